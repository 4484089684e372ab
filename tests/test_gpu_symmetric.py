"""Builds with densities marked symmetric (esmf_fock_build_sym).

A symmetric density takes one matrix-core column instead of two, so up to 16
densities share one pass over the integrals (the paper's nine ESMF densities,
two of them symmetric, in one pass).  For exactly symmetric flagged
densities every column a flagged build uses carries the same values as the
corresponding column of the unflagged build, so the results must be bitwise
equal to esmf_fock_build's run with the same work plan, and within the FP64
tolerance of the oracle.  A wide group (more than 8 densities) always runs
the two-visit plan, so the bitwise comparisons here run every build on that
plan (ESMF_PLAN=0; it is the default of stored integrals, integral-direct
stores default to the fused plan); the fused plan is compared within
rounding.
"""
import numpy as np
import pytest

import workloads as wl
from gpu_util import announce, dev, host, maxabs

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


@pytest.fixture(autouse=True)
def two_visit_plan(monkeypatch):
    monkeypatch.setenv("ESMF_PLAN", "0")


@pytest.fixture(scope="module")
def pa():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2002_00322_amd as pa
    return pa


def _dens(n, flags, seed):
    rng = np.random.default_rng(seed)
    D = rng.standard_normal((len(flags), n, n)) / n
    for i, f in enumerate(flags):
        if f:
            D[i] = D[i] + D[i].T  # exactly symmetric
    return D


def _both(pa, st, D, flags, prec=0):
    import torch
    d = dev(D)
    j0, k0 = pa.fock_build(st, d, prec=prec)
    j1, k1 = pa.fock_build(st, d, prec=prec, symmetric=flags)
    torch.cuda.synchronize()
    return host(j0), host(k0), host(j1), host(k1)


CASES = [
    ("esmf9", (1, 0, 1, 0, 0, 0, 0, 0, 0)),          # one wide pass (16 K columns)
    ("sym12", (1,) * 12),                             # one wide pass (12 K columns)
    ("sym16", (1,) * 16),                             # one wide pass
    ("sym17", (1,) * 17),                             # wide 16 + narrow 1
    ("sym1", (1,)),
    ("mix13", (0, 1, 1, 0, 1, 0, 0, 1, 1, 1, 0, 1, 0)),
    ("none10", (0,) * 10),                            # no flag set: groups of 8
    ("tail", (0,) * 7 + (1,) * 3),                    # 7*2 + 2 = 16 columns, then 1
]


@pytest.mark.parametrize("name,flags", CASES)
def test_flagged_build_bitwise_equal_chain400(pa, oracle_mod, name, flags):
    c = wl.config2()
    n = c["alpha"].shape[0]
    announce(f"symmetric-flag build {name}: m={len(flags)} chain400")
    st = pa.EriStore(c["centers"], c["alpha"], c["tau"])
    D = _dens(n, flags, 500 + len(flags))
    J0, K0, J1, K1 = _both(pa, st, D, flags)
    assert np.array_equal(J0, J1) and np.array_equal(K0, K1), (maxabs(J0, J1), maxabs(K0, K1))
    if name in ("esmf9", "sym17"):
        Jr, Kr = oracle_mod.jk_canonical(c["centers"], c["alpha"], c["tau"], D)
        assert maxabs(J1, Jr) < TOL64 and maxabs(K1, Kr) < TOL64
    st.release()


@pytest.mark.parametrize("case", ["box40", "edge13", "edge37"])
def test_flagged_build_against_oracle_small(pa, oracle_mod, case):
    if case == "box40":
        c = wl.config1()
    else:
        nn = int(case[4:])
        A, al = wl.random_box(nn, seed=nn, box=6.0)
        c = dict(centers=A, alpha=al, tau=1e-10)
    n = c["alpha"].shape[0]
    flags = (1, 0, 1, 0, 0, 0, 0, 0, 0, 1, 1)
    D = _dens(n, flags, 70 + n)
    announce(f"symmetric-flag build vs oracle: {case}, m={len(flags)}")
    st = pa.EriStore(c["centers"], c["alpha"], c["tau"])
    J0, K0, J1, K1 = _both(pa, st, D, flags)
    Jr, Kr = oracle_mod.jk_canonical(c["centers"], c["alpha"], c["tau"], D)
    assert maxabs(J1, Jr) < TOL64 and maxabs(K1, Kr) < TOL64
    assert np.array_equal(J0, J1) and np.array_equal(K0, K1)
    st.release()


@pytest.mark.parametrize("prec", ["mixed", "store32", "direct"])
def test_flagged_build_other_paths(pa, prec):
    c = wl.config2()
    n = c["alpha"].shape[0]
    flags = (1, 0, 1, 0, 0, 0, 0, 0, 0)
    storage = {"mixed": pa.STORE_FP32, "store32": pa.STORE_FP32, "direct": pa.STORE_DIRECT}[prec]
    p = {"mixed": pa.PREC_MIXED, "store32": pa.PREC_STORE32, "direct": pa.PREC_FP64}[prec]
    announce(f"symmetric-flag build, {prec}: esmf9 chain400")
    st = pa.EriStore(c["centers"], c["alpha"], c["tau"], storage=storage)
    D = _dens(n, flags, 91)
    J0, K0, J1, K1 = _both(pa, st, D, flags, prec=p)
    assert np.array_equal(J0, J1) and np.array_equal(K0, K1), (maxabs(J0, J1), maxabs(K0, K1))
    st.release()


def test_flag_on_nonsymmetric_density_keeps_j(pa):
    # J is exact for any flagged density; K of a flagged non-symmetric one is
    # unspecified (finite here), the unflagged densities are unaffected
    import torch
    c = wl.config2()
    n = c["alpha"].shape[0]
    D = _dens(n, (0,) * 9, 17)
    flags = (1, 0, 0, 0, 0, 0, 0, 0, 0)
    announce("flag on a non-symmetric density")
    st = pa.EriStore(c["centers"], c["alpha"], c["tau"])
    J0, K0, J1, K1 = _both(pa, st, D, flags)
    assert np.array_equal(J0, J1)
    assert np.array_equal(K0[1:], K1[1:])
    assert np.all(np.isfinite(K1[0]))
    with pytest.raises(pa.InvalidArgument):
        pa.fock_build(st, dev(D), symmetric=flags[:5])
    torch.cuda.synchronize()
    st.release()


def test_esmf_nine_in_one_pass_slab1000(pa, oracle_mod):
    # the paper's configuration: the nine densities of a gradient evaluation
    # built in one loop over the retained pairs; sampled against the oracle
    # and bitwise against the two-pass build
    import torch
    c = wl.config3()
    es = wl.esmf_state(1000, 40, 9)
    announce("ESMF nine densities in one pass: slab1000")
    st = pa.EriStore(c["centers"], c["alpha"], c["tau"])
    d = pa.nine_densities(*(dev(es[k]) for k in ("theta", "gamma", "sigma", "mu", "R", "Phi")))
    torch.cuda.synchronize()
    D = host(d)
    assert np.array_equal(D[0], D[0].T) and np.array_equal(D[2], D[2].T)
    j1, k1 = pa.fock_build(st, d, symmetric=pa.ESMF_SYMMETRIC)
    torch.cuda.synchronize()
    J1, K1 = host(j1), host(k1)
    del j1, k1
    j0, k0 = pa.fock_build(st, d)
    torch.cuda.synchronize()
    assert np.array_equal(host(j0), J1) and np.array_equal(host(k0), K1)
    rng = np.random.default_rng(8)
    cnt = 30
    i, p, q = rng.integers(0, 9, cnt), rng.integers(0, 1000, cnt), rng.integers(0, 1000, cnt)
    Jr, Kr = oracle_mod.jk_entries(c["centers"], c["alpha"], c["tau"], D, i, p, q)
    assert np.max(np.abs(J1[i, p, q] - Jr)) < TOL64 and np.max(np.abs(K1[i, p, q] - Kr)) < TOL64
    st.release()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_default_fused_plan_agrees_with_flagged_build(pa, monkeypatch, prec):
    # the unflagged build on the fused plan sums the same products in another
    # order than the flagged (wide, two-visit) build: equal to FP64 rounding
    # (FP32 chains for mixed)
    c = wl.config2()
    n = c["alpha"].shape[0]
    flags = (1, 0, 1, 0, 0, 0, 0, 0, 0)
    storage = pa.STORE_FP64 if prec == "fp64" else pa.STORE_FP32
    p = pa.PREC_FP64 if prec == "fp64" else pa.PREC_MIXED
    announce(f"fused unflagged vs two-visit flagged, {prec}: esmf9 chain400")
    st = pa.EriStore(c["centers"], c["alpha"], c["tau"], storage=storage)
    D = _dens(n, flags, 93)
    monkeypatch.setenv("ESMF_PLAN", "1")
    J0, K0, J1, K1 = _both(pa, st, D, flags, prec=p)
    scale = max(np.abs(J0).max(), np.abs(K0).max())
    tol = 1e-13 if prec == "fp64" else 1e-8 / scale
    announce(f"fused vs two-visit {prec}: max|dJ|={maxabs(J0, J1):.3e} max|dK|={maxabs(K0, K1):.3e}")
    assert maxabs(J0, J1) < tol * scale and maxabs(K0, K1) < tol * scale
    st.release()


@pytest.mark.parametrize("seed", range(12))
def test_seeded_small_builds_against_oracle(pa, oracle_mod, seed):
    # seeded molecules of 3..48 functions (ragged tiles), 1..12 densities
    # with seeded symmetric flags, three thresholds: each group's column set
    # (packed narrow columns, 4x4x4 K products for up to 8 columns, wide
    # groups) held to the oracle, on the FP64 and integral-direct stores, and
    # the flagged build bitwise equal to the unflagged one
    import torch
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(3, 49))
    m = int(rng.integers(1, 13))
    tau = float(rng.choice([0.0, 1e-10, 1e-6]))
    A, al = wl.random_box(n, seed=2000 + seed, box=float(rng.uniform(3.0, 9.0)))
    flags = tuple(int(x) for x in rng.integers(0, 2, m))
    D = _dens(n, flags, 3000 + seed)
    announce(f"seeded build {seed}: n={n} m={m} tau={tau:g} flags={flags}")
    Jr, Kr = oracle_mod.jk_canonical(A, al, tau, D)
    for storage in (pa.STORE_FP64, pa.STORE_DIRECT):
        st = pa.EriStore(A, al, tau, storage=storage)
        J0, K0, J1, K1 = _both(pa, st, D, flags)
        assert maxabs(J1, Jr) < TOL64 and maxabs(K1, Kr) < TOL64, (storage, maxabs(J1, Jr), maxabs(K1, Kr))
        assert np.array_equal(J0, J1) and np.array_equal(K0, K1), storage
        st.release()
    torch.cuda.synchronize()
