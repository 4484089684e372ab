"""The nine ESMF densities and the two-body energy on the GPU, through the C ABI.

Densities: each product is held element by element to the oracle's within
8 (N + No + Nv) eps times the same product of absolute values (for A and B the
sum of both terms'), a bound on the rounding of products whose inner
dimensions are at most N, No and Nv.
Energy: from the same J and K, the GPU reduction is held to the oracle's
within 1e-13 of the sum of the absolute terms; from the GPU's own FP64 build,
within the J/K tolerance of the FP64 build (1e-10) times the sum of the
absolute densities it multiplies.
"""
import numpy as np
import pytest

import workloads as wl
from gpu_util import announce, dev, host, maxabs

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps
TOL64 = 1e-10


@pytest.fixture(scope="module")
def pa():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2002_00322_amd as pa
    return pa


def _gpu_densities(pa, st):
    import torch
    d = pa.nine_densities(*(dev(st[k]) for k in ("theta", "gamma", "sigma", "mu", "R", "Phi")))
    torch.cuda.synchronize()
    return d


def _abs_bound(oracle_mod, st):
    a = {k: np.abs(st[k]) for k in ("theta", "gamma", "sigma", "mu", "R", "Phi")}
    z = {k: np.zeros_like(v) for k, v in a.items()}
    M = oracle_mod.nine_densities(a["theta"], a["gamma"], a["sigma"], a["mu"], a["R"], a["Phi"])
    # A and B: add the magnitudes of their two terms instead of subtracting
    M[2] = (oracle_mod.nine_densities(z["theta"], a["gamma"], a["sigma"], a["mu"], a["R"], a["Phi"])[2]
            - oracle_mod.nine_densities(a["theta"], z["gamma"], a["sigma"], a["mu"], a["R"], a["Phi"])[2])
    M[8] = (oracle_mod.nine_densities(a["theta"], a["gamma"], a["sigma"], a["mu"], z["R"], a["Phi"])[8]
            - oracle_mod.nine_densities(a["theta"], a["gamma"], a["sigma"], a["mu"], a["R"], z["Phi"])[8])
    return M


def _check_densities(oracle_mod, st, D):
    n = st["theta"].shape[1]
    no, nv = st["sigma"].shape
    ref = oracle_mod.nine_densities(st["theta"], st["gamma"], st["sigma"], st["mu"], st["R"], st["Phi"])
    bound = 8.0 * (n + no + nv) * EPS * _abs_bound(oracle_mod, st) + 1e-300
    err = np.abs(D - ref)
    worst = [float(np.max(err[i] / bound[i])) for i in range(9)]
    announce(f"densities N={n} No={no} Nv={nv}: worst err/bound per density "
             + " ".join(f"{w:.2g}" for w in worst))
    assert all(w <= 1.0 for w in worst), worst
    return ref


@pytest.mark.parametrize("n,no,seed", [(2, 1, 1), (3, 1, 2), (17, 5, 3), (40, 20, 4), (33, 16, 5),
                                       (100, 37, 6), (257, 64, 7), (400, 40, 8), (1000, 40, 9),
                                       (1500, 150, 10), (2113, 67, 11)])
def test_nine_densities_match_oracle(pa, oracle_mod, n, no, seed):
    st = wl.esmf_state(n, no, seed)
    D = host(_gpu_densities(pa, st))
    _check_densities(oracle_mod, st, D)
    # D1 and A exactly symmetric (a build may mark them so)
    assert np.array_equal(D[0], D[0].T) and np.array_equal(D[2], D[2].T)


def test_nine_densities_general_sizes(pa, oracle_mod):
    # No + Nv need not equal N; rows need not be orthonormal
    import torch
    rng = np.random.default_rng(77)
    n, no, nv = 23, 7, 9
    st = dict(theta=rng.standard_normal((no, n)), gamma=rng.standard_normal((nv, n)),
              sigma=rng.standard_normal((no, nv)), mu=rng.standard_normal((no, nv)),
              R=rng.standard_normal((no, n)), Phi=rng.standard_normal((nv, n)))
    announce("densities with No + Nv != N")
    D = host(_gpu_densities(pa, st))
    _check_densities(oracle_mod, st, D)
    # a preallocated output is filled in place; stale contents do not leak
    out = torch.full((9, n, n), float("nan"), dtype=torch.float64, device="cuda:0")
    got = pa.nine_densities(*(dev(st[k]) for k in ("theta", "gamma", "sigma", "mu", "R", "Phi")), d=out)
    torch.cuda.synchronize()
    assert got.data_ptr() == out.data_ptr() and np.array_equal(host(out), D)


def _energy_terms_sum(D, J, K, n2, c0):
    F1, F2 = np.abs(2 * J[0] - K[0]), np.abs(2 * J[1] - K[1])
    return float(abs(n2) * np.sum(F1 * np.abs(D[0])) + 4 * abs(c0) * np.sum(F1 * np.abs(D[1]))
                 + 2 * np.sum(F1 * np.abs(D[2])) + 2 * np.sum(F2 * np.abs(D[1])))


def _jk_bound(D, n2, c0):
    # |dE| from |dJ|, |dK| <= TOL64 entrywise: |dF| <= 3 TOL64
    return 3 * TOL64 * float(abs(n2) * np.sum(np.abs(D[0])) + 4 * abs(c0) * np.sum(np.abs(D[1]))
                             + 2 * np.sum(np.abs(D[2])) + 2 * np.sum(np.abs(D[1])))


@pytest.mark.parametrize("case", ["box40", "chain400"])
def test_energy_pipeline_matches_oracle(pa, oracle_mod, case):
    # densities -> one grouped FP64 build of all nine -> E_2, all on the GPU
    import torch
    c = wl.config1() if case == "box40" else wl.config2()
    n = c["alpha"].shape[0]
    no = 20 if case == "box40" else 40
    st = wl.esmf_state(n, no, 600 + n)
    announce(f"ESMF pipeline {case}: N={n} No={no}, nine densities in one build")
    eri = pa.EriStore(c["centers"], c["alpha"], c["tau"])
    d = _gpu_densities(pa, st)
    j, k = pa.fock_build(eri, d)
    e2 = pa.energy_two_body(d, j, k, st["n2"], st["c0"])
    torch.cuda.synchronize()
    D, J, K = host(d), host(j), host(k)
    Dr = _check_densities(oracle_mod, st, D)
    Jr, Kr = oracle_mod.jk_canonical(c["centers"], c["alpha"], c["tau"], Dr)
    assert np.max(np.abs(J - Jr)) < TOL64 and np.max(np.abs(K - Kr)) < TOL64
    er = oracle_mod.energy_two_body(Jr, Kr, Dr, st["n2"], st["c0"])
    got = float(e2.item())
    announce(f"{case}: E2 gpu={got:.15e} oracle={er:.15e} diff={got - er:.2e}")
    assert abs(got - er) <= _jk_bound(Dr, st["n2"], st["c0"]) + 1e-13 * _energy_terms_sum(Dr, Jr, Kr, st["n2"], st["c0"])
    # the reduction alone: the oracle's J, K and densities on the device
    e2o = pa.energy_two_body(dev(Dr), dev(Jr[:2]), dev(Kr[:2]), st["n2"], st["c0"])
    torch.cuda.synchronize()
    assert abs(float(e2o.item()) - er) <= 1e-13 * _energy_terms_sum(Dr, Jr, Kr, st["n2"], st["c0"])
    eri.release()


def test_energy_hf_limit(pa, oracle_mod):
    # sigma = 0, c0 = N2 = 1: D2 = A = 0 and E_2 = F[D1] . D1
    import torch
    c = wl.config1()
    st = wl.esmf_state(40, 12, 31, sigma_norm=0.0, c0=1.0)
    st["sigma"][:] = 0.0
    announce("ESMF energy, HF limit (box40)")
    eri = pa.EriStore(c["centers"], c["alpha"], c["tau"])
    d = _gpu_densities(pa, st)
    j, k = pa.fock_build(eri, d[:2].contiguous())
    e2 = pa.energy_two_body(d, j, k, 1.0, 1.0)
    torch.cuda.synchronize()
    D = host(d)
    assert np.all(D[1] == 0) and np.all(D[2] == 0)
    Jr, Kr = oracle_mod.jk_canonical(c["centers"], c["alpha"], c["tau"], D[:1])
    ref = float(np.sum((2 * Jr[0] - Kr[0]) * D[0]))
    assert abs(float(e2.item()) - ref) <= 3 * TOL64 * np.sum(np.abs(D[0])) + 1e-13 * abs(ref)
    eri.release()


def test_full_size_slab1000_sampled(pa, oracle_mod):
    # the benchmark workload: slab1000 (N=1000), No=40, all nine densities in
    # one grouped build; sampled J/K entries against the oracle, the energy
    # against a host evaluation of the same formula from the GPU's J, K
    import torch
    c = wl.config3()
    st = wl.esmf_state(1000, 40, 9)
    announce("ESMF terms at slab1000: nine densities, one build, energy")
    eri = pa.EriStore(c["centers"], c["alpha"], c["tau"])
    d = _gpu_densities(pa, st)
    j, k = pa.fock_build(eri, d)
    e2 = pa.energy_two_body(d, j, k, st["n2"], st["c0"])
    torch.cuda.synchronize()
    D, J, K = host(d), host(j), host(k)
    _check_densities(oracle_mod, st, D)
    rng = np.random.default_rng(5)
    cnt = 36
    i, p, q = rng.integers(0, 9, cnt), rng.integers(0, 1000, cnt), rng.integers(0, 1000, cnt)
    Jr, Kr = oracle_mod.jk_entries(c["centers"], c["alpha"], c["tau"], D, i, p, q)
    assert np.max(np.abs(J[i, p, q] - Jr)) < TOL64 and np.max(np.abs(K[i, p, q] - Kr)) < TOL64
    eh = oracle_mod.energy_two_body(J, K, D, st["n2"], st["c0"])
    assert abs(float(e2.item()) - eh) <= 1e-13 * _energy_terms_sum(D, J, K, st["n2"], st["c0"])
    eri.release()


def test_energy_is_deterministic(pa):
    import torch
    n = 300
    rng = np.random.default_rng(3)
    d, j, k = dev(rng.standard_normal((3, n, n))), dev(rng.standard_normal((2, n, n))), \
        dev(rng.standard_normal((2, n, n)))
    announce("ESMF energy: repeated calls, bitwise")
    vals = [float(pa.energy_two_body(d, j, k, 1.3, -0.4).item()) for _ in range(3)]
    torch.cuda.synchronize()
    assert vals[0] == vals[1] == vals[2]


# ---- the energy gradient and the GVP two-pass form --------------------------

def _grad_gpu(pa, st, d, j, k):
    import torch
    g = pa.energy_gradient(*(dev(st[x]) for x in ("theta", "gamma", "sigma", "G")), d, j, k, st["c0"], st["n2"])
    torch.cuda.synchronize()
    return {x: host(v) for x, v in g.items()}


def _grad_err(got, ref):
    out = {}
    for x in ("sigma", "theta", "gamma"):
        out[x] = float(np.max(np.abs(got[x] - ref[x])) / max(1.0, np.max(np.abs(ref[x]))))
    e = got["energy"]
    for i, x in enumerate(("E1", "E2", "E", "c0")):
        out[x] = float(abs(e[i] - ref[x]) / max(1.0, abs(ref[x])))
    return out


@pytest.mark.parametrize("case", ["box40", "chain400", "edge13"])
def test_energy_gradient_assembly_matches_oracle(pa, oracle_mod, case):
    # the same J, K on both sides: the GPU assembly (GEMMs, dots, quotient)
    # against the oracle's formulas, relative to the largest entry
    if case == "box40":
        c, no = wl.config1(), 20
    elif case == "chain400":
        c, no = wl.config2(), 40
    else:
        A, al = wl.random_box(13, seed=13, box=6.0)
        c, no = dict(centers=A, alpha=al, tau=1e-10), 4
    n = c["alpha"].shape[0]
    st = wl.esmf_state(n, no, 800 + n)
    D = oracle_mod.nine_densities(st["theta"], st["gamma"], st["sigma"], st["mu"], st["R"], st["Phi"])
    J, K = oracle_mod.jk_canonical(c["centers"], c["alpha"], c["tau"], D[:3])
    ref = oracle_mod.energy_gradient(st["G"], J, K, D, st["theta"], st["gamma"], st["sigma"], st["c0"], st["n2"])
    announce(f"energy gradient assembly: {case} N={n} No={no}")
    got = _grad_gpu(pa, st, dev(D[:3]), dev(J), dev(K))
    err = _grad_err(got, ref)
    announce(f"{case}: relative errors {err}")
    assert all(v < 1e-12 for v in err.values()), err


@pytest.mark.parametrize("n,no", [(1500, 150), (1601, 33)])
def test_energy_gradient_assembly_large(pa, oracle_mod, n, no):
    # sizes whose products run on the 64 x 64 tiles (and ragged tails): the
    # assembly from seeded J, K (any J, K define the same formulas) against
    # the oracle's, relative to the largest entry
    st = wl.esmf_state(n, no, 900 + n)
    D = oracle_mod.nine_densities(st["theta"], st["gamma"], st["sigma"], st["mu"], st["R"], st["Phi"])
    rng = np.random.default_rng(n)
    J = rng.standard_normal((3, n, n)) * 0.1
    K = rng.standard_normal((3, n, n)) * 0.1
    J = 0.5 * (J + J.transpose(0, 2, 1))
    ref = oracle_mod.energy_gradient(st["G"], J, K, D[:3], st["theta"], st["gamma"], st["sigma"], st["c0"], st["n2"])
    announce(f"energy gradient assembly: seeded J, K, N={n} No={no}")
    got = _grad_gpu(pa, st, dev(D[:3]), dev(J), dev(K))
    err = _grad_err(got, ref)
    announce(f"N={n}: relative errors {err}")
    assert all(v < 1e-12 for v in err.values()), err


def test_gvp_two_pass_chain400(pa, oracle_mod):
    # Sec. "Derivatives of GVP-based Objective Function": pass 1 builds the
    # three densities of the energy (D1, A symmetric), the energy gradient
    # replaces the multipliers (mu = dE/dsigma, R = dE/dTheta,
    # Phi = dE/dGamma), pass 2 builds the six densities that depend on it.
    import torch
    c = wl.config2()
    n, no = 400, 40
    st = wl.esmf_state(n, no, 4242)
    announce("GVP two-pass form: chain400")
    eri = pa.EriStore(c["centers"], c["alpha"], c["tau"])
    T, Gm, S = (dev(st[x]) for x in ("theta", "gamma", "sigma"))
    z = dict(mu=torch.zeros_like(S), R=torch.zeros_like(T), Phi=torch.zeros_like(Gm))
    d1 = pa.nine_densities(T, Gm, S, z["mu"], z["R"], z["Phi"])
    d3 = d1[:3].contiguous()
    j3, k3 = pa.fock_build(eri, d3, symmetric=(1, 0, 1))
    g = pa.energy_gradient(T, Gm, S, dev(st["G"]), d3, j3, k3, st["c0"], st["n2"])
    d2 = pa.nine_densities(T, Gm, S, g["sigma"], g["theta"], g["gamma"])
    d6 = d2[3:].contiguous()
    j6, k6 = pa.fock_build(eri, d6)
    torch.cuda.synchronize()
    # oracle chain from the same state
    D = oracle_mod.nine_densities(st["theta"], st["gamma"], st["sigma"], st["mu"], st["R"], st["Phi"])
    J3, K3 = oracle_mod.jk_canonical(c["centers"], c["alpha"], c["tau"], D[:3])
    assert maxabs(host(j3), J3) < TOL64 and maxabs(host(k3), K3) < TOL64
    ref = oracle_mod.energy_gradient(st["G"], J3, K3, D, st["theta"], st["gamma"], st["sigma"], st["c0"],
                                     st["n2"])
    got = {x: host(v) for x, v in g.items()}
    err = _grad_err(got, ref)
    announce(f"GVP pass-1 gradient relative errors {err}")
    assert all(v < 1e-9 for v in err.values()), err
    D2 = oracle_mod.nine_densities(st["theta"], st["gamma"], st["sigma"], ref["sigma"], ref["theta"], ref["gamma"])
    dd = float(np.max(np.abs(host(d6) - D2[3:])) / np.max(np.abs(D2[3:])))
    announce(f"GVP pass-2 densities: relative error {dd:.2e}")
    assert dd < 1e-9
    # pass 2's build against the oracle on the densities it was given
    J6, K6 = oracle_mod.jk_canonical(c["centers"], c["alpha"], c["tau"], host(d6))
    assert maxabs(host(j6), J6) < TOL64 and maxabs(host(k6), K6) < TOL64
    eri.release()


def test_energy_gradient_rejects_bad_arguments(pa):
    import torch
    n, no = 12, 3
    st = wl.esmf_state(n, no, 5)
    T, Gm, S, G = (dev(st[x]) for x in ("theta", "gamma", "sigma", "G"))
    d = dev(np.zeros((3, n, n)))
    announce("energy gradient: argument errors")
    with pytest.raises(pa.InvalidArgument):
        pa.energy_gradient(T, Gm, S, G, d[:2], d, d, st["c0"], st["n2"])
    with pytest.raises(pa.InvalidArgument):
        pa.energy_gradient(T, Gm, S, G, d, d, d, st["c0"], 0.0)
    with pytest.raises(pa.InvalidArgument):
        pa.energy_gradient(T, Gm, S, G[:, :5].contiguous(), d, d, d, st["c0"], st["n2"])
    torch.cuda.synchronize()


def test_gvp_two_pass_slab1000_sampled(pa, oracle_mod):
    # the bench's GVP step at full size: pass 1 (D1, D2, A; two marked
    # symmetric) and pass 2 (the six densities from the gradient) sampled
    # against the oracle's definition; the gradient assembly against the
    # oracle's formulas on the same J, K
    import torch
    c = wl.config3()
    n, no = 1000, 40
    st = wl.esmf_state(n, no, 9)
    announce("GVP two-pass form at slab1000: sampled")
    eri = pa.EriStore(c["centers"], c["alpha"], c["tau"])
    T, Gm, S, G = (dev(st[x]) for x in ("theta", "gamma", "sigma", "G"))
    z = [torch.zeros_like(S), torch.zeros_like(T), torch.zeros_like(Gm)]
    d3 = pa.nine_densities(T, Gm, S, *z)[:3].contiguous()
    j3, k3 = pa.fock_build(eri, d3, symmetric=(1, 0, 1))
    g = pa.energy_gradient(T, Gm, S, G, d3, j3, k3, st["c0"], st["n2"])
    d6 = pa.nine_densities(T, Gm, S, g["sigma"], g["theta"], g["gamma"])[3:].contiguous()
    j6, k6 = pa.fock_build(eri, d6)
    torch.cuda.synchronize()
    D3, J3, K3, D6, J6, K6 = (host(x) for x in (d3, j3, k3, d6, j6, k6))
    rng = np.random.default_rng(17)
    for D, J, K, m in ((D3, J3, K3, 3), (D6, J6, K6, 6)):
        cnt = 20
        i, p, q = rng.integers(0, m, cnt), rng.integers(0, n, cnt), rng.integers(0, n, cnt)
        Jr, Kr = oracle_mod.jk_entries(c["centers"], c["alpha"], c["tau"], D, i, p, q)
        assert np.max(np.abs(J[i, p, q] - Jr)) < TOL64 and np.max(np.abs(K[i, p, q] - Kr)) < TOL64
    ref = oracle_mod.energy_gradient(st["G"], J3, K3, D3, st["theta"], st["gamma"], st["sigma"], st["c0"],
                                     st["n2"])
    err = _grad_err({x: host(v) for x, v in g.items()}, ref)
    announce(f"slab1000 gradient assembly, relative errors {err}")
    assert all(v < 1e-12 for v in err.values()), err
    D6r = oracle_mod.nine_densities(st["theta"], st["gamma"], st["sigma"], host(g["sigma"]), host(g["theta"]),
                                    host(g["gamma"]))[3:]
    assert np.max(np.abs(D6 - D6r)) <= 1e-12 * np.max(np.abs(D6r))
    eri.release()
