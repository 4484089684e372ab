"""Element-by-element parity at the benchmark's full sizes.

slab1000 (25x10x2 slab, N = 1000, m = 8, tau = 1e-10) is built by the HIP
path in FP64, STORE32 and MIXED, and every J and K element of every density
is compared with the oracle's full grouped build of Eq. J_and_K (about two
minutes of host time, computed once per session in chunks of outer pairs).
MIXED also runs on the FP64 store (integrals rounded to FP32 as they load).
The 64-molecule batch (chains, N 50..600, m 2..10) is held to the oracle in
all three precisions (MIXED on both stores), every molecule in full.

Tolerances (absolute, max over densities and elements): 1e-10 for FP64
builds, 1e-8 for the FP32-storage builds.  max|dF| with F = 2J - K is
announced too.
"""
import time

import numpy as np
import pytest

import workloads as wl
from gpu_util import announce, dev, host, maxabs

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-8


@pytest.fixture(scope="module")
def pa():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2002_00322_amd as pa
    return pa


def oracle_full(oracle_mod, c, chunks=8):
    """The oracle's grouped build over all unique quartets, split into ranges
    of the outer pair index of about equal work (the work of pair a grows
    like a), each range reported as it ends."""
    n = c["alpha"].shape[0]
    npair = n * (n + 1) // 2
    cuts = [0] + [int(npair * np.sqrt(x / chunks)) for x in range(1, chunks)] + [npair]
    J = np.zeros(c["D"].shape)
    K = np.zeros(c["D"].shape)
    total = 0
    t0 = time.time()
    for a, b in zip(cuts[:-1], cuts[1:]):
        Jc, Kc, nv = oracle_mod.jk_canonical_range(c["centers"], c["alpha"], c["tau"], c["D"], a, b)
        J += Jc
        K += Kc
        total += nv
        announce(f"oracle {c['name']}: outer pairs [{a}, {b}) done, {total} quartets, "
                 f"{time.time() - t0:.1f} s")
    return J, K, total


def report(name, J, K, Jr, Kr):
    ej, ek = maxabs(J, Jr), maxabs(K, Kr)
    ef = maxabs(2.0 * J - K, 2.0 * Jr - Kr)
    announce(f"{name}: max|dJ|={ej:.3e} max|dK|={ek:.3e} max|dF|={ef:.3e}")
    return ej, ek, ef


@pytest.fixture(scope="module")
def slab_ref(oracle_mod):
    c = wl.config3()
    announce("slab1000: full oracle build (FP64, all unique quartets)")
    J, K, nv = oracle_full(oracle_mod, c)
    return c, J, K, nv


@pytest.mark.timeout(900)
def test_slab1000_fp64_every_element(pa, slab_ref):
    import torch
    c, Jr, Kr, nv = slab_ref
    announce("slab1000 fp64: prepare and build")
    st = pa.EriStore(c["centers"], c["alpha"], c["tau"])
    assert abs(st.info()["nquartets_kept"] - nv) <= 8
    d = dev(c["D"])
    j, k = pa.fock_build(st, d)
    torch.cuda.synchronize()
    ej, ek, _ = report("slab1000 fp64", host(j), host(k), Jr, Kr)
    # MIXED on the same FP64 store: integrals rounded to FP32 as they load
    jm, km = pa.fock_build(st, d, prec=pa.PREC_MIXED)
    torch.cuda.synchronize()
    mj, mk, _ = report("slab1000 mixed on the FP64 store", host(jm), host(km), Jr, Kr)
    st.release()
    assert ej < TOL64 and ek < TOL64
    assert mj < TOL32 and mk < TOL32 and max(mj, mk) > 1e-14


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec_name", ["store32", "mixed"])
def test_slab1000_fp32_storage_every_element(pa, slab_ref, prec_name):
    import torch
    c, Jr, Kr, _ = slab_ref
    prec = pa.PREC_STORE32 if prec_name == "store32" else pa.PREC_MIXED
    announce(f"slab1000 {prec_name}: prepare and build")
    st = pa.EriStore(c["centers"], c["alpha"], c["tau"], storage=pa.STORE_FP32)
    d = dev(c["D"])
    j, k = pa.fock_build(st, d, prec=prec)
    torch.cuda.synchronize()
    ej, ek, _ = report(f"slab1000 {prec_name}", host(j), host(k), Jr, Kr)
    st.release()
    assert ej < TOL32 and ek < TOL32
    assert max(ej, ek) > 1e-14   # the FP32 integrals leave a trace


@pytest.fixture(scope="module")
def batch_ref(oracle_mod):
    mols = wl.batch_workload()
    t0 = time.time()
    refs = [oracle_mod.jk_canonical(c["centers"], c["alpha"], c["tau"], c["D"]) for c in mols]
    announce(f"batch64: oracle for {len(mols)} molecules in {time.time() - t0:.1f} s")
    return mols, refs


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec_name", ["fp64", "store32", "mixed", "mixed_fp64_store"])
def test_batch64_every_molecule_against_oracle(pa, batch_ref, prec_name):
    import torch
    mols, refs = batch_ref
    prec = {"fp64": pa.PREC_FP64, "store32": pa.PREC_STORE32, "mixed": pa.PREC_MIXED,
            "mixed_fp64_store": pa.PREC_MIXED}[prec_name]
    storage = pa.STORE_FP64 if prec_name in ("fp64", "mixed_fp64_store") else pa.STORE_FP32
    tol = TOL64 if prec_name == "fp64" else TOL32
    announce(f"batch64 {prec_name}: {len(mols)} molecules in one batched build")
    stores = [pa.EriStore(c["centers"], c["alpha"], c["tau"], storage=storage) for c in mols]
    s = torch.cuda.Stream()
    ds = [dev(c["D"]) for c in mols]
    js = [torch.full_like(d, float("nan")) for d in ds]
    ks = [torch.full_like(d, float("nan")) for d in ds]
    torch.cuda.synchronize()
    pa.fock_build_batched(stores, ds, js, ks, prec=prec, stream=s)
    s.synchronize()
    worst = (0.0, 0.0, 0.0, "")
    bad = []
    for c, (Jr, Kr), j, k in zip(mols, refs, js, ks):
        J, K = host(j), host(k)
        ej, ek = maxabs(J, Jr), maxabs(K, Kr)
        ef = maxabs(2.0 * J - K, 2.0 * Jr - Kr)
        if max(ej, ek) > max(worst[0], worst[1]):
            worst = (ej, ek, ef, c["name"])
        if not (ej < tol and ek < tol):
            bad.append((c["name"], ej, ek))
    announce(f"batch64 {prec_name}: worst {worst[3]} max|dJ|={worst[0]:.3e} max|dK|={worst[1]:.3e} "
             f"max|dF|={worst[2]:.3e}")
    for st in stores:
        st.release()
    assert not bad, bad
