"""Batched builds (esmf_fock_build_batched) through the C ABI.

A batched build must give, bitwise, what one build per molecule gives (same
kernels, same fixed reduction order), and the per-molecule builds are held to
the FP64 oracle here and in the single-build parity tests.  The graph path is
replayed several times with eager work and synchronisations between replays;
every replay is checked against the eager per-molecule result.
"""
import numpy as np
import pytest

import workloads as wl
from gpu_util import announce, dev, host, maxabs

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


@pytest.fixture(scope="module")
def pa():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2002_00322_amd as pa
    return pa


@pytest.fixture(scope="module")
def mols():
    return wl.batch_workload()


def _stores(pa, mols, storage):
    return [pa.EriStore(c["centers"], c["alpha"], c["tau"], storage=storage) for c in mols]


def _single(pa, stores, ds, prec, stream):
    import torch
    out = []
    with torch.cuda.stream(stream):
        for st, d in zip(stores, ds):
            j, k = pa.fock_build(st, d, prec=prec, stream=stream)
            out.append((j, k))
    stream.synchronize()
    return [(host(j), host(k)) for j, k in out]


def _batched(pa, stores, ds, prec, stream):
    import torch
    with torch.cuda.stream(stream):
        js = [torch.full_like(d, float("nan")) for d in ds]
        ks = [torch.full_like(d, float("nan")) for d in ds]
    stream.synchronize()
    pa.fock_build_batched(stores, ds, js, ks, prec=prec, stream=stream)
    stream.synchronize()
    return [(host(j), host(k)) for j, k in zip(js, ks)]


def test_batched_fp64_equals_single_and_oracle(pa, mols, oracle_mod):
    import torch
    announce(f"batched fp64: {len(mols)} molecules, N {min(c['alpha'].shape[0] for c in mols)}.."
             f"{max(c['alpha'].shape[0] for c in mols)}")
    stores = _stores(pa, mols, pa.STORE_FP64)
    s = torch.cuda.Stream()
    ds = [dev(c["D"]) for c in mols]
    ref = _single(pa, stores, ds, pa.PREC_FP64, s)
    got = _batched(pa, stores, ds, pa.PREC_FP64, s)
    for i, ((jr, kr), (jg, kg)) in enumerate(zip(ref, got)):
        assert np.array_equal(jr, jg) and np.array_equal(kr, kg), f"molecule {i} {mols[i]['name']}"
    # the first call tuned the plan and captured it as a graph on this stream
    rep = pa.batched_report()
    announce(f"batched report: {rep}")
    assert rep["graph"] and rep["units"] >= len(mols) and rep["items"] > 0
    assert len(rep["tuner"]) >= 2 and all(v["ms"] > 0 for v in rep["tuner"])
    chosen = [v for v in rep["tuner"] if (v["plan"], v["occupancy"], v["skip_zero"]) ==
              (rep["plan"], rep["occupancy"], rep["skip_zero"])]
    assert chosen and chosen[0]["ms"] == min(v["ms"] for v in rep["tuner"])
    # a replay reports the same plan
    _batched(pa, stores, ds, pa.PREC_FP64, s)
    assert pa.batched_report()["graph"]
    # the three smallest molecules in full against the oracle
    order = np.argsort([c["alpha"].shape[0] for c in mols])[:3]
    for i in order:
        c = mols[i]
        Jo, Ko = oracle_mod.jk_canonical(c["centers"], c["alpha"], c["tau"], c["D"])
        assert maxabs(got[i][0], Jo) < TOL64 and maxabs(got[i][1], Ko) < TOL64, c["name"]
    for st in stores:
        st.release()


def test_batched_graph_replays_with_eager_work_between(pa, mols):
    import torch
    sub = mols[:12]
    announce(f"batched graph replays: {len(sub)} molecules")
    stores = _stores(pa, sub, pa.STORE_FP64)
    s = torch.cuda.Stream()
    rng = np.random.default_rng(77)
    js = [torch.empty((c["D"].shape[0],) + c["D"].shape[1:], dtype=torch.float64, device="cuda:0")
          for c in sub]
    ks = [torch.empty_like(j) for j in js]
    ds = [dev(c["D"]) for c in sub]
    for rep in range(5):
        # new density values in place (same pointers) on even replays, new
        # tensors (new pointers) on odd ones
        if rep % 2 == 0:
            for d in ds:
                d.copy_(torch.from_numpy(rng.standard_normal(tuple(d.shape)) / 40.0).to(d.device))
        else:
            ds = [d.clone() for d in ds]
        torch.cuda.synchronize()
        pa.fock_build_batched(stores, ds, js, ks, stream=s)
        # eager work on the same stream between replays
        with torch.cuda.stream(s):
            junk = torch.randn(512, 512, device="cuda:0", dtype=torch.float64)
            junk = junk @ junk
        s.synchronize()
        ref = _single(pa, stores, ds, pa.PREC_FP64, s)
        for i, (jr, kr) in enumerate(ref):
            assert np.array_equal(host(js[i]), jr), f"replay {rep} molecule {i} J"
            assert np.array_equal(host(ks[i]), kr), f"replay {rep} molecule {i} K"
        announce(f"replay {rep} ok")
    for st in stores:
        st.release()


def test_batched_plan_cache_and_release(pa, mols):
    import torch
    a, b = mols[:5], mols[5:9]
    announce("plan cache: alternating batches, release of a member")
    sa = _stores(pa, a, pa.STORE_FP64)
    sb = _stores(pa, b, pa.STORE_FP64)
    s = torch.cuda.Stream()
    da = [dev(c["D"]) for c in a]
    db = [dev(c["D"]) for c in b]
    ra0 = _single(pa, sa, da, pa.PREC_FP64, s)
    rb0 = _single(pa, sb, db, pa.PREC_FP64, s)
    # a plan's first build tunes it, which may cut every member's work items
    # anew: the same products summed in another order
    ga = _batched(pa, sa, da, pa.PREC_FP64, s)
    gb = _batched(pa, sb, db, pa.PREC_FP64, s)
    for x, y in zip(ga + gb, ra0 + rb0):
        sc = max(np.abs(y[0]).max(), np.abs(y[1]).max())
        assert maxabs(x[0], y[0]) <= 1e-13 * sc and maxabs(x[1], y[1]) <= 1e-13 * sc
    # from then on single builds (on the cuts the plans chose) and every
    # replay of either cached plan agree bitwise
    ra = _single(pa, sa, da, pa.PREC_FP64, s)
    rb = _single(pa, sb, db, pa.PREC_FP64, s)
    for _ in range(3):
        ga = _batched(pa, sa, da, pa.PREC_FP64, s)
        gb = _batched(pa, sb, db, pa.PREC_FP64, s)
        for x, y in zip(ga + gb, ra + rb):
            assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])
    # a different subset (a new plan) after releasing a member of batch a:
    # its members' cuts were chosen already, so it keeps them
    sa[0].release()
    ga = _batched(pa, sa[1:], da[1:], pa.PREC_FP64, s)
    for x, y in zip(ga, ra[1:]):
        assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])
    # the default (NULL) stream runs without a graph, and says so
    torch.cuda.synchronize()
    js = [torch.empty_like(d) for d in db]
    ks = [torch.empty_like(d) for d in db]
    pa.fock_build_batched(sb, db, js, ks)
    torch.cuda.synchronize()
    assert not pa.batched_report()["graph"]
    for i, (jr, kr) in enumerate(rb):
        assert np.array_equal(host(js[i]), jr) and np.array_equal(host(ks[i]), kr)
    for st in sa[1:] + sb:
        st.release()


@pytest.mark.parametrize("prec_name", ["mixed", "store32"])
def test_batched_fp32_storage_equals_single(pa, mols, prec_name):
    import torch
    prec = pa.PREC_MIXED if prec_name == "mixed" else pa.PREC_STORE32
    sub = mols[:16]
    announce(f"batched {prec_name}: {len(sub)} molecules")
    stores = _stores(pa, sub, pa.STORE_FP32)
    s = torch.cuda.Stream()
    ds = [dev(c["D"]) for c in sub]
    ref = _single(pa, stores, ds, prec, s)
    got = _batched(pa, stores, ds, prec, s)
    for i, ((jr, kr), (jg, kg)) in enumerate(zip(ref, got)):
        assert np.array_equal(jr, jg) and np.array_equal(kr, kg), f"molecule {i}"
    for st in stores:
        st.release()


def test_batched_rejects_bad_member_before_enqueue(pa, mols):
    import torch
    sub = mols[:3]
    stores = _stores(pa, sub, pa.STORE_FP64)
    ds = [dev(c["D"]) for c in sub]
    js = [torch.full_like(d, 7.0) for d in ds]
    ks = [torch.full_like(d, 7.0) for d in ds]
    ks[2] = js[2]  # aliasing outputs of the last molecule
    torch.cuda.synchronize()
    with pytest.raises(pa.InvalidArgument, match="molecule 2"):
        pa.fock_build_batched(stores, ds, js, ks)
    torch.cuda.synchronize()
    for j in js[:2] + ks[:2]:
        assert bool((j == 7.0).all()), "outputs were written although the call failed"
    # STORE32 over FP64 storage is refused the same way
    with pytest.raises(pa.InvalidArgument):
        pa.fock_build_batched(stores, ds, [torch.empty_like(d) for d in ds],
                              [torch.empty_like(d) for d in ds], prec=pa.PREC_STORE32)
    for st in stores:
        st.release()
