"""Integral-direct builds (ESMF_STORE_DIRECT) through the C ABI.

A direct handle stores no integrals: every build recomputes each kept
integral inside the contraction from the resident pair data, with the same
formula and screen as the store fill.  Its results are held to the FP64 oracle
(1e-10, as every FP64 build) and to the stored FP64 build of the same molecule
(the same integrals and the same contraction order, so they agree to rounding
of the integrals: 1e-14 relative to the largest entry).
"""
import numpy as np
import pytest

import workloads as wl
from gpu_util import announce, check_tune_report, dev, host, maxabs

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


@pytest.fixture(scope="module")
def pa():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2002_00322_amd as pa
    return pa


def _pair(pa, c, prec=0):
    import torch
    out = []
    for storage in (pa.STORE_FP64, pa.STORE_DIRECT):
        st = pa.EriStore(c["centers"], c["alpha"], c["tau"], storage=storage)
        j, k = pa.fock_build(st, dev(c["D"]), prec=prec)
        torch.cuda.synchronize()
        out.append((st, host(j), host(k)))
    return out


def _cases():
    yield "box40", wl.config1()
    yield "chain400", wl.config2()
    for n, m, tau, seed in [(1, 1, 0.0, 3), (2, 2, 0.0, 4), (13, 3, 1e-10, 5), (37, 11, 1e-6, 6),
                            (64, 1, 1e-10, 7)]:
        A, al = wl.random_box(n, seed=seed, box=6.0)
        D = wl.random_densities(n, m, seed=seed + 100, scale=0.1)
        yield f"edge{n}", dict(centers=A, alpha=al, tau=tau, D=D)
    # unit-exponent s functions at distances sqrt(T) from the first, T over
    # the Boys function's grid table and beyond 36 (its point-charge form)
    Ts = np.array([0.0, 1e-6, 0.03125, 0.0625, 1.0, 5.0, 17.96875, 35.96875, 36.0, 36.001, 40.0, 100.0])
    A = np.zeros((Ts.size + 1, 3))
    A[1:, 0] = np.sqrt(Ts)
    yield "boysrange", dict(centers=A, alpha=np.ones(Ts.size + 1), tau=0.0,
                            D=wl.random_densities(Ts.size + 1, 3, seed=77, scale=0.1))


@pytest.mark.parametrize("name", [n for n, _ in _cases()])
def test_direct_equals_stored_and_oracle(pa, oracle_mod, name):
    c = dict(_cases())[name]
    announce(f"direct vs stored FP64: {name}")
    (s0, J0, K0), (s1, J1, K1) = _pair(pa, c)
    scale = max(1.0, np.max(np.abs(J0)), np.max(np.abs(K0)))
    dj, dk = maxabs(J1, J0), maxabs(K1, K0)
    announce(f"{name}: direct - stored max|dJ|={dj:.3e} max|dK|={dk:.3e} "
             f"bitwise={np.array_equal(J0, J1) and np.array_equal(K0, K1)}")
    assert dj <= 1e-14 * scale and dk <= 1e-14 * scale
    Jr, Kr = oracle_mod.jk_canonical(c["centers"], c["alpha"], c["tau"], c["D"])
    assert maxabs(J1, Jr) < TOL64 and maxabs(K1, Kr) < TOL64
    i0, i1 = s0.info(), s1.info()
    assert i1["storage"] == pa.STORE_DIRECT and i1["nelements_stored"] == 0
    assert i1["nquartets_kept"] == i0["nquartets_kept"] and i1["nblocks"] == i0["nblocks"]
    s0.release()
    s1.release()


@pytest.mark.parametrize("plan", ["0", "1"])
def test_direct_equals_stored_bitwise_on_one_plan(pa, monkeypatch, plan):
    # with the same work plan (two visits, or fused) for both handles the
    # direct build sums the same products in the same order as the stored
    # one: the integrals are the stored values, bit for bit
    import torch
    monkeypatch.setenv("ESMF_PLAN", plan)
    c = wl.config2()
    announce(f"direct vs stored FP64, work plan {plan}: chain400")
    s0 = pa.EriStore(c["centers"], c["alpha"], c["tau"])
    s1 = pa.EriStore(c["centers"], c["alpha"], c["tau"], storage=pa.STORE_DIRECT)
    d = dev(c["D"])
    j0, k0 = pa.fock_build(s0, d)
    j1, k1 = pa.fock_build(s1, d)
    torch.cuda.synchronize()
    assert torch.equal(j0, j1) and torch.equal(k0, k1)
    s0.release()
    s1.release()


def test_direct_handle_rules(pa):
    import torch
    c = wl.config2()
    announce("direct handle: lookup, precisions, tuner, footprint")
    st = pa.EriStore(c["centers"], c["alpha"], c["tau"], storage=pa.STORE_DIRECT)
    stored = pa.EriStore(c["centers"], c["alpha"], c["tau"])
    # no integrals are held: the footprint is the pair data and the plan
    assert st.info()["device_bytes"] < stored.info()["device_bytes"]
    with pytest.raises(pa.NotSupported):
        st.lookup(np.zeros(1, np.int32), np.zeros(1, np.int32), np.zeros(1, np.int32),
                  np.zeros(1, np.int32))
    d = dev(c["D"])
    for prec in (pa.PREC_MIXED, pa.PREC_STORE32):
        with pytest.raises(pa.InvalidArgument):
            pa.fock_build(st, d, prec=prec)
    j0, k0 = pa.fock_build(st, d)
    torch.cuda.synchronize()
    rep = pa.fock_tune(st, d.shape[0])
    check_tune_report(rep, 4)
    j1, k1 = pa.fock_build(st, d)
    torch.cuda.synchronize()
    # the tuner may change the work plan: the same products in another order
    scale = float(max(j0.abs().max(), k0.abs().max()))
    assert maxabs(host(j0), host(j1)) <= 1e-13 * scale and maxabs(host(k0), host(k1)) <= 1e-13 * scale
    st.release()
    stored.release()


def test_direct_screening_drops_everything(pa):
    import torch
    announce("direct: tau above every bound")
    A, al = wl.chain(10)
    D = wl.random_densities(20, 2, seed=1)
    st = pa.EriStore(A, al, 1e6, storage=pa.STORE_DIRECT)
    assert st.info()["nblocks"] == 0
    j, k = pa.fock_build(st, dev(D))
    torch.cuda.synchronize()
    assert np.all(host(j) == 0) and np.all(host(k) == 0)
    st.release()


def test_direct_batched_equals_single(pa):
    import torch
    mols = wl.batch_workload()[:10]
    announce(f"direct batched: {len(mols)} molecules")
    stores = [pa.EriStore(c["centers"], c["alpha"], c["tau"], storage=pa.STORE_DIRECT) for c in mols]
    s = torch.cuda.Stream()
    ds = [dev(c["D"]) for c in mols]
    with torch.cuda.stream(s):
        ref = [pa.fock_build(st, d, stream=s) for st, d in zip(stores, ds)]
        js = [torch.full_like(d, float("nan")) for d in ds]
        ks = [torch.full_like(d, float("nan")) for d in ds]
    s.synchronize()
    pa.fock_build_batched(stores, ds, js, ks, stream=s)
    s.synchronize()
    for i, ((jr, kr), j, k) in enumerate(zip(ref, js, ks)):
        assert np.array_equal(host(j), host(jr)) and np.array_equal(host(k), host(kr)), f"molecule {i}"
    # direct and stored handles do not mix in one batch
    mixed = stores[:2] + [pa.EriStore(mols[2]["centers"], mols[2]["alpha"], mols[2]["tau"])]
    with pytest.raises(pa.InvalidArgument, match="molecule 2"):
        pa.fock_build_batched(mixed, ds[:3], [torch.empty_like(d) for d in ds[:3]],
                              [torch.empty_like(d) for d in ds[:3]])
    mixed[2].release()
    for st in stores:
        st.release()


def test_direct_server_equals_builds_alone(pa):
    import torch
    sess = []
    for nc, m in [(25, 4), (60, 8)]:
        c, a = wl.chain(nc)
        sess.append(dict(centers=c, alpha=a, tau=1e-10, m=m))
    announce("direct server: 2 sessions x 2 iterations")
    srv = pa.Server(nstreams=2, max_group=4, workspace_limit_bytes=1 << 30, storage=pa.STORE_DIRECT)
    ids = [srv.open_session(s["centers"], s["alpha"], s["tau"])[0] for s in sess]
    reqs = []
    for it in range(2):
        for s, sid in zip(sess, ids):
            n = s["alpha"].shape[0]
            d = dev(wl.transition_densities(n, s["m"], min(40, n // 2), 7000 + n, 9000 + 131 * it))
            j, k = torch.empty_like(d), torch.empty_like(d)
            torch.cuda.synchronize()
            reqs.append((s, d, j, k, srv.submit(sid, d, j, k)))
    for r in reqs:
        srv.wait(r[-1])
    for s, d, j, k, _ in reqs:
        st = pa.EriStore(s["centers"], s["alpha"], s["tau"], storage=pa.STORE_DIRECT)
        jr, kr = pa.fock_build(st, d)
        torch.cuda.synchronize()
        assert np.array_equal(host(j), host(jr)) and np.array_equal(host(k), host(kr))
        st.release()
    srv.destroy()


@pytest.mark.timeout(900)
def test_direct_where_the_store_does_not_fit(pa, oracle_mod):
    # the 10x10x5 slab: its FP64 store and the workspace of a stored build
    # together exceed the device (both read from the integral-direct handle's
    # info: the block list and plans are those a stored handle would have),
    # so only the integral-direct handle can build it.  That handle holds the
    # pair data and plans; its build is held to the oracle on sampled entries
    # (near-diagonal ones, where J and K are largest, and random ones)
    import torch
    c = wl.config3_deep()
    torch.cuda.empty_cache()
    announce("slab10x10x5 integral-direct: prepare")
    st = pa.EriStore(c["centers"], c["alpha"], c["tau"], storage=pa.STORE_DIRECT)
    info = st.info()
    free, total = torch.cuda.mem_get_info()
    m = c["D"].shape[0]
    outputs = 3 * 8 * m * 1000 * 1000
    stored_need = info["fp64_store_bytes"] + info["workspace_bytes_plan"][0] + outputs
    need = info["workspace_bytes"] + outputs
    announce(f"slab10x10x5: {info['nquartets_kept']} quartets in {info['nblocks']} blocks; FP64 store "
             f"{info['fp64_store_bytes'] / 1e9:.1f} GB + stored-build workspace "
             f"{info['workspace_bytes_plan'][0] / 1e9:.1f} GB against {total / 1e9:.1f} GB of device; "
             f"direct handle {info['device_bytes'] / 1e9:.2f} GB, workspace {info['workspace_bytes'] / 1e9:.1f} GB, "
             f"free {free / 1e9:.1f} GB")
    assert info["nelements_stored"] == 0 and info["fp64_store_bytes"] > 8 * info["nquartets_kept"]
    assert stored_need > total and info["device_bytes"] < 0.05 * info["fp64_store_bytes"]
    assert need < free, "the direct build of this slab must fit in the device's free memory"
    d = dev(c["D"])
    j, k = pa.fock_build(st, d)
    torch.cuda.synchronize()
    J, K = host(j), host(k)
    rng = np.random.default_rng(55)
    cnt = 48
    i = rng.integers(0, 8, cnt)
    p = rng.integers(0, 1000, cnt)
    q = np.where(np.arange(cnt) < cnt // 2, np.clip(p + rng.integers(-3, 4, cnt), 0, 999), rng.integers(0, 1000, cnt))
    Jr, Kr = oracle_mod.jk_entries(c["centers"], c["alpha"], c["tau"], c["D"], i, p, q)
    ej, ek = np.max(np.abs(J[i, p, q] - Jr)), np.max(np.abs(K[i, p, q] - Kr))
    announce(f"slab10x10x5 direct: sampled max|dJ|={ej:.3e} max|dK|={ek:.3e} (|K| up to {np.abs(Kr).max():.3e})")
    assert ej < TOL64 and ek < TOL64
    assert maxabs(J, J.transpose(0, 2, 1)) < 1e-13
    del j, k, d
    st.release()
