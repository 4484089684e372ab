"""Stores over Cartesian s, p and d functions (esmf_eri_prepare_cart).

The contraction is the same as for s functions; what is new is the integral
fill (McMurchie-Davidson on the GPU) and the Schwarz factors it screens
with.  Stored integrals are held to the oracle's Cartesian integrals
(1e-12 relative to the largest), builds to the oracle's J and K (1e-10, as
every FP64 build), FP32 stores to FP32 rounding.
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


CASES = {
    "spd_box3": lambda: wl.spd_box(3, seed=7, box=3.0),        # 42 functions
    "spd_chain5": lambda: wl.spd_chain(5),                     # 70 functions, ragged tiles
    "p_only": lambda: wl.cart_basis(np.random.default_rng(3).uniform(0, 4, (4, 3)), ((1, 0.7),)),
    "d_only": lambda: wl.cart_basis(np.random.default_rng(4).uniform(0, 4, (3, 3)), ((2, 0.5), (2, 1.7))),
    # p and d shells of exponent 1 on a line: (aa|bb) of same-site pairs has
    # T = |A - B|^2 = 0, 0.5, 4, 17.97, 35.9, 60 (the F_n grid table and the
    # form beyond 36), mixed pairs everything between
    "pd_line": lambda: wl.cart_basis([[x, 0.0, 0.0] for x in np.sqrt([0.0, 0.5, 4.0, 17.96875, 35.9, 60.0])],
                                     ((1, 1.0), (2, 1.0))),
}


@pytest.mark.parametrize("name", list(CASES))
def test_stored_cartesian_integrals_match_oracle(pa, oracle_mod, name):
    A, al, L = CASES[name]()
    n = al.shape[0]
    announce(f"Cartesian store {name}: N={n}")
    st = pa.EriStore(A, al, 0.0, lmn=L)
    rng = np.random.default_rng(11)
    idx = rng.integers(0, n, (400, 4))
    got = st.lookup(idx[:, 0], idx[:, 1], idx[:, 2], idx[:, 3])
    ref = np.array([oracle_mod.eri(A, al, *q, lmn=L) for q in idx])
    scale = np.max(np.abs(ref))
    err = np.max(np.abs(got - ref))
    announce(f"{name}: max |d(pq|rs)| = {err:.3e} (largest {scale:.3e})")
    assert err <= 1e-12 * scale
    Q = oracle_mod.schwarz(A, al, lmn=L)
    assert abs(st.info()["q_max"] - np.max(Q)) <= 1e-12 * np.max(Q)
    st.release()


@pytest.mark.parametrize("name,tau", [("spd_box3", 0.0), ("spd_chain5", 1e-10), ("p_only", 1e-8),
                                      ("d_only", 0.0), ("pd_line", 0.0)])
def test_cartesian_build_matches_oracle(pa, oracle_mod, name, tau):
    import torch
    A, al, L = CASES[name]()
    n = al.shape[0]
    D = wl.random_densities(n, 3, seed=n, scale=1.0 / n)
    announce(f"Cartesian build {name}: N={n} m=3 tau={tau}")
    st = pa.EriStore(A, al, tau, lmn=L)
    j, k = pa.fock_build(st, dev(D))
    torch.cuda.synchronize()
    Jr, Kr = oracle_mod.jk_canonical(A, al, tau, D, lmn=L)
    dj, dk = maxabs(host(j), Jr), maxabs(host(k), Kr)
    announce(f"{name}: max|dJ|={dj:.3e} max|dK|={dk:.3e}")
    assert dj < TOL64 and dk < TOL64
    nq = oracle_mod.count(A, al, tau, lmn=L)[1]
    assert st.info()["nquartets_kept"] == nq
    st.release()


def test_cartesian_chain_sampled(pa, oracle_mod):
    # 20 sites, 280 functions: sampled entries of J and K by the definition
    import torch
    A, al, L = wl.spd_chain(20)
    n = al.shape[0]
    D = wl.random_densities(n, 4, seed=5, scale=1.0 / n)
    announce(f"Cartesian chain: N={n} m=4, sampled")
    st = pa.EriStore(A, al, 1e-10, lmn=L)
    j, k = pa.fock_build(st, dev(D))
    torch.cuda.synchronize()
    rng = np.random.default_rng(2)
    cnt = 24
    i, p, q = rng.integers(0, 4, cnt), rng.integers(0, n, cnt), rng.integers(0, n, cnt)
    Jr, Kr = oracle_mod.jk_entries(A, al, 1e-10, D, i, p, q, lmn=L)
    J, K = host(j), host(k)
    assert np.max(np.abs(J[i, p, q] - Jr)) < TOL64 and np.max(np.abs(K[i, p, q] - Kr)) < TOL64
    st.release()


def test_cartesian_fp32_store_and_batched(pa, oracle_mod):
    # STORE32 on the same molecule: FP64 arithmetic on the FP32-rounded
    # integrals, bounded by their rounding; a batched build with an s-only
    # and a Cartesian molecule equals the single builds bitwise
    import torch
    A, al, L = wl.spd_box(3, seed=7, box=3.0)
    n = al.shape[0]
    D = wl.random_densities(n, 2, seed=9, scale=1.0 / n)
    announce("Cartesian FP32 store and batched build")
    s64 = pa.EriStore(A, al, 0.0, lmn=L)
    s32 = pa.EriStore(A, al, 0.0, lmn=L, storage=pa.STORE_FP32)
    d = dev(D)
    j64, k64 = pa.fock_build(s64, d)
    j32, k32 = pa.fock_build(s32, d, prec=pa.PREC_STORE32)
    torch.cuda.synchronize()
    T = oracle_mod.eri_tensor(A, al, 0.0, lmn=L)
    # each stored integral rounds to FP32 (relative 2^-24); bound the effect
    bJ = np.einsum("rs,rspq->pq", np.abs(D[0]), np.abs(T)) * 2.0 ** -24
    assert np.all(np.abs(host(j32)[0] - host(j64)[0]) <= 8 * bJ + 1e-14)
    A2, al2 = wl.chain(30)
    D2 = wl.random_densities(60, 3, seed=3, scale=1.0 / 60)
    s2 = pa.EriStore(A2, al2, 1e-10)
    stores, ds = [s64, s2], [d, dev(D2)]
    refs = [pa.fock_build(x, y) for x, y in zip(stores, ds)]
    js = [torch.empty_like(x) for x in ds]
    ks = [torch.empty_like(x) for x in ds]
    torch.cuda.synchronize()
    # the first batched build tunes the plan (and may cut the members' work
    # items anew: the same sums in another order); after it, single and
    # batched builds agree bitwise
    pa.fock_build_batched(stores, ds, js, ks)
    torch.cuda.synchronize()
    for (jr, kr), jb, kb in zip(refs, js, ks):
        sc = float(max(jr.abs().max(), kr.abs().max()))
        assert float((jr - jb).abs().max()) <= 1e-13 * sc and float((kr - kb).abs().max()) <= 1e-13 * sc
    refs = [pa.fock_build(x, y) for x, y in zip(stores, ds)]
    pa.fock_build_batched(stores, ds, js, ks)
    torch.cuda.synchronize()
    for (jr, kr), jb, kb in zip(refs, js, ks):
        assert torch.equal(jr, jb) and torch.equal(kr, kb)
    for x in (s64, s32, s2):
        x.release()


# ---- contracted functions (esmf_eri_prepare_contracted) ---------------------

def _contracted(nsites, seed, box=3.0, shells=None):
    sites = np.random.default_rng(seed).uniform(0.0, box, (nsites, 3))
    return wl.contracted_basis(sites) if shells is None else wl.contracted_basis(sites, shells)


@pytest.mark.parametrize("nsites,seed", [(2, 1), (3, 2)])
def test_contracted_store_and_build_match_oracle(pa, oracle_mod, nsites, seed):
    import torch
    cen, L, off, pe, pc = _contracted(nsites, seed)
    n = cen.shape[0]
    basis = oracle_mod.contraction(cen, L, off, pe, pc)
    announce(f"contracted store: {nsites} sites, N={n}, {off[-1]} primitives")
    st = pa.EriStore.contracted(cen, L, off, pe, pc, 0.0)
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, n, (120, 4))
    got = st.lookup(idx[:, 0], idx[:, 1], idx[:, 2], idx[:, 3])
    ref = np.array([oracle_mod.eri_contracted(basis, *q) for q in idx])
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(got - ref)) <= 1e-12 * scale, np.max(np.abs(got - ref))
    D = wl.random_densities(n, 3, seed=seed + 40, scale=1.0 / n)
    j, k = pa.fock_build(st, dev(D))
    torch.cuda.synchronize()
    Jr, Kr = oracle_mod.jk_contracted(basis, D)
    dj, dk = maxabs(host(j), Jr), maxabs(host(k), Kr)
    announce(f"contracted build: max|dJ|={dj:.3e} max|dK|={dk:.3e}")
    assert dj < TOL64 and dk < TOL64
    st.release()


def test_contracted_length_one_equals_primitive_store(pa):
    # one primitive of coefficient 1 per function: the same integrals as the
    # primitive Cartesian store, bitwise
    import torch
    A, al, L = wl.spd_box(3, seed=7, box=3.0)
    n = al.shape[0]
    announce("contracted of length one vs primitive Cartesian store")
    s1 = pa.EriStore(A, al, 1e-10, lmn=L)
    s2 = pa.EriStore.contracted(A, L, np.arange(n + 1), al, np.ones(n), 1e-10)
    d = dev(wl.random_densities(n, 2, seed=3, scale=1.0 / n))
    j1, k1 = pa.fock_build(s1, d)
    j2, k2 = pa.fock_build(s2, d)
    torch.cuda.synchronize()
    assert torch.equal(j1, j2) and torch.equal(k1, k2)
    assert s1.info()["nquartets_kept"] == s2.info()["nquartets_kept"]
    for st in (s1, s2):
        st.release()


def test_contracted_single_s_primitives_keep_their_sign(pa, oracle_mod):
    # one s primitive per function with coefficients of either sign: each
    # normalised function is sign(c) g, so functions of negative coefficient
    # flip the sign of their integrals; the store must not take them as g
    import torch
    n = 24
    A, al = wl.random_box(n, seed=31, box=4.0)
    rng = np.random.default_rng(32)
    coef = rng.uniform(0.5, 2.0, n) * np.where(rng.random(n) < 0.5, -1.0, 1.0)
    L = np.zeros((n, 3), np.int32)
    off = np.arange(n + 1)
    basis = oracle_mod.contraction(A, L, off, al, coef)
    announce("contracted single s primitives of either sign, N=24")
    st = pa.EriStore.contracted(A, L, off, al, coef, 0.0)
    idx = rng.integers(0, n, (200, 4))
    got = st.lookup(idx[:, 0], idx[:, 1], idx[:, 2], idx[:, 3])
    ref = np.array([oracle_mod.eri_contracted(basis, *q) for q in idx])
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    D = wl.random_densities(n, 2, seed=33, scale=1.0 / n)
    j, k = pa.fock_build(st, dev(D))
    torch.cuda.synchronize()
    Jr, Kr = oracle_mod.jk_contracted(basis, D)
    assert maxabs(host(j), Jr) < TOL64 and maxabs(host(k), Kr) < TOL64
    st.release()


def test_contracted_screened_chain(pa, oracle_mod):
    # 8 sites on a line (88 functions), tau 1e-10: the screened build against
    # the unscreened oracle within the screening bound tau * sum |D|
    import torch
    sites = np.zeros((8, 3))
    sites[:, 0] = 1.4 * np.arange(8)
    cen, L, off, pe, pc = wl.contracted_basis(sites)
    n = cen.shape[0]
    basis = oracle_mod.contraction(cen, L, off, pe, pc)
    D = wl.random_densities(n, 2, seed=12, scale=1.0 / n)
    announce(f"contracted chain: N={n}, tau 1e-10")
    st = pa.EriStore.contracted(cen, L, off, pe, pc, 1e-10)
    j, k = pa.fock_build(st, dev(D))
    torch.cuda.synchronize()
    Jr, Kr = oracle_mod.jk_contracted(basis, D)
    bound = TOL64 + 1e-10 * np.sum(np.abs(D), axis=(1, 2)).max()
    assert maxabs(host(j), Jr) < bound and maxabs(host(k), Kr) < bound
    st.release()


def test_contracted_rejects_bad_arguments(pa):
    cen, L, off, pe, pc = _contracted(1, 0)
    announce("contracted: argument errors")
    bad_off = off.copy()
    bad_off[1] = bad_off[0]  # a function without primitives
    with pytest.raises(pa.InvalidArgument):
        pa.EriStore.contracted(cen, L, bad_off, pe, pc, 0.0)
    bad_e = pe.copy()
    bad_e[0] = -1.0
    with pytest.raises(pa.InvalidArgument):
        pa.EriStore.contracted(cen, L, off, bad_e, pc, 0.0)
    with pytest.raises(pa.NotSupported):
        pa.EriStore.contracted(cen, L, off, pe, pc, 0.0, storage=pa.STORE_DIRECT)


def test_server_session_over_contracted_basis(pa):
    # a serving session over a contracted basis gives the single build's
    # results, bitwise, next to an s-type session
    import torch
    sites = np.zeros((6, 3))
    sites[:, 0] = 1.4 * np.arange(6)
    cen, L, off, pe, pc = wl.contracted_basis(sites)
    n = cen.shape[0]
    A2, al2 = wl.chain(20)
    announce(f"server: contracted session N={n} with an s session N=40")
    srv = pa.Server(nstreams=2, max_group=4, workspace_limit_bytes=1 << 30)
    s1, _ = srv.open_session_contracted(cen, L, off, pe, pc, 1e-10)
    s2, _ = srv.open_session(A2, al2, 1e-10)
    d1 = dev(wl.random_densities(n, 3, seed=1, scale=1.0 / n))
    d2 = dev(wl.random_densities(40, 2, seed=2, scale=1.0 / 40))
    outs = [(torch.empty_like(d1), torch.empty_like(d1)), (torch.empty_like(d2), torch.empty_like(d2))]
    torch.cuda.synchronize()
    r1 = srv.submit(s1, d1, *outs[0])
    r2 = srv.submit(s2, d2, *outs[1])
    srv.wait(r1)
    srv.wait(r2)
    st1 = pa.EriStore.contracted(cen, L, off, pe, pc, 1e-10)
    st2 = pa.EriStore(A2, al2, 1e-10)
    ref1 = pa.fock_build(st1, d1)
    ref2 = pa.fock_build(st2, d2)
    torch.cuda.synchronize()
    for (j, k), (jr, kr) in zip(outs, (ref1, ref2)):
        assert torch.equal(j, jr) and torch.equal(k, kr)
    st1.release()
    st2.release()
    srv.destroy()


def test_cartesian_mixed_and_store32_within_1e8(pa):
    # the FP32-storage paths on an s/p/d basis with transition densities
    # (N_o = 40): within 1e-8 of the FP64 build on every J and K element
    import torch
    A, al, L = wl.spd_chain(20)
    n = al.shape[0]
    d = dev(wl.transition_densities(n, 8, 40, 811, 812))
    announce(f"Cartesian chain N={n}: MIXED and STORE32 against FP64")
    s64 = pa.EriStore(A, al, 1e-10, lmn=L)
    s32 = pa.EriStore(A, al, 1e-10, lmn=L, storage=pa.STORE_FP32)
    j64, k64 = pa.fock_build(s64, d)
    out = {}
    for name, prec in (("mixed", pa.PREC_MIXED), ("store32", pa.PREC_STORE32)):
        j, k = pa.fock_build(s32, d, prec=prec)
        torch.cuda.synchronize()
        out[name] = (float((j - j64).abs().max()), float((k - k64).abs().max()))
    announce(f"max |dJ|, |dK| vs FP64: {out}")
    for dj, dk in out.values():
        assert dj <= 1e-8 and dk <= 1e-8
    s64.release()
    s32.release()
