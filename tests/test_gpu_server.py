"""Serving loop (esmf_server_*) through the C ABI.

Every request's result must equal, bitwise, the same build done alone with
esmf_fock_build (the grouped launch runs the same kernels with the same fixed
reduction order), whatever group or stream it ran in.  Admission is checked
against the exact store footprints the server reports.
"""
import numpy as np
import pytest

import workloads as wl
from gpu_util import announce, dev, host

pytestmark = pytest.mark.gpu

WS = 2 << 30   # workspace arena of the test servers


@pytest.fixture(scope="module")
def pa():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2002_00322_amd as pa
    return pa


def _sessions():
    """Small sessions of the serving mix: chains and a two-layer slab."""
    out = []
    for i, nc in enumerate([25, 60, 110]):
        c, a = wl.chain(nc)
        out.append(dict(name=f"chain{2 * nc}", centers=c, alpha=a, tau=1e-10, m=[4, 8, 4][i]))
    c, a = wl.slab(3, 10, 2, seed=611)
    out.append(dict(name="slab120", centers=c, alpha=a, tau=1e-10, m=8))
    c, a = wl.random_box(37, seed=612)
    out.append(dict(name="box37", centers=c, alpha=a, tau=0.0, m=11))
    return out


def _density(s, it):
    n = s["alpha"].shape[0]
    return wl.transition_densities(n, s["m"], min(40, n // 2), 7000 + n, 9000 + 131 * it)


def _alone(pa, s, d, prec):
    import torch
    st = pa.EriStore(s["centers"], s["alpha"], s["tau"],
                     storage=pa.STORE_FP64 if prec == pa.PREC_FP64 else pa.STORE_FP32)
    j, k = pa.fock_build(st, d, prec=prec)
    torch.cuda.synchronize()
    out = host(j), host(k)
    st.release()
    return out


@pytest.mark.parametrize("prec_name", ["fp64", "mixed", "store32"])
def test_server_results_equal_builds_alone(pa, prec_name):
    import torch
    prec = {"fp64": pa.PREC_FP64, "mixed": pa.PREC_MIXED, "store32": pa.PREC_STORE32}[prec_name]
    sess = _sessions()
    announce(f"server {prec_name}: {len(sess)} sessions x 3 iterations")
    srv = pa.Server(prec=prec, nstreams=3, max_group=8, max_inflight=2, workspace_limit_bytes=WS)
    ids = [srv.open_session(s["centers"], s["alpha"], s["tau"])[0] for s in sess]
    reqs = []
    for it in range(3):
        for s, sid in zip(sess, ids):
            d = dev(_density(s, it))
            j = torch.empty_like(d)
            k = torch.empty_like(d)
            torch.cuda.synchronize()
            reqs.append((s, it, d, j, k, srv.submit(sid, d, j, k)))
    lats = [srv.wait(r[-1]) for r in reqs]
    assert all(x > 0 for x in lats)
    st = srv.stats()
    assert st["requests_completed"] == len(reqs) and st["sessions_open"] == len(sess)
    for s, it, d, j, k, _ in reqs:
        jr, kr = _alone(pa, s, d, prec)
        assert np.array_equal(host(j), jr), f"{s['name']} iteration {it} J"
        assert np.array_equal(host(k), kr), f"{s['name']} iteration {it} K"
    for sid in ids:
        srv.close_session(sid)
    assert srv.stats()["resident_bytes"] == 0
    srv.destroy()


def test_server_groups_pending_requests(pa):
    import torch
    sess = _sessions()[:3]
    announce("server grouping: one stream, one group in flight, a burst of requests")
    srv = pa.Server(nstreams=1, max_group=16, max_inflight=1, workspace_limit_bytes=WS)
    ids = [srv.open_session(s["centers"], s["alpha"], s["tau"])[0] for s in sess]
    held = []
    for it in range(4):
        for s, sid in zip(sess, ids):
            d = dev(_density(s, it))
            held.append((s, d, torch.empty_like(d), torch.empty_like(d)))
    torch.cuda.synchronize()
    rids = [srv.submit(sid, d, j, k) for (s, d, j, k), sid in zip(held, ids * 4)]
    for r in rids:
        srv.wait(r)
    st = srv.stats()
    assert st["groups_launched"] < len(rids) and st["max_group_size"] >= 2, st
    for s, d, j, k in held[:3]:
        jr, kr = _alone(pa, s, d, pa.PREC_FP64)
        assert np.array_equal(host(j), jr) and np.array_equal(host(k), kr)
    srv.destroy()


def test_server_admission_by_footprint(pa):
    import torch
    small, big = _sessions()[0], _sessions()[3]
    probe = pa.Server(workspace_limit_bytes=WS)
    _, fp_small = probe.open_session(small["centers"], small["alpha"], small["tau"])
    _, fp_big = probe.open_session(big["centers"], big["alpha"], big["tau"])
    probe.destroy()
    assert 0 < fp_small < fp_big
    announce(f"admission: footprints {fp_small} / {fp_big} bytes")
    srv = pa.Server(hbm_budget_bytes=fp_big + fp_small // 2, workspace_limit_bytes=WS)
    s1, _ = srv.open_session(small["centers"], small["alpha"], small["tau"])
    with pytest.raises(pa.OutOfMemory) as e:
        srv.open_session(big["centers"], big["alpha"], big["tau"])
    assert e.value.footprint == fp_big          # fits the budget, not what is left of it
    assert srv.stats()["sessions_rejected"] == 1
    # a session whose store alone exceeds the budget is refused for good
    tiny = pa.Server(hbm_budget_bytes=fp_small - 1, workspace_limit_bytes=WS)
    with pytest.raises(pa.OutOfMemory) as e2:
        tiny.open_session(small["centers"], small["alpha"], small["tau"])
    assert e2.value.footprint == fp_small
    tiny.destroy()
    # a request in flight holds the session; closing waits for it
    d = dev(_density(small, 0))
    j, k = torch.empty_like(d), torch.empty_like(d)
    torch.cuda.synchronize()
    r = srv.submit(s1, d, j, k)
    srv.close_session(s1)
    srv.wait(r)
    assert srv.stats()["resident_bytes"] == 0
    s2, fp = srv.open_session(big["centers"], big["alpha"], big["tau"])
    assert fp == fp_big and srv.stats()["resident_bytes"] == fp_big
    srv.close_session(s2)
    srv.destroy()


def test_server_argument_errors(pa):
    import torch
    s = _sessions()[0]
    srv = pa.Server(workspace_limit_bytes=WS)
    sid, _ = srv.open_session(s["centers"], s["alpha"], s["tau"])
    n = s["alpha"].shape[0]
    d = torch.zeros((2, n, n), dtype=torch.float64, device="cuda:0")
    with pytest.raises(pa.InvalidArgument):
        srv.submit(sid + 100, d, torch.empty_like(d), torch.empty_like(d))
    j = torch.empty_like(d)
    with pytest.raises(pa.InvalidArgument):
        srv.submit(sid, d, j, j)
    with pytest.raises(pa.InvalidArgument):
        srv.wait(123456)
    with pytest.raises(pa.InvalidArgument):
        srv.close_session(sid + 100)
    assert srv.stats()["requests_submitted"] == 0
    srv.destroy()


def test_server_refuses_request_larger_than_its_arena(pa):
    import torch
    s = _sessions()[3]
    srv = pa.Server(workspace_limit_bytes=1 << 20)
    sid, _ = srv.open_session(s["centers"], s["alpha"], s["tau"])
    d = dev(_density(s, 0))
    with pytest.raises(pa.OutOfMemory, match="workspace"):
        srv.submit(sid, d, torch.empty_like(d), torch.empty_like(d))
    assert srv.stats()["requests_submitted"] == 0
    srv.destroy()


def test_server_build_follows_the_producer_stream(pa):
    # the density is written on the caller's stream behind slow work and
    # submitted at once, with no host synchronisation: the build must read
    # the written density (the server's streams wait for the producer event)
    import torch
    s = _sessions()[3]
    srv = pa.Server(nstreams=2, max_group=4, max_inflight=2, workspace_limit_bytes=WS)
    sid, _ = srv.open_session(s["centers"], s["alpha"], s["tau"])
    src = dev(_density(s, 5))
    d = torch.full_like(src, float("nan"))
    j, k = torch.empty_like(d), torch.empty_like(d)
    junk = torch.randn(4096, 4096, device="cuda:0", dtype=torch.float64)
    torch.cuda.synchronize()
    announce("server producer stream: density written behind six 4096^2 FP64 products, submitted without a sync")
    prod = torch.cuda.Stream()
    with torch.cuda.stream(prod):
        for _ in range(6):
            junk = junk @ junk * 1e-3
        d.copy_(src)
        r = srv.submit(sid, d, j, k)      # stream=None: the current stream, prod
    srv.wait(r)
    torch.cuda.synchronize()
    jr, kr = _alone(pa, s, src, pa.PREC_FP64)
    assert np.array_equal(host(j), jr) and np.array_equal(host(k), kr)
    srv.destroy()
