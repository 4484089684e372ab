"""CPU checks of the host planner (csrc/plan.cpp), built with g++ under
AddressSanitizer and UndefinedBehaviorSanitizer and driven by
tests/native/plan_check.cpp, from the oracle's Schwarz factors.

What is checked, exactly (integers and powers of two, no tolerance):
- the block list with its degeneracy weights covers Eq. J_and_K: every
  ordered quartet (ab|cd) of functions with Q_ab Q_cd > tau receives total
  weight 1 over the 8 index permutations that every stored slot applies
  (the updates of Sec. "Shell-Pair Screening"'s grouped loop), and no other
  quartet receives any;
- each work plan (two visits per block, or fused) visits every block once per
  visit kind, in the documented order, in items of the bra's blocks;
- every partial slot belongs to the target its accumulator writes, is
  written by exactly one accumulator, and the slot ranges leave no slot
  unwritten (the reduction sums every slot of a target);
- the operand-tile and reduction lists contain what the blocks read and
  the targets that receive partials.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.cpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2002_00322_amd", "csrc")
TILE = 8


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("plan") / "plan_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", CSRC, os.path.join(ROOT, "tests", "native", "plan_check.cpp"),
           os.path.join(CSRC, "plan.cpp"), "-o", exe]
    subprocess.check_call(cmd)
    return exe


def _run(driver, tmp_path, centers, alpha, q, tau, kind, seg, band, xcd=8):
    n = alpha.shape[0]
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(fin, "wb") as f:
        np.array([n, kind, seg, band, xcd], dtype=np.int32).tofile(f)
        np.array([tau], dtype=np.float64).tofile(f)
        np.ascontiguousarray(centers, dtype=np.float64).tofile(f)
        np.ascontiguousarray(alpha, dtype=np.float64).tofile(f)
        np.ascontiguousarray(q, dtype=np.float64).tofile(f)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([driver, str(fin), str(fout)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    raw = open(fout, "rb").read()
    pos = 0
    out = {}

    def take(dtype):
        nonlocal pos
        cnt = int(np.frombuffer(raw, np.int64, 1, pos)[0])
        pos += 8
        a = np.frombuffer(raw, dtype, cnt, pos).copy()
        pos += cnt * np.dtype(dtype).itemsize
        return a
    for name, dt in (("slot_fn", np.int32), ("bt", np.int32), ("weight", np.float64), ("entries", np.int32),
                     ("items", np.int32), ("eslot", np.int32), ("kptr", np.int64), ("jptr", np.int64),
                     ("used", np.int32), ("red", np.int32)):
        out[name] = take(dt)
    out["nkslots"], out["njslots"] = (int(x) for x in np.frombuffer(raw, np.int64, 2, pos))
    out["rc"] = int(np.frombuffer(raw, np.int32, 1, pos + 16)[0])
    out["bt"] = out["bt"].reshape(-1, 4)
    out["items"] = out["items"].reshape(-1, 8)
    out["eslot"] = out["eslot"].reshape(-1, 6)
    return out


def _cases():
    c1 = wl.config1()
    A, al = wl.chain(30)
    Bc, Ba = wl.slab(3, 3, 2, seed=5)
    Rc, Ra = wl.random_box(29, seed=17, box=6.0)
    return [("box40 tau 0", c1["centers"], c1["alpha"], 0.0),
            ("chain60 tau 1e-10", A, al, 1e-10),
            ("slab36 tau 1e-6", Bc, Ba, 1e-6),
            ("box29 tau 1e-3", Rc, Ra, 1e-3)]


def _check_blocks(p, q, tau, n):
    """Total weight per ordered function quartet over the 8 permutations
    applied by every stored slot, against the screen."""
    slot_fn, bt, w = p["slot_fn"], p["bt"], p["weight"]
    assert np.all(np.isin(w, [1.0, 0.5, 0.25, 0.125]))
    W = np.zeros((n, n, n, n))
    idx = np.arange(TILE)
    for (I, J, K, L), wb in zip(bt, w):
        a = slot_fn[I * TILE + idx]
        b = slot_fn[J * TILE + idx]
        c = slot_fn[K * TILE + idx]
        d = slot_fn[L * TILE + idx]
        A, B, C, D = np.meshgrid(a, b, c, d, indexing="ij")
        keep = (A >= 0) & (B >= 0) & (C >= 0) & (D >= 0)
        A, B, C, D = A[keep], B[keep], C[keep], D[keep]
        # the screen inside a block: a slot holds its integral iff Q_ab Q_cd > tau
        kept = q[A, B] * q[C, D] > tau
        A, B, C, D = A[kept], B[kept], C[kept], D[kept]
        for (x, y, z, t) in ((A, B, C, D), (B, A, C, D), (A, B, D, C), (B, A, D, C),
                             (C, D, A, B), (D, C, A, B), (C, D, B, A), (D, C, B, A)):
            np.add.at(W, (x, y, z, t), wb)
    want = (q[:, :, None, None] * q[None, None, :, :] > tau).astype(float)
    assert np.array_equal(W, want), np.argwhere(W != want)[:5]
    # canonical order: I >= J, K >= L, (IJ) >= (KL), bra-major then (K, L)
    tp = lambda X, Y: X * (X + 1) // 2 + Y  # noqa: E731
    assert np.all(bt[:, 0] >= bt[:, 1]) and np.all(bt[:, 2] >= bt[:, 3])
    assert np.all(tp(bt[:, 0], bt[:, 1]) >= tp(bt[:, 2], bt[:, 3]))
    key = tp(bt[:, 0], bt[:, 1]).astype(np.int64) << 32 | tp(bt[:, 2], bt[:, 3])
    assert np.all(np.diff(key) > 0)


def _check_plan(p, kind, seg, band):
    bt, items, es, entries = p["bt"], p["items"], p["eslot"], p["entries"]
    nb = bt.shape[0]
    T = len(p["slot_fn"]) // TILE
    assert p["rc"] == 0
    # items partition the entries; two-visit: every block once per visit
    spans = sorted((int(it[0]), int(it[1])) for it in items)
    assert spans[0][0] == 0 and spans[-1][1] == len(entries)
    assert all(a[1] == b[0] for a, b in zip(spans[:-1], spans[1:]))
    visits = [0, 1] if kind == 0 else [2]
    for v in visits:
        seen = np.concatenate([entries[it[0]:it[1]] for it in items if it[4] == v] or [np.zeros(0, np.int32)])
        assert np.array_equal(np.sort(seen), np.arange(nb)), f"visit {v}"
    slot_owner_k = {}
    slot_owner_j = {}

    def own(d, slot, inst, tgt, ptr):
        assert ptr[tgt] <= slot < ptr[tgt + 1], (slot, tgt)
        if slot in d:
            assert d[slot] == inst, (slot, d[slot], inst)
        d[slot] = inst
    for ii, it in enumerate(items):
        e0, e1, I, J, visit, _, jslot0, _ = (int(x) for x in it)
        blk = entries[e0:e1]
        assert e1 > e0 and np.all(bt[blk, 0] == I) and np.all(bt[blk, 1] == J)
        K, L = bt[blk, 2], bt[blk, 3]
        if visit == 0:
            order = np.lexsort((L, K))
        elif visit == 1:
            order = np.lexsort((K, L))
        else:
            order = np.lexsort((L, K))
            assert len(set(L.tolist())) <= band
        assert np.array_equal(order, np.arange(len(blk))), f"item {ii} order"
        key = L if visit == 1 else K
        runs = np.concatenate([[0], np.nonzero(np.diff(key))[0] + 1, [len(blk)]])
        if visit == 2:
            assert len(blk) <= seg or len(runs) == 2   # longer only as one K-run
        else:
            assert len(blk) <= seg
        if visit != 1:
            own(slot_owner_j, jslot0, ("J_IJ", ii), I * T + J, p["jptr"])
        else:
            assert jslot0 == -1
        for r0, r1 in zip(runs[:-1], runs[1:]):
            ka = es[e0 + r0:e0 + r1, 0]
            kb = es[e0 + r0:e0 + r1, 1]
            assert np.all(ka == ka[0]) and np.all(kb == kb[0])
            own(slot_owner_k, int(ka[0]), ("Ka", ii, r0), I * T + int(key[r0]), p["kptr"])
            own(slot_owner_k, int(kb[0]), ("Kb", ii, r0), J * T + int(key[r0]), p["kptr"])
        for x in range(len(blk)):
            row = es[e0 + x]
            if visit == 0:
                assert row[2] == -1
            else:
                own(slot_owner_j, int(row[2]), ("J_KL", e0 + x), int(K[x]) * T + int(L[x]), p["jptr"])
            if visit == 2:
                bpos = int(row[5])
                assert 0 <= bpos < band
                own(slot_owner_k, int(row[3]), ("La", ii, bpos), I * T + int(L[x]), p["kptr"])
                own(slot_owner_k, int(row[4]), ("Lb", ii, bpos), J * T + int(L[x]), p["kptr"])
            else:
                assert row[3] == -1 and row[4] == -1
        if visit == 2:
            # one band position per distinct L, in order of first occurrence
            firsts = []
            for x in range(len(blk)):
                if int(L[x]) not in firsts:
                    firsts.append(int(L[x]))
                assert int(es[e0 + x, 5]) == firsts.index(int(L[x]))
    # every slot written by exactly one accumulator, none left unwritten
    assert sorted(slot_owner_k) == list(range(p["nkslots"]))
    assert sorted(slot_owner_j) == list(range(p["njslots"]))
    assert p["kptr"][-1] == p["nkslots"] and p["jptr"][-1] == p["njslots"]
    # operand tiles read and reduction pairs
    used = set()
    for I, J, K, L in bt:
        used |= {J * T + L, I * T + L, J * T + K, I * T + K, K * T + L, I * T + J}
    assert np.array_equal(p["used"], np.array(sorted(used), dtype=np.int32))
    red = []
    for X in range(T):
        for Y in range(X + 1):
            xy, yx = X * T + Y, Y * T + X
            if (p["kptr"][xy + 1] > p["kptr"][xy] or p["kptr"][yx + 1] > p["kptr"][yx]
                    or p["jptr"][xy + 1] > p["jptr"][xy]):
                red.append(xy)
    assert np.array_equal(p["red"], np.array(red, dtype=np.int32))


@pytest.mark.parametrize("case", range(4))
@pytest.mark.parametrize("kind,seg,band", [(0, 64, 0), (0, 3, 0), (1, 64, 4), (1, 5, 4), (1, 2, 2), (1, 1000, 1)])
def test_plan_covers_every_screened_quartet(driver, tmp_path, oracle_mod, case, kind, seg, band):
    name, centers, alpha, tau = _cases()[case]
    n = alpha.shape[0]
    q = oracle_mod.schwarz(centers, alpha)
    p = _run(driver, tmp_path, centers, alpha, q, tau, kind, seg, band)
    # the tile plan holds every function once, ghosts padding tiles
    sf = p["slot_fn"]
    assert len(sf) % TILE == 0 and np.array_equal(np.sort(sf[sf >= 0]), np.arange(n))
    _check_blocks(p, q, tau, n)
    _check_plan(p, kind, seg, band)


def test_plan_drops_everything_above_every_bound(driver, tmp_path, oracle_mod):
    A, al = wl.chain(10)
    q = oracle_mod.schwarz(A, al)
    p = _run(driver, tmp_path, A, al, q, 1e6, 1, 64, 4)
    assert p["bt"].shape[0] == 0 and p["items"].shape[0] == 0 and p["nkslots"] == 0 and p["rc"] == 0


def test_oracle_under_sanitizers(tmp_path):
    # the oracle's C, built with AddressSanitizer and UndefinedBehaviorSanitizer
    # (OpenMP on), runs every routine once on small inputs
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_check")
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp", "-ffp-contract=off",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           os.path.join(ROOT, "tests", "native", "oracle_check.c"),
                           os.path.join(ROOT, "oracle", "esmf_oracle.c"), "-lm", "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", OMP_NUM_THREADS="4")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    assert "max |literal - grouped|" in r.stdout
