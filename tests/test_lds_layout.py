"""The LDS layout of a block in the contraction kernels: the bank functions
of csrc/fock_mfma.hip (translated from the source) make every matrix-core
fragment read of the six views free of bank conflicts for the lane groups
they are designed for (16 lanes of 8-byte elements, 32 lanes of 4-byte
ones), and map each aligned group of positions onto itself."""
import os
import re
from collections import Counter

import pytest

pytestmark = pytest.mark.cpu

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2002_00322_amd", "csrc",
                   "fock_mfma.hip")


def _swizzle(f32):
    """The kernel's Swz<F32>::pos as a Python function, translated from the
    source text (its statements are C integer expressions on i, j, k, l)."""
    text = open(SRC).read()
    body = text.split("struct Swz<%s> {" % ("true" if f32 else "false"), 1)[1].split("\n};", 1)[0]
    bits = int(re.search(r"kBits = (\d+)", body).group(1))
    stmts = body.split("{", 1)[1].rsplit("}", 1)[0]
    lines = []
    for st in stmts.split(";"):
        st = st.strip()
        if not st:
            continue
        st = re.sub(r"^int ", "", st)
        st = re.sub(r"\(([^()]*)\) \? (\d+) : (\d+)", r"(\2 if (\1) else \3)", st)
        st = st.replace("return ", "_out = ")
        lines.append(st)
    code = "\n".join(lines)

    def pos(i, j, k, l):
        env = {"i": i, "j": j, "k": k, "l": l}
        exec(code, {}, env)
        return env["_out"]
    return pos, bits


def _views(P):
    # lane l of wave w reads A[l % 16][l / 16] of step S: rows (x1, x2) of row
    # tile w, reduction index 4 S + l / 16 = (y1, y2)
    for vis in (0, 1):
        for which in (0, 1, 2):
            for w in range(4):
                for S in range(16):
                    out = []
                    for lane in range(64):
                        fr, fk = lane & 15, lane >> 4
                        x1, x2 = (16 * w + fr) >> 3, fr & 7
                        y1, y2 = S >> 1, 4 * (S & 1) + fk
                        if vis == 0:
                            t = [(x1, y1, x2, y2), (y1, x1, x2, y2), (x1, x2, y1, y2)][which]
                        else:
                            t = [(x1, y1, y2, x2), (y1, x1, y2, x2), (y1, y2, x1, x2)][which]
                        out.append(P(*t))
                    yield (vis, which, w, S), out


@pytest.mark.parametrize("f32", [False, True])
def test_bank_function_is_a_bijection_per_group(f32):
    pos, bits = _swizzle(f32)
    assert bits == (5 if f32 else 4)
    allpos = [pos(i, j, k, l) for i in range(8) for j in range(8) for k in range(8) for l in range(8)]
    assert sorted(allpos) == list(range(4096))
    for n, p in enumerate(allpos):
        assert p >> bits == n >> bits


@pytest.mark.parametrize("f32", [False, True])
def test_fragment_reads_are_free_of_bank_conflicts(f32):
    # 8-byte elements: each 16 lanes over 16 bank pairs; 4-byte elements: 32
    # lanes over 32 banks
    pos, bits = _swizzle(f32)
    groups = [(32, 32)] if f32 else [(16, 16)]
    for key, addr in _views(pos):
        for size, slots in groups:
            for g0 in range(0, 64, size):
                c = Counter(a % slots for a in addr[g0:g0 + size])
                assert max(c.values()) == 1, (f32, key, size)


def test_granule_stores_are_free_of_bank_conflicts():
    # 8-byte layout: the lanes of 16 consecutive granules store the same
    # element u of their granules (zero-fill, integral-direct evaluation)
    pos, bits = _swizzle(False)
    for w in range(4):
        for u in range(16):
            addr = [pos(g >> 5, (g >> 2) & 7, 2 * (g & 3) + (u >> 3), u & 7)
                    for g in range(64 * w, 64 * w + 64)]
            for g0 in range(0, 64, 16):
                assert len({a % 16 for a in addr[g0:g0 + 16]}) == 16, (w, u)


def _expr(pattern):
    """A C integer expression of the kernel source, as a Python function of
    the names it uses (>>, <<, &, +, * read the same in both languages)."""
    text = open(SRC).read()
    m = re.search(pattern, text)
    assert m, pattern
    return m.group(1)


def test_narrow_j_operand_interleave_matches_the_4x4x4_reads():
    # The operand prep stores column c of a narrow (8-column) J tile row at
    # 2 (c % 4) + c / 4; lane l of step S reads two adjacent values there as
    # the B operands of the two 4x4x4 products: they must be columns l % 4
    # and 4 + l % 4 of reduction row 4 S + l / 16 (the row its A operand
    # holds), and the two products' outputs must cover the 16x8 J tile of a
    # row tile once (lane l holds rows 4 ((l / 4) % 4) + l / 16, columns l % 4
    # and 4 + l % 4)
    perm = _expr(r"jw == 8 \? (2 \* \(c & 3\) \+ \(c >> 2\)) : c")
    read = _expr(r"f\.bj = \*\(const d2\*\)\(sBJ \+ (32 \* S \+ 8 \* \(lane >> 4\) \+ 2 \* \(lane & 3\))\)")
    store_row = _expr(r"\(16 \* rt \+ (4 \* \(\(lane >> 2\) & 3\) \+ \(lane >> 4\))\) \* 8 \+ \(lane & 3\)")
    where = {}
    for k in range(64):
        for c in range(8):
            where[8 * k + eval(perm, {"c": c})] = (k, c)
    assert sorted(where) == list(range(512))
    for S in range(16):
        for lane in range(64):
            x = eval(read, {"S": S, "lane": lane})
            assert x % 2 == 0   # 16-byte aligned pair
            assert where[x] == (4 * S + (lane >> 4), lane & 3)
            assert where[x + 1] == (4 * S + (lane >> 4), 4 + (lane & 3))
    cover = Counter()
    for lane in range(64):
        r = eval(store_row, {"lane": lane})
        cover[(r, lane & 3)] += 1
        cover[(r, 4 + (lane & 3))] += 1
    assert sorted(cover) == [(r, c) for r in range(16) for c in range(8)] and set(cover.values()) == {1}


def test_narrow_k_operand_interleave_matches_the_4x4x4_reads():
    # A narrow K column set (kq > 0) has its X tile rows written with column
    # cx = 4 (c % 4) + c / 4 at position c (an involution); lane l of step S
    # reads kq adjacent values from kb = 64 S + 16 (l / 16) + 4 (l % 4): value
    # h must be column 4h + l % 4 of reduction row 4 S + l / 16
    cx = _expr(r"const int cx = u\.kq > 0 \? (4 \* \(c & 3\) \+ \(c >> 2\)) : c;")
    read = _expr(r"const int kb = (64 \* S \+ 16 \* \(lane >> 4\) \+ 4 \* \(lane & 3\));")
    col = {c: eval(cx, {"c": c}) for c in range(16)}
    assert sorted(col.values()) == list(range(16))
    assert all(col[col[c]] == c for c in range(16))   # an involution
    for S in range(16):
        for lane in range(64):
            x = eval(read, {"S": S, "lane": lane})
            assert x % 2 == 0
            for h in range(2):
                k, pos = divmod(x + h, 16)
                assert (k, col[pos]) == (4 * S + (lane >> 4), 4 * h + (lane & 3))
