"""The device Boys function's grid table and method, on the CPU.

The device evaluates G(T) = (2/sqrt(pi)) F0(T) for 0 <= T <= 36 by the
tabulated Taylor expansion of McMurchie and Davidson about the nearest grid
point T_g = g / 16, from a table of G_7(T_g) and (2/sqrt(pi)) exp(-T_g) and the
downward recursion (csrc/eri_device.h, boys_g).  Here:
- the committed header is what its generator writes;
- the table's first entry is its closed form (F_n(0) = 1 / (2n + 1));
- the tabulated F_7 matches the oracle's F_n series at every grid point;
- the method, restated in float64 with the device's operation order, matches
  the oracle's F0 (erf and its series) to 1e-15 relative over [0, 36];
- the second table (F_15, for the Cartesian integrals' F_0 .. F_8, csrc/kernels.hip,
  boys_fn8) likewise: closed form at 0, the oracle's series at every grid
  point, and the restated method against the oracle's F_0 .. F_8.
"""
import importlib.util
import math
import os

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.cpu

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2002_00322_amd", "csrc")


def _gen():
    spec = importlib.util.spec_from_file_location("boys_table_gen", os.path.join(CSRC, "boys_table_gen.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.fixture(scope="module")
def gen():
    return _gen()


@pytest.fixture(scope="module")
def tab(gen):
    return np.array(gen.table())


def test_committed_header_is_the_generated_one(gen):
    with open(os.path.join(CSRC, "boys_table.h")) as f:
        assert f.read() == gen.header_text()


def test_first_entry_is_the_closed_form(gen, tab):
    c = 2.0 / math.sqrt(math.pi)
    assert gen.ORDER == 7 and gen.PER_UNIT == 16 and tab.shape == (36 * 16 + 1, 2)
    assert tab[0, 1] == c
    assert abs(tab[0, 0] - c / 15.0) <= 1e-16 * tab[0, 0]


def test_tabulated_f7_matches_the_oracle_series(tab):
    c = 2.0 / math.sqrt(math.pi)
    for g in range(tab.shape[0]):
        T = g / 16.0
        f = oracle.boys_fn(7, T)
        assert abs(tab[g, 0] / c - f[7]) <= 2e-15 * f[7], g
        assert abs(tab[g, 1] / c - math.exp(-T)) <= 5e-16 * math.exp(-T), g


def _device_method(tab, T):
    """boys_g of csrc/eri_device.h, element-wise in float64, same order of
    operations."""
    g = np.rint(np.minimum(T, 36.0) * 16.0)
    Tg = g * (1.0 / 16.0)
    x = Tg - T
    e = tab[g.astype(np.int64)]
    ex = e[:, 1]
    t2 = 2.0 * Tg
    gk = e[:, 0].copy()
    s = gk.copy()
    for k in range(6, -1, -1):
        gk = (t2 * gk + ex) * (1.0 / (2 * k + 1))
        s = gk + (x * (1.0 / (k + 1))) * s
    return s


def test_method_matches_oracle_f0(tab):
    c = 2.0 / math.sqrt(math.pi)
    rng = np.random.default_rng(20)
    grid = np.arange(577) / 16.0
    T = np.concatenate([rng.uniform(0.0, 36.0, 40000), rng.uniform(0.0, 0.02, 4000),
                        grid, np.minimum(grid + 1.0 / 32.0 - 1e-13, 36.0), [0.0, 1e-300, 1e-9, 36.0]])
    ref = np.array([c * oracle.boys_f0(t) for t in T])
    got = _device_method(tab, T)
    rel = np.abs(got - ref) / ref
    assert rel.max() < 1e-15, (rel.max(), T[rel.argmax()])


def test_method_meets_the_point_charge_limit_at_36(tab):
    # above T = 36 the device takes G(T) = 1 / sqrt(T) (erf(6) is 1.0 in
    # float64); the table form meets it there
    g36 = _device_method(tab, np.array([36.0]))[0]
    assert abs(g36 - 1.0 / 6.0) <= 2e-16


def test_restated_method_is_the_device_source():
    # the statements _device_method restates, as they stand in boys_g
    with open(os.path.join(CSRC, "eri_device.h")) as f:
        src = f.read()
    for stmt in ("const double g = rint(fmin(T, 36.0) * kBoysPerUnit);",
                 "const double Tg = g * (1.0 / kBoysPerUnit);",
                 "const double x = Tg - T;",
                 "const double t2 = 2.0 * Tg;",
                 "for (int k = kBoysOrder - 1; k >= 0; --k) {",
                 "gk = (t2 * gk + ex) * (1.0 / (2 * k + 1));",
                 "s = gk + (x * (1.0 / (k + 1))) * s;",
                 "const double g = T > 36.0 ? rsqrt(d2) : gt;"):
        assert stmt in src, stmt


@pytest.fixture(scope="module")
def tab_high(gen):
    return np.array(gen.table_high())


def test_high_table_first_entry_and_series(gen, tab_high):
    assert gen.ORDER_HIGH == 15 and tab_high.shape == (36 * 16 + 1, 2)
    assert tab_high[0, 1] == 1.0 and abs(tab_high[0, 0] - 1.0 / 31.0) <= 1e-16 / 31.0
    for g in range(tab_high.shape[0]):
        T = g / 16.0
        f = oracle.boys_fn(15, T)
        assert abs(tab_high[g, 0] - f[15]) <= 2e-15 * f[15], g
        assert abs(tab_high[g, 1] - math.exp(-T)) <= 2e-16 * math.exp(-T), g


def _device_fn8(tab_high, T):
    """boys_fn8 of csrc/kernels.hip for one T, float64, same order of
    operations."""
    F = [0.0] * 9
    et = math.exp(-T)
    if T <= 36.0:
        g = float(np.rint(T * 16.0))
        Tg = g * (1.0 / 16.0)
        x = Tg - T
        e0, e1 = tab_high[int(g)]
        t2 = 2.0 * Tg
        f = [0.0] * 8
        f[7] = e0
        for k in range(14, 7, -1):
            f[k - 8] = (t2 * f[k - 7] + e1) * (1.0 / (2 * k + 1))
        s = f[7]
        for j in range(6, -1, -1):
            s = f[j] + (x * (1.0 / (j + 1))) * s
        F[8] = s
        t2x = 2.0 * T
        for n in range(7, -1, -1):
            F[n] = (t2x * F[n + 1] + et) * (1.0 / (2 * n + 1))
    else:
        F[0] = 0.5 * math.sqrt(math.pi / T)
        for n in range(8):
            F[n + 1] = ((2 * n + 1) * F[n] - et) / (2.0 * T)
    return np.array(F)


def test_cartesian_method_matches_oracle_fn(tab_high):
    rng = np.random.default_rng(21)
    Ts = np.concatenate([rng.uniform(0.0, 36.0, 4000), rng.uniform(0.0, 0.02, 400), np.arange(577) / 16.0,
                         [0.0, 1e-300, 36.0, 36.001, 40.0, 200.0, 1e5]])
    worst = 0.0
    for T in Ts:
        ref = oracle.boys_fn(8, T)
        worst = max(worst, float(np.max(np.abs(_device_fn8(tab_high, T) - ref) / ref)))
    assert worst < 5e-15, worst


def test_restated_cartesian_method_is_the_device_source():
    with open(os.path.join(CSRC, "kernels.hip")) as f:
        src = f.read()
    for stmt in ("if (T <= 36.0) {",
                 "const double g = rint(T * kBoysPerUnit);",
                 "f[7] = e[0];",
                 "for (int k = 14; k >= 8; --k) f[k - 8] = (t2 * f[k - 7] + e[1]) * (1.0 / (2 * k + 1));",
                 "for (int j = 6; j >= 0; --j) s = f[j] + (x * (1.0 / (j + 1))) * s;",
                 "for (int n = 7; n >= 0; --n) F[n] = (t2x * F[n + 1] + et) * (1.0 / (2 * n + 1));",
                 "F[0] = 0.5 * sqrt(kPi / T);",
                 "for (int n = 0; n < 8; ++n) F[n + 1] = ((double)(2 * n + 1) * F[n] - et) / (2.0 * T);"):
        assert stmt in src, stmt
