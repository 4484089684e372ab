"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Nothing here re-types the oracle's formulas: the integral is checked against a
numerical quadrature of an independently derived representation, closed forms
and limits; the contraction bookkeeping against the literal definition
(Eq. J_and_K) summed by numpy over the full tensor; and the J/K results against
the structure the definition implies (symmetries, bilinearity, energy
derivatives, the paper's worked Theta-derivative and its HF limit).
"""
import math

import numpy as np
import pytest
from scipy import integrate

import workloads as wl

pytestmark = pytest.mark.cpu


def _quad_boys(T):
    v, _ = integrate.quad(lambda u: math.exp(-T * u * u), 0.0, 1.0, epsabs=0, epsrel=1.2e-14,
                          limit=200)
    return v


@pytest.mark.parametrize("T", [0.0, 1e-14, 1e-6, 3e-3, 9.999e-3, 1e-2, 0.3, 1.0, 7.5, 30.0,
                               60.0, 400.0])
def test_boys_f0_against_quadrature(oracle_mod, T):
    # F0(T) = int_0^1 exp(-T u^2) du by definition
    assert abs(oracle_mod.boys_f0(T) - _quad_boys(T)) <= 5e-15 * max(1.0, _quad_boys(T))


def test_boys_branches_meet(oracle_mod):
    # the series branch (T < 1e-2) and the erf branch meet at the switch: the jump
    # across it equals the slope dF0/dT = -int_0^1 u^2 exp(-T u^2) du times the step
    T0, d = 1e-2, 1e-12
    a = oracle_mod.boys_f0(T0 - d)
    b = oracle_mod.boys_f0(T0)
    f1, _ = integrate.quad(lambda u: u * u * math.exp(-T0 * u * u), 0.0, 1.0)
    assert abs((a - b) - d * f1) < 2e-16


def _norm(a):
    return (2 * a / math.pi) ** 0.75


def _eri_by_quadrature(A, al, p, q, r, s):
    """(pq|rs) from 1/r12 = (2/sqrt(pi)) int_0^inf exp(-t^2 r12^2) dt: the
    Gaussian integrals over r1, r2 done analytically for each t, the t-integral
    numerically. Independent of the Boys-function closed form."""
    def prod(i, j):
        z = al[i] + al[j]
        P = (al[i] * A[i] + al[j] * A[j]) / z
        E = _norm(al[i]) * _norm(al[j]) * math.exp(-al[i] * al[j] / z * np.sum((A[i] - A[j]) ** 2))
        return z, P, E
    z, P, E1 = prod(p, q)
    e, Q, E2 = prod(r, s)
    R2 = float(np.sum((P - Q) ** 2))

    def f(t):
        den = z * e + t * t * (z + e)
        return (math.pi ** 2 / den) ** 1.5 * math.exp(-z * e * t * t * R2 / den)
    v, _ = integrate.quad(f, 0.0, np.inf, epsabs=0, epsrel=1e-13, limit=400)
    return E1 * E2 * 2.0 / math.sqrt(math.pi) * v


def test_eri_against_quadrature(oracle_mod):
    A, al = wl.random_box(12, seed=7)
    rng = np.random.default_rng(3)
    for _ in range(40):
        p, q, r, s = (int(x) for x in rng.integers(0, 12, 4))
        ref = _eri_by_quadrature(A, al, p, q, r, s)
        got = oracle_mod.eri(A, al, p, q, r, s)
        assert abs(got - ref) <= 1e-11 * abs(ref) + 1e-300, (p, q, r, s, got, ref)


def test_eri_single_centre_closed_form(oracle_mod):
    # one normalised s function: (aa|aa) = 2 sqrt(alpha/pi)
    for a in [0.1, 0.3, 1.5, 10.0]:
        A = np.zeros((1, 3))
        al = np.array([a])
        assert abs(oracle_mod.eri(A, al, 0, 0, 0, 0) - 2 * math.sqrt(a / math.pi)) < 1e-15 * 4


def test_eri_point_charge_limit(oracle_mod):
    # far apart charge distributions interact as point charges:
    # (pq|rs) = S_pq S_rs / |P - Q|, S_pq = E_pq (pi/zeta)^(3/2); exact in FP64 once
    # erfc(sqrt(T)) < 1e-17 (T > 40)
    A = np.array([[0.0, 0, 0], [0.5, 0, 0], [60.0, 1, 0], [60.3, 1.2, 0]])
    al = np.array([1.2, 0.8, 2.0, 0.9])

    def S(i, j):
        z = al[i] + al[j]
        E = _norm(al[i]) * _norm(al[j]) * math.exp(-al[i] * al[j] / z * np.sum((A[i] - A[j]) ** 2))
        return E * (math.pi / z) ** 1.5, (al[i] * A[i] + al[j] * A[j]) / z
    s1, P = S(0, 1)
    s2, Q = S(2, 3)
    ref = s1 * s2 / math.sqrt(np.sum((P - Q) ** 2))
    got = oracle_mod.eri(A, al, 0, 1, 2, 3)
    assert abs(got - ref) <= 1e-14 * abs(ref)


def test_eri_eightfold_symmetry_bitwise(oracle_mod):
    A, al = wl.random_box(9, seed=11)
    T = oracle_mod.eri_tensor(A, al, 0.0)
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1), (3, 2, 1, 0)]:
        assert np.array_equal(T, T.transpose(perm))


def test_schwarz_bound_holds(oracle_mod):
    A, al = wl.random_box(12, seed=5)
    T = oracle_mod.eri_tensor(A, al, 0.0)
    Q = oracle_mod.schwarz(A, al)
    bound = Q[:, :, None, None] * Q[None, None, :, :]
    assert np.all(np.abs(T) <= bound * (1 + 1e-14))
    assert np.allclose(np.sqrt(np.einsum("pqpq->pq", T)), Q, rtol=0, atol=0)


def _literal_numpy(T, D):
    # Eq. J_and_K written out: J[D]_pq = sum_rs D_rs (rs|pq); K[D]_pq = sum_rs D_rs (pr|qs)
    J = np.einsum("rs,rspq->pq", D, T)
    K = np.einsum("rs,prqs->pq", D, T)
    return J, K


def _tau_dropping(Q, frac):
    prod = np.sort((Q[:, :, None, None] * Q[None, None]).ravel())
    return float(prod[int(frac * len(prod))])


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("drop", [0.0, 0.3])
def test_canonical_loop_equals_brute_force(oracle_mod, seed, drop):
    A, al = wl.random_box(14, seed=seed)
    Q = oracle_mod.schwarz(A, al)
    tau = 0.0 if drop == 0.0 else _tau_dropping(Q, drop)
    T = oracle_mod.eri_tensor(A, al, tau)
    D = wl.random_densities(14, 3, seed=seed + 50, scale=1.0)
    J, K = oracle_mod.jk_canonical(A, al, tau, D)
    for i in range(3):
        Jr, Kr = _literal_numpy(T, D[i])
        assert np.max(np.abs(J[i] - Jr)) < 1e-13 * max(1, np.abs(Jr).max())
        assert np.max(np.abs(K[i] - Kr)) < 1e-13 * max(1, np.abs(Kr).max())


def test_k_orientation_is_discriminated(oracle_mod):
    # the swapped reading K[D^T] differs from K[D] for non-symmetric D, so the
    # brute-force test above fixes the orientation of Eq. J_and_K
    A, al = wl.random_box(10, seed=4)
    T = oracle_mod.eri_tensor(A, al, 0.0)
    D = wl.random_densities(10, 1, seed=9, scale=1.0)[0]
    _, K = oracle_mod.jk_canonical(A, al, 0.0, D)
    _, Kr = _literal_numpy(T, D)
    _, Kt = _literal_numpy(T, D.T.copy())
    assert np.max(np.abs(K[0] - Kr)) < 1e-13
    assert np.max(np.abs(Kr - Kt)) > 1e-3


def test_literal_c_equals_canonical_config1(oracle_mod):
    c = wl.config1()
    J1, K1 = oracle_mod.jk_literal(c["centers"], c["alpha"], c["tau"], c["D"])
    J2, K2 = oracle_mod.jk_canonical(c["centers"], c["alpha"], c["tau"], c["D"])
    assert np.max(np.abs(J1 - J2)) < 1e-13
    assert np.max(np.abs(K1 - K2)) < 1e-13


def test_literal_c_equals_canonical_screened(oracle_mod):
    A, al = wl.chain(12)
    D = wl.random_densities(24, 2, seed=77, scale=0.1)
    for tau in [1e-10, 1e-4]:
        J1, K1 = oracle_mod.jk_literal(A, al, tau, D)
        J2, K2 = oracle_mod.jk_canonical(A, al, tau, D)
        assert np.max(np.abs(J1 - J2)) < 1e-14
        assert np.max(np.abs(K1 - K2)) < 1e-14


def test_entries_equal_full_build(oracle_mod):
    A, al = wl.chain(30)
    D = wl.transition_densities(60, 3, 10, 5, 6)
    J, K = oracle_mod.jk_canonical(A, al, 1e-10, D)
    rng = np.random.default_rng(0)
    i = rng.integers(0, 3, 50)
    p = rng.integers(0, 60, 50)
    q = rng.integers(0, 60, 50)
    Je, Ke = oracle_mod.jk_entries(A, al, 1e-10, D, i, p, q)
    assert np.max(np.abs(Je - J[i, p, q])) < 1e-15
    assert np.max(np.abs(Ke - K[i, p, q])) < 1e-15


def test_quartet_count_matches_independent_count(oracle_mod):
    c = wl.config2()
    Q = oracle_mod.schwarz(c["centers"], c["alpha"])
    iu = np.tril_indices(Q.shape[0])
    qp = np.sort(Q[iu])
    tau = c["tau"]
    # unordered pairs {a, b} (a == b allowed) with qa*qb > tau, by sorted search
    with np.errstate(divide="ignore"):
        idx = np.searchsorted(qp, tau / qp, side="right")
    ordered = int((len(qp) - idx).sum())
    diag = int((qp * qp > tau).sum())
    npairs, nq = oracle_mod.count(c["centers"], c["alpha"], tau)
    assert nq == (ordered + diag) // 2
    assert npairs == int((Q[iu] * Q.max() > tau).sum())


@pytest.fixture(scope="module")
def box_jk(oracle_mod):
    c = wl.config1()
    A, al = c["centers"], c["alpha"]
    D = c["D"]
    J, K = oracle_mod.jk_canonical(A, al, 0.0, D)
    return A, al, D, J, K


def test_jk_structure(oracle_mod, box_jk):
    A, al, D, J, K = box_jk
    Jt, Kt = oracle_mod.jk_canonical(A, al, 0.0, np.ascontiguousarray(D.transpose(0, 2, 1)))
    for i in range(D.shape[0]):
        assert np.max(np.abs(J[i] - J[i].T)) < 1e-14            # J symmetric
        assert np.max(np.abs(J[i] - Jt[i])) < 1e-14             # J[D] = J[D^T]
        assert np.max(np.abs(K[i].T - Kt[i])) < 1e-14           # K[D]^T = K[D^T]
    S = D[0] + D[0].T
    _, Ks = oracle_mod.jk_canonical(A, al, 0.0, S)
    assert np.max(np.abs(Ks[0] - Ks[0].T)) < 1e-14              # K symmetric for symmetric D


def test_jk_linear_and_bilinear(oracle_mod, box_jk):
    A, al, D, J, K = box_jk
    comb = 0.7 * D[0] - 1.3 * D[1]
    Jc, Kc = oracle_mod.jk_canonical(A, al, 0.0, comb)
    assert np.max(np.abs(Jc[0] - (0.7 * J[0] - 1.3 * J[1]))) < 1e-14
    assert np.max(np.abs(Kc[0] - (0.7 * K[0] - 1.3 * K[1]))) < 1e-14
    # D1 . J[D2] = D2 . J[D1] and D1 . K[D2] = D2 . K[D1]
    assert abs(np.sum(D[0] * J[1]) - np.sum(D[1] * J[0])) < 1e-13
    assert abs(np.sum(D[0] * K[1]) - np.sum(D[1] * K[0])) < 1e-13


def test_energy_derivatives_by_finite_difference(oracle_mod):
    # E_J(D) = 1/2 sum D_ab (ab|cd) D_cd, E_K(D) = 1/2 sum D_bd (ab|cd) D_ac are
    # quadratic; their gradients are J[D] and K[D] for any D, and a central
    # difference of a quadratic is exact for every step.
    A, al = wl.random_box(12, seed=21)
    T = oracle_mod.eri_tensor(A, al, 0.0)
    rng = np.random.default_rng(8)
    D = rng.standard_normal((12, 12))
    Dl = rng.standard_normal((12, 12))

    def EJ(X):
        return 0.5 * np.einsum("ab,abcd,cd->", X, T, X)

    def EK(X):
        return 0.5 * np.einsum("bd,abcd,ac->", X, T, X)
    J, K = oracle_mod.jk_canonical(A, al, 0.0, D)
    for h in [1.0, 0.1]:
        gj = (EJ(D + h * Dl) - EJ(D - h * Dl)) / (2 * h)
        gk = (EK(D + h * Dl) - EK(D - h * Dl)) / (2 * h)
        assert abs(gj - np.sum(Dl * J[0])) < 1e-12 * max(1, abs(gj))
        assert abs(gk - np.sum(Dl * K[0])) < 1e-12 * max(1, abs(gk))


def _fock(oracle_mod, A, al, tau, X):
    J, K = oracle_mod.jk_canonical(A, al, tau, X)
    return 2 * J[0] - K[0]


def test_paper_theta_derivative(oracle_mod):
    # Appendix, Eq. eng2_der_theta_kp4 (N2 factored out):
    #   d/dTheta_kp ( F[Theta^T Theta] . Theta^T Theta ) = 4 (Theta F[Theta^T Theta])_kp
    A, al = wl.random_box(10, seed=31)
    rng = np.random.default_rng(12)
    Th = rng.standard_normal((3, 10)) * 0.5

    def f(X):
        P = X.T @ X
        return np.sum(_fock(oracle_mod, A, al, 0.0, P) * P)
    G = 4 * Th @ _fock(oracle_mod, A, al, 0.0, Th.T @ Th)
    h = 1e-4
    for (k, p) in [(0, 0), (1, 4), (2, 9), (0, 7)]:
        E = np.zeros_like(Th)
        E[k, p] = h
        # 4-point central difference (error O(h^4))
        fd = (-f(Th + 2 * E) + 8 * f(Th + E) - 8 * f(Th - E) + f(Th - 2 * E)) / (12 * h)
        assert abs(fd - G[k, p]) < 1e-8 * max(1, abs(G[k, p])), (k, p, fd, G[k, p])


def test_hf_limit_energy(oracle_mod):
    # Eq. esmf_eng_hf: with sigma = 0 and U = I the two-electron energy is
    # F[P] . P, P = C_occ C_occ^T; it equals sum_abcd (2 P_ab P_cd - P_ac P_bd)(ab|cd)
    A, al = wl.random_box(12, seed=41)
    T = oracle_mod.eri_tensor(A, al, 0.0)
    C = wl.orthonormal(12, 3)
    P = C[:, :4] @ C[:, :4].T
    e2 = np.sum(_fock(oracle_mod, A, al, 0.0, P) * P)
    ref = 2 * np.einsum("ab,abcd,cd->", P, T, P) - np.einsum("ac,abcd,bd->", P, T, P)
    assert abs(e2 - ref) < 1e-12 * abs(ref)


def test_positivity(oracle_mod, box_jk):
    A, al, D, J, K = box_jk
    for i in range(D.shape[0]):
        assert np.sum(D[i] * J[i]) >= 0          # Coulomb metric is positive semidefinite
    C = wl.orthonormal(40, 9)
    P = C[:, :10] @ C[:, :10].T
    _, Kp = oracle_mod.jk_canonical(A, al, 0.0, P)
    assert np.sum(P * Kp[0]) >= 0


def test_screening_error_bound(oracle_mod):
    # dropping a quartet changes an entry by |D_cd (ab|cd)| <= |D_cd| Q_ab Q_cd <= tau |D_cd|
    A, al = wl.chain(60)
    D = wl.transition_densities(120, 2, 20, 71, 72)
    J0, K0 = oracle_mod.jk_canonical(A, al, 0.0, D)
    for tau in [1e-10, 1e-6, 1e-3]:
        Jt, Kt = oracle_mod.jk_canonical(A, al, tau, D)
        for i in range(2):
            b = tau * np.abs(D[i]).sum()
            assert np.max(np.abs(Jt[i] - J0[i])) <= b * (1 + 1e-9) + 1e-15
            assert np.max(np.abs(Kt[i] - K0[i])) <= b * (1 + 1e-9) + 1e-15
    # and the largest threshold does drop something
    assert np.max(np.abs(Jt - J0)) > 0


def test_golden_box40_entries(oracle_mod):
    # stored by tests/golden/make_golden.py (oracle only); guards the oracle
    # against unintended changes of its arithmetic
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "box40_entries.txt")
    rows = np.loadtxt(path)
    c = wl.config1()
    i, p, q = (rows[:, k].astype(int) for k in range(3))
    J, K = oracle_mod.jk_entries(c["centers"], c["alpha"], c["tau"], c["D"], i, p, q)
    assert np.max(np.abs(J - rows[:, 3])) < 1e-15
    assert np.max(np.abs(K - rows[:, 4])) < 1e-15
