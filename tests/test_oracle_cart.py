"""Pins of the oracle's integrals over Cartesian s, p and d functions.

The McMurchie-Davidson integrals (oracle_eri_cart) are checked against what
holds independently of that scheme:
- F_n(T) against numerical quadrature of its defining integral;
- four s functions: the s-type closed form;
- a p function is a centre derivative of an s function,
  x_A exp(-a r_A^2) = (1/2a) d/dA_x exp(-a r_A^2), and d functions are
  second derivatives (x_A y_A: the mixed one; x_A^2: the second one plus
  1/2a times the s function), so p and d integrals equal five-point
  differences of the s closed form in the centre coordinates;
- rotating the geometry rotates the p components as a vector;
- the 8-fold index symmetry and the Schwarz bound.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import workloads as wl

pytestmark = pytest.mark.cpu


@pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")
@pytest.mark.parametrize("T", [0.0, 1e-8, 0.01, 0.7, 5.0, 20.0, 34.9, 35.1, 60.0, 300.0])
def test_boys_fn_against_quadrature(oracle_mod, T):
    F = oracle_mod.boys_fn(8, T)
    for n in range(9):
        ref, _ = integrate.quad(lambda u: u ** (2 * n) * math.exp(-T * u * u), 0.0, 1.0, epsabs=0,
                                epsrel=1.2e-14, limit=200)
        assert abs(F[n] - ref) <= 3e-14 * max(ref, 1e-300) + 1e-300, (n, T, F[n], ref)


def _four(seed):
    rng = np.random.default_rng(seed)
    A = rng.uniform(0.0, 2.5, (4, 3))
    al = np.exp(rng.uniform(np.log(0.2), np.log(3.0), 4))
    return A, al


def test_all_s_equals_closed_form(oracle_mod):
    for seed in range(5):
        A, al = _four(seed)
        L = np.zeros((4, 3), int)
        ref = oracle_mod.eri(A, al, 0, 1, 2, 3)
        got = oracle_mod.eri(A, al, 0, 1, 2, 3, lmn=L)
        assert abs(got - ref) <= 1e-14 * abs(ref)


def _s_int(oracle_mod, A, al, which, shift):
    B = A.copy()
    B[which[0]] += shift
    return oracle_mod.eri(B, al, 0, 1, 2, 3)


def _d1(f, h):
    return (-f(2 * h) + 8 * f(h) - 8 * f(-h) + f(-2 * h)) / (12 * h)


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("pos", range(4))
@pytest.mark.parametrize("xyz", range(3))
def test_p_function_is_a_centre_derivative(oracle_mod, seed, pos, xyz):
    # normalised: phi_p = sqrt(4a) x_A exp(..) N_s, so
    # (p..|..) = (1/sqrt(a)) d/dA_x (s..|..)
    A, al = _four(seed)
    L = np.zeros((4, 3), int)
    L[pos, xyz] = 1
    got = oracle_mod.eri(A, al, 0, 1, 2, 3, lmn=L)
    e = np.zeros(3)
    e[xyz] = 1.0

    def f(h):
        B = A.copy()
        B[pos] += h * e
        return oracle_mod.eri(B, al, 0, 1, 2, 3)
    ref = _d1(f, 1e-3) / math.sqrt(al[pos])
    scale = abs(oracle_mod.eri(A, al, 0, 1, 2, 3))
    assert abs(got - ref) <= 1e-9 * scale, (got, ref)


@pytest.mark.parametrize("seed", range(3))
def test_d_functions_are_second_centre_derivatives(oracle_mod, seed):
    A, al = _four(seed + 10)
    s0 = oracle_mod.eri(A, al, 0, 1, 2, 3)
    h = 2e-3
    for pos in range(4):
        a = al[pos]

        def sh(dx, dy):
            B = A.copy()
            B[pos, 0] += dx
            B[pos, 1] += dy
            return oracle_mod.eri(B, al, 0, 1, 2, 3)
        # x_A y_A: phi = 4a x_A y_A e N_s = (1/a) d2/dAx dAy (s)
        mixed = (sh(h, h) - sh(h, -h) - sh(-h, h) + sh(-h, -h)) / (4 * h * h)
        L = np.zeros((4, 3), int)
        L[pos] = [1, 1, 0]
        assert abs(oracle_mod.eri(A, al, 0, 1, 2, 3, lmn=L) - mixed / a) <= 1e-5 * abs(s0)
        # x_A^2: phi = (4a / sqrt 3) x_A^2 e N_s, x_A^2 e = (d2/dAx2 e + 2a e) / 4a^2
        second = (-sh(2 * h, 0) + 16 * sh(h, 0) - 30 * s0 + 16 * sh(-h, 0) - sh(-2 * h, 0)) / (12 * h * h)
        L[pos] = [2, 0, 0]
        ref = (second + 2 * a * s0) / (math.sqrt(3.0) * a)
        assert abs(oracle_mod.eri(A, al, 0, 1, 2, 3, lmn=L) - ref) <= 1e-5 * abs(s0)


def _rotation(seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def test_p_components_rotate_as_a_vector(oracle_mod):
    # (p_i s|p_j s) in a rotated frame = Rot_ik Rot_jl (p_k s|p_l s)
    A, al = _four(21)
    Rot = _rotation(5)
    M = np.zeros((3, 3))
    Mr = np.zeros((3, 3))
    Ar = A @ Rot.T
    for i in range(3):
        for j in range(3):
            L = np.zeros((4, 3), int)
            L[0, i] = 1
            L[2, j] = 1
            M[i, j] = oracle_mod.eri(A, al, 0, 1, 2, 3, lmn=L)
            Mr[i, j] = oracle_mod.eri(Ar, al, 0, 1, 2, 3, lmn=L)
    assert np.max(np.abs(Mr - Rot @ M @ Rot.T)) <= 1e-13 * np.max(np.abs(M))


def _shell_basis(n_centres, seed, lmax=2):
    """Centres with an s, a p and (lmax 2) a d shell of one exponent each."""
    rng = np.random.default_rng(seed)
    C = rng.uniform(0.0, 3.0, (n_centres, 3))
    comps = [[0, 0, 0]]
    if lmax >= 1:
        comps += [[1, 0, 0], [0, 1, 0], [0, 0, 1]]
    if lmax >= 2:
        comps += [[2, 0, 0], [1, 1, 0], [1, 0, 1], [0, 2, 0], [0, 1, 1], [0, 0, 2]]
    cen, al, L = [], [], []
    for c in C:
        a = float(np.exp(rng.uniform(np.log(0.3), np.log(2.0))))
        for l in comps:
            cen.append(c)
            al.append(a)
            L.append(l)
    return np.array(cen), np.array(al), np.array(L, dtype=np.int32)


def test_cartesian_tensor_symmetry_and_schwarz(oracle_mod):
    A, al, L = _shell_basis(2, 3)
    T = oracle_mod.eri_tensor(A, al, 0.0, lmn=L)
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1)]:
        assert np.max(np.abs(T - T.transpose(perm))) <= 1e-14 * np.max(np.abs(T))
    Q = oracle_mod.schwarz(A, al, lmn=L)
    n = al.shape[0]
    bound = Q.reshape(n, n, 1, 1) * Q.reshape(1, 1, n, n)
    assert np.all(np.abs(T) <= bound * (1 + 1e-12) + 1e-300)


def test_cartesian_canonical_build_equals_literal(oracle_mod):
    A, al, L = _shell_basis(3, 4)
    n = al.shape[0]
    D = np.random.default_rng(1).standard_normal((2, n, n)) / n
    for tau in (0.0, 1e-4):
        J1, K1 = oracle_mod.jk_literal(A, al, tau, D, lmn=L)
        J2, K2 = oracle_mod.jk_canonical(A, al, tau, D, lmn=L)
        assert np.max(np.abs(J1 - J2)) < 1e-13 and np.max(np.abs(K1 - K2)) < 1e-13
    T = oracle_mod.eri_tensor(A, al, 0.0, lmn=L)
    J3 = np.einsum("rs,rspq->pq", D[0], T)
    K3 = np.einsum("rs,prqs->pq", D[0], T)
    J2, K2 = oracle_mod.jk_canonical(A, al, 0.0, D, lmn=L)
    assert np.max(np.abs(J2[0] - J3)) < 1e-13 and np.max(np.abs(K2[0] - K3)) < 1e-13


# ---- contracted functions ---------------------------------------------------

@pytest.mark.parametrize("lmn", [(0, 0, 0), (1, 0, 0), (0, 1, 1), (2, 0, 0)])
def test_primitive_overlap_against_quadrature(oracle_mod, lmn):
    # <g_a|g_b> by 1-D quadratures of the unnormalised factors, normalised by
    # the same quadratures at a = b
    a, b = 0.7, 2.3

    def mom(x, y, l):
        v, _ = integrate.quad(lambda t: t ** (2 * l) * math.exp(-(x + y) * t * t), -np.inf, np.inf,
                              epsabs=0, epsrel=1e-13)
        return v
    raw = np.prod([mom(a, b, l) for l in lmn])
    na = np.prod([mom(a, a, l) for l in lmn])
    nb = np.prod([mom(b, b, l) for l in lmn])
    assert abs(oracle_mod.primitive_overlap(a, b, lmn) - raw / math.sqrt(na * nb)) < 1e-12
    assert abs(oracle_mod.primitive_overlap(a, a, lmn) - 1.0) < 1e-14


def test_contraction_of_one_primitive_is_the_primitive(oracle_mod):
    A, al, L = _shell_basis(2, 8)
    n = al.shape[0]
    basis = oracle_mod.contraction(A, L, np.arange(n + 1), al, np.full(n, 2.5))
    assert np.allclose(basis[3], np.eye(n), rtol=0, atol=1e-15)
    for q in [(0, 1, 2, 3), (4, 5, 6, 7), (1, 9, 3, 12)]:
        assert abs(oracle_mod.eri_contracted(basis, *q) - oracle_mod.eri(A, al, *q, lmn=L)) < 1e-15


def test_contracted_functions_are_normalised(oracle_mod):
    # <phi|phi> = sum C_a C_b <g_a|g_b> = 1 and (phi phi|..) scales as the
    # square of the function: doubling all coefficients changes nothing
    import workloads as wl
    cen, L, off, pe, pc = wl.contracted_basis(np.zeros((1, 3)))
    b1 = oracle_mod.contraction(cen, L, off, pe, pc)
    b2 = oracle_mod.contraction(cen, L, off, pe, 2 * pc)
    assert np.allclose(b1[3], b2[3], rtol=1e-15, atol=0)
    for i in range(cen.shape[0]):
        ks = np.nonzero(b1[3][:, i])[0]
        s = sum(b1[3][a, i] * b1[3][b, i] * oracle_mod.primitive_overlap(pe[a], pe[b], L[i]) for a in ks for b in ks)
        assert abs(s - 1.0) < 1e-14


def test_contracted_build_against_contracted_tensor(oracle_mod):
    # J, K from the primitive build of C D C^T against the definition over
    # the contracted tensor assembled integral by integral
    import workloads as wl
    cen, L, off, pe, pc = wl.contracted_basis(np.array([[0.0, 0.0, 0.0], [1.3, 0.4, -0.2]]),
                                              shells=wl.CONTRACTED_SHELLS[:3])
    basis = oracle_mod.contraction(cen, L, off, pe, pc)
    n = cen.shape[0]
    T = np.zeros((n, n, n, n))
    for p in range(n):
        for q in range(n):
            for r in range(n):
                for s in range(n):
                    T[p, q, r, s] = oracle_mod.eri_contracted(basis, p, q, r, s)
    D = np.random.default_rng(4).standard_normal((2, n, n)) / n
    J, K = oracle_mod.jk_contracted(basis, D)
    assert np.max(np.abs(J[1] - np.einsum("rs,rspq->pq", D[1], T))) < 1e-13
    assert np.max(np.abs(K[1] - np.einsum("rs,prqs->pq", D[1], T))) < 1e-13
