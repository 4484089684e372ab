"""ctypes front end of ``esmf_oracle.c`` (plain FP64 C + OpenMP).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every routine follows
the definitions of arXiv:2002.00322 Sec. "Notation" (Eq. J_and_K) and
Sec. "Shell-Pair Screening"; the C file documents each step.
"""
import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "esmf_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_i64p = ctypes.POINTER(ctypes.c_int64)


def build(force=True):
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
    if force or not os.path.exists(_LIB_PATH):
        subprocess.check_call(cmd)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_boys_f0.restype = ctypes.c_double
    lib.oracle_boys_f0.argtypes = [ctypes.c_double]
    lib.oracle_boys_fn.restype = None
    lib.oracle_boys_fn.argtypes = [ctypes.c_int, ctypes.c_double, _dp]
    lib.oracle_eri.restype = ctypes.c_double
    lib.oracle_eri.argtypes = [_dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.oracle_eri_cart.restype = ctypes.c_double
    lib.oracle_eri_cart.argtypes = [_dp, _dp, _ip, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    # each routine in two forms: s functions, and Cartesian functions (_cart,
    # with the [n][3] angular-momentum array after the exponents)
    sigs = {
        "oracle_schwarz": (None, [ctypes.c_int, _dp, _dp, _dp]),
        "oracle_eri_tensor": (ctypes.c_int, [ctypes.c_int, _dp, _dp, ctypes.c_double, _dp]),
        "oracle_count": (None, [ctypes.c_int, _dp, _dp, ctypes.c_double, _i64p, _i64p]),
        "oracle_jk_literal": (ctypes.c_int, [ctypes.c_int, _dp, _dp, ctypes.c_double, ctypes.c_int,
                                             _dp, _dp, _dp]),
        "oracle_jk_entries": (ctypes.c_int, [ctypes.c_int, _dp, _dp, ctypes.c_double, ctypes.c_int,
                                             _dp, ctypes.c_int, _ip, _ip, _ip, _dp, _dp]),
        "oracle_jk_canonical_range": (ctypes.c_int, [ctypes.c_int, _dp, _dp, ctypes.c_double,
                                                     ctypes.c_int, _dp, _dp, _dp, ctypes.c_int64,
                                                     ctypes.c_int64, _i64p]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(lib, name)
        f.restype, f.argtypes = res, args
        g = getattr(lib, name + "_cart")
        g.restype, g.argtypes = res, args[:3] + [_ip] + args[3:]
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_num_threads.argtypes = []
    _lib = lib
    return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(_dp)


def _basis(centers, alpha, lmn):
    """(centers, exponents, angular-momentum array or None) as C arrays."""
    c, a = _f64(centers), _f64(alpha)
    if lmn is None:
        return c, a, None
    L = np.ascontiguousarray(lmn, dtype=np.int32)
    assert L.shape == (a.shape[0], 3) and L.min() >= 0 and L.max() <= 2
    return c, a, L


def _call(name, c, a, L, *rest):
    lib = _load()
    if L is None:
        return getattr(lib, name)(a.shape[0], _ptr(c), _ptr(a), *rest)
    return getattr(lib, name + "_cart")(a.shape[0], _ptr(c), _ptr(a), L.ctypes.data_as(_ip), *rest)


def boys_f0(T):
    return _load().oracle_boys_f0(float(T))


def boys_fn(nmax, T):
    """F_0(T) .. F_nmax(T)."""
    F = np.empty(int(nmax) + 1)
    _load().oracle_boys_fn(int(nmax), float(T), _ptr(F))
    return F


def eri(centers, alpha, p, q, r, s, lmn=None):
    """(pq|rs) for normalised s primitives, or Cartesian functions with the
    given (l, m, n) per function (chemists' notation)."""
    c, a, L = _basis(centers, alpha, lmn)
    if L is None:
        return _load().oracle_eri(_ptr(c), _ptr(a), int(p), int(q), int(r), int(s))
    return _load().oracle_eri_cart(_ptr(c), _ptr(a), L.ctypes.data_as(_ip), int(p), int(q), int(r), int(s))


def schwarz(centers, alpha, lmn=None):
    c, a, L = _basis(centers, alpha, lmn)
    n = a.shape[0]
    Q = np.empty((n, n))
    _call("oracle_schwarz", c, a, L, _ptr(Q))
    return Q


def eri_tensor(centers, alpha, tau=0.0, lmn=None):
    """Dense masked (pq|rs) tensor, shape (n,n,n,n); small n only."""
    c, a, L = _basis(centers, alpha, lmn)
    n = a.shape[0]
    T = np.empty((n, n, n, n))
    if _call("oracle_eri_tensor", c, a, L, float(tau), _ptr(T)) != 0:
        raise MemoryError("oracle_eri_tensor")
    return T


def count(centers, alpha, tau, lmn=None):
    """(retained pairs, retained unique quartets) under the screen."""
    c, a, L = _basis(centers, alpha, lmn)
    np_, nq = ctypes.c_int64(), ctypes.c_int64()
    _call("oracle_count", c, a, L, float(tau), ctypes.byref(np_), ctypes.byref(nq))
    return np_.value, nq.value


def _dens(D, n):
    D = _f64(D)
    if D.ndim == 2:
        D = D[None]
    assert D.shape[1:] == (n, n)
    return D


def jk_literal(centers, alpha, tau, D, lmn=None):
    """J and K by the plain quadruple sum of Eq. J_and_K (O(m N^4))."""
    c, a, L = _basis(centers, alpha, lmn)
    n = a.shape[0]
    D = _dens(D, n)
    J = np.empty_like(D)
    K = np.empty_like(D)
    if _call("oracle_jk_literal", c, a, L, float(tau), D.shape[0], _ptr(D), _ptr(J), _ptr(K)) != 0:
        raise MemoryError("oracle_jk_literal")
    return J, K


def jk_canonical_range(centers, alpha, tau, D, pair_begin=0, pair_end=None, lmn=None):
    """Grouped build over unique quartets whose outer pair index is in range.

    Returns (J, K, n_quartets_visited)."""
    c, a, L = _basis(centers, alpha, lmn)
    n = a.shape[0]
    D = _dens(D, n)
    if pair_end is None:
        pair_end = n * (n + 1) // 2
    J = np.empty_like(D)
    K = np.empty_like(D)
    nv = ctypes.c_int64()
    if _call("oracle_jk_canonical_range", c, a, L, float(tau), D.shape[0], _ptr(D), _ptr(J), _ptr(K),
             int(pair_begin), int(pair_end), ctypes.byref(nv)) != 0:
        raise MemoryError("oracle_jk_canonical_range")
    return J, K, nv.value


def jk_canonical(centers, alpha, tau, D, lmn=None):
    """The paper's grouped build: one loop over unique screened quartets."""
    J, K, _ = jk_canonical_range(centers, alpha, tau, D, lmn=lmn)
    return J, K


def jk_entries(centers, alpha, tau, D, dens, rows, cols, lmn=None):
    """J_i[p][q] and K_i[p][q] at the listed (i, p, q) by the definition."""
    c, a, L = _basis(centers, alpha, lmn)
    n = a.shape[0]
    D = _dens(D, n)
    dens = np.ascontiguousarray(dens, dtype=np.int32)
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    cnt = dens.shape[0]
    Jo = np.empty(cnt)
    Ko = np.empty(cnt)
    rc = _call("oracle_jk_entries", c, a, L, float(tau), D.shape[0], _ptr(D), cnt, dens.ctypes.data_as(_ip),
               rows.ctypes.data_as(_ip), cols.ctypes.data_as(_ip), _ptr(Jo), _ptr(Ko))
    if rc != 0:
        raise ValueError("oracle_jk_entries: bad index or allocation failure")
    return Jo, Ko


def primitive_overlap(a, b, lmn):
    """<g_a|g_b> of two normalised Cartesian primitives on one centre with the
    same powers: the product over directions of the 1-D moments
    int x^(2l) exp(-(a+b) x^2) dx = Gamma(l + 1/2) / (a+b)^(l + 1/2), times the
    primitives' normalisations (each fixed by <g|g> = 1 in the same way)."""
    def raw(x, y):
        return np.prod([math.gamma(l + 0.5) / (x + y) ** (l + 0.5) for l in lmn])
    return raw(a, b) / math.sqrt(raw(a, a) * raw(b, b))


def contraction(centers, lmn, prim_offset, prim_exp, prim_coef):
    """A contracted basis as its primitive basis and the matrix C [P, N] with
    phi_i = sum_k C[k, i] g_k, each phi_i normalised: returns (primitive
    centres [P, 3], exponents [P], powers [P, 3], C)."""
    centers, lmn = np.asarray(centers, float), np.asarray(lmn, int)
    off = np.asarray(prim_offset, int)
    e, cf = np.asarray(prim_exp, float), np.asarray(prim_coef, float)
    n, P = centers.shape[0], off[-1]
    C = np.zeros((P, n))
    pc = np.zeros((P, 3))
    pl = np.zeros((P, 3), int)
    for i in range(n):
        ks = range(off[i], off[i + 1])
        nrm = sum(cf[a] * cf[b] * primitive_overlap(e[a], e[b], lmn[i]) for a in ks for b in ks)
        for k in ks:
            C[k, i] = cf[k] / math.sqrt(nrm)
            pc[k] = centers[i]
            pl[k] = lmn[i]
    return pc, e.copy(), pl, C


def eri_contracted(basis, p, q, r, s):
    """(pq|rs) over contracted functions: sum of C-weighted primitive integrals."""
    pc, pe, pl, C = basis
    v = 0.0
    for a in np.nonzero(C[:, p])[0]:
        for b in np.nonzero(C[:, q])[0]:
            for c in np.nonzero(C[:, r])[0]:
                for d in np.nonzero(C[:, s])[0]:
                    v += C[a, p] * C[b, q] * C[c, r] * C[d, s] * eri(pc, pe, a, b, c, d, lmn=pl)
    return v


def jk_contracted(basis, D):
    """Unscreened J and K over contracted functions, from the primitive build
    of the densities C D C^T (J[D] = C^T J_prim[C D C^T] C, likewise K, by
    linearity of Eq. J_and_K in the integrals)."""
    pc, pe, pl, C = basis
    D = np.asarray(D, float)
    if D.ndim == 2:
        D = D[None]
    Dp = np.einsum("ki,mij,lj->mkl", C, D, C)
    Jp, Kp = jk_canonical(pc, pe, 0.0, Dp, lmn=pl)
    return np.einsum("ki,mkl,lj->mij", C, Jp, C), np.einsum("ki,mkl,lj->mij", C, Kp, C)


def nine_densities(theta, gamma, sigma, mu, R, Phi):
    """The nine generalised densities of one ESMF gradient evaluation
    (Sec. "Shell-Pair Screening", the list of nine Fock builds), each written
    as the product of the notation table's matrices, in list order:
    Theta^T Theta, Theta^T sigma Gamma, A, R^T Theta, R^T sigma Gamma,
    Theta^T mu Gamma, Theta^T sigma Phi, Theta^T mu sigma^T Theta, B, with
    A = Gamma^T sigma^T sigma Gamma - Theta^T sigma sigma^T Theta and
    B = Phi^T sigma^T sigma Gamma - R^T sigma sigma^T Theta (the reading of the
    table's B whose first term conforms)."""
    T, G, s, u, Rm, P = (np.asarray(x, dtype=np.float64) for x in (theta, gamma, sigma, mu, R, Phi))
    A = G.T @ s.T @ s @ G - T.T @ s @ s.T @ T
    B = P.T @ s.T @ s @ G - Rm.T @ s @ s.T @ T
    return np.stack([T.T @ T, T.T @ s @ G, A, Rm.T @ T, Rm.T @ s @ G, T.T @ u @ G, T.T @ s @ P,
                     T.T @ u @ s.T @ T, B])


def energy_two_body(J, K, D, n2, c0):
    """E_2 of Eq. esmf_energy_2b from D1 = Theta^T Theta, D2 = Theta^T sigma Gamma,
    A (the first three of D) and J, K of D1 and D2:
    N2 F[D1].D1 + 4 c0 F[D1].D2 + 2 F[D1].A + 2 F[D2].D2, with F = 2J - K
    (Eq. J_and_K) and X.Y the element-wise inner product.  The last term is
    read as F[D2].D2: the printed F[D2].D1 is linear in sigma, while that
    term belongs to the block quadratic in sigma; the sigma-derivative of the
    energy in the Appendix carries the 4 Theta F[D2] Gamma^T that F[D2].D2
    produces."""
    F1 = 2.0 * J[0] - K[0]
    F2 = 2.0 * J[1] - K[1]
    D1, D2, A = D[0], D[1], D[2]
    return float(n2 * np.sum(F1 * D1) + 4.0 * c0 * np.sum(F1 * D2) + 2.0 * np.sum(F1 * A)
                 + 2.0 * np.sum(F2 * D2))


def energy_one_body(G, D, n2, c0):
    """E_1 of Eq. esmf_energy_1b, each trace written as an inner product with
    the symmetric one-electron matrix G: G . (2 N2 D1 + 4 c0 D2 + 2 A)."""
    G = np.asarray(G, dtype=np.float64)
    return float(np.sum(G * (2.0 * n2 * D[0] + 4.0 * c0 * D[1] + 2.0 * D[2])))


def energy_gradient(G, J, K, D, theta, gamma, sigma, c0, n2):
    """The ESMF energy E = (E_1 + E_2) / N2 (Eq. esmf_eng) and its first
    derivatives with respect to c0, sigma, Theta and Gamma (the Appendix's
    energy derivatives), from the J and K of D1, D2 and A (the first three
    densities).  Written from E_1 (Eq. esmf_energy_1b) and E_2 (Eq.
    esmf_energy_2b, last term F[D2].D2) with F[X].Y = F[Y].X, F[X^T] = F[X]^T
    and, for H = G + F[D1], the chain rule through D1 = Theta^T Theta,
    D2 = Theta^T sigma Gamma, A and N2 = c0^2 + 2 |sigma|^2.
    Returns dict(E1, E2, E, c0, sigma, theta, gamma)."""
    G, T, Gm, s = (np.asarray(x, dtype=np.float64) for x in (G, theta, gamma, sigma))
    F1 = 2.0 * J[0] - K[0]
    F2 = 2.0 * J[1] - K[1]
    FA = 2.0 * J[2] - K[2]
    D1, D2, A = D[0], D[1], D[2]
    e1 = energy_one_body(G, D, n2, c0)
    e2 = energy_two_body(J, K, D, n2, c0)
    e = (e1 + e2) / n2
    H = G + F1
    # derivatives of E_1 + E_2
    d_c0 = 4.0 * c0 * np.sum(G * D1) + 4.0 * np.sum(G * D2) + 2.0 * c0 * np.sum(F1 * D1) + 4.0 * np.sum(F1 * D2)
    d_sigma = (4.0 * (2.0 * np.sum(G * D1) + np.sum(F1 * D1)) * s
               + 4.0 * c0 * T @ H @ Gm.T + 4.0 * s @ Gm @ H @ Gm.T - 4.0 * T @ H @ T.T @ s
               + 4.0 * T @ F2 @ Gm.T)
    d_theta = (4.0 * n2 * T @ H + 4.0 * c0 * s @ Gm @ H - 4.0 * s @ s.T @ T @ H
               + 4.0 * c0 * T @ (F2 + F2.T) + 2.0 * T @ (FA + FA.T) + 4.0 * s @ Gm @ F2.T)
    d_gamma = 4.0 * c0 * s.T @ T @ H + 4.0 * s.T @ s @ Gm @ H + 4.0 * s.T @ T @ F2
    # quotient by N2 (dN2/dc0 = 2 c0, dN2/dsigma = 4 sigma)
    return dict(E1=e1, E2=e2, E=e, c0=float((d_c0 - 2.0 * c0 * e) / n2),
                sigma=(d_sigma - 4.0 * e * s) / n2, theta=d_theta / n2, gamma=d_gamma / n2)


def num_threads():
    return _load().oracle_num_threads()
