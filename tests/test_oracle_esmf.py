"""Pins of the oracle's ESMF densities and two-body energy.

The closed forms (the notation table's A and B, the list of nine Fock builds,
Eq. esmf_energy_2b) are checked against the wave function they come from, not
against a retyping of themselves:
- the ESMF state c0 |Phi> + sum_{ia,spin} sigma_ia a+_a a_i |Phi> is built
  in an explicit fermion Fock space (occupation bit strings, operator signs by
  counting), and its one-particle density and the expectation value of the
  two-electron operator over the MO integrals are summed by brute force;
- the densities that carry Lagrange multipliers are the first-order changes
  of D1, D2 and A along the multiplier directions (the L_3 and L_2 pieces of
  the Appendix are such directional derivatives), taken by exact central
  differences of these quadratic functions.
"""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.cpu


# ---- a small fermion Fock space -------------------------------------------
# spin orbital 2p + s (s = 0 alpha, 1 beta) of spatial orbital p; a
# determinant is an int bit string, operators act from the right.

def _annihilate(det, q):
    if not (det >> q) & 1:
        return None, 0
    sign = -1 if bin(det & ((1 << q) - 1)).count("1") % 2 else 1
    return det & ~(1 << q), sign


def _create(det, p):
    if (det >> p) & 1:
        return None, 0
    sign = -1 if bin(det & ((1 << p) - 1)).count("1") % 2 else 1
    return det | (1 << p), sign


def _apply(ops, state):
    """ops: [(kind, spin_orbital)] applied right to left; state: {det: coef}."""
    out = {}
    for det, c in state.items():
        d, s = det, c
        for kind, o in reversed(ops):
            d, sg = (_create if kind == "+" else _annihilate)(d, o)
            if d is None:
                break
            s *= sg
        if d is not None:
            out[d] = out.get(d, 0.0) + s
    return out


def _dot(a, b):
    return sum(c * b.get(d, 0.0) for d, c in a.items())


def _esmf_wavefunction(no, nv, c0, sigma):
    ref = 0
    for i in range(no):
        ref |= (1 << (2 * i)) | (1 << (2 * i + 1))
    psi = {ref: c0}
    for i in range(no):
        for a in range(nv):
            for s in (0, 1):
                t = _apply([("+", 2 * (no + a) + s), ("-", 2 * i + s)], {ref: sigma[i, a]})
                for d, c in t.items():
                    psi[d] = psi.get(d, 0.0) + c
    return psi


def _one_particle_density(psi, n):
    g = np.zeros((n, n))
    for p in range(n):
        for q in range(n):
            for s in (0, 1):
                g[p, q] += _dot(psi, _apply([("+", 2 * p + s), ("-", 2 * q + s)], psi))
    return g


def _two_body_expectation(psi, h):
    """<psi| 1/2 sum (pq|rs) a+_{p s} a+_{r t} a_{s' t} a_{q s} |psi> over
    chemists' MO integrals h[p, q, r, s]."""
    n = h.shape[0]
    e = 0.0
    for p in range(n):
        for q in range(n):
            for r in range(n):
                for s in range(n):
                    v = h[p, q, r, s]
                    if v == 0.0:
                        continue
                    for sa in (0, 1):
                        for sb in (0, 1):
                            ops = [("+", 2 * p + sa), ("+", 2 * r + sb), ("-", 2 * s + sb), ("-", 2 * q + sa)]
                            e += 0.5 * v * _dot(psi, _apply(ops, psi))
    return e


def test_fock_space_signs():
    # {a_p, a+_q} = delta_pq on every basis state of 4 spin orbitals
    for det in range(16):
        for p in range(4):
            for q in range(4):
                st = {det: 1.0}
                x = _apply([("-", p), ("+", q)], st)
                y = _apply([("+", q), ("-", p)], st)
                tot = {d: x.get(d, 0.0) + y.get(d, 0.0) for d in set(x) | set(y)}
                tot = {d: c for d, c in tot.items() if c != 0.0}
                assert tot == ({det: 1.0} if p == q else {})


def _state(n, no, seed):
    st = wl.esmf_state(n, no, seed, sigma_norm=0.6, c0=0.7)
    assert st["theta"].shape == (no, n) and st["gamma"].shape == (n - no, n)
    V = np.vstack([st["theta"], st["gamma"]])
    assert np.allclose(V @ V.T, np.eye(n), atol=1e-14)
    return st, V


@pytest.mark.parametrize("n,no,seed", [(4, 1, 3), (5, 2, 4), (6, 2, 5)])
def test_densities_against_one_particle_density(oracle_mod, n, no, seed):
    # E_1 of Eq. esmf_energy_1b is G . (2 N2 D1 + 4 c0 D2 + 2 A), so the
    # state's symmetric one-particle density in the AO basis is
    # 2 N2 D1 + 2 c0 (D2 + D2^T) + 2 A, and its norm is N2
    st, V = _state(n, no, seed)
    psi = _esmf_wavefunction(no, n - no, st["c0"], st["sigma"])
    assert abs(_dot(psi, psi) - st["n2"]) < 1e-14
    g_ao = V.T @ _one_particle_density(psi, n) @ V
    D = oracle_mod.nine_densities(st["theta"], st["gamma"], st["sigma"], st["mu"], st["R"], st["Phi"])
    assert D.shape == (9, n, n)
    want = 2 * st["n2"] * D[0] + 2 * st["c0"] * (D[1] + D[1].T) + 2 * D[2]
    assert np.max(np.abs(g_ao - want)) < 1e-13
    # the off-diagonal block alone: <Phi| E_pq |CIS> in the AO basis is 2 D2
    ref = {k: v for k, v in psi.items() if k == max(psi, key=lambda d: d if psi[d] == st["c0"] else -1)}
    assert len(ref) == 1
    cis = {d: c for d, c in psi.items() if d not in ref}
    t = np.zeros((n, n))
    for p in range(n):
        for q in range(n):
            for s in (0, 1):
                t[p, q] += _dot({d: 1.0 for d in ref}, _apply([("+", 2 * p + s), ("-", 2 * q + s)], cis))
    assert np.max(np.abs(V.T @ t @ V - 2 * D[1])) < 1e-14


@pytest.mark.parametrize("n,no,seed,c0", [(4, 1, 31, 0.7), (5, 2, 32, -1.1), (6, 3, 33, 0.25)])
def test_energy_one_body_against_fock_space(oracle_mod, n, no, seed, c0):
    # E_1 of Eq. esmf_energy_1b is <Psi|sum_pq G_pq E_pq|Psi> of the
    # unnormalised ESMF state, with E_pq = sum_spin a+_p a_q: the trace of G
    # (an arbitrary symmetric matrix here, not the workloads' stand-in) with
    # the state's one-particle density, summed in the Fock space over MO
    # indices and brought to the AO basis with V
    st = wl.esmf_state(n, no, seed, sigma_norm=0.5, c0=c0)
    V = np.vstack([st["theta"], st["gamma"]])
    rng = np.random.default_rng(seed + 5)
    G = rng.standard_normal((n, n))
    G = G + G.T
    psi = _esmf_wavefunction(no, n - no, st["c0"], st["sigma"])
    g_mo = _one_particle_density(psi, n)
    e_fs = float(np.sum((V @ G @ V.T) * g_mo))
    D = oracle_mod.nine_densities(st["theta"], st["gamma"], st["sigma"], st["mu"], st["R"], st["Phi"])
    e1 = oracle_mod.energy_one_body(G, D, st["n2"], st["c0"])
    assert abs(e1 - e_fs) < 1e-13 * max(1.0, abs(e_fs)), (e1, e_fs)
    # with sigma = 0 and c0 = 1 it is 2 Tr[P G] with P = Theta^T Theta (Eq. esmf_eng_hf)
    st["sigma"][:] = 0.0
    D0 = oracle_mod.nine_densities(st["theta"], st["gamma"], st["sigma"], st["mu"], st["R"], st["Phi"])
    P = st["theta"].T @ st["theta"]
    assert abs(oracle_mod.energy_one_body(G, D0, 1.0, 1.0) - 2.0 * np.trace(P @ G)) < 1e-13 * np.abs(G).sum()


@pytest.mark.parametrize("n,no,seed,c0", [(4, 1, 11, 0.7), (5, 2, 12, 0.7), (5, 2, 13, -1.3), (6, 3, 14, 0.2)])
def test_energy_two_body_against_fock_space(oracle_mod, n, no, seed, c0):
    # Eq. esmf_energy_2b is <Psi|V_ee|Psi> of the unnormalised ESMF state (with
    # its last term read as 2 F[D2].D2; the printed 2 F[D2].D1 misses by
    # F[D2].(D2 - D1), the difference the first case below shows)
    A, al = wl.random_box(n, seed=seed, box=3.0)
    T = oracle_mod.eri_tensor(A, al, 0.0)
    st = wl.esmf_state(n, no, seed, sigma_norm=0.5, c0=c0)
    V = np.vstack([st["theta"], st["gamma"]])
    h = np.einsum("pa,qb,rc,sd,abcd->pqrs", V, V, V, V, T, optimize=True)
    psi = _esmf_wavefunction(no, n - no, st["c0"], st["sigma"])
    e_fs = _two_body_expectation(psi, h)
    D = oracle_mod.nine_densities(st["theta"], st["gamma"], st["sigma"], st["mu"], st["R"], st["Phi"])
    J, K = oracle_mod.jk_canonical(A, al, 0.0, D[:2])
    e2 = oracle_mod.energy_two_body(J, K, D, st["n2"], st["c0"])
    assert abs(e2 - e_fs) < 1e-12 * max(1.0, abs(e_fs)), (e2, e_fs)


def test_energy_two_body_hf_limit(oracle_mod):
    # sigma = 0, c0 = 1 (Eq. esmf_eng_hf): E_2 = F[P] . P with P = Theta^T Theta,
    # which is 2 sum (ii|jj) - sum (ij|ji) over occupied MOs
    n, no = 7, 3
    A, al = wl.random_box(n, seed=51, box=4.0)
    T = oracle_mod.eri_tensor(A, al, 0.0)
    st = wl.esmf_state(n, no, 52, sigma_norm=0.0, c0=1.0)
    st["sigma"][:] = 0.0
    D = oracle_mod.nine_densities(st["theta"], st["gamma"], st["sigma"], st["mu"], st["R"], st["Phi"])
    J, K = oracle_mod.jk_canonical(A, al, 0.0, D[:2])
    e2 = oracle_mod.energy_two_body(J, K, D, 1.0, 1.0)
    Th = st["theta"]
    h = np.einsum("pa,qb,rc,sd,abcd->pqrs", Th, Th, Th, Th, T, optimize=True)
    ref = 2 * np.einsum("iijj->", h) - np.einsum("ijji->", h)
    assert abs(e2 - ref) < 1e-12 * abs(ref)
    assert np.all(D[1] == 0) and np.all(D[2] == 0)


def _d(f, x, dx):
    # central difference; exact (up to rounding) for f of degree <= 2 in the step
    return (f(x + dx) - f(x - dx)) / 2.0


@pytest.mark.parametrize("n,no,seed", [(6, 2, 21), (9, 4, 22)])
def test_multiplier_densities_are_directional_derivatives(oracle_mod, n, no, seed):
    # L_3 of the Appendix is the first-order change of the energy when Theta
    # and Gamma move along R and Phi; L_2 the change when sigma moves along
    # mu.  Densities 4-9 are the first-order changes of D1, D2 and A.
    st = wl.esmf_state(n, no, seed)
    T, G, s, u, R, P = (st[k] for k in ("theta", "gamma", "sigma", "mu", "R", "Phi"))
    D = oracle_mod.nine_densities(T, G, s, u, R, P)

    def nd(Tx=T, Gx=G, sx=s):
        return oracle_mod.nine_densities(Tx, Gx, sx, u, R, P)
    tol = 1e-14 * max(1.0, np.max(np.abs(D)))
    # Theta -> Theta + e R: D1 changes by D4 + D4^T, D2 by D5
    d_t = _d(lambda x: nd(Tx=x), T, R)
    assert np.max(np.abs(d_t[0] - (D[3] + D[3].T))) < tol
    assert np.max(np.abs(d_t[1] - D[4])) < tol
    # Gamma -> Gamma + e Phi: D2 changes by D7
    d_g = _d(lambda x: nd(Gx=x), G, P)
    assert np.max(np.abs(d_g[1] - D[6])) < tol
    # both at once: A changes by B + B^T (the reading of the table's B whose
    # first factor conforms: Phi^T sigma^T sigma Gamma)
    d_tg = (nd(Tx=T + R, Gx=G + P)[2] - nd(Tx=T - R, Gx=G - P)[2]) / 2.0
    assert np.max(np.abs(d_tg - (D[8] + D[8].T))) < tol
    # sigma -> sigma + e mu: D2 changes by D6; the Theta^T sigma sigma^T Theta
    # part of A by D8 + D8^T
    d_s = _d(lambda x: nd(sx=x), s, u)
    assert np.max(np.abs(d_s[1] - D[5])) < tol
    # (with Gamma = 0, A is - Theta^T sigma sigma^T Theta)
    ss = lambda x: nd(sx=x, Gx=np.zeros_like(G))[2]  # noqa: E731
    assert np.max(np.abs(_d(ss, s, u) + (D[7] + D[7].T))) < tol
    # D1, A symmetric; D1 idempotent-like: D1 D1 = D1 for orthonormal rows
    assert np.max(np.abs(D[0] - D[0].T)) < tol and np.max(np.abs(D[2] - D[2].T)) < tol
    assert np.max(np.abs(D[0] @ D[0] - D[0])) < 1e-13


def test_printed_b_does_not_conform():
    # the table prints B's first term as Theta^T sigma^T sigma Gamma: Theta^T is
    # [N, No] and sigma^T [Nv, No], which multiply only when No = Nv
    st = wl.esmf_state(6, 2, 1)
    with pytest.raises(ValueError):
        st["theta"].T @ st["sigma"].T


# ---- the energy and its first derivatives ----------------------------------

def _num(oracle_mod, A, al, G, theta, gamma, sigma, c0):
    """E_1 + E_2 at (c0, sigma, Theta, Gamma), from fresh oracle builds."""
    z = np.zeros_like(sigma)
    D = oracle_mod.nine_densities(theta, gamma, sigma, z, np.zeros_like(theta), np.zeros_like(gamma))
    J, K = oracle_mod.jk_canonical(A, al, 0.0, D[:2])
    n2 = c0 * c0 + 2.0 * np.sum(sigma * sigma)
    return oracle_mod.energy_one_body(G, D, n2, c0) + oracle_mod.energy_two_body(J, K, D, n2, c0)


def _stencil5(f, h=1.0):
    # (-f(2h) + 8 f(h) - 8 f(-h) + f(-2h)) / 12h: exact for polynomials of degree <= 4
    return (-f(2 * h) + 8 * f(h) - 8 * f(-h) + f(-2 * h)) / (12 * h)


@pytest.mark.parametrize("n,no,seed", [(8, 3, 61), (9, 2, 62)])
def test_energy_gradient_exact_differences(oracle_mod, n, no, seed):
    # E_1 + E_2 is a polynomial of degree <= 4 in each of c0, sigma, Theta and
    # Gamma separately, so a five-point difference along any direction of one
    # block gives its directional derivative exactly (up to rounding); the
    # oracle's gradient of E = (E_1 + E_2) / N2 must reproduce it through
    # d(E_1 + E_2) = N2 dE + E dN2.
    A, al = wl.random_box(n, seed=seed, box=4.0)
    st = wl.esmf_state(n, no, seed, sigma_norm=0.4, c0=0.8)
    T, Gm, s, c0, G = st["theta"], st["gamma"], st["sigma"], st["c0"], st["G"]
    D = oracle_mod.nine_densities(T, Gm, s, st["mu"], st["R"], st["Phi"])
    J, K = oracle_mod.jk_canonical(A, al, 0.0, D[:3])
    g = oracle_mod.energy_gradient(G, J, K, D, T, Gm, s, c0, st["n2"])
    n2, E = st["n2"], g["E"]
    num0 = _num(oracle_mod, A, al, G, T, Gm, s, c0)
    assert abs(num0 - n2 * E) < 1e-12 * abs(num0)
    rng = np.random.default_rng(seed + 7)
    dT, dG, ds = (rng.standard_normal(x.shape) for x in (T, Gm, s))
    scale = abs(num0)
    fd = _stencil5(lambda h: _num(oracle_mod, A, al, G, T + h * dT, Gm, s, c0))
    assert abs(fd - n2 * np.sum(g["theta"] * dT)) < 1e-11 * scale
    fd = _stencil5(lambda h: _num(oracle_mod, A, al, G, T, Gm + h * dG, s, c0))
    assert abs(fd - n2 * np.sum(g["gamma"] * dG)) < 1e-11 * scale
    fd = _stencil5(lambda h: _num(oracle_mod, A, al, G, T, Gm, s + h * ds, c0))
    assert abs(fd - (n2 * np.sum(g["sigma"] * ds) + E * np.sum(4 * s * ds))) < 1e-11 * scale
    fd = _stencil5(lambda h: _num(oracle_mod, A, al, G, T, Gm, s, c0 + h))
    assert abs(fd - (n2 * g["c0"] + E * 2 * c0)) < 1e-11 * scale


def test_energy_gradient_of_the_quotient(oracle_mod):
    # dE itself (a rational function): small-step five-point differences
    n, no = 8, 3
    A, al = wl.random_box(n, seed=71, box=4.0)
    st = wl.esmf_state(n, no, 72, sigma_norm=0.4, c0=0.8)
    T, Gm, s, c0, G = st["theta"], st["gamma"], st["sigma"], st["c0"], st["G"]
    D = oracle_mod.nine_densities(T, Gm, s, st["mu"], st["R"], st["Phi"])
    J, K = oracle_mod.jk_canonical(A, al, 0.0, D[:3])
    g = oracle_mod.energy_gradient(G, J, K, D, T, Gm, s, c0, st["n2"])

    def E(sx, cx):
        return _num(oracle_mod, A, al, G, T, Gm, sx, cx) / (cx * cx + 2 * np.sum(sx * sx))
    ds = np.random.default_rng(3).standard_normal(s.shape)
    ds /= np.linalg.norm(ds)
    # unit direction, h = 2e-4: truncation ~h^4, rounding ~eps |E| / h
    h = 2e-4
    fd = (-E(s + 2 * h * ds, c0) + 8 * E(s + h * ds, c0) - 8 * E(s - h * ds, c0) + E(s - 2 * h * ds, c0)) / (12 * h)
    assert abs(fd - np.sum(g["sigma"] * ds)) < 1e-8 * max(1.0, abs(fd))
    fd = (-E(s, c0 + 2 * h) + 8 * E(s, c0 + h) - 8 * E(s, c0 - h) + E(s, c0 - 2 * h)) / (12 * h)
    assert abs(fd - g["c0"]) < 1e-8 * max(1.0, abs(fd))
    # the paper's printed Theta-derivative has F[A] - F[A]^T, which vanishes
    # for symmetric A: the exact gradient carries 2 Theta (F[A] + F[A]^T) / N2
    FA = 2 * J[2] - K[2]
    assert np.max(np.abs(FA - FA.T)) < 1e-14 * np.max(np.abs(FA))
    assert np.max(np.abs(T @ (FA + FA.T))) > 1e-3
