"""Seeded synthetic molecules and densities.

The paper's molecules and basis sets (PySCF integrals over cc-pVDZ / 6-31G*,
Sec. "Computational Details") are not available here; these generators stand
in for them with single-primitive s-type bases whose sizes, spatial structure
and density shapes follow the workloads the build is measured on:

  random_box   -- N s functions, centres uniform in a cube, log-uniform exponents
  chain        -- linear chain of centres, several exponents per centre
  slab         -- jittered 3-D lattice of centres, several exponents per centre
  random_densities      -- dense non-symmetric D, entries N(0,1)*scale
  transition_densities  -- D_i = C_occ W_i C_virt^T with C orthonormal (QR of a
                           seeded Gaussian matrix, columns sign-fixed so that
                           diag(R) > 0) and W_i Gaussian with variance
                           1/(N_o N_v), i.e. ||W_i||_F ~ 1 like a normalised
                           CIS vector; this is the shape of the paper's
                           transition density Theta^T sigma Gamma (Eq.
                           esmf_energy_2b) in the AO basis.

Functions are returned as (centers[N,3] in bohr, exponents[N]) in the order
(centre, exponent) -- centre-major.
"""
import numpy as np

__all__ = [
    "random_box", "chain", "slab", "random_densities", "transition_densities",
    "config1", "config2", "config3", "config3_deep", "batch_workload", "serving_sessions",
    "SPACING", "CHAIN_EXPONENTS", "orthonormal", "session_density", "esmf_state",
    "CART_COMPONENTS", "SPD_SHELLS", "cart_basis", "spd_chain", "spd_box", "CONTRACTED_SHELLS",
    "contracted_basis",
]

SPACING = 1.4
CHAIN_EXPONENTS = (0.3, 1.5)


def random_box(n, seed, box=10.0, amin=0.1, amax=10.0):
    rng = np.random.default_rng(seed)
    centers = rng.uniform(0.0, box, size=(n, 3))
    alpha = np.exp(rng.uniform(np.log(amin), np.log(amax), size=n))
    return centers, alpha


def _expand(sites, exps):
    exps = np.asarray(exps, dtype=np.float64)
    centers = np.repeat(np.asarray(sites, dtype=np.float64), len(exps), axis=0)
    alpha = np.tile(exps, len(sites))
    return centers, alpha


def chain(ncentres, spacing=SPACING, exps=CHAIN_EXPONENTS):
    sites = np.zeros((ncentres, 3))
    sites[:, 0] = spacing * np.arange(ncentres)
    return _expand(sites, exps)


def slab(nx, ny, nz, seed, spacing=SPACING, jitter=0.2, exps=CHAIN_EXPONENTS):
    rng = np.random.default_rng(seed)
    g = np.array([(x, y, z) for x in range(nx) for y in range(ny) for z in range(nz)],
                 dtype=np.float64) * spacing
    g += rng.uniform(-jitter, jitter, size=g.shape)
    return _expand(g, exps)


def random_densities(n, m, seed, scale=1.0 / 40.0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, n, n)) * scale


def orthonormal(n, seed):
    rng = np.random.default_rng(seed)
    q, r = np.linalg.qr(rng.standard_normal((n, n)))
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s[None, :]


def transition_densities(n, m, n_occ, seed_c, seed_w):
    n_occ = int(min(n_occ, n // 2))
    C = orthonormal(n, seed_c)
    Co, Cv = C[:, :n_occ], C[:, n_occ:]
    nv = n - n_occ
    rng = np.random.default_rng(seed_w)
    W = rng.standard_normal((m, n_occ, nv)) / np.sqrt(n_occ * nv)
    return np.ascontiguousarray(np.einsum("pi,mia,qa->mpq", Co, W, Cv, optimize=True))


def esmf_state(n, n_occ, seed, sigma_norm=0.3, c0=0.9, mult_scale=0.05):
    """A seeded ESMF state for the nine-density terms (the matrices of the
    paper's notation table): V = U^T C drawn orthogonal (rows sign-fixed),
    Theta = its first N_o rows, Gamma the other N_v = n - N_o rows; sigma
    Gaussian with Frobenius norm sigma_norm; c0 given, N2 = c0^2 + 2|sigma|^2;
    the multipliers mu [N_o, N_v], R [N_o, n], Phi [N_v, n] Gaussian with
    entries of size mult_scale; G a symmetric one-electron matrix.  Returns a
    dict of float64 arrays and scalars."""
    n_occ = int(n_occ)
    nv = n - n_occ
    V = orthonormal(n, seed).T
    rng = np.random.default_rng(seed + 1)
    sigma = rng.standard_normal((n_occ, nv))
    sigma *= sigma_norm / np.linalg.norm(sigma)
    mu = rng.standard_normal((n_occ, nv)) * mult_scale
    R = rng.standard_normal((n_occ, n)) * mult_scale
    Phi = rng.standard_normal((nv, n)) * mult_scale
    # a symmetric stand-in for the one-electron matrix (core Hamiltonian):
    # negative diagonal, decaying couplings
    Gr = rng.standard_normal((n, n)) * 0.1
    G = 0.5 * (Gr + Gr.T) - np.diag(rng.uniform(0.5, 2.0, n))
    return dict(theta=np.ascontiguousarray(V[:n_occ]), gamma=np.ascontiguousarray(V[n_occ:]),
                sigma=sigma, mu=mu, R=R, Phi=Phi, c0=float(c0),
                n2=float(c0 * c0 + 2.0 * np.sum(sigma * sigma)), G=G)


# Cartesian components of a shell of angular momentum l (l + m + n = l).
CART_COMPONENTS = {
    0: [(0, 0, 0)],
    1: [(1, 0, 0), (0, 1, 0), (0, 0, 1)],
    2: [(2, 0, 0), (1, 1, 0), (1, 0, 1), (0, 2, 0), (0, 1, 1), (0, 0, 2)],
}
# Shells (l, exponent) on every site of the s/p/d workloads: two s, two p and
# one d primitive shell, the shape of a split-valence set with polarisation
# (14 Cartesian functions per site).
SPD_SHELLS = ((0, 1.6), (0, 0.35), (1, 0.9), (1, 0.25), (2, 0.8))


def cart_basis(sites, shells=SPD_SHELLS):
    """Every shell on every site, expanded into its Cartesian components.
    Returns (centers [N, 3], exponents [N], lmn [N, 3] int32)."""
    cen, al, lmn = [], [], []
    for site in np.asarray(sites, dtype=np.float64):
        for l, a in shells:
            for comp in CART_COMPONENTS[l]:
                cen.append(site)
                al.append(a)
                lmn.append(comp)
    return np.array(cen), np.array(al), np.array(lmn, dtype=np.int32)


def spd_chain(nsites, spacing=SPACING):
    sites = np.zeros((nsites, 3))
    sites[:, 0] = spacing * np.arange(nsites)
    return cart_basis(sites)


def spd_box(nsites, seed, box=5.0):
    return cart_basis(np.random.default_rng(seed).uniform(0.0, box, (nsites, 3)))


# Contracted shells (l, [(exponent, coefficient of the normalised
# primitive), ...]) on every site of the contracted workloads: a three-
# primitive s, a one-primitive s, a two-primitive p and a one-primitive d
# shell, the shape of a split-valence set with polarisation (the
# coefficients are of the kind such sets carry, not taken from one).
CONTRACTED_SHELLS = (
    (0, ((3.4, 0.16), (0.62, 0.54), (0.17, 0.44))),
    (0, ((0.12, 1.0),)),
    (1, ((0.9, 0.42), (0.25, 0.71))),
    (2, ((0.8, 1.0),)),
)


def contracted_basis(sites, shells=CONTRACTED_SHELLS):
    """Every contracted shell on every site, one function per Cartesian
    component.  Returns (centers [N, 3], lmn [N, 3], prim_offset [N+1],
    prim_exp [P], prim_coef [P])."""
    cen, lmn, off, pe, pc = [], [], [0], [], []
    for site in np.asarray(sites, dtype=np.float64):
        for l, prims in shells:
            for comp in CART_COMPONENTS[l]:
                cen.append(site)
                lmn.append(comp)
                for e, c in prims:
                    pe.append(e)
                    pc.append(c)
                off.append(len(pe))
    return (np.array(cen), np.array(lmn, dtype=np.int32), np.array(off, dtype=np.int32), np.array(pe),
            np.array(pc))


def config1():
    """40 s functions in a 10 bohr box, m=4 random densities, no screening."""
    c, a = random_box(40, seed=1)
    return dict(name="box40", centers=c, alpha=a, tau=0.0,
                D=random_densities(40, 4, seed=101))


def config2():
    """Chain of 200 centres (N=400), m=8 transition densities, tau=1e-10."""
    c, a = chain(200)
    return dict(name="chain400", centers=c, alpha=a, tau=1e-10,
                D=transition_densities(400, 8, 40, 202, 203))


def config3():
    """25x10x2 jittered slab (N=1000), m=8 transition densities, tau=1e-10."""
    c, a = slab(25, 10, 2, seed=301)
    return dict(name="slab1000", centers=c, alpha=a, tau=1e-10,
                D=transition_densities(1000, 8, 40, 302, 303))


def config3_deep():
    """10x10x5 jittered slab (N=1000), m=8 transition densities, tau=1e-10:
    three times slab1000's screened quartets, whose FP64 store would not fit
    one GPU's HBM (the integral-direct workload)."""
    c, a = slab(10, 10, 5, seed=305)
    return dict(name="slab10x10x5", centers=c, alpha=a, tau=1e-10,
                D=transition_densities(1000, 8, 40, 306, 307))


def batch_workload(nmol=64, seed0=401, nmin=25, nmax=300, mmin=2, mmax=10):
    """Independent chain molecules: N = 2 N_c with N_c ~ U{nmin..nmax},
    m ~ U{mmin..mmax}, N_o = min(40, N/2), tau = 1e-10."""
    mols = []
    for i in range(nmol):
        rng = np.random.default_rng(seed0 + i)
        nc = int(rng.integers(nmin, nmax + 1))
        m = int(rng.integers(mmin, mmax + 1))
        c, a = chain(nc)
        n = a.shape[0]
        D = transition_densities(n, m, min(40, n // 2), seed0 + 1000 + i, seed0 + 2000 + i)
        mols.append(dict(name=f"chain{n}_m{m}", centers=c, alpha=a, tau=1e-10, D=D))
    return mols


def serving_sessions(nsess=32, seed0=501, nmin=100, nmax=1500, iters=20):
    """Concurrent synthetic ESMF optimisations: each a chain or a two-layer slab
    (nx x 10 x 2, N rounded to a multiple of 40) with probability 1/2,
    N ~ U[nmin, nmax], m in {4, 8}.  Densities are drawn per iteration by
    ``session_density``."""
    out = []
    for i in range(nsess):
        rng = np.random.default_rng(seed0 + i)
        kind = "chain" if rng.random() < 0.5 else "slab"
        n = int(rng.integers(nmin, nmax + 1))
        m = int(rng.choice([4, 8]))
        if kind == "chain":
            c, a = chain(max(n // 2, 1))
        else:
            nx = max(1, int(round(n / 40.0)))
            c, a = slab(nx, 10, 2, seed=seed0 + 100 + i)
        out.append(dict(name=f"s{i}_{kind}{a.shape[0]}_m{m}", kind=kind, centers=c, alpha=a,
                        tau=1e-10, m=m, iters=iters, seed=seed0 + i))
    return out


def session_density(sess, it):
    n = sess["alpha"].shape[0]
    return transition_densities(n, sess["m"], min(40, n // 2), sess["seed"] + 7000,
                                sess["seed"] + 9000 + 131 * it)
