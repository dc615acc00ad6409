"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds input generators only: no part of the solver, the operator
or the loop estimators.  It feeds the HIP library and the CPU oracle the same
gauge field; random numbers that the method itself draws (the Z4 noise) are
not made here but by each side from the published SplitMix64 definition.

Gauge links stand in for the paper's 32^3 x 64 ensemble, which is not
available: i.i.d. near-identity SU(3) links U = exp(i eps H), with
H = sum_a h_a lambda_a / 2 traceless Hermitian, h_a ~ N(0, 1) (numpy PCG64
stream of the given seed), lambda_a the Gell-Mann matrices.
"""
import numpy as np

_GELL_MANN = np.zeros((8, 3, 3), dtype=np.complex128)
_GELL_MANN[0][0, 1] = _GELL_MANN[0][1, 0] = 1
_GELL_MANN[1][0, 1], _GELL_MANN[1][1, 0] = -1j, 1j
_GELL_MANN[2][0, 0], _GELL_MANN[2][1, 1] = 1, -1
_GELL_MANN[3][0, 2] = _GELL_MANN[3][2, 0] = 1
_GELL_MANN[4][0, 2], _GELL_MANN[4][2, 0] = -1j, 1j
_GELL_MANN[5][1, 2] = _GELL_MANN[5][2, 1] = 1
_GELL_MANN[6][1, 2], _GELL_MANN[6][2, 1] = -1j, 1j
_GELL_MANN[7] = np.diag([1, 1, -2]) / np.sqrt(3)


def volume(L):
    return int(np.prod(L))


def gauge_links(L, eps, seed, chunk=1 << 20):
    """Links U[mu, site, 3, 3] (complex128), site = x + Lx*(y + Ly*(z + Lz*t))."""
    V = volume(L)
    rng = np.random.Generator(np.random.PCG64(seed))
    h = rng.standard_normal((4 * V, 8))
    U = np.empty((4 * V, 3, 3), dtype=np.complex128)
    for a in range(0, 4 * V, chunk):
        b = min(a + chunk, 4 * V)
        H = np.einsum("na,aij->nij", h[a:b], _GELL_MANN / 2)
        w, Q = np.linalg.eigh(H)
        U[a:b] = (Q * np.exp(1j * eps * w)[:, None, :]) @ Q.conj().transpose(0, 2, 1)
    return U.reshape(4, V, 3, 3)


def unit_links(L):
    V = volume(L)
    U = np.zeros((4, V, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1
    return U


def random_su3(n, seed):
    """n Haar-ish random SU(3) matrices (QR of complex Gaussians, det fixed to 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Z = rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))
    Q, R = np.linalg.qr(Z)
    d = np.diagonal(R, axis1=1, axis2=2)
    Q = Q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(Q)
    return Q / (det ** (1.0 / 3.0))[:, None, None]


def gauge_transform(L, U, g):
    """U_mu(x) -> g(x) U_mu(x) g(x+mu)^dag (periodic neighbours)."""
    V = volume(L)
    out = np.empty_like(U)
    idx = np.arange(V)
    c = [idx % L[0], (idx // L[0]) % L[1], (idx // (L[0] * L[1])) % L[2],
         idx // (L[0] * L[1] * L[2])]
    for mu in range(4):
        cc = list(c)
        cc[mu] = (cc[mu] + 1) % L[mu]
        fwd = cc[0] + L[0] * (cc[1] + L[1] * (cc[2] + L[2] * cc[3]))
        out[mu] = g @ U[mu] @ g[fwd].conj().transpose(0, 2, 1)
    return out


def random_spinor(L, seed, n=None):
    """Gaussian complex spinor field(s) (V, 4, 3) or (n, V, 4, 3)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = ((n,) if n is not None else ()) + (volume(L), 4, 3)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# The lattice workloads of the method (kappa normalisation: eps = 2 kappa mu).
CONFIGS = {
    "c1": dict(L=(4, 4, 4, 8), eps_links=0.3, seed=101, kappa=0.124, two_kappa_mu=0.01),
    "c2": dict(L=(16, 16, 16, 32), eps_links=0.2, seed=102, kappa=0.124, two_kappa_mu=0.0028),
    "c3": dict(L=(32, 32, 32, 64), eps_links=0.15, seed=103, kappa=0.1245,
               two_kappa_mu=0.0014),
    "c4a": dict(L=(8, 8, 8, 16), eps_links=0.3, seed=1041, kappa=0.124, two_kappa_mu=0.005),
    "c4b": dict(L=(12, 12, 12, 24), eps_links=0.2, seed=1042, kappa=0.124,
                two_kappa_mu=0.005),
    "c4c": dict(L=(16, 16, 16, 32), eps_links=0.15, seed=1043, kappa=0.124,
                two_kappa_mu=0.005),
    "c5": dict(L=(32, 32, 32, 64), eps_links=0.2, seed=105, kappa=0.124, two_kappa_mu=0.0028),
}
NOISE_SEEDS = {"c1": 201, "c2": 202, "c3": 203}
