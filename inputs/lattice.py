"""Seeded gauge fields, sources and setup starting vectors.

Every generator draws from ``numpy.random.Generator(PCG64(seed))`` in canonical
index order, so the same seed gives the same array on any machine.

Gauge recipe (synthetic stand-in for a production ensemble): on every link draw
eight i.i.d. N(0,1) numbers h_a, form the traceless Hermitian matrix
``H = sum_a h_a lambda_a / 2`` with the Gell-Mann matrices, and set
``U = exp(i * eps * H)`` (computed through the eigendecomposition of H, so U is
unitary with unit determinant to rounding).  Optionally smooth with APE-style
steps: ``V = (1 - alpha) U + (alpha / 6) * (sum of the six staples)``, applied to
all links at once, then projected back to SU(3) by the polar factor
``W = V (V^+ V)^(-1/2)`` divided by the principal cube root of ``det W``.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Sequence, Tuple

import numpy as np


@dataclass(frozen=True)
class LatticeShape:
    """Extents of the 4D lattice (x, y, z, t) and of the fifth dimension."""

    L: Tuple[int, int, int, int]
    Ls: int

    @property
    def V4(self) -> int:
        return int(np.prod(self.L))

    @property
    def V5(self) -> int:
        return self.V4 * self.Ls


def fermion_shape(L: Sequence[int], Ls: int) -> Tuple[int, ...]:
    """Array shape of a canonical 5D fermion field: (Lt, Lz, Ly, Lx, Ls, 4, 3)."""
    Lx, Ly, Lz, Lt = L
    return (Lt, Lz, Ly, Lx, Ls, 4, 3)


def gauge_shape(L: Sequence[int]) -> Tuple[int, ...]:
    """Array shape of a canonical gauge field: (Lt, Lz, Ly, Lx, 4, 3, 3)."""
    Lx, Ly, Lz, Lt = L
    return (Lt, Lz, Ly, Lx, 4, 3, 3)


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3)."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam


def _expi_hermitian(H: np.ndarray, eps: float) -> np.ndarray:
    """exp(i*eps*H) for a stack of Hermitian matrices, via eigh."""
    w, Q = np.linalg.eigh(H)
    ph = np.exp(1j * eps * w)
    return np.einsum("...ij,...j,...kj->...ik", Q, ph, Q.conj())


def random_su3_field(L: Sequence[int], eps: float, seed: int) -> np.ndarray:
    """U = exp(i eps H) per link, H traceless Hermitian Gaussian (see module doc)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shp = gauge_shape(L)[:-2]  # (Lt, Lz, Ly, Lx, 4)
    h = rng.standard_normal(shp + (8,))
    H = np.einsum("...a,aij->...ij", h, gell_mann()) * 0.5
    return _expi_hermitian(H, eps)


def _shift(a: np.ndarray, mu: int, sign: int) -> np.ndarray:
    """Periodic neighbour field: returns f with f(x) = a(x + sign*mu_hat)."""
    axis = 3 - mu  # arrays are ordered (t, z, y, x, ...)
    return np.roll(a, -sign, axis=axis)


def _dag(m: np.ndarray) -> np.ndarray:
    return np.conj(np.swapaxes(m, -1, -2))


def _project_su3(V: np.ndarray) -> np.ndarray:
    """Polar projection W = V (V^+V)^(-1/2), then W / det(W)^(1/3) (principal)."""
    M = _dag(V) @ V
    w, Q = np.linalg.eigh(M)
    inv_sqrt = np.einsum("...ij,...j,...kj->...ik", Q, 1.0 / np.sqrt(w), Q.conj())
    W = V @ inv_sqrt
    det = np.linalg.det(W)
    return W / (det ** (1.0 / 3.0))[..., None, None]


def ape_smear(U: np.ndarray, steps: int, alpha: float = 0.5) -> np.ndarray:
    """APE-style smoothing with SU(3) projection, all links updated at once."""
    for _ in range(steps):
        Unew = np.empty_like(U)
        for mu in range(4):
            Umu = U[..., mu, :, :]
            stap = np.zeros_like(Umu)
            for nu in range(4):
                if nu == mu:
                    continue
                Unu = U[..., nu, :, :]
                # upper staple: U_nu(x) U_mu(x+nu) U_nu(x+mu)^+
                stap += Unu @ _shift(Umu, nu, +1) @ _dag(_shift(Unu, mu, +1))
                # lower staple: U_nu(x-nu)^+ U_mu(x-nu) U_nu(x-nu+mu)
                Unu_m = _shift(Unu, nu, -1)
                stap += _dag(Unu_m) @ _shift(Umu, nu, -1) @ _shift(_shift(Unu, nu, -1), mu, +1)
            Unew[..., mu, :, :] = _project_su3((1 - alpha) * Umu + (alpha / 6.0) * stap)
        U = Unew
    return U


def prepare_gauge(L: Sequence[int], eps: float, seed: int, ape_steps: int = 0,
                  alpha: float = 0.5) -> np.ndarray:
    """Seeded SU(3) field, optionally APE-smoothed; canonical complex128 layout."""
    U = random_su3_field(L, eps, seed)
    if ape_steps:
        U = ape_smear(U, ape_steps, alpha)
    return np.ascontiguousarray(U)


def gaussian_fermion(L: Sequence[int], Ls: int, seed: int, n: int | None = None) -> np.ndarray:
    """Gaussian complex field(s): Re, Im i.i.d. N(0,1) in canonical order.

    With ``n`` given, returns ``n`` fields stacked on a leading axis.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    shp = fermion_shape(L, Ls) if n is None else (n,) + fermion_shape(L, Ls)
    re = rng.standard_normal(shp)
    im = rng.standard_normal(shp)
    return re + 1j * im


def point_sources(L: Sequence[int], Ls: int, site=(0, 0, 0, 0)) -> np.ndarray:
    """The 12 spin-colour point sources of a 4D quark field, lifted to 5D.

    Source (alpha, a) is placed at 4D site ``site`` (x, y, z, t): spins 0,1
    (positive chirality) on the wall s = Ls-1, spins 2,3 on the wall s = 0, so
    that the 4D quark field built from the walls is the unit vector e_(alpha,a).
    Returns shape (12, Lt, Lz, Ly, Lx, Ls, 4, 3), index 3*alpha + a.
    """
    x, y, z, t = site
    out = np.zeros((12,) + fermion_shape(L, Ls), dtype=np.complex128)
    for alpha in range(4):
        s = Ls - 1 if alpha < 2 else 0
        for a in range(3):
            out[3 * alpha + a, t, z, y, x, s, alpha, a] = 1.0
    return out


def random_starts(L: Sequence[int], Ls: int, nvec: int, seed: int) -> np.ndarray:
    """Random starting vectors of the adaptive setup, shape (nvec, *fermion)."""
    return gaussian_fermion(L, Ls, seed, n=nvec)


def random_coarse_starts(Lc: Sequence[int], nv: int, n: int, seed: int) -> np.ndarray:
    """Random starting vectors on a coarse lattice (a third multigrid level's
    setup): shape (n, Lt_c, Lz_c, Ly_c, Lx_c, 2, nv), Re, Im i.i.d. N(0,1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shp = (n,) + tuple(Lc[::-1]) + (2, nv)
    return rng.standard_normal(shp) + 1j * rng.standard_normal(shp)


def random_gauge_transform(L: Sequence[int], seed: int, eps: float = 1.0) -> np.ndarray:
    """One random SU(3) matrix per 4D site, shape (Lt, Lz, Ly, Lx, 3, 3)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Lx, Ly, Lz, Lt = L
    h = rng.standard_normal((Lt, Lz, Ly, Lx, 8))
    H = np.einsum("...a,aij->...ij", h, gell_mann()) * 0.5
    return _expi_hermitian(H, eps)
