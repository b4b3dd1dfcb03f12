"""Galerkin coarse operator D_c = R D P as a 9-point stencil.  TEST INFRASTRUCTURE ONLY.

Paper, Sec. 2 (V-cycle, third step): the coarse problem uses the operator
R A P.  Sec. 4 (last paragraph): coarsening the unsquared operator keeps a
one-hop stencil -- with blocks spanning all of the fifth dimension and D
nearest-neighbour in 4D, a coarse site couples only to itself and its eight
4D neighbours.

Definition: (D_c)[(B,i),(B',j)] = < Vhat_(B,i), D Vhat_(B',j) >, stored as
Dc[B][d] (2Nv x 2Nv) with d = 0 the block itself, d = 1+2mu the block B+mu and
d = 2+2mu the block B-mu, so that (D_c y)(B) = sum_d Dc[B][d] y(B + delta_d)
with periodic coarse wrap.

Reading that keeps aliased extents exact (coarse extent 1 or 2, where B+mu
and B-mu, or B itself, coincide): a fine hop from x to x+mu belongs to
d = +mu exactly when x lies on the upper face of its block
(x_mu mod b_mu = b_mu - 1); a hop from x to x-mu belongs to d = -mu exactly
when x lies on the lower face (x_mu mod b_mu = 0).  Everything else (the
diagonal, the fifth-dimension hops and block-interior hops) is d = 0.
"""

from __future__ import annotations

import numpy as np

from . import dwf as _dwf
from .transfer import coarse_dims, prolong, restrict


def _face_mask(L, block, mu: int, upper: bool) -> np.ndarray:
    """Boolean (T,Z,Y,X) mask of sites on the upper/lower block face in direction mu."""
    Lx, Ly, Lz, Lt = L
    coords = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    xmu = coords[3 - mu]
    b = block[mu]
    return (xmu % b == b - 1) if upper else (xmu % b == 0)


def face_hop(psi: np.ndarray, U: np.ndarray, L, block, mu: int, upper: bool,
             bc=(1, 1, 1, 1), dagger: bool = False) -> np.ndarray:
    """The single hop of D (or D^+) in direction +mu or -mu, kept only on the block face."""
    sgn = -1.0 if not dagger else 1.0
    Umu = U[..., mu, :, :]
    if upper:
        h = _dwf.spin_mul(_dwf.I4 + sgn * _dwf.GAMMA[mu],
                          _dwf.colour_mul(Umu, _dwf.shift(psi, mu, +1, bc)))
    else:
        h = _dwf.spin_mul(_dwf.I4 - sgn * _dwf.GAMMA[mu],
                          _dwf.shift(_dwf.colour_mul(_dwf.dagger3(Umu), psi), mu, -1, bc))
    m = _face_mask(L, block, mu, upper)
    return -0.5 * h * m[..., None, None, None]


def _unit_coarse(Lc, Nv: int, chi: int, k: int) -> np.ndarray:
    c = np.zeros(tuple(Lc[::-1]) + (2, Nv), dtype=np.complex128)
    c[..., chi, k] = 1.0
    return c


def build_coarse_op(Vhat: np.ndarray, U: np.ndarray, M5: float, mf: float, block,
                    bc=(1, 1, 1, 1)) -> np.ndarray:
    """Dc with shape (Tc, Zc, Yc, Xc, 9, 2Nv, 2Nv); row/column index chi*Nv + k.

    Column j of Dc[B][d] is the restriction to block B of D_d applied to the
    prolongation of the coarse vector that is 1 in component j on every coarse
    site; D_d only reads block B + delta_d, so this isolates that block.
    """
    Nv = Vhat.shape[0]
    T, Zd, Y, X = Vhat.shape[1:5]
    L = (X, Y, Zd, T)
    Lc = coarse_dims(L, block)
    n2 = 2 * Nv
    Dc = np.zeros(tuple(Lc[::-1]) + (9, n2, n2), dtype=np.complex128)
    for chi in range(2):
        for k in range(Nv):
            j = chi * Nv + k
            pe = prolong(_unit_coarse(Lc, Nv, chi, k), Vhat, block)
            full = _dwf.apply_dwf(pe, U, M5, mf, bc)
            rest = full.copy()
            for mu in range(4):
                for upper, d in ((True, 1 + 2 * mu), (False, 2 + 2 * mu)):
                    part = face_hop(pe, U, L, block, mu, upper, bc)
                    rest -= part
                    Dc[..., d, :, j] = restrict(part, Vhat, block).reshape(Dc.shape[:4] + (n2,))
            Dc[..., 0, :, j] = restrict(rest, Vhat, block).reshape(Dc.shape[:4] + (n2,))
    return Dc


def _coarse_shift(c: np.ndarray, mu: int, sign: int) -> np.ndarray:
    """g(B) = c(B + sign*mu_hat), periodic; arrays ordered (T, Z, Y, X, ...)."""
    return np.roll(c, -sign, axis=3 - mu)


def apply_coarse(c: np.ndarray, Dc: np.ndarray, dagger: bool = False) -> np.ndarray:
    """y(B) = sum_d Dc[B][d] c(B + delta_d)  (or the adjoint stencil when dagger).

    c has shape (Tc,Zc,Yc,Xc, 2, Nv); the flat coarse index is chi*Nv + k.
    The adjoint uses (D_c^+)(B, B+delta) = Dc[B+delta][opposite d]^+.
    """
    shp = c.shape
    v = c.reshape(shp[:4] + (-1,))
    y = np.zeros_like(v)
    if not dagger:
        y += np.einsum("...ij,...j->...i", Dc[..., 0, :, :], v)
        for mu in range(4):
            y += np.einsum("...ij,...j->...i", Dc[..., 1 + 2 * mu, :, :], _coarse_shift(v, mu, +1))
            y += np.einsum("...ij,...j->...i", Dc[..., 2 + 2 * mu, :, :], _coarse_shift(v, mu, -1))
    else:
        DcH = np.conj(np.swapaxes(Dc, -1, -2))
        y += np.einsum("...ij,...j->...i", DcH[..., 0, :, :], v)
        for mu in range(4):
            # output B reads input at B+mu through the block stored at B+mu for direction -mu
            y += np.einsum("...ij,...j->...i", _coarse_shift(DcH[..., 2 + 2 * mu, :, :], mu, +1),
                           _coarse_shift(v, mu, +1))
            y += np.einsum("...ij,...j->...i", _coarse_shift(DcH[..., 1 + 2 * mu, :, :], mu, -1),
                           _coarse_shift(v, mu, -1))
    return y.reshape(shp)


class Coarse:
    """D_c bundle with an application counter."""

    def __init__(self, Dc: np.ndarray):
        self.Dc = Dc
        self.napply = 0

    def __call__(self, c):
        self.napply += 1
        return apply_coarse(c, self.Dc)

    def dag(self, c):
        self.napply += 1
        return apply_coarse(c, self.Dc, dagger=True)
