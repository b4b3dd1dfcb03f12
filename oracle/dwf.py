"""Shamir domain-wall operator, FP64 reference.  TEST INFRASTRUCTURE ONLY.

The paper (Sec. 2, fifth-dimension paragraph; Sec. 4) describes D as a 5D
nearest-neighbour operator -- one site couples to itself and its ten unit
neighbours -- with low modes bound to the two walls by chirality, but never
writes it.  The reading used here is the standard Shamir form:

    (D psi)(x,s) = (D_W psi)(x,s) + psi(x,s) - P_- psi(x,s+1) - P_+ psi(x,s-1)
    with the walls closed by the quark mass:
        P_- psi(x,Ls) := -m_f P_- psi(x,0),   P_+ psi(x,-1) := -m_f P_+ psi(x,Ls-1)
    (D_W psi)(x,s) = (4 - M5) psi(x,s)
        - 1/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu,s) + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu,s) ]
    P_+- = (1 +- g_5)/2.

Gamma matrices are in the chiral basis: g_k = [[0, -i s_k], [i s_k, 0]] for
k = x, y, z and g_t = [[0, 1], [1, 0]], so g_5 = g_x g_y g_z g_t = diag(1,1,-1,-1):
P_+ keeps spins {0,1}, P_- keeps spins {2,3}.

Boundary conditions: periodic; ``bc[mu] = -1`` multiplies every hop that crosses
the lattice boundary in direction mu.

The adjoint is written out term by term (it is not obtained from the
gamma_5 R_5 symmetry, which the tests check separately).

Field shapes: psi (Lt, Lz, Ly, Lx, Ls, 4, 3); U (Lt, Lz, Ly, Lx, 4, 3, 3).
"""

from __future__ import annotations

import numpy as np

_s1 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_s2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_s3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)
_Z2 = np.zeros((2, 2), dtype=np.complex128)
_I2 = np.eye(2, dtype=np.complex128)

GAMMA = np.array(
    [np.block([[_Z2, -1j * s], [1j * s, _Z2]]) for s in (_s1, _s2, _s3)]
    + [np.block([[_Z2, _I2], [_I2, _Z2]])]
)
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
I4 = np.eye(4, dtype=np.complex128)
PPLUS = 0.5 * (I4 + GAMMA5)
PMINUS = 0.5 * (I4 - GAMMA5)


def spin_mul(G: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """Apply a 4x4 spin matrix to every site: out[..., i, c] = G[i, j] psi[..., j, c]."""
    return np.matmul(G, psi)


def colour_mul(Umu: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """out(x, s, i) = Umu(x) @ psi(x, s, i); Umu (T,Z,Y,X,3,3), psi (T,Z,Y,X,Ls,4,3)."""
    T, Zd, Y, X, Ls, ns, nc = psi.shape
    flat = psi.reshape(T, Zd, Y, X, Ls * ns, nc)
    return np.matmul(flat, np.swapaxes(Umu, -1, -2)).reshape(psi.shape)


def dagger3(M: np.ndarray) -> np.ndarray:
    return np.conj(np.swapaxes(M, -1, -2))


def shift(f: np.ndarray, mu: int, sign: int, bc=(1, 1, 1, 1)) -> np.ndarray:
    """Neighbour field g(x) = f(x + sign*mu_hat), with bc[mu] on boundary-crossing hops.

    Arrays are ordered (t, z, y, x, ...), so direction mu lives on axis 3 - mu.
    """
    axis = 3 - mu
    g = np.roll(f, -sign, axis=axis)
    if bc[mu] != 1:
        L = f.shape[axis]
        idx = [slice(None)] * f.ndim
        idx[axis] = L - 1 if sign > 0 else 0
        g[tuple(idx)] *= bc[mu]
    return g


def wilson_hop(psi: np.ndarray, U: np.ndarray, bc=(1, 1, 1, 1), dagger: bool = False) -> np.ndarray:
    """The hopping part of D_W (or of its adjoint), applied on every s-slice."""
    out = np.zeros_like(psi)
    sgn = -1.0 if not dagger else 1.0
    for mu in range(4):
        Umu = U[..., mu, :, :]
        fwd = colour_mul(Umu, shift(psi, mu, +1, bc))             # U_mu(x) psi(x+mu)
        bwd = shift(colour_mul(dagger3(Umu), psi), mu, -1, bc)    # U_mu(x-mu)^+ psi(x-mu)
        out += spin_mul(I4 + sgn * GAMMA[mu], fwd)
        out += spin_mul(I4 - sgn * GAMMA[mu], bwd)
    return -0.5 * out


def fifth_hop(psi: np.ndarray, mf: float, dagger: bool = False) -> np.ndarray:
    """The fifth-dimension hop with the mass-closed walls (or its adjoint).

    D:   -P_- psi(s+1) - P_+ psi(s-1), walls +m_f P_- psi(0) at s=Ls-1 and
         +m_f P_+ psi(Ls-1) at s=0.
    D^+: the roles of P_+ and P_- are exchanged.
    """
    Ls = psi.shape[4]
    P_up, P_dn = (PMINUS, PPLUS) if not dagger else (PPLUS, PMINUS)
    c_up = -np.ones(Ls)
    c_up[Ls - 1] = mf          # psi(s+1) at s = Ls-1 is psi(0) across the wall
    c_dn = -np.ones(Ls)
    c_dn[0] = mf               # psi(s-1) at s = 0 is psi(Ls-1) across the wall
    up = spin_mul(P_up, np.roll(psi, -1, axis=4)) * c_up[:, None, None]
    dn = spin_mul(P_dn, np.roll(psi, 1, axis=4)) * c_dn[:, None, None]
    return up + dn


def apply_dwf(psi: np.ndarray, U: np.ndarray, M5: float, mf: float,
              bc=(1, 1, 1, 1), dagger: bool = False) -> np.ndarray:
    """D psi (or D^+ psi) for the Shamir operator above."""
    return ((5.0 - M5) * psi + wilson_hop(psi, U, bc, dagger) + fifth_hop(psi, mf, dagger))


def gamma5_R5(psi: np.ndarray) -> np.ndarray:
    """(g_5 R_5 psi)(s) = g_5 psi(Ls-1-s)."""
    return spin_mul(GAMMA5, psi[..., ::-1, :, :])


def apply_wilson(psi4: np.ndarray, U: np.ndarray, mass: float, bc=(1, 1, 1, 1)) -> np.ndarray:
    """Textbook 4D Wilson operator (4 + m) - 1/2 sum hops, on fields (T,Z,Y,X,4,3).

    Used only to pin the Ls = 1 reduction of D.
    """
    psi5 = psi4[..., None, :, :]
    return ((4.0 + mass) * psi5 + wilson_hop(psi5, U, bc))[..., 0, :, :]


class DWF:
    """Convenience bundle of (U, M5, m_f, bc) with the operator and its adjoint."""

    def __init__(self, U: np.ndarray, M5: float, mf: float, bc=(1, 1, 1, 1)):
        self.U = U
        self.M5 = float(M5)
        self.mf = float(mf)
        self.bc = tuple(int(b) for b in bc)
        self.napply = 0

    def __call__(self, psi: np.ndarray) -> np.ndarray:
        self.napply += 1
        return apply_dwf(psi, self.U, self.M5, self.mf, self.bc, False)

    def dag(self, psi: np.ndarray) -> np.ndarray:
        self.napply += 1
        return apply_dwf(psi, self.U, self.M5, self.mf, self.bc, True)
