"""Two-dimensional U(1) domain-wall operator and its squared multigrid.
TEST INFRASTRUCTURE ONLY.

The paper's first test problem (Sec. 3, Fig. 2): a quenched U(1) gauge field
in two dimensions, 20^2 x 8, a null space of 16 vectors, blocks of 4^2 sites
spanning the fifth dimension, quark masses 0.01 .. 0.10, the multigrid
against CG on the squared operator, cost counted in applications of the
squared fine operator, and the coarse residual as a function of coarse
applications.  The paper writes none of the operator; the reading is the
4D one of ``dwf`` taken to two dimensions:

    (D psi)(x,s) = (3 - M5) psi(x,s)
        - 1/2 sum_{mu = x, y} [ (1 - g_mu) U_mu(x) psi(x+mu,s)
                               + (1 + g_mu) conj(U_mu(x-mu)) psi(x-mu,s) ]
        - P_- psi(x,s+1) - P_+ psi(x,s-1),
    walls closed by the quark mass as in 4D:
        P_- psi(x,Ls) := -m_f P_- psi(x,0),  P_+ psi(x,-1) := -m_f P_+ psi(x,Ls-1).

(3 - M5 is the 2D Wilson diagonal 2 - M5 plus the 1 of the fifth dimension.)
Dirac matrices: g_x = sigma_1, g_y = sigma_2, g_5 = sigma_3 = -i g_x g_y, so
P_+ keeps spin 0 and P_- spin 1.  The adjoint is written out term by term.

Everything else is the squared method of ``squared`` on this operator: the
basis from CG on D^+D v = 0, split by chirality (the spin index) and
orthonormalised per block; A_c = P^+ D^+D P; the V-cycle of Sec. 2 on
D^+D preconditioning flexible GCR on D x = b.  With blocks of extent >= 2,
A_c couples a coarse site to the 9 sites ``OFFSETS2`` (self, four unit
neighbours, four diagonal neighbours), for the same reason as the 33 in 4D.

Shapes: psi (Ly, Lx, Ls, 2); U (Ly, Lx, 2) unit complex numbers; coarse
vectors (Yc, Xc, 2, Nv); the stencil (Yc, Xc, 9, 2Nv, 2Nv).
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np

from . import setup as _setup
from . import solvers as _sol
from . import squared as _sq
from . import transfer as _tr

SIGMA1 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
SIGMA2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
SIGMA3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)
GAMMA2 = np.array([SIGMA1, SIGMA2])
GAMMA5_2 = SIGMA3
I2 = np.eye(2, dtype=np.complex128)
PPLUS2 = 0.5 * (I2 + GAMMA5_2)
PMINUS2 = 0.5 * (I2 - GAMMA5_2)


def spin_mul2(G: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """out[..., i] = G[i, j] psi[..., j]."""
    return np.einsum("ij,...j->...i", G, psi)


def shift2(f: np.ndarray, mu: int, sign: int, bc=(1, 1)) -> np.ndarray:
    """g(x) = f(x + sign*mu_hat); arrays are (y, x, ...), so mu lives on axis 1 - mu."""
    axis = 1 - mu
    g = np.roll(f, -sign, axis=axis)
    if bc[mu] != 1:
        L = f.shape[axis]
        idx = [slice(None)] * f.ndim
        idx[axis] = L - 1 if sign > 0 else 0
        g[tuple(idx)] *= bc[mu]
    return g


def wilson_hop2(psi: np.ndarray, U: np.ndarray, bc=(1, 1), dagger: bool = False) -> np.ndarray:
    out = np.zeros_like(psi)
    sgn = -1.0 if not dagger else 1.0
    for mu in range(2):
        Umu = U[..., mu][..., None, None]
        fwd = Umu * shift2(psi, mu, +1, bc)                 # U_mu(x) psi(x+mu)
        bwd = shift2(np.conj(Umu) * psi, mu, -1, bc)        # conj(U_mu(x-mu)) psi(x-mu)
        out += spin_mul2(I2 + sgn * GAMMA2[mu], fwd)
        out += spin_mul2(I2 - sgn * GAMMA2[mu], bwd)
    return -0.5 * out


def fifth_hop2(psi: np.ndarray, mf: float, dagger: bool = False) -> np.ndarray:
    """-P_- psi(s+1) - P_+ psi(s-1) with the walls closed by +m_f (adjoint: the
    projectors exchanged)."""
    Ls = psi.shape[2]
    P_up, P_dn = (PMINUS2, PPLUS2) if not dagger else (PPLUS2, PMINUS2)
    c_up = -np.ones(Ls)
    c_up[Ls - 1] = mf
    c_dn = -np.ones(Ls)
    c_dn[0] = mf
    up = spin_mul2(P_up, np.roll(psi, -1, axis=2)) * c_up[:, None]
    dn = spin_mul2(P_dn, np.roll(psi, 1, axis=2)) * c_dn[:, None]
    return up + dn


def apply_dwf2(psi: np.ndarray, U: np.ndarray, M5: float, mf: float, bc=(1, 1),
               dagger: bool = False) -> np.ndarray:
    """D psi (or D^+ psi); psi may carry leading axes."""
    if psi.ndim > 4:
        return np.array([apply_dwf2(p, U, M5, mf, bc, dagger) for p in psi])
    return (3.0 - M5) * psi + wilson_hop2(psi, U, bc, dagger) + fifth_hop2(psi, mf, dagger)


def gamma5_R5_2(psi: np.ndarray) -> np.ndarray:
    """(g_5 R_5 psi)(s) = g_5 psi(Ls-1-s)."""
    return spin_mul2(GAMMA5_2, psi[..., ::-1, :])


class DWF2:
    """(U, M5, m_f, bc) with the 2D operator and its adjoint; counts applications."""

    def __init__(self, U: np.ndarray, M5: float, mf: float, bc=(1, 1)):
        self.U = U
        self.M5 = float(M5)
        self.mf = float(mf)
        self.bc = tuple(int(b) for b in bc)
        self.napply = 0

    def __call__(self, psi):
        self.napply += 1
        return apply_dwf2(psi, self.U, self.M5, self.mf, self.bc, False)

    def dag(self, psi):
        self.napply += 1
        return apply_dwf2(psi, self.U, self.M5, self.mf, self.bc, True)


# ---------------------------------------------------------------- transfer

def block_split2(f: np.ndarray, block) -> np.ndarray:
    """View (..., Ly, Lx, Ls, 2) as (..., Yc, Xc, by, bx, Ls, 2)."""
    bx, by = block
    lead = f.shape[:-4]
    Ly, Lx, Ls, ns = f.shape[-4:]
    if Ly % by or Lx % bx:
        raise ValueError("block does not divide the lattice")
    n = len(lead)
    g = f.reshape(lead + (Ly // by, by, Lx // bx, bx, Ls, ns))
    return g.transpose(list(range(n)) + [n + i for i in (0, 2, 1, 3, 4, 5)])


def block_merge2(g: np.ndarray) -> np.ndarray:
    n = g.ndim - 6
    lead = g.shape[:n]
    Yc, Xc, by, bx, Ls, ns = g.shape[n:]
    perm = list(range(n)) + [n + i for i in (0, 2, 1, 3, 4, 5)]
    return g.transpose(perm).reshape(lead + (Yc * by, Xc * bx, Ls, ns))


def build_basis2d(V: np.ndarray, block) -> np.ndarray:
    """Chirality split (spin 0 | spin 1) and Gram-Schmidt (twice) per block."""
    Nv = V.shape[0]
    g = block_split2(V, block)                       # (Nv, Yc, Xc, by, bx, Ls, 2)
    out = np.zeros_like(g)
    for chi in range(2):
        part = g[..., chi]                           # (Nv, Yc, Xc, by, bx, Ls)
        Yc, Xc = part.shape[1:3]
        panels = np.moveaxis(part.reshape(Nv, Yc, Xc, -1), 0, -1)   # (Yc, Xc, rows, Nv)
        Q = _tr.orthonormalise_panels(panels)
        out[..., chi] = np.moveaxis(Q, -1, 0).reshape(part.shape)
    return np.ascontiguousarray(block_merge2(out))


def restrict2d(x: np.ndarray, Vhat: np.ndarray, block) -> np.ndarray:
    """c[B, chi, k] = sum over block B, all s, spin chi of conj(Vhat_k) x."""
    gv = block_split2(Vhat, block)
    gx = block_split2(x, block)
    Nv = Vhat.shape[0]
    Yc, Xc = gx.shape[:2]
    out = np.empty((Yc, Xc, 2, Nv), dtype=np.complex128)
    for chi in range(2):
        prod = np.conj(gv[..., chi]) * gx[None, ..., chi]
        out[..., chi, :] = np.moveaxis(prod.reshape(Nv, Yc, Xc, -1).sum(-1), 0, -1)
    return out


def prolong2d(c: np.ndarray, Vhat: np.ndarray, block) -> np.ndarray:
    """x = sum over (chi, k) of Vhat_k on spin chi times c[B, chi, k]."""
    gv = block_split2(Vhat, block)
    g = np.zeros(gv.shape[1:], dtype=np.complex128)
    for chi in range(2):
        coef = np.moveaxis(c[..., chi, :], -1, 0)             # (Nv, Yc, Xc)
        g[..., chi] = np.einsum("kYX,kYXabs->YXabs", coef, gv[..., chi])
    return block_merge2(g)


# ---------------------------------------------------------------- coarse operator

OFFSETS2 = [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (1, -1), (-1, 1), (-1, -1)]


def _coarse_roll2(c: np.ndarray, o) -> np.ndarray:
    """g(X) = c(X + o), periodic, arrays (Yc, Xc, ...)."""
    g = c
    for mu in range(2):
        if o[mu]:
            g = np.roll(g, -o[mu], axis=1 - mu)
    return g


def build_sq_coarse_op2d(Vhat: np.ndarray, U: np.ndarray, M5: float, mf: float, block,
                         bc=(1, 1)) -> np.ndarray:
    """A_c column by column, R D^+D P e_(B, j), read off on the 9 sites B - o.

    Needs coarse extents >= 3 and block extents >= 2; anything the column
    reaches beyond those 9 sites raises.
    """
    Nv = Vhat.shape[0]
    Ly, Lx = Vhat.shape[1:3]
    Yc, Xc = Ly // block[1], Lx // block[0]
    if min(Yc, Xc) < 3 or min(block) < 2:
        raise ValueError("the probed stencil needs coarse extents >= 3 and block extents >= 2")
    n2 = 2 * Nv
    Ac = np.zeros((Yc, Xc, len(OFFSETS2), n2, n2), dtype=np.complex128)
    for B in np.ndindex(Yc, Xc):
        for chi in range(2):
            for k in range(Nv):
                e = np.zeros((Yc, Xc, 2, Nv), dtype=np.complex128)
                e[B + (chi, k)] = 1.0
                pe = prolong2d(e, Vhat, block)
                w = restrict2d(apply_dwf2(apply_dwf2(pe, U, M5, mf, bc), U, M5, mf, bc, dagger=True),
                               Vhat, block).reshape(Yc, Xc, n2)
                seen = np.zeros((Yc, Xc), dtype=bool)
                j = chi * Nv + k
                for oi, o in enumerate(OFFSETS2):
                    Xs = ((B[0] - o[1]) % Yc, (B[1] - o[0]) % Xc)   # y(B - o) = Ac[B - o][o] e(B)
                    Ac[Xs + (oi, slice(None), j)] = w[Xs]
                    seen[Xs] = True
                rest = np.abs(w[~seen]).max() if (~seen).any() else 0.0
                if rest > 1e-12 * np.abs(w).max():
                    raise ValueError("A_c column reaches beyond the 9-site stencil")
    return Ac


def apply_sq_coarse2d(c: np.ndarray, Ac: np.ndarray) -> np.ndarray:
    """y(X) = sum_o Ac[X][o] c(X + o); c has shape (Yc, Xc, 2, Nv)."""
    shp = c.shape
    v = c.reshape(shp[:2] + (-1,))
    y = np.zeros_like(v)
    for oi, o in enumerate(OFFSETS2):
        y += np.einsum("...ij,...j->...i", Ac[..., oi, :, :], _coarse_roll2(v, o))
    return y.reshape(shp)


class ExplicitCoarse2D:
    """A_c applied as R D^+D P (the definition; any extents); counts applications."""

    def __init__(self, A, Vhat, block):
        self.A, self.Vhat, self.block = A, Vhat, block
        self.napply = 0

    def __call__(self, c):
        self.napply += 1
        return restrict2d(self.A.dag(self.A(prolong2d(c, self.Vhat, self.block))), self.Vhat, self.block)


class StencilCoarse2D:
    def __init__(self, Ac):
        self.Ac = Ac
        self.napply = 0

    def __call__(self, c):
        self.napply += 1
        return apply_sq_coarse2d(c, self.Ac)


# ---------------------------------------------------------------- multigrid

class TwoLevelSquared2D(_sq.TwoLevelSquared):
    """The squared V-cycle of Sec. 2 with the 2D transfer; records the coarse
    CG iteration count of every cycle (the coarse-level cost of Fig. 2)."""

    def __init__(self, *args, **kw):
        super().__init__(*args, **kw)
        self.coarse_iters: List[int] = []

    def vcycle(self, g: np.ndarray) -> np.ndarray:
        if self.nu_pre > 0:
            x1, r1 = _sq.mr_hpd_steps(self.N, g, self.nu_pre)
        else:
            x1, r1 = np.zeros_like(g), g.copy()
        x2, it = _sq.cg(self.coarse, restrict2d(r1, self.Vhat, self.block), self.coarse_tol, self.coarse_maxiter)
        self.coarse_iters.append(it)
        xc = x1 + prolong2d(x2, self.Vhat, self.block)
        if self.nu_post > 0:
            x3, _ = _sq.mr_hpd_steps(self.N, g - self.N(xc), self.nu_post)
            return xc + x3
        return xc


@dataclass
class U1Params:
    block: tuple = (4, 4)
    nvec: int = 16
    sweeps: int = 1
    sweep0_iters: int = 100
    sweep_iters: int = 4
    nu_pre: int = 4
    nu_post: int = 4
    coarse_tol: float = 0.1
    coarse_maxiter: int = 200
    sweep0_check: int = 0


@dataclass
class U1MG:
    A: DWF2
    params: U1Params
    V: np.ndarray = None
    Vhat: np.ndarray = None
    coarse: object = None
    null_residuals: List[float] = None

    def rebuild(self, V: np.ndarray, stencil: bool = False):
        self.V = V
        self.Vhat = build_basis2d(V, self.params.block)
        if stencil:
            self.coarse = StencilCoarse2D(build_sq_coarse_op2d(self.Vhat, self.A.U, self.A.M5, self.A.mf,
                                                               self.params.block, self.A.bc))
        else:
            self.coarse = ExplicitCoarse2D(self.A, self.Vhat, self.params.block)

    def preconditioner(self) -> TwoLevelSquared2D:
        p = self.params
        return TwoLevelSquared2D(self.A, self.Vhat, p.block, self.coarse, p.coarse_tol, p.coarse_maxiter,
                                 p.nu_pre, p.nu_post)


def u1_setup(A: DWF2, V0: np.ndarray, params: U1Params, stencil: bool = False) -> U1MG:
    """Sweep 0: CG on D^+D v = 0 from each start, normalise, build; later
    sweeps: flexible GCR with the current multigrid on D x = 0 from each
    vector (sweep_iters steps), keep what is left, normalise, rebuild."""
    if V0.shape[0] != params.nvec:
        raise ValueError("expected nvec random starts")
    mg = U1MG(A, params, null_residuals=[])
    V = np.array([_setup.sweep0(A, v, params.sweep0_iters, params.sweep0_check) for v in V0])
    V = np.array([v / _sol.norm(v) for v in V])
    mg.rebuild(V, stencil)
    mg.null_residuals.append(float(np.median([_setup.null_residual(A, v) for v in V])))
    zero = np.zeros_like(V[0])
    for _ in range(params.sweeps - 1):
        M = mg.preconditioner()
        V = np.array([_sol.gcr_fixed(A, zero, v, params.sweep_iters, M=M)[0] for v in V])
        V = np.array([v / _sol.norm(v) for v in V])
        mg.rebuild(V, stencil)
        mg.null_residuals.append(float(np.median([_setup.null_residual(A, v) for v in V])))
    return mg


def u1_solve(mg: U1MG, b: np.ndarray, tol: float = 1e-10, maxiter: int = 200, restart: int = 8):
    """Flexible GCR on D x = b with the squared two-level preconditioner; returns
    (x, report, the preconditioner with its coarse iteration counts)."""
    M = mg.preconditioner()
    x, rep = _sol.gcr(mg.A, b, tol, maxiter, restart, M=M)
    return x, rep, M
