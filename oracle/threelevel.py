"""Three-level squared-operator multigrid.  TEST INFRASTRUCTURE ONLY.

Paper Sec. 2 (after the five steps of the V-cycle): the coarse solve of step
3 can itself be done by the same multigrid, recursively; Sec. 3 (Fig. 2
right) motivates it by the coarse operator's own critical slowing down.  The
two-level method here is ``squared`` (A = D^+ D, A_c = P^+ A P); this module
adds the level below A_c, written from the same definitions one level down:

* level-2 near-null vectors w_j of A_c: CG on A_c w = 0 from random coarse
  starts (the Krylov solver of Sec. 2's adaptive paragraph, applied to A_c);
* level-2 basis: each w_j split by the coarse chirality index (the first of
  the two axes of a coarse site's dof) and orthonormalised per block of
  coarse sites (thin QR with positive real diagonal), as ``transfer`` does
  on the fine level;
* R2 = W^+, P2 = W, A_cc = R2 A_c P2 (Hermitian positive definite; with
  blocks of extent >= 2 again a 33-offset stencil);
* level-2 cycle K2 on A_c e = f: nu minimal-residual steps on A_c, R2, CG on
  A_cc, P2, the residual recomputed with A_c, nu more steps;
* the level-1 coarse solve becomes gamma sweeps of the stationary iteration
  e <- e + K2(f - A_c e) from e = 0: gamma = 1 is the V-cycle, gamma = 2 the
  W-cycle (the coarse level visited twice per fine cycle).

Coarse vectors have shape (Tc, Zc, Yc, Xc, 2, Nv); level-2 vectors
(Tcc, Zcc, Ycc, Xcc, 2, Nv2).  Blocks ``block2`` are in coarse sites.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import solvers as _sol
from . import squared as _sq
from . import transfer as _tr


def _split(Lc, b2):
    """Coarse shape (Tc, Zc, Yc, Xc) -> index blocks: returns Lcc (x, y, z, t order)."""
    Lcc = tuple(Lc[m] // b2[m] for m in range(4))
    if any(Lcc[m] * b2[m] != Lc[m] for m in range(4)):
        raise ValueError("block2 must divide the coarse lattice")
    return Lcc


def _blocked(c: np.ndarray, b2) -> np.ndarray:
    """(..., Tc, Zc, Yc, Xc, 2, Nv) -> (..., Tcc, Zcc, Ycc, Xcc, 2, bt*bz*by*bx*Nv): each block's rows,
    ordered (t, z, y, x within the block, then k), per chirality."""
    *lead, Tc, Zc, Yc, Xc, two, nv = c.shape
    bx, by, bz, bt = b2
    v = c.reshape(*lead, Tc // bt, bt, Zc // bz, bz, Yc // by, by, Xc // bx, bx, two, nv)
    n = len(lead)
    perm = list(range(n)) + [n + 0, n + 2, n + 4, n + 6, n + 8, n + 1, n + 3, n + 5, n + 7, n + 9]
    v = v.transpose(perm)
    return v.reshape(*lead, Tc // bt, Zc // bz, Yc // by, Xc // bx, two, bt * bz * by * bx * nv)


def _unblocked(v: np.ndarray, b2, nv) -> np.ndarray:
    """Inverse of _blocked."""
    *lead, Tcc, Zcc, Ycc, Xcc, two, rows = v.shape
    bx, by, bz, bt = b2
    n = len(lead)
    w = v.reshape(*lead, Tcc, Zcc, Ycc, Xcc, two, bt, bz, by, bx, nv)
    perm = list(range(n)) + [n + 0, n + 5, n + 1, n + 6, n + 2, n + 7, n + 3, n + 8, n + 4, n + 9]
    w = w.transpose(perm)
    return w.reshape(*lead, Tcc * bt, Zcc * bz, Ycc * by, Xcc * bx, two, nv)


def build_basis2(W: np.ndarray, b2) -> np.ndarray:
    """Chirality split + per-block thin QR (positive real diagonal) of the level-2
    near-null vectors W (n, Tc, Zc, Yc, Xc, 2, Nv); returns What of the same shape,
    What[j] holding column (block, chi, j) on block's chirality-chi rows."""
    n = W.shape[0]
    B = _blocked(W, b2)                       # (n, Tcc, Zcc, Ycc, Xcc, 2, rows)
    P = np.moveaxis(B, 0, -1)                 # (..., 2, rows, n): one panel per (block, chi)
    Q, R = np.linalg.qr(P)
    d = np.diagonal(R, axis1=-2, axis2=-1)
    ph = d / np.abs(d)                        # make diag(R) positive real
    Q = Q * ph[..., None, :]
    return _unblocked(np.moveaxis(Q, -1, 0), b2, W.shape[-1])


def restrict2(c: np.ndarray, What: np.ndarray, b2) -> np.ndarray:
    """R2 c: (Tc,Zc,Yc,Xc,2,Nv) -> (Tcc,Zcc,Ycc,Xcc,2,Nv2), out[B,chi,j] = <What_j|_(B,chi), c>."""
    Bc = _blocked(c, b2)                      # (Tcc,..,2,rows)
    BW = _blocked(What, b2)                   # (Nv2, Tcc,..,2,rows)
    return np.einsum("j...r,...r->...j", BW.conj(), Bc)


def prolong2(cc: np.ndarray, What: np.ndarray, b2) -> np.ndarray:
    """P2 cc: sum_j What_j cc[B(X), chi, j]."""
    BW = _blocked(What, b2)
    out = np.einsum("j...r,...j->...r", BW, cc)
    return _unblocked(out, b2, What.shape[-1])


def cg_null_steps(Ac, w0: np.ndarray, niter: int) -> np.ndarray:
    """niter CG steps on A_c w = 0 from w0 (CG on the correction d of A_c d = -A_c w0)."""
    d, _ = _sq.cg(Ac, -Ac(w0), 0.0, niter)
    return w0 + d


class ExplicitCoarse2:
    """A_cc applied as R2 A_c P2 (the definition)."""

    def __init__(self, Ac, What, b2):
        self.Ac, self.What, self.b2 = Ac, What, b2

    def __call__(self, cc):
        return restrict2(self.Ac(prolong2(cc, self.What, self.b2)), self.What, self.b2)


def build_stencil2(Ac, What, b2) -> np.ndarray:
    """A_cc as the 33-offset stencil of ``squared`` (Tcc,Zcc,Ycc,Xcc,33,n2,n2), read
    off column by column: column (B, chi, j) is R2 A_c applied to What_j
    restricted to block B and chirality chi.  Where the level-2 lattice has
    extent 1 or 2 several offsets name the same neighbour; the whole coupling
    then sits in the first of them (in OFFSETS order) and the others are zero."""
    nv2 = What.shape[0]
    Tc, Zc, Yc, Xc = What.shape[1:5]
    Lc = (Xc, Yc, Zc, Tc)
    Lcc = _split(Lc, b2)
    n2 = 2 * nv2
    S = np.zeros(tuple(Lcc[::-1]) + (33, n2, n2), dtype=np.complex128)
    BW = _blocked(What, b2)
    for bt in range(Lcc[3]):
        for bz in range(Lcc[2]):
            for by in range(Lcc[1]):
                for bx in range(Lcc[0]):
                    for chi in range(2):
                        for j in range(nv2):
                            col = np.zeros(BW.shape[1:], dtype=np.complex128)
                            col[bt, bz, by, bx, chi] = BW[j, bt, bz, by, bx, chi]
                            y = restrict2(Ac(_unblocked(col, b2, What.shape[-1])), What, b2)
                            taken = set()
                            for oi, o in enumerate(_sq.OFFSETS):
                                # destination D with D + o = source B (o = (x, y, z, t))
                                D = tuple((np.array((bx, by, bz, bt)) - np.array(o)) % np.array(Lcc))
                                key = D
                                if key in taken:
                                    continue
                                taken.add(key)
                                S[D[3], D[2], D[1], D[0], oi, :, chi * nv2 + j] = \
                                    y[D[3], D[2], D[1], D[0]].reshape(n2)
    return S


class ThreeLevelSquared(_sq.TwoLevelSquared):
    """``squared``'s V-cycle with its coarse solve replaced by gamma sweeps of
    e <- e + K2(f - A_c e) (gamma = 1: V-cycle, 2: W-cycle)."""

    def __init__(self, A, Vhat, block, coarse, nu_pre, nu_post, What, b2, coarse2, nu2: int, tol2: float,
                 maxiter2: int, gamma: int):
        super().__init__(A, Vhat, block, coarse, 0.0, 0, nu_pre, nu_post)
        self.What, self.b2, self.coarse2 = What, b2, coarse2
        self.nu2, self.tol2, self.maxiter2, self.gamma = nu2, tol2, maxiter2, gamma

    def k2(self, f: np.ndarray) -> np.ndarray:
        """Level-2 cycle on A_c e = f."""
        Ac = self.coarse
        if self.nu2 > 0:
            e1, r1 = _sq.mr_hpd_steps(Ac, f, self.nu2)
        else:
            e1, r1 = np.zeros_like(f), f.copy()
        y, _ = _sq.cg(self.coarse2, restrict2(r1, self.What, self.b2), self.tol2, self.maxiter2)
        e = e1 + prolong2(y, self.What, self.b2)
        if self.nu2 > 0:
            e3, _ = _sq.mr_hpd_steps(Ac, f - Ac(e), self.nu2)
            e = e + e3
        return e

    def coarse_solve(self, f: np.ndarray) -> np.ndarray:
        e = np.zeros_like(f)
        for g in range(self.gamma):
            e = e + self.k2(f if g == 0 else f - self.coarse(e))
        return e

    def vcycle(self, g: np.ndarray) -> np.ndarray:
        if self.nu_pre > 0:
            x1, r1 = _sq.mr_hpd_steps(self.N, g, self.nu_pre)
        else:
            x1, r1 = np.zeros_like(g), g.copy()
        x2 = self.coarse_solve(_tr.restrict(r1, self.Vhat, self.block))
        xc = x1 + _tr.prolong(x2, self.Vhat, self.block)
        if self.nu_post > 0:
            x3, _ = _sq.mr_hpd_steps(self.N, g - self.N(xc), self.nu_post)
            return xc + x3
        return xc


@dataclass
class Level2Params:
    block: tuple = (2, 2, 2, 2)   # coarse sites per level-2 block
    nvec: int = 8                 # level-2 basis columns per chirality
    null_iters: int = 50          # CG steps on A_c w = 0 per start
    nu: int = 2                   # MR steps on A_c before and after the level-2 correction
    coarse_tol: float = 0.1       # CG on A_cc
    coarse_maxiter: int = 200
    gamma: int = 1                # 1: V-cycle, 2: W-cycle


@dataclass
class ThreeLevelMG:
    mg: _sq.SquaredMG
    p2: Level2Params
    W: np.ndarray = None
    What: np.ndarray = None
    coarse2: object = None

    def preconditioner(self) -> ThreeLevelSquared:
        p = self.mg.params
        return ThreeLevelSquared(self.mg.A, self.mg.Vhat, p.block, self.mg.coarse, p.nu_pre, p.nu_post,
                                 self.What, self.p2.block, self.coarse2, self.p2.nu, self.p2.coarse_tol,
                                 self.p2.coarse_maxiter, self.p2.gamma)


def level2_setup(mg: _sq.SquaredMG, W0: np.ndarray, p2: Level2Params) -> ThreeLevelMG:
    """Level-2 near-null vectors (CG on A_c w = 0 from each start, normalised),
    their basis and A_cc on top of a squared two-level setup."""
    W = np.array([cg_null_steps(mg.coarse, w, p2.null_iters) for w in W0])
    W = np.array([w / _sol.norm(w) for w in W])
    What = build_basis2(W, p2.block)
    return ThreeLevelMG(mg, p2, W, What, ExplicitCoarse2(mg.coarse, What, p2.block))


def three_level_solve(t: ThreeLevelMG, b: np.ndarray, tol: float = 1e-10, maxiter: int = 200, restart: int = 8):
    """Flexible GCR on D x = b with the three-level squared preconditioner."""
    return _sol.gcr(t.mg.A, b, tol, maxiter, restart, M=t.preconditioner())
