"""Squared-operator Galerkin multigrid.  TEST INFRASTRUCTURE ONLY.

The paper ran its multigrid (and its CG control) on the squared operator
N = D^+ D (Sec. 3, first paragraph: the cost is counted in applications of
the squared fine operator; Sec. 4, last paragraph: the coarse operator of
the squared operator couples a coarse site to sites up to two hops away).
This module is that method, written from its definition:

* basis: the near-null vectors v_k of D^+ D (sweep 0 of the adaptive setup),
  chirality split and block orthonormalised as in ``transfer`` -- no
  pairing with reflections, since N is Hermitian and its left and right
  near-null vectors coincide;
* coarse operator: A_c = P^+ N P = (D P)^+ (D P), Hermitian positive
  definite;
* V-cycle (Sec. 2, its five steps) on N f = g: minimal-residual smoothing on
  N, restriction, a CG solve of A_c, prolongation, the residual recomputed
  with N, post-smoothing;
* outer solver: flexible GCR on D x = b (Sec. 3) with the right
  preconditioner M(r) = V-cycle applied to g = D^+ r, so M approximates
  N^-1 D^+ = D^-1.

With 4D blocks of extent >= 2 that span the fifth dimension, A_c couples a
coarse site X only to X + o for the 33 offsets o in ``OFFSETS`` (self, the
eight unit neighbours and the 24 diagonal neighbours +-mu +-nu, mu < nu):
two hops of D reach the neighbouring block in one or two directions, never
two blocks away in one direction, because the two hops of one direction
land on opposite faces of the block in between.  The paper counts 17 sites
at up to two hops (self, 8 one-hop and, by that count, 8 straight two-hop
sites); the Galerkin definition with such blocks gives instead no straight
two-hop coupling and 24 diagonal ones, 33 in all -- the reading taken here,
pinned by the support test.

Layouts as in ``transfer`` and ``coarse``: coarse vectors (Tc,Zc,Yc,Xc,2,Nv);
the stencil Ac has shape (Tc,Zc,Yc,Xc,33,2Nv,2Nv) with
(A_c y)(X) = sum_o Ac[X][o] y(X + o), periodic.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np

from . import dwf as _dwf
from . import setup as _setup
from . import solvers as _sol
from . import transfer as _tr


def _offsets():
    """Offsets in (x, y, z, t) order: 0 self; 1 + 2 mu = +mu, 2 + 2 mu = -mu;
    then for mu < nu the four diagonals (+mu+nu, +mu-nu, -mu+nu, -mu-nu)."""
    out = [(0, 0, 0, 0)]
    for mu in range(4):
        for sgn in (1, -1):
            o = [0, 0, 0, 0]
            o[mu] = sgn
            out.append(tuple(o))
    for mu in range(4):
        for nu in range(mu + 1, 4):
            for s1, s2 in ((1, 1), (1, -1), (-1, 1), (-1, -1)):
                o = [0, 0, 0, 0]
                o[mu], o[nu] = s1, s2
                out.append(tuple(o))
    return out


OFFSETS = _offsets()
NOFF = len(OFFSETS)  # 33


class Normal:
    """N = A^+ A, Hermitian; counts nothing itself (A may)."""

    def __init__(self, A):
        self.A = A

    def __call__(self, v):
        return self.A.dag(self.A(v))

    def dag(self, v):
        return self(v)


def _coarse_roll(c: np.ndarray, o) -> np.ndarray:
    """g(X) = c(X + o), periodic, arrays ordered (T, Z, Y, X, ...)."""
    g = c
    for mu in range(4):
        if o[mu]:
            g = np.roll(g, -o[mu], axis=3 - mu)
    return g


def build_sq_coarse_op(Vhat: np.ndarray, U: np.ndarray, M5: float, mf: float, block,
                       bc=(1, 1, 1, 1)) -> np.ndarray:
    """Ac from its definition: column (B, j) of A_c is R D^+ D P e_(B,j).

    Every coarse extent must be >= 3 so that the 33 sites X = B - o that the
    column reaches are distinct and the column can be read off site by site;
    the block extents must be >= 2.  Any part of the column outside those 33
    sites raises (it would contradict the two-hop support).
    """
    Nv = Vhat.shape[0]
    T, Zd, Y, X = Vhat.shape[1:5]
    L = (X, Y, Zd, T)
    Lc = _tr.coarse_dims(L, block)
    if min(Lc) < 3 or min(block) < 2:
        raise ValueError("the probed stencil needs coarse extents >= 3 and block extents >= 2")
    n2 = 2 * Nv
    shp = tuple(Lc[::-1]) + (2, Nv)
    Ac = np.zeros(tuple(Lc[::-1]) + (NOFF, n2, n2), dtype=np.complex128)
    for B in np.ndindex(*Lc[::-1]):
        for chi in range(2):
            for k in range(Nv):
                e = np.zeros(shp, dtype=np.complex128)
                e[B + (chi, k)] = 1.0
                pe = _tr.prolong(e, Vhat, block)
                w = _tr.restrict(_dwf.apply_dwf(_dwf.apply_dwf(pe, U, M5, mf, bc), U, M5, mf, bc, dagger=True),
                                 Vhat, block).reshape(tuple(Lc[::-1]) + (n2,))
                seen = np.zeros(Lc[::-1], dtype=bool)
                j = chi * Nv + k
                for oi, o in enumerate(OFFSETS):
                    # y(B - o) = Ac[B - o][o] e(B)
                    Xs = tuple((B[a] - o[3 - a]) % Lc[3 - a] for a in range(4))
                    Ac[Xs + (oi, slice(None), j)] = w[Xs]
                    seen[Xs] = True
                rest = np.abs(w[~seen]).max() if (~seen).any() else 0.0
                if rest > 1e-12 * np.abs(w).max():
                    raise ValueError("A_c column reaches beyond the 33-site stencil")
    return Ac


def apply_sq_coarse(c: np.ndarray, Ac: np.ndarray) -> np.ndarray:
    """y(X) = sum_o Ac[X][o] c(X + o); c has shape (Tc,Zc,Yc,Xc,2,Nv)."""
    shp = c.shape
    v = c.reshape(shp[:4] + (-1,))
    y = np.zeros_like(v)
    for oi, o in enumerate(OFFSETS):
        y += np.einsum("...ij,...j->...i", Ac[..., oi, :, :], _coarse_roll(v, o))
    return y.reshape(shp)


class ExplicitCoarse:
    """A_c applied as R N P (the definition; any coarse extents)."""

    def __init__(self, A, Vhat, block):
        self.N, self.Vhat, self.block = Normal(A), Vhat, block
        self.napply = 0

    def __call__(self, c):
        self.napply += 1
        return _tr.restrict(self.N(_tr.prolong(c, self.Vhat, self.block)), self.Vhat, self.block)

    def dag(self, c):
        return self(c)


def mr_hpd_steps(N, f: np.ndarray, niter: int):
    """Minimal residual on the Hermitian operator N: p = N r, alpha = <p, r>/<p, p>,
    x += alpha r, r -= alpha p (each step minimises |f - N x| along r)."""
    x = np.zeros_like(f)
    r = f.copy()
    for _ in range(niter):
        p = N(r)
        pp = _sol.vdot(p, p).real
        if pp == 0.0:
            break
        alpha = _sol.vdot(p, r) / pp
        x += alpha * r
        r -= alpha * p
    return x, r


def cg(Aop, b: np.ndarray, tol: float, maxiter: int):
    """Conjugate gradients on a Hermitian positive definite operator, from x = 0,
    to |r| <= tol |b| (tested every iteration) or maxiter iterations."""
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = _sol.vdot(r, r).real
    bb = rr
    it = 0
    while it < maxiter and rr > tol * tol * bb:
        q = Aop(p)
        pq = _sol.vdot(p, q).real
        if pq <= 0.0:
            break
        alpha = rr / pq
        x += alpha * p
        r -= alpha * q
        rn = _sol.vdot(r, r).real
        p = r + (rn / rr) * p
        rr = rn
        it += 1
    return x, it


class TwoLevelSquared:
    """M(r) = V(D^+ r), V the five-step V-cycle (Sec. 2) on N = D^+ D:
    x1 = S1^nu1(N, g); g2 = R(g - N x1); x2 = CG(A_c, g2); g3 = g - N(x1 + P x2);
    result x1 + P x2 + S3^nu3(N, g3)."""

    def __init__(self, A, Vhat, block, coarse, coarse_tol: float, coarse_maxiter: int, nu_pre: int, nu_post: int):
        self.A, self.N = A, Normal(A)
        self.Vhat, self.block = Vhat, block
        self.coarse = coarse
        self.coarse_tol, self.coarse_maxiter = coarse_tol, coarse_maxiter
        self.nu_pre, self.nu_post = nu_pre, nu_post

    def vcycle(self, g: np.ndarray) -> np.ndarray:
        if self.nu_pre > 0:
            x1, r1 = mr_hpd_steps(self.N, g, self.nu_pre)
        else:
            x1, r1 = np.zeros_like(g), g.copy()
        x2, _ = cg(self.coarse, _tr.restrict(r1, self.Vhat, self.block), self.coarse_tol, self.coarse_maxiter)
        xc = x1 + _tr.prolong(x2, self.Vhat, self.block)
        if self.nu_post > 0:
            x3, _ = mr_hpd_steps(self.N, g - self.N(xc), self.nu_post)
            return xc + x3
        return xc

    def __call__(self, r: np.ndarray) -> np.ndarray:
        return self.vcycle(self.A.dag(r))


@dataclass
class SquaredParams:
    block: tuple = (2, 2, 2, 2)
    nvec: int = 16                  # adaptive vectors = basis columns per chirality
    sweeps: int = 1
    sweep0_iters: int = 100
    sweep_iters: int = 4
    nu_pre: int = 4
    nu_post: int = 4
    coarse_tol: float = 0.1
    coarse_maxiter: int = 200
    sweep0_check: int = 0


@dataclass
class SquaredMG:
    A: _dwf.DWF
    params: SquaredParams
    V: np.ndarray = None
    Vhat: np.ndarray = None
    coarse: object = None
    null_residuals: List[float] = None

    def rebuild(self, V: np.ndarray, stencil: bool = False):
        self.V = V
        self.Vhat = _tr.build_basis(V, self.params.block)
        if stencil:
            Ac = build_sq_coarse_op(self.Vhat, self.A.U, self.A.M5, self.A.mf, self.params.block, self.A.bc)
            self.coarse = lambda c: apply_sq_coarse(c, Ac)
        else:
            self.coarse = ExplicitCoarse(self.A, self.Vhat, self.params.block)

    def preconditioner(self) -> TwoLevelSquared:
        p = self.params
        return TwoLevelSquared(self.A, self.Vhat, p.block, self.coarse, p.coarse_tol, p.coarse_maxiter,
                               p.nu_pre, p.nu_post)


def squared_setup(A: _dwf.DWF, V0: np.ndarray, params: SquaredParams, stencil: bool = False) -> SquaredMG:
    """Sweep 0: CG on D^+D v = 0 from each start (the Krylov solver of Sec. 2's
    adaptive paragraph), normalise, build; sweeps >= 1: the squared multigrid
    applied to D x = 0 from each vector (flexible GCR, sweep_iters steps), keep
    what is left, normalise, rebuild."""
    if V0.shape[0] != params.nvec:
        raise ValueError("expected nvec random starts")
    mg = SquaredMG(A, params, null_residuals=[])
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


def squared_solve(mg: SquaredMG, b: np.ndarray, tol: float = 1e-10, maxiter: int = 200, restart: int = 8):
    """Flexible GCR on D x = b with the squared two-level preconditioner."""
    return _sol.gcr(mg.A, b, tol, maxiter, restart, M=mg.preconditioner())
