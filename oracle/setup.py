"""Adaptive near-null vector setup and the full two-level solver.  TEST INFRASTRUCTURE ONLY.

Paper, Sec. 2 (adaptive paragraph): run a Krylov solver on A x = 0 from a
random x; what survives is what the solver does not remove; build the
multigrid from that batch of vectors, apply the multigrid itself to the same
problem, keep what it fails to remove, and repeat.

Reading of the steps (the paper gives no counts):
* sweep 0: ``sweep0_iters`` iterations of CG on the normal equations of
  A v = 0 (the Krylov solver of the paper's Sec. 3, applied to D^+D) from
  each random start;
* sweeps 1..: ``sweep_iters`` iterations of the MG-preconditioned flexible GCR
  on A v = 0 from the current v (so v <- error left by the current MG);
* every vector is normalised after each sweep, the whole batch then rebuilds
  the basis and D_c;
* the basis is closed under gamma_5 R_5: the nh adaptive vectors are joined
  by their fifth-dimension reflections (R_5 v)(s) = v(Ls-1-s), giving
  Nv = 2 nh columns per chirality.  If D v ~ 0 then gamma_5 R_5 v is a left
  near-null vector (D^+ = gamma_5 R_5 D gamma_5 R_5), and with the chirality
  split the block span then holds both left and right near-null vectors, so
  D_c = P^+ D P inherits the gamma_5 R_5 symmetry of D.  Without this the
  Galerkin coarse operator of the unsquared D fails to give a convergent
  two-level method (the paper itself coarsened D^+D and names direct
  coarsening of D as open, Sec. 4).

Random starting vectors are inputs (generated elsewhere, identical for both
sides of a comparison).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np

from . import coarse as _coarse
from . import dwf as _dwf
from . import solvers as _sol
from . import transfer as _tr


@dataclass
class MGParams:
    block: tuple = (2, 2, 2, 2)
    nvec: int = 8                   # Nv: columns per chirality = 2 * adaptive vectors
    sweeps: int = 3                 # total sweeps including sweep 0
    sweep0_iters: int = 100
    sweep_iters: int = 4
    nu_pre: int = 4
    nu_post: int = 4
    smoother: str = "mr_normal"     # "mr" (on D) or "mr_normal" (along D^+ r)
    coarse_solver: str = "cgne"     # "gcr" or "cgne"
    coarse_tol: float = 0.1
    coarse_maxiter: int = 100
    coarse_restart: int = 16
    sweep0_check: int = 0           # > 0: sweep 0 keeps its best iterate (cgnr_null_best)


def _smoother_fn(kind: str):
    if kind == "mr":
        return _sol.mr_steps
    if kind == "mr_normal":
        return _sol.mr_normal_steps
    raise ValueError(kind)


@dataclass
class MG:
    A: _dwf.DWF
    params: MGParams
    Vhat: np.ndarray = None
    Dc: np.ndarray = None
    coarse: _coarse.Coarse = None
    null_residuals: List[float] = field(default_factory=list)
    sweep_norms: List[List[float]] = field(default_factory=list)   # |v| before each normalisation

    def rebuild(self, V: np.ndarray):
        self.Vhat = _tr.build_basis(reflect_pairs(V), self.params.block)
        self.Dc = _coarse.build_coarse_op(self.Vhat, self.A.U, self.A.M5, self.A.mf,
                                          self.params.block, self.A.bc)
        self.coarse = _coarse.Coarse(self.Dc)

    def R(self, x):
        return _tr.restrict(x, self.Vhat, self.params.block)

    def P(self, c):
        return _tr.prolong(c, self.Vhat, self.params.block)

    def preconditioner(self) -> _sol.TwoLevel:
        p = self.params
        if p.coarse_solver == "gcr":
            cs = _sol.coarse_gcr_solver(self.coarse, p.coarse_tol, p.coarse_maxiter, p.coarse_restart)
        else:
            cs = _sol.coarse_cgne_solver(self.coarse, p.coarse_tol, p.coarse_maxiter)
        return _sol.TwoLevel(self.A, self.R, self.P, cs, _smoother_fn(p.smoother), p.nu_pre, p.nu_post)


def reflect_pairs(V: np.ndarray) -> np.ndarray:
    """[v_0 .. v_{nh-1}, R5 v_0 .. R5 v_{nh-1}] with (R5 v)(s) = v(Ls-1-s)."""
    return np.concatenate([V, V[..., ::-1, :, :]], axis=0)


def cgnr_null_steps(A, x0: np.ndarray, niter: int) -> np.ndarray:
    """``niter`` CG iterations on A^+A x = 0 from x0 (two applications each)."""
    x = x0.copy()
    r = -A.dag(A(x))
    p = r.copy()
    rr = _sol.vdot(r, r).real
    for _ in range(niter):
        Ap = A.dag(A(p))
        pAp = _sol.vdot(p, Ap).real
        if pAp == 0.0 or rr == 0.0:
            break
        a = rr / pAp
        x += a * p
        r -= a * Ap
        rn = _sol.vdot(r, r).real
        p = r + (rn / rr) * p
        rr = rn
    return x


def cgnr_null_best(A, x0: np.ndarray, niter: int, check: int) -> np.ndarray:
    """Sweep 0 with a stopping rule: the CG iterations of ``cgnr_null_steps``;
    of the iterates after every ``check`` iterations and after the last one,
    the one with the smallest null residual |A x| / |x| is returned (the
    earliest on a tie).  The Krylov sweep is meant to stop while x holds the
    modes the solver removes slowly (Sec. 2, adaptive paragraph); once CG
    resolves the lowest modes as well, |A x| / |x| rises again."""
    x = x0.copy()
    r = -A.dag(A(x))
    p = r.copy()
    rr = _sol.vdot(r, r).real
    best, best_q = x0.copy(), np.inf
    for k in range(1, niter + 1):
        Ap = A.dag(A(p))
        pAp = _sol.vdot(p, Ap).real
        if pAp == 0.0 or rr == 0.0:
            break
        a = rr / pAp
        x += a * p
        r -= a * Ap
        rn = _sol.vdot(r, r).real
        p = r + (rn / rr) * p
        rr = rn
        if k % check == 0 or k == niter:
            q = null_residual(A, x)
            if q < best_q or (k == niter and best_q == np.inf):
                best, best_q = x.copy(), q
    return best


def sweep0(A, x0: np.ndarray, niter: int, check: int = 0) -> np.ndarray:
    """Sweep 0 of the adaptive setup: the last CG iterate, or with check > 0
    the best one (``cgnr_null_best``)."""
    return cgnr_null_best(A, x0, niter, check) if check > 0 else cgnr_null_steps(A, x0, niter)


def null_residual(A, v: np.ndarray) -> float:
    """|A v| / |v|, the quality measure of a near-null vector."""
    return _sol.norm(A(v)) / _sol.norm(v)


def adaptive_setup(A: _dwf.DWF, V0: np.ndarray, params: MGParams) -> MG:
    """Sweep 0 with the smoother, then MG-error sweeps, rebuilding after each."""
    mg = MG(A, params)
    if V0.shape[0] * 2 != params.nvec:
        raise ValueError("expected nvec/2 random starts (each is paired with its reflection)")
    V = np.array(V0, dtype=np.complex128, copy=True)
    zero = np.zeros_like(V[0])
    norms = []
    for k in range(V.shape[0]):
        x = sweep0(A, V[k], params.sweep0_iters, params.sweep0_check)
        norms.append(_sol.norm(x))
        V[k] = x / norms[-1]
    mg.sweep_norms.append(norms)
    mg.rebuild(V)
    mg.null_residuals.append(float(np.median([null_residual(A, v) for v in V])))
    for _ in range(params.sweeps - 1):
        M = mg.preconditioner()
        norms = []
        for k in range(V.shape[0]):
            x, _ = _sol.gcr_fixed(A, zero, V[k], params.sweep_iters, M=M)
            norms.append(_sol.norm(x))
            V[k] = x / norms[-1]
        mg.sweep_norms.append(norms)
        mg.rebuild(V)
        mg.null_residuals.append(float(np.median([null_residual(A, v) for v in V])))
    mg.V = V
    return mg


def mg_solve(mg: MG, b: np.ndarray, tol: float = 1e-10, maxiter: int = 200, restart: int = 8):
    """Flexible GCR on D x = b preconditioned by the two-level V-cycle."""
    M = mg.preconditioner()
    return _sol.gcr(mg.A, b, tol, maxiter, restart, M=M)
