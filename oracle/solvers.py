"""Krylov solvers and the V-cycle.  TEST INFRASTRUCTURE ONLY.

Paper references:
* Sec. 2 (V-cycle): five steps with nu1, nu2, nu3 iterations of solvers S1,
  S2, S3; the coarse step acts on R A P.
* Sec. 3 (first paragraph): the cost measure is the number of fine-operator
  applications; the control is CG on the squared operator.
* Sec. 3 (second paragraph): a 2-level V-cycle preconditions a flexible outer
  Krylov solver, generalised conjugate residual (GCR).

Readings: residuals are r = b - A x throughout (the paper writes both signs);
the smoother S1 = S3 is a fixed number of minimal-residual steps; the coarse
solver S2 runs to a relative residual or an iteration cap.

Operators are callables on numpy arrays; ``A.dag`` is the adjoint when needed.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np


def vdot(a: np.ndarray, b: np.ndarray) -> complex:
    """<a, b> = sum conj(a) b."""
    return complex(np.vdot(a.ravel(), b.ravel()))


def norm(a: np.ndarray) -> float:
    return float(np.linalg.norm(a.ravel()))


# ---------------------------------------------------------------- smoothers

def mr_steps(A, b: np.ndarray, niter: int, x0: Optional[np.ndarray] = None):
    """Minimal residual on A x = b: p = A r, alpha = <p,r>/<p,p>, x += alpha r, r -= alpha p.

    Returns (x, r) with r the recursively updated residual b - A x.
    """
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b.copy() if x0 is None else b - A(x0)
    for _ in range(niter):
        p = A(r)
        pp = vdot(p, p).real
        if pp == 0.0:
            break
        alpha = vdot(p, r) / pp
        x += alpha * r
        r -= alpha * p
    return x, r


def mr_normal_steps(A, b: np.ndarray, niter: int, x0: Optional[np.ndarray] = None):
    """Minimal residual along p = A^+ r: alpha = |p|^2 / |A p|^2, x += alpha p, r -= alpha A p.

    Each step minimises |b - A x| over the direction A^+ r (steepest descent
    on the normal equations); |r| never increases.  Two applications per step.
    """
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b.copy() if x0 is None else b - A(x0)
    for _ in range(niter):
        p = A.dag(r)
        q = A(p)
        qq = vdot(q, q).real
        if qq == 0.0:
            break
        alpha = vdot(p, p).real / qq
        x += alpha * p
        r -= alpha * q
    return x, r


# ---------------------------------------------------------------- GCR family

@dataclass
class SolveReport:
    converged: bool = False
    iters: int = 0
    true_relres: float = float("nan")
    history: List[float] = field(default_factory=list)


def gcr(A, b: np.ndarray, tol: float, maxiter: int, restart: int,
        M: Optional[Callable] = None, x0: Optional[np.ndarray] = None,
        true_residual_at_restart: bool = True):
    """(Flexible) GCR with right preconditioner M, restarted every ``restart`` steps.

    Per step: z = M(r); q = A z; orthogonalise q against the stored q_i by
    modified Gram-Schmidt, applying the same combination to z; normalise;
    alpha = <q, r>; x += alpha z; r -= alpha q.  At each restart the residual is
    recomputed as b - A x.  Stops when |r|/|b| < tol (iterated residual) and
    then confirms with the true residual, restarting if that is not met.
    """
    bn = norm(b)
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b.copy() if x0 is None else b - A(x)
    rep = SolveReport()
    if bn == 0.0:
        rep.converged, rep.true_relres = True, 0.0
        return x, rep
    Q: List[np.ndarray] = []
    Z: List[np.ndarray] = []
    rep.history.append(norm(r) / bn)
    while rep.iters < maxiter:
        z = M(r) if M is not None else r.copy()
        q = A(z)
        for qi, zi in zip(Q, Z):
            beta = vdot(qi, q)
            q = q - beta * qi
            z = z - beta * zi
        qn = norm(q)
        if qn == 0.0:
            break
        q /= qn
        z /= qn
        alpha = vdot(q, r)
        x += alpha * z
        r -= alpha * q
        Q.append(q)
        Z.append(z)
        rep.iters += 1
        rel = norm(r) / bn
        rep.history.append(rel)
        restart_now = len(Q) >= restart
        if rel < tol or restart_now:
            if true_residual_at_restart:
                r = b - A(x)
                rel = norm(r) / bn
            Q.clear()
            Z.clear()
            if rel < tol:
                rep.converged = True
                break
    rep.true_relres = norm(b - A(x)) / bn if true_residual_at_restart else norm(r) / bn
    return x, rep


def gcr_fixed(A, b: np.ndarray, x0: np.ndarray, niter: int, M: Optional[Callable] = None):
    """Exactly ``niter`` flexible-GCR steps from x0, no restart and no stopping test.

    Used by the adaptive setup on A x = 0, where |b| = 0 gives no relative scale.
    """
    x = x0.copy()
    r = b - A(x)
    Q: List[np.ndarray] = []
    Z: List[np.ndarray] = []
    for _ in range(niter):
        z = M(r) if M is not None else r.copy()
        q = A(z)
        for qi, zi in zip(Q, Z):
            beta = vdot(qi, q)
            q = q - beta * qi
            z = z - beta * zi
        qn = norm(q)
        if qn == 0.0:
            break
        q /= qn
        z /= qn
        alpha = vdot(q, r)
        x += alpha * z
        r -= alpha * q
        Q.append(q)
        Z.append(z)
    return x, r


def cgne(A, b: np.ndarray, tol: float, maxiter: int, x0: Optional[np.ndarray] = None):
    """CG on the normal equations A A^+ y = b, x = A^+ y (CGNE), stopping on |b - A x|/|b|.

    This is the control of the paper's Sec. 3: CG on the squared operator.
    Each iteration costs two applications (A^+ then A).
    """
    bn = norm(b)
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b.copy() if x0 is None else b - A(x)
    rep = SolveReport()
    p = A.dag(r)
    rr = vdot(r, r).real
    rep.history.append(np.sqrt(rr) / bn)
    while rep.iters < maxiter and np.sqrt(rr) / bn >= tol:
        Ap = A(p)
        pp = vdot(p, p).real
        alpha = rr / pp
        x += alpha * p
        r -= alpha * Ap
        rr_new = vdot(r, r).real
        p = A.dag(r) + (rr_new / rr) * p
        rr = rr_new
        rep.iters += 1
        rep.history.append(np.sqrt(rr) / bn)
    rep.true_relres = norm(b - A(x)) / bn
    rep.converged = rep.true_relres < tol
    return x, rep


# ---------------------------------------------------------------- V-cycle

class TwoLevel:
    """The five-step V-cycle of the paper's Sec. 2, as a preconditioner M(b).

    x1 = S1^nu1(A, b); b2 = R(b - A x1); x2 = S2(R A P, b2);
    b3 = b - A(P x2 + x1); x = x1 + P x2 + S3^nu3(A, b3).

    ``smoother(A, b, nu)`` returns (x, r); ``coarse_solve(b2)`` returns x2.
    b - A x1 is the smoother's own residual; b3 is formed with one more
    application of A, as the step is written.
    """

    def __init__(self, A, R, P, coarse_solve, smoother, nu_pre: int, nu_post: int):
        self.A, self.R, self.P = A, R, P
        self.coarse_solve = coarse_solve
        self.smoother = smoother
        self.nu_pre, self.nu_post = nu_pre, nu_post

    def __call__(self, b: np.ndarray) -> np.ndarray:
        if self.nu_pre > 0:
            x1, r1 = self.smoother(self.A, b, self.nu_pre)
        else:
            x1, r1 = np.zeros_like(b), b.copy()
        b2 = self.R(r1)
        x2 = self.coarse_solve(b2)
        xc = x1 + self.P(x2)
        if self.nu_post > 0:
            b3 = b - self.A(xc)
            x3, _ = self.smoother(self.A, b3, self.nu_post)
            return xc + x3
        return xc


def coarse_gcr_solver(Ac, tol: float, maxiter: int, restart: int):
    """S2 as unpreconditioned GCR on D_c to a relative residual ``tol``."""
    def solve(b2):
        x, _ = gcr(Ac, b2, tol, maxiter, restart, M=None, true_residual_at_restart=False)
        return x
    return solve


def coarse_cgne_solver(Ac, tol: float, maxiter: int):
    """S2 as CG on the normal equations of D_c."""
    def solve(b2):
        x, _ = cgne(Ac, b2, tol, maxiter)
        return x
    return solve
