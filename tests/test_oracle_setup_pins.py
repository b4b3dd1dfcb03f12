"""Pins of the oracle's smoother and adaptive-setup steps (CPU only).

Paper, Sec. 2: the smoother S1 = S3 is a minimal-residual iteration; the
adaptive setup first runs a Krylov solver on A x = 0 from random vectors, then
applies the multigrid built from them to the same problem.  Each step below is
a minimisation over a small subspace, so each is pinned against numpy's dense
least-squares routine on that subspace, built from applications of the
operator alone (no formula of the oracle is re-typed here).
"""
import numpy as np

from inputs import gaussian_fermion, prepare_gauge, random_starts
from oracle import dwf
from oracle import setup as osu
from oracle import solvers as osv
from oracle import transfer as ot

M5 = 1.8


def _lstsq_min(cols, target):
    """argmin_c |target - sum_j c_j cols[j]|, every array flattened."""
    Amat = np.stack([c.ravel() for c in cols], axis=1)
    c, *_ = np.linalg.lstsq(Amat, target.ravel(), rcond=None)
    return c


def test_mr_normal_step_is_the_one_dimensional_least_squares_minimiser():
    """Each step of the smoother minimises |b - A x| along A^+ r (a wrong or
    halved step length, or a step along r instead of A^+ r, fails)."""
    L, Ls, mf = (4, 2, 2, 2), 4, 0.05
    A = dwf.DWF(prepare_gauge(L, 0.4, 5), M5, mf)
    b = gaussian_fermion(L, Ls, 6)
    x = np.zeros_like(b)
    for k in range(1, 4):
        r = b - A(x)
        p = A.dag(r)
        c = _lstsq_min([A(p)], r)
        x = x + c[0] * p
        xk, rk = osv.mr_normal_steps(A, b, k)
        assert np.linalg.norm(xk - x) / np.linalg.norm(x) < 1e-12
        # the returned residual is the true one
        assert np.linalg.norm(rk - (b - A(xk))) / np.linalg.norm(b) < 1e-12


def test_cgnr_null_steps_minimise_over_the_krylov_space():
    """k CG iterations on A^+A x = 0 from x0 give the minimiser of |A x| over
    x0 + K_k(A^+A, r0), r0 = -A^+A x0 (CG minimises the A^+A-norm of the error,
    and the exact solution is 0)."""
    L, Ls, mf = (2, 2, 2, 4), 4, 0.02
    A = dwf.DWF(prepare_gauge(L, 0.5, 7), M5, mf)
    x0 = random_starts(L, Ls, 1, 8)[0]
    r0 = -A.dag(A(x0))
    for k in (1, 3, 6):
        K = [r0]
        for _ in range(k - 1):
            K.append(A.dag(A(K[-1])))
        Q, _ = np.linalg.qr(np.stack([v.ravel() for v in K], axis=1))
        cols = [Q[:, j].reshape(x0.shape) for j in range(k)]
        c = _lstsq_min([A(q) for q in cols], -A(x0))
        xref = x0 + sum(cj * q for cj, q in zip(c, cols))
        xk = osu.cgnr_null_steps(A, x0, k)
        assert np.linalg.norm(xk - xref) / np.linalg.norm(xref) < 1e-10, k
        assert np.linalg.norm(A(xk)) < np.linalg.norm(A(x0))


def _linear_two_level(A, Vhat, block):
    """The V-cycle with no smoothing and a coarse solve to rounding: the linear map P D_c^-1 R."""
    from oracle import coarse as oc
    Dc = oc.build_coarse_op(Vhat, A.U, A.M5, A.mf, block)
    cs = osv.coarse_cgne_solver(oc.Coarse(Dc), 1e-15, 5000)
    R = lambda x: ot.restrict(x, Vhat, block)
    P = lambda c: ot.prolong(c, Vhat, block)
    return osv.TwoLevel(A, R, P, cs, osv.mr_normal_steps, 0, 0), R, P, Dc


def test_fixed_flexible_gcr_is_minimum_residual_over_the_multigrid_krylov_space():
    """The sweeps after sweep 0 run k flexible-GCR steps with the V-cycle M
    from a starting vector x0 (Sec. 2: the multigrid applied to A x = 0).  With
    a linear M and b = 0 the result is the minimiser of |A x| over
    x0 + M K_k(A M, -A x0), computed here by dense least squares on that space.
    M is the coarse correction P D_c^-1 R plus a multiple of the identity (the
    coarse correction alone is a projector, M A M = M, whose Krylov space stops
    growing after one step)."""
    L, Ls, mf, block = (2, 2, 2, 4), 4, 0.02, (1, 1, 2, 2)
    A = dwf.DWF(prepare_gauge(L, 0.4, 9), M5, mf)
    Vhat = ot.build_basis(osu.reflect_pairs(random_starts(L, Ls, 2, 10)), block)
    T, R, P, _ = _linear_two_level(A, Vhat, block)
    M = lambda r: T(r) + 0.3 * r
    x0 = random_starts(L, Ls, 1, 14)[0]
    for k in (1, 2, 4):
        K = [-A(x0)]
        for _ in range(k - 1):
            K.append(A(M(K[-1])))
        Q, _ = np.linalg.qr(np.stack([w.ravel() for w in K], axis=1))
        dirs = [M(Q[:, i].reshape(x0.shape)) for i in range(k)]
        c = _lstsq_min([A(d) for d in dirs], -A(x0))
        xref = x0 + sum(ci * d for ci, d in zip(c, dirs))
        x, r = osv.gcr_fixed(A, np.zeros_like(x0), x0, k, M=M)
        assert np.linalg.norm(x - xref) / np.linalg.norm(xref) < 1e-9, k
        assert np.linalg.norm(r + A(x)) / np.linalg.norm(A(x)) < 1e-9, k


def test_adaptive_sweep_keeps_only_what_the_multigrid_fails_to_remove():
    """Sec. 2: after sweep 0 the multigrid built from the vectors is applied to
    A x = 0 starting from each vector, and what it fails to remove is kept.
    Every vector lies in its own coarse space, so with no smoothing and an
    exact coarse solve one step removes it entirely (the norms the setup
    records before normalising vanish), while sweep 0 alone keeps them.  An
    inverse-iteration sweep (solving A e = v) or a wrong sign of the starting
    residual would leave them of order one."""
    L, Ls, mf, block = (2, 2, 2, 4), 4, 0.02, (1, 1, 2, 2)
    A = dwf.DWF(prepare_gauge(L, 0.4, 9), M5, mf)
    V0 = random_starts(L, Ls, 2, 10)
    prm = osu.MGParams(block=block, nvec=4, sweeps=2, sweep0_iters=4, sweep_iters=1, nu_pre=0, nu_post=0,
                       coarse_tol=1e-15, coarse_maxiter=5000)
    mg = osu.adaptive_setup(A, V0, prm)
    assert len(mg.sweep_norms) == 2
    assert min(mg.sweep_norms[0]) > 1e-3
    assert max(mg.sweep_norms[1]) < 1e-10
    # with the V-cycle's smoothing on, the sweep keeps a part of each vector
    # that is of order one and lowers |A v| before normalisation
    prm.nu_pre = prm.nu_post = 2
    prm.coarse_tol, prm.coarse_maxiter = 0.1, 100
    mg = osu.adaptive_setup(A, V0, prm)
    assert min(mg.sweep_norms[1]) > 1e-6


def test_adaptive_sweep_with_exact_coarse_solve_removes_the_coarse_space():
    """One flexible-GCR step with M = P D_c^-1 R on A x = 0 from a vector that
    lies in the coarse space returns (up to rounding) zero: M A v = v for v in
    range(P) because R A P = D_c.  A dropped term in the V-cycle or a wrong
    sign in the sweep's starting residual leaves a nonzero remainder."""
    L, Ls, mf, block = (2, 2, 2, 4), 4, 0.02, (1, 1, 2, 2)
    A = dwf.DWF(prepare_gauge(L, 0.4, 11), M5, mf)
    V = random_starts(L, Ls, 3, 12)
    Vhat = ot.build_basis(osu.reflect_pairs(V), block)
    M, R, P, Dc = _linear_two_level(A, Vhat, block)
    c = np.random.default_rng(13).standard_normal(Dc.shape[:4] + (2, Vhat.shape[0])) + 0j
    v = P(c)
    x, r = osv.gcr_fixed(A, np.zeros_like(v), v, 1, M=M)
    assert np.linalg.norm(x) / np.linalg.norm(v) < 1e-10
    assert np.linalg.norm(r) / np.linalg.norm(A(v)) < 1e-10


def test_sweep0_stopping_rule_picks_the_best_checked_iterate():
    """cgnr_null_best against brute force: the same number of CG iterations
    run afresh for every checked count, the smallest |A x|/|x| among them;
    with one check at the end it is plain sweep 0."""
    L, Ls = (6, 6, 6, 6), 8
    A = dwf.DWF(prepare_gauge(L, 0.3, 11, ape_steps=2), M5, 0.001)
    v = random_starts(L, Ls, 1, 21)[0]
    niter, check = 100, 25
    cands = [k for k in range(check, niter + 1, check)]
    xs = [osu.cgnr_null_steps(A, v, k) for k in cands]
    q = [osu.null_residual(A, x) for x in xs]
    assert cands[int(np.argmin(q))] == 75  # an intermediate iterate wins here (the ratio rises after it)
    want = xs[int(np.argmin(q))]
    got = osu.cgnr_null_best(A, v, niter, check)
    assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)
    last = osu.cgnr_null_best(A, v, 40, 1000)
    assert np.array_equal(last, osu.cgnr_null_steps(A, v, 40))
    assert np.array_equal(osu.sweep0(A, v, 40), osu.cgnr_null_steps(A, v, 40))
