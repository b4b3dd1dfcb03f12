"""Pins of the three-level squared multigrid oracle (CPU only).

Paper Sec. 2: the coarse solve may itself be a multigrid cycle.  Pins: the
level-2 basis is orthonormal per (block, chirality) and spans the
chirality-split near-null vectors; R2 P2 = 1; A_cc read off as a 33-offset
stencil reproduces R2 A_c P2 exactly on level-2 lattices with extents 1, 2
and 3 and is Hermitian positive definite; the CG null steps minimise the
A_c-energy over their Krylov space (dense least squares); with a complete
level-2 basis and exact inner solves the three-level cycle equals the
two-level one with an exact coarse solve; V- and W-cycle solves reach a true
residual of 1e-10.
"""
import numpy as np
import pytest

from inputs import gaussian_fermion, prepare_gauge, random_coarse_starts, random_starts
from oracle import dwf
from oracle import squared as osq
from oracle import threelevel as o3
from oracle import transfer as ot

M5 = 1.8


def _level1(L, Ls, mf, block, nvec, seed):
    U = prepare_gauge(L, 0.35, seed)
    A = dwf.DWF(U, M5, mf)
    V = random_starts(L, Ls, nvec, seed + 1)
    Vh = ot.build_basis(V, block)
    Ac = osq.ExplicitCoarse(A, Vh, block)  # R D^+D P (its stencil form needs coarse extents >= 3)
    Lc = tuple(L[m] // block[m] for m in range(4))
    return A, Vh, Ac, Lc


def _dense(op, shape):
    n = int(np.prod(shape))
    cols = []
    for j in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[j] = 1.0
        cols.append(op(e.reshape(shape)).ravel())
    return np.array(cols).T


@pytest.mark.parametrize("L,b2", [((4, 4, 4, 4), (2, 2, 2, 2)),    # level-2 extents 1
                                  ((4, 4, 4, 4), (1, 1, 2, 2)),    # extents 2, 2, 1, 1
                                  ((6, 4, 4, 4), (1, 2, 2, 1))])   # extents 3, 1, 1, 2
def test_stencil2_is_r2_ac_p2(L, b2):
    Ls, mf, block, nvec, nv2 = 4, 0.05, (2, 2, 2, 2), 4, 3
    A, Vh, Ac, Lc = _level1(L, Ls, mf, block, nvec, 40)
    W = random_coarse_starts(Lc, nvec, nv2, 41)
    Wh = o3.build_basis2(W, b2)
    # orthonormal per (block, chirality), and the span holds the split W
    Lcc = tuple(Lc[m] // b2[m] for m in range(4))
    rng = np.random.default_rng(42)
    cc = rng.standard_normal(Lcc[::-1] + (2, nv2)) + 1j * rng.standard_normal(Lcc[::-1] + (2, nv2))
    assert np.abs(o3.restrict2(o3.prolong2(cc, Wh, b2), Wh, b2) - cc).max() < 1e-13
    for w in W:
        for chi in (0, 1):
            wc = np.zeros_like(w)
            wc[..., chi, :] = w[..., chi, :]
            back = o3.prolong2(o3.restrict2(wc, Wh, b2), Wh, b2)
            assert np.abs(back - wc).max() < 1e-12 * np.abs(wc).max()
    S = o3.build_stencil2(Ac, Wh, b2)
    ex = o3.ExplicitCoarse2(Ac, Wh, b2)
    for _ in range(2):
        x = rng.standard_normal(cc.shape) + 1j * rng.standard_normal(cc.shape)
        want = ex(x)
        assert np.linalg.norm(osq.apply_sq_coarse(x, S) - want) <= 1e-12 * np.linalg.norm(want)
    M = _dense(ex, cc.shape)
    assert np.abs(M - M.conj().T).max() < 1e-12 * np.abs(M).max()
    assert np.linalg.eigvalsh(M).min() > 0


def test_cg_null_steps_minimise_the_energy():
    """k CG steps on A_c w = 0 from w0 give argmin of w^+ A_c w over
    w0 + span{A_c w0, ..., A_c^k w0} (dense least squares on that space)."""
    L, Ls, mf, block, nvec = (4, 4, 4, 4), 4, 0.05, (2, 2, 2, 2), 4
    A, Vh, Ac, Lc = _level1(L, Ls, mf, block, nvec, 43)
    w0 = random_coarse_starts(Lc, nvec, 1, 44)[0]
    shape = w0.shape
    M = _dense(Ac, shape)
    x0 = w0.ravel()
    for k in (1, 2, 4):
        got = o3.cg_null_steps(Ac, w0, k).ravel()
        K = [M @ x0]
        for _ in range(k - 1):
            K.append(M @ K[-1])
        Q, _ = np.linalg.qr(np.array(K).T)  # orthonormal basis of the Krylov space
        c = np.linalg.solve(Q.conj().T @ M @ Q, -(Q.conj().T @ (M @ x0)))
        want = x0 + Q @ c
        assert np.linalg.norm(got - want) < 1e-9 * np.linalg.norm(x0), k
        # a plain dropped term would fail: the energy is below that of w0 and of one step less
        assert (want.conj() @ M @ want).real < (x0.conj() @ M @ x0).real


def test_complete_level2_basis_gives_the_two_level_cycle():
    """Blocks of one coarse site holding all 2 Nv of its dof: R2 is unitary, so
    with exact inner solves K2 inverts A_c and the three-level cycle equals the
    two-level cycle with an exact coarse solve."""
    L, Ls, mf, block, nvec = (4, 4, 4, 4), 4, 0.05, (2, 2, 2, 2), 3
    A, Vh, Ac, Lc = _level1(L, Ls, mf, block, nvec, 45)
    W = random_coarse_starts(Lc, nvec, nvec, 46)
    b2 = (1, 1, 1, 1)
    Wh = o3.build_basis2(W, b2)
    S = o3.build_stencil2(Ac, Wh, b2)
    Acc = lambda c: osq.apply_sq_coarse(c, S)  # noqa: E731
    t3 = o3.ThreeLevelSquared(A, Vh, block, Ac, 2, 2, Wh, b2, Acc, 2, 1e-15, 500, 1)
    t2 = osq.TwoLevelSquared(A, Vh, block, Ac, 1e-15, 500, 2, 2)
    g = gaussian_fermion(L, Ls, 47)
    a, b = t3(g), t2(g)
    assert np.linalg.norm(a - b) < 1e-9 * np.linalg.norm(b)


@pytest.mark.parametrize("gamma", [1, 2])
def test_three_level_solves_converge(gamma):
    L, Ls, mf, block = (4, 4, 4, 4), 4, 0.05, (2, 2, 2, 2)
    U = prepare_gauge(L, 0.35, 48)
    A = dwf.DWF(U, M5, mf)
    prm = osq.SquaredParams(block=block, nvec=8, sweep0_iters=60, nu_pre=3, nu_post=3, coarse_tol=0.1,
                            coarse_maxiter=100)
    mg = osq.squared_setup(A, random_starts(L, Ls, 8, 49), prm)
    Lc = tuple(L[m] // block[m] for m in range(4))
    shape = tuple(Lc[::-1]) + (2, 8)
    Md = _dense(mg.coarse, shape)  # R D^+D P once, as a matrix (the same operator, faster)
    mg.coarse = lambda c: (Md @ c.ravel()).reshape(c.shape)
    t = o3.level2_setup(mg, random_coarse_starts(Lc, 8, 4, 50),
                        o3.Level2Params(block=(1, 1, 2, 2), nvec=4, null_iters=30, nu=2, coarse_tol=0.1,
                                        coarse_maxiter=100, gamma=gamma))
    b = gaussian_fermion(L, Ls, 51)
    x, rep = o3.three_level_solve(t, b, 1e-10, 300, 8)
    assert rep.converged
    assert np.linalg.norm(b - A(x)) / np.linalg.norm(b) < 1e-10
