"""Pins of the oracle's squared-operator multigrid (CPU only).

Paper: Sec. 3 (first paragraph: CG and the multigrid act on the squared
operator D^+D) and Sec. 4 (the coarse operator of the squared operator
reaches sites two hops away).  Pins: the 33-site support with blocks of
extent >= 2, the stencil equal to R D^+D P applied explicitly, Hermiticity
and positivity, gauge invariance, the smoother and CG steps against dense
least squares / dense solves, the V-cycle with a complete basis returning
D^-1, the coarse correction as an N-orthogonal projector, and a full solve
against a dense LU solve.
"""
import numpy as np
import pytest

from inputs import gaussian_fermion, prepare_gauge, random_gauge_transform, random_starts
from oracle import dwf
from oracle import squared as sq
from oracle import transfer as ot

M5 = 1.8


def _rc(shape, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)


def test_offsets_are_the_two_hop_block_stencil():
    offs = sq.OFFSETS
    assert len(offs) == len(set(offs)) == 33
    assert offs[0] == (0, 0, 0, 0)
    assert all(sum(abs(c) for c in o) <= 2 and max(abs(c) for c in o) <= 1 for o in offs)
    assert sum(1 for o in offs if sum(abs(c) for c in o) == 1) == 8
    assert sum(1 for o in offs if sum(abs(c) for c in o) == 2) == 24


def _case(L=(6, 6, 6, 6), Ls=2, block=(2, 2, 2, 2), nv=2, seed=30, mf=0.04, bc=(1, 1, 1, 1)):
    U = prepare_gauge(L, 0.5, seed)
    Vh = ot.build_basis(random_starts(L, Ls, nv, seed + 1), block)
    return U, Vh, sq.build_sq_coarse_op(Vh, U, M5, mf, block, bc)


@pytest.fixture(scope="module")
def case6():
    return _case()


def test_stencil_equals_r_dd_p(case6):
    """The 33-offset stencil applied to a random coarse vector equals R D^+ D P
    applied explicitly (the definition), in both antiperiodic and periodic bc."""
    U, Vh, Ac = case6
    c = _rc(Ac.shape[:4] + (2, Vh.shape[0]), 32)
    A = dwf.DWF(U, M5, 0.04)
    ref = sq.ExplicitCoarse(A, Vh, (2, 2, 2, 2))(c)
    assert np.linalg.norm(sq.apply_sq_coarse(c, Ac) - ref) / np.linalg.norm(ref) < 1e-13
    L, block, bc = (6, 6, 6, 6), (2, 2, 2, 2), (1, -1, 1, -1)
    Ac2 = sq.build_sq_coarse_op(Vh, U, M5, 0.04, block, bc)
    ref2 = sq.ExplicitCoarse(dwf.DWF(U, M5, 0.04, bc), Vh, block)(c)
    assert np.linalg.norm(sq.apply_sq_coarse(c, Ac2) - ref2) / np.linalg.norm(ref2) < 1e-13


def test_support_is_33_sites(case6):
    """A coarse point source reaches exactly 33 coarse sites (blocks of extent 2):
    none two blocks away in one direction, all 24 diagonal neighbours."""
    U, Vh, Ac = case6
    c = np.zeros(Ac.shape[:4] + (2, Vh.shape[0]), complex)
    c[1, 1, 1, 1] = _rc((2, Vh.shape[0]), 33)
    y = sq.apply_sq_coarse(c, Ac)
    hit = {tuple(int(v) for v in idx) for idx in np.argwhere(np.abs(y).sum(axis=(-1, -2)) > 1e-13)}
    want = {(1 + o[3], 1 + o[2], 1 + o[1], 1 + o[0]) for o in sq.OFFSETS}
    assert hit == {(t % 3, z % 3, y_ % 3, x % 3) for t, z, y_, x in want}
    assert len(hit) == 33


def test_hermitian_positive_definite(case6):
    U, Vh, Ac = case6
    n = int(np.prod(Ac.shape[:4])) * 2 * Vh.shape[0]
    shp = Ac.shape[:4] + (2, Vh.shape[0])
    M = np.array([sq.apply_sq_coarse(np.eye(n, dtype=complex)[j].reshape(shp), Ac).ravel() for j in range(n)]).T
    assert np.abs(M - M.conj().T).max() < 1e-13 * np.abs(M).max()
    assert np.linalg.eigvalsh(M).min() > 0.0


def test_gauge_invariance():
    L, Ls, block, nv = (6, 6, 6, 6), 2, (2, 2, 2, 2), 1
    U = prepare_gauge(L, 0.5, 34)
    V = random_starts(L, Ls, nv, 35)
    Om = random_gauge_transform(L, 36)
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[..., mu, :, :] = Om @ U[..., mu, :, :] @ np.conj(np.swapaxes(np.roll(Om, -1, axis=3 - mu), -1, -2))
    Vg = np.einsum("...ab,k...sib->k...sia", Om, V)
    A1 = sq.build_sq_coarse_op(ot.build_basis(V, block), U, M5, 0.02, block)
    A2 = sq.build_sq_coarse_op(ot.build_basis(Vg, block), Ug, M5, 0.02, block)
    assert np.abs(A1 - A2).max() < 1e-13 * np.abs(A1).max()


def test_mr_hpd_step_is_the_one_dimensional_least_squares_minimiser():
    L, Ls = (4, 2, 2, 2), 4
    N = sq.Normal(dwf.DWF(prepare_gauge(L, 0.4, 37), M5, 0.05))
    f = gaussian_fermion(L, Ls, 38)
    x = np.zeros_like(f)
    for k in range(1, 4):
        r = f - N(x)
        Nr = N(r)
        c, *_ = np.linalg.lstsq(Nr.reshape(-1, 1), r.ravel(), rcond=None)
        x = x + c[0] * r
        xk, rk = sq.mr_hpd_steps(N, f, k)
        assert np.linalg.norm(xk - x) / np.linalg.norm(x) < 1e-12
        assert np.linalg.norm(rk - (f - N(xk))) / np.linalg.norm(f) < 1e-12


def test_cg_is_the_galerkin_solution_on_the_krylov_space():
    """k CG steps give x_k in K_k(A, b) with A x_k - b orthogonal to K_k (the
    Galerkin condition, solved here densely on an orthonormal Krylov basis);
    run to a small tolerance CG equals numpy's dense solve."""
    rng = np.random.default_rng(39)
    B = rng.standard_normal((40, 40)) + 1j * rng.standard_normal((40, 40))
    A = B.conj().T @ B + 0.5 * np.eye(40)
    b = rng.standard_normal(40) + 1j * rng.standard_normal(40)
    op = lambda v: A @ v
    for k in (1, 3, 7):
        K = [b]
        for _ in range(k - 1):
            K.append(A @ K[-1])
        Q, _ = np.linalg.qr(np.stack(K, axis=1))
        xg = Q @ np.linalg.solve(Q.conj().T @ A @ Q, Q.conj().T @ b)
        xk, it = sq.cg(op, b, 1e-300, k)
        assert it == k
        assert np.linalg.norm(xk - xg) / np.linalg.norm(xg) < 1e-10
    x, _ = sq.cg(op, b, 1e-13, 1000)
    assert np.linalg.norm(x - np.linalg.solve(A, b)) / np.linalg.norm(x) < 1e-10


def _dense_D(U, Ls, mf):
    L = U.shape[:4]
    n = 12 * int(np.prod(L)) * Ls
    shape = tuple(L) + (Ls, 4, 3)
    return np.array([dwf.apply_dwf(np.eye(n, dtype=complex)[j].reshape(shape), U, M5, mf).ravel()
                     for j in range(n)]).T


def test_vcycle_with_complete_basis_is_d_inverse():
    """2^4 x Ls 2 with 1^4 blocks and Nv = 12 (every dof of a block and
    chirality): P is unitary, the exact coarse solve inverts N, and M(r) =
    N^-1 D^+ r = D^-1 r, checked against a dense solve."""
    L, Ls, block, nv, mf = (2, 2, 2, 2), 2, (1, 1, 1, 1), 12, 0.05
    U = prepare_gauge(L, 0.4, 40)
    A = dwf.DWF(U, M5, mf)
    Vh = ot.build_basis(random_starts(L, Ls, nv, 41), block)
    coarse = sq.ExplicitCoarse(A, Vh, block)
    M = sq.TwoLevelSquared(A, Vh, block, coarse, 1e-15, 5000, 2, 2)
    r = gaussian_fermion(L, Ls, 42)
    D = _dense_D(U, Ls, mf)
    want = np.linalg.solve(D, r.ravel()).reshape(r.shape)
    assert np.linalg.norm(M(r) - want) / np.linalg.norm(want) < 1e-9


def test_coarse_correction_is_an_n_orthogonal_projector():
    """With no smoothing and an exact coarse solve, E = 1 - P A_c^-1 R N is
    idempotent and N-self-adjoint (<N E x, y> = <N x, E y>)."""
    L, Ls, block, nv, mf = (4, 2, 2, 2), 2, (2, 2, 1, 1), 3, 0.05
    U = prepare_gauge(L, 0.4, 43)
    A = dwf.DWF(U, M5, mf)
    N = sq.Normal(A)
    Vh = ot.build_basis(random_starts(L, Ls, nv, 44), block)
    T = sq.TwoLevelSquared(A, Vh, block, sq.ExplicitCoarse(A, Vh, block), 1e-15, 5000, 0, 0)
    E = lambda x: x - T.vcycle(N(x))
    x = gaussian_fermion(L, Ls, 45)
    y = gaussian_fermion(L, Ls, 46)
    Ex = E(x)
    assert np.linalg.norm(E(Ex) - Ex) / np.linalg.norm(Ex) < 1e-10
    a = np.vdot(N(Ex), y)
    b = np.vdot(N(x), E(y))
    assert abs(a - b) / abs(a) < 1e-10


def test_squared_mg_solve_matches_dense_lu():
    L, Ls, block, mf = (2, 2, 2, 4), 4, (2, 2, 2, 2), 0.05
    U = prepare_gauge(L, 0.4, 47)
    A = dwf.DWF(U, M5, mf)
    prm = sq.SquaredParams(block=block, nvec=12, sweep0_iters=100, nu_pre=4, nu_post=4, coarse_tol=0.1)
    mg = sq.squared_setup(A, random_starts(L, Ls, 12, 48), prm)
    b = gaussian_fermion(L, Ls, 49)
    x, rep = sq.squared_solve(mg, b, 1e-10, 300, 8)
    assert rep.converged and rep.true_relres < 1e-10
    xd = np.linalg.solve(_dense_D(U, Ls, mf), b.ravel()).reshape(b.shape)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-7
