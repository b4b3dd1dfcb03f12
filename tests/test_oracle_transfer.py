"""Pins of the oracle's transfer operators, coarse operator and solvers (CPU only).

Paper: Sec. 1 (R P = 1), Sec. 2 (blocks over all of Ls, V-cycle), Sec. 3
(flexible GCR, CG on the squared operator), Sec. 4 (one-hop coarse stencil of
the unsquared operator).  Pins are library routines (numpy QR, lstsq, dense
solves), invariants and exact special cases.
"""
import numpy as np
import pytest

from inputs import gaussian_fermion, prepare_gauge, random_gauge_transform, random_starts
from oracle import coarse as oc
from oracle import dwf
from oracle import setup as osu
from oracle import solvers as osv
from oracle import transfer as ot

M5 = 1.8


def _rng_coarse(shape, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)


def test_basis_equals_numpy_qr():
    """The block basis is the thin QR factor (positive real diagonal) of each chirality panel."""
    L, Ls, block, nv = (4, 4, 2, 2), 4, (2, 2, 2, 2), 6
    V = random_starts(L, Ls, nv, 3)
    Vh = ot.build_basis(V, block)
    A = ot._chiral_panels(V, block)
    Q, R = np.linalg.qr(A)
    d = np.diagonal(R, axis1=-2, axis2=-1)
    Q = Q * (d / np.abs(d))[..., None, :]
    assert np.abs(ot._chiral_panels(Vh, block) - Q).max() < 1e-13


def test_rp_is_identity_and_r_is_p_adjoint():
    L, Ls, block, nv = (4, 4, 4, 2), 6, (2, 2, 2, 2), 8
    V = random_starts(L, Ls, nv, 4)
    Vh = ot.build_basis(V, block)
    c = _rng_coarse((1, 2, 2, 2, 2, nv), 5)
    x = gaussian_fermion(L, Ls, 6)
    assert np.linalg.norm(ot.restrict(ot.prolong(c, Vh, block), Vh, block) - c) / np.linalg.norm(c) < 1e-14
    lhs = np.vdot(ot.restrict(x, Vh, block), c)
    rhs = np.vdot(x, ot.prolong(c, Vh, block))
    assert abs(lhs - rhs) / abs(rhs) < 1e-13


def test_span_contains_the_input_vectors():
    """P R v_k = v_k: every near-null vector lies in the block span (Sec. 2)."""
    L, Ls, block, nv = (4, 4, 2, 2), 4, (2, 2, 2, 2), 5
    V = random_starts(L, Ls, nv, 8)
    Vh = ot.build_basis(V, block)
    for k in range(nv):
        back = ot.prolong(ot.restrict(V[k], Vh, block), Vh, block)
        assert np.linalg.norm(back - V[k]) / np.linalg.norm(V[k]) < 1e-13


def test_rank_deficiency_detected():
    L, Ls, block = (2, 2, 2, 2), 2, (2, 2, 2, 2)
    V = random_starts(L, Ls, 3, 9)
    V[2] = 2.0 * V[0]
    with pytest.raises(ot.RankDeficientError):
        ot.build_basis(V, block)


def _coarse_case(L=(4, 4, 6, 6), Ls=4, block=(2, 2, 2, 2), nv=6, seed=12, bc=(1, 1, 1, 1)):
    U = prepare_gauge(L, 0.5, seed)
    V = random_starts(L, Ls, nv, seed + 1)
    Vh = ot.build_basis(V, block)
    return U, Vh, oc.build_coarse_op(Vh, U, M5, 0.03, block, bc)


@pytest.mark.parametrize("L,block,bc", [
    ((4, 4, 6, 6), (2, 2, 2, 2), (1, 1, 1, 1)),     # coarse extents 2, 2, 3, 3
    ((4, 4, 4, 4), (2, 2, 2, 2), (1, -1, 1, -1)),   # all extents 2: +mu and -mu alias
    ((2, 4, 2, 4), (2, 2, 2, 2), (1, 1, 1, 1)),     # coarse extent 1 in x, z: d aliases to self
])
def test_coarse_operator_is_r_d_p(L, block, bc):
    Ls, nv = 4, 6
    U = prepare_gauge(L, 0.5, 12)
    Vh = ot.build_basis(random_starts(L, Ls, nv, 13), block)
    Dc = oc.build_coarse_op(Vh, U, M5, 0.03, block, bc)
    Lc = tuple(L[m] // block[m] for m in range(4))
    y = _rng_coarse(Lc[::-1] + (2, nv), 14)
    ref = ot.restrict(dwf.apply_dwf(ot.prolong(y, Vh, block), U, M5, 0.03, bc), Vh, block)
    assert np.linalg.norm(oc.apply_coarse(y, Dc) - ref) / np.linalg.norm(ref) < 1e-13
    # adjoint stencil
    x = _rng_coarse(Lc[::-1] + (2, nv), 15)
    a = np.vdot(x, oc.apply_coarse(y, Dc))
    b = np.vdot(oc.apply_coarse(x, Dc, dagger=True), y)
    assert abs(a - b) / abs(a) < 1e-13


def test_coarse_dense_galerkin_tiny():
    """On 2^4 x Ls4 with 2^4 blocks (one coarse site) the stencil sums to the dense P^+ D P."""
    L, Ls, block, nv = (2, 2, 2, 2), 4, (2, 2, 2, 2), 8
    U = prepare_gauge(L, 0.4, 16)
    Vh = ot.build_basis(random_starts(L, Ls, nv, 17), block)
    Dc = oc.build_coarse_op(Vh, U, M5, 0.05, block)
    P = np.array([Vh[k].ravel() * m for m in (np.tile(np.repeat([1, 1, 0, 0], 3), 16 * Ls),
                                              np.tile(np.repeat([0, 0, 1, 1], 3), 16 * Ls)) for k in range(nv)]).T
    n = 12 * 16 * Ls
    D = np.array([dwf.apply_dwf(np.eye(n, dtype=complex)[j].reshape(2, 2, 2, 2, Ls, 4, 3), U, M5, 0.05).ravel() for j in range(n)]).T
    dense = P.conj().T @ D @ P
    assert np.abs(Dc[0, 0, 0, 0].sum(axis=0) - dense).max() < 1e-13


def test_coarse_stencil_support_is_nine_sites():
    L, Ls, block, nv = (6, 6, 6, 6), 2, (2, 2, 2, 2), 2
    U = prepare_gauge(L, 0.4, 18)
    Vh = ot.build_basis(random_starts(L, Ls, nv, 19), block)
    Dc = oc.build_coarse_op(Vh, U, M5, 0.05, block)
    c = np.zeros((3, 3, 3, 3, 2, nv), complex)
    c[1, 1, 1, 1] = _rng_coarse((2, nv), 20)
    y = oc.apply_coarse(c, Dc)
    assert len(np.argwhere(np.abs(y).sum(axis=(-1, -2)) > 1e-14)) == 9


def test_coarse_operator_gauge_invariant():
    L, Ls, block, nv = (4, 4, 4, 4), 4, (2, 2, 2, 2), 4
    U = prepare_gauge(L, 0.5, 21)
    V = random_starts(L, Ls, nv, 22)
    Om = random_gauge_transform(L, 23)
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[..., mu, :, :] = Om @ U[..., mu, :, :] @ np.conj(np.swapaxes(np.roll(Om, -1, axis=3 - mu), -1, -2))
    Vg = np.einsum("...ab,k...sib->k...sia", Om, V)
    D1 = oc.build_coarse_op(ot.build_basis(V, block), U, M5, 0.02, block)
    D2 = oc.build_coarse_op(ot.build_basis(Vg, block), Ug, M5, 0.02, block)
    assert np.abs(D1 - D2).max() < 1e-13


# ---------------------------------------------------------------- solvers

class _Dense:
    def __init__(self, A):
        self.A = A
        self.napply = 0

    def __call__(self, v):
        self.napply += 1
        return (self.A @ v.ravel()).reshape(v.shape)

    def dag(self, v):
        self.napply += 1
        return (self.A.conj().T @ v.ravel()).reshape(v.shape)


def test_mr_exact_for_scaled_identity_and_monotone():
    A = _Dense(2.5j * np.eye(30))
    b = _rng_coarse(30, 1)
    x, r = osv.mr_steps(A, b, 1)
    assert np.linalg.norm(A(x) - b) < 1e-13
    r0 = np.random.default_rng(2)
    M = r0.standard_normal((40, 40)) + 1j * r0.standard_normal((40, 40)) + 8 * np.eye(40)
    A2 = _Dense(M)
    prev = np.linalg.norm(b := _rng_coarse(40, 3))
    for k in range(1, 8):
        _, rk = osv.mr_normal_steps(A2, b, k)
        assert np.linalg.norm(rk) <= prev * (1 + 1e-14)
        prev = np.linalg.norm(rk)


def test_gcr_is_minimum_residual_over_krylov_space():
    """k steps of (unpreconditioned, unrestarted) GCR give min |b - A x| over K_k(A, b)."""
    r = np.random.default_rng(4)
    n = 60
    M = r.standard_normal((n, n)) + 1j * r.standard_normal((n, n)) + 6 * np.eye(n)
    b = _rng_coarse(n, 5)
    for k in (1, 3, 6):
        x, _ = osv.gcr_fixed(_Dense(M), b, np.zeros(n, complex), k)
        K = np.array([np.linalg.matrix_power(M, j) @ b for j in range(k)]).T
        c, *_ = np.linalg.lstsq(M @ K, b, rcond=None)
        assert abs(np.linalg.norm(b - M @ x) - np.linalg.norm(b - M @ K @ c)) < 1e-10 * np.linalg.norm(b)


def test_cgne_matches_dense_solve():
    r = np.random.default_rng(6)
    n = 50
    M = r.standard_normal((n, n)) + 1j * r.standard_normal((n, n)) + 5 * np.eye(n)
    b = _rng_coarse(n, 7)
    x, rep = osv.cgne(_Dense(M), b, 1e-12, 500)
    assert np.linalg.norm(x - np.linalg.solve(M, b)) / np.linalg.norm(x) < 1e-10


def test_vcycle_with_complete_basis_is_exact():
    """Sec. 2 V-cycle with P unitary (1^4 blocks, all 48 dof) and an exact coarse solve gives A^-1 b."""
    L, Ls, block, nv = (2, 2, 2, 2), 4, (1, 1, 1, 1), 24
    U = prepare_gauge(L, 0.5, 24)
    A = dwf.DWF(U, M5, 0.02)
    Vh = ot.build_basis(random_starts(L, Ls, nv, 25), block)
    Dc = oc.build_coarse_op(Vh, U, M5, 0.02, block)
    n = 16 * 2 * nv
    Mc = np.array([oc.apply_coarse(np.eye(n, dtype=complex)[j].reshape(2, 2, 2, 2, 2, nv), Dc).ravel() for j in range(n)]).T
    Minv = np.linalg.inv(Mc)
    cs = lambda b2: (Minv @ b2.ravel()).reshape(b2.shape)
    b = gaussian_fermion(L, Ls, 26)
    for nu in (0, 3):
        T = osv.TwoLevel(A, lambda x: ot.restrict(x, Vh, block), lambda c: ot.prolong(c, Vh, block), cs,
                         osv.mr_normal_steps, nu, nu)
        x = T(b)
        assert np.linalg.norm(b - A(x)) / np.linalg.norm(b) < 1e-12


def test_coarse_correction_is_a_projector():
    """With nu1 = nu3 = 0 and an exact coarse solve, E = 1 - P Dc^-1 R A satisfies E E = E."""
    L, Ls, block, nv = (2, 2, 2, 4), 2, (2, 2, 2, 2), 4
    U = prepare_gauge(L, 0.5, 27)
    A = dwf.DWF(U, M5, 0.05)
    Vh = ot.build_basis(random_starts(L, Ls, nv, 28), block)
    Dc = oc.build_coarse_op(Vh, U, M5, 0.05, block)
    n = 2 * 2 * nv
    Mc = np.array([oc.apply_coarse(np.eye(n, dtype=complex)[j].reshape(2, 1, 1, 1, 2, nv), Dc).ravel() for j in range(n)]).T
    Minv = np.linalg.inv(Mc)
    T = osv.TwoLevel(A, lambda x: ot.restrict(x, Vh, block), lambda c: ot.prolong(c, Vh, block),
                     lambda b2: (Minv @ b2.ravel()).reshape(b2.shape), osv.mr_normal_steps, 0, 0)
    E = lambda e: e - T(A(e))
    e = gaussian_fermion(L, Ls, 29)
    assert np.linalg.norm(E(E(e)) - E(e)) / np.linalg.norm(E(e)) < 1e-12


def test_mg_solve_matches_dense_lu_on_tiny_lattice():
    """Full two-level MG-FGCR on 2^4 x Ls4 reaches 1e-10 and agrees with a dense LU solve."""
    L, Ls = (2, 2, 2, 2), 4
    U = prepare_gauge(L, 0.4, 30)
    A = dwf.DWF(U, M5, 0.01)
    # 1^4 blocks, 8 adaptive vectors + reflections: the smallest coarse space that
    # converges here (larger blocks stagnate at restart 8 on this 768-dof problem)
    params = osu.MGParams(block=(1, 1, 1, 1), nvec=16, sweeps=1, sweep0_iters=50)
    mg = osu.adaptive_setup(A, random_starts(L, Ls, 8, 31), params)
    b = gaussian_fermion(L, Ls, 32)
    x, rep = osu.mg_solve(mg, b, 1e-10, 300, 8)
    assert rep.converged and rep.true_relres < 1e-10
    n = 12 * 16 * Ls
    D = np.array([dwf.apply_dwf(np.eye(n, dtype=complex)[j].reshape(x.shape), U, M5, 0.01).ravel() for j in range(n)]).T
    xlu = np.linalg.solve(D, b.ravel())
    kappa = np.linalg.cond(D)
    assert np.linalg.norm(x.ravel() - xlu) / np.linalg.norm(xlu) < kappa * 1e-10
