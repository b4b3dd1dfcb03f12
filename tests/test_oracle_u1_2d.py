"""Pins of the 2D U(1) oracle (the paper's Sec. 3 test problem, Fig. 2) and
of its gauge-field generator, against what the mathematics fixes:

* the free operator on a plane wave equals its momentum-space form, a
  2 Ls x 2 Ls matrix built here from the Fourier transform of each term
  (periodic and antiperiodic directions, D and D^+);
* at M5 = 1, m_f = 0 the free operator annihilates the constant spin-0 field
  on the wall s = Ls - 1, and with m_f it maps it to m_f times the spin-0
  field on s = 0 (the wall coupling);
* gamma_5 R_5 hermiticity, D^+ = G D G, on a random U(1) field, which checks
  the term-by-term adjoint independently; the adjoint identity; gauge
  covariance;
* the Dirac matrices: the Pauli matrices sigma_1, sigma_2 with
  gamma_5 = -i g_x g_y = sigma_3 and the Clifford relations;
* the block basis: orthonormal panels, R P = 1, and P R
  reproducing every near-null vector it was built from;
* the probed 9-offset A_c equal to R D^+D P applied directly, and Hermitian;
* with a complete basis (as many vectors as a block's dof per chirality) and
  an exact coarse solve, the V-cycle preconditioner is D^-1 itself, checked
  against a dense solve;
* the Metropolis generator's mean plaquette against the infinite-volume
  value I_1(beta) / I_0(beta) of the 2D U(1) Wilson action.
"""

import numpy as np
import pytest
from scipy.special import i0, i1

from inputs import (gaussian_fermion2d, plaquette_angles, point_sources2d, quenched_u1_2d, random_starts2d,
                    random_u1_transform)
from oracle import solvers as sol
from oracle import u1_2d as o


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def momentum_matrix(p, Ls, M5, mf, dagger):
    """K(p) acting on phi (Ls, 2) for psi(x, s) = exp(i p.x) phi(s), U = 1:
    each hop psi(x +- mu) contributes exp(+- i p_mu)."""
    n = 2 * Ls
    K = np.zeros((n, n), dtype=np.complex128)
    g = [np.array([[0, 1], [1, 0]], dtype=np.complex128), np.array([[0, -1j], [1j, 0]], dtype=np.complex128)]
    sg = -1.0 if not dagger else 1.0
    site = (3.0 - M5) * np.eye(2, dtype=np.complex128)
    for mu in range(2):
        site = site - 0.5 * ((np.eye(2) + sg * g[mu]) * np.exp(1j * p[mu])
                             + (np.eye(2) - sg * g[mu]) * np.exp(-1j * p[mu]))
    Pp, Pm = np.diag([1.0, 0.0]), np.diag([0.0, 1.0])
    up, dn = (Pm, Pp) if not dagger else (Pp, Pm)
    for s in range(Ls):
        K[2 * s:2 * s + 2, 2 * s:2 * s + 2] += site
        t = (s + 1) % Ls
        K[2 * s:2 * s + 2, 2 * t:2 * t + 2] += (mf if s == Ls - 1 else -1.0) * up
        t = (s - 1) % Ls
        K[2 * s:2 * s + 2, 2 * t:2 * t + 2] += (mf if s == 0 else -1.0) * dn
    return K


@pytest.mark.parametrize("bc,dagger", [((1, 1), False), ((1, -1), False), ((-1, 1), True), ((1, 1), True)])
def test_free_plane_wave_matches_momentum_space(bc, dagger):
    L, Ls, M5, mf = (6, 4), 3, 1.3, 0.07
    rng = np.random.default_rng(5)
    U = np.ones((L[1], L[0], 2), dtype=np.complex128)
    for nx, ny in ((0, 0), (1, 2), (5, 3)):
        p = [2 * np.pi * (nx + (0.5 if bc[0] < 0 else 0.0)) / L[0],
             2 * np.pi * (ny + (0.5 if bc[1] < 0 else 0.0)) / L[1]]
        phi = rng.standard_normal((Ls, 2)) + 1j * rng.standard_normal((Ls, 2))
        y, x = np.meshgrid(np.arange(L[1]), np.arange(L[0]), indexing="ij")
        wave = np.exp(1j * (p[0] * x + p[1] * y))
        psi = wave[..., None, None] * phi
        got = o.apply_dwf2(psi, U, M5, mf, bc, dagger)
        want = wave[..., None, None] * (momentum_matrix(p, Ls, M5, mf, dagger) @ phi.reshape(-1)).reshape(Ls, 2)
        assert rel(got, want) < 1e-13


def test_dirac_matrices():
    g = o.GAMMA2
    for mu in range(2):
        for nu in range(2):
            assert np.abs(g[mu] @ g[nu] + g[nu] @ g[mu] - 2.0 * (mu == nu) * np.eye(2)).max() == 0.0
    assert np.abs(o.GAMMA5_2 - (-1j) * g[0] @ g[1]).max() == 0.0
    assert np.abs(o.GAMMA5_2 - np.diag([1.0, -1.0])).max() == 0.0


def test_free_wall_mode():
    L, Ls = (4, 6), 5
    U = np.ones((L[1], L[0], 2), dtype=np.complex128)
    e = np.zeros((L[1], L[0], Ls, 2), dtype=np.complex128)
    e[:, :, Ls - 1, 0] = 1.0
    assert np.abs(o.apply_dwf2(e, U, 1.0, 0.0)).max() < 1e-15
    f = np.zeros_like(e)
    f[:, :, 0, 0] = 1.0
    assert np.abs(o.apply_dwf2(e, U, 1.0, 0.25) - 0.25 * f).max() < 1e-15


@pytest.fixture(scope="module")
def field():
    return quenched_u1_2d((6, 4), 2.0, 3, sweeps=20)


def test_gamma5_r5_hermiticity_and_adjoint(field):
    U, Ls, M5, mf = field, 4, 1.0, 0.05
    psi = gaussian_fermion2d((6, 4), Ls, 9)
    chi = gaussian_fermion2d((6, 4), Ls, 10)
    lhs = o.apply_dwf2(psi, U, M5, mf, (1, -1), dagger=True)
    rhs = o.gamma5_R5_2(o.apply_dwf2(o.gamma5_R5_2(psi), U, M5, mf, (1, -1)))
    assert rel(lhs, rhs) < 1e-14
    a = np.vdot(chi, o.apply_dwf2(psi, U, M5, mf, (1, -1)))
    b = np.vdot(o.apply_dwf2(chi, U, M5, mf, (1, -1), dagger=True), psi)
    assert abs(a - b) < 1e-12 * abs(a)


def test_gauge_covariance(field):
    U, Ls = field, 3
    g = random_u1_transform((6, 4), 4)
    Ug = np.empty_like(U)
    Ug[..., 0] = g * U[..., 0] * np.conj(np.roll(g, -1, axis=1))
    Ug[..., 1] = g * U[..., 1] * np.conj(np.roll(g, -1, axis=0))
    psi = gaussian_fermion2d((6, 4), Ls, 2)
    got = o.apply_dwf2(g[..., None, None] * psi, Ug, 0.9, 0.1)
    want = g[..., None, None] * o.apply_dwf2(psi, U, 0.9, 0.1)
    assert rel(got, want) < 1e-14


def test_basis_transfer_identities(field):
    L, Ls, block, nv = (6, 4), 3, (2, 2), 5
    V = random_starts2d(L, Ls, nv, 8)
    Vh = o.build_basis2d(V, block)
    g = o.block_split2(Vh, block)
    for chi in range(2):
        panel = np.moveaxis(g[..., chi].reshape(nv, 2, 3, -1), 0, -1)  # (Yc, Xc, rows, nv)
        gram = np.einsum("yxrk,yxrl->yxkl", np.conj(panel), panel)
        assert np.abs(gram - np.eye(nv)).max() < 1e-13
    c = np.random.default_rng(1).standard_normal((2, 3, 2, nv)) + 0j
    assert rel(o.restrict2d(o.prolong2d(c, Vh, block), Vh, block), c) < 1e-14
    for k in range(nv):
        for chi in range(2):
            vk = np.zeros_like(V[k])
            vk[..., chi] = V[k][..., chi]
            assert rel(o.prolong2d(o.restrict2d(vk, Vh, block), Vh, block), vk) < 1e-12


def test_probed_stencil_equals_galerkin_product(field):
    L, Ls, block, nv = (6, 6), 2, (2, 2), 3
    U = quenched_u1_2d(L, 2.0, 4, sweeps=20)
    V = random_starts2d(L, Ls, nv, 6)
    Vh = o.build_basis2d(V, block)
    A = o.DWF2(U, 1.0, 0.05, (1, -1))
    Ac = o.build_sq_coarse_op2d(Vh, U, 1.0, 0.05, block, (1, -1))
    ex = o.ExplicitCoarse2D(A, Vh, block)
    rng = np.random.default_rng(3)
    c = rng.standard_normal((3, 3, 2, nv)) + 1j * rng.standard_normal((3, 3, 2, nv))
    assert rel(o.apply_sq_coarse2d(c, Ac), ex(c)) < 1e-13
    d = rng.standard_normal((3, 3, 2, nv)) + 1j * rng.standard_normal((3, 3, 2, nv))
    a = np.vdot(d, o.apply_sq_coarse2d(c, Ac))
    b = np.vdot(o.apply_sq_coarse2d(d, Ac), c)
    assert abs(a - b) < 1e-12 * abs(a)


def test_complete_basis_vcycle_is_the_inverse():
    L, Ls, block = (4, 4), 2, (2, 2)
    nv = 2 * 2 * Ls  # a block's dof per chirality: every column of the panel
    U = quenched_u1_2d(L, 2.0, 5, sweeps=20)
    A = o.DWF2(U, 1.0, 0.1)
    p = o.U1Params(block=block, nvec=nv, sweep0_iters=3, nu_pre=2, nu_post=2, coarse_tol=1e-14,
                   coarse_maxiter=2000)
    mg = o.u1_setup(A, random_starts2d(L, Ls, nv, 2), p)
    n = L[0] * L[1] * Ls * 2
    Dm = np.zeros((n, n), dtype=np.complex128)
    for i in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[i] = 1.0
        Dm[:, i] = o.apply_dwf2(e.reshape(L[1], L[0], Ls, 2), U, 1.0, 0.1).reshape(-1)
    r = gaussian_fermion2d(L, Ls, 4)
    z = mg.preconditioner()(r)
    assert rel(z.reshape(-1), np.linalg.solve(Dm, r.reshape(-1))) < 1e-10


def test_squared_multigrid_solves():
    L, Ls = (8, 8), 4
    U = quenched_u1_2d(L, 4.0, 7, sweeps=50)
    A = o.DWF2(U, 1.0, 0.02)
    p = o.U1Params(block=(4, 4), nvec=4, sweep0_iters=40, nu_pre=3, nu_post=3, coarse_tol=0.1)
    mg = o.u1_setup(A, random_starts2d(L, Ls, 4, 21), p)
    b = point_sources2d(L, Ls)[0]
    x, rep, M = o.u1_solve(mg, b, 1e-10, 200, 8)
    assert rep.converged
    assert rel(o.apply_dwf2(x, U, 1.0, 0.02), b) < 1e-10
    assert len(M.coarse_iters) == rep.iters


def test_metropolis_plaquette_matches_bessel_ratio():
    beta = 4.0
    vals = [np.cos(plaquette_angles(np.angle(quenched_u1_2d((20, 20), beta, s, sweeps=200)))).mean()
            for s in range(12)]
    assert abs(np.mean(vals) - i1(beta) / i0(beta)) < 0.015
    U = quenched_u1_2d((4, 6), beta, 1, sweeps=5)
    assert np.abs(np.abs(U) - 1.0).max() < 1e-15
