"""Pins of the oracle's domain-wall operator (CPU only).

The paper (Sec. 2 fifth-dimension paragraph, Sec. 4) never writes D; these
tests pin the oracle's reading (Shamir form, chiral gamma basis) to facts that
do not come from the oracle's own code: the Clifford algebra, the
momentum-space closed form of the free operator, the textbook Wilson operator
at Ls = 1, the p = 0 determinant, adjointness, gamma_5 R_5 hermiticity, gauge
covariance and the size of the stencil (one site plus ten neighbours).
"""
import itertools

import numpy as np
import pytest

from inputs import gaussian_fermion, prepare_gauge, random_gauge_transform
from oracle import dwf

M5 = 1.8


def test_gamma_matrices_clifford_and_chiral_basis():
    g = dwf.GAMMA
    for a, b in itertools.product(range(4), range(4)):
        assert np.allclose(g[a] @ g[b] + g[b] @ g[a], 2.0 * (a == b) * np.eye(4), atol=1e-15)
    for a in range(4):
        assert np.allclose(g[a], g[a].conj().T)
    assert np.allclose(dwf.GAMMA5, np.diag([1, 1, -1, -1]))
    assert np.allclose(dwf.PPLUS, np.diag([1, 1, 0, 0]))
    assert np.allclose(dwf.PMINUS, np.diag([0, 0, 1, 1]))


def _free_links(L):
    U = np.zeros(tuple(L[::-1]) + (4, 3, 3), dtype=np.complex128)
    U[...] = np.eye(3)
    return U


def _closed_form(p, Ls, mf, dagger=False):
    """4Ls x 4Ls momentum-space matrix of the free Shamir operator (derived by hand).

    D(p)_{ss'} = d_{ss'}[(1 - M5 + sum(1 - cos p)) + i sum g_mu sin p_mu]
                 - d_{s',s+1} P_- - d_{s',s-1} P_+
                 + m_f (d_{s,Ls-1} d_{s',0} P_- + d_{s,0} d_{s',Ls-1} P_+).
    """
    Pp = np.diag([1, 1, 0, 0]).astype(complex)
    Pm = np.diag([0, 0, 1, 1]).astype(complex)
    s1 = np.array([[0, 1], [1, 0]]); s2 = np.array([[0, -1j], [1j, 0]]); s3 = np.array([[1, 0], [0, -1]])
    Z = np.zeros((2, 2)); I2 = np.eye(2)
    G = [np.block([[Z, -1j * s], [1j * s, Z]]) for s in (s1, s2, s3)] + [np.block([[Z, I2], [I2, Z]])]
    D = np.zeros((Ls, 4, Ls, 4), dtype=complex)
    for s in range(Ls):
        D[s, :, s, :] = (1 - M5 + np.sum(1 - np.cos(p))) * np.eye(4) + 1j * sum(G[m] * np.sin(p[m]) for m in range(4))
        if s + 1 < Ls:
            D[s, :, s + 1, :] -= Pm
        if s >= 1:
            D[s, :, s - 1, :] -= Pp
    D[Ls - 1, :, 0, :] += mf * Pm
    D[0, :, Ls - 1, :] += mf * Pp
    D = D.reshape(4 * Ls, 4 * Ls)
    return D.conj().T.reshape(Ls, 4, Ls, 4) if dagger else D.reshape(Ls, 4, Ls, 4)


@pytest.mark.parametrize("L,Ls,mf,bc,n", [
    ((4, 4, 4, 4), 8, 0.01, (1, 1, 1, 1), (1, 2, 0, 3)),
    ((4, 6, 2, 8), 5, 0.1, (1, 1, 1, -1), (3, 1, 1, 2)),
    ((3, 4, 5, 6), 3, 0.3, (-1, 1, -1, 1), (2, 0, 4, 5)),
])
@pytest.mark.parametrize("dagger", [False, True])
def test_free_field_closed_form(L, Ls, mf, bc, n, dagger):
    # momenta allowed by the boundary conditions: 2 pi n / L, or (2n+1) pi / L when antiperiodic
    p = np.array([(2 * n[m] + (1 if bc[m] < 0 else 0)) * np.pi / L[m] for m in range(4)])
    rng = np.random.default_rng(7)
    chi = rng.standard_normal((Ls, 4, 3)) + 1j * rng.standard_normal((Ls, 4, 3))
    t, z, y, x = np.meshgrid(*[np.arange(l) for l in L[::-1]], indexing="ij")
    ph = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    psi = ph[..., None, None, None] * chi
    out = dwf.apply_dwf(psi, _free_links(L), M5, mf, bc, dagger=dagger)
    ref = ph[..., None, None, None] * np.einsum("sitj,tjc->sic", _closed_form(p, Ls, mf, dagger), chi)
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref) < 1e-13


def test_p0_chirality_block_determinant():
    """At p = 0 each chirality block is bidiagonal with a twisted corner: |det| = |(1-M5)^Ls + m_f|."""
    for Ls, mf in ((4, 0.1), (8, 0.01), (16, 0.001)):
        D = _closed_form(np.zeros(4), Ls, mf)
        for chi in (0, 1):
            sl = slice(2 * chi, 2 * chi + 1)   # one spin of the chirality (the two spins are identical)
            blk = D[:, sl, :, sl].reshape(Ls, Ls)
            assert abs(abs(np.linalg.det(blk)) - abs((1 - M5) ** Ls + mf)) < 1e-12


def test_ls1_is_textbook_wilson():
    """Ls = 1 reduces D to the Wilson operator with mass 1 - M5 + m_f (random gauge field)."""
    L = (4, 4, 4, 4)
    U = prepare_gauge(L, 0.5, 3)
    psi = gaussian_fermion(L, 1, 4)
    mf = 0.07
    d = dwf.apply_dwf(psi, U, M5, mf)
    w = dwf.apply_wilson(psi[..., 0, :, :], U, 1 - M5 + mf)
    assert np.linalg.norm(d[..., 0, :, :] - w) / np.linalg.norm(w) < 1e-14


def test_ls1_free_wilson_spectrum():
    """Free Wilson D^+D eigenvalues: (m + sum(1-cos p))^2 + sum sin^2 p, from the Clifford algebra."""
    L = (4, 4, 2, 2)
    mass = 1 - M5 + 0.05
    U = _free_links(L)
    n = 12 * int(np.prod(L))
    cols = []
    for j in range(n):
        e = np.zeros(n, complex)
        e[j] = 1
        cols.append(dwf.apply_dwf(e.reshape(tuple(L[::-1]) + (1, 4, 3)), U, M5, 0.05).ravel())
    A = np.array(cols).T
    ev = np.sort(np.linalg.eigvalsh(A.conj().T @ A))
    ref = []
    for n4 in itertools.product(*[range(l) for l in L]):
        p = 2 * np.pi * np.array(n4) / np.array(L)
        ref += [(mass + np.sum(1 - np.cos(p))) ** 2 + np.sum(np.sin(p) ** 2)] * 12
    assert np.allclose(ev, np.sort(ref), atol=1e-12)


@pytest.mark.parametrize("bc", [(1, 1, 1, 1), (1, -1, 1, -1)])
def test_adjoint_and_gamma5_r5_hermiticity(bc):
    L, Ls = (4, 4, 2, 6), 6
    U = prepare_gauge(L, 0.6, 5)
    x = gaussian_fermion(L, Ls, 6)
    y = gaussian_fermion(L, Ls, 7)
    Dy = dwf.apply_dwf(y, U, M5, 0.02, bc)
    Ddx = dwf.apply_dwf(x, U, M5, 0.02, bc, dagger=True)
    assert abs(np.vdot(x, Dy) - np.vdot(Ddx, y)) / abs(np.vdot(x, Dy)) < 1e-13
    H = dwf.gamma5_R5(dwf.apply_dwf(dwf.gamma5_R5(x), U, M5, 0.02, bc))
    assert np.linalg.norm(H - Ddx) / np.linalg.norm(Ddx) < 1e-14


def test_gauge_covariance():
    L, Ls = (4, 4, 4, 2), 4
    U = prepare_gauge(L, 0.5, 8)
    psi = gaussian_fermion(L, Ls, 9)
    Om = random_gauge_transform(L, 10)
    Ug = np.empty_like(U)
    for mu in range(4):
        Om_fwd = np.roll(Om, -1, axis=3 - mu)
        Ug[..., mu, :, :] = Om @ U[..., mu, :, :] @ np.conj(np.swapaxes(Om_fwd, -1, -2))
    rot = lambda f: np.einsum("...ab,...sib->...sia", Om, f)
    lhs = dwf.apply_dwf(rot(psi), Ug, M5, 0.01)
    rhs = rot(dwf.apply_dwf(psi, U, M5, 0.01))
    assert np.linalg.norm(lhs - rhs) / np.linalg.norm(rhs) < 1e-13


def test_stencil_is_site_plus_ten_neighbours():
    """Paper Sec. 4: a site couples to itself and its 10 unit neighbours in 5D."""
    L, Ls = (4, 3, 5, 3), 5
    U = prepare_gauge(L, 0.4, 11)
    src = np.zeros(tuple(L[::-1]) + (Ls, 4, 3), dtype=complex)
    rng = np.random.default_rng(0)
    src[1, 2, 1, 2, 2] = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    out = dwf.apply_dwf(src, U, M5, 0.05)
    support = np.argwhere(np.abs(out).sum(axis=(-1, -2)) > 1e-14)
    assert len(support) == 11
    # the wall: a source on s = 0 reaches s = Ls-1 through the mass term
    src2 = np.zeros_like(src)
    src2[0, 0, 0, 0, 0] = rng.standard_normal((4, 3))
    out2 = dwf.apply_dwf(src2, U, M5, 0.05)
    assert np.abs(out2[0, 0, 0, 0, Ls - 1]).sum() > 0
    assert len(np.argwhere(np.abs(out2).sum(axis=(-1, -2)) > 1e-14)) == 11
