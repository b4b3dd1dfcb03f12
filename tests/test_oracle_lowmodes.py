"""Pins of the oracle's low modes and coverage (CPU only).

Paper Sec. 2, Fig. 1 right: the coarse space of a basis built from low modes
holds those modes exactly.  Pins: the dense eigenpairs satisfy N e = lambda e
with the operator applied directly and are orthonormal; coverage lies in
[0, 1], is 1 for fields in the span of the basis (and for every field with a
complete basis), and P R is an orthogonal projector (Pythagoras).
"""
import numpy as np

from inputs import gaussian_fermion, prepare_gauge, random_starts
from oracle import dwf
from oracle import lowmodes as olm
from oracle import transfer as ot

M5 = 1.8


def test_dense_eigenpairs_satisfy_the_eigen_equation():
    L, Ls, mf = (2, 2, 2, 4), 4, 0.05
    A = dwf.DWF(prepare_gauge(L, 0.4, 70), M5, mf)
    shape = tuple(L[::-1]) + (Ls, 4, 3)
    lam, E = olm.lowest_modes(A, shape, 6)
    assert np.all(np.diff(lam) >= 0) and lam[0] > 0
    for l, e in zip(lam, E):
        assert np.linalg.norm(A.dag(A(e)) - l * e) < 1e-12 * max(1.0, l)
    G = np.array([[np.vdot(a, b) for b in E] for a in E])
    assert np.abs(G - np.eye(6)).max() < 1e-12


def test_coverage_of_the_basis_vectors_and_a_complete_basis():
    L, Ls, block = (4, 2, 2, 2), 4, (2, 2, 2, 2)
    V = random_starts(L, Ls, 5, 71)
    Vh = ot.build_basis(V, block)
    assert np.allclose(olm.coverage(V, Vh, block), 1.0, atol=1e-13)
    x = gaussian_fermion(L, Ls, 72, n=4)
    c = olm.coverage(x, Vh, block)
    assert np.all(c >= 0) and np.all(c <= 1 + 1e-14) and np.all(c < 0.5)
    # P R is an orthogonal projector: |P R x|^2 + |(1 - P R) x|^2 = |x|^2
    for xi, ci in zip(x, c):
        pe = ot.prolong(ot.restrict(xi, Vh, block), Vh, block)
        assert abs(ci * np.vdot(xi, xi).real + np.vdot(xi - pe, xi - pe).real - np.vdot(xi, xi).real) < 1e-10
    # complete basis: 1^4 blocks, Nv = 6 Ls (every dof of a block and chirality)
    Lc, Lsc = (2, 2, 2, 2), 2
    Vc = random_starts(Lc, Lsc, 6 * Lsc, 73)
    Vhc = ot.build_basis(Vc, (1, 1, 1, 1))
    assert np.allclose(olm.coverage(gaussian_fermion(Lc, Lsc, 74, n=3), Vhc, (1, 1, 1, 1)), 1.0, atol=1e-12)


def test_basis_of_the_lowest_modes_covers_them_exactly():
    """Fig. 1's construction: the basis made of the lowest k modes holds each of
    them entirely; the next modes are held in part."""
    L, Ls, mf, block = (2, 2, 2, 4), 4, 0.05, (2, 2, 2, 2)
    A = dwf.DWF(prepare_gauge(L, 0.4, 75), M5, mf)
    shape = tuple(L[::-1]) + (Ls, 4, 3)
    lam, E = olm.lowest_modes(A, shape, 12)
    Vh = ot.build_basis(E[:4], block)
    c = olm.coverage(E, Vh, block)
    assert np.allclose(c[:4], 1.0, atol=1e-12)
    assert np.all(c[4:] < 1.0 - 1e-6)
