"""Seeded synthetic inputs: SU(3) links, APE-style smoothing, sources (CPU only)."""
import numpy as np

from inputs import gaussian_fermion, gell_mann, point_sources, prepare_gauge, random_starts


def test_gell_mann_basis():
    lam = gell_mann()
    for a in range(8):
        assert np.allclose(lam[a], lam[a].conj().T) and abs(np.trace(lam[a])) < 1e-15
        for b in range(8):
            assert abs(np.trace(lam[a] @ lam[b]) - 2.0 * (a == b)) < 1e-14


def test_links_are_su3_and_seeded():
    for ape in (0, 2):
        U = prepare_gauge((4, 4, 2, 2), 0.6, 5, ape_steps=ape)
        I = np.eye(3)
        assert np.abs(U @ np.conj(np.swapaxes(U, -1, -2)) - I).max() < 1e-13
        assert np.abs(np.linalg.det(U) - 1.0).max() < 1e-13
    assert np.array_equal(prepare_gauge((2, 2, 2, 2), 0.3, 7), prepare_gauge((2, 2, 2, 2), 0.3, 7))
    assert not np.array_equal(prepare_gauge((2, 2, 2, 2), 0.3, 7), prepare_gauge((2, 2, 2, 2), 0.3, 8))


def test_ape_smoothing_reduces_disorder():
    """Smoothing moves links towards the staple average: the mean plaquette rises."""
    def plaq(U):
        tot = 0.0
        for mu in range(4):
            for nu in range(mu + 1, 4):
                Umu, Unu = U[..., mu, :, :], U[..., nu, :, :]
                P = Umu @ np.roll(Unu, -1, axis=3 - mu) @ np.conj(np.swapaxes(np.roll(Umu, -1, axis=3 - nu), -1, -2)) \
                    @ np.conj(np.swapaxes(Unu, -1, -2))
                tot += np.trace(P, axis1=-2, axis2=-1).real.mean() / 3
        return tot / 6
    U0 = prepare_gauge((4, 4, 4, 4), 0.6, 9)
    U2 = prepare_gauge((4, 4, 4, 4), 0.6, 9, ape_steps=2)
    assert plaq(U2) > plaq(U0)


def test_sources():
    b = gaussian_fermion((2, 2, 2, 2), 4, 3)
    assert b.shape == (2, 2, 2, 2, 4, 4, 3) and b.dtype == np.complex128
    ps = point_sources((2, 2, 2, 2), 4)
    assert ps.shape[0] == 12 and np.allclose(np.abs(ps).sum(axis=tuple(range(1, 8))), 1.0)
    assert random_starts((2, 2, 2, 2), 4, 3, 1).shape == (3, 2, 2, 2, 2, 4, 4, 3)
