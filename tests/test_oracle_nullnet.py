"""Pins of the oracle's proposal network (CPU only): finite differences of the
hand-derived backward, gauge covariance of the output, and the lift's wall profile
(the p = 0 free-field null vector of each chirality, paper Sec. 2 last paragraph)."""
import numpy as np
import pytest

from inputs import gaussian_fermion, prepare_gauge, random_gauge_transform, random_starts
from oracle import dwf
from oracle import nullnet as nn
from oracle import transfer as ot

M5 = 1.8


def _weights(rng, sizes, scale=0.3):
    return [scale * rng.standard_normal((9, o, i)) / np.sqrt(9 * i) for i, o in zip(sizes[:-1], sizes[1:])]


def _noise(rng, C, L):
    shp = (C,) + tuple(L[::-1]) + (3,)
    return rng.standard_normal(shp) + 1j * rng.standard_normal(shp)


def test_gauge_covariance():
    L = (4, 4, 2, 2)
    rng = np.random.default_rng(1)
    U = prepare_gauge(L, 0.5, 3)
    Ws = _weights(rng, [3, 5, 5, 8])
    eta = _noise(rng, 3, L)
    Om = random_gauge_transform(L, 4)
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[..., mu, :, :] = Om @ U[..., mu, :, :] @ np.conj(np.swapaxes(np.roll(Om, -1, axis=3 - mu), -1, -2))
    rot = lambda f: np.einsum("...ab,c...b->c...a", Om, f)
    out1, _ = nn.forward(rot(eta), Ug, Ws)
    out2, _ = nn.forward(eta, U, Ws)
    assert np.abs(out1 - rot(out2)).max() < 1e-12 * np.abs(out2).max()


def test_backward_matches_finite_differences():
    L = (2, 2, 2, 4)
    rng = np.random.default_rng(2)
    U = prepare_gauge(L, 0.5, 5)
    Ws = _weights(rng, [2, 4, 4, 4])
    eta = _noise(rng, 2, L)
    G = _noise(rng, 4, L)
    f = lambda Ws_, eta_: np.real(np.vdot(G, nn.forward(eta_, U, Ws_)[0]))
    out, cache = nn.forward(eta, U, Ws)
    dWs, deta = nn.backward(G, U, Ws, cache)
    h = 1e-6
    for l in range(3):
        for idx in [(0, 0, 0), (3, 1, 1), (8, 2, 1)]:
            Wp = [w.copy() for w in Ws]; Wm = [w.copy() for w in Ws]
            Wp[l][idx] += h; Wm[l][idx] -= h
            fd = (f(Wp, eta) - f(Wm, eta)) / (2 * h)
            assert abs(fd - dWs[l][idx]) < 1e-6 * max(1.0, abs(fd))
    for idx in [(0, 0, 0, 0, 0, 0), (1, 3, 0, 1, 1, 2)]:
        for unit in (1.0, 1j):
            ep = eta.copy(); em = eta.copy()
            ep[idx] += h * unit; em[idx] -= h * unit
            fd = (f(Ws, ep) - f(Ws, em)) / (2 * h)
            an = np.real(np.conj(deta[idx]) * unit)
            assert abs(fd - an) < 1e-6 * max(1.0, abs(fd))


def test_loss_gradient_matches_finite_differences():
    L, Ls, block, nh = (2, 2, 2, 4), 4, (2, 2, 2, 2), 3
    rng = np.random.default_rng(3)
    Vh = ot.build_basis(random_starts(L, Ls, 6, 7), block)
    f = rng.standard_normal((nh,) + tuple(L[::-1]) + (4, 3)) + 1j * rng.standard_normal((nh,) + tuple(L[::-1]) + (4, 3))
    Lval, g = nn.loss_and_grad(f, Vh, block, Ls, M5, lam=0.7)
    h = 1e-6
    for idx in [(0, 0, 0, 0, 0, 0, 0), (2, 1, 1, 0, 1, 3, 2), (1, 3, 0, 1, 0, 2, 1)]:
        for unit in (1.0, 1j):
            fp = f.copy(); fm = f.copy()
            fp[idx] += h * unit; fm[idx] -= h * unit
            fd = (nn.loss_and_grad(fp, Vh, block, Ls, M5, 0.7)[0] - nn.loss_and_grad(fm, Vh, block, Ls, M5, 0.7)[0]) / (2 * h)
            assert abs(fd - np.real(np.conj(g[idx]) * unit)) < 1e-6 * max(1.0, abs(fd))
    # a proposal inside the target space costs nothing in the first term
    assert Lval >= 0


def test_lift_is_the_free_null_profile():
    """At p = 0 in the free field, the lifted profile is annihilated by D up to the wall terms m_f and (1-M5)^Ls."""
    L, Ls = (2, 2, 2, 2), 16
    U = np.zeros(tuple(L[::-1]) + (4, 3, 3), complex); U[...] = np.eye(3)
    f = np.zeros((1,) + tuple(L[::-1]) + (4, 3), complex)
    f[..., :, 0] = 1.0        # constant in x: p = 0
    v = nn.lift(f, Ls, M5)[0]
    Dv = dwf.apply_dwf(v, U, M5, 0.0)
    # only the wall sites carry a residual, of size |1-M5|^Ls relative to the profile maximum
    interior = np.abs(Dv[..., 1:Ls - 1, :, :]).max()
    assert interior < 1e-12
    assert np.abs(Dv).max() <= abs(1 - M5) ** (Ls - 1) * 1.0001


def test_lift_adjoint():
    rng = np.random.default_rng(5)
    f = rng.standard_normal((2, 2, 2, 2, 2, 4, 3)) + 0j
    g = rng.standard_normal((2, 2, 2, 2, 2, 6, 4, 3)) + 1j * rng.standard_normal((2, 2, 2, 2, 2, 6, 4, 3))
    lhs = np.vdot(g, nn.lift(f, 6, M5))
    rhs = np.vdot(nn.lift_adjoint(g, M5), f)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
