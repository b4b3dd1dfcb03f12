"""Gauge-covariant proposal network for near-null vectors.  TEST INFRASTRUCTURE ONLY.

Not in the paper.  The paper finds near-null vectors by running a Krylov
solver on A x = 0 (Sec. 2, adaptive paragraph) and notes that every low mode
of the domain-wall operator has the same fifth-dimension structure, bound to
one wall or the other by chirality (Sec. 2, last paragraph).  This network
proposes the 4D part of such vectors from the gauge field; the fifth
dimension is the free-field wall profile.  FP64 forward and hand-derived
backward; the GPU implements the same steps.

Fields are lists/arrays of 4D colour vectors, shape (C, T, Z, Y, X, 3).

Layer:   out_o(x) = sum_{d=0..8} sum_i W[d, o, i] (T_d in_i)(x),  W real,
         T_0 = 1,  T_{1+2mu} f(x) = U_mu(x) f(x+mu),  T_{2+2mu} f(x) = U_mu(x-mu)^+ f(x-mu).
         T_d commutes with gauge transformations, so the layer is covariant.
Gate:    g(f) = f * a / (1 + a),  a = |f(x)|^2 (colour norm; invariant).
Net:     four layers, the gate after each of the first three.
Output:  channel o = 4 k + alpha is spin alpha of proposal k (a 4D spinor f_k).
Lift:    v_k(x, s) = P_+ f_k(x) w^(Ls-1-s) + P_- f_k(x) w^s,  w = 1 - M5
         (the p = 0 free-field null profile: P_+ bound to s = Ls-1, P_- to s = 0).
Loss:    L = mean_k |(1 - Pi) v_k|^2 / |v_k|^2
           + lam * mean_{j<k} |<f_j, f_k>|^2 / (|f_j|^2 |f_k|^2)
         with Pi the block projector onto a target coarse space (P R of a
         basis from the adaptive setup); the first term asks every proposal to
         lie in that space, the second keeps the proposals from collapsing
         onto one direction.
"""

from __future__ import annotations

import numpy as np

from . import dwf as _dwf
from . import transfer as _tr


def _roll(f: np.ndarray, mu: int, sign: int) -> np.ndarray:
    """g(x) = f(x + sign mu) for fields (..., T, Z, Y, X, 3)."""
    axis = f.ndim - 2 - mu   # X is axis -2, Y -3, Z -4, T -5
    return np.roll(f, -sign, axis=axis)


def _cmul(Umu: np.ndarray, f: np.ndarray) -> np.ndarray:
    """U(x) f(x) for U (T,Z,Y,X,3,3), f (C,T,Z,Y,X,3)."""
    return np.einsum("...ab,c...b->c...a", Umu, f)


def _cmulh(Umu: np.ndarray, f: np.ndarray) -> np.ndarray:
    """U(x)^+ f(x)."""
    return np.einsum("...ba,c...b->c...a", np.conj(Umu), f)


def transports(f: np.ndarray, U: np.ndarray) -> list:
    """[T_d f for d = 0..8] with the ordering self, +x, -x, +y, -y, ..."""
    out = [f]
    for mu in range(4):
        Umu = U[..., mu, :, :]
        out.append(_cmul(Umu, _roll(f, mu, +1)))            # U_mu(x) f(x+mu)
        out.append(_roll(_cmulh(Umu, f), mu, -1))           # U_mu(x-mu)^+ f(x-mu)
    return out


def opposite(d: int) -> int:
    return 0 if d == 0 else ((d - 1) ^ 1) + 1


def layer(f: np.ndarray, U: np.ndarray, W: np.ndarray):
    X = transports(f, U)
    out = sum(np.einsum("oi,i...->o...", W[d], X[d]) for d in range(9))
    return out, X


def gate(f: np.ndarray):
    a = np.sum(np.abs(f) ** 2, axis=-1, keepdims=True)
    return f * a / (1 + a)


def gate_backward(f: np.ndarray, G: np.ndarray) -> np.ndarray:
    """Gradient of Re<G, gate(f)> with respect to f (real inner product convention)."""
    a = np.sum(np.abs(f) ** 2, axis=-1, keepdims=True)
    re = np.sum(np.real(np.conj(G) * f), axis=-1, keepdims=True)
    return G * a / (1 + a) + 2 * re / (1 + a) ** 2 * f


def forward(eta: np.ndarray, U: np.ndarray, Ws: list):
    """Returns (output, cache) for input channels eta (C0, T,Z,Y,X, 3)."""
    cache = []
    h = eta
    for l, W in enumerate(Ws):
        pre, X = layer(h, U, W)
        cache.append((h, X, pre))
        h = gate(pre) if l < len(Ws) - 1 else pre
    return h, cache


def backward(G: np.ndarray, U: np.ndarray, Ws: list, cache: list):
    """Gradients of L with dL = Re<G, d out>: returns (dWs, d eta)."""
    dWs = [None] * len(Ws)
    g = G
    for l in range(len(Ws) - 1, -1, -1):
        h, X, pre = cache[l]
        if l < len(Ws) - 1:
            g = gate_backward(pre, g)
        W = Ws[l]
        gm = np.conj(g).reshape(g.shape[0], -1)
        dWs[l] = np.stack([np.real(gm @ X[d].reshape(X[d].shape[0], -1).T) for d in range(9)])
        gin = np.zeros_like(h)
        for d in range(9):
            gX = np.einsum("oi,o...->i...", W[d], g)
            gin += transports_one(gX, U, opposite(d))
        g = gin
    return dWs, g


def transports_one(f: np.ndarray, U: np.ndarray, d: int) -> np.ndarray:
    """T_d f alone (T_d^+ = T_opposite(d))."""
    if d == 0:
        return f
    mu = (d - 1) // 2
    Umu = U[..., mu, :, :]
    if d % 2 == 1:
        return _cmul(Umu, _roll(f, mu, +1))
    return _roll(_cmulh(Umu, f), mu, -1)


def to_spinors(out: np.ndarray, nh: int) -> np.ndarray:
    """Channels 4k + alpha -> spinors f_k, shape (nh, T,Z,Y,X, 4, 3)."""
    C = out.shape[0]
    assert C == 4 * nh
    o = out.reshape((nh, 4) + out.shape[1:])          # (nh, 4, T,Z,Y,X, 3)
    return np.moveaxis(o, 1, -2)                      # (nh, T,Z,Y,X, 4, 3)


def from_spinors(f: np.ndarray) -> np.ndarray:
    nh = f.shape[0]
    o = np.moveaxis(f, -2, 1)
    return o.reshape((4 * nh,) + o.shape[2:])


def wall_profile(Ls: int, M5: float):
    w = 1.0 - M5
    s = np.arange(Ls)
    return w ** (Ls - 1 - s), w ** s        # (for P_+, for P_-)


def lift(f: np.ndarray, Ls: int, M5: float) -> np.ndarray:
    """(nh, T,Z,Y,X, 4, 3) -> (nh, T,Z,Y,X, Ls, 4, 3)."""
    wp, wm = wall_profile(Ls, M5)
    v = np.zeros(f.shape[:5] + (Ls, 4, 3), dtype=np.complex128)
    v[..., 0:2, :] = f[..., None, 0:2, :] * wp[:, None, None]
    v[..., 2:4, :] = f[..., None, 2:4, :] * wm[:, None, None]
    return v


def lift_adjoint(g: np.ndarray, M5: float) -> np.ndarray:
    Ls = g.shape[5]
    wp, wm = wall_profile(Ls, M5)
    f = np.zeros(g.shape[:5] + (4, 3), dtype=np.complex128)
    f[..., 0:2, :] = np.einsum("...sac,s->...ac", g[..., 0:2, :], wp)
    f[..., 2:4, :] = np.einsum("...sac,s->...ac", g[..., 2:4, :], wm)
    return f


def loss_and_grad(f: np.ndarray, Vhat: np.ndarray, block, Ls: int, M5: float, lam: float = 1.0):
    """Loss of the spinor proposals f (nh, ...) and its gradient dL/df (dL = Re<g, df>)."""
    nh = f.shape[0]
    v = lift(f, Ls, M5)
    L = 0.0
    gv = np.zeros_like(v)
    for k in range(nh):
        pv = _tr.prolong(_tr.restrict(v[k], Vhat, block), Vhat, block)
        N = np.vdot(v[k], v[k]).real
        Q = np.vdot(pv, pv).real
        L += (1.0 - Q / N) / nh
        gv[k] = -(2.0 / N) * (pv - (Q / N) * v[k]) / nh
    gf = np.stack([lift_adjoint(gv[k:k + 1], M5)[0] for k in range(nh)])
    npair = nh * (nh - 1) / 2
    Nf = np.array([np.vdot(f[k], f[k]).real for k in range(nh)])
    for j in range(nh):
        for k in range(j + 1, nh):
            c = np.vdot(f[j], f[k])
            a2 = abs(c) ** 2
            L += lam * a2 / (Nf[j] * Nf[k]) / npair
            sc = lam * 2.0 / (Nf[j] * Nf[k]) / npair
            gf[j] += sc * (np.conj(c) * f[k] - (a2 / Nf[j]) * f[j])
            gf[k] += sc * (c * f[j] - (a2 / Nf[k]) * f[k])
    return L, gf


def propose(eta, U, Ws, nh, Ls, M5):
    out, _ = forward(eta, U, Ws)
    return lift(to_spinors(out, nh), Ls, M5)
