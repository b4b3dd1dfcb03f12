"""Block near-null basis, restrictor and prolongator.  TEST INFRASTRUCTURE ONLY.

Paper, Sec. 1 (definition of R and P): R maps fine vectors to coarse vectors,
P maps back, and R P = 1 on the coarse space.  Sec. 2 (choice of subspace):
the near-null vectors are cut into blocks, one block per coarse site, and the
coarse space is the span of all those pieces.  Sec. 2 (domain-wall paragraph):
every block covers the entire fifth dimension, so the coarse lattice is 4D.

Readings (the paper is silent on these):

* chirality split: each vector v_k contributes two columns per block,
  P_+ v_k and P_- v_k (spins {0,1} and {2,3}), so a coarse site carries 2*Nv
  degrees of freedom, independent of Ls;
* orthonormalisation: modified Gram-Schmidt applied twice per column, columns
  in ascending k, positive real diagonal -- the unique thin QR factor Q of
  every full-rank block panel;
* P c = sum over (block, chirality, k) of Q-columns times c, and R = P^+, so
  R P = 1 holds because every panel is orthonormal.

Layouts: fine fields (Lt,Lz,Ly,Lx,Ls,4,3); the basis ``Vhat`` has shape
(Nv, Lt,Lz,Ly,Lx,Ls,4,3) with both chirality columns of vector k stored in
field k (they live on disjoint spin components); coarse vectors have shape
(Tc, Zc, Yc, Xc, 2, Nv) with chirality 0 = P_+.
"""

from __future__ import annotations

import numpy as np

RANK_TOL = 1e-12


class RankDeficientError(ValueError):
    """A block panel lost (numerically) all of a column during orthonormalisation."""


def block_split(f: np.ndarray, block) -> np.ndarray:
    """View (..., T,Z,Y,X,Ls,4,3) as (..., Tc,Zc,Yc,Xc, bt,bz,by,bx, Ls,4,3)."""
    bx, by, bz, bt = block
    lead = f.shape[:-7]
    T, Zd, Y, X, Ls, ns, nc = f.shape[-7:]
    if T % bt or Zd % bz or Y % by or X % bx:
        raise ValueError("block does not divide the lattice")
    n = len(lead)
    g = f.reshape(lead + (T // bt, bt, Zd // bz, bz, Y // by, by, X // bx, bx, Ls, ns, nc))
    perm = list(range(n)) + [n + i for i in (0, 2, 4, 6, 1, 3, 5, 7, 8, 9, 10)]
    return g.transpose(perm)


def block_merge(g: np.ndarray) -> np.ndarray:
    """Inverse of :func:`block_split`."""
    n = g.ndim - 11
    lead = g.shape[:n]
    Tc, Zc, Yc, Xc, bt, bz, by, bx, Ls, ns, nc = g.shape[n:]
    perm = list(range(n)) + [n + i for i in (0, 4, 1, 5, 2, 6, 3, 7, 8, 9, 10)]
    return g.transpose(perm).reshape(lead + (Tc * bt, Zc * bz, Yc * by, Xc * bx, Ls, ns, nc))


def coarse_dims(L, block):
    return tuple(L[m] // block[m] for m in range(4))


def _chiral_panels(V: np.ndarray, block) -> np.ndarray:
    """Panels A[chi, Tc,Zc,Yc,Xc, rows, k]: the chirality-chi part of v_k on each block."""
    Nv = V.shape[0]
    g = block_split(V, block)  # (Nv, Tc,Zc,Yc,Xc, bt,bz,by,bx, Ls,4,3)
    panels = []
    for chi in range(2):
        part = g[..., 2 * chi:2 * chi + 2, :]          # spins of this chirality
        Tc, Zc, Yc, Xc = part.shape[1:5]
        flat = part.reshape(Nv, Tc, Zc, Yc, Xc, -1)     # rows = (bt,bz,by,bx,Ls,2,3)
        panels.append(np.moveaxis(flat, 0, -1))         # (Tc,Zc,Yc,Xc, rows, Nv)
    return np.stack(panels)


def orthonormalise_panels(A: np.ndarray) -> np.ndarray:
    """Modified Gram-Schmidt, two passes per column, ascending k, on every panel.

    ``A`` has shape (..., rows, Nv); returns Q of the same shape with Q^+ Q = 1
    per panel and positive real R diagonal.  Raises RankDeficientError when a
    column keeps less than RANK_TOL of its norm.
    """
    Q = np.array(A, dtype=np.complex128, copy=True)
    Nv = Q.shape[-1]
    for k in range(Nv):
        q = Q[..., k]
        n0 = np.linalg.norm(q, axis=-1)
        for _ in range(2):
            for j in range(k):
                qj = Q[..., j]
                coef = np.sum(np.conj(qj) * q, axis=-1)
                q = q - coef[..., None] * qj
        nrm = np.linalg.norm(q, axis=-1)
        if np.any(nrm <= RANK_TOL * n0) or np.any(n0 == 0):
            raise RankDeficientError(f"column {k} is numerically dependent on its predecessors")
        Q[..., k] = q / nrm[..., None]
    return Q


def build_basis(V: np.ndarray, block) -> np.ndarray:
    """Chirality-split, block-orthonormal basis Vhat from near-null vectors V (Nv, field)."""
    Nv = V.shape[0]
    Q = orthonormalise_panels(_chiral_panels(V, block))   # (2, Tc,Zc,Yc,Xc, rows, Nv)
    g = np.zeros_like(block_split(V, block))
    for chi in range(2):
        q = np.moveaxis(Q[chi], -1, 0)                     # (Nv, Tc,Zc,Yc,Xc, rows)
        shp = g[..., 2 * chi:2 * chi + 2, :].shape
        g[..., 2 * chi:2 * chi + 2, :] = q.reshape(shp)
    return np.ascontiguousarray(block_merge(g))


def restrict(x: np.ndarray, Vhat: np.ndarray, block) -> np.ndarray:
    """c[B, chi, k] = sum over block B, all s, spins of chirality chi, colour of conj(Vhat_k) x."""
    gv = block_split(Vhat, block)       # (Nv, Tc,Zc,Yc,Xc, b.., Ls,4,3)
    gx = block_split(x, block)          # (Tc,Zc,Yc,Xc, b.., Ls,4,3)
    Nv = Vhat.shape[0]
    Tc, Zc, Yc, Xc = gx.shape[:4]
    out = np.empty((Tc, Zc, Yc, Xc, 2, Nv), dtype=np.complex128)
    for chi in range(2):
        sl = slice(2 * chi, 2 * chi + 2)
        prod = np.conj(gv[..., sl, :]) * gx[None, ..., sl, :]
        out[..., chi, :] = np.moveaxis(prod.reshape(Nv, Tc, Zc, Yc, Xc, -1).sum(-1), 0, -1)
    return out


def prolong(c: np.ndarray, Vhat: np.ndarray, block) -> np.ndarray:
    """x = sum over (chi, k) of Vhat_k restricted to chirality chi, times c[B, chi, k]."""
    gv = block_split(Vhat, block)
    g = np.zeros(gv.shape[1:], dtype=np.complex128)
    for chi in range(2):
        sl = slice(2 * chi, 2 * chi + 2)
        coef = np.moveaxis(c[..., chi, :], -1, 0)          # (Nv, Tc,Zc,Yc,Xc)
        g[..., sl, :] = np.einsum("kTZYX,kTZYXabcdsij->TZYXabcdsij", coef, gv[..., sl, :])
    return block_merge(g)
