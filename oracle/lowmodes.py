"""Low modes of D^+D and their coverage by the coarse space.  TEST INFRASTRUCTURE ONLY.

Paper, Sec. 2 (the choice of coarse space, Fig. 1 right): with a coarse
space spanned by a few low modes cut into blocks, those modes are in it
exactly and most of the next ones nearly so.  The oracle computes, on
lattices small enough for a dense matrix, N = D^+ D column by column, its
eigenpairs with a dense Hermitian eigensolver, and the fraction
|P R e|^2 / |e|^2 of a field e inside the span of a block basis.
"""

from __future__ import annotations

import numpy as np

from . import transfer as _tr


def dense_normal(A, shape) -> np.ndarray:
    """N = D^+ D as a dense matrix, column j = N e_j (fields of the given shape, flattened)."""
    n = int(np.prod(shape))
    cols = []
    for j in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[j] = 1.0
        cols.append(A.dag(A(e.reshape(shape))).ravel())
    return np.array(cols).T


def lowest_modes(A, shape, nev: int):
    """The nev smallest eigenvalues of D^+ D (ascending) and unit eigenvectors (nev, *shape)."""
    w, v = np.linalg.eigh(dense_normal(A, shape))
    return w[:nev], np.array([v[:, i].reshape(shape) for i in range(nev)])


def coverage(E: np.ndarray, Vhat: np.ndarray, block) -> np.ndarray:
    """|P R e|^2 / |e|^2 for each field e of E (the coarse space of the basis Vhat)."""
    out = []
    for e in E:
        pe = _tr.prolong(_tr.restrict(e, Vhat, block), Vhat, block)
        out.append(float(np.vdot(pe, pe).real / np.vdot(e, e).real))
    return np.array(out)
