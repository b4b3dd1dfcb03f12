"""Seeded inputs of the two-dimensional U(1) test problem.

The paper's first test (Sec. 3, Fig. 2) runs on a quenched U(1) gauge field in
two dimensions, 20^2 sites with Ls = 8.  That ensemble is not available; a
stand-in of the same kind is generated here: the Wilson plaquette action
S = -beta sum_P cos(theta_P) sampled by Metropolis updates of the link angles.

Canonical layout of the 2D problem (C order, complex128):

* 2D site index ``x2 = y*Lx + x``; direction mu = 0, 1 is x, y.
* fermion field: shape ``(Ly, Lx, Ls, 2)`` = (site, s, spin).
* gauge field: shape ``(Ly, Lx, 2)`` = U_mu(x) = exp(i theta_mu(x)).

Metropolis recipe: start from angles uniform in [-pi, pi); one sweep visits
the links in four sets (x-links on even rows, x-links on odd rows, y-links on
even columns, y-links on odd columns).  Links of one set share no plaquette,
so each set is updated at once: every link of the set proposes
theta + u, u uniform in [-step, step], and accepts with probability
min(1, exp(-dS)), dS the change of its two plaquettes.  Per set the draws
are the proposals for the whole (Ly, Lx) array of that direction, then the
acceptance uniforms for the same array, both from
``numpy.random.Generator(PCG64(seed))``; entries outside the set are unused.
Both extents must be even (with sweeps = 0, the random start, any extents).
"""

from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np


def fermion2d_shape(L: Sequence[int], Ls: int) -> Tuple[int, ...]:
    Lx, Ly = L
    return (Ly, Lx, Ls, 2)


def plaquette_angles(theta: np.ndarray) -> np.ndarray:
    """theta_P(x) = theta_x(x) + theta_y(x + x^) - theta_x(x + y^) - theta_y(x),
    periodic; ``theta`` has shape (Ly, Lx, 2)."""
    tx, ty = theta[..., 0], theta[..., 1]
    return tx + np.roll(ty, -1, axis=1) - np.roll(tx, -1, axis=0) - ty


def quenched_u1_2d(L: Sequence[int], beta: float, seed: int, sweeps: int = 500,
                   step: float = 1.5) -> np.ndarray:
    """A U(1) gauge field after ``sweeps`` Metropolis sweeps of the Wilson action."""
    Lx, Ly = L
    if sweeps > 0 and (Lx % 2 or Ly % 2):
        raise ValueError("both extents must be even")
    rng = np.random.Generator(np.random.PCG64(seed))
    theta = rng.uniform(-np.pi, np.pi, size=(Ly, Lx, 2))
    yy, xx = np.meshgrid(np.arange(Ly), np.arange(Lx), indexing="ij")
    for _ in range(sweeps):
        for mu in (0, 1):
            for parity in (0, 1):
                mask = ((yy if mu == 0 else xx) % 2) == parity
                prop = rng.uniform(-step, step, size=(Ly, Lx))
                acc = rng.uniform(0.0, 1.0, size=(Ly, Lx))
                new = theta.copy()
                new[..., mu] = np.where(mask, theta[..., mu] + prop, theta[..., mu])
                c_old = np.cos(plaquette_angles(theta))
                c_new = np.cos(plaquette_angles(new))
                d = c_new - c_old
                # the two plaquettes of a link: x-link at (x, y) lies in P(x, y)
                # and P(x, y - 1); y-link at (x, y) in P(x, y) and P(x - 1, y)
                other = np.roll(d, 1, axis=0) if mu == 0 else np.roll(d, 1, axis=1)
                dS = -beta * (d + other)
                take = mask & (acc < np.exp(-np.maximum(dS, -50.0)))
                theta[..., mu] = np.where(take, new[..., mu], theta[..., mu])
    theta = np.mod(theta + np.pi, 2.0 * np.pi) - np.pi
    return np.exp(1j * theta)


def gaussian_fermion2d(L: Sequence[int], Ls: int, seed: int, n: int | None = None) -> np.ndarray:
    """Gaussian complex 2D field(s): Re, Im i.i.d. N(0,1) in canonical order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shp = fermion2d_shape(L, Ls) if n is None else (n,) + fermion2d_shape(L, Ls)
    return rng.standard_normal(shp) + 1j * rng.standard_normal(shp)


def point_sources2d(L: Sequence[int], Ls: int, site=(0, 0)) -> np.ndarray:
    """The two spin point sources of a 2D quark field, lifted to the walls:
    spin 0 (positive chirality) on s = Ls-1, spin 1 on s = 0.  Shape
    (2, Ly, Lx, Ls, 2)."""
    x, y = site
    out = np.zeros((2,) + fermion2d_shape(L, Ls), dtype=np.complex128)
    out[0, y, x, Ls - 1, 0] = 1.0
    out[1, y, x, 0, 1] = 1.0
    return out


def random_starts2d(L: Sequence[int], Ls: int, nvec: int, seed: int) -> np.ndarray:
    """Random starting vectors of the 2D setup, shape (nvec, Ly, Lx, Ls, 2)."""
    return gaussian_fermion2d(L, Ls, seed, n=nvec)


def random_u1_transform(L: Sequence[int], seed: int) -> np.ndarray:
    """One random phase per 2D site, shape (Ly, Lx)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Lx, Ly = L
    return np.exp(1j * rng.uniform(-np.pi, np.pi, size=(Ly, Lx)))
