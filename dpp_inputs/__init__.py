"""Seeded synthetic inputs for the four-field double porosity/permeability (DPP)
workloads.

This module produces problem *data* only: box sizes, per-cell permeabilities,
the mass-transfer coefficient, nodal boundary pressures taken from the
closed-form manufactured solutions, and random directions.  It contains none
of the discretization or solver arithmetic, so both the GPU library and the
CPU oracle can consume its arrays without sharing any of the method.

Numbering spec (both sides implement it independently):
  * nodes of an n_x x n_y (x n_z) box on [0,L]^d: id = i + (n_x+1)(j + (n_y+1)k),
    coordinates (i h_x, j h_y, k h_z), x fastest;
  * 3D cells: hexahedron h = i + n_x(j + n_y k) is split into 6 tetrahedra
    6h+s, s indexing the permutations of the axes in lexicographic order;
  * 2D cells: square h = i + n_x j is split into triangles 2h and 2h+1;
  * with Q1 elements (elem = "q1") the cells are the boxes themselves: cell h
    is hexahedron / square h.
  * the local vertices of the simplex of permutation pi at hex corner c (the
    hex's node with the smallest indices) are v_0 = c and v_k = v_(k-1) +
    e_(pi(k-1)) (a path through the box along the permuted axes);
  * DG-VMS (elem = "dg", discontinuous P1 on those simplices): every simplex
    e owns its d + 1 vertex slots, slot e(d+1) + v for local vertex v; the
    unknown vector is [u1 | p1 | u2 | p2] over slots (velocities slot-major,
    components interleaved), as over nodes for P1.

Manufactured solutions: Section "Two-dimensional study" and "Three-dimensional
study" of the paper (the 3D micro-pressure carries mu/(beta k2); the printed
k1 there is a typo, see the appendix listing which uses 1/(beta*0.1)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Problem", "node_coords", "cells_per_box", "mms_fields", "mms_problem",
    "grf_log10", "grf_problem", "CONFIGS", "make_config", "batch_configs",
    "random_directions",
]


@dataclass
class Problem:
    """One DPP instance: a box and its coefficient / boundary data (host arrays).

    k1, k2: per-cell permeabilities [n_cells]; beta: scalar or [n_cells];
    p0_1, p0_2: nodal pressures [n_nodes] (only boundary nodes are used);
    body: gamma*b per cell [n_cells, dim] or None;
    face_bc: None (every box face a pressure boundary) or int8 [2, 2*dim]:
      face_bc[i, 2a + s] = 1 makes face s (0: x_a = 0, 1: x_a = L_a) a velocity
      boundary of network i, whose normal velocity is prescribed;
    u_bc_1, u_bc_2: nodal velocities [n_nodes, dim] whose normal components are
      imposed on the velocity faces (None for a network without one);
    elem: "p1" (Kuhn simplices, P1), "q1" (box cells, Q1) or "dg" (Kuhn
    simplices, discontinuous P1 of the DG-VMS form: every simplex owns its
    d + 1 vertex slots; nodal p0 data are read at the boundary vertices).
    """
    dim: int
    n: tuple
    L: tuple
    mu: float
    k1: np.ndarray
    k2: np.ndarray
    beta: object
    p0_1: np.ndarray
    p0_2: np.ndarray
    body: object = None
    gamma: float = 1.0
    meta: dict = field(default_factory=dict)
    face_bc: object = None
    u_bc_1: object = None
    u_bc_2: object = None
    elem: str = "p1"

    @property
    def n_nodes(self):
        return int(np.prod([m + 1 for m in self.n]))

    @property
    def n_cells(self):
        return cells_per_box(self.dim, self.elem) * int(np.prod(self.n))

    @property
    def n_slots(self):
        """Unknown positions per field component: nodes, or (DG) simplex vertex slots."""
        return (self.dim + 1) * self.n_cells if self.elem == "dg" else self.n_nodes

    @property
    def n_dof(self):
        return (2 * self.dim + 2) * self.n_slots


def cells_per_box(dim: int, elem: str = "p1") -> int:
    if elem == "q1":
        return 1
    return 6 if dim == 3 else 2


def node_coords(dim, n, L=None):
    """Coordinates [n_nodes, dim] in the spec numbering (x fastest)."""
    n = tuple(int(v) for v in n)
    L = tuple(float(v) for v in (L or (1.0,) * dim))
    axes = [np.arange(n[a] + 1, dtype=np.float64) * (L[a] / n[a]) for a in range(dim)]
    grids = np.meshgrid(*axes, indexing="ij")
    # meshgrid 'ij' gives axis 0 = x slowest; transpose so x is fastest in C order
    cols = [g.transpose(tuple(range(dim))[::-1]).reshape(-1) for g in grids]
    return np.stack(cols, axis=1)


def mms_fields(dim, X, k1, k2, beta, mu):
    """Closed-form manufactured DPP solution at points X [m, dim].

    Returns (p1, p2, u1, u2); u_i = -(k_i/mu) grad p_i and the pressures satisfy
    the mass balances with eta = sqrt(beta (k1+k2)/(k1 k2)).
    """
    X = np.asarray(X, dtype=np.float64)
    eta = math.sqrt(beta * (k1 + k2) / (k1 * k2))
    x = X[:, 0]
    y = X[:, 1]
    ex = np.exp(np.pi * x)
    if dim == 2:
        harm = ex * np.sin(np.pi * y)
        ey = np.exp(eta * y)
        p1 = (mu / np.pi) * harm - (mu / (beta * k1)) * ey
        p2 = (mu / np.pi) * harm + (mu / (beta * k2)) * ey
        u1 = -k1 * np.stack([ex * np.sin(np.pi * y),
                             ex * np.cos(np.pi * y) - eta / (beta * k1) * ey], axis=1)
        u2 = -k2 * np.stack([ex * np.sin(np.pi * y),
                             ex * np.cos(np.pi * y) + eta / (beta * k2) * ey], axis=1)
        return p1, p2, u1, u2
    z = X[:, 2]
    sy, sz = np.sin(np.pi * y), np.sin(np.pi * z)
    ey, ez = np.exp(eta * y), np.exp(eta * z)
    p1 = (mu / np.pi) * ex * (sy + sz) - (mu / (beta * k1)) * (ey + ez)
    p2 = (mu / np.pi) * ex * (sy + sz) + (mu / (beta * k2)) * (ey + ez)
    u1 = -k1 * np.stack([ex * (sy + sz),
                         ex * np.cos(np.pi * y) - eta / (beta * k1) * ey,
                         ex * np.cos(np.pi * z) - eta / (beta * k1) * ez], axis=1)
    u2 = -k2 * np.stack([ex * (sy + sz),
                         ex * np.cos(np.pi * y) + eta / (beta * k2) * ey,
                         ex * np.cos(np.pi * z) + eta / (beta * k2) * ez], axis=1)
    return p1, p2, u1, u2


def mms_problem(dim, n, k1=1.0, k2=0.1, beta=1.0, mu=1.0, L=None, bc_params=None,
                flux_faces=None, elem="p1"):
    """Homogeneous manufactured-solution instance: constant k1, k2, beta.

    bc_params (k1, k2, beta, mu) overrides the parameters used for the boundary
    pressures (heterogeneous-permeability workloads keep the homogeneous MMS
    boundary data).  flux_faces: None, or [2, 2*dim] face flags (see Problem)
    whose velocity faces take the exact normal velocities.  elem: "p1", "q1" or
    "dg".
    """
    n = tuple(int(v) for v in (n if np.ndim(n) else (n,) * dim))
    L = tuple(L or (1.0,) * dim)
    nc = cells_per_box(dim, elem) * int(np.prod(n))
    X = node_coords(dim, n, L)
    bk1, bk2, bb, bmu = bc_params or (k1, k2, beta, mu)
    p1, p2, u1, u2 = mms_fields(dim, X, bk1, bk2, bb, bmu)
    prob = Problem(dim=dim, n=n, L=L, mu=float(mu),
                   k1=np.full(nc, float(k1)), k2=np.full(nc, float(k2)),
                   beta=float(beta), p0_1=p1, p0_2=p2,
                   meta=dict(mms=(bk1, bk2, bb, bmu)), elem=elem)
    if flux_faces is not None:
        fb = np.asarray(flux_faces, dtype=np.int8).reshape(2, 2 * dim)
        prob.face_bc = fb
        prob.u_bc_1 = u1 if fb[0].any() else None
        prob.u_bc_2 = u2 if fb[1].any() else None
    return prob


def grf_log10(n, dim, seed, mean, std, ell=0.1, L=None):
    """Stationary Gaussian random field on the hex/square centres of the box.

    Squared-exponential covariance exp(-r^2 / (2 ell^2)), sampled by circulant
    embedding on a periodic grid of twice the box size, cropped to the box.
    Returns mean + std * field, one value per hex (x fastest) [prod(n)].
    """
    n = tuple(int(v) for v in (n if np.ndim(n) else (n,) * dim))
    L = tuple(L or (1.0,) * dim)
    h = [L[a] / n[a] for a in range(dim)]
    shape = tuple(2 * n[a] for a in reversed(range(dim)))  # C order: z, y, x
    hh = list(reversed(h))
    # periodic distances on the embedding grid
    r2 = np.zeros(shape)
    for ax in range(dim):
        m = shape[ax]
        idx = np.arange(m)
        dist = np.minimum(idx, m - idx) * hh[ax]
        sh = [1] * dim
        sh[ax] = m
        r2 = r2 + (dist ** 2).reshape(sh)
    cov = np.exp(-r2 / (2.0 * ell * ell))
    lam = np.fft.fftn(cov).real
    lam = np.clip(lam, 0.0, None)
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.standard_normal(shape)
    fld = np.fft.ifftn(np.sqrt(lam) * np.fft.fftn(w)).real
    crop = fld[tuple(slice(0, n[a]) for a in reversed(range(dim)))]
    return mean + std * crop.reshape(-1)


def hex_to_cells(values_per_hex, dim, elem="p1"):
    """Give each cell of a hex/square (its simplices, or the box itself with
    Q1 elements) the value of its hex/square."""
    return np.repeat(np.asarray(values_per_hex, dtype=np.float64), cells_per_box(dim, elem))


def grf_problem(dim, n, seeds=(1001, 1002), means=(0.0, -2.0), std=1.0, ell=0.1,
                beta=1.0, mu=1.0, bc_params=(1.0, 1e-2, 1.0, 1.0), elem="p1"):
    """Log-normal heterogeneous permeabilities, homogeneous-MMS boundary data."""
    base = mms_problem(dim, n, k1=1.0, k2=1e-2, beta=beta, mu=mu, bc_params=bc_params, elem=elem)
    l1 = grf_log10(base.n, dim, seeds[0], means[0], std, ell)
    l2 = grf_log10(base.n, dim, seeds[1], means[1], std, ell)
    base.k1 = hex_to_cells(10.0 ** l1, dim, elem)
    base.k2 = hex_to_cells(10.0 ** l2, dim, elem)
    base.meta.update(grf=dict(seeds=seeds, means=means, std=std, ell=ell))
    return base


def batch_configs(count=64, seed=2024, nmin=32, nmax=256):
    """Uneven 2D batch: n ~ U{nmin..nmax}, beta ~ logU[0.1,10], k2/k1 ~ logU[1e-3,1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = rng.integers(nmin, nmax + 1, size=count)
    betas = 10.0 ** rng.uniform(-1.0, 1.0, size=count)
    ratios = 10.0 ** rng.uniform(-3.0, 0.0, size=count)
    return [mms_problem(2, int(ns[i]), k1=1.0, k2=float(ratios[i]), beta=float(betas[i]))
            for i in range(count)]


def random_directions(count, size, seed0=4000):
    """Unit directions d_j ~ N(0, I)/||.|| with seeds seed0 .. seed0+count-1."""
    out = []
    for j in range(count):
        rng = np.random.Generator(np.random.PCG64(seed0 + j))
        v = rng.standard_normal(size)
        out.append(v / np.linalg.norm(v))
    return out


def random_vector(size, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(size)


# Named workloads (sizes and parameters of the paper's experiments and of the
# five measured configurations).
CONFIGS = {
    "c1_2d16": dict(kind="mms", dim=2, n=16, k1=1.0, k2=0.1, beta=1.0, mu=1.0),
    "c2_3d64": dict(kind="mms", dim=3, n=64, k1=1.0, k2=1e-2, beta=1.0, mu=1.0),
    "c3_3d96_grf": dict(kind="grf", dim=3, n=96),
    "c4_batch64": dict(kind="batch", count=64, seed=2024),
    "c5_3d48_grf": dict(kind="grf", dim=3, n=48),
    # the 64^3 manufactured solution with velocity faces: network 1 prescribes
    # u.n on the x faces, network 2 on the y and z = 0 faces
    "c2f_3d64_flux": dict(kind="mms", dim=3, n=64, k1=1.0, k2=1e-2, beta=1.0, mu=1.0,
                          flux_faces=[[1, 1, 0, 0, 0, 0], [0, 0, 1, 1, 1, 0]]),
    # pure flux: velocity faces everywhere in both networks (singular K)
    "c2p_3d64_pureflux": dict(kind="mms", dim=3, n=64, k1=1.0, k2=1e-2, beta=1.0, mu=1.0,
                              flux_faces=[[1] * 6, [1] * 6]),
    # Q1 hexahedra (the HEX columns of the 3D study): the 64^3 manufactured
    # solution and the 96^3 log-normal box on box cells
    "h2_3d64_q1": dict(kind="mms", dim=3, n=64, k1=1.0, k2=1e-2, beta=1.0, mu=1.0, elem="q1"),
    "h3_3d96_grf_q1": dict(kind="grf", dim=3, n=96, elem="q1"),
    # DG-VMS (discontinuous P1 on the Kuhn simplices): the appendix DG-VMS
    # listing's data (k1 = 1, k2 = 0.1, beta = mu = 1), 3D and 2D;
    # the largest DG-VMS rows of the h-size tables: TET h = 1/20 (1,536,000
    # DOF) and TRI h = 1/160 (921,600 DOF)
    "g2_3d20_dg": dict(kind="mms", dim=3, n=20, k1=1.0, k2=0.1, beta=1.0, mu=1.0, elem="dg"),
    "g1_2d160_dg": dict(kind="mms", dim=2, n=160, k1=1.0, k2=0.1, beta=1.0, mu=1.0, elem="dg"),
}


def make_config(name, n=None):
    """Build the Problem of a named workload (optionally at a different n)."""
    c = CONFIGS[name]
    if c["kind"] == "mms":
        return mms_problem(c["dim"], n or c["n"], k1=c["k1"], k2=c["k2"],
                           beta=c["beta"], mu=c["mu"], flux_faces=c.get("flux_faces"),
                           elem=c.get("elem", "p1"))
    if c["kind"] == "grf":
        return grf_problem(c["dim"], n or c["n"], elem=c.get("elem", "p1"))
    raise ValueError("batch workloads are built with batch_configs()")
