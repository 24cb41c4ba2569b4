"""Seeded synthetic meshes and coefficients for the five benchmark workloads.

Everything here is input data.  Random draws use
``numpy.random.default_rng(SeedSequence([workload_id, stream]))`` with streams
0 = vertex jitter, 1 = materials, 2 = degrees, 3 = point sources.

Workloads (one per entry of ``CONFIGS``):
  1  2D acoustics, unit square, 8x8 squares split into 128 triangles, k=2, rho=c=1,
     one backward-Euler step dt=0.01 (small parity case).
  2  3D acoustics, unit cube, 24^3 cubes x 6 Kuhn tetrahedra = 82,944, jitter +-0.2h,
     k=3, rho=1, c ~ U[1,2], 3-stage DIRK, dt=0.01.
  3  3D elastodynamics (velocity + symmetric stress), 16^3 x 6 = 24,576 jittered tets,
     k=4, rho=1, lambda ~ U[1,3], mu ~ U[0.5,1.5].
  4  3D acoustics, 40x40x25 boxes x 5 tets = 200,000 jittered tets, k ~ U{1..5},
     c ~ U[1,2], 32 point-source right-hand sides.
  5  3D Maxwell (E, H), 32^3 x 6 = 196,608 jittered tets, k=3, eps=mu=1,
     sigma ~ U[0, 0.1].
"""
from __future__ import annotations

from dataclasses import dataclass, field
from itertools import permutations

import numpy as np

__all__ = [
    "Problem",
    "unit_square_tris",
    "kuhn_cube_tets",
    "five_tet_box",
    "jitter_vertices",
    "make_problem",
    "CONFIGS",
]


def _rng(cfg_id: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(cfg_id), int(stream)]))


def _signed_volumes(xyz: np.ndarray, ev: np.ndarray) -> np.ndarray:
    """Signed d-volume factor det[x1-x0, ..., xd-x0] of each simplex (orientation test)."""
    x0 = xyz[ev[:, 0]]
    cols = [xyz[ev[:, i]] - x0 for i in range(1, ev.shape[1])]
    return np.linalg.det(np.stack(cols, axis=-1))


def _orient_positive(xyz: np.ndarray, ev: np.ndarray) -> np.ndarray:
    """Swap the last two vertices of every negatively oriented simplex."""
    ev = ev.copy()
    neg = _signed_volumes(xyz, ev) < 0
    ev[neg, -1], ev[neg, -2] = ev[neg, -2].copy(), ev[neg, -1].copy()
    return ev


def unit_square_tris(n: int):
    """Unit square, n x n squares, each split along its (i,j)-(i+1,j+1) diagonal."""
    g = np.linspace(0.0, 1.0, n + 1)
    X, Y = np.meshgrid(g, g, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel()], axis=1)

    def vid(i, j):
        return i * (n + 1) + j

    tris = []
    for i in range(n):
        for j in range(n):
            a, b, c, d = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
            tris.append((a, b, c))
            tris.append((a, c, d))
    ev = np.asarray(tris, dtype=np.int64)
    return xyz, _orient_positive(xyz, ev)


def kuhn_cube_tets(n: int):
    """Unit cube, n^3 cubes, each split into the 6 Kuhn (Freudenthal) tetrahedra.

    Every tetrahedron of a cube is a monotone lattice path from corner (0,0,0) to (1,1,1);
    all cubes use the same split, so the mesh is conforming.
    """
    g = np.linspace(0.0, 1.0, n + 1)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    m = n + 1
    I, J, K = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    tets = []
    for perm in permutations(range(3)):
        corner = np.zeros(3, dtype=np.int64)
        path = [corner.copy()]
        for ax in perm:
            corner[ax] += 1
            path.append(corner.copy())
        ids = [(I + p[0]) * m * m + (J + p[1]) * m + (K + p[2]) for p in path]
        tets.append(np.stack(ids, axis=1))
    # element order: cube-major, then the 6 paths
    ev = np.stack(tets, axis=1).reshape(-1, 4).astype(np.int64)
    return xyz, _orient_positive(xyz, ev)


_EVEN5 = [((0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1)),
          ((1, 0, 0), (0, 0, 0), (1, 1, 0), (1, 0, 1)),
          ((0, 1, 0), (0, 0, 0), (1, 1, 0), (0, 1, 1)),
          ((0, 0, 1), (0, 0, 0), (1, 0, 1), (0, 1, 1)),
          ((1, 1, 1), (1, 1, 0), (1, 0, 1), (0, 1, 1))]
_ODD5 = [((1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 1)),
         ((0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)),
         ((1, 1, 0), (1, 0, 0), (0, 1, 0), (1, 1, 1)),
         ((1, 0, 1), (1, 0, 0), (0, 0, 1), (1, 1, 1)),
         ((0, 1, 1), (0, 1, 0), (0, 0, 1), (1, 1, 1))]


def five_tet_box(nx: int, ny: int, nz: int):
    """Unit cube cut into nx x ny x nz boxes, each split into 5 tetrahedra.

    Boxes alternate between the two 5-tet splits in a checkerboard pattern so that the
    face diagonals of neighbouring boxes coincide (conforming mesh).
    """
    gx, gy, gz = (np.linspace(0.0, 1.0, q + 1) for q in (nx, ny, nz))
    X, Y, Z = np.meshgrid(gx, gy, gz, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    I, J, K = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    par = (I + J + K) % 2
    sy, sx = nz + 1, (ny + 1) * (nz + 1)
    out = np.empty((I.size, 5, 4), dtype=np.int64)
    for split, mask in ((_EVEN5, par == 0), (_ODD5, par == 1)):
        for t, tet in enumerate(split):
            for v, (a, b, c) in enumerate(tet):
                out[mask, t, v] = (I[mask] + a) * sx + (J[mask] + b) * sy + (K[mask] + c)
    ev = out.reshape(-1, 4)
    return xyz, _orient_positive(xyz, ev)


def jitter_vertices(xyz: np.ndarray, h, frac: float, rng: np.random.Generator) -> np.ndarray:
    """Move every vertex coordinate by U[-frac*h, frac*h], except coordinates lying on the
    boundary of the unit box (0 or 1), which stay exact so that the domain is unchanged."""
    h = np.broadcast_to(np.asarray(h, dtype=np.float64), (xyz.shape[1],))
    d = rng.uniform(-1.0, 1.0, size=xyz.shape) * (frac * h)[None, :]
    on_bnd = (np.abs(xyz) < 1e-14) | (np.abs(xyz - 1.0) < 1e-14)
    d[on_bnd] = 0.0
    return xyz + d


@dataclass
class Problem:
    """A seeded workload: mesh + per-element coefficients + run parameters."""
    cfg_id: int
    name: str
    physics: str            # "acoustic" | "elastic" | "maxwell"
    dim: int
    xyz: np.ndarray         # [n_vert, dim] float64
    elem_vert: np.ndarray   # [n_elem, dim+1] int64, positively oriented
    elem_par: np.ndarray    # [n_elem, 2 or 3] float64
    degree: np.ndarray      # [n_elem] int8
    dt: float
    scheme: str             # "be" (backward Euler) | "dirk33"
    steps: int
    nrhs: int = 1
    sources: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    par_names: tuple = ()
    bface_tag: np.ndarray | None = None   # [n_elem, dim+1] int8: 1 = Neumann boundary face

    @property
    def n_elem(self) -> int:
        return int(self.elem_vert.shape[0])

    @property
    def uniform_k(self):
        k0 = int(self.degree[0])
        return k0 if np.all(self.degree == k0) else None


def make_problem(cfg_id: int, n: int | None = None, nxyz=None, k: int | None = None,
                 jitter: float | None = None) -> Problem:
    """Build workload ``cfg_id`` (1..5).  ``n``/``nxyz``/``k`` override the mesh resolution
    and degree so that tests can run the same recipe on small meshes."""
    if cfg_id == 1:
        n = 8 if n is None else n
        xyz, ev = unit_square_tris(n)
        if jitter:
            xyz = jitter_vertices(xyz, 1.0 / n, jitter, _rng(cfg_id, 0))
        ne = ev.shape[0]
        par = np.ones((ne, 2))
        kk = 2 if k is None else k
        return Problem(1, "acoustic2d", "acoustic", 2, xyz, ev, par,
                       np.full(ne, kk, np.int8), 0.01, "be", 1, par_names=("rho", "c"))
    if cfg_id in (2, 3, 5):
        n = {2: 24, 3: 16, 5: 32}[cfg_id] if n is None else n
        xyz, ev = kuhn_cube_tets(n)
        xyz = jitter_vertices(xyz, 1.0 / n, 0.2 if jitter is None else jitter, _rng(cfg_id, 0))
        ne = ev.shape[0]
        r = _rng(cfg_id, 1)
        if cfg_id == 2:
            par = np.stack([np.ones(ne), r.uniform(1.0, 2.0, ne)], axis=1)
            kk = 3 if k is None else k
            return Problem(2, "acoustic3d", "acoustic", 3, xyz, ev, par,
                           np.full(ne, kk, np.int8), 0.01, "dirk33", 10,
                           par_names=("rho", "c"))
        if cfg_id == 3:
            lam = r.uniform(1.0, 3.0, ne)
            mu = r.uniform(0.5, 1.5, ne)
            par = np.stack([np.ones(ne), lam, mu], axis=1)
            kk = 4 if k is None else k
            return Problem(3, "elastic3d", "elastic", 3, xyz, ev, par,
                           np.full(ne, kk, np.int8), 0.01, "dirk33", 5,
                           par_names=("rho", "lambda", "mu"))
        par = np.stack([np.ones(ne), np.ones(ne), r.uniform(0.0, 0.1, ne)], axis=1)
        kk = 3 if k is None else k
        return Problem(5, "maxwell3d", "maxwell", 3, xyz, ev, par,
                       np.full(ne, kk, np.int8), 0.01, "dirk33", 10,
                       par_names=("eps", "mu", "sigma"))
    if cfg_id == 4:
        nx, ny, nz = (40, 40, 25) if nxyz is None else nxyz
        xyz, ev = five_tet_box(nx, ny, nz)
        hmin = 1.0 / max(nx, ny, nz)
        xyz = jitter_vertices(xyz, hmin, 0.2 if jitter is None else jitter, _rng(4, 0))
        ne = ev.shape[0]
        par = np.stack([np.ones(ne), _rng(4, 1).uniform(1.0, 2.0, ne)], axis=1)
        deg = _rng(4, 2).integers(1, 6, ne).astype(np.int8)
        if k is not None:
            deg[:] = k
        src = _rng(4, 3).uniform(0.1, 0.9, size=(32, 3))
        return Problem(4, "acoustic3d_pvar", "acoustic", 3, xyz, ev, par, deg, 0.01, "be", 1,
                       nrhs=32, sources=src, par_names=("rho", "c"))
    raise ValueError(f"unknown workload id {cfg_id}")


CONFIGS = {
    1: dict(name="acoustic2d", elems=128),
    2: dict(name="acoustic3d", elems=82944),
    3: dict(name="elastic3d", elems=24576),
    4: dict(name="acoustic3d_pvar", elems=200000),
    5: dict(name="maxwell3d", elems=196608),
}


def tag_box_faces(problem: Problem, planes) -> np.ndarray:
    """Neumann tags [n_elem, dim+1] (local face f = the face opposite vertex f) for the boundary
    faces of the unit box lying on the given planes, e.g. [(0, 0.0), (2, 1.0)] for x = 0 and
    z = 1; every other face gets 0.  Sets problem.bface_tag and returns it."""
    ev, xyz = problem.elem_vert, problem.xyz
    nv = ev.shape[1]
    tag = np.zeros(ev.shape, dtype=np.int8)
    for f in range(nv):
        fv = xyz[np.delete(ev, f, axis=1)]          # [ne, d, dim]
        for axis, val in planes:
            on = np.all(np.abs(fv[:, :, axis] - val) < 1e-12, axis=1)
            tag[on, f] = 1
    problem.bface_tag = tag
    return tag

