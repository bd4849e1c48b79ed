"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds geometry and random numbers only: triangulated spheres and
ellipsoids shaped like the polygonal unit spheres of the paper's experiments
(Section 2, the n = 32768 sphere with piecewise-constant bases), and seeded
right-hand sides.  It contains none of the compression method's arithmetic
(no quadrature, no kernel evaluation, no clustering), so both the CPU oracle
and the HIP path may import it.

Mesh recipe (icosahedral refinement):
  * level 0 is the regular icosahedron with vertices (0, +-1, +-phi) and their
    cyclic permutations, scaled to radius r;
  * every triangle (a, b, c) of level l becomes four children at indices
    4p + k: (a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca), where ab is
    the midpoint of edge a-b projected back onto the sphere;
  * new midpoint vertices are appended in first-encounter order;
  * all triangles are oriented with outward normals ((b-a) x (c-a) . a > 0).
Level l has 20 * 4**l triangles and 10 * 4**l + 2 vertices.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Mesh", "QuadMesh", "icosphere", "ellipsoid", "quadratic", "jitter", "mean_edge_length",
    "rhs_normal", "workload",
]


@dataclass
class Mesh:
    """A flat-triangle surface mesh.

    verts: (nv, 3) float64 vertex coordinates.
    tris:  (nt, 3) int32 vertex indices, 0-based, outward orientation.
    """
    verts: np.ndarray
    tris: np.ndarray

    @property
    def nv(self) -> int:
        return int(self.verts.shape[0])

    @property
    def nt(self) -> int:
        return int(self.tris.shape[0])

    def copy(self) -> "Mesh":
        return Mesh(self.verts.copy(), self.tris.copy())


def _icosahedron():
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([
        [-1, phi, 0], [1, phi, 0], [-1, -phi, 0], [1, -phi, 0],
        [0, -1, phi], [0, 1, phi], [0, -1, -phi], [0, 1, -phi],
        [phi, 0, -1], [phi, 0, 1], [-phi, 0, -1], [-phi, 0, 1],
    ], dtype=np.float64)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    # enforce outward orientation
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    s = np.einsum("ij,ij->i", np.cross(b - a, c - a), a)
    f[s < 0] = f[s < 0][:, [0, 2, 1]]
    return v, f


def icosphere(level: int, radius: float = 1.0) -> Mesh:
    """Icosahedral sphere of the given refinement level (see module docstring)."""
    verts, tris = _icosahedron()
    verts = [tuple(p) for p in verts]
    tris = [tuple(int(i) for i in t) for t in tris]
    for _ in range(level):
        cache = {}
        new_tris = []

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            idx = cache.get(key)
            if idx is None:
                pa, pb = verts[a], verts[b]
                m = [(pa[k] + pb[k]) * 0.5 for k in range(3)]
                nrm = math.sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2])
                verts.append((m[0] / nrm, m[1] / nrm, m[2] / nrm))
                idx = len(verts) - 1
                cache[key] = idx
            return idx

        for (a, b, c) in tris:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new_tris.extend([(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)])
        tris = new_tris
    v = np.asarray(verts, dtype=np.float64) * float(radius)
    t = np.asarray(tris, dtype=np.int32)
    return Mesh(v, t)


def ellipsoid(level: int, axes=(1.0, 0.7, 0.4)) -> Mesh:
    """Icosphere of the given level with vertices scaled by the semi-axes."""
    m = icosphere(level)
    m.verts = m.verts * np.asarray(axes, dtype=np.float64)[None, :]
    return m


@dataclass
class QuadMesh:
    """Quadratic (curved) triangles on the vertices of a flat mesh.

    nodes: (nv + ne, 3) float64: the nv vertices, then one node per edge.
    tris:  (nt, 6) int32: vertices v0, v1, v2 (the flat mesh's order), then the
           nodes of the edges v0-v1, v1-v2, v2-v0.
    """
    nodes: np.ndarray
    tris: np.ndarray
    nv: int

    @property
    def nt(self) -> int:
        return int(self.tris.shape[0])

    @property
    def nn(self) -> int:
        return int(self.nodes.shape[0])


def quadratic(mesh: Mesh, surface: str = "sphere", axes=(1.0, 1.0, 1.0)) -> QuadMesh:
    """Edge nodes for curved triangles: the midpoint of every edge, moved onto
    the surface the mesh approximates -- "sphere" (radial projection onto the
    sphere of the vertices' radius), "ellipsoid" (the semi-axes `axes`: the
    midpoint mapped to the unit sphere, projected, mapped back) or "flat" (kept
    on the straight edge).  Edges are numbered in order of first appearance
    in (triangle, edge) order."""
    t = mesh.tris.astype(np.int64)
    e = np.stack([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]], axis=1).reshape(-1, 2)
    key = np.sort(e, axis=1)
    _, first, inv = np.unique(key[:, 0] * (mesh.nv + 1) + key[:, 1], return_index=True, return_inverse=True)
    order = np.argsort(first, kind="stable")            # renumber by first appearance
    rank = np.empty_like(order)
    rank[order] = np.arange(order.size)
    eid = rank[inv.reshape(-1)]
    ends = key[first[order]]
    mid = 0.5 * (mesh.verts[ends[:, 0]] + mesh.verts[ends[:, 1]])
    if surface == "sphere":
        r = np.linalg.norm(mesh.verts[ends[:, 0]], axis=1)
        mid = mid / np.linalg.norm(mid, axis=1, keepdims=True) * r[:, None]
    elif surface == "ellipsoid":
        a = np.asarray(axes, dtype=np.float64)[None, :]
        u = mid / a
        mid = u / np.linalg.norm(u, axis=1, keepdims=True) * a
    elif surface != "flat":
        raise ValueError("surface must be sphere, ellipsoid or flat")
    nodes = np.concatenate([mesh.verts, mid])
    tri6 = np.concatenate([mesh.tris.astype(np.int64), mesh.nv + eid.reshape(-1, 3)], axis=1).astype(np.int32)
    return QuadMesh(nodes, tri6, mesh.nv)


def mean_edge_length(mesh: Mesh) -> float:
    t = mesh.tris.astype(np.int64)
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    e = np.unique(np.sort(e, axis=1), axis=0)
    d = mesh.verts[e[:, 0]] - mesh.verts[e[:, 1]]
    return float(np.mean(np.linalg.norm(d, axis=1)))


def jitter(mesh: Mesh, sigma: float, seed: int) -> Mesh:
    """Copy of the mesh with every vertex moved by N(0, sigma^2) per coordinate."""
    rng = np.random.default_rng(seed)
    out = mesh.copy()
    out.verts = out.verts + rng.normal(0.0, sigma, size=out.verts.shape)
    return out


def rhs_normal(n: int, nrhs: int = 1, seed: int = 0) -> np.ndarray:
    """Seeded N(0,1) vectors, shape (n,) for one right-hand side else (n, nrhs)."""
    rng = np.random.default_rng(seed)
    if nrhs == 1:
        return rng.standard_normal(n)
    return np.ascontiguousarray(rng.standard_normal((nrhs, n)).T)


def workload(name: str):
    """Named synthetic workloads: returns (mesh, parameters dict).

    sphere_l3  : unit sphere, 1280 triangles, leaf 32, eta 2, Green order 3, eps 1e-6
    sphere_l5  : unit sphere, 20480 triangles, leaf 64, eta 2, eps 1e-5, 16 RHS;
                 Green order 4 (at order 3 the Green quadrature, not eps, limits
                 the error of single admissible blocks)
    sphere_l7  : unit sphere, 327680 triangles, leaf 64, eta 2 (mixed precision solve)
    ellip_l6   : ellipsoid (1, 0.7, 0.4), 81920 triangles, jitter N(0, (1e-3 h)^2), seed 1
    sphere_l8  : unit sphere, 1310720 triangles, leaf 64, eta 2; Green order 5,
                 omega margin 1.5 diam / eta, eps 1e-5, coupling entries with the
                 order-2 regular rule, symmetric triangle rules for disjoint pairs
                 (6 points regular, 3 coupling) -- the cheapest setting measured at
                 <= 1e-4 relative error of the product on this mesh
    """
    if name == "sphere_l3":
        return icosphere(3), dict(leaf=32, eta=2.0, green_m=3, eps=1e-6)
    if name == "sphere_l5":
        return icosphere(5), dict(leaf=64, eta=2.0, green_m=4, eps=1e-5)
    if name == "sphere_l7":
        return icosphere(7), dict(leaf=64, eta=2.0, green_m=3, eps=1e-4)
    if name == "ellip_l6":
        m = ellipsoid(6)
        h = mean_edge_length(m)
        return jitter(m, 1e-3 * h, seed=1), dict(leaf=64, eta=2.0, green_m=3, eps=1e-5)
    if name == "sphere_l8":
        return icosphere(8), dict(leaf=64, eta=2.0, green_m=5, eps=1e-5, omega_scale=1.5, q_c=2, sym_rules=1)
    raise KeyError(name)
