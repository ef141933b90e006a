"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only builds inputs: closed triangle meshes (icosahedral and
octahedral spheres, ellipsoids), incidence directions and seeded random
density vectors.  It contains none of the boundary-element arithmetic, so the
oracle and the GPU path can both draw their inputs from here without sharing
any of the method.

Conventions
-----------
* Meshes are returned as ``(V, T)`` with ``V`` a float64 ``(nv, 3)`` array of
  vertex coordinates and ``T`` an int32 ``(nt, 3)`` array of vertex indices.
* Every triangle is wound counter-clockwise when seen from outside the body,
  so ``(v1 - v0) x (v2 - v0)`` points out of the body into the fluid.
"""
from __future__ import annotations

import math
from typing import Dict, Tuple

import numpy as np

__all__ = [
    "icosphere",
    "octasphere",
    "ellipsoid",
    "spheroid_rings",
    "fibonacci_directions",
    "complex_normal",
    "uneven_batch",
    "orient_outward",
    "workload",
    "WORKLOADS",
]


def orient_outward(V: np.ndarray, T: np.ndarray) -> np.ndarray:
    """Flip triangles of a star-shaped (about the origin) closed mesh so that
    their right-hand normals point away from the origin."""
    T = np.array(T, dtype=np.int32, copy=True)
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    nrm = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", nrm, (a + b + c) / 3.0) < 0
    T[flip, 1], T[flip, 2] = T[flip, 2].copy(), T[flip, 1].copy()
    return T


def _faces_from_edge_length(V: np.ndarray, edge: float) -> np.ndarray:
    """All vertex triples whose three pairwise distances equal ``edge``
    (the faces of a regular polyhedron)."""
    n = len(V)
    d = np.linalg.norm(V[:, None, :] - V[None, :, :], axis=-1)
    adj = np.abs(d - edge) < 1e-9
    faces = []
    for i in range(n):
        for j in range(i + 1, n):
            if not adj[i, j]:
                continue
            for k in range(j + 1, n):
                if adj[i, k] and adj[j, k]:
                    faces.append((i, j, k))
    return np.array(faces, dtype=np.int32)


def _subdivide(V: np.ndarray, T: np.ndarray, levels: int, radius: float):
    """Midpoint subdivision; every new vertex is pushed onto the sphere."""
    verts = [tuple(v) for v in V]
    tris = [tuple(t) for t in T]
    for _ in range(levels):
        cache: Dict[Tuple[int, int], int] = {}

        def mid(i: int, j: int) -> int:
            key = (i, j) if i < j else (j, i)
            m = cache.get(key)
            if m is None:
                p = np.add(verts[i], verts[j]) * 0.5
                p = p * (radius / np.linalg.norm(p))
                verts.append(tuple(p))
                m = len(verts) - 1
                cache[key] = m
            return m

        new = []
        for a, b, c in tris:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        tris = new
    return np.array(verts, dtype=np.float64), np.array(tris, dtype=np.int32)


def icosphere(subdiv: int, radius: float = 0.5):
    """Icosahedral sphere: 20 * 4**subdiv flat triangles, 10 * 4**subdiv + 2
    vertices, all vertices on the sphere of the given radius."""
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    base = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            base += [(0.0, s1, s2 * phi), (s1, s2 * phi, 0.0), (s2 * phi, 0.0, s1)]
    V = np.array(base, dtype=np.float64)
    T = _faces_from_edge_length(V, 2.0)
    V = V * (radius / np.linalg.norm(V[0]))
    T = orient_outward(V, T)
    V, T = _subdivide(V, T, subdiv, radius)
    return V, orient_outward(V, T)


def octasphere(subdiv: int, radius: float = 1.0):
    """Octahedral sphere: 8 * 4**subdiv flat triangles (512, 2048, 8192 for
    subdiv 3, 4, 5)."""
    V = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]],
                 dtype=np.float64)
    T = _faces_from_edge_length(V, math.sqrt(2.0))
    V = V * radius
    T = orient_outward(V, T)
    V, T = _subdivide(V, T, subdiv, radius)
    return V, orient_outward(V, T)


def ellipsoid(subdiv: int, semi_axes=(0.5, 0.5, 0.5)):
    """Ellipsoid meshed as a unit icosphere scaled along x, y, z.  Positive
    scaling keeps the outward winding."""
    V, T = icosphere(subdiv, 1.0)
    return V * np.asarray(semi_axes, dtype=np.float64)[None, :], T


def spheroid_rings(h: float, a: float = 2.5, b: float = 0.5):
    """Near-uniform mesh of the prolate spheroid x^2/a^2 + (y^2 + z^2)/b^2 = 1
    (long axis x) with edges of about h: rings of constant x spaced h apart
    in arc length along the meridian, each with about 2 pi rho / h points
    (alternate rings offset by half a step), consecutive rings zipped into
    triangles in angular order, one vertex at each pole.  (A scaled sphere
    mesh would stretch its elements a / b times along the axis.)"""
    t = np.linspace(0.0, math.pi, 200001)
    ds = np.hypot(a * np.sin(t), b * np.cos(t))
    s = np.concatenate([[0.0], np.cumsum(0.5 * (ds[1:] + ds[:-1]) * (t[1] - t[0]))])
    m = max(4, int(round(s[-1] / h)))
    ti = np.interp(np.linspace(0.0, s[-1], m + 1), s, t)
    verts = [np.array([[a, 0.0, 0.0]])]
    rings = []  # (first vertex, count, angles)
    nv = 1
    for i in range(1, m):
        rho, x = b * math.sin(ti[i]), a * math.cos(ti[i])
        n = max(3, int(round(2.0 * math.pi * rho / h)))
        ang = 2.0 * math.pi * (np.arange(n) + 0.5 * (i % 2)) / n
        verts.append(np.stack([np.full(n, x), rho * np.cos(ang), rho * np.sin(ang)], axis=1))
        rings.append((nv, n, ang))
        nv += n
    verts.append(np.array([[-a, 0.0, 0.0]]))
    south = nv
    V = np.concatenate(verts)
    tris = []
    f0, n0, _ = rings[0]
    j = np.arange(n0)
    tris.append(np.stack([np.zeros(n0, dtype=np.int64), f0 + j, f0 + (j + 1) % n0], axis=1))
    for (fa, na, aa), (fb, nb, ab) in zip(rings[:-1], rings[1:]):
        # walk both rings in angular order; each step advances one of them
        ev = np.concatenate([aa[1:], [aa[0] + 2.0 * math.pi], ab[1:], [ab[0] + 2.0 * math.pi]])
        typ = np.concatenate([np.zeros(na, dtype=np.int64), np.ones(nb, dtype=np.int64)])[np.argsort(ev, kind="stable")]
        ia = np.cumsum(typ == 0) - (typ == 0)
        jb = np.cumsum(typ == 1) - (typ == 1)
        A0, A1 = fa + ia % na, fa + (ia + 1) % na
        B0, B1 = fb + jb % nb, fb + (jb + 1) % nb
        tris.append(np.where((typ == 0)[:, None], np.stack([A0, A1, B0], axis=1), np.stack([A0, B1, B0], axis=1)))
    fl, nl, _ = rings[-1]
    j = np.arange(nl)
    tris.append(np.stack([np.full(nl, south), fl + (j + 1) % nl, fl + j], axis=1))
    T = np.concatenate(tris).astype(np.int32)
    return V, orient_outward(V, T)


def graded_sphere(subdiv: int, bands=((0.3, 1), (0.7, 2)), radius: float = 0.5):
    """Icosphere of `subdiv` whose triangles are refined further towards the
    +z pole: a triangle whose centroid has z > zb * radius gets `extra` more
    midpoint subdivisions for the largest such (zb, extra) in `bands`, so the
    edge length drops by 2**extra over the cap.  Triangles of one refinement
    class share their new vertices; between classes the mesh has hanging
    vertices (collocation with constant elements needs no conformity).  The
    default gives 4,952 triangles for subdiv 3 with a 4:1 edge ratio."""
    V, T = icosphere(subdiv, radius)
    cz = V[T].mean(axis=1)[:, 2] / radius
    extra = np.zeros(len(T), dtype=np.int64)
    for zb, e in bands:
        extra[cz > zb] = np.maximum(extra[cz > zb], e)
    tris = [T[extra == 0]]
    for e in sorted(set(extra.tolist()) - {0}):
        V, Te = _subdivide(V, T[extra == e], e, radius)
        tris.append(Te)
    T = np.concatenate(tris).astype(np.int32)
    return V, orient_outward(V, T)


def fibonacci_directions(n: int) -> np.ndarray:
    """n unit vectors on a Fibonacci sphere: z_j = 1 - (2j+1)/n,
    azimuth_j = j * pi * (3 - sqrt(5))."""
    j = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * j + 1.0) / n
    ph = j * math.pi * (3.0 - math.sqrt(5.0))
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([s * np.cos(ph), s * np.sin(ph), z], axis=1)


def complex_normal(n: int, nrhs: int = 1, seed: int = 0) -> np.ndarray:
    """Complex standard normal samples (E|x|^2 = 1), shape (n,) or (n, nrhs),
    from numpy's default_rng(seed)."""
    rng = np.random.default_rng(seed)
    shape = (n,) if nrhs == 1 else (n, nrhs)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2.0)


# Named synthetic workloads.  A rigid sphere of diameter D = 1 (radius 0.5)
# meshed as an icosphere, a unit plane wave along +z, Burton-Miller coupling
# i/k (fluid-side normal), compression threshold eps = 1e-4, at most 64
# elements per leaf,
# GMRES(50) to a relative residual of 1e-5.
WORKLOADS = {
    "sphere1280_kD10": dict(subdiv=3, radius=0.5, k=10.0, eps=1e-4, direction=(0.0, 0.0, 1.0)),
    # the headline configuration: every SVD truncated at the paper's eps
    # (eqs. (eq_epsg), (eq_epsk)) instead of the library's default eps / 10
    "sphere81920_kD100": dict(subdiv=6, radius=0.5, k=100.0, eps=1e-4, direction=(0.0, 0.0, 1.0),
                              plan=dict(svd_eps=1e-4)),
    "sphere5120_kD20": dict(subdiv=4, radius=0.5, k=20.0, eps=1e-4, direction=(0.0, 0.0, 1.0)),
    "sphere20480_kD50": dict(subdiv=5, radius=0.5, k=50.0, eps=1e-4, direction=(0.0, 0.0, 1.0)),
    "sphere20480_kD100": dict(subdiv=5, radius=0.5, k=100.0, eps=1e-4, direction=(0.0, 0.0, 1.0)),
}


def uneven_batch(n: int = 32, seed: int = 3, subdivs=(4, 5, 6)):
    """Seeded uneven multi-mesh batch: n meshes, the first half spheres of
    radius 0.5, the second half ellipsoids with semi-axes U[0.3, 0.7];
    subdivision uniform in `subdivs` (5,120 / 20,480 / 81,920 triangles),
    kD uniform in [20, 100] with D = 2 x the largest semi-axis.  Returns a
    list of (V, T, k, info)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        s = int(rng.choice(subdivs))
        if i < n // 2:
            axes = np.array([0.5, 0.5, 0.5])
            V, T = icosphere(s, 0.5)
        else:
            axes = rng.uniform(0.3, 0.7, size=3)
            V, T = ellipsoid(s, tuple(axes))
        kD = float(rng.uniform(20.0, 100.0))
        k = kD / (2.0 * float(axes.max()))
        out.append((V, T, k, dict(subdiv=s, semi_axes=axes.tolist(), kD=kD, n=len(T))))
    return out


def workload(name: str):
    """Return (V, T, params) for a named workload."""
    p = dict(WORKLOADS[name])
    V, T = icosphere(p["subdiv"], p["radius"])
    return V, T, p
