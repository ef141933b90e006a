"""The synthetic mesh generators: the prolate spheroid ring mesher gives a
closed, consistently wound, near-uniform surface whose area converges to the
spheroid's closed-form area."""
import math

import numpy as np

import workloads as W


def _spheroid_area(a, b):
    e = math.sqrt(1.0 - (b / a) ** 2)
    return 2.0 * math.pi * b * b * (1.0 + a / (b * e) * math.asin(e))


def test_spheroid_rings_is_a_closed_outward_uniform_surface():
    a, b = 2.5, 0.5
    for h in (0.05, 0.025):
        V, T = W.spheroid_rings(h, a, b)
        # on the surface
        assert np.allclose((V[:, 0] / a) ** 2 + (V[:, 1] ** 2 + V[:, 2] ** 2) / b**2, 1.0, atol=1e-12)
        # closed 2-manifold of genus 0: every edge in exactly two triangles,
        # once in each direction (consistent winding), Euler characteristic 2
        E = np.concatenate([T[:, [0, 1]], T[:, [1, 2]], T[:, [2, 0]]]).astype(np.int64)
        key = E[:, 0] * len(V) + E[:, 1]
        rev = E[:, 1] * len(V) + E[:, 0]
        assert len(np.unique(key)) == len(key)
        assert np.array_equal(np.sort(key), np.sort(rev))
        assert len(V) - len(key) // 2 + len(T) == 2
        # outward: right-hand normals point away from the axis side of the centroid
        p0, p1, p2 = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
        nrm = np.cross(p1 - p0, p2 - p0)
        c = (p0 + p1 + p2) / 3.0
        grad = np.stack([c[:, 0] / a**2, c[:, 1] / b**2, c[:, 2] / b**2], axis=1)
        assert np.all(np.einsum("ij,ij->i", nrm, grad) > 0)
        # near-uniform: edges within a factor 2 of h, no sliver
        el = np.linalg.norm(np.stack([p1 - p0, p2 - p1, p0 - p2]), axis=2)
        assert el.max() < 2.0 * h and el.min() > 0.3 * h
        assert (el.max(axis=0) / el.min(axis=0)).max() < 2.0
        area = 0.5 * np.linalg.norm(nrm, axis=1).sum()
        assert abs(area / _spheroid_area(a, b) - 1.0) < 2.0 * h * h
