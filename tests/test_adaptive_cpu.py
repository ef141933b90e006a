"""Adaptive trees (Section 3.2: leaves on any level) on the host: the tree
and list phase through fda_inspect.  The U, V, W and X lists together must
reach every ordered element pair exactly once; leaves sit on several
levels of a graded mesh that a uniform tree refuses; a uniform mesh built
adaptively is still covered exactly."""
import math

import numpy as np
import pytest

import workloads as W


def _inspect(V, T, k, **kw):
    from paper_1403_4747_amd import inspect

    return inspect(V, T, k, 1e-4, **kw)


def test_graded_sphere_mesh():
    V, T = W.graded_sphere(3)
    assert len(T) == 4952
    assert np.allclose(np.linalg.norm(V, axis=1), 0.5, atol=1e-12)
    p0, p1, p2 = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    nrm = np.cross(p1 - p0, p2 - p0)
    c = (p0 + p1 + p2) / 3.0
    assert np.all(np.einsum("ij,ij->i", nrm, c) > 0)  # outward
    el = np.linalg.norm(np.stack([p1 - p0, p2 - p1, p0 - p2]), axis=2)
    assert el.max() / el.min() > 4.0  # graded: 4:1 in edge length
    # refined towards +z: the finest triangles lie in the top cap
    small = el.max(axis=0) < 1.5 * el.min()
    assert np.all(c[small, 2] > 0.3 * 0.5)
    # area converges to the sphere's (flat triangles inside the sphere)
    area = 0.5 * np.linalg.norm(nrm, axis=1).sum()
    assert 0.97 * math.pi < area < math.pi


@pytest.mark.parametrize("s,k", [(3, 10.0), (4, 20.0)])
def test_adaptive_tree_covers_every_pair_once(s, k):
    V, T = W.graded_sphere(s)
    n = len(T)
    st = _inspect(V, T, k, adaptive=1)
    assert st["near_nnz"] + st["far_elem_pairs"] == n * n
    nz = [l for l, c in enumerate(st["leaves"]) if c > 0]
    assert len(nz) >= 3, st["leaves"]  # leaves on several levels
    assert sum(st["leaves"]) == st["nleaf"]
    # W and X lists are duals: a (target leaf, source box) W pair is an X
    # entry seen from the source side
    assert st["w_pairs"] == st["x_pairs"] > 0
    assert st["max_leaf_count"] <= 256
    assert sum(st["m2l_pairs"]) > 0


def test_uniform_tree_refuses_the_graded_mesh():
    from paper_1403_4747_amd import FDAError

    V, T = W.graded_sphere(3)
    with pytest.raises(FDAError) as e:
        _inspect(V, T, 10.0)
    assert e.value.code == -2 and "256" in str(e.value)


@pytest.mark.parametrize("name", ["sphere5120_kD20", "sphere20480_kD100"])
def test_adaptive_build_of_a_uniform_mesh(name):
    """On a quasi-uniform sphere the adaptive tree stops some boxes early;
    coverage stays exact and directional levels keep no leaves."""
    V, T, prm = W.workload(name)
    n = len(T)
    u = _inspect(V, T, prm["k"])
    a = _inspect(V, T, prm["k"], adaptive=1)
    assert a["near_nnz"] + a["far_elem_pairs"] == n * n
    assert a["depth"] == u["depth"] and a["nleaf"] <= u["nleaf"]
    for l, h in enumerate(a["hf"]):
        if h:
            assert a["leaves"][l] == 0


def test_adaptive_option_is_validated():
    from paper_1403_4747_amd import FDAError

    V, T, prm = W.workload("sphere1280_kD10")
    with pytest.raises(FDAError) as e:
        _inspect(V, T, prm["k"], adaptive=2)
    assert e.value.code == -1
