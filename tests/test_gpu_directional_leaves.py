"""Leaves on a directional level (Section 3.2, completely adaptive trees;
Algorithm, Step 2: the S2M of a high-frequency leaf, per direction).

The 5,120-triangle ellipsoid of the seeded uneven batch at kD = 97 has about
two elements per wavelength: boxes narrow enough to be leaves are already
directional, so every leaf keeps one outgoing and one incoming state per
direction slot (24 slots here), with its own S2M and L2T per slot.  The fast
matvec, the Neumann right-hand side and the GMRES solution are checked
against the dense oracle, for the uniform and the adaptive tree, FP64 and
FP32.
"""
import sys

import numpy as np
import pytest

import _parity as P
import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mesh():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    V, T, k, info = W.uneven_batch(32)[25]
    assert info["n"] == 5120 and info["kD"] > 97
    return V, T, k


_ORACLE = {}


def _oracle_y(V, T, k, x):
    if "y" not in _ORACLE:
        _ORACLE["y"] = O.matvec(V, T, k, x)
    return _ORACLE["y"]


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _hf_leaf_levels(st):
    return [l for l in range(st["depth"] + 1) if st["hf"][l] and st["leaves"][l] > 0]


@pytest.mark.parametrize("adaptive,prec", [(0, "fp64"), (1, "fp64"), (0, "fp32")])
def test_directional_leaves_matvec_matches_oracle(mesh, adaptive, prec):
    from paper_1403_4747_amd import Plan

    V, T, k = mesh
    x = W.complex_normal(len(T), 1, seed=0)
    _say(f"[directional leaves] N={len(T)} k={k:.2f} adaptive={adaptive} {prec}")
    with Plan(V, T, k, 1e-4, adaptive=adaptive, prec=prec) as p:
        st = p.stats()
        _say("depth", st["depth"], "hf", st["hf"][:st["depth"] + 1], "leaves", st["leaves"][:st["depth"] + 1],
             "slots", st["active_dirs"][:st["depth"] + 1])
        assert _hf_leaf_levels(st)
        y = p.matvec(_dev(x)).cpu().numpy()
        y2 = p.matvec(_dev(x)).cpu().numpy()
    yr = _oracle_y(V, T, k, x)
    e, r = P.check(y, yr)
    _say(f"rel err {e:.3e} row err {r:.3e}")
    assert np.array_equal(y, y2)


def test_directional_leaves_neumann_rhs_matches_oracle(mesh):
    """b = B g with B's S2M per direction slot on the directional leaves,
    against the oracle's B on the same Neumann data (an interior point
    source's normal derivative)."""
    from paper_1403_4747_amd import Plan

    V, T, k = mesh
    _, g = O.point_source_data(V, T, k, np.array([0.05, -0.02, 0.03]))
    rows = np.sort(np.random.default_rng(7).choice(len(T), size=512, replace=False))
    with Plan(V, T, k, 1e-4, neumann_rhs=1) as p:
        assert _hf_leaf_levels(p.stats())
        b = p.rhs_neumann(_dev(g)).cpu().numpy()
    br = O.neumann_rhs(V, T, k, g, row_idx=rows)
    e, r = P.check(b[rows], br)
    _say(f"neumann rhs rel err {e:.3e}")


def test_directional_leaves_solution_matches_oracle(mesh):
    """GMRES(50) to 1e-5 on the plane-wave problem: the surface field within
    1e-3 of the oracle's dense solution."""
    from paper_1403_4747_amd import Plan

    V, T, k = mesh
    d = np.array([0.0, 0.0, 1.0])
    with Plan(V, T, k, 1e-4) as p:
        b = p.rhs_planewave(d)
        u, info = p.solve(b, tol=1e-5, restart=50)
        u = u.cpu().numpy()
    _say("solve", {q: info[q] for q in ("iterations", "rel_residual", "converged")})
    assert info["converged"]
    A = O.assemble(V, T, k)
    ur = O.solve_dense(A, O.rhs_planewave(V, T, k, d))
    e = float(np.linalg.norm(u - ur) / np.linalg.norm(ur))
    _say(f"solution rel err {e:.3e}")
    assert e <= 1e-3
