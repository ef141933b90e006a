"""GMRES solution at the headline size against the oracle's own solution.

The rigid sphere of 81,920 triangles at kD = 100 under a plane wave along +z
(Section 5; eq. (eq_bm) with zero Neumann data), solved by bm_solve to a
relative residual of 1e-5 in the benchmark's configuration (every SVD
truncated at the paper's eps), in the plain FP64 form and in the FP32 form
with block Jacobi.  The expected surface field is the oracle's matrix-free
MGS-GMRES(50) solution, written by tests/golden/make_reference_solution.py
(oracle only; its provenance is stored in the file).  Bounds: the surface
field within 1e-3 of the oracle's (relative 2-norm), and within the
discretisation error of the Mie series.
"""
import os
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

REF = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sphere81920_k100_solution.npz")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ref():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(REF):
        pytest.skip("the oracle's reference solution has not been generated")
    z = np.load(REF, allow_pickle=False)
    V, T, prm = W.workload("sphere81920_kD100")
    import hashlib

    h = hashlib.sha256()
    h.update(np.ascontiguousarray(V, dtype=np.float64).tobytes())
    h.update(np.ascontiguousarray(T, dtype=np.int32).tobytes())
    assert str(z["mesh_sha256"]) == h.hexdigest(), "the stored solution is for another mesh"
    assert float(z["k"]) == prm["k"] and float(z["rel_residual"]) <= 1e-6
    return V, T, prm, z["u"]


@pytest.mark.parametrize("prec,precond", [("fp64", "none"), ("fp32", "block_jacobi")])
def test_headline_solution_matches_oracle_solution(ref, prec, precond):
    from paper_1403_4747_amd import Plan

    V, T, prm, uref = ref
    k = prm["k"]
    _say("[headline solve]", prec, precond)
    with Plan(V, T, k, prm["eps"], prec=prec, **prm["plan"]) as p:
        b = p.rhs_planewave(prm["direction"])
        x, info = p.solve(b, tol=1e-5, restart=50, precond=precond)
        u = x.cpu().numpy()
        b = b.cpu().numpy()
    _say("solve", {q: info[q] for q in ("iterations", "rel_residual", "seconds", "converged")})
    assert info["converged"] and info["rel_residual"] <= 1e-5
    # the product at the solution (a smooth, far-field-heavy vector): the
    # oracle's rows of A u against b on sampled rows, within the matvec bound
    # plus the solver tolerance
    rows = np.sort(np.random.default_rng(13).choice(len(T), size=2048, replace=False))
    res = float(np.linalg.norm(O.matvec(V, T, k, u, row_idx=rows) - b[rows]) / np.linalg.norm(b[rows]))
    _say(f"oracle residual of the solution on {len(rows)} rows {res:.3e}")
    assert res <= 1e-4 + 1e-5
    e = float(np.linalg.norm(u - uref) / np.linalg.norm(uref))
    cen = O.geometry(V, T)[0]
    um = O.mie_rigid_sphere(0.5, k, cen[:, 2] / np.linalg.norm(cen, axis=1))
    em = float(np.linalg.norm(u - um) / np.linalg.norm(um))
    eo = float(np.linalg.norm(uref - um) / np.linalg.norm(um))
    _say(f"vs oracle solution {e:.3e}; vs Mie {em:.3e} (oracle vs Mie {eo:.3e})")
    assert e <= 1e-3
    # the GPU solution is as close to the Mie series as the oracle's own
    assert abs(em - eo) <= 1e-3 and em <= 5e-2
