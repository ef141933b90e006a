"""Edge cases of the HIP path through the C ABI: degenerate and tiny meshes,
ragged trees, zero data, padded leading dimensions, the largest nrhs,
argument errors, other geometries and the FP32 plan's multi-column product."""
import ctypes
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _plan(V, T, k, eps=1e-4, **kw):
    from paper_1403_4747_amd import Plan

    return Plan(V, T, k, eps, **kw)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_single_triangle_is_the_half_identity_plus_self_term():
    _say("[edge] single triangle")
    V = np.array([[0.0, 0.0, 0.0], [0.1, 0.0, 0.0], [0.0, 0.1, 0.0]])
    T = np.array([[0, 1, 2]], dtype=np.int32)
    k = 3.0
    A = O.assemble(V, T, k)
    x = np.array([0.7 - 0.2j])
    with _plan(V, T, k) as p:
        assert p.stats()["nleaf"] == 1
        y = p.matvec(_dev(x)).cpu().numpy()
    assert abs(y[0] - A[0, 0] * x[0]) <= 1e-12 * abs(A[0, 0] * x[0])


def test_icosahedron_all_near_equals_dense():
    _say("[edge] icosahedron N=20")
    V, T = W.icosphere(0, 0.5)
    k = 2.0
    A = O.assemble(V, T, k)
    x = W.complex_normal(len(T), 1, seed=3)
    with _plan(V, T, k) as p:
        y = p.matvec(_dev(x)).cpu().numpy()
    assert _rel(y, A @ x) <= 1e-12


def test_zero_vector_and_zero_rhs():
    _say("[edge] zero input, zero right-hand side")
    V, T, prm = W.workload("sphere5120_kD20")
    with _plan(V, T, prm["k"], prm["eps"]) as p:
        z = torch.zeros(len(T), dtype=torch.complex128, device="cuda")
        y = p.matvec(z)
        assert torch.count_nonzero(y).item() == 0
        x, info = p.solve(z, tol=1e-6)
        assert info["converged"] and info["iterations"] == 0 and torch.count_nonzero(x).item() == 0


@pytest.mark.parametrize("name,max_leaf", [("sphere5120_kD20", 128), ("sphere5120_kD20", 16)])
def test_leaf_capacity_variants_match_oracle(name, max_leaf):
    """Leaf capacity 128 (a shallower tree whose leaves hold up to 117
    elements, above the 64 of one MFMA-sized block) and 16 (the leaf-width
    floor keeps the default depth) on the 5,120-triangle sphere at kD = 20."""
    _say(f"[edge] {name} max_leaf={max_leaf}")
    V, T, prm = W.workload(name)
    k = prm["k"]
    x = W.complex_normal(len(T), 1, seed=4)
    with _plan(V, T, k, prm["eps"], max_leaf=max_leaf) as p:
        st = p.stats()
        y = p.matvec(_dev(x)).cpu().numpy()
        b = p.rhs_planewave(prm["direction"])
        u1, i1 = p.solve(b, tol=1e-6, precond="block_jacobi")
        u0, i0 = p.solve(b, tol=1e-6)
    if max_leaf > 64:
        assert st["max_leaf_count"] > 64
    yr = O.matvec(V, T, k, x)
    assert _rel(y, yr) <= 1e-4
    assert i0["converged"] and i1["converged"]
    assert float(torch.linalg.norm(u1 - u0) / torch.linalg.norm(u0)) <= 1e-4


def test_both_svd_methods_match_oracle():
    """The build's batched SVDs by one-sided Jacobi (svd_method 1, the
    default) and by bidiagonalisation + QR (0) truncate to the same ranks,
    and both products meet the oracle on the 5,120-triangle sphere at
    kD = 20 (their difference is a rotation inside the kept subspaces,
    orders below the matvec bound)."""
    _say("[edge] svd_method 0 and 1")
    V, T, prm = W.workload("sphere5120_kD20")
    k = prm["k"]
    x = W.complex_normal(len(T), 1, seed=6)
    ys, ranks = [], []
    for meth in (0, 1):
        with _plan(V, T, k, prm["eps"], svd_method=meth) as p:
            st = p.stats()
            ranks.append((st["rank_up"], st["rank_dn"], st["m2l_rank_max"]))
            ys.append(p.matvec(_dev(x)).cpu().numpy())
    yr = O.matvec(V, T, k, x)
    # a singular value within rounding of the truncation threshold could be
    # kept by one method and dropped by the other: ranks agree to one
    for a0, a1 in zip(ranks[0], ranks[1]):
        assert all(abs(int(u) - int(v)) <= 1 for u, v in zip(a0, a1)), ranks
    for y in ys:
        assert _rel(y, yr) <= 1e-4
    assert _rel(ys[1], ys[0]) <= 5e-5


def test_padded_leading_dimension_through_the_c_abi():
    """x and y with leading dimension ld = N + 7 (column-major N x nrhs):
    the product equals the contiguous one and the padding is untouched."""
    from paper_1403_4747_amd import library

    _say("[edge] ld = N + 7 via fda_matvec")
    V, T, prm = W.workload("sphere1280_kD10")
    n, nr, ld = len(T), 3, len(T) + 7
    x = W.complex_normal(n, nr, seed=5)  # (n, nr)
    xp = np.full((nr, ld), 9.0 + 9.0j)
    xp[:, :n] = x.T
    with _plan(V, T, prm["k"], prm["eps"]) as p:
        want = p.matvec(_dev(x.T)).cpu().numpy()
        xd = _dev(xp)
        yd = torch.full((nr, ld), -5.0 - 5.0j, dtype=torch.complex128, device="cuda")
        s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        rc = library().fda_matvec(p._h, xd.data_ptr(), yd.data_ptr(), nr, ld, s)
        assert rc == 0
        # ld < N is rejected
        assert library().fda_matvec(p._h, xd.data_ptr(), yd.data_ptr(), nr, n - 1, s) < 0
        torch.cuda.synchronize()
        y = yd.cpu().numpy()
    assert np.max(np.abs(y[:, :n] - want)) <= 1e-13 * np.max(np.abs(want))
    assert np.all(y[:, n:] == -5.0 - 5.0j)


def test_nrhs_at_and_above_the_limit():
    from paper_1403_4747_amd import FDAError

    _say("[edge] nrhs = nrhs_max and nrhs_max + 1")
    V, T, prm = W.workload("sphere1280_kD10")
    n = len(T)
    with _plan(V, T, prm["k"], prm["eps"], nrhs_max=8) as p:
        X = _dev(W.complex_normal(n, 8, seed=6).T)
        Y = p.matvec(X).cpu().numpy()
        y0 = p.matvec(X[5].contiguous()).cpu().numpy()
        assert np.max(np.abs(Y[5] - y0)) <= 1e-13 * np.max(np.abs(y0))
        with pytest.raises(FDAError):
            p.matvec(_dev(W.complex_normal(n, 9, seed=7).T))


def test_argument_errors_on_gpu_entry_points():
    from paper_1403_4747_amd import FDAError, library

    _say("[edge] argument errors")
    V, T, prm = W.workload("sphere1280_kD10")
    n = len(T)
    L = library()
    with _plan(V, T, prm["k"], prm["eps"]) as p:
        b = p.rhs_planewave(prm["direction"])
        x = torch.empty_like(b)
        for kw in (dict(restart=0), dict(maxit=0), dict(tol=0.0), dict(tol=-1.0), dict(restart=501)):
            with pytest.raises(FDAError):
                p.solve(b, **kw)
        with pytest.raises(KeyError):
            p.solve(b, precond="ilu")
        s = ctypes.c_void_p(0)
        d = (ctypes.c_double * 3)(0.0, 0.0, 1.0)
        assert L.bm_rhs_planewave(p._h, ctypes.cast(d, ctypes.c_void_p), 0, b.data_ptr(), n, s) < 0
        assert L.fda_matvec(p._h, None, x.data_ptr(), 1, n, s) < 0
        assert L.fda_matvec(None, b.data_ptr(), x.data_ptr(), 1, n, s) < 0
        with pytest.raises(TypeError):
            p.matvec(b.to(torch.complex64))
        with pytest.raises(ValueError):
            p.matvec(b[: n - 1].contiguous())
        # an output tensor of another shape than the input (the library would
        # write nrhs x N values into it), or the input itself, is refused
        X4 = torch.zeros((4, n), dtype=torch.complex128, device="cuda")
        for bad in (torch.empty_like(b), torch.empty((2, n), dtype=torch.complex128, device="cuda")):
            with pytest.raises(ValueError):
                p.matvec(X4, out=bad if bad.dim() == 2 else bad)
        with pytest.raises(ValueError):
            p.matvec(b, out=torch.empty((1, n), dtype=torch.complex128, device="cuda"))
        with pytest.raises(ValueError):
            p.matvec(b, out=b)
        with pytest.raises(ValueError):
            p.solve(X4, out=torch.empty_like(b))
        with pytest.raises(ValueError):
            p.profile(X4, reps=1, out=torch.empty_like(b))
    # build errors: k <= 0, eps out of range, vertex index out of range
    from paper_1403_4747_amd import Plan

    for args in ((V, T, -1.0, 1e-4), (V, T, 10.0, 1.5)):
        with pytest.raises(FDAError):
            Plan(*args)
    Tbad = T.copy()
    Tbad[0, 0] = len(V) + 3
    with pytest.raises(FDAError):
        Plan(V, Tbad, 10.0, 1e-4)


@pytest.mark.parametrize("geom", ["ellipsoid", "octasphere"])
def test_other_geometries_match_oracle(geom):
    """The FDA matvec on an ellipsoid (semi-axes 0.6, 0.4, 0.3; 5,120
    triangles, kD = 24) and an octahedral sphere (8,192 triangles, kD = 20)
    against the oracle on sampled rows."""
    _say(f"[edge] {geom}")
    if geom == "ellipsoid":
        V, T = W.ellipsoid(4, (0.6, 0.4, 0.3))
        k = 24.0 / 1.2
    else:
        V, T = W.octasphere(5, 0.5)
        k = 20.0
    n = len(T)
    x = W.complex_normal(n, 1, seed=8)
    rows = np.sort(np.random.default_rng(9).choice(n, size=200, replace=False))
    with _plan(V, T, k, 1e-4) as p:
        y = p.matvec(_dev(x)).cpu().numpy()
    yr = O.matvec(V, T, k, x, row_idx=rows)
    assert _rel(y[rows], yr) <= 1e-4


def test_fp32_plan_multi_column_equals_single_and_is_deterministic():
    _say("[edge] FP32 plan, 4 columns")
    V, T, prm = W.workload("sphere5120_kD20")
    n = len(T)
    X = _dev(W.complex_normal(n, 4, seed=10).T)
    with _plan(V, T, prm["k"], prm["eps"], prec="fp32") as p:
        Y = p.matvec(X).cpu().numpy()
        Y2 = p.matvec(X).cpu().numpy()
        y2 = p.matvec(X[2].contiguous()).cpu().numpy()
    assert np.array_equal(Y, Y2)
    assert np.max(np.abs(Y[2] - y2)) <= 1e-6 * np.max(np.abs(y2))
