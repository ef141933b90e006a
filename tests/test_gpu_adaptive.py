"""Adaptive trees on the GPU (Section 3.2: leaves on any non-directional
level; leaf pairs on different levels that no interaction list separates,
the U, W and X lists of adaptive FMMs, evaluated directly): the fast
matvec, the Neumann right-hand side and GMRES against the dense oracle, on
graded spheres (4:1 in edge length, which a uniform tree refuses) and on a
uniform sphere built adaptively."""
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


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _plan(V, T, k, eps=1e-4, **kw):
    from paper_1403_4747_amd import Plan

    return Plan(V, T, k, eps, adaptive=1, **kw)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _check_adaptive_stats(st):
    assert sum(1 for c in st["leaves"] if c > 0) >= 2, st["leaves"]
    assert st["w_pairs"] == st["x_pairs"] > 0
    assert st["near_nnz"] + st["far_elem_pairs"] == st["n"] ** 2
    assert st["m2l_flops"] > 0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_graded_sphere_matvec_matches_oracle(prec):
    """4,952-triangle graded sphere, kD = 10, two columns: every row within
    the matvec bound 1e-4 (relative 2-norm) of the dense oracle."""
    V, T = W.graded_sphere(3)
    k = 10.0
    X = W.complex_normal(len(T), 2, seed=61)  # (n, 2)
    _say(f"[adaptive] graded sphere N={len(T)} kD=10 {prec}")
    with _plan(V, T, k, prec=prec) as p:
        st = p.stats()
        _say("leaves per level", st["leaves"], "U/W/X", st["u_pairs"], st["w_pairs"], st["x_pairs"])
        _check_adaptive_stats(st)
        Y = p.matvec(_dev(X.T)).cpu().numpy()
        y1 = p.matvec(_dev(X[:, 1])).cpu().numpy()
        y1b = p.matvec(_dev(X[:, 1])).cpu().numpy()
    for c in range(2):
        err = _rel(Y[c], O.matvec(V, T, k, X[:, c]))
        _say("rel err", c, err)
        assert err < 1e-4
    assert np.array_equal(y1, y1b)  # deterministic
    assert np.max(np.abs(Y[1] - y1)) <= (1e-13 if prec == "fp64" else 1e-6) * np.max(np.abs(y1))


@pytest.mark.parametrize("s,k,rows", [(4, 60.0, 256), (5, 100.0, 96)])
def test_graded_sphere_directional_sampled_rows(s, k, rows):
    """Graded spheres with directional levels above the leaves (19,760
    triangles at kD = 60, 79,106 at kD = 100): sampled rows against the
    oracle row by row, relative 2-norm <= 1e-4."""
    V, T = W.graded_sphere(s)
    x = W.complex_normal(len(T), 1, seed=62)
    _say(f"[adaptive] graded sphere N={len(T)} kD={k:g}, {rows} sampled rows")
    with _plan(V, T, k) as p:
        st = p.stats()
        _say("leaves per level", st["leaves"], "hf", st["hf"], "pairs", st["m2l_pairs"])
        _check_adaptive_stats(st)
        assert any(st["hf"][l] and st["m2l_pairs"][l] > 0 for l in range(st["depth"] + 1))
        y = p.matvec(_dev(x)).cpu().numpy()
    r = np.sort(np.random.default_rng(6).choice(len(T), size=rows, replace=False))
    yr = O.matvec(V, T, k, x, row_idx=r)
    err = _rel(y[r], yr)
    _say("rel err", err)
    assert err < 1e-4


def test_uniform_sphere_built_adaptively_matches_oracle():
    """5,120-triangle sphere at kD = 20 with an adaptive tree (some boxes stop
    a level early, so W and X lists appear): within 1e-4 of the oracle, and
    of the uniform plan's product."""
    from paper_1403_4747_amd import Plan

    V, T, prm = W.workload("sphere5120_kD20")
    k = prm["k"]
    x = W.complex_normal(len(T), 1, seed=63)
    _say("[adaptive] sphere5120_kD20 adaptive vs uniform")
    with _plan(V, T, k, prm["eps"]) as p:
        st = p.stats()
        _check_adaptive_stats(st)
        ya = p.matvec(_dev(x)).cpu().numpy()
    with Plan(V, T, k, prm["eps"]) as q:
        yu = q.matvec(_dev(x)).cpu().numpy()
    yr = O.matvec(V, T, k, x)
    assert _rel(ya, yr) < 1e-4
    assert _rel(ya, yu) < 2e-4


def test_graded_sphere_solve_satisfies_the_oracle_system():
    """Plane-wave scattering on the graded sphere: GMRES on the adaptive plan
    (with and without block Jacobi) converges to a u whose dense-oracle
    residual is within the matvec bound."""
    V, T = W.graded_sphere(3)
    k = 10.0
    _say("[adaptive] graded sphere solve")
    with _plan(V, T, k) as p:
        b = p.rhs_planewave((0.0, 0.0, 1.0))
        u, info = p.solve(b, tol=1e-6)
        ub, infob = p.solve(b, tol=1e-6, precond="block_jacobi")
    assert info["converged"] and infob["converged"]
    _say("iterations", info["iterations"], "with block Jacobi", infob["iterations"])
    u, ub, b = u.cpu().numpy(), ub.cpu().numpy(), b.cpu().numpy()
    assert _rel(b, O.rhs_planewave(V, T, k, (0.0, 0.0, 1.0))) < 1e-12
    assert _rel(O.matvec(V, T, k, u), b) < 1e-4
    assert _rel(ub, u) < 1e-4


def test_graded_sphere_neumann_rhs_matches_oracle():
    """B g (the right-hand operator for Neumann data) on the adaptive plan:
    leaf S2M of B at every leaf level."""
    V, T = W.graded_sphere(3)
    k = 10.0
    g = W.complex_normal(len(T), 1, seed=64)
    _say("[adaptive] graded sphere Neumann right-hand side")
    with _plan(V, T, k, neumann_rhs=1) as p:
        bg = p.rhs_neumann(_dev(g)).cpu().numpy()
    assert _rel(bg, O.neumann_rhs(V, T, k, g)) < 1e-4


def test_adaptive_plans_in_a_batch_graph_and_a_torch_graph():
    """Adaptive plans (several S2M / L2T launches, two near-field launches)
    inside one captured HIP graph with a uniform plan (fda_batch), and a
    matvec captured into a torch CUDA graph: every replay equals the eager
    product, with eager work between the replays."""
    from paper_1403_4747_amd import Batch, Plan

    _say("[adaptive] batch graph: graded sphere FP64 + FP32 adaptive, uniform sphere")
    Vg, Tg = W.graded_sphere(3)
    Vu, Tu, pu = W.workload("sphere1280_kD10")
    plans = [_plan(Vg, Tg, 10.0), _plan(Vg, Tg, 10.0, prec="fp32"), Plan(Vu, Tu, pu["k"], pu["eps"])]
    xs, ys, want = [], [], []
    for i, p in enumerate(plans):
        x = torch.from_numpy(np.ascontiguousarray(W.complex_normal(p.n, 2, seed=70 + i).T)).to("cuda")
        xs.append(x)
        ys.append(torch.zeros_like(x))
        want.append(p.matvec(x).cpu().numpy())
    b = Batch(plans, xs, ys)
    for rep in range(3):
        for y in ys:
            y.zero_()
        b.launch()
        torch.cuda.synchronize()
        for i in range(len(plans)):
            assert np.array_equal(ys[i].cpu().numpy(), want[i]), (rep, i)
        z = plans[0].matvec(torch.ones_like(xs[0]))
        torch.cuda.synchronize()
        assert torch.isfinite(z.real).all()
    b.close()
    _say("[adaptive] torch CUDA graph of one adaptive matvec, 3 replays")
    p = plans[0]
    x = xs[0][0].contiguous()
    y = torch.zeros_like(x)
    w = p.matvec(x).cpu().numpy()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s, capture_error_mode="thread_local"):
            p.matvec(x, out=y)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        y.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy(), w), rep
        p.matvec(torch.ones_like(x))
        torch.cuda.synchronize()
    for q in plans:
        q.close()


def test_near_rows_longer_than_4096_columns():
    """Leaves of up to 256 elements on the graded sphere (4,952 triangles,
    kD = 10) give near-field rows of 4,952 columns (every element): the
    long-row kernel, which reads x through the column list, matches the
    dense oracle on every entry (FP64 and FP32 plans)."""
    V, T = W.graded_sphere(3)
    k = 10.0
    _say("[adaptive] rows above 4,096 columns")
    x = W.complex_normal(len(T), 1, seed=44)
    yr = O.matvec(V, T, k, x)
    for prec in ("fp64", "fp32"):
        with _plan(V, T, k, max_leaf=256, prec=prec) as p:
            st = p.stats()
            assert st["max_near_cols"] > 4096
            y = p.matvec(_dev(x)).cpu().numpy()
        _say(prec, "max cols", st["max_near_cols"], "rel err", P.rel_err(y, yr))
        P.check(y, yr, regress=P.REGRESS)
