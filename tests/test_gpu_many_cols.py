"""The merged low-rank M2L in its many-column form (from 8 right-hand
sides in FP64 plans, 16 in FP32 ones): phase 1 stores Z = V^ S per
interaction pair and a destination-major kernel sums U^ Z over every
incoming state's list on the matrix cores.
Every column of such a product must equal the single-column product (which
reduces per-pair kd-row scratch columns instead) to rounding, for column
counts that fill one, two and four 16-column tiles, leave a ragged tile, and
span two column blocks; sampled rows are checked against the oracle."""
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


# FP64: the two forms sum the same terms in different orders (rounding);
# FP32: operators and states are stored in single precision
_TOL = {"fp64": 1e-12, "fp32": 2e-6}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_many_column_products_equal_single_columns(prec):
    from paper_1403_4747_amd import Plan

    # the smallest named workload whose plan has low-rank M2L levels
    for name in ("sphere5120_kD20", "sphere20480_kD50"):
        V, T, prm = W.workload(name)
        p = Plan(V, T, prm["k"], prm["eps"], prec=prec, nrhs_max=70)
        if max(p.stats()["m2l_rank_max"]) > 0:
            break
        p.close()
    else:
        pytest.fail("no workload with low-rank M2L levels")
    n = len(T)
    _say(f"[many-cols] {name}")
    with p:
        for nrhs in (8, 16, 33, 64, 70):
            _say(f"[many-cols] {prec} nrhs={nrhs}")
            X = W.complex_normal(n, nrhs, seed=40 + nrhs).T  # (nrhs, N)
            Xd = _dev(X)
            Y = p.matvec(Xd).cpu().numpy()
            assert np.array_equal(Y, p.matvec(Xd).cpu().numpy())  # deterministic
            for c in sorted({0, min(15, nrhs - 1), nrhs // 2, nrhs - 1}):
                y1 = p.matvec(_dev(X[c])).cpu().numpy()
                err = np.max(np.abs(Y[c] - y1)) / np.max(np.abs(y1))
                assert err <= _TOL[prec], (nrhs, c, err)
        # one column of a 64-column product against the oracle's rows
        X = W.complex_normal(n, 64, seed=99).T
        Y = p.matvec(_dev(X)).cpu().numpy()
    rows = np.sort(np.random.default_rng(5).choice(n, size=256, replace=False))
    yr = O.matvec(V, T, prm["k"], X[37].copy(), row_idx=rows)
    rel = float(np.linalg.norm(Y[37][rows] - yr) / np.linalg.norm(yr))
    _say(f"[many-cols] {prec} column 37 of 64 vs oracle rows: {rel:.2e}")
    assert rel <= 1e-4


@pytest.mark.parametrize("case", ["graded_adaptive", "directional_leaves_adaptive"])
def test_many_column_products_on_adaptive_trees(case):
    """40 columns (both many-column forms in an FP64 plan) on adaptive trees:
    the graded sphere (leaves on several levels, U / W / X lists) and the
    5,120-triangle ellipsoid at kD = 97 whose leaves sit on directional
    levels; every sampled column equals its single-column product."""
    from paper_1403_4747_amd import Plan

    if case == "graded_adaptive":
        V, T = W.graded_sphere(3)
        k = 20.0
    else:
        V, T, k, info = W.uneven_batch(32)[25]
        assert info["n"] == 5120
    n = len(T)
    _say(f"[many-cols] {case} N={n} k={k:.2f}")
    X = W.complex_normal(n, 40, seed=77).T
    with Plan(V, T, k, 1e-4, adaptive=1, nrhs_max=40) as p:
        Y = p.matvec(_dev(X)).cpu().numpy()
        for c in (0, 17, 39):
            y1 = p.matvec(_dev(X[c])).cpu().numpy()
            err = np.max(np.abs(Y[c] - y1)) / np.max(np.abs(y1))
            assert err <= _TOL["fp64"], (case, c, err)
