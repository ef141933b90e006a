"""A deep directional case on a non-spherical body: the prolate spheroid
(2.5, 0.5, 0.5) of the large benchmark case, meshed by the ring mesher with
215,018 triangles, at kD = 250 (directional levels 1-4), leaves at least two
longest edges wide as in that case: the FDA matvec against the oracle on
1,024 sampled rows (FP64 and FP32 plans; one oracle product serves both)
and GMRES to 1e-5 for an oblique plane wave."""
import math
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


_ORACLE = {}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_spheroid_kD250_matches_oracle_and_solves(prec):
    from paper_1403_4747_amd import Plan

    V, T = W.spheroid_rings(0.0108)
    n, k = len(T), 250.0 / 5.0
    _say(f"[spheroid] N={n} kD=250 {prec}")
    x = W.complex_normal(n, 1, seed=61)
    rows = np.sort(np.random.default_rng(62).choice(n, size=1024, replace=False))
    th = math.radians(30.0)
    with Plan(V, T, k, 1e-4, prec=prec, leaf_min_h=2.0) as p:
        st = p.stats()
        assert sum(st["hf"]) >= 3 and st["max_leaf_count"] <= 64
        y = p.matvec(torch.from_numpy(x).to("cuda")).cpu().numpy()
        _, info = p.solve(p.rhs_planewave((math.cos(th), math.sin(th), 0.0)), tol=1e-5)
    if "yr" not in _ORACLE:
        _ORACLE["yr"] = O.matvec(V, T, k, x, row_idx=rows)
    yr = _ORACLE["yr"]
    _say("rel err", P.rel_err(y[rows], yr), "row err", P.row_err(y[rows], yr), "its", info["iterations"])
    P.check(y[rows], yr, regress=P.REGRESS)
    assert info["converged"] and info["iterations"] < 100
