"""The merged M2L launch configuration (fda_m2l_get_config / set_config)
and its autotuner (fda_autotune): kernel variant and item order leave the
product unchanged bit for bit, the width per level changes it only by
rounding (the k-split of the first product), the tuner leaves a valid
configuration behind, and bad configurations are rejected without changing
the plan."""
import sys

import numpy as np
import pytest

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


def _plan_with_lowrank(prec):
    """The smallest named workload whose plan has low-rank M2L levels."""
    from paper_1403_4747_amd import Plan

    for name in ("sphere5120_kD20", "sphere20480_kD50"):
        V, T, prm = W.workload(name)
        p = Plan(V, T, prm["k"], prm["eps"], prec=prec)
        if p.m2l_config()["width"]:
            return name, p, len(T)
        p.close()
    pytest.fail("no workload with low-rank M2L levels")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_every_m2l_configuration_gives_the_same_product(prec):
    name, p, n = _plan_with_lowrank(prec)
    _say(f"[tune] {name} {prec}: all variants x orders x widths")
    with p:
        cfg0 = p.m2l_config()
        assert cfg0["variant"] == 0 and cfg0["xcd_order"] == 1
        assert set(cfg0["width"].values()) == {32}
        levels = list(cfg0["width"])
        X = torch.from_numpy(np.ascontiguousarray(W.complex_normal(n, 2, seed=41).T)).to("cuda")
        want = {32: p.matvec(X).cpu().numpy()}
        p.set_m2l_config(width={l: 16 for l in levels})
        want[16] = p.matvec(X).cpu().numpy()
        rel = np.linalg.norm(want[16] - want[32]) / np.linalg.norm(want[32])
        assert rel <= (1e-13 if prec == "fp64" else 1e-5), rel
        for w in (32, 16):
            for variant in range(4):
                for xcd in (1, 0):
                    got_cfg = p.set_m2l_config(variant=variant, xcd_order=xcd, width={l: w for l in levels})
                    assert got_cfg == dict(variant=variant, xcd_order=xcd, width={l: w for l in levels})
                    y = p.matvec(X).cpu().numpy()
                    assert np.array_equal(y, want[w]), (variant, xcd, w)


def test_autotune_keeps_the_product_and_reports():
    name, p, n = _plan_with_lowrank("fp64")
    _say(f"[tune] {name}: autotune")
    with p:
        x = torch.from_numpy(W.complex_normal(n, 1, seed=42)).to("cuda")
        want = p.matvec(x).cpu().numpy()
        r = p.autotune(reps=5)
        nl = r["nlevels"]
        assert nl == len(p.m2l_config()["width"]) > 0
        assert r["candidates"] == 1 + 3 + 1 + nl  # start, other variants, other order, one width flip per level
        assert r["ms_before"] > 0 and r["ms_after"] > 0
        assert r["best"] == p.m2l_config()
        y = p.matvec(x).cpu().numpy()
        if set(r["best"]["width"].values()) == {32}:
            assert np.array_equal(y, want)
        else:
            assert np.linalg.norm(y - want) <= 1e-13 * np.linalg.norm(want)
        _, info = p.solve(p.rhs_planewave(W.workload(name)[2]["direction"]), tol=1e-6)
        assert info["converged"]


def test_bad_configurations_are_rejected_and_change_nothing():
    from paper_1403_4747_amd import FDAError

    name, p, n = _plan_with_lowrank("fp64")
    _say(f"[tune] {name}: argument errors")
    with p:
        cfg0 = p.m2l_config()
        lev = next(iter(cfg0["width"]))
        for kw in (dict(variant=4), dict(variant=-1), dict(xcd_order=2), dict(width={lev: 24}),
                   dict(width={lev: 0})):
            with pytest.raises(FDAError):
                p.set_m2l_config(**kw)
            assert p.m2l_config() == cfg0
        with pytest.raises(FDAError):
            p.autotune(reps=0)
