"""Several meshes in one captured HIP graph (fda_batch_*): every replay
equals the plans' own products and the dense oracle's, with eager work
between the replays; calls that would reallocate what the graph references
are refused while the batch exists."""
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


def _meshes():
    V1, T1, p1 = W.workload("sphere1280_kD10")
    V2, T2, p2 = W.workload("sphere5120_kD20")
    V3, T3 = W.ellipsoid(3, (0.6, 0.4, 0.3))
    V4, T4 = W.octasphere(3, 0.5)
    return [(V1, T1, p1["k"], 1, "fp64"), (V2, T2, p2["k"], 3, "fp64"), (V3, T3, 12.0, 1, "fp32"),
            (V4, T4, 8.0, 2, "fp64")]


def test_batch_graph_replays_equal_the_single_products():
    from paper_1403_4747_amd import Batch, Plan

    _say("[batch] 4 meshes (1280, 5120, 1280 ellipsoid FP32, 512 octasphere)")
    plans, xs, ys, want = [], [], [], []
    for i, (V, T, k, nr, prec) in enumerate(_meshes()):
        p = Plan(V, T, k, 1e-4, prec=prec)
        x = W.complex_normal(len(T), nr, seed=20 + i)  # (N,) for one column, (N, nr) otherwise
        x = torch.from_numpy(np.ascontiguousarray(x if nr == 1 else x.T)).to("cuda")
        plans.append(p)
        xs.append(x)
        ys.append(torch.zeros_like(x))
        want.append(p.matvec(x).cpu().numpy())
    # the oracle's products of the same inputs (every row of each mesh)
    for i, (V, T, k, nr, prec) in enumerate(_meshes()):
        yr = O.matvec(V, T, k, xs[i].cpu().numpy().T if nr > 1 else xs[i].cpu().numpy())
        yr = yr.T if nr > 1 else yr
        _say(f"mesh {i}: N={len(T)} {prec} rel err {P.rel_err(want[i], yr):.2e}")
        P.check(want[i], yr, regress=P.REGRESS)
    b = Batch(plans, xs, ys)
    for rep in range(3):
        for y in ys:
            y.zero_()
        b.launch()
        torch.cuda.synchronize()
        for i in range(len(plans)):
            got = ys[i].cpu().numpy()
            assert np.array_equal(got, want[i]), (rep, i)
        # eager work between replays: other products on the same plans
        z = plans[1].matvec(torch.ones_like(xs[1]))
        torch.cuda.synchronize()
        assert torch.isfinite(z.real).all()
    # new inputs in the captured buffers are picked up by the next replay
    xs[0].mul_(2.0)
    b.launch()
    torch.cuda.synchronize()
    assert np.allclose(ys[0].cpu().numpy(), 2.0 * want[0], rtol=1e-13, atol=0)
    b.close()
    for p in plans:
        p.close()


def test_batch_rejects_a_repeated_plan():
    from paper_1403_4747_amd import Batch, FDAError, Plan

    V, T, prm = W.workload("sphere1280_kD10")
    p = Plan(V, T, prm["k"], prm["eps"])
    x = torch.zeros(len(T), dtype=torch.complex128, device="cuda")
    y = torch.zeros_like(x)
    y2 = torch.zeros_like(x)
    with pytest.raises(FDAError):
        Batch([p, p], [x, x], [y, y2])
    p.close()


def test_batch_keeps_its_buffers_in_place():
    """While a batch exists, calls that would reallocate the work buffers or
    the M2L work list it references fail cleanly; the batch still replays to
    the same products, and after it is freed the calls work again."""
    from paper_1403_4747_amd import Batch, FDAError, Plan

    V, T, prm = W.workload("sphere5120_kD20")
    p = Plan(V, T, prm["k"], prm["eps"], nrhs_max=4)
    x = torch.from_numpy(W.complex_normal(len(T), 1, seed=40)).to("cuda")
    y = torch.zeros_like(x)
    want = p.matvec(x).cpu().numpy()
    b = Batch([p], [x], [y])
    x2 = torch.zeros((2, len(T)), dtype=torch.complex128, device="cuda")
    with pytest.raises(FDAError):
        p.matvec(x2)  # two columns: the buffers hold one
    cfg = p.m2l_config()
    lv = next(iter(cfg["width"]))
    with pytest.raises(FDAError):
        p.set_m2l_config(width={lv: 16 if cfg["width"][lv] == 32 else 32})
    with pytest.raises(FDAError):
        p.autotune(reps=2)
    assert p.m2l_config() == cfg
    p.matvec(x)  # one column still fits
    b.launch()
    torch.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy(), want)
    b.close()
    Y = p.matvec(x2)
    torch.cuda.synchronize()
    assert Y.shape == x2.shape
    p.close()
