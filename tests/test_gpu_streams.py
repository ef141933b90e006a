"""Stream behaviour of fda_matvec: the near field runs on the plan's own
stream beside the far field; the product must equal the one-stream product
(the stage-timing path) bit for bit, on any caller stream, and a matvec
captured into a torch CUDA graph (where everything stays on the captured
stream) must replay to the eager result."""
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


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_overlapped_product_equals_one_stream_product(prec):
    from paper_1403_4747_amd import Plan

    _say(f"[streams] sphere5120_kD20 {prec}: side-stream near field vs one stream")
    V, T, prm = W.workload("sphere5120_kD20")
    n = len(T)
    X = _dev(W.complex_normal(n, 3, seed=31).T)
    with Plan(V, T, prm["k"], prm["eps"], prec=prec) as p:
        assert p.stats()["nleaf"] > 1
        y_overlap = p.matvec(X).cpu().numpy()
        y_seq = torch.empty_like(X)
        p.profile(X, reps=1, out=y_seq)  # every stage on the caller's stream
        y_seq = y_seq.cpu().numpy()
        # a non-default caller stream with work queued ahead of the product
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            X2 = X * 1.0
            y_other = p.matvec(X2)
        s.synchronize()
        y_other = y_other.cpu().numpy()
    assert np.array_equal(y_overlap, y_seq)
    assert np.array_equal(y_other, y_seq)


def test_torch_graph_capture_replays_the_eager_product():
    from paper_1403_4747_amd import Plan

    _say("[streams] torch CUDA graph of one matvec, 3 replays")
    V, T, prm = W.workload("sphere5120_kD20")
    n = len(T)
    with Plan(V, T, prm["k"], prm["eps"]) as p:
        x = _dev(W.complex_normal(n, 1, seed=32))
        y = torch.zeros_like(x)
        want = p.matvec(x).cpu().numpy()  # also sizes the plan's work buffers before capture
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
            assert np.array_equal(y.cpu().numpy(), want), rep
            z = p.matvec(torch.ones_like(x))  # eager product between replays
            torch.cuda.synchronize()
            assert torch.isfinite(z.real).all()
        x.mul_(2.0)
        g.replay()
        torch.cuda.synchronize()
        assert np.allclose(y.cpu().numpy(), 2.0 * want, rtol=1e-13, atol=0)
