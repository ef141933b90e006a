"""GPU test of the allocation-free entry point fda_mlp_forward_noalloc.

The entry point runs the network's forward pass with its hidden activations
in a static per-device array instead of allocated work buffers.  Its output
must equal fda_mlp_forward's (the same kernels, so bit for bit) on two calls
in a row, the second with fewer rows than the first, and sizes above the
static array's limit must be refused before anything is launched.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HIDDEN = 256
MAX_ROWS = (8 << 20) // (2 * HIDDEN)  # 2 x rows x hidden floats of static scratch


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def net():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1403_4747_amd import Mlp

    m = Mlp(hidden=HIDDEN, seed=3)
    yield m
    m.close()


def _rows(n, seed):
    g = np.random.default_rng(seed)
    return torch.from_numpy(g.standard_normal((n, 272)).astype(np.float32)).to("cuda")


def test_noalloc_forward_equals_forward_on_two_calls(net):
    for n, seed in ((3000, 0), (700, 1)):
        _say("[noalloc] rows", n)
        X = _rows(n, seed)
        ref = net.forward(X)
        out = torch.full((n, 128), float("nan"), dtype=torch.float32, device="cuda")
        net.forward_noalloc(X, out)
        torch.cuda.synchronize()
        a, b = ref.cpu().numpy(), out.cpu().numpy()
        assert np.all(np.isfinite(b))
        assert np.array_equal(a, b), float(np.max(np.abs(a - b)))


def test_noalloc_forward_at_its_largest_size(net):
    _say("[noalloc] rows", MAX_ROWS)
    X = _rows(MAX_ROWS, 2)
    out = torch.empty((MAX_ROWS, 128), dtype=torch.float32, device="cuda")
    net.forward_noalloc(X, out)
    ref = net.forward(X)
    torch.cuda.synchronize()
    assert np.array_equal(ref.cpu().numpy(), out.cpu().numpy())


def test_noalloc_forward_refuses_sizes_beyond_its_scratch(net):
    from paper_1403_4747_amd import FDAError

    n = MAX_ROWS + 1
    X = torch.zeros((n, 272), dtype=torch.float32, device="cuda")
    out = torch.zeros((n, 128), dtype=torch.float32, device="cuda")
    with pytest.raises(FDAError) as e:
        net.forward_noalloc(X, out)
    assert e.value.code == -1 and "static scratch" in str(e.value)
    assert float(out.abs().sum()) == 0.0
