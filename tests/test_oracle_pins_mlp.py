"""Pins of the learned-preconditioner oracle (oracle/mlp_ref.py) against
facts that do not come from the oracle itself: exact bfloat16 values, a
hand-evaluated network, central differences of the loss, the closed form of
Adam's first step and the block-Jacobi reduction."""
import numpy as np
import pytest

from oracle import mlp_ref as R


def test_bf16_round_exact_cases():
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -7, -2.5, 65504.0, 3.0e38, 3.4e38,
                  np.inf, -np.inf, 0.0, 1.0 + 2.0 ** -8 + 2.0 ** -20], dtype=np.float32)
    got = R.bf16_round(x)
    assert got[0] == 1.0 and got[1] == 1.0
    assert got[2] == np.float32(1.0 + 2.0 ** -6)
    assert got[3] == np.float32(1.0 + 2.0 ** -7)
    assert got[4] == -2.5
    assert got[5] == 65536.0  # 65504 = 1.9990234375 * 2^15 rounds up to 2^16 at 8 significant bits
    assert np.isinf(got[7]) and got[7] > 0  # above the largest bfloat16 (about 3.3895e38)
    assert got[8] == np.inf and got[9] == -np.inf and got[10] == 0.0
    assert got[11] == np.float32(1.0 + 2.0 ** -7)  # just above the tie rounds up
    # every output is a bfloat16: low 16 bits zero
    fin = np.isfinite(got)
    assert np.all(got[fin].view(np.uint32) & 0xFFFF == 0)
    # relative error of a random sample is at most the unit roundoff 2^-8 (8 significant bits)
    r = np.random.default_rng(0).standard_normal(10000).astype(np.float32)
    assert np.max(np.abs(R.bf16_round(r) - r) / np.abs(r)) <= 2.0 ** -8 + 1e-12
    assert np.isnan(R.bf16_round(np.float32(np.nan)))


def test_forward_hand_evaluated_width2():
    h = 2
    p = np.zeros(R.num_params(h), dtype=np.float32)
    W1, b1, W2, b2, W3, b3 = R.split(p, h)
    W1[0, 0], W1[1, 1] = 1.0, -1.0
    b1[:] = [0.5, 0.25]
    W2[0, 0], W2[1, 0], W2[1, 1] = 2.0, 1.0, 1.0
    b2[:] = [0.0, -1.0]
    W3[0, 0], W3[1, 5] = 1.0, 3.0
    b3[7] = 0.125
    X = np.zeros((2, R.MLP_IN))
    X[0, 0], X[0, 1] = 1.0, -2.0   # H1 = relu([1.5, 2.25]) ; H2 = relu([3 + 2.25, 2.25 - 1]) = [5.25, 1.25]
    X[1, 0], X[1, 1] = -3.0, 4.0   # H1 = relu([-2.5, -3.75]) = 0 ; H2 = relu([0, -1]) = 0
    Y, _, _ = R.forward(p, X, h, bf16=False)
    assert Y[0, 0] == pytest.approx(5.25) and Y[0, 5] == pytest.approx(3.75) and Y[0, 7] == pytest.approx(0.125)
    assert np.count_nonzero(Y[0]) == 3
    assert np.count_nonzero(Y[1]) == 1 and Y[1, 7] == pytest.approx(0.125)


def test_forward_bf16_rounds_layer_inputs_hand_evaluated():
    """The width-2 network of the test above with bfloat16 layer inputs:
    x = 1 + 3 / 512 rounds to 1 + 1 / 128 (bfloat16 keeps 7 fraction bits,
    ties to even), and the hidden values then stay exactly representable."""
    h = 2
    p = np.zeros(R.num_params(h), dtype=np.float32)
    W1, b1, W2, b2, W3, b3 = R.split(p, h)
    W1[0, 0], W1[1, 1] = 1.0, -1.0
    b1[:] = [0.5, 0.25]
    W2[0, 0], W2[1, 0], W2[1, 1] = 2.0, 1.0, 1.0
    b2[:] = [0.0, -1.0]
    W3[0, 0], W3[1, 5] = 1.0, 3.0
    X = np.zeros((1, R.MLP_IN))
    X[0, 0], X[0, 1] = 1.0 + 3.0 / 512, -2.0
    # bf16(x0) = 1 + 1/128: H1 = [1.5 + 1/128, 2.25]; H2 = [5.25 + 1/64, 1.25];
    # the last layer's input 5.265625 = 1.01010001b x 4 lies halfway between
    # two bfloat16 values and rounds to the even one, 5.25
    Y, H1, H2 = R.forward(p, X, h, bf16=True)
    assert H1[0, 0] == 1.5 + 1.0 / 128 and H1[0, 1] == 2.25
    assert H2[0, 0] == 5.25 + 1.0 / 64 and H2[0, 1] == 1.25
    assert Y[0, 0] == 5.25 and Y[0, 5] == 3.75
    Yf, _, _ = R.forward(p, X, h, bf16=False)
    assert Yf[0, 0] == pytest.approx(5.25 + 6.0 / 512)


@pytest.mark.parametrize("bf16", [False, True])
def test_gradient_matches_central_differences(bf16):
    rng = np.random.default_rng(1)
    h, rows = 5, 7
    p = (0.3 * rng.standard_normal(R.num_params(h))).astype(np.float32)
    if bf16:  # differentiate where the rounding is the identity: weights already bfloat16
        p = R.bf16_round(p)
    X = rng.standard_normal((rows, R.MLP_IN))
    T = rng.standard_normal((rows, R.MLP_OUT))
    M = (rng.random((rows, R.MLP_OUT)) < 0.7).astype(np.float64)
    L, g = R.loss_and_gradient(p, X, T, M, h, bf16=False)
    pd = p.astype(np.float64)
    idx = rng.choice(p.size, size=60, replace=False)
    # the loss as a plain function of FP64 parameters, written out without the oracle
    def loss(q):
        W1 = q[:R.MLP_IN * h].reshape(R.MLP_IN, h)
        o = R.MLP_IN * h
        b1 = q[o:o + h]; o += h
        W2 = q[o:o + h * h].reshape(h, h); o += h * h
        b2 = q[o:o + h]; o += h
        W3 = q[o:o + h * R.MLP_OUT].reshape(h, R.MLP_OUT); o += h * R.MLP_OUT
        b3 = q[o:]
        Y = np.maximum(np.maximum(X @ W1 + b1, 0) @ W2 + b2, 0) @ W3 + b3
        return np.sum((M * (Y - T)) ** 2) / (rows * R.MLP_OUT)
    assert loss(pd) == pytest.approx(L, rel=1e-12)
    for i in idx:
        e = 1e-6
        qp, qm = pd.copy(), pd.copy()
        qp[i] += e
        qm[i] -= e
        fd = (loss(qp) - loss(qm)) / (2 * e)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_adam_first_step_is_signed_learning_rate():
    rng = np.random.default_rng(2)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p1, m, v = R.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr=1e-2, eps=0.0)
    assert np.allclose(p1, p - 1e-2 * np.sign(g), rtol=0, atol=1e-15)
    # second step with the same gradient moves by the same amount again
    p2, _, _ = R.adam_step(p1, g, m, v, 2, lr=1e-2, eps=0.0)
    assert np.allclose(p2, p - 2e-2 * np.sign(g), rtol=0, atol=1e-14)


def test_features_and_block_jacobi_reduction():
    rng = np.random.default_rng(3)
    n = 37
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 8 * np.eye(n)
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    f, s, z = R.leaf_features(v, A, 0.7, 0.12)
    assert abs(s) == pytest.approx(np.linalg.norm(v))
    j = np.argmax(np.abs(v))
    assert np.angle(s) == pytest.approx(np.angle(v[j]))
    assert np.allclose(A @ z, v)
    assert np.allclose(f[0:n] ** 2 + f[64:64 + n] ** 2, np.abs(v) ** 2 / abs(s) ** 2)
    # the largest entry is real and positive in the scaled frame
    assert f[j] > 0 and f[64 + j] == pytest.approx(0.0, abs=1e-15)
    assert np.all(f[n:64] == 0) and np.all(f[64 + n:128] == 0) and np.all(f[128 + n:192] == 0)
    assert list(f[256:260]) == pytest.approx([0.7, 0.12, n / 64, 1.0]) and np.all(f[260:] == 0)
    # identity block: z = v
    f2, _, _ = R.leaf_features(v, np.eye(n), 0.7, 0.12)
    assert np.allclose(f2[128:256], f2[0:128])
    # complex scaling of v leaves the features unchanged and scales s
    a = 0.3 - 2.1j
    f3, s3, z3 = R.leaf_features(a * v, A, 0.7, 0.12)
    assert np.allclose(f3, f) and s3 == pytest.approx(a * s) and np.allclose(z3, a * z)
    # a chunk of the leaf: rows 10..29, z restricted to them
    f4, s4, z4 = R.leaf_features(v, A, 0.7, 0.12, i0=10, n=20)
    assert np.allclose(z4, z[10:30]) and abs(s4) == pytest.approx(np.linalg.norm(v[10:30]))
    assert f4[258] == pytest.approx(20 / 64)
    # a zero last layer leaves exactly the block-Jacobi correction
    h = 8
    p = (0.2 * rng.standard_normal(R.num_params(h))).astype(np.float32)
    W1, b1, W2, b2, W3, b3 = R.split(p, h)
    W3[:] = 0
    b3[:] = 0
    Y, _, _ = R.forward(p, f[None, :], h)
    assert np.array_equal(R.precond_apply(z, s, Y[0]), z)
    # the target of an exact correction e = z is zero, and of e = z + t v is t v / s
    t, m = R.leaf_targets(z, z, s)
    assert np.all(t == 0) and m.sum() == 2 * n
    t, m = R.leaf_targets(z + 0.5 * v, z, s)
    assert np.allclose(t[:n] + 1j * t[64:64 + n], 0.5 * v / s)
    # a network that outputs that target reproduces e exactly
    assert np.allclose(R.precond_apply(z, s, t), z + 0.5 * v)
    # row ranges split leaves above 64 elements into 64-element chunks
    assert R.row_ranges(np.array([0, 30, 160])) == [(0, 0, 30), (1, 30, 64), (1, 94, 64), (1, 158, 2)]
