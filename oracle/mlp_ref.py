"""Oracle of the learned per-leaf preconditioner (TEST INFRASTRUCTURE ONLY).

Plain numpy, FP64.  Nothing in the product path imports this module; only
tests, the smoke check and the benchmark's CPU leg do.  It shares no code
with the HIP library.

The paper solves its Burton-Miller systems with unpreconditioned GMRES
(Section 5); the preconditioner below is an addition on top of the
block-Jacobi one (inverse of each leaf's self-interaction block).  A row R
is a chunk of at most 64 consecutive elements of a leaf L of the octree (the
whole leaf when n_L <= 64).  For a residual v:

    z    = A_LL^-1 v_L, restricted to the row: z_R        (block Jacobi)
    s_R  = |v_R| v_j / |v_j|, j the row's largest entry (first on ties)
    f_R  = [Re, Im of v_R / s_R, Re, Im of z_R / s_R]   (each padded to 64)
           ++ [w_L / lambda, h_max / lambda, n_R / 64, 1, 0 ... 0]   (272)
    c_R  = W3^T relu(W2^T relu(W1^T f_R + b1) + b2) + b3             (128)
    M(v)_R = z_R + s_R (c_R[:64] + i c_R[64:])[:n_R]

so that M(a v) = a M(v) for every complex a.  Training minimises the
masked mean squared error between c_R and the normalised correction
(e_R - z_R)/s_R of pairs (r, e = A^-1 r).

Parameters are one flat array: W1 (272 x h, input-major), b1 (h), W2
(h x h), b2 (h), W3 (h x 128), b3 (128).  Inference uses bfloat16 copies of
W1, W2, W3 (round to nearest, ties to even) and rounds each layer's input
the same way (a bfloat16 product), with wider accumulation; the biases and
the ReLU keep full precision.

Pins (tests/test_oracle_pins_mlp.py): the backward pass against central
differences of the loss, bfloat16 rounding against exactly representable
cases, a hand-evaluated width-2 network, and the block-Jacobi reduction when
the last layer is zero.
"""
from __future__ import annotations

import numpy as np

MLP_IN, MLP_OUT, LEAF = 272, 128, 64

__all__ = ["MLP_IN", "MLP_OUT", "LEAF", "num_params", "split", "bf16_round", "row_scale", "leaf_features", "row_ranges",
           "leaf_targets", "forward", "loss_and_gradient", "adam_step", "precond_apply"]


def num_params(h: int) -> int:
    return MLP_IN * h + h + h * h + h + h * MLP_OUT + MLP_OUT


def split(p: np.ndarray, h: int):
    """Flat parameters -> (W1, b1, W2, b2, W3, b3) views."""
    shapes = [(MLP_IN, h), (h,), (h, h), (h,), (h, MLP_OUT), (MLP_OUT,)]
    out, o = [], 0
    for s in shapes:
        n = int(np.prod(s))
        out.append(p[o:o + n].reshape(s))
        o += n
    assert o == p.size
    return out


def bf16_round(x) -> np.ndarray:
    """float32 -> nearest bfloat16 (ties to even), returned as float32.
    NaN stays NaN; values past the largest bfloat16 round to infinity."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    nan = np.isnan(a)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).copy()
    out[nan] = np.nan
    return out


def row_scale(vR: np.ndarray) -> complex:
    """s_R = |v_R| times the unit phase of the row's largest entry (the first
    one on ties); 0 for v_R = 0.  Dividing by s makes the features, and so
    the preconditioner, equivariant under complex scaling of v."""
    nv = float(np.linalg.norm(vR))
    if nv == 0:
        return 0j
    j = int(np.argmax(np.abs(vR) ** 2))
    return nv * vR[j] / abs(vR[j])


def leaf_features(vL: np.ndarray, A_LL: np.ndarray, width_lam: float, hmax_lam: float, i0: int = 0, n: int = None):
    """Features (272,), scale s_R and z_R of the row R = elements
    i0 .. i0+n-1 of leaf L (the whole leaf by default; n <= 64).  z is the
    block-Jacobi correction of the whole leaf restricted to the row."""
    nL = vL.size
    n = nL - i0 if n is None else n
    assert 0 < n <= LEAF and i0 + n <= nL and A_LL.shape == (nL, nL)
    z = np.linalg.solve(A_LL, vL)[i0:i0 + n]
    vR = vL[i0:i0 + n]
    s = row_scale(vR)
    inv = 1.0 / s if s != 0 else 0.0
    f = np.zeros(MLP_IN)
    f[0:n] = (vR * inv).real
    f[64:64 + n] = (vR * inv).imag
    f[128:128 + n] = (z * inv).real
    f[192:192 + n] = (z * inv).imag
    f[256:260] = [width_lam, hmax_lam, n / 64.0, 1.0]
    return f, s, z


def row_ranges(leaf_off: np.ndarray):
    """(leaf, first tree position, count) of every row: leaves split into
    chunks of at most 64 consecutive elements, in leaf order."""
    out = []
    for L in range(len(leaf_off) - 1):
        for e in range(int(leaf_off[L]), int(leaf_off[L + 1]), LEAF):
            out.append((L, e, min(LEAF, int(leaf_off[L + 1]) - e)))
    return out


def leaf_targets(eR: np.ndarray, zR: np.ndarray, s: complex):
    """Target (128,) and mask (128,) of one row: (e_R - z_R) / s_R."""
    n = eR.size
    t = np.zeros(MLP_OUT)
    m = np.zeros(MLP_OUT)
    d = (eR - zR) * (1.0 / s if s != 0 else 0.0)
    t[:n], t[64:64 + n] = d.real, d.imag
    m[:n] = m[64:64 + n] = 1.0
    return t, m


def _weights(p, h, bf16):
    W1, b1, W2, b2, W3, b3 = (np.asarray(q, dtype=np.float64) for q in split(np.asarray(p, np.float32), h))
    if bf16:
        W1, W2, W3 = (bf16_round(W).astype(np.float64) for W in (W1, W2, W3))
    return W1, b1, W2, b2, W3, b3


def forward(p: np.ndarray, X: np.ndarray, h: int, bf16: bool = True):
    """Y (rows x 128) and the hidden activations (H1, H2).  With bf16 each
    layer is a bfloat16 product: its input (X, H1, H2) and its weights are
    rounded to bfloat16 and multiplied exactly (wider accumulation); the
    bias, the ReLU and the returned H1, H2 stay unrounded."""
    W1, b1, W2, b2, W3, b3 = _weights(p, h, bf16)
    X = np.asarray(X, dtype=np.float64)
    rnd = (lambda A: bf16_round(A).astype(np.float64)) if bf16 else (lambda A: A)
    H1 = np.maximum(rnd(X) @ W1 + b1, 0.0)
    H2 = np.maximum(rnd(H1) @ W2 + b2, 0.0)
    return rnd(H2) @ W3 + b3, H1, H2


def loss_and_gradient(p: np.ndarray, X, T, M, h: int, bf16: bool = True):
    """L = sum (M (Y - T))^2 / (rows * 128) and dL/dp (flat, FP64).  With
    bf16 the forward pass and the products with the weights use the rounded
    weights; the derivative treats the rounding as the identity."""
    W1, b1, W2, b2, W3, b3 = _weights(p, h, bf16)
    X = np.asarray(X, dtype=np.float64)
    Y, H1, H2 = forward(p, X, h, bf16)
    cnt = X.shape[0] * MLP_OUT
    D = np.asarray(M, np.float64) * (Y - np.asarray(T, np.float64))
    L = float(np.sum(D * D) / cnt)
    dY = 2.0 * np.asarray(M, np.float64) * D / cnt
    gW3, gb3 = H2.T @ dY, dY.sum(0)
    dH2 = (dY @ W3.T) * (H2 > 0)
    gW2, gb2 = H1.T @ dH2, dH2.sum(0)
    dH1 = (dH2 @ W2.T) * (H1 > 0)
    gW1, gb1 = X.T @ dH1, dH1.sum(0)
    g = np.concatenate([q.ravel() for q in (gW1, gb1, gW2, gb2, gW3, gb3)])
    return L, g


def adam_step(p, g, m, v, t: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, Algorithm 1) at step t >= 1; returns
    the new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def precond_apply(zR: np.ndarray, s: complex, yR: np.ndarray):
    """M(v)_R = z_R + s_R c_R from the network output row y_R (128,)."""
    n = zR.size
    return zR + s * (yR[:n] + 1j * yR[64:64 + n])
