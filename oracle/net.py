"""FP64 CPU oracle of the learned sinogram preconditioner (test
infrastructure: only tests, the smoke check and the benchmark's CPU leg use
it).

The preconditioner is the extension the method admits on the back
projector side: BA-GKB (Sec. 3.2, Alg. "BA-GKB") only needs B and B^T, so a
linear sinogram filter F inside it, M = B F A with M^T = A^T F^T B^T, keeps
the algorithm unchanged.  F is the frozen-mask linearisation of a small 1D
convolutional network N applied along the detector axis of every view
(every detector row in 3D):

    N(y) = W4 * relu(W3 * relu(W2 * relu(W1 * y)))

with four bias-free layers (1 -> C -> C -> C -> 1 channels, kernel K, zero
"same" padding, stride 1).  With the ReLU masks D_l = [z_l(b) > 0] of the
measured sinogram b frozen,

    F y   = W4 * D3 (W3 * D2 (W2 * D1 (W1 * y)))
    F^T z = W1^T * D1 (W2^T * D2 (W3^T * D3 (W4^T * z)))

F is linear, F b = N(b) (ReLU is positively homogeneous and D_l z_l = relu(z_l)),
and F^T is its exact transpose.

Precision points mirrored from the GPU path:
  * all weights are used rounded to bfloat16 (round to nearest even);
  * inference (F, F^T, N(b) inside GKB): activations exact (the GPU splits
    each FP32 activation into three bfloat16 terms);
  * training: the inputs of layers 2 and 3 (forward) and the gradients
    entering the transposed layers 3 and 2 and the weight gradients of
    layers 2 and 3 are rounded to bfloat16; layers 1 and 4 stay exact.
Training losses per sample, averaged over the batch: the learned filtered
back projection ||B N(b) - x||^2 / ||x||^2, or the operator objective
||B F_b (A x) - x||^2 / ||x||^2 of the filter frozen at the measured b and
applied to the noise-free data A x (what M = B F A needs); Adam with bias
correction (Kingma and Ba 2015).

Arrays: a sinogram batch is [rows, L] (rows = views (x detector rows),
L = detector columns); activations are [rows, C, L]; weights W[l] have shape
[c_out, c_in, K]; the flat weight vector concatenates W1..W4 in that order
(row-major), 2*C*K + 2*C*C*K values.
"""
from __future__ import annotations

import numpy as np


def bf16(x):
    """Round to the nearest bfloat16 (8 significant bits), ties to even."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)  # x = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(m * 256.0) / 256.0, e)


def shapes(C: int = 32, K: int = 9):
    return [(C, 1, K), (C, C, K), (C, C, K), (1, C, K)]


def split_weights(flat, C: int = 32, K: int = 9):
    out, o = [], 0
    for s in shapes(C, K):
        n = int(np.prod(s))
        out.append(np.asarray(flat[o:o + n], dtype=np.float64).reshape(s))
        o += n
    assert o == len(flat)
    return out


def conv(a, W):
    """z[r, co, p] = sum_ci sum_t W[co, ci, t] a[r, ci, p + t - K//2], zero outside [0, L)."""
    R, Ci, L = a.shape
    Co, Ci2, K = W.shape
    assert Ci == Ci2
    h = K // 2
    ap = np.zeros((R, Ci, L + 2 * h))
    ap[:, :, h:h + L] = a
    z = np.zeros((R, Co, L))
    for t in range(K):
        z += np.einsum("oc,rcl->rol", W[:, :, t], ap[:, :, t:t + L])
    return z


def conv_t(g, W):
    """Transpose of conv in its input: a[r, ci, p] = sum_co sum_t W[co, ci, t] g[r, co, p - t + K//2]."""
    R, Co, L = g.shape
    Co2, Ci, K = W.shape
    assert Co == Co2
    h = K // 2
    a = np.zeros((R, Ci, L + 2 * h))
    for t in range(K):
        a[:, :, t:t + L] += np.einsum("oc,rol->rcl", W[:, :, t], g)
    return a[:, :, h:h + L]


def wgrad(a, g, K: int = 9):
    """Gradient of <conv(a, W), g> in W: dW[co, ci, t] = sum_r sum_p g[r, co, p] a[r, ci, p + t - K//2]."""
    R, Ci, L = a.shape
    h = K // 2
    ap = np.zeros((R, Ci, L + 2 * h))
    ap[:, :, h:h + L] = a
    return np.stack([np.einsum("rol,rcl->oc", g, ap[:, :, t:t + L]) for t in range(K)], axis=2)


def forward(Ws, y, train: bool = False):
    """N(y) for y [rows, L].  Returns (out [rows, L], z list, masks list).
    train: bfloat16 rounding of the inputs of layers 2 and 3."""
    Wb = [bf16(W) for W in Ws]
    a = np.asarray(y, dtype=np.float64)[:, None, :]
    zs, masks = [], []
    for l in range(4):
        inp = bf16(a) if (train and l in (1, 2)) else a
        z = conv(inp, Wb[l])
        zs.append(z)
        if l < 3:
            m = z > 0
            masks.append(m)
            a = np.where(m, z, 0.0)
    return zs[3][:, 0, :], zs, masks


def masks_of(Ws, b):
    """Frozen ReLU masks D1..D3 of the measured sinogram b (inference precision)."""
    return forward(Ws, b)[2]


def apply_F(Ws, masks, y):
    """F y with the frozen masks."""
    Wb = [bf16(W) for W in Ws]
    a = np.asarray(y, dtype=np.float64)[:, None, :]
    for l in range(4):
        z = conv(a, Wb[l])
        a = np.where(masks[l], z, 0.0) if l < 3 else z
    return a[:, 0, :]


def apply_Ft(Ws, masks, z):
    """F^T z with the frozen masks."""
    Wb = [bf16(W) for W in Ws]
    g = np.asarray(z, dtype=np.float64)[:, None, :]
    for l in (3, 2, 1, 0):
        g = conv_t(g, Wb[l])
        if l > 0:
            g = np.where(masks[l - 1], g, 0.0)
    return g[:, 0, :]


def forward_frozen(Ws, y, masks, train: bool = False):
    """F y with given masks, in the training precision when train is set.
    Returns (out, z list, masks)."""
    Wb = [bf16(W) for W in Ws]
    a = np.asarray(y, dtype=np.float64)[:, None, :]
    zs = []
    for l in range(4):
        inp = bf16(a) if (train and l in (1, 2)) else a
        z = conv(inp, Wb[l])
        zs.append(z)
        if l < 3:
            a = np.where(masks[l], z, 0.0)
    return zs[3][:, 0, :], zs, masks


def net_grad(Ws, y, gout, train: bool = True, masks=None):
    """Gradient of <N(y), gout> in the weights (list of arrays), with the
    training rounding points when train is set; with masks given, of
    <F y, gout> for the filter frozen at those masks (masks held fixed)."""
    Wb = [bf16(W) for W in Ws]
    if masks is None:
        out, zs, masks = forward(Ws, y, train=train)
    else:
        out, zs, masks = forward_frozen(Ws, y, masks, train=train)
    acts = [np.asarray(y, dtype=np.float64)[:, None, :]]
    for l in range(3):
        acts.append(np.where(masks[l], zs[l], 0.0))
    r = bf16 if train else (lambda v: v)
    dW = [None] * 4
    g = np.asarray(gout, dtype=np.float64)[:, None, :]
    for l in (3, 2, 1, 0):
        mfma = l in (1, 2)
        inp = r(acts[l]) if mfma else acts[l]
        dW[l] = wgrad(inp, r(g) if mfma else g, Wb[l].shape[2])
        if l > 0:
            g = conv_t(r(g) if (train and l in (2, 1)) else g, Wb[l])
            g = np.where(masks[l - 1], g, 0.0)
    return out, dW


def loss_and_grad(Ws, op_B, op_Bt, bs, xs, train: bool = True):
    """Mean over the batch of ||B N(b_i) - x_i||^2 / ||x_i||^2 and its
    gradient in the weights.  bs: [batch, rows, L]; xs: [batch, n];
    op_B / op_Bt: the back projector and its transpose (flat vectors)."""
    nb = len(bs)
    total = 0.0
    grads = None
    for b, x in zip(bs, xs):
        out = forward(Ws, b, train=train)[0]
        x = np.asarray(x, dtype=np.float64).reshape(-1)
        res = np.asarray(op_B(out.reshape(-1))).reshape(-1) - x
        xx = float(x @ x)
        total += float(res @ res) / xx
        gout = np.asarray(op_Bt(res)).reshape(out.shape) * (2.0 / xx / nb)
        _, dW = net_grad(Ws, b, gout, train=train)
        grads = dW if grads is None else [g0 + g1 for g0, g1 in zip(grads, dW)]
    return total / nb, grads


def frozen_loss_and_grad(Ws, op_A, op_B, op_Bt, bs, xs, train: bool = True):
    """Operator objective of the filter GKB applies: with the masks of the
    measured b_i frozen, mean over the batch of
    ||B F_{b_i} (A x_i) - x_i||^2 / ||x_i||^2 and its gradient in the
    weights (masks held fixed).  bs: [batch, rows, L]; xs: [batch, n]."""
    nb = len(bs)
    total = 0.0
    grads = None
    for b, x in zip(bs, xs):
        x = np.asarray(x, dtype=np.float64).reshape(-1)
        masks = masks_of(Ws, b)
        y = np.asarray(op_A(x)).reshape(np.shape(b))
        out = forward_frozen(Ws, y, masks, train=train)[0]
        res = np.asarray(op_B(out.reshape(-1))).reshape(-1) - x
        xx = float(x @ x)
        total += float(res @ res) / xx
        gout = np.asarray(op_Bt(res)).reshape(out.shape) * (2.0 / xx / nb)
        _, dW = net_grad(Ws, y, gout, train=train, masks=masks)
        grads = dW if grads is None else [g0 + g1 for g0, g1 in zip(grads, dW)]
    return total / nb, grads


def adam(w, g, m, v, step: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam step (FP64) on flat arrays; returns new (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def identity_weights(C: int = 32, K: int = 9):
    """Weights with N(y) = relu(y) - relu(-y) = y: channel 0 passes y,
    channel 1 passes -y, the middle layers copy channels 0 and 1, the last
    layer subtracts them."""
    Ws = [np.zeros(s) for s in shapes(C, K)]
    h = K // 2
    Ws[0][0, 0, h], Ws[0][1, 0, h] = 1.0, -1.0
    for l in (1, 2):
        Ws[l][0, 0, h] = Ws[l][1, 1, h] = 1.0
    Ws[3][0, 0, h], Ws[3][0, 1, h] = 1.0, -1.0
    return Ws


def flatten(Ws):
    return np.concatenate([np.asarray(W, dtype=np.float64).reshape(-1) for W in Ws])
