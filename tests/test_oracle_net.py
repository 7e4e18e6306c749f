"""Pins of the learned-preconditioner oracle (oracle/net.py) against facts
that do not depend on it: bfloat16 rounding cases and PyTorch's own
bfloat16 conversion, NumPy's correlate, the transposition identities of
convolution, positive homogeneity (F b = N(b)), a closed-form identity
network, central finite differences of the training loss, and the first
Adam step's closed form."""
import numpy as np
import pytest

from oracle import net


def test_bf16_rounding_cases():
    assert net.bf16(1.0 + 2.0 ** -8) == 1.0  # tie to even
    assert net.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6  # tie to even (upwards)
    assert net.bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert net.bf16(-3.0) == -3.0 and net.bf16(0.0) == 0.0
    torch = pytest.importorskip("torch")
    r = np.random.default_rng(0)
    x = (r.standard_normal(10000) * np.exp(r.uniform(-20, 20, 10000))).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(net.bf16(x.astype(np.float64)), ref)


def test_conv_is_correlation_with_zero_padding():
    r = np.random.default_rng(1)
    a = r.standard_normal(23)
    w = r.standard_normal(9)
    z = net.conv(a[None, None, :], w[None, None, :])[0, 0]
    ref = np.correlate(np.concatenate([np.zeros(4), a, np.zeros(4)]), w, mode="valid")
    assert np.allclose(z, ref, rtol=0, atol=1e-13)


def test_transposition_identities():
    r = np.random.default_rng(2)
    a = r.standard_normal((3, 5, 17))
    W = r.standard_normal((4, 5, 9))
    g = r.standard_normal((3, 4, 17))
    lhs = float(np.sum(net.conv(a, W) * g))
    assert abs(lhs - float(np.sum(a * net.conv_t(g, W)))) <= 1e-12 * abs(lhs)
    assert abs(lhs - float(np.sum(W * net.wgrad(a, g)))) <= 1e-12 * abs(lhs)


def random_weights(seed, C=32, K=9):
    r = np.random.default_rng(seed)
    return [r.standard_normal(s) * np.sqrt(2.0 / (s[1] * s[2])) for s in net.shapes(C, K)]


def test_frozen_linearisation():
    Ws = random_weights(3)
    r = np.random.default_rng(4)
    b = r.standard_normal((6, 40))
    masks = net.masks_of(Ws, b)
    Nb = net.forward(Ws, b)[0]
    Fb = net.apply_F(Ws, masks, b)
    assert np.allclose(Fb, Nb, rtol=0, atol=1e-13 * np.abs(Nb).max())
    y = r.standard_normal(b.shape)
    z = r.standard_normal(b.shape)
    lhs = float(np.sum(net.apply_F(Ws, masks, y) * z))
    rhs = float(np.sum(y * net.apply_Ft(Ws, masks, z)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # linear in y
    Fy, Fz = net.apply_F(Ws, masks, y), net.apply_F(Ws, masks, z)
    assert np.allclose(net.apply_F(Ws, masks, 2 * y - 3 * z), 2 * Fy - 3 * Fz, atol=1e-12)


def test_identity_network():
    Ws = net.identity_weights()
    r = np.random.default_rng(5)
    y = r.standard_normal((4, 31))
    assert np.array_equal(net.forward(Ws, y)[0], y)
    masks = net.masks_of(Ws, y)
    z = r.standard_normal(y.shape)
    assert np.array_equal(net.apply_F(Ws, masks, z), z)
    assert np.array_equal(net.apply_Ft(Ws, masks, z), z)


def test_loss_gradient_against_finite_differences():
    C, K, L, rows = 2, 3, 16, 3
    r = np.random.default_rng(6)
    Ws = [r.standard_normal(s) for s in net.shapes(C, K)]
    # the weights enter through bfloat16; use bfloat16 values so that the
    # perturbed weights are the only change (exact arithmetic otherwise)
    Ws = [net.bf16(W) for W in Ws]
    n = 10
    Bm = r.standard_normal((n, rows * L))
    bs = r.standard_normal((2, rows, L))
    xs = r.standard_normal((2, n))
    opB = lambda v: Bm @ v  # noqa: E731
    opBt = lambda v: Bm.T @ v  # noqa: E731

    def loss(Wlist):
        # exact-precision loss (train=False); weights are not re-rounded here
        tot = 0.0
        for b, x in zip(bs, xs):
            a = b[:, None, :]
            for l in range(4):
                z = net.conv(a, Wlist[l])
                a = np.maximum(z, 0.0) if l < 3 else z
            res = Bm @ a[:, 0, :].reshape(-1) - x
            tot += float(res @ res) / float(x @ x)
        return tot / len(bs)

    val, grads = net.loss_and_grad(Ws, opB, opBt, bs, xs, train=False)
    assert val == pytest.approx(loss(Ws), rel=1e-12)
    h = 1e-6
    for l in range(4):
        for idx in np.ndindex(*Ws[l].shape):
            Wp = [W.copy() for W in Ws]
            Wm = [W.copy() for W in Ws]
            Wp[l][idx] += h
            Wm[l][idx] -= h
            fd = (loss(Wp) - loss(Wm)) / (2 * h)
            assert abs(fd - grads[l][idx]) <= 1e-6 * max(1.0, abs(fd)), (l, idx)


def test_adam_first_step_closed_form():
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    w1, m, v = net.adam(w, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    # m_hat = g, v_hat = g^2: the first step moves each weight by lr * g / (|g| + eps)
    assert np.allclose(w1, w - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_training_rounding_points_change_little():
    # the bfloat16 rounding of the training path perturbs the gradient at the
    # level of bfloat16's precision, not more
    Ws = random_weights(7)
    r = np.random.default_rng(8)
    y = r.standard_normal((4, 33))
    gout = r.standard_normal((4, 33))
    _, g_exact = net.net_grad(Ws, y, gout, train=False)
    _, g_train = net.net_grad(Ws, y, gout, train=True)
    for ge, gt in zip(g_exact, g_train):
        assert np.linalg.norm(gt - ge) <= 0.05 * np.linalg.norm(ge)


def test_frozen_objective_gradient_against_finite_differences():
    # masks held fixed: the objective is a smooth function of the weights
    C, K, L, rows = 2, 3, 16, 3
    r = np.random.default_rng(12)
    Ws = [net.bf16(r.standard_normal(s)) for s in net.shapes(C, K)]
    n = 10
    Am = r.standard_normal((rows * L, n))
    Bm = r.standard_normal((n, rows * L))
    xs = r.standard_normal((2, n))
    bs = [(Am @ x).reshape(rows, L) + 0.1 * r.standard_normal((rows, L)) for x in xs]
    val, grads = net.frozen_loss_and_grad(Ws, lambda v: Am @ v, lambda v: Bm @ v, lambda v: Bm.T @ v, bs, xs,
                                          train=False)
    masks = [net.masks_of(Ws, b) for b in bs]

    def loss(Wlist):
        # exact arithmetic (the oracle's weights enter through bfloat16, which
        # would swallow the finite-difference step)
        tot = 0.0
        for b, x, mk in zip(bs, xs, masks):
            a = (Am @ x).reshape(rows, L)[:, None, :]
            for l in range(4):
                z = net.conv(a, Wlist[l])
                a = np.where(mk[l], z, 0.0) if l < 3 else z
            res = Bm @ a[:, 0, :].reshape(-1) - x
            tot += float(res @ res) / float(x @ x)
        return tot / len(xs)

    assert val == pytest.approx(loss(Ws), rel=1e-12)
    h = 1e-6
    for l in range(4):
        for idx in np.ndindex(*Ws[l].shape):
            Wp = [W.copy() for W in Ws]
            Wm = [W.copy() for W in Ws]
            Wp[l][idx] += h
            Wm[l][idx] -= h
            fd = (loss(Wp) - loss(Wm)) / (2 * h)
            assert abs(fd - grads[l][idx]) <= 1e-6 * max(1.0, abs(fd)), (l, idx)
