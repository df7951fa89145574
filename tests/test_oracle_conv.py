"""Pins of the FP64 conv-net reference (learned local solve)."""
import numpy as np

from oracle.conv import Adam, ConvNet, conv3d, conv3d_backward


def test_forward_matches_direct_sum():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((2, 3, 4, 5, 6))
    W = rng.standard_normal((4, 3, 3, 3, 3))
    b = rng.standard_normal(4)
    Y = conv3d(X, W, b)
    for (bb, o, z, y, x) in [(0, 0, 0, 0, 0), (1, 3, 3, 4, 5), (0, 2, 1, 2, 3), (1, 1, 3, 0, 2)]:
        s = b[o]
        for i in range(3):
            for dz in range(3):
                for dy in range(3):
                    for dx in range(3):
                        zz, yy, xx = z + dz - 1, y + dy - 1, x + dx - 1
                        if 0 <= zz < 4 and 0 <= yy < 5 and 0 <= xx < 6:
                            s += W[o, i, dz, dy, dx] * X[bb, i, zz, yy, xx]
        assert abs(Y[bb, o, z, y, x] - s) < 1e-12


def test_gradients_against_finite_differences():
    rng = np.random.default_rng(1)
    net = ConvNet([2, 3, 2], seed=3)
    net.b = [rng.standard_normal(3) * 0.1, rng.standard_normal(2) * 0.1]
    X = rng.standard_normal((2, 2, 4, 4, 4))
    Y = rng.standard_normal((2, 2, 4, 4, 4))
    mask = (rng.random((1, 2, 4, 4, 4)) > 0.3).astype(float)
    loss, gW, gb, gX = net.loss_and_grads(X, Y, mask)

    def L():
        out = net.forward(X)
        d = (out - Y) * mask
        return 0.5 * np.sum(d * d) / X.shape[0]

    eps = 1e-6
    for l in range(2):
        for idx in [(0, 0, 0, 0, 0), (1, 1, 2, 1, 0), (0, 1, 1, 1, 1)]:
            idx = tuple(min(k, s - 1) for k, s in zip(idx, net.W[l].shape))
            w0 = net.W[l][idx]
            net.W[l][idx] = w0 + eps; lp = L()
            net.W[l][idx] = w0 - eps; lm = L()
            net.W[l][idx] = w0
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - gW[l][idx]) <= 1e-7 * max(1.0, abs(fd)), (l, idx)
        for o in range(net.b[l].size):
            b0 = net.b[l][o]
            net.b[l][o] = b0 + eps; lp = L()
            net.b[l][o] = b0 - eps; lm = L()
            net.b[l][o] = b0
            assert abs((lp - lm) / (2 * eps) - gb[l][o]) <= 1e-7 * max(1.0, abs(gb[l][o]))
    for idx in [(0, 0, 0, 0, 0), (1, 1, 3, 2, 1)]:
        x0 = X[idx]
        X[idx] = x0 + eps; lp = L()
        X[idx] = x0 - eps; lm = L()
        X[idx] = x0
        assert abs((lp - lm) / (2 * eps) - gX[idx]) <= 1e-7 * max(1.0, abs(gX[idx]))


def test_adam_first_step_is_signed_lr():
    """After one step with bias correction, each weight moves by lr * g/(|g|+eps')."""
    p = [np.array([1.0, -2.0, 0.5])]
    g = [np.array([0.3, -4.0, 1e-3])]
    opt = Adam(p, lr=0.01)
    out = opt.step(p, g)[0]
    assert np.allclose(out, p[0] - 0.01 * np.sign(g[0]), rtol=0, atol=1e-7)


def test_adam_three_steps_by_hand():
    """Three steps with b1 != b2 and changing gradients, against values worked
    out by hand in exact fractions (b1 = 1/2, b2 = 3/4, lr = 1, eps = 0,
    gradients 1, -1, 2 from w = 0):
      t=1: m = 1/2,   v = 1/4,     m^ = 1,    v^ = 1       -> w = -1
      t=2: m = -1/4,  v = 7/16,    m^ = -1/3, v^ = 1       -> w = -2/3
      t=3: m = 7/8,   v = 85/64,   m^ = 1,    v^ = 85/37   -> w = -2/3 - sqrt(37/85)
    Swapping b1 and b2 changes the second step (m^ = -1/7)."""
    w = [np.array([0.0])]
    opt = Adam(w, lr=1.0, b1=0.5, b2=0.75, eps=0.0)
    expect = [-1.0, -2.0 / 3.0, -2.0 / 3.0 - np.sqrt(37.0 / 85.0)]
    for g, e in zip([1.0, -1.0, 2.0], expect):
        w = opt.step(w, [np.array([g])])
        assert abs(w[0][0] - e) < 1e-15, (w[0][0], e)
    assert np.allclose(opt.m[0], [7.0 / 8.0], rtol=0, atol=1e-16)
    assert np.allclose(opt.v[0], [85.0 / 64.0], rtol=0, atol=1e-16)


def test_adam_moments_closed_form():
    """Over five steps with random gradients, the moments equal their closed
    forms m_t = (1-b1) sum_k b1^(t-k) g_k, v_t = (1-b2) sum_k b2^(t-k) g_k^2,
    and the update uses the bias corrections 1 - b^t (default betas)."""
    rng = np.random.default_rng(4)
    G = rng.standard_normal((5, 7))
    p0 = rng.standard_normal(7)
    b1, b2, lr, eps = 0.9, 0.999, 3e-3, 1e-8
    opt = Adam([p0], lr=lr)
    p = [p0.copy()]
    for t in range(1, 6):
        prev = p[0]
        p = opt.step(p, [G[t - 1]])
        k = np.arange(1, t + 1)
        m = (1 - b1) * np.sum(b1 ** (t - k)[:, None] * G[:t], 0)
        v = (1 - b2) * np.sum(b2 ** (t - k)[:, None] * G[:t] ** 2, 0)
        assert np.allclose(opt.m[0], m, rtol=1e-14, atol=0)
        assert np.allclose(opt.v[0], v, rtol=1e-14, atol=0)
        step = lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
        assert np.allclose(prev - p[0], step, rtol=1e-12, atol=1e-18)
