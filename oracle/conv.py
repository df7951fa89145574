"""Dense FP64 3-D convolution network: forward, backward, loss and Adam (CPU).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The learned local solve replaces A_i^{-1} in eq. (2.2) on interior subdomains
by a small network N; FGMRES tolerates the resulting variable preconditioner.
The network is plain:

    layer l:  Y = conv3x3x3(X, W_l) + b_l  (zero padding 1, stride 1),
              ReLU after every layer but the last,
    loss:     L = 1/(2 B) * sum_b || mask * (N(x_b) - y_b) ||^2,
    Adam:     m = b1 m + (1-b1) g,  v = b2 v + (1-b2) g^2,
              w -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Shapes: X[B, C, D, H, W]; W_l[C_out, C_in, 3, 3, 3]; b_l[C_out].

Pins (``tests/test_oracle_conv.py``): forward against a direct sum over
taps for single entries; every gradient against central finite differences.
"""
from __future__ import annotations

import numpy as np

TAPS = [(dz, dy, dx) for dz in range(3) for dy in range(3) for dx in range(3)]


def conv3d(X, W, b):
    """Y[b, o, z, y, x] = b[o] + sum_{i, t} W[o, i, t] X[b, i, (z, y, x) + t - 1]."""
    B, C, D, H, Wd = X.shape
    Xp = np.zeros((B, C, D + 2, H + 2, Wd + 2))
    Xp[:, :, 1:-1, 1:-1, 1:-1] = X
    Y = np.zeros((B, W.shape[0], D, H, Wd)) + b[None, :, None, None, None]
    for dz, dy, dx in TAPS:
        Xs = Xp[:, :, dz:dz + D, dy:dy + H, dx:dx + Wd]
        Y += np.einsum("oi,bizyx->bozyx", W[:, :, dz, dy, dx], Xs)
    return Y


def conv3d_backward(X, W, dY):
    """Gradients (dX, dW, db) of conv3d for an upstream gradient dY."""
    B, C, D, H, Wd = X.shape
    Xp = np.zeros((B, C, D + 2, H + 2, Wd + 2))
    Xp[:, :, 1:-1, 1:-1, 1:-1] = X
    dXp = np.zeros_like(Xp)
    dW = np.zeros_like(W)
    for dz, dy, dx in TAPS:
        Xs = Xp[:, :, dz:dz + D, dy:dy + H, dx:dx + Wd]
        dW[:, :, dz, dy, dx] = np.einsum("bozyx,bizyx->oi", dY, Xs)
        dXp[:, :, dz:dz + D, dy:dy + H, dx:dx + Wd] += np.einsum(
            "oi,bozyx->bizyx", W[:, :, dz, dy, dx], dY)
    db = dY.sum(axis=(0, 2, 3, 4))
    return dXp[:, :, 1:-1, 1:-1, 1:-1], dW, db


class ConvNet:
    """Stack of conv3x3x3 layers with ReLU between them."""

    def __init__(self, channels, seed=0, weights=None):
        self.channels = list(channels)
        if weights is not None:
            self.W = [np.array(w, dtype=np.float64) for w in weights[0]]
            self.b = [np.array(v, dtype=np.float64) for v in weights[1]]
        else:
            rng = np.random.default_rng(seed)
            self.W, self.b = [], []
            for cin, cout in zip(self.channels[:-1], self.channels[1:]):
                scale = np.sqrt(2.0 / (27 * cin))
                self.W.append(rng.standard_normal((cout, cin, 3, 3, 3)) * scale)
                self.b.append(np.zeros(cout))

    def forward(self, X, keep=False, act_round=None):
        """act_round: optional map applied to every layer's output (after the
        ReLU), the storage format of a network that keeps its activations in
        a narrower type; None keeps them exact."""
        acts = [X]
        h = X
        L = len(self.W)
        for l in range(L):
            h = conv3d(h, self.W[l], self.b[l])
            if l < L - 1:
                h = np.maximum(h, 0.0)
            if act_round is not None:
                h = act_round(h)
            acts.append(h)
        return (h, acts) if keep else h

    def loss_and_grads(self, X, Y, mask, act_round=None):
        """Loss and exact gradients of the network as evaluated, i.e. with
        the activations as act_round leaves them (straight through the
        rounding, which is how a network storing rounded activations trains)."""
        out, acts = self.forward(X, keep=True, act_round=act_round)
        B = X.shape[0]
        diff = (out - Y) * mask
        loss = 0.5 * float(np.sum(diff * diff)) / B
        g = diff * mask / B
        gW = [None] * len(self.W)
        gb = [None] * len(self.W)
        for l in range(len(self.W) - 1, -1, -1):
            if l < len(self.W) - 1:
                g = g * (acts[l + 1] > 0.0)
            dX, gW[l], gb[l] = conv3d_backward(acts[l], self.W[l], g)
            g = dX
        return loss, gW, gb, g


class Adam:
    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [np.zeros_like(p) for p in params]
        self.v = [np.zeros_like(p) for p in params]
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        out = []
        for k, (p, g) in enumerate(zip(params, grads)):
            self.m[k] = self.b1 * self.m[k] + (1 - self.b1) * g
            self.v[k] = self.b2 * self.v[k] + (1 - self.b2) * g * g
            mh = self.m[k] / (1 - self.b1 ** self.t)
            vh = self.v[k] / (1 - self.b2 ** self.t)
            out.append(p - self.lr * mh / (np.sqrt(vh) + self.eps))
        return out
