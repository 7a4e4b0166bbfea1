"""Learned initial density: a small periodic 3D convolutional network (FP64 oracle).

TEST INFRASTRUCTURE ONLY (see the package header).  The network maps the
superposition-of-atoms start density to a correction:
  x   = n0 / nbar,  nbar = N_e / Omega
  h1  = silu(conv1(x)),  h2 = silu(conv2(h1)),  h3 = silu(conv3(h2)),  y = conv4(h3)
  dn  = nbar * (y - mean(y))                  (integrates to zero)
  n   = max(n0 + dn, 0) rescaled so that (Omega/N) sum n = N_e
conv: 3x3x3 cross-correlation with circular (periodic) padding,
  out[co, r] = b[co] + sum_ci sum_d W[co, ci, d] x[ci, (r + d) mod S],
  d in {-1, 0, 1}^3, W stored as (co, ci, 3, 3, 3) with index d + 1;
silu(a) = a / (1 + exp(-a)).  Channels 1 -> 16 -> 16 -> 16 -> 1.
Training loss per sample (target t = (n_conv - n0) / nbar):
  L = mean_r (y - mean(y) - t)^2, averaged over the batch; Adam on the weights.
The steps are written out plainly with numpy.roll for the periodic shifts;
gradients are pinned by central finite differences in the tests.
"""
from __future__ import annotations

import numpy as np

CHANNELS = (1, 16, 16, 16, 1)
OFFSETS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def init_params(seed: int = 501):
    """Seeded initial weights (drawn by the shared input generator)."""
    from workloads import net_init_params
    return net_init_params(seed)


def shifted(x, d):
    """y[..., r] = x[..., (r + d) mod S] over the last three axes."""
    return np.roll(x, shift=(-d[0], -d[1], -d[2]), axis=(-3, -2, -1))


def conv(x, W, b):
    """x: (ci, S0, S1, S2) -> (co, S0, S1, S2)."""
    co, ci = W.shape[0], W.shape[1]
    out = np.zeros((co,) + x.shape[1:])
    for d in OFFSETS:
        xs = shifted(x, d)
        Wd = W[:, :, d[0] + 1, d[1] + 1, d[2] + 1]          # (co, ci)
        out += np.tensordot(Wd, xs, axes=(1, 0))
    return out + b[:, None, None, None]


def conv_backward(x, W, dout):
    """Gradients of sum(dout * conv(x, W, b)) wrt x, W and b."""
    co, ci = W.shape[0], W.shape[1]
    dx = np.zeros_like(x)
    dW = np.zeros_like(W)
    for d in OFFSETS:
        xs = shifted(x, d)
        dW[:, :, d[0] + 1, d[1] + 1, d[2] + 1] = np.tensordot(dout, xs, axes=([1, 2, 3], [1, 2, 3]))
        Wd = W[:, :, d[0] + 1, d[1] + 1, d[2] + 1]
        # out[r] uses x[r + d]  =>  dx[s] += W^T dout[s - d]
        dx += np.tensordot(Wd, shifted(dout, (-d[0], -d[1], -d[2])), axes=(0, 0))
    db = dout.sum(axis=(1, 2, 3))
    return dx, dW, db


def sigmoid(a):
    return 1.0 / (1.0 + np.exp(-a))


def silu(a):
    return a * sigmoid(a)


def silu_grad(a):
    s = sigmoid(a)
    return s * (1.0 + a * (1.0 - s))


def forward(params, x):
    """Returns y and the cache (inputs and pre-activations of every layer)."""
    cache = []
    h = x
    for l, (W, b) in enumerate(params):
        a = conv(h, W, b)
        cache.append((h, a))
        h = silu(a) if l < 3 else a
    return h, cache


def loss_and_grads(params, x, t):
    """Loss mean((y - mean(y) - t)^2) and its gradients for one sample."""
    y, cache = forward(params, x)
    e = y[0] - y[0].mean() - t
    N = e.size
    L = float(np.mean(e * e))
    dy = (2.0 / N) * (e - e.mean())
    g = dy[None]
    grads = [None] * 4
    for l in range(3, -1, -1):
        h, a = cache[l]
        if l < 3:
            g = g * silu_grad(a)
        dx, dW, db = conv_backward(h, params[l][0], g)
        grads[l] = (dW, db)
        g = dx
    return L, grads


def predict_density(params, n0, n_electrons, omega):
    """Learned start density (inference, with the safety post-processing)."""
    nbar = n_electrons / omega
    y, _ = forward(params, (n0 / nbar)[None])
    dn = nbar * (y[0] - y[0].mean())
    n = np.maximum(n0 + dn, 0.0)
    return n * (n_electrons / (omega / n.size * n.sum()))


class Adam:
    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        self.v = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        out = []
        for l, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
            new = []
            for j, (p, g) in enumerate(((W, gW), (b, gb))):
                m = self.b1 * self.m[l][j] + (1 - self.b1) * g
                v = self.b2 * self.v[l][j] + (1 - self.b2) * g * g
                self.m[l] = tuple(m if jj == j else self.m[l][jj] for jj in range(2))
                self.v[l] = tuple(v if jj == j else self.v[l][jj] for jj in range(2))
                mh = m / (1 - self.b1 ** self.t)
                vh = v / (1 - self.b2 ** self.t)
                new.append(p - self.lr * mh / (np.sqrt(vh) + self.eps))
            out.append(tuple(new))
        return out
