"""FP64 numpy oracle of the surrogate MLP (test infrastructure only).

The surrogate maps [3 sweep parameters, 32-bin radial density histogram at
iteration t] to the histogram at t + 50.  Layers: Linear -> GELU (three
hidden layers of width 256) -> Linear; loss = mean squared error over all
batch x output elements; optimiser = Adam with bias correction.  GELU is the
exact form x * Phi(x) with Phi the standard normal CDF.

Parameter layout (the flat vector exchanged with the GPU library): for each
layer in order, W as [out, in] row-major, then b as [out].
"""
import math

import numpy as np
from scipy.special import erf

DIMS = (35, 256, 256, 256, 32)


def n_params(dims=DIMS):
    return sum(dims[i + 1] * dims[i] + dims[i + 1] for i in range(len(dims) - 1))


def unflatten(theta, dims=DIMS):
    out, o = [], 0
    for i in range(len(dims) - 1):
        fi, fo = dims[i], dims[i + 1]
        W = theta[o:o + fo * fi].reshape(fo, fi); o += fo * fi
        b = theta[o:o + fo]; o += fo
        out.append((W, b))
    return out


def flatten(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def forward(theta, x, dims=DIMS):
    """Returns the output and the cache needed by backward."""
    layers = unflatten(np.asarray(theta, dtype=np.float64), dims)
    h = np.asarray(x, dtype=np.float64)
    cache = []
    for li, (W, b) in enumerate(layers):
        z = h @ W.T + b
        cache.append((h, z))
        h = gelu(z) if li < len(layers) - 1 else z
    return h, cache


def loss(theta, x, y, dims=DIMS):
    yhat, _ = forward(theta, x, dims)
    return float(np.mean((yhat - np.asarray(y, dtype=np.float64)) ** 2))


def grads(theta, x, y, dims=DIMS):
    """Loss and its gradient with respect to the flat parameter vector."""
    layers = unflatten(np.asarray(theta, dtype=np.float64), dims)
    yhat, cache = forward(theta, x, dims)
    y = np.asarray(y, dtype=np.float64)
    L = float(np.mean((yhat - y) ** 2))
    g = 2.0 * (yhat - y) / yhat.size  # dL/dyhat
    out = []
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        h, z = cache[li]
        dz = g if li == len(layers) - 1 else g * gelu_grad(z)
        dW = dz.T @ h
        db = dz.sum(axis=0)
        out.append((dW, db))
        g = dz @ W
    out.reverse()
    return L, flatten(out)


class Adam:
    """Adam with bias correction (Kingma and Ba, 2015) on FP64 parameters."""

    def __init__(self, theta, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.theta = np.array(theta, dtype=np.float64)
        self.m = np.zeros_like(self.theta)
        self.v = np.zeros_like(self.theta)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps

    def step(self, g):
        self.t += 1
        self.m = self.b1 * self.m + (1.0 - self.b1) * g
        self.v = self.b2 * self.v + (1.0 - self.b2) * g * g
        mh = self.m / (1.0 - self.b1 ** self.t)
        vh = self.v / (1.0 - self.b2 ** self.t)
        self.theta = self.theta - self.lr * mh / (np.sqrt(vh) + self.eps)
        return self.theta
