"""CPU FP64 oracle for the learned warm start: a small multilayer perceptron
over per-node features, its mean-squared-error loss, back-propagation and the
Adam update.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only users.  The product library never imports
this module and shares no code with it.

The paper has no learned component; the network is an addition to its method.
What this module computes is fixed here, in plain definitions:

* Parameters are one flat vector holding, layer after layer, the weight matrix
  W_l (out x in, row-major) and then the bias b_l.
* Hidden layers: a_l = silu(W_l a_{l-1} + b_l) with silu(z) = z / (1 + e^-z);
  the last layer is affine (no activation).
* Loss: the mean of (y - t)^2 over all B x out entries.
* Gradients: the chain rule written out layer by layer (reverse mode).
* Adam with bias correction: m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
  p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
* Features of a node at x in the periodic unit cell around a grain of radius
  r centred at (1/2, 1/2, 1/2): the minimum-image offset d = x - c (three
  values), the signed distance |d| - r to the grain surface, and the cell
  porosity phi (Section 2 describes the cell; the choice of features is part
  of the addition).
* Network outputs (v_x, v_y, v_z, p) / (U, P) map to a solver state: v = U y
  on interior nodes, v = 0 on the grain (the no-slip condition), p = P y_3
  with its node mean removed (the pressure is fixed only up to a constant).

Everything is float64 and unblocked; numpy's matmul is the only library
primitive.  Parity pins: central finite differences of the loss, torch's
float64 autograd of the same network, closed forms of silu and of Adam's
first steps, and geometric identities of the features.
"""
from __future__ import annotations

import numpy as np

SIZES = (5, 128, 128, 128, 4)


def param_count(sizes=SIZES) -> int:
    return sum(o * i + o for i, o in zip(sizes[:-1], sizes[1:]))


def unpack(theta, sizes=SIZES):
    """Views (W_l, b_l) into the flat parameter vector."""
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (param_count(sizes),)
    out, at = [], 0
    for i, o in zip(sizes[:-1], sizes[1:]):
        W = theta[at:at + o * i].reshape(o, i)
        at += o * i
        b = theta[at:at + o]
        at += o
        out.append((W, b))
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_prime(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(theta, x, sizes=SIZES):
    """y [B][out] and the per-layer pre-activations and inputs for backward."""
    a = np.asarray(x, dtype=np.float64)
    layers = unpack(theta, sizes)
    zs, ins = [], []
    for l, (W, b) in enumerate(layers):
        ins.append(a)
        z = a @ W.T + b
        zs.append(z)
        a = silu(z) if l + 1 < len(layers) else z
    return a, (zs, ins)


def backward(theta, cache, dy, sizes=SIZES):
    """Gradient of sum(dy * y) with respect to every parameter, flat."""
    zs, ins = cache
    layers = unpack(theta, sizes)
    grads = [None] * len(layers)
    d = np.asarray(dy, dtype=np.float64)  # dL/dz of the last (affine) layer
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        grads[l] = (d.T @ ins[l], d.sum(axis=0))
        if l > 0:
            d = (d @ W) * silu_prime(zs[l - 1])
    return np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])


def mse(y, t):
    """Loss and its gradient with respect to y."""
    y = np.asarray(y, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    e = y - t
    return float(np.mean(e * e)), 2.0 * e / e.size


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def features(pos, r, phi):
    """pos [n][3] in the unit cell -> [n][5] (offset from the grain centre by
    minimum image, signed distance to the grain surface, porosity)."""
    pos = np.asarray(pos, dtype=np.float64)
    d = pos - 0.5
    d = d - np.round(d)
    dist = np.sqrt((d * d).sum(axis=1))
    return np.column_stack([d, dist - r, np.full(len(pos), float(phi))])


def to_state(y, n_int, U, P):
    """Network outputs [n][4] -> (v [3][n], p [n]) as described above."""
    y = np.asarray(y, dtype=np.float64)
    n = len(y)
    v = np.zeros((3, n))
    v[:, :n_int] = U * y[:n_int, :3].T
    p = P * y[:, 3]
    return v, p - p.mean()
