"""Reference MLP for the learned continued-fraction terminator -- TEST INFRASTRUCTURE ONLY.

The network is not in the paper; it extends the Haydock recursion (section 3.2): from the
first m = 32 coefficient pairs it predicts the next 224, so that the continued fraction
(eq. loss.fcn with G = [w - H]^-1) can be evaluated to depth 256 from 32 H*v.

Encoding, per sequence (a_0.., b_1..):
  c = mean(a_16..a_31), s = mean(b_17..b_32)            (the tail of the known part)
  input  x = [(a_n - c)/s for n < 32] + [b_{n+1}/s for n < 32]                    (64)
  output y = [(a_n - c)/s for 32 <= n < 256] + [log(b_{n+1}/s) for 32 <= n < 256]  (448)
so b stays positive after decoding.

Network 64 -> 256 -> 256 -> 256 -> 448, ReLU on the hidden layers, mean-squared error with
an optional weight per output position, Adam (Kingma & Ba) with beta1 = 0.9, beta2 = 0.999,
eps = 1e-8.  Parameters are packed
[W1 (64x256), b1, W2 (256x256), b2, W3 (256x256), b3, W4 (256x448), b4], each W stored
[in][out] so that a layer computes x W + b.  FP64 throughout.
"""
from __future__ import annotations

import numpy as np

M_IN = 32
N_OUT = 224
SIZES = [64, 256, 256, 256, 448]
BETA1, BETA2, ADAM_EPS = 0.9, 0.999, 1e-8


def layer_shapes():
    return [(SIZES[i], SIZES[i + 1]) for i in range(len(SIZES) - 1)]


def n_params():
    return sum(i * o + o for i, o in layer_shapes())


def unpack(p):
    out, off = [], 0
    for i, o in layer_shapes():
        w = p[off:off + i * o].reshape(i, o)
        off += i * o
        b = p[off:off + o]
        off += o
        out.append((w, b))
    return out


def init_params(rng):
    """He-normal weights, zero biases (drawn by the caller's generator)."""
    parts = []
    for i, o in layer_shapes():
        parts.append(rng.standard_normal(i * o) * np.sqrt(2.0 / i))
        parts.append(np.zeros(o))
    return np.concatenate(parts)


def encode(a, b):
    """Features and targets from coefficient arrays a[.., >=256], b[.., >=256] (b[j] = b_{j+1})."""
    a = np.atleast_2d(a)
    b = np.atleast_2d(b)
    c = a[:, 16:32].mean(axis=1, keepdims=True)
    s = b[:, 16:32].mean(axis=1, keepdims=True)
    x = np.concatenate([(a[:, :M_IN] - c) / s, b[:, :M_IN] / s], axis=1)
    t = None
    if a.shape[1] >= M_IN + N_OUT:
        t = np.concatenate([(a[:, M_IN:M_IN + N_OUT] - c) / s,
                            np.log(b[:, M_IN:M_IN + N_OUT] / s)], axis=1)
    return x, t, c[:, 0], s[:, 0]


def decode(y, a_known, b_known, c, s):
    """Extended coefficients: the known 32 pairs followed by the 224 predicted ones."""
    a_pred = y[:, :N_OUT] * s[:, None] + c[:, None]
    b_pred = np.exp(y[:, N_OUT:]) * s[:, None]
    return (np.concatenate([a_known[:, :M_IN], a_pred], axis=1),
            np.concatenate([b_known[:, :M_IN], b_pred], axis=1))


def forward(p, x):
    """Returns the output and the list of layer activations (input first)."""
    acts = [x]
    h = x
    layers = unpack(p)
    for li, (w, b) in enumerate(layers):
        z = h @ w + b
        h = np.maximum(z, 0.0) if li < len(layers) - 1 else z
        acts.append(h)
    return h, acts


def loss_and_grad(p, x, t, weights=None):
    """Mean-squared error over all outputs, each output position j weighted by weights[j]
    (default 1), and its gradient w.r.t. the packed parameters:
    loss = sum_{s, j} w_j (y_sj - t_sj)^2 / (n_seq * 448)."""
    y, acts = forward(p, x)
    n = y.size
    r = y - t
    wr = r if weights is None else r * np.asarray(weights, dtype=np.float64)[None, :]
    loss = float(np.sum(wr * r) / n)
    g = 2.0 * wr / n
    layers = unpack(p)
    grads = []
    for li in range(len(layers) - 1, -1, -1):
        w, _ = layers[li]
        h_in = acts[li]
        grads.append((h_in.T @ g, g.sum(axis=0)))
        if li > 0:
            g = (g @ w.T) * (acts[li] > 0.0)
    grads.reverse()
    return loss, np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in grads])


def adam_step(p, g, m, v, t, lr):
    """One Adam update (t counts from 1).  Returns new (p, m, v)."""
    m = BETA1 * m + (1.0 - BETA1) * g
    v = BETA2 * v + (1.0 - BETA2) * g * g
    mh = m / (1.0 - BETA1 ** t)
    vh = v / (1.0 - BETA2 ** t)
    return p - lr * mh / (np.sqrt(vh) + ADAM_EPS), m, v
