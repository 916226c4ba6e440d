"""Learned surrogate of k frozen-flow FD substeps: plain FP64 reference.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` (and nothing in the product).

What the network computes (the method addition of the learned part; the paper
has no surrogate). Grids are channels-last arrays x[B, D, H, W, C] in (z, y, x,
channel) order, the node order of the solver's fields.

* conv(x, w, b)[v, o] = b[o] + sum over taps (a, p, q) in {0,1,2}^3 and input
  channels i of x[v + (a, p, q), i] * w[a, p, q, i, o]  (a "valid" 3x3x3
  convolution: each spatial extent shrinks by two).
* Four layers, channels 6 -> 32 -> 32 -> 32 -> 2, ReLU after the first three;
  the last layer is linear. A 40^3 input tile gives a 32^3 output tile.
* Input channels per node: psi / psi_inf, phi / phi_s, rhoN, and u_x, u_y, u_z
  divided by u_s (u_z = 0 in 2-D). Output channels: the change of psi and of
  phi over the k substeps, divided by dpsi_s and dphi_s.
* Loss: the mean over output nodes and both channels of the squared error.
* Adam with bias correction (Kingma and Ba, 2015), on FP32-like master weights
  (here FP64).

Parameter vector order (also the order of the C ABI): for each layer in turn,
the weights w[a, p, q, i, o] in row-major order, then the biases b[o].
"""
from __future__ import annotations

import numpy as np

LAYERS = ((6, 32), (32, 32), (32, 32), (32, 2))
HALO = len(LAYERS)          # each layer trims one node per side


def n_params() -> int:
    return sum(27 * ci * co + co for ci, co in LAYERS)


def init_params(seed: int = 0, out_scale: float = 0.1):
    """He-normal weights (std sqrt(2 / (27 Cin))), zero biases; the last layer
    scaled by out_scale so the untrained network predicts a small change."""
    rng = np.random.default_rng(seed)
    ps = []
    for li, (ci, co) in enumerate(LAYERS):
        w = rng.standard_normal((3, 3, 3, ci, co)) * np.sqrt(2.0 / (27 * ci))
        if li == len(LAYERS) - 1:
            w *= out_scale
        ps.append([w, np.zeros(co)])
    return ps


def flatten(ps) -> np.ndarray:
    return np.concatenate([np.concatenate([w.reshape(-1), b]) for w, b in ps])


def unflatten(v) -> list:
    v = np.asarray(v, dtype=np.float64)
    ps, o = [], 0
    for ci, co in LAYERS:
        nw = 27 * ci * co
        w = v[o:o + nw].reshape(3, 3, 3, ci, co)
        o += nw
        b = v[o:o + co].copy()
        o += co
        ps.append([w.copy(), b])
    assert o == v.size
    return ps


def conv(x, w, b):
    B, D, H, W, _ = x.shape
    out = np.zeros((B, D - 2, H - 2, W - 2, w.shape[-1])) + b
    for a in range(3):
        for p in range(3):
            for q in range(3):
                out += x[:, a:a + D - 2, p:p + H - 2, q:q + W - 2, :] @ w[a, p, q]
    return out


def conv_grad_input(dy, w, in_shape):
    """Adjoint of conv in x: dx[v + tap, i] += dy[v, o] w[tap, i, o]."""
    dx = np.zeros(in_shape)
    _, Do, Ho, Wo, _ = dy.shape
    for a in range(3):
        for p in range(3):
            for q in range(3):
                dx[:, a:a + Do, p:p + Ho, q:q + Wo, :] += dy @ w[a, p, q].T
    return dx


def conv_grad_weight(x, dy):
    """Adjoint of conv in w: dw[tap, i, o] = sum_v x[v + tap, i] dy[v, o]; db[o] = sum_v dy[v, o]."""
    _, Do, Ho, Wo, co = dy.shape
    ci = x.shape[-1]
    dw = np.zeros((3, 3, 3, ci, co))
    dyf = dy.reshape(-1, co)
    for a in range(3):
        for p in range(3):
            for q in range(3):
                dw[a, p, q] = x[:, a:a + Do, p:p + Ho, q:q + Wo, :].reshape(-1, ci).T @ dyf
    return dw, dyf.sum(0)


def forward(ps, x):
    """Output and the layer inputs (kept for the backward pass)."""
    acts = [x]
    h = x
    for li, (w, b) in enumerate(ps):
        y = conv(h, w, b)
        h = np.maximum(y, 0.0) if li < len(ps) - 1 else y
        acts.append(h)
    return h, acts


def loss_and_grads(ps, x, t):
    """Mean squared error of the output against t, and its gradient for every
    weight and bias (backpropagation through the layers above)."""
    o, acts = forward(ps, x)
    r = o - t
    L = float((r * r).mean())
    dy = 2.0 * r / r.size
    grads = [None] * len(ps)
    for li in range(len(ps) - 1, -1, -1):
        w, _ = ps[li]
        dw, db = conv_grad_weight(acts[li], dy)
        grads[li] = [dw, db]
        if li > 0:
            dx = conv_grad_input(dy, w, acts[li].shape)
            dy = dx * (acts[li] > 0.0)      # ReLU of the layer below
    return L, grads


def adam(ps, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step; state = dict(t, m, v) with m, v flat arrays (created when empty)."""
    g = flatten(grads)
    p = flatten(ps)
    if not state:
        state.update(t=0, m=np.zeros_like(p), v=np.zeros_like(p))
    state["t"] += 1
    t = state["t"]
    state["m"] = beta1 * state["m"] + (1.0 - beta1) * g
    state["v"] = beta2 * state["v"] + (1.0 - beta2) * g * g
    mh = state["m"] / (1.0 - beta1 ** t)
    vh = state["v"] / (1.0 - beta2 ** t)
    return unflatten(p - lr * mh / (np.sqrt(vh) + eps))


def features(psi, phi, rhoN, u, scales):
    """Input channels of one grid (arrays of shape (nz, ny, nx), u of shape (d, nz, ny, nx))."""
    psi_inf, phi_s, u_s = scales["psi_inf"], scales["phi_s"], scales["u_s"]
    ch = [psi / psi_inf, phi / phi_s, rhoN]
    for a in range(3):
        ch.append(u[a] / u_s if a < u.shape[0] else np.zeros_like(psi))
    return np.stack(ch, axis=-1)


def pad_periodic(x, h=HALO):
    """Periodic halo of h nodes on the three spatial axes of x[D, H, W, C]."""
    return np.pad(x, ((h, h), (h, h), (h, h), (0, 0)), mode="wrap")


def predict_fields(ps, psi, phi, rhoN, u, scales):
    """psi and phi after k substeps as the network predicts them on a periodic grid."""
    x = pad_periodic(features(psi, phi, rhoN, u, scales))[None]
    o, _ = forward(ps, x)
    return psi + scales["dpsi_s"] * o[0, ..., 0], phi + scales["dphi_s"] * o[0, ..., 1]
