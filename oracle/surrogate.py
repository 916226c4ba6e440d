"""Learned surrogate of k frozen-flow FD substeps: plain FP64 reference.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` (and nothing in the product).

What the network computes (the method addition of the learned part; the paper
has no surrogate). Grids are channels-last arrays x[B, D, H, W, C] in (z, y, x,
channel) order, the node order of the solver's fields.

* conv(x, w, b)[v, o] = b[o] + sum over taps (a, p, q) in {0,1,2}^3 and input
  channels i of x[v + (a, p, q), i] * w[a, p, q, i, o]  (a "valid" 3x3x3
  convolution: each spatial extent shrinks by two).
* Four layers, channels 6 -> 32 -> 32 -> 32 -> 7, ReLU after the first three;
  the last layer is linear. A 40^3 input tile gives a 32^3 output tile.
* Input channels per node: psi / psi_inf, phi / phi_s, rhoN, and u_x, u_y, u_z
  divided by u_s (u_z = 0 in 2-D).
* Output channels (conservative form): per node n, raw flux coefficients
  f_psi_a, f_phi_a (a = x, y, z) and an exchange coefficient s. The fluxes of
  the conserved densities W psi and X phi (W = G + fd_eps, X = 1 - rhoN +
  fd_eps, the weights of eqs 20-21, held over the substeps) through the face
  between n and n + e_a carry the face weight of their field, and the exchange
  from bulk to interface carries the interface weight, as the transport terms
  and the source G j of eqs 20-21 do:
      Fpsi_a[n] = (W[n] + W[n + e_a])/2 f_psi_a[n],  Fphi_a[n] = (X[n] + X[n + e_a])/2 f_phi_a[n],
      S[n] = W[n] s[n].
  The changes of the conserved densities over the k substeps are
      dM_psi[n] = dpsi_s (-sum_a (Fpsi_a[n] - Fpsi_a[n - e_a]) + S[n])
      dM_phi[n] = dphi_s (-sum_a (Fphi_a[n] - Fphi_a[n - e_a])) - dpsi_s S[n]
  so sum_n (dM_psi + dM_phi) = 0 on a periodic grid whatever the network
  outputs: the total surfactant of eqs 20-21 is conserved by construction.
  psi and phi change by dM_psi / W and dM_phi / X. On a tile of T^3 output
  nodes the changes exist on the interior nodes [1, T - 2]^3 (every face they
  need lies inside the tile).
* Targets: W dpsi / dpsi_s and X dphi / dphi_s on the interior nodes. Loss: the
  mean over them and both fields of the squared error of the changes above.
* Adam with bias correction (Kingma and Ba, 2015), on FP32-like master weights
  (here FP64).

Parameter vector order (also the order of the C ABI): for each layer in turn,
the weights w[a, p, q, i, o] in row-major order, then the biases b[o].
"""
from __future__ import annotations

import numpy as np

LAYERS = ((6, 32), (32, 32), (32, 32), (32, 7))
NOUT = LAYERS[-1][1]        # 3 + 3 fluxes and the exchange
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


def _interior(shape, axis=None, d=0):
    """Slices of the interior nodes (1 .. extent - 2 along each spatial axis) of a
    [B, D, H, W, ...] grid, shifted by d along the spatial axis `axis` (0 = x,
    the last one; 1 = y; 2 = z)."""
    sl = [slice(1, e - 1) for e in shape[1:4]]
    if axis is not None:
        e = shape[3 - axis]
        sl[2 - axis] = slice(1 + d, e - 1 + d)
    return (slice(None),) + tuple(sl)


def conserved_changes(o, W, X, ratio):
    """Scaled changes (A_psi, A_phi) = (dM_psi / dpsi_s, dM_phi / dphi_s) of the
    conserved densities on the interior nodes of the output o[B, T, T, T, 7],
    with the weights W, X[B, T, T, T]; ratio = dpsi_s / dphi_s."""
    I = _interior(o.shape)
    Ap = W[I] * o[I + (6,)]
    Af = -ratio * W[I] * o[I + (6,)]
    for a in range(3):
        up, lo = _interior(o.shape, a, 1), _interior(o.shape, a, -1)
        for A, Wt, c in ((Ap, W, a), (Af, X, 3 + a)):
            A -= 0.5 * (Wt[I] + Wt[up]) * o[I + (c,)]     # out through the upper face
            A += 0.5 * (Wt[lo] + Wt[I]) * o[lo + (c,)]    # in through the lower face
    return Ap, Af


def conserved_changes_adjoint(g_psi, g_phi, W, X, ratio, shape):
    """Adjoint of `conserved_changes` in o: the gradient with respect to o of
    sum(g_psi A_psi + g_phi A_phi)."""
    do = np.zeros(shape)
    I = _interior(shape)
    do[I + (6,)] += W[I] * (g_psi - ratio * g_phi)
    for a in range(3):
        up, lo = _interior(shape, a, 1), _interior(shape, a, -1)
        for g, Wt, c in ((g_psi, W, a), (g_phi, X, 3 + a)):
            do[I + (c,)] -= 0.5 * (Wt[I] + Wt[up]) * g
            do[lo + (c,)] += 0.5 * (Wt[lo] + Wt[I]) * g
    return do


def loss_and_grads(ps, x, t, ratio=1.0):
    """Mean squared error of the conserved changes against the targets
    t[B, T, T, T, 4] = (W dpsi / dpsi_s, X dphi / dphi_s, W, X) on the interior
    nodes, and its gradient for every weight and bias (backpropagation through
    the conservative form and the layers above)."""
    o, acts = forward(ps, x)
    W, X = t[..., 2], t[..., 3]
    Ap, Af = conserved_changes(o, W, X, ratio)
    I = _interior(o.shape)
    rp, rf = Ap - t[I + (0,)], Af - t[I + (1,)]
    n = 2 * rp.size
    L = float(((rp * rp).sum() + (rf * rf).sum()) / n)
    dy = conserved_changes_adjoint(2.0 * rp / n, 2.0 * rf / n, W, X, ratio, o.shape)
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


def predict_fields(ps, psi, phi, rhoN, u, G, scales):
    """psi and phi after k substeps as the network predicts them on a periodic grid
    (every face and neighbour taken periodically)."""
    x = pad_periodic(features(psi, phi, rhoN, u, scales))[None]
    o, _ = forward(ps, x)
    W = (G + scales["fd_eps"])[None]
    X = (1.0 - rhoN + scales["fd_eps"])[None]
    # one periodic layer around the grid makes every node an interior node
    wrap = lambda a: np.pad(a, ((0, 0), (1, 1), (1, 1), (1, 1)) + ((0, 0),) * (a.ndim - 4), mode="wrap")
    Ap, Af = conserved_changes(wrap(o), wrap(W), wrap(X), scales["dpsi_s"] / scales["dphi_s"])
    return psi + scales["dpsi_s"] * Ap[0] / W[0], phi + scales["dphi_s"] * Af[0] / X[0]
