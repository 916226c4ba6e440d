"""Snapshot tiles from the solver and training of the learned surrogate.

Orchestration only: the features, the frozen-flow FD substeps that make the
targets, the tile crops, the network and Adam all run in liblbfd.so's kernels.
Tiles are torch device tensors (inputs as int16 tensors holding BF16 bit
patterns, targets FP32).
"""
from __future__ import annotations

import numpy as np

from . import lbfd


def feature_buffers(solver):
    import torch

    p = solver.p
    nf = (p["nz"] + 8) * (p["ny"] + 8) * (p["nx"] + 8) * 16
    feat = torch.empty(nf, dtype=torch.int16, device=solver.device)
    snap = torch.empty(2 * solver.N, dtype=torch.float32, device=solver.device)
    return feat, snap


def tile_origins(solver, T: int, n_tiles: int, rng, interface_share: float = 0.75, g_min: float = 0.05):
    """Output corners of n_tiles tiles: a share of them centred on random nodes of
    the interface (|grad rhoN| >= g_min, where psi and phi change), the rest
    uniform over the grid. On a grid with a few small bubbles a uniform draw
    would give mostly tiles where nothing happens."""
    p = solver.p
    hi = np.array([p["nx"] - T + 1, p["ny"] - T + 1, p["nz"] - T + 1])
    org = rng.integers(0, hi, size=(n_tiles, 3))
    n_if = int(round(interface_share * n_tiles))
    if n_if > 0:
        G = solver.field("G")
        z, y, x = np.nonzero(G >= g_min)
        if x.size:
            pick = rng.integers(0, x.size, size=n_if)
            c = np.stack([x[pick], y[pick], z[pick]], axis=1) - T // 2
            org[:n_if] = np.clip(c, 0, hi - 1)
    return org.astype(np.int32)


def snapshot_tiles(solver, sg, n_tiles: int, rng, bufs=None, interface_share: float = 0.75, out=None):
    """n_tiles training tiles of the solver's current state: inputs from the
    state now, targets from the state after k frozen-flow FD substeps (the
    solver's psi and phi are left advanced by those substeps). out: optional
    (X, Y) device tensors of n_tiles tiles to fill (a slice of a larger set)."""
    import torch

    T = sg.cfg["tile"]
    feat, snap = bufs if bufs is not None else feature_buffers(solver)
    org = tile_origins(solver, T, n_tiles, rng, interface_share)
    sg.features(solver, feat)
    sg.snapshot(solver, snap)
    solver.fd_substeps(sg.cfg["k"])
    if out is not None:
        X, Y = out
        if tuple(X.shape) != (n_tiles, T + 8, T + 8, T + 8, 16) or tuple(Y.shape) != (n_tiles, T, T, T, 4):
            raise ValueError("snapshot_tiles: out tensors of the wrong shape")
    else:
        X = torch.empty((n_tiles, T + 8, T + 8, T + 8, 16), dtype=torch.int16, device=solver.device)
        Y = torch.empty((n_tiles, T, T, T, 4), dtype=torch.float32, device=solver.device)
    mb = sg.cfg["max_batch"]
    for a in range(0, n_tiles, mb):
        b = min(n_tiles, a + mb)
        sg.tiles(solver, feat, snap, org[a:b], X[a:b], Y[a:b])
    return X, Y


def change_scales(solver, k: int, quantile: float = 0.999):
    """Scales of the target channels from one probe: the given quantile of
    |change| of psi and phi over k frozen-flow substeps (the probe's substeps
    are applied to the solver)."""
    psi0, phi0 = solver.field("psi"), solver.field("phi")
    solver.fd_substeps(k)
    dpsi = np.abs(solver.field("psi") - psi0)
    dphi = np.abs(solver.field("phi") - phi0)
    return float(max(np.quantile(dpsi, quantile), 1e-12)), float(max(np.quantile(dphi, quantile), 1e-12))


def train(sg, X, Y, steps: int, batch: int, rng, log_every: int = 0, lr_final: float | None = None):
    """Adam steps on random minibatches of the tiles; returns the loss history
    (one value per logged step, each read back from the device).

    lr_final: the step size falls from the network's configured one to lr_final
    along a half cosine over the run (None: constant)."""
    import math

    import torch

    n = X.shape[0]
    hist = []
    lr0 = sg.cfg["lr"]
    for it in range(steps):
        if lr_final is not None:
            sg.set_lr(lr_final + 0.5 * (lr0 - lr_final) * (1.0 + math.cos(math.pi * it / max(1, steps - 1))))
        idx = torch.as_tensor(rng.choice(n, size=min(batch, n), replace=False), device=X.device)
        xb = X.index_select(0, idx).contiguous()
        yb = Y.index_select(0, idx).contiguous()
        want = log_every > 0 and (it % log_every == 0 or it == steps - 1)
        loss = sg.train_step(xb, yb, want_loss=want)
        if want:
            hist.append((it, loss))
    if lr_final is not None:
        sg.set_lr(lr0)   # the configured step size again for later calls
    return hist


def conserved_changes(o, Y, ratio):
    """The conservative form of the network's tile output o[B, T, T, T, 7] (the
    changes of W psi / dpsi_s and X phi / dphi_s on the interior nodes), with the
    weights W, X of the targets Y[..., 2:4]; for the error measure only (training
    and application evaluate it in the library's kernels)."""
    W, X = Y[..., 2], Y[..., 3]
    I = (slice(None), slice(1, -1), slice(1, -1), slice(1, -1))

    def sh(a, axis, d):
        sl = [slice(1, -1)] * 3
        sl[2 - axis] = slice(1 + d, a.shape[3 - axis] - 1 + d)
        return a[(slice(None),) + tuple(sl)]

    Ap = W[I] * o[I + (6,)]
    Af = -ratio * W[I] * o[I + (6,)]
    for a in range(3):
        for A, Wt, c in ((Ap, W, a), (Af, X, 3 + a)):
            A -= 0.5 * (Wt[I] + sh(Wt, a, 1)) * o[I + (c,)]
            A += 0.5 * (sh(Wt, a, -1) + Wt[I]) * sh(o[..., c], a, -1)
    return Ap, Af


def tile_error(sg, X, Y):
    """Relative L2 error of the network's conserved changes on the tiles' interior
    nodes against the targets, and that of predicting no change at all."""
    import torch

    mb = sg.cfg["max_batch"]
    T = sg.cfg["tile"]
    ratio = sg.cfg["dpsi_s"] / sg.cfg["dphi_s"]
    I = (slice(None), slice(1, -1), slice(1, -1), slice(1, -1))
    num = den = 0.0
    for a in range(0, X.shape[0], mb):
        b = min(X.shape[0], a + mb)
        out = torch.empty((b - a, T, T, T, lbfd.SG_NOUT), dtype=torch.float32, device=X.device)
        sg.forward(X[a:b].contiguous(), out)
        Ap, Af = conserved_changes(out, Y[a:b], ratio)
        tp, tf = Y[a:b][I + (0,)], Y[a:b][I + (1,)]
        num += float(((Ap - tp) ** 2).sum().item() + ((Af - tf) ** 2).sum().item())
        den += float((tp ** 2).sum().item() + (tf ** 2).sum().item())
    return float(np.sqrt(num / max(den, 1e-300))), 1.0


def initial_params(seed: int = 0, out_scale: float = 0.1):
    """He-normal weights, zero biases, a small last layer (parameter order of the C ABI)."""
    rng = np.random.default_rng(seed)
    layers = ((6, 32), (32, 32), (32, 32), (32, lbfd.SG_NOUT))
    parts = []
    for li, (ci, co) in enumerate(layers):
        w = rng.standard_normal(27 * ci * co) * np.sqrt(2.0 / (27 * ci))
        if li == len(layers) - 1:
            w *= out_scale
        parts += [w, np.zeros(co)]
    return np.concatenate(parts).astype(np.float32)


__all__ = ["feature_buffers", "tile_origins", "snapshot_tiles", "change_scales", "train", "conserved_changes",
           "tile_error", "initial_params", "lbfd"]
