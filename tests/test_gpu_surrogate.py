"""The learned surrogate on the GPU (include/lbfd_surrogate.h) against the FP64
references: frozen-flow FD substeps against the oracle, the network's output
and gradient against oracle/surrogate.py evaluated with the same BF16 roundings
the kernels make (inputs, weights, layer outputs and output gradients rounded
to BF16; sums in FP64), training, and the fallback of surrogate mode."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import surrogate as OS
from tests.parity import say, state_errors

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbfd():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_15242_amd import lbfd as L

    L.load()
    return L


def bf16(a):
    """Nearest-even BF16 value of each entry (as float64)."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def bf16_tensor(a):
    """BF16 bit patterns of a float array as a device int16 tensor."""
    import torch

    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    h = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    return torch.from_numpy(h.view(np.int16).copy()).cuda()


def padded_input(x6):
    """[..., 6] inputs padded with zeros to the 16 channels of the kernels."""
    pad = np.zeros(x6.shape[:-1] + (16,))
    pad[..., :6] = x6
    return pad


def gpu_params(ps):
    """The oracle's parameters as the kernels hold them: BF16 weights, FP32 biases."""
    return [[bf16(w), np.float32(b).astype(np.float64)] for w, b in ps]


def ref_forward(ps, x):
    h = x
    acts = [x]
    for li, (w, b) in enumerate(ps):
        y = OS.conv(h, w, b)
        h = bf16(np.maximum(y, 0.0)) if li < len(ps) - 1 else y
        acts.append(h)
    return h, acts


def ref_gradient(ps, x, t, ratio):
    """Loss of the conservative form and its gradient, with the kernels' BF16
    roundings of the output gradient and of the layer gradients."""
    o, acts = ref_forward(ps, x)
    W, X = t[..., 2], t[..., 3]
    Ap, Af = OS.conserved_changes(o, W, X, ratio)
    I = (slice(None), slice(1, -1), slice(1, -1), slice(1, -1))
    rp, rf = Ap - t[I + (0,)], Af - t[I + (1,)]
    n = 2 * rp.size
    dy = bf16(OS.conserved_changes_adjoint(2.0 * rp / n, 2.0 * rf / n, W, X, ratio, o.shape))
    dy = np.concatenate([dy, np.zeros(dy.shape[:-1] + (32 - OS.NOUT,))], axis=-1)   # padded output channels
    grads = [None] * len(ps)
    for li in range(len(ps) - 1, -1, -1):
        w, _ = ps[li]
        wpad = w if w.shape[-1] == 32 else np.concatenate([w, np.zeros(w.shape[:-1] + (32 - w.shape[-1],))], axis=-1)
        dw, db = OS.conv_grad_weight(acts[li], dy)
        co = w.shape[-1]
        grads[li] = [dw[..., :co], db[:co]]
        if li > 0:
            dx = OS.conv_grad_input(dy, wpad, acts[li].shape)
            dy = bf16(dx * (acts[li] > 0.0))
    return float(((rp * rp).sum() + (rf * rf).sum()) / n), grads


def make_sg(L, **kw):
    return L.Surrogate(**kw)


@pytest.mark.parametrize("case", ["periodic3d", "odd2d", "walled3d"])
def test_frozen_substeps_match_oracle(lbfd, case):
    """k FD substeps with the flow frozen, FP64, against the oracle's; the LB
    populations do not move."""
    if case == "periodic3d":
        p, q = W.make(dict(lattice=W.D3Q19, nx=20, ny=18, nz=16, sigma0=0.01, E0=0.5, Ds=0.05, Db=0.05,
                           rhoR0=0.5, muR0=0.1, gravity=[0, 0, -1e-5], precision="fp64"),
                      dict(drops=[(9.5, 8.5, 7.5, 5.0)], width=3.0, psi0=0.1, phi0_out=0.05, phi0_in=0.0))
    elif case == "odd2d":
        p, q = W.droplet_adsorption(n=70, radius=11.0, ny=37)
    else:
        p, q = W.bubble_rise(nx=24, ny=20, nz=32, radius=6.0, precision="fp64")
    say(f"[frozen substeps] {case}")
    s = lbfd.Solver(p).init_fields(q).step(5)
    o = oracle.Oracle(dict(p, precision="fp64")).init(q).step(5)
    f0 = s.field("f")
    s.fd_substeps(8)
    o.fd_substeps(8)
    errs = state_errors(s, o)
    say(errs)
    assert max(errs.values()) < 1e-10, errs
    assert np.array_equal(s.field("f"), f0)
    assert s.observables()["status"] == 0


def test_forward_matches_reference(lbfd):
    import torch

    rng = np.random.default_rng(11)
    ps = gpu_params(OS.init_params(3, out_scale=1.0))
    x6 = bf16(rng.uniform(-1.0, 1.0, (2, 11, 12, 13, 6)))
    sg = make_sg(lbfd, tile=4, max_batch=2)
    sg.set_params(OS.flatten(ps))
    out = torch.empty((2, 3, 4, 5, OS.NOUT), dtype=torch.float32, device="cuda")
    sg.forward(bf16_tensor(padded_input(x6)), out)
    ref, _ = ref_forward(ps, x6)
    err = float(np.abs(out.cpu().numpy() - ref).max() / np.abs(ref).max())
    say(f"forward max rel err {err:.2e}")
    assert err < 5e-3
    # parameters round-trip through the master copy
    assert np.array_equal(sg.get_params(), np.float32(OS.flatten(ps)))


@pytest.mark.parametrize("T,B", [(4, 2), (32, 8)])
def test_gradient_matches_reference(lbfd, T, B):
    """The full gradient of the conservative loss: a tiny tile, and the tiles of
    the training launch the surrogate benchmark times (32^3 outputs, 8 tiles:
    128 stages of 256 nodes per tile in the weight gradient)."""
    import torch

    rng = np.random.default_rng(12)
    ps = gpu_params(OS.init_params(4, out_scale=1.0))
    x6 = bf16(rng.uniform(-1.0, 1.0, (B, T + 8, T + 8, T + 8, 6)))
    t = rng.standard_normal((B, T, T, T, 4)).astype(np.float32)
    t[..., 2:] = rng.uniform(0.05, 2.0, (B, T, T, T, 2))     # the weights W, X
    sg = make_sg(lbfd, tile=T, max_batch=B, dpsi_s=0.02, dphi_s=0.005)
    sg.set_params(OS.flatten(ps))
    loss, g = sg.gradient(bf16_tensor(padded_input(x6)), torch.from_numpy(t).cuda())
    Lr, gr = ref_gradient(ps, x6, t.astype(np.float64), 0.02 / 0.005)
    say(f"loss gpu {loss:.6e} ref {Lr:.6e}")
    assert abs(loss - Lr) <= 1e-3 * Lr
    o = 0
    for li, (w, b) in enumerate(gr):
        for name, ref in (("w", w), ("b", b)):
            n = ref.size
            got = g[o:o + n].reshape(ref.shape)
            o += n
            err = float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-30))
            say(f"layer {li} {name}: max rel err {err:.2e}")
            assert err < 2e-2, (li, name, err)
    assert o == g.size


def test_step_size_setter_scales_the_first_adam_step(lbfd):
    """lbfd_sg_set_lr: Adam's first step from fresh moments moves each weight by
    lr g / (|g| + eps), so a quarter of the step size moves it a quarter as far;
    a step size that is not positive is rejected."""
    import torch

    rng = np.random.default_rng(13)
    T = 4
    x6 = bf16(rng.uniform(-1.0, 1.0, (2, T + 8, T + 8, T + 8, 6)))
    t = rng.standard_normal((2, T, T, T, 4)).astype(np.float32)
    t[..., 2:] = rng.uniform(0.05, 2.0, (2, T, T, T, 2))
    x, tt = bf16_tensor(padded_input(x6)), torch.from_numpy(t).cuda()
    p0 = np.float32(OS.flatten(gpu_params(OS.init_params(4, out_scale=1.0))))
    lr = 1e-3
    sg = make_sg(lbfd, tile=T, max_batch=2, lr=lr, dpsi_s=0.02, dphi_s=0.005)
    moves = []
    for f in (1.0, 0.25):
        sg.set_params(p0)   # fresh moments and step count
        sg.set_lr(lr * f)
        sg.train_step(x, tt, want_loss=False)
        moves.append(sg.get_params().astype(np.float64) - p0)
    d1, d2 = moves
    big = np.abs(d1) > 0.5 * lr
    say(f"{int(big.sum())} of {p0.size} weights moved by more than lr / 2")
    assert big.sum() > 0.5 * p0.size
    assert np.abs(d2[big] - 0.25 * d1[big]).max() <= 1e-3 * lr
    for bad in (0.0, -1e-3, float("nan"), float("inf")):
        with pytest.raises(lbfd.LbfdError):
            sg.set_lr(bad)


def _bubbles(lbfd, n=40, seed=1):
    p, q = W.multi_bubble(n=n, count=2, diameter=12.0, seed=seed, precision="fp32")
    return lbfd.Solver(p).init_fields(q), p


def test_training_lowers_the_error(lbfd):
    """Tiles from the solver's own snapshots; Adam on the GPU lowers the loss and
    the trained network's error on tiles of a later snapshot is well below that
    of predicting no change."""
    from paper_2311_15242_amd import sgtrain

    rng = np.random.default_rng(5)
    s, p = _bubbles(lbfd)
    s.step(40)
    dps, dph = sgtrain.change_scales(s, 8)
    sg = make_sg(lbfd, tile=16, max_batch=8, k=8, dpsi_s=dps, dphi_s=dph, phi_s=0.5, u_s=0.005, lr=2e-3)
    sg.set_params(sgtrain.initial_params(0))
    bufs = sgtrain.feature_buffers(s)
    Xs, Ys = [], []
    for i in range(6):
        s.step(15)
        X, Y = sgtrain.snapshot_tiles(s, sg, 16, rng, bufs)
        Xs.append(X)
        Ys.append(Y)
    import torch

    X, Y = torch.cat(Xs), torch.cat(Ys)
    s.step(15)
    Xh, Yh = sgtrain.snapshot_tiles(s, sg, 16, rng, bufs)
    e0, _ = sgtrain.tile_error(sg, Xh, Yh)
    hist = sgtrain.train(sg, X, Y, 300, 8, rng, log_every=50)
    e1, _ = sgtrain.tile_error(sg, Xh, Yh)
    say(f"loss {hist[0][1]:.3e} -> {hist[-1][1]:.3e}; held-out error {e0:.3f} -> {e1:.3f}")
    assert hist[-1][1] < 0.5 * hist[0][1]
    assert e1 < 0.6 and e1 < e0


def test_advance_fallback_is_the_fd_update(lbfd):
    """Weights that predict nonsense fail the range check every time (the
    conservative form keeps the total whatever the weights); surrogate mode then
    equals frozen-flow FD substeps followed by LB steps with psi held, bit for
    bit."""
    rng = np.random.default_rng(6)
    p, q = W.multi_bubble(n=24, count=1, diameter=10.0, seed=2, precision="fp32")
    a = lbfd.Solver(p).init_fields(q).step(6)
    b = lbfd.Solver(p).init_fields(q).step(6)
    sg = make_sg(lbfd, tile=8, max_batch=1, k=4, field=(24, 24, 24), dpsi_s=1.0, dphi_s=1.0)
    sg.set_params((rng.standard_normal(sg.n) * 3.0).astype(np.float32))
    rep = sg.advance(a, 3)
    say(rep)
    assert rep["blocks"] == 3 and rep["fallbacks"] == 3 and rep["accepted"] == 0
    for _ in range(3):
        b.fd_substeps(4)
        b.set_fd(False).step(4).set_fd(True)
    for name in ("f", "psi", "phi", "u", "rhoN"):
        assert np.array_equal(a.field(name), b.field(name)), name
    assert a.observables()["step"] == b.observables()["step"] == 18


def test_advance_passes_the_strict_drift_check(lbfd):
    """With the drift check at 1e-6 a network with small outputs is kept every
    time: the conservative form changes the total surfactant only by rounding
    before the rescaling, and the applied update is the network's own."""
    from paper_2311_15242_amd import sgtrain

    p, q = W.multi_bubble(n=24, count=1, diameter=10.0, seed=3, precision="fp32")
    s = lbfd.Solver(p).init_fields(q).step(6)
    psi0 = s.field("psi")
    sg = make_sg(lbfd, tile=8, max_batch=1, k=4, field=(24, 24, 24), drift_tol=1e-6)
    sg.set_params(sgtrain.initial_params(1, out_scale=0.01))
    rep = sg.advance(s, 3)
    say(rep)
    assert rep["accepted"] == 3 and rep["fallbacks"] == 0
    assert rep["max_drift"] <= 1e-6
    assert s.observables()["status"] == 0
    assert np.abs(s.field("psi") - psi0).max() > 0


def test_advance_accepts_and_conserves(lbfd):
    """With the check opened up every application is kept. Each kept update is
    rescaled to the initial total; during the k LB steps that follow, psi and phi
    are held while the weights G and 1 - rhoN move with the interface, so the
    total at the end of a block is close to, not equal to, the initial one."""
    p, q = W.multi_bubble(n=24, count=1, diameter=10.0, seed=3, precision="fp32")
    s = lbfd.Solver(p).init_fields(q).step(6)
    M0 = s.observables()["total_surf"]
    from paper_2311_15242_amd import sgtrain

    sg = make_sg(lbfd, tile=8, max_batch=1, k=4, field=(24, 24, 24), drift_tol=1.0)
    sg.set_params(sgtrain.initial_params(1, out_scale=0.01))
    rep = sg.advance(s, 2)
    say(rep)
    assert rep["accepted"] == 2 and rep["fallbacks"] == 0
    ob = s.observables()
    assert ob["status"] == 0 and ob["step"] == 14
    assert abs(ob["total_surf"] - M0) <= 1e-3 * M0


@pytest.mark.parametrize("shape,batch", [((11, 14, 75), 1), ((45, 13, 71), 1), ((9, 10, 70), 2)])
def test_forward_wide_grid_matches_reference(lbfd, shape, batch):
    """Grids at least 60 output nodes wide run the z-marching kernel (columns of
    30 x 4 output nodes over 32 planes, weights in registers, input planes in LDS);
    ragged in every direction, the second grid spans two column heights and the
    third is a batch of two grids."""
    import torch

    rng = np.random.default_rng(13)
    ps = gpu_params(OS.init_params(5, out_scale=1.0))
    d, h, w = shape
    x6 = bf16(rng.uniform(-1.0, 1.0, (batch, d, h, w, 6)))
    sg = make_sg(lbfd, tile=16, max_batch=batch, field=(w - 8, h - 8, d - 8))
    sg.set_params(OS.flatten(ps))
    out = torch.empty((batch, d - 8, h - 8, w - 8, OS.NOUT), dtype=torch.float32, device="cuda")
    sg.forward(bf16_tensor(padded_input(x6)), out)
    ref, _ = ref_forward(ps, x6)
    err = float(np.abs(out.cpu().numpy() - ref).max() / np.abs(ref).max())
    say(f"wide forward {shape} max rel err {err:.2e}")
    assert err < 5e-3


def test_forward_full_grid_sampled(lbfd):
    """The whole-grid forward at the benchmark's size (256^3 output nodes from a
    264^3 input, the launch the surrogate benchmark times) against the reference
    at sampled output nodes: the eight corners, points on the faces and edges
    and random interior nodes, each from its own 9^3 input window."""
    import torch

    n, H = 256, 4
    m = n + 2 * H
    rng = np.random.default_rng(17)
    x6 = rng.uniform(-1.0, 1.0, (m, m, m, 6)).astype(np.float32)
    u = x6.view(np.uint32).astype(np.uint64)
    bits = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    del u
    full = np.zeros((m, m, m, 16), dtype=np.uint16)
    full[..., :6] = bits
    del bits
    x = torch.from_numpy(full.view(np.int16)).cuda().view(1, m, m, m, 16)
    del full
    ps = gpu_params(OS.init_params(7, out_scale=1.0))
    sg = make_sg(lbfd, tile=16, max_batch=1, field=(n, n, n))
    sg.set_params(OS.flatten(ps))
    out = torch.empty((1, n, n, n, OS.NOUT), dtype=torch.float32, device="cuda")
    sg.forward(x, out)
    torch.cuda.synchronize()
    e = (0, n // 2, n - 1)
    pts = {(a, b, c) for a in (0, n - 1) for b in (0, n - 1) for c in (0, n - 1)}
    pts |= {(a, b, c) for a in e for b in e for c in e}
    pts |= {tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(24)}
    got, ref = [], []
    for (z, y, xx) in sorted(pts):
        win = bf16(x6[z:z + 2 * H + 1, y:y + 2 * H + 1, xx:xx + 2 * H + 1])[None]
        r, _ = ref_forward(ps, win)
        ref.append(r[0, 0, 0, 0])
        got.append(out[0, z, y, xx].cpu().numpy())
    got, ref = np.array(got), np.array(ref)
    err = float(np.abs(got - ref).max() / np.abs(ref).max())
    say(f"full-grid forward {n}^3, {len(pts)} sampled nodes: max rel err {err:.2e}")
    assert err < 5e-3
