"""Pins of the FP64 surrogate reference (oracle/surrogate.py) to things other
than itself: the convolution written out as loops, closed forms, adjoint
identities, central finite differences of the loss, and Adam's first step."""
import numpy as np
import pytest

from oracle import surrogate as S


def conv_loops(x, w, b):
    B, D, H, W, ci = x.shape
    co = w.shape[-1]
    out = np.zeros((B, D - 2, H - 2, W - 2, co))
    for n in range(B):
        for z in range(D - 2):
            for y in range(H - 2):
                for xx in range(W - 2):
                    for o in range(co):
                        s = b[o]
                        for a in range(3):
                            for p in range(3):
                                for q in range(3):
                                    for i in range(ci):
                                        s += x[n, z + a, y + p, xx + q, i] * w[a, p, q, i, o]
                        out[n, z, y, xx, o] = s
    return out


def test_conv_matches_loops():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 4, 5, 6, 3))
    w = rng.standard_normal((3, 3, 3, 3, 2))
    b = rng.standard_normal(2)
    assert np.abs(S.conv(x, w, b) - conv_loops(x, w, b)).max() < 1e-12


def test_conv_delta_kernel_is_a_crop():
    """A kernel that is the identity channel map at the centre tap returns the
    interior of the input (plus the bias)."""
    rng = np.random.default_rng(2)
    x = rng.standard_normal((1, 6, 5, 7, 4))
    w = np.zeros((3, 3, 3, 4, 4))
    w[1, 1, 1] = np.eye(4)
    b = np.array([0.5, -1.0, 0.0, 2.0])
    assert np.array_equal(S.conv(x, w, b), x[:, 1:-1, 1:-1, 1:-1, :] + b)


def test_adjoint_identities():
    """<conv(x, w), y> = <x, grad_input(y, w)> = <w, grad_weight(x, y)> (zero bias)."""
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 5, 6, 7, 3))
    w = rng.standard_normal((3, 3, 3, 3, 4))
    y = rng.standard_normal((2, 3, 4, 5, 4))
    lhs = float((S.conv(x, w, np.zeros(4)) * y).sum())
    dx = S.conv_grad_input(y, w, x.shape)
    dw, db = S.conv_grad_weight(x, y)
    assert abs(lhs - float((x * dx).sum())) < 1e-10 * abs(lhs)
    assert abs(lhs - float((w * dw).sum())) < 1e-10 * abs(lhs)
    assert np.allclose(db, y.reshape(-1, 4).sum(0), rtol=1e-14, atol=0)


def test_gradients_match_central_differences():
    rng = np.random.default_rng(4)
    ps = S.init_params(5, out_scale=1.0)
    x = rng.standard_normal((2, 12, 12, 11, 6))
    t = rng.standard_normal((2, 4, 4, 3, 4))
    t[..., 2:] = rng.uniform(0.1, 2.0, (2, 4, 4, 3, 2))      # the weights W, X
    ratio = 1.7
    L, grads = S.loss_and_grads(ps, x, t, ratio)
    flat, g = S.flatten(ps), S.flatten(grads)
    idx = rng.choice(flat.size, 40, replace=False)
    # include biases of every layer
    o = 0
    for ci, co in S.LAYERS:
        o += 27 * ci * co
        idx = np.append(idx, o)
        o += co
    for k in idx:
        h = 1e-6 * max(1.0, abs(flat[k]))
        up, dn = flat.copy(), flat.copy()
        up[k] += h
        dn[k] -= h
        fd = (S.loss_and_grads(S.unflatten(up), x, t, ratio)[0] - S.loss_and_grads(S.unflatten(dn), x, t, ratio)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(abs(g[k]), 1e-3 * np.abs(g).max()), (k, fd, g[k])


def test_adam_first_step_closed_form():
    """From zero moments the bias-corrected first step is -lr g / (|g| + eps)."""
    ps = S.init_params(6)
    rng = np.random.default_rng(7)
    grads = S.unflatten(rng.standard_normal(S.n_params()))
    st = {}
    lr, eps = 1e-3, 1e-8
    new = S.adam(ps, grads, st, lr, eps=eps)
    g = S.flatten(grads)
    assert np.allclose(S.flatten(new) - S.flatten(ps), -lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-18)


def test_parameter_layout():
    ps = S.init_params(8)
    assert S.n_params() == 27 * (6 * 32 + 32 * 32 * 2 + 32 * 7) + 32 * 3 + 7 == 66631
    assert np.array_equal(S.flatten(S.unflatten(S.flatten(ps))), S.flatten(ps))


def test_periodic_prediction_is_translation_equivariant():
    """On a periodic grid the predicted fields shift with the inputs."""
    rng = np.random.default_rng(9)
    ps = S.init_params(10, out_scale=1.0)
    sc = dict(psi_inf=1.0, phi_s=0.1, u_s=0.01, dpsi_s=0.01, dphi_s=0.001, fd_eps=1e-6)
    shape = (6, 7, 8)
    psi, phi, rN = rng.random(shape), 0.1 * rng.random(shape), rng.uniform(-1, 1, shape)
    G = 0.3 * rng.random(shape)
    u = 0.01 * rng.standard_normal((3,) + shape)
    a = S.predict_fields(ps, psi, phi, rN, u, G, sc)
    sh = lambda f: np.roll(f, (1, -2, 3), axis=(-3, -2, -1))
    b = S.predict_fields(ps, sh(psi), sh(phi), sh(rN), sh(u), sh(G), sc)
    assert np.abs(sh(a[0]) - b[0]).max() < 1e-12 and np.abs(sh(a[1]) - b[1]).max() < 1e-12


def _periodic_case(seed):
    rng = np.random.default_rng(seed)
    sc = dict(psi_inf=1.0, phi_s=0.1, u_s=0.01, dpsi_s=0.02, dphi_s=0.003, fd_eps=1e-6)
    shape = (6, 7, 8)
    return (rng.random(shape), 0.1 * rng.random(shape), rng.uniform(-1, 1, shape),
            0.01 * rng.standard_normal((3,) + shape), 0.3 * rng.random(shape), sc)


def test_prediction_conserves_the_total_surfactant():
    """Whatever the weights, the flux form changes sum(W psi + X phi) only by
    rounding (eqs 20-21: the divergences telescope on the periodic grid and
    the exchange moves conserved density between the fields)."""
    psi, phi, rN, u, G, sc = _periodic_case(11)
    ps = S.init_params(12, out_scale=5.0)
    W, X = G + sc["fd_eps"], 1.0 - rN + sc["fd_eps"]
    p2, f2 = S.predict_fields(ps, psi, phi, rN, u, G, sc)
    M0, M1 = (W * psi + X * phi).sum(), (W * p2 + X * f2).sum()
    assert np.abs(p2 - psi).max() > 1e-3                      # the update is not small
    assert abs(M1 - M0) < 1e-13 * M0


def test_pure_exchange_closed_form():
    """All weights zero and only the exchange bias b_S: every node moves
    dpsi_s b_S W of conserved density from the bulk field to the interface field."""
    psi, phi, rN, u, G, sc = _periodic_case(13)
    ps = S.init_params(14)
    for w, b in ps:
        w[...] = 0.0
        b[...] = 0.0
    ps[-1][1][6] = 0.25
    W, X = G + sc["fd_eps"], 1.0 - rN + sc["fd_eps"]
    p2, f2 = S.predict_fields(ps, psi, phi, rN, u, G, sc)
    assert np.abs(W * (p2 - psi) - sc["dpsi_s"] * 0.25 * W).max() < 1e-15
    assert np.abs(X * (f2 - phi) + sc["dpsi_s"] * 0.25 * W).max() < 1e-15


def test_conserved_changes_adjoint_identity():
    rng = np.random.default_rng(15)
    o = rng.standard_normal((2, 5, 6, 7, 7))
    W, X = rng.uniform(0.1, 1.0, (2, 5, 6, 7)), rng.uniform(0.1, 2.0, (2, 5, 6, 7))
    gp, gf = rng.standard_normal((2, 3, 4, 5)), rng.standard_normal((2, 3, 4, 5))
    Ap, Af = S.conserved_changes(o, W, X, 2.5)
    lhs = float((gp * Ap).sum() + (gf * Af).sum())
    do = S.conserved_changes_adjoint(gp, gf, W, X, 2.5, o.shape)
    assert abs(lhs - float((do * o).sum())) < 1e-12 * abs(lhs)


def test_uniform_flux_and_linear_flux_closed_forms():
    """With unit weights a uniform flux has no divergence, a flux growing by c per
    node along an axis removes c from every node; with a weight that is linear
    along x and a uniform coefficient f, the face fluxes grow by f times the slope."""
    o = np.zeros((1, 5, 6, 7, 7))
    one = np.ones((1, 5, 6, 7))
    o[..., 0] = 3.0
    o[..., 4] = -2.0
    Ap, Af = S.conserved_changes(o, one, one, 1.0)
    assert np.abs(Ap).max() == 0.0 and np.abs(Af).max() == 0.0
    o[..., 0] = 0.5 * np.arange(7)[None, None, None, :]
    Ap, _ = S.conserved_changes(o, one, one, 1.0)
    assert np.allclose(Ap, -0.5, rtol=0, atol=1e-15)
    o[...] = 0.0
    o[..., 1] = 2.0                       # uniform y coefficient
    Wy = 1.0 + 0.25 * np.arange(6)[None, None, :, None] * one
    Ap, _ = S.conserved_changes(o, Wy, one, 1.0)
    assert np.allclose(Ap, -2.0 * 0.25, rtol=0, atol=1e-14)
