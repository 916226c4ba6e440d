"""Independent NumPy brute-force evaluation of one time step on a tiny periodic
grid, used to check the oracle. Test code only.

It is written differently from the oracle on purpose: whole-array ``np.roll``
shifts instead of per-node ghost lookups, the transformation matrices built
from their defining polynomials (not the printed tables), moment-space
operators as matrix products over the whole grid, and the implicit diffusion
step as a dense matrix solved exactly with ``numpy.linalg.solve``.
"""
from __future__ import annotations

import numpy as np

# Velocity order of the printed transformation matrices (Appendix A).
VEL2 = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (-1, 0, 0), (0, -1, 0),
        (1, 1, 0), (-1, 1, 0), (-1, -1, 0), (1, -1, 0)]
VEL3 = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
        (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
        (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
        (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]


def lattice(three: bool):
    e = np.array(VEL3 if three else VEL2, dtype=np.int64)
    c2 = (e ** 2).sum(1)
    if three:
        w = np.where(c2 == 0, 1 / 3, np.where(c2 == 1, 1 / 18, 1 / 36))
        x, y, z = e[:, 0], e[:, 1], e[:, 2]
        rows = [np.ones_like(x), x, y, z, c2, 2 * x * x - y * y - z * z, y * y - z * z,
                x * y, x * z, y * z, x * x * y, x * y * y, x * x * z, x * z * z, y * y * z, y * z * z,
                x * x * y * y, x * x * z * z, y * y * z * z]
    else:
        w = np.where(c2 == 0, 4 / 9, np.where(c2 == 1, 1 / 9, 1 / 36))
        x, y = e[:, 0], e[:, 1]
        # Lallemand-Luo orthogonal basis: 1, e, eps, jx, qx, jy, qy, pxx, pxy
        rows = [np.ones_like(x), -4 + 3 * c2, (8 - 21 * c2 + 9 * c2 * c2) // 2, x, (-5 + 3 * c2) * x,
                y, (-5 + 3 * c2) * y, x * x - y * y, x * y]
    M = np.array(rows, dtype=np.float64)
    return e, w.astype(np.float64), M


def shift(a, d):
    """a(x + d) on a periodic grid; a has shape (..., nz, ny, nx)."""
    return np.roll(a, shift=(-d[2], -d[1], -d[0]), axis=(-3, -2, -1))


def grad(chi, e, w, D):
    out = []
    for a in range(D):
        acc = np.zeros_like(chi)
        for i in range(len(w)):
            if e[i, a]:
                acc = acc + w[i] * e[i, a] * shift(chi, e[i])
        out.append(3.0 * acc)
    return np.array(out)


def meq(rho, u, alpha, cs2, D):
    ux, uy = u[0], u[1]
    uz = u[2] if D == 3 else np.zeros_like(ux)
    u2 = ux * ux + uy * uy + uz * uz
    if D == 2:
        return np.array([rho, rho * (-3.6 * alpha - 0.4 + 3 * u2), rho * (5.4 * alpha - 1.4 - 3 * u2),
                         rho * ux, rho * (-1.8 * alpha - 0.2) * ux, rho * uy, rho * (-1.8 * alpha - 0.2) * uy,
                         rho * (ux * ux - uy * uy), rho * ux * uy])
    p = rho * cs2
    base = 1 - alpha - u2
    return np.array([rho, rho * ux, rho * uy, rho * uz, 3 * p + rho * u2,
                     rho * (2 * ux * ux - uy * uy - uz * uz), rho * (uy * uy - uz * uz),
                     rho * ux * uy, rho * ux * uz, rho * uy * uz,
                     p * uy, p * ux, p * uz, p * ux, p * uz, p * uy,
                     rho * (base + 2 * (ux * ux + uy * uy)) / 6, rho * (base + 2 * (ux * ux + uz * uz)) / 6,
                     rho * (base + 2 * (uy * uy + uz * uz)) / 6])


def weno_div(Psi, u, D, eps, upwind_eps=0.0):
    out = np.zeros_like(Psi[0])
    for a in range(D):
        d = np.zeros(3, dtype=int)

        def P(k):
            dd = d.copy()
            dd[a] = k
            return shift(Psi[a], dd)
        p = {k: P(k) for k in range(-2, 3)}
        dp = {k: p[k + 1] - p[k] for k in (-2, -1, 0, 1)}
        d2 = {k: p[k + 1] - 2 * p[k] + p[k - 1] for k in (-1, 0, 1)}
        wm = 1 / (1 + 2 * ((eps + d2[-1] ** 2) / (eps + d2[0] ** 2)) ** 2)
        wp = 1 / (1 + 2 * ((eps + d2[1] ** 2) / (eps + d2[0] ** 2)) ** 2)
        Dm = 0.5 * (dp[-1] + dp[0]) - 0.5 * wm * (dp[-2] - 2 * dp[-1] + dp[0])
        Dp = 0.5 * (dp[-1] + dp[0]) - 0.5 * wp * (dp[1] - 2 * dp[0] + dp[-1])
        ua = u[a]
        ue = upwind_eps
        out = out + np.where(ua > ue, Dm, np.where(ua < -ue, Dp, 0.5 * (Dm + Dp)))
    return out


def implicit_matrix(W, Dc, D):
    """Dense matrix of diag(W) - (Dc/2) L_W on a periodic grid (eq 28)."""
    shape = W.shape
    N = W.size
    idx = np.arange(N).reshape(shape)
    A = np.diag(W.reshape(-1).copy())
    for a in range(D):
        for s in (-1, 1):
            d = np.zeros(3, dtype=int)
            d[a] = s
            nb = shift(idx, d).reshape(-1)
            wf = 0.5 * (W.reshape(-1) + W.reshape(-1)[nb])
            for n in range(N):
                A[n, n] += 0.5 * Dc * wf[n]
                A[n, nb[n]] -= 0.5 * Dc * wf[n]
    return A


def step(p, st):
    """One step from state dict st = {fR, fB (Q,nz,ny,nx), psi, phi, Sprev, Bprev, step, M0}."""
    three = p["lattice"] == 1
    D = 3 if three else 2
    e, w, M = lattice(three)
    Minv = np.linalg.inv(M)
    Q = len(w)
    alpha = np.array([p["alphaR"], 1 - p["rhoR0"] / p["rhoB0"] * (1 - p["alphaR"])])
    cs2 = (0.5 if three else 0.6) * (1 - alpha)
    fR, fB = st["fR"], st["fB"]
    psi, phi = st["psi"], st["phi"]
    rR, rB = fR.sum(0), fB.sum(0)
    rho = rR + rB
    rN = (rR / p["rhoR0"] - rB / p["rhoB0"]) / (rR / p["rhoR0"] + rB / p["rhoB0"])
    f = fR + fB
    jv = np.einsum("ia,i...->a...", e[:, :D].astype(float), f)
    g = grad(rN, e, w, D)
    G = np.sqrt((g ** 2).sum(0))
    nrm = -g / np.sqrt(G ** 2 + p["eps_n"] ** 2)
    kappa = -sum(grad(nrm[a], e, w, D)[a] for a in range(D))
    gpsi = grad(psi, e, w, D)
    E0, s0, pinf = p["E0"], p["sigma0"], p["psi_inf"]
    smin = p["sigma_min_ratio"] * s0
    if E0 == 0:
        Fs = -0.5 * s0 * kappa * g
    else:
        cmc = pinf * (1 - np.exp(-(1 - p["sigma_min_ratio"]) / E0))
        below = psi < cmc
        sig = s0 * (1 + E0 * np.log(np.where(below, 1 - psi / pinf, 1.0)))
        ndg = (nrm * gpsi).sum(0)
        mar = 0.5 * G * s0 * E0 / np.where(below, pinf - psi, 1.0)
        Fs = np.where(below, -0.5 * sig * kappa * g - mar * (gpsi - ndg * nrm), -0.5 * smin * kappa * g)
    Fb = np.array([(rho - p["rhoB0"]) * p["gravity"][a] for a in range(D)])
    F = Fs + Fb
    u = (jv + 0.5 * F) / rho
    mu = 1 / ((1 + rN) / (2 * p["muR0"]) + (1 - rN) / (2 * p["muB0"]))
    sv = 1 / (mu / (rR * cs2[0] + rB * cs2[1]) + 0.5)

    m = np.einsum("ri,i...->r...", M, f)
    me = meq(rR, u, alpha[0], cs2[0], D) + meq(rB, u, alpha[1], cs2[1], D)
    C = np.zeros_like(m)
    for k, rk in enumerate((rR, rB)):
        coef = (1.8 * alpha[k] - 0.8) if not three else ((1 - cs2[k]) if p["q_literal"] else (1 - 3 * cs2[k]))
        Qa = [coef * grad(rk * u[a], e, w, D)[a] for a in range(D)]
        if three:
            C[4] += Qa[0] + Qa[1] + Qa[2]
            C[5] += 2 * Qa[0] - Qa[1] - Qa[2]
            C[6] += Qa[1] - Qa[2]
        else:
            C[1] += 3 * Qa[0] + 3 * Qa[1]
            C[7] += Qa[0] - Qa[1]
    ef = e[:, :D].astype(float)
    eu = np.einsum("ia,a...->i...", ef, u)
    eF = np.einsum("ia,a...->i...", ef, F)
    uF = (u * F).sum(0)
    Fi = w[:, None, None, None] * (3 * (eF - uF) + 9 * eu * eF)
    Fm = np.einsum("ri,i...->r...", M, Fi)
    if three:
        S = np.ones((Q,) + sv.shape)
        S[5:10] = sv
    else:
        S = np.array([np.full_like(sv, v) for v in (0, 1.25, 1.14, 0, 1.6, 0, 1.6, 0, 0)])
        S[7] = sv
        S[8] = sv
    dm = -S * (m - me) + (1 - 0.5 * S) * (C + Fm)
    fdag = f + np.einsum("ir,r...->i...", Minv, dm)
    ce = np.where(G > 0, np.einsum("ia,a...->i...", ef, g) / np.where(G > 0, G, 1), 0.0)
    if p.get("recolour_literal", 0):
        wgt = w[:, None, None, None] * np.ones_like(rho)
    else:
        zero = np.zeros((D,) + rho.shape)
        wgt = (np.einsum("ir,r...->i...", Minv, meq(rR, zero, alpha[0], cs2[0], D))
               + np.einsum("ir,r...->i...", Minv, meq(rB, zero, alpha[1], cs2[1], D))) / rho
    rec = p["beta"] * wgt * (rR * rB / rho) * ce
    fRr = rR / rho * fdag + rec
    fBr = rB / rho * fdag - rec
    fR1 = np.array([shift(fRr[i], -e[i]) for i in range(Q)])
    fB1 = np.array([shift(fBr[i], -e[i]) for i in range(Q)])
    out = dict(fR=fR1, fB=fB1, psi=psi.copy(), phi=phi.copy(), Sprev=st["Sprev"].copy(),
               Bprev=st["Bprev"].copy(), step=st["step"] + 1, M0=st["M0"], u=u, F=F, fdag=fdag)
    if not p["fd_enable"]:
        return out
    rR1, rB1 = fR1.sum(0), fB1.sum(0)
    rN1 = (rR1 / p["rhoR0"] - rB1 / p["rhoB0"]) / (rR1 / p["rhoR0"] + rB1 / p["rhoB0"])
    eps = p.get("fd_eps", 0.0)
    G1 = np.sqrt((grad(rN1, e, w, D) ** 2).sum(0)) + eps
    psi1, phi1, Sn, Bn, rhsP, Mt = fd_update(p, st, G + eps, 1 - rN + eps, G1, 1 - rN1 + eps, u, D)
    out.update(psi=psi1, phi=phi1, Sprev=Sn, Bprev=Bn, G1=G1, rhsP=rhsP, Mt=Mt)
    return out


def fd_update(p, st, Gw, X0, G1, X1, u, D):
    """One FD transport update (eqs 20-28) from psi, phi, Sprev, Bprev of st with
    the weights Gw, X0 (time t) and G1, X1 (time t+1), dense direct solves."""
    psi, phi = st["psi"], st["phi"]
    pinf = p["psi_inf"]
    divPsi = weno_div(psi * Gw * u, u, D, p["weno_eps"], p.get("upwind_eps", 0.0))
    divPhi = weno_div(phi * X0 * u, u, D, p["weno_eps"], p.get("upwind_eps", 0.0))
    if p["source_mode"] == 1:
        jj = p["ra"] * pinf * phi
    else:
        jj = p["ra"] * phi * (pinf - psi) - p["rd"] * psi
    Sn = -divPsi + Gw * jj
    Bn = -divPhi - Gw * jj
    if st["step"] == 0:
        eS, eB = Sn, Bn
    else:
        eS, eB = 1.5 * Sn - 0.5 * st["Sprev"], 1.5 * Bn - 0.5 * st["Bprev"]
    A0p = implicit_matrix(Gw, -p["Ds"], D)      # diag(G) + (Ds/2) L_G
    A0f = implicit_matrix(X0, -p["Db"], D)
    rhsP = A0p @ psi.reshape(-1) + eS.reshape(-1)
    rhsF = A0f @ phi.reshape(-1) + eB.reshape(-1)
    res = []
    for W1, Dc, rhs, old in ((G1, p["Ds"], rhsP, psi), (X1, p["Db"], rhsF, phi)):
        A = implicit_matrix(W1, Dc, D)
        dead = np.diag(A) <= 0
        A[dead, :] = 0
        A[dead, dead] = 1
        b = rhs.copy()
        b[dead] = old.reshape(-1)[dead]
        res.append(np.linalg.solve(A, b).reshape(psi.shape))
    psi1, phi1 = res
    Mt = (G1 * psi1 + X1 * phi1).sum()
    if p["rescale"] and st["M0"] != 0:
        psi1, phi1 = psi1 * st["M0"] / Mt, phi1 * st["M0"] / Mt
    return psi1, phi1, Sn, Bn, rhsP, Mt


def fd_substeps(p, st, k):
    """k FD updates with the flow frozen at state st (rhoN, G and u of its
    populations; the new-level weights equal the old ones)."""
    three = p["lattice"] == 1
    D = 3 if three else 2
    base = step(dict(p, fd_enable=0), st)     # u of the current populations
    e, w, _ = lattice(three)
    rR, rB = st["fR"].sum(0), st["fB"].sum(0)
    rN = (rR / p["rhoR0"] - rB / p["rhoB0"]) / (rR / p["rhoR0"] + rB / p["rhoB0"])
    eps = p.get("fd_eps", 0.0)
    Gw = np.sqrt((grad(rN, e, w, D) ** 2).sum(0)) + eps
    X0 = 1 - rN + eps
    cur = dict(st)
    for _ in range(k):
        psi1, phi1, Sn, Bn, _, _ = fd_update(p, cur, Gw, X0, Gw, X0, base["u"], D)
        cur = dict(cur, psi=psi1, phi=phi1, Sprev=Sn, Bprev=Bn)
    return cur
