"""Synthetic workloads shared by the HIP path and the oracle.

This module holds only problem set-ups: lattice parameters, initial geometry
and seeded random draws. It contains none of the method's arithmetic. The
mapping from the paper's dimensionless groups to lattice parameters follows
their definitions in Sec 3.3 (Ca, Re, Pe_s, Pe_b, Bi, k, h, x_in) and Sec 3.4
(Eo, Mo); each derived value is computed in the open below.

A workload is a pair of plain dicts ``(params, init)``. ``params`` mirrors the
C parameter blocks of both implementations field by field; ``init`` describes
the initial drops and concentrations.
"""
from __future__ import annotations

import copy
import json
import math
import os
import sys

import numpy as np

D2Q9, D3Q19 = 0, 1
PERIODIC, WALL = 0, 1
PRECISIONS = ("fp64", "fp32", "fp16dev", "bf16dev")

BASE_PARAMS = dict(
    lattice=D2Q9, nx=64, ny=64, nz=1,
    bc=[PERIODIC, PERIODIC, PERIODIC],
    wall_u=[[0.0, 0.0, 0.0] for _ in range(6)],   # -x,+x,-y,+y,-z,+z
    rhoR0=1.0, rhoB0=1.0, muR0=1.0 / 6.0, muB0=1.0 / 6.0,
    alphaR=None,                 # None: standard value (4/9 in 2-D, 1/3 in 3-D)
    beta=0.7,                    # recolouring segregation parameter (Sec 2.1)
    sigma0=0.01, E0=0.5, psi_inf=1.0, sigma_min_ratio=0.1,
    Ds=0.02, Db=0.02, ra=0.1, rd=0.05, source_mode=0,
    gravity=[0.0, 0.0, 0.0],
    sor_omega=1.0, sor_tol=1e-13, sor_max_sweeps=60,   # omega: 1.2 in Sec 2.2; the solve is converged either way
    weno_eps=1e-6, rescale=1, fd_enable=1, q_literal=0, eps_n=1e-12, recolour_literal=0,
    fd_eps=1e-10,                # background support of the FD weights (FP32 modes: 1e-6)
    upwind_eps=1e-12,            # |u| band in which the WENO upwind weights are 1/2 each
    buoyancy_ref=0,              # buoyancy reference density: 0 = rhoB0 (Sec 3.4), 1 = domain mean
    eos_mode=0,                  # 0: Langmuir eq 8 with the CMC floor; 1: linear law of Sec 3.2
    precision="fp64",
)

BASE_INIT = dict(drops=[], width=3.0, psi0=0.0, phi0_out=0.0, phi0_in=0.0, shear_rate=0.0)


def finalize(params: dict) -> dict:
    """Fill defaults that depend on the lattice (the standard alpha)."""
    p = copy.deepcopy(BASE_PARAMS)
    p.update(copy.deepcopy(params))
    if p["alphaR"] is None:
        p["alphaR"] = 4.0 / 9.0 if p["lattice"] == D2Q9 else 1.0 / 3.0
    if p["lattice"] == D2Q9:
        p["nz"] = 1
    if p["precision"] != "fp64" and "sor_tol" not in params:
        p["sor_tol"] = 1e-6
    if p["precision"] != "fp64" and "fd_eps" not in params:
        p["fd_eps"] = 1e-6
    return p


def make(params: dict, init: dict):
    q = copy.deepcopy(BASE_INIT)
    q.update(copy.deepcopy(init))
    return finalize(params), q


# ----------------------------------------------------------------------------
# Stationary droplet with adsorption (periodic D2Q9 box, 128 x 128, R = 25).
# "C = 0.1 in units of the Langmuir constant": with K = ra/rd = 2 the raw bulk
# concentration is 0.05 (K phi = 0.1); literal_c=True takes 0.1 instead.
# ----------------------------------------------------------------------------
def droplet_adsorption(n=128, radius=25.0, precision="fp64", literal_c=False, **over):
    params = dict(lattice=D2Q9, nx=n, ny=n, rhoR0=1.0, rhoB0=1.0,
                  muR0=1.0 / 6.0, muB0=1.0 / 6.0, sigma0=0.01, E0=0.5, psi_inf=1.0,
                  Ds=0.02, Db=0.02, ra=0.1, rd=0.05, precision=precision)
    params.update(over)
    ny = params.get("ny", n)
    init = dict(drops=[((n - 1) / 2.0, (ny - 1) / 2.0, 0.0, radius)], width=3.0, psi0=0.0,
                phi0_out=0.1 if literal_c else 0.05, phi0_in=0.0)
    return make(params, init)


# ----------------------------------------------------------------------------
# Droplet in simple shear between walls moving at -/+ u_w (Sec 3.3 groups).
# U = shear * R (the paper's U = u_w/2 when H = 4R), L = R.
# ----------------------------------------------------------------------------
def shear_droplet(nx=512, ny=256, radius=40.0, u_w=0.02, Ca=0.2, Re=1.0, lam=1.0,
                  Pe_s=10.0, Pe_b=1.0, Bi=1.0, E0=0.3, x_in=0.5, h=0.5, k=1.0,
                  precision="fp64", **over):
    shear = 2.0 * u_w / ny
    U = shear * radius
    muB = U * radius / Re                       # Re = rho U L / mu, rho = 1
    sigma0 = muB * U / Ca                       # Ca = mu U / sigma0
    psi0 = x_in * 1.0                           # x_in = psi0 / psi_inf
    phi0 = psi0 / (h * radius)                  # h = psi0 / (phi0 R)
    rd = Bi * shear                             # Bi = rd / shear
    ra = k * rd / phi0                          # k = ra phi0 / rd
    params = dict(lattice=D2Q9, nx=nx, ny=ny, bc=[PERIODIC, WALL, PERIODIC],
                  wall_u=[[0, 0, 0], [0, 0, 0], [-u_w, 0, 0], [u_w, 0, 0], [0, 0, 0], [0, 0, 0]],
                  rhoR0=1.0, rhoB0=1.0, muR0=lam * muB, muB0=muB, sigma0=sigma0, E0=E0,
                  psi_inf=1.0, Ds=U * radius / Pe_s, Db=U * radius / Pe_b, ra=ra, rd=rd,
                  precision=precision)
    params.update(over)
    init = dict(drops=[((nx - 1) / 2.0, (ny - 1) / 2.0, 0.0, radius)], width=3.0, psi0=psi0,
                phi0_out=phi0, phi0_in=0.0, shear_rate=shear)
    return make(params, init)


# ----------------------------------------------------------------------------
# Buoyancy-driven bubble rise in a walled column (Sec 3.4 groups), D3Q19.
# Eo = drho g (2R)^2 / sigma, Mo = drho g mu^4 / (rho^2 sigma^3) fixes mu at
# Eo = 1. Reading for the surfactant time scale: t_ref = sqrt(2R/g) at the
# Eo of the run, U = R/t_ref, L = R, Bi = rd t_ref.
# ----------------------------------------------------------------------------
def bubble_rise(nx=128, ny=128, nz=384, radius=16.0, Eo=10.0, Mo=0.1, Bi=1.0,
                E0=0.5, Pe=10.0, k=1.0, phi0=0.5, sigma0=0.004, rho_ratio=0.1,
                mu_ratio=0.1, clean=False, lattice=D3Q19, precision="bf16dev", zc=None, **over):
    rhoR0, rhoB0 = rho_ratio, 1.0
    drho = rhoB0 - rhoR0
    g1 = 1.0 * sigma0 / (drho * (2 * radius) ** 2)      # g at Eo = 1
    muB = (Mo * rhoB0 ** 2 * sigma0 ** 3 / (drho * g1)) ** 0.25
    g = Eo * sigma0 / (drho * (2 * radius) ** 2)
    t_ref = math.sqrt(2 * radius / g)
    rd = 0.0 if clean else Bi / t_ref
    ra = 0.0 if clean else k * rd / phi0
    D = radius * (radius / t_ref) / Pe
    grav = [0.0, 0.0, 0.0]
    if lattice == D3Q19:
        grav[2] = -g
        bc = [WALL, WALL, PERIODIC]
        centre = ((nx - 1) / 2.0, (ny - 1) / 2.0, zc if zc is not None else 3.0 * radius)
    else:
        grav[1] = -g
        bc = [WALL, PERIODIC, PERIODIC]
        centre = ((nx - 1) / 2.0, zc if zc is not None else 3.0 * radius, 0.0)
    params = dict(lattice=lattice, nx=nx, ny=ny, nz=nz if lattice == D3Q19 else 1, bc=bc,
                  rhoR0=rhoR0, rhoB0=rhoB0, muR0=mu_ratio * muB, muB0=muB,
                  sigma0=sigma0, E0=0.0 if clean else E0, psi_inf=1.0,
                  Ds=D, Db=D, ra=ra, rd=rd, gravity=grav, precision=precision)
    params.update(over)
    init = dict(drops=[(centre[0], centre[1], centre[2], radius)], width=3.0, psi0=0.0,
                phi0_out=0.0 if clean else phi0, phi0_in=0.0)
    return make(params, init)


# ----------------------------------------------------------------------------
# Adsorption onto a stationary 3-D droplet (Sec 3.1). The paper simulates one
# octant of a 5R cube with symmetry planes through the drop centre and periodic
# far faces; mirror planes at 0 and periodicity 5R place a drop every 5R, so the
# same problem is a whole drop at the centre of a periodic 5R cube (8 times the
# nodes, no symmetry boundary). Both fluids of density 1 and viscosity 0.1,
# sigma0 = 0.1, E0 = 0.5, Ds = Db = 0.1, the adsorption-only source
# j = ra psi_inf phi with ra = 0.2 (source_mode = 1), psi0 = 0, phi0 = 0.0005
# in the blue fluid and 0 in the drop; psi_inf = 1 (not given in the paper).
# ----------------------------------------------------------------------------
def adsorption_3d(R=30, precision="fp64", **over):
    n = 5 * R
    params = dict(lattice=D3Q19, nx=n, ny=n, nz=n, bc=[PERIODIC, PERIODIC, PERIODIC],
                  rhoR0=1.0, rhoB0=1.0, muR0=0.1, muB0=0.1, sigma0=0.1, E0=0.5, psi_inf=1.0,
                  Ds=0.1, Db=0.1, ra=0.2, rd=0.0, source_mode=1, precision=precision)
    params.update(over)
    c = (n - 1) / 2.0
    init = dict(drops=[(c, c, c, float(R))], width=3.0, psi0=0.0, phi0_out=0.0005, phi0_in=0.0)
    return make(params, init)


# ----------------------------------------------------------------------------
# Droplet migration in an imposed surfactant gradient (Sec 3.2): a red drop of
# radius R at the centre of a (w R) x (w R) x 10R box with walls in x and y and
# periodic z; both fluids of density 1 and viscosity 0.1, sigma0 = 0.001,
# E0 = 0.5 with the linear tension law (eos_mode = 1), Ds = 0.1. The surfactant
# is insoluble and held: the FD part is off and psi is the linear ramp of eq 31
# (migration_psi), so the centre of the drop sits at psi = x_in psi_inf = 0.5.
# ----------------------------------------------------------------------------
def ygb_migration(R=30, width=5, precision="fp32", **over):
    nx = ny = int(round(width * R))
    nz = 10 * R
    params = dict(lattice=D3Q19, nx=nx, ny=ny, nz=nz, bc=[WALL, WALL, PERIODIC],
                  rhoR0=1.0, rhoB0=1.0, muR0=0.1, muB0=0.1, sigma0=0.001, E0=0.5, psi_inf=1.0,
                  Ds=0.1, Db=0.1, ra=0.0, rd=0.0, fd_enable=0, eos_mode=1, precision=precision)
    params.update(over)
    init = dict(drops=[((nx - 1) / 2.0, (ny - 1) / 2.0, nz / 2.0, float(R))], width=3.0, psi0=0.5,
                phi0_out=0.0, phi0_in=0.0)
    return make(params, init)


def migration_psi(p):
    """Eq 31 on the nodes: psi = psi_inf z / L_z with L_z = nz (node z at height
    z; the ramp restarts at the periodic seam, far from the drop). Shape
    (nz, ny, nx)."""
    z = np.arange(p["nz"], dtype=np.float64)
    col = p["psi_inf"] * z / p["nz"]
    return np.broadcast_to(col[:, None, None], (p["nz"], p["ny"], p["nx"])).copy()


# ----------------------------------------------------------------------------
# Periodic box with several bubbles at seeded non-overlapping positions (the
# snapshot source of the learned surrogate): D3Q19, the bubble column's
# parameters (density and viscosity ratio 10, Mo at Eo = 1, Pe = 10, k = 1,
# phi0 = 0.5, E0 = 0.5), Eo and Bi as given. Positions are drawn in order with
# numpy's default_rng(seed) inside the box, rejecting any bubble closer than 1.5
# diameters (periodic distance) to an earlier one.
# ----------------------------------------------------------------------------
def multi_bubble(n=256, count=8, diameter=24.0, Eo=10.0, Bi=1.0, seed=0, precision="fp32", **over):
    radius = diameter / 2.0
    rng = np.random.default_rng(seed)
    centres = []
    tries = 0
    while len(centres) < count:
        tries += 1
        if tries > 100000:
            raise ValueError("bubbles do not fit")
        c = rng.uniform(radius + 2.0, n - radius - 2.0, 3)   # whole bubbles (the initial profile does not wrap)
        ok = True
        for d in centres:
            dd = np.abs(c - np.asarray(d))
            dd = np.minimum(dd, n - dd)
            if float(np.sqrt((dd * dd).sum())) < 1.5 * diameter:
                ok = False
                break
        if ok:
            centres.append(tuple(float(v) for v in c))
    p, q = bubble_rise(nx=n, ny=n, nz=n, radius=radius, Eo=Eo, Bi=Bi, precision=precision, **over)
    p["bc"] = [PERIODIC, PERIODIC, PERIODIC]
    q = dict(q, drops=[(x, y, z, radius) for x, y, z in centres])
    return p, q


# ----------------------------------------------------------------------------
# Seeded batch of uneven 2-D bubble-rise instances (draw order W, H, Eo, Bi).
# ----------------------------------------------------------------------------
def batch_manifest(count=64, seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        W = int(rng.integers(128, 257))
        H = int(rng.integers(256, 769))
        Eo = float(math.exp(rng.uniform(math.log(1.0), math.log(50.0))))
        Bi = float(math.exp(rng.uniform(math.log(0.01), math.log(10.0))))
        out.append(dict(W=W, H=H, Eo=Eo, Bi=Bi))
    return out


# The 64 draws of batch_manifest(64, 0), stored once so that every run uses the
# same instances (rewrite with ``python workloads.py --write-manifest``).
BATCH_MANIFEST = os.path.join(os.path.dirname(os.path.abspath(__file__)), "bubble_rise_batch64.json")


def load_manifest(path: str = BATCH_MANIFEST):
    with open(path) as fh:
        return json.load(fh)["instances"]


def batch_instances(manifest, precision="bf16dev", scale=1.0):
    """2-D bubble-rise instances of a manifest: a W x H column walled in x,
    periodic in y, bubble diameter W / 5, the 3-D column's other parameters.
    ``scale`` shrinks W and H (small test batches of the same mix)."""
    out = []
    for m in manifest:
        W = max(16, int(round(m["W"] * scale)))
        H = max(32, int(round(m["H"] * scale)))
        out.append(bubble_rise(nx=W, ny=H, radius=W / 10.0, Eo=m["Eo"], Bi=m["Bi"], lattice=D2Q9,
                               precision=precision))
    return out


# ----------------------------------------------------------------------------
# Random states for property tests: populations near equilibrium weights with
# a colour split, psi in [0, 0.5 psi_inf], phi in [0, 0.1]. Pure data.
# ----------------------------------------------------------------------------
def random_state(shape_q_nodes, weights, seed, amp=0.02, red_share=None):
    rng = np.random.default_rng(seed)
    Q, N = shape_q_nodes
    base = np.asarray(weights, dtype=np.float64)[:, None] * np.ones((1, N))
    f = base * (1.0 + amp * rng.standard_normal((Q, N)))
    share = rng.uniform(0.0, 1.0, N) if red_share is None else np.full(N, red_share)
    return f * share[None, :], f * (1.0 - share[None, :])


def random_scalar(n, seed, lo=0.0, hi=1.0):
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, n)


# Named configurations (lattice sizes as in the measurement plan).
def config(name: str, precision: str | None = None):
    if name == "droplet128":
        return droplet_adsorption(precision=precision or "fp64")
    if name == "shear512x256":
        return shear_droplet(precision=precision or "fp64")
    if name == "bubble128x128x384":
        return bubble_rise(precision=precision or "bf16dev")
    raise KeyError(name)


if __name__ == "__main__":
    if sys.argv[1:] == ["--write-manifest"]:
        with open(BATCH_MANIFEST, "w") as fh:
            json.dump(dict(seed=0, count=64, draws="W ~ U{128..256}, H ~ U{256..768}, Eo ~ logU[1, 50], "
                                                   "Bi ~ logU[0.01, 10], in that order per instance",
                           instances=batch_manifest(64, 0)), fh, indent=1)
            fh.write("\n")
