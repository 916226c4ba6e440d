"""Write the stored expected values of the long parity cases.

Every value here comes from the FP64 oracle alone (``oracle/``, with the
workloads of ``workloads.py``); nothing is taken from the HIP path. The GPU
tests run the same workloads and compare against these files:

* ``bubble_column_500.npz`` -- the 3-D bubble column (D3Q19 128 x 128 x 384,
  density and viscosity ratio 10, Eo = 10, Bi = 1; Sec 3.4 groups) after 500
  steps of the FP64 method (fd_eps 1e-10, SOR tolerance 1e-13): u, rhoN,
  G psi and X phi on the plane y = 63 for z < 128 (the bubble and its wake),
  and the observables after 50, 100, 200 and 500 steps.

* ``shear_deformation_20k.json`` -- the drop in simple shear (D2Q9 512 x 256,
  walls at -/+ 0.02, R = 40, Sec 3.3 groups) at two corners of the parameter
  range (Ca 0.1, Bi 0.1, E0 0.1 and Ca 0.4, Bi 1, E0 0.5), 20 000 FP64 steps:
  the deformation D = (L - B)/(L + B) of the second moments, the centroid and
  the velocity of eq 33 every 1000 steps.

Usage: ``python tests/golden/make_golden.py bubble`` (about 90 minutes on 8
cores), ``... shear CASE`` (one case, about an hour). The output is
deterministic up to the oracle's OpenMP reduction order in the observables
(1e-15 relative).
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

BUBBLE_FILE = os.path.join(HERE, "bubble_column_500.npz")
BUBBLE_CHECKS = (50, 100, 200, 500)
BUBBLE_PLANE_Y = 63
BUBBLE_ZMAX = 128


def bubble_column():
    p, q = W.bubble_rise(precision="fp64")
    o = oracle.Oracle(p).init(q)
    obs = {}
    done = 0
    t0 = time.time()
    for c in BUBBLE_CHECKS:
        o.step(c - done)
        done = c
        obs[c] = o.observables()
        print(f"step {c} ({time.time() - t0:.0f} s): velocity {obs[c]['velocity']}", flush=True)
    rN = o.field("rhoN")
    sl = (slice(0, BUBBLE_ZMAX), BUBBLE_PLANE_Y, slice(None))
    u = o.field("u")
    out = dict(u=np.stack([u[a][sl] for a in range(3)]), rhoN=rN[sl], Gpsi=(o.field("G") * o.field("psi"))[sl],
               Xphi=((1.0 - rN) * o.field("phi"))[sl], initial_total=np.float64(o.initial_total),
               obs=np.array(json.dumps({str(k): v for k, v in obs.items()})))
    np.savez_compressed(BUBBLE_FILE, **out)
    print("wrote", BUBBLE_FILE, flush=True)


SHEAR_FILE = os.path.join(HERE, "shear_deformation_20k.json")
SHEAR_CASES = {"ca0.1_bi0.1_e0.1": dict(Ca=0.1, Bi=0.1, E0=0.1), "ca0.4_bi1_e0.5": dict(Ca=0.4, Bi=1.0, E0=0.5)}
SHEAR_STEPS, SHEAR_EVERY = 20000, 1000


def shear_case(name):
    p, q = W.shear_droplet(precision="fp64", **SHEAR_CASES[name])
    o = oracle.Oracle(p).init(q)
    rec = []
    t0 = time.time()
    for c in range(0, SHEAR_STEPS + 1, SHEAR_EVERY):
        if c:
            o.step(SHEAR_EVERY)
        ob = o.observables()
        rec.append(dict(step=c, deformation=oracle.deformation(ob["second"], 2), centroid=ob["centroid"][:2],
                        velocity=ob["velocity"][:2], psi_av=ob["psi_av"], total_surf=ob["total_surf"]))
        print(f"{name} step {c} ({time.time() - t0:.0f} s): D {rec[-1]['deformation']:.6f}", flush=True)
    table = {}
    if os.path.exists(SHEAR_FILE):
        with open(SHEAR_FILE) as fh:
            table = json.load(fh)
    table[name] = dict(params=SHEAR_CASES[name], steps=SHEAR_STEPS, every=SHEAR_EVERY, records=rec)
    with open(SHEAR_FILE, "w") as fh:
        json.dump(table, fh, indent=1)
        fh.write("\n")
    print("wrote", SHEAR_FILE, flush=True)


if __name__ == "__main__":
    what = sys.argv[1:] or ["bubble"]
    if what[0] == "bubble":
        bubble_column()
    elif what[0] == "shear":
        for name in what[1:] or list(SHEAR_CASES):
            shear_case(name)
