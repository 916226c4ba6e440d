"""Field-by-field comparison of the GPU solver with the oracle (test helper).

Errors are max-norm errors relative to the largest magnitude of the oracle's
field. psi and phi are compared through the conserved densities G psi and
X phi (G = |grad rhoN|, X = 1 - rhoN): where G (or X) vanishes the implicit
rows are nearly empty and psi (phi) is only weakly determined, while the
weighted fields are bounded by the solver residual."""
from __future__ import annotations

import sys

import numpy as np


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(b).max(), 1e-300))


def state_errors(s, o, names=("f", "rhoR", "rhoB", "rhoN", "u", "Gpsi", "Xphi")):
    out = {}
    for n in names:
        if n == "Gpsi":
            a, b = s.field("G") * s.field("psi"), o.field("G") * o.field("psi")
        elif n == "Xphi":
            a, b = (1 - s.field("rhoN")) * s.field("phi"), (1 - o.field("rhoN")) * o.field("phi")
        else:
            a, b = s.field(n), o.field(n)
        out[n] = rel(a, b)
    return out


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()
