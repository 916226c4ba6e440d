"""ctypes wrapper of the FP64 CPU oracle (``lbfd_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of the benchmark. The product package never imports it.

The wrapper declares its own C structures; it shares no header with the HIP
library. Parameters come from the plain dicts of ``workloads``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbfd_oracle.c")
_SO = os.path.join(_HERE, "liblbfd_oracle.so")

FIELDS = dict(f=0, fR=1, fB=2, rhoR=3, rhoB=4, rhoN=5, u=6, psi=7, phi=8, force=9, G=10,
              Sprev=11, Bprev=12, kappa=13)
PRECISIONS = {"fp64": 0}


def build(verbose=False):
    """Compile the oracle with plain FP64 semantics (no contraction, no fast-math)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-std=c11", "-Wall", "-o", _SO + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(_SO + ".tmp", _SO)
    return _SO


class _Params(C.Structure):
    _fields_ = [
        ("lattice", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("bc", C.c_int32 * 3), ("wall_u", (C.c_double * 3) * 6),
        ("rhoR0", C.c_double), ("rhoB0", C.c_double), ("muR0", C.c_double), ("muB0", C.c_double),
        ("alphaR", C.c_double), ("beta", C.c_double),
        ("sigma0", C.c_double), ("E0", C.c_double), ("psi_inf", C.c_double),
        ("sigma_min_ratio", C.c_double),
        ("Ds", C.c_double), ("Db", C.c_double), ("ra", C.c_double), ("rd", C.c_double),
        ("source_mode", C.c_int32), ("gravity", C.c_double * 3),
        ("sor_omega", C.c_double), ("sor_tol", C.c_double), ("sor_max_sweeps", C.c_int32),
        ("weno_eps", C.c_double), ("rescale", C.c_int32), ("fd_enable", C.c_int32),
        ("q_literal", C.c_int32), ("eps_n", C.c_double), ("recolour_literal", C.c_int32),
        ("fd_eps", C.c_double), ("upwind_eps", C.c_double), ("buoyancy_ref", C.c_int32),
        ("eos_mode", C.c_int32),
    ]


class _Init(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("cx", C.c_double * 16), ("cy", C.c_double * 16), ("cz", C.c_double * 16),
        ("r", C.c_double * 16), ("width", C.c_double), ("psi0", C.c_double),
        ("phi0_out", C.c_double), ("phi0_in", C.c_double), ("shear_rate", C.c_double),
    ]


class _Obs(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("mass_R", C.c_double), ("mass_B", C.c_double),
        ("total_surf", C.c_double), ("drift_pre", C.c_double),
        ("velocity", C.c_double * 3), ("centroid", C.c_double * 3), ("second", C.c_double * 6),
        ("wsum", C.c_double), ("nsum", C.c_double),
        ("psi_av", C.c_double), ("psi_min", C.c_double), ("psi_max", C.c_double),
        ("p_in", C.c_double), ("p_out", C.c_double),
        ("sor_sweeps", C.c_int32 * 2), ("status", C.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_SO)
        P = C.POINTER
        dp = P(C.c_double)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [P(_Params)]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_init.argtypes = [C.c_void_p, P(_Init)]
        L.orc_step.argtypes = [C.c_void_p, C.c_int64]
        L.orc_fd_substeps.argtypes = [C.c_void_p, C.c_int64]
        L.orc_nodes.restype = C.c_int64
        L.orc_nodes.argtypes = [C.c_void_p]
        L.orc_lattice_q.argtypes = [C.c_void_p]
        L.orc_threads.restype = C.c_int
        L.orc_threads.argtypes = []
        L.orc_set_threads.restype = None
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_initial_total.restype = C.c_double
        L.orc_initial_total.argtypes = [C.c_void_p]
        L.orc_get_field.argtypes = [C.c_void_p, C.c_int, dp]
        L.orc_set_field.argtypes = [C.c_void_p, C.c_int, dp]
        L.orc_set_clock.argtypes = [C.c_void_p, C.c_int64, C.c_double]
        L.orc_observables.argtypes = [C.c_void_p, P(_Obs)]
        L.orc_lattice.argtypes = [C.c_void_p, P(C.c_int), P(C.c_int), P(C.c_int), dp, dp, dp, dp, dp]
        L.orc_moment_eq.argtypes = [C.c_void_p, C.c_int, C.c_double, dp, dp]
        L.orc_sigma.restype = C.c_double
        L.orc_sigma.argtypes = [C.c_void_p, C.c_double]
        L.orc_op_deriv.argtypes = [C.c_void_p, dp, C.c_int, C.c_int, dp]
        L.orc_op_weno_div.argtypes = [C.c_void_p, dp, dp, dp]
        L.orc_op_diffusion.argtypes = [C.c_void_p, dp, dp, dp]
        L.orc_op_solve.argtypes = [C.c_void_p, dp, C.c_double, dp, dp]
        L.orc_collide_only.argtypes = [C.c_void_p, dp, dp, dp]
        _lib = L
    return _lib


def _ptr(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def threads() -> int:
    """OpenMP threads the oracle's node loops use."""
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's node loops (timing runs)."""
    lib().orc_set_threads(int(n))


def params_struct(p: dict) -> _Params:
    s = _Params()
    s.lattice, s.nx, s.ny, s.nz = p["lattice"], p["nx"], p["ny"], p["nz"]
    for a in range(3):
        s.bc[a] = p["bc"][a]
        s.gravity[a] = p["gravity"][a]
    for w in range(6):
        for a in range(3):
            s.wall_u[w][a] = p["wall_u"][w][a]
    for k in ("rhoR0", "rhoB0", "muR0", "muB0", "alphaR", "beta", "sigma0", "E0", "psi_inf",
              "sigma_min_ratio", "Ds", "Db", "ra", "rd", "sor_omega", "sor_tol", "weno_eps", "eps_n", "fd_eps", "upwind_eps"):
        setattr(s, k, float(p[k]))
    for k in ("source_mode", "sor_max_sweeps", "rescale", "fd_enable", "q_literal", "recolour_literal"):
        setattr(s, k, int(p[k]))
    s.buoyancy_ref = int(p.get("buoyancy_ref", 0))
    s.eos_mode = int(p.get("eos_mode", 0))
    return s


def init_struct(q: dict) -> _Init:
    s = _Init()
    s.n = len(q["drops"])
    for d, (cx, cy, cz, r) in enumerate(q["drops"]):
        s.cx[d], s.cy[d], s.cz[d], s.r[d] = cx, cy, cz, r
    s.width, s.psi0, s.phi0_out, s.phi0_in = q["width"], q["psi0"], q["phi0_out"], q["phi0_in"]
    s.shear_rate = q.get("shear_rate", 0.0)
    return s


class Oracle:
    """FP64 CPU solver: ``Oracle(params).init(init).step(n)``; fields come back
    as numpy arrays of shape (nz, ny, nx), with a leading Q or D axis for
    populations and vectors."""

    def __init__(self, params: dict):
        self.p = dict(params)
        self._ps = params_struct(self.p)
        self.h = lib().orc_create(C.byref(self._ps))
        if not self.h:
            raise ValueError("oracle rejected the parameters")
        self.N = int(lib().orc_nodes(self.h))
        self.Q = int(lib().orc_lattice_q(self.h))
        self.D = 3 if self.p["lattice"] == 1 else 2
        self.shape = (self.p["nz"], self.p["ny"], self.p["nx"])

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.orc_destroy(h)
            self.h = None

    def init(self, init: dict):
        st = lib().orc_init(self.h, C.byref(init_struct(init)))
        if st != 0:
            raise ValueError(f"orc_init failed ({st})")
        return self

    def step(self, n=1):
        st = lib().orc_step(self.h, int(n))
        if st != 0:
            raise RuntimeError(f"orc_step failed ({st})")
        return self

    def fd_substeps(self, k):
        """k FD updates of psi and phi with the flow frozen at the current state."""
        st = lib().orc_fd_substeps(self.h, int(k))
        if st != 0:
            raise RuntimeError(f"orc_fd_substeps failed ({st})")
        return self

    def _count(self, name):
        if name in ("f", "fR", "fB"):
            return self.Q
        if name in ("u", "force"):
            return self.D
        return 1

    def field(self, name: str) -> np.ndarray:
        c = self._count(name)
        out = np.zeros(c * self.N, dtype=np.float64)
        st = lib().orc_get_field(self.h, FIELDS[name], _ptr(out))
        if st != 0:
            raise ValueError(name)
        return out.reshape((c,) + self.shape) if c > 1 else out.reshape(self.shape)

    def set_field(self, name: str, arr):
        a = np.ascontiguousarray(arr, dtype=np.float64).reshape(-1)
        assert a.size == self._count(name) * self.N
        st = lib().orc_set_field(self.h, FIELDS[name], _ptr(a))
        if st != 0:
            raise ValueError(name)

    def set_clock(self, step: int, M0: float):
        lib().orc_set_clock(self.h, int(step), float(M0))

    @property
    def initial_total(self):
        return float(lib().orc_initial_total(self.h))

    def observables(self) -> dict:
        o = _Obs()
        lib().orc_observables(self.h, C.byref(o))
        return obs_dict(o)

    # --- operator-level access for the pin tests -------------------------------
    def lattice(self):
        Q, D = C.c_int(), C.c_int()
        e = (C.c_int * 57)()
        w = np.zeros(19)
        M = np.zeros(361)
        Mi = np.zeros(361)
        al = np.zeros(2)
        cs = np.zeros(2)
        lib().orc_lattice(self.h, C.byref(Q), C.byref(D), e, _ptr(w), _ptr(M), _ptr(Mi), _ptr(al), _ptr(cs))
        q = Q.value
        return dict(Q=q, D=D.value, e=np.array(e[: 3 * q]).reshape(q, 3), w=w[:q].copy(),
                    M=M[: q * q].reshape(q, q).copy(), Minv=Mi[: q * q].reshape(q, q).copy(),
                    alpha=al.copy(), cs2=cs.copy())

    def moment_eq(self, k, rho, u):
        uu = np.zeros(3)
        uu[: len(u)] = u
        m = np.zeros(19)
        lib().orc_moment_eq(self.h, int(k), float(rho), _ptr(uu), _ptr(m))
        return m[: self.Q].copy()

    def sigma(self, psi):
        return float(lib().orc_sigma(self.h, float(psi)))

    def deriv(self, chi, axis, odd_axis=-1):
        c = np.ascontiguousarray(chi, dtype=np.float64).reshape(-1)
        out = np.zeros(self.N)
        lib().orc_op_deriv(self.h, _ptr(c), int(odd_axis), int(axis), _ptr(out))
        return out.reshape(self.shape)

    def weno_div(self, Psi, u):
        P = np.zeros((3, self.N))
        U = np.zeros((3, self.N))
        P[: self.D] = np.asarray(Psi, dtype=np.float64).reshape(self.D, -1)
        U[: self.D] = np.asarray(u, dtype=np.float64).reshape(self.D, -1)
        out = np.zeros(self.N)
        lib().orc_op_weno_div(self.h, _ptr(P), _ptr(U), _ptr(out))
        return out.reshape(self.shape)

    def diffusion(self, W, chi):
        Wc = np.ascontiguousarray(W, dtype=np.float64).reshape(-1)
        c = np.ascontiguousarray(chi, dtype=np.float64).reshape(-1)
        out = np.zeros(self.N)
        lib().orc_op_diffusion(self.h, _ptr(Wc), _ptr(c), _ptr(out))
        return out.reshape(self.shape)

    def solve(self, W, Dc, rhs, guess):
        Wc = np.ascontiguousarray(W, dtype=np.float64).reshape(-1)
        r = np.ascontiguousarray(rhs, dtype=np.float64).reshape(-1)
        x = np.array(guess, dtype=np.float64).reshape(-1).copy()
        sweeps = lib().orc_op_solve(self.h, _ptr(Wc), float(Dc), _ptr(r), _ptr(x))
        return x.reshape(self.shape), sweeps

    def collide_only(self):
        fd = np.zeros(self.Q * self.N)
        fr = np.zeros(self.Q * self.N)
        fb = np.zeros(self.Q * self.N)
        lib().orc_collide_only(self.h, _ptr(fd), _ptr(fr), _ptr(fb))
        s = (self.Q,) + self.shape
        return fd.reshape(s), fr.reshape(s), fb.reshape(s)


def obs_dict(o) -> dict:
    return dict(step=o.step, mass_R=o.mass_R, mass_B=o.mass_B, total_surf=o.total_surf,
                drift_pre=o.drift_pre, velocity=list(o.velocity), centroid=list(o.centroid),
                second=list(o.second), wsum=o.wsum, nsum=o.nsum, psi_av=o.psi_av,
                psi_min=o.psi_min, psi_max=o.psi_max, p_in=o.p_in, p_out=o.p_out,
                sor_sweeps=list(o.sor_sweeps), status=o.status)


def deformation(second, D):
    """D = (L - B)/(L + B) from the eigenvalues of the central second-moment
    tensor (axes proportional to their square roots)."""
    xx, yy, zz, xy, xz, yz = second
    if D == 2:
        T = np.array([[xx, xy], [xy, yy]])
    else:
        T = np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])
    lam = np.linalg.eigvalsh(T)
    L, B = np.sqrt(max(lam[-1], 0.0)), np.sqrt(max(lam[0], 0.0))
    return (L - B) / (L + B) if L + B > 0 else 0.0
