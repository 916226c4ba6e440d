"""Python binding of the C ABI in include/lbfd.h (argument marshalling only).

Every step of the solver runs in the HIP kernels of liblbfd.so. PyTorch only
provides the device workspace (one uint8 tensor) and the stream. If the
library is missing this module raises; there is no other code path.
"""
from __future__ import annotations

import ctypes as C
import json
import math
import os

import numpy as np

from . import build as _build

LBFD_OK, LBFD_EINVAL, LBFD_ENOMEM, LBFD_EHIP, LBFD_ENONFINITE, LBFD_ESOR, LBFD_EWORKSPACE = 0, -1, -2, -3, -4, -5, -6
LBFD_EUNSUPPORTED, LBFD_ESCRATCH = -7, -8
SCRATCH_DOUBLES = 8 << 20   # LBFD_SCRATCH_DOUBLES: capacity of lbfd_read_field_noalloc
PRECISION = {"fp64": 0, "fp32": 1, "fp16dev": 2, "bf16dev": 3}
FIELDS = dict(f=0, rhoR=3, rhoB=4, rhoN=5, u=6, psi=7, phi=8, force=9, G=10, Sprev=11, Bprev=12)
EXPORTED = ["lbfd_workspace_bytes", "lbfd_create", "lbfd_init_fields", "lbfd_set_state", "lbfd_step",
            "lbfd_observables", "lbfd_read_field", "lbfd_profile", "lbfd_profile_read", "lbfd_destroy",
            "lbfd_strerror", "lbfd_batch_workspace_bytes", "lbfd_batch_create", "lbfd_batch_instance",
            "lbfd_batch_step", "lbfd_batch_destroy", "lbfd_set_graphs", "lbfd_batch_set_graphs",
            "lbfd_fd_substeps", "lbfd_set_fd", "lbfd_write_field", "lbfd_read_field_noalloc",
            "lbfd_set_tuning", "lbfd_get_tuning", "lbfd_batch_set_tuning",
            "lbfd_sg_n_params", "lbfd_sg_workspace_bytes", "lbfd_sg_create", "lbfd_sg_set_params",
            "lbfd_sg_get_params", "lbfd_sg_forward", "lbfd_sg_gradient", "lbfd_sg_train_step", "lbfd_sg_features",
            "lbfd_sg_snapshot", "lbfd_sg_tiles", "lbfd_sg_advance", "lbfd_sg_destroy", "lbfd_sg_set_drift_tol",
            "lbfd_sg_set_lr"]


class LbfdError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__(f"{what}: {strerror(status)} ({status})")


class Params(C.Structure):
    _fields_ = [
        ("lattice", C.c_int32), ("precision", C.c_int32),
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("bc", C.c_int32 * 3), ("wall_u", (C.c_double * 3) * 6),
        ("rhoR0", C.c_double), ("rhoB0", C.c_double), ("muR0", C.c_double), ("muB0", C.c_double),
        ("alphaR", C.c_double), ("beta", C.c_double), ("sigma0", C.c_double), ("E0", C.c_double),
        ("psi_inf", C.c_double), ("sigma_min_ratio", C.c_double),
        ("Ds", C.c_double), ("Db", C.c_double), ("ra", C.c_double), ("rd", C.c_double),
        ("source_mode", C.c_int32), ("gravity", C.c_double * 3),
        ("sor_omega", C.c_double), ("sor_tol", C.c_double), ("sor_max_sweeps", C.c_int32),
        ("weno_eps", C.c_double), ("rescale", C.c_int32), ("fd_enable", C.c_int32),
        ("q_literal", C.c_int32), ("eps_n", C.c_double), ("recolour_literal", C.c_int32),
        ("fd_eps", C.c_double), ("upwind_eps", C.c_double), ("buoyancy_ref", C.c_int32),
        ("eos_mode", C.c_int32),
    ]


class Init(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("cx", C.c_double * 16), ("cy", C.c_double * 16), ("cz", C.c_double * 16),
        ("r", C.c_double * 16), ("width", C.c_double), ("psi0", C.c_double),
        ("phi0_out", C.c_double), ("phi0_in", C.c_double), ("shear_rate", C.c_double),
    ]


class Obs(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("mass_R", C.c_double), ("mass_B", C.c_double),
        ("total_surf", C.c_double), ("drift_pre", C.c_double),
        ("velocity", C.c_double * 3), ("centroid", C.c_double * 3), ("second", C.c_double * 6),
        ("wsum", C.c_double), ("nsum", C.c_double), ("psi_av", C.c_double),
        ("psi_min", C.c_double), ("psi_max", C.c_double), ("p_in", C.c_double), ("p_out", C.c_double),
        ("deformation", C.c_double), ("sor_sweeps", C.c_int32 * 2), ("status", C.c_int32),
    ]


_lib = None


class Tuning(C.Structure):
    _fields_ = [("rows", C.c_int32), ("sor_wg_per_cu", C.c_int32), ("sor_narrow", C.c_int32)]


# Launch shape of the library's defaults (64 x 4 node tiles, 8 SOR workgroups per
# compute unit, 256 for sweeps past the third) and the table of tuned shapes the
# autotuner writes (tuning.json next to this module), keyed by tuning_key.
DEFAULT_TUNING = dict(rows=4, sor_wg_per_cu=8, sor_narrow=256)
TUNING_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")


def tuning_key(params: dict, instances: int = 0, nodes: int | None = None) -> str:
    """Table key of a workload: lattice, storage, size class round(log2 nodes), and
    for a batch its instance count (nodes: the batch's total)."""
    lat = "D3Q19" if params["lattice"] == 1 else "D2Q9"
    n = nodes if nodes is not None else params["nx"] * params["ny"] * params["nz"]
    key = f"{lat}/{params.get('precision', 'fp64')}/n2^{int(round(math.log2(max(n, 1))))}"
    return f"batch{instances}/{key}" if instances else key


def tuned_shape(key: str, path: str = TUNING_FILE):
    """The tuned launch shape of a key, or None."""
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        table = json.load(fh)
    e = table.get("entries", {}).get(key)
    return dict(e["tuning"]) if e else None


def _tuning_struct(t: dict) -> Tuning:
    s = Tuning()
    s.rows, s.sor_wg_per_cu, s.sor_narrow = int(t["rows"]), int(t["sor_wg_per_cu"]), int(t["sor_narrow"])
    return s


class SgParams(C.Structure):
    _fields_ = [("tile", C.c_int32), ("max_batch", C.c_int32), ("field", C.c_int32 * 3), ("k", C.c_int32),
                ("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("adam_eps", C.c_double),
                ("psi_inf", C.c_double), ("phi_s", C.c_double), ("u_s", C.c_double), ("dpsi_s", C.c_double),
                ("dphi_s", C.c_double), ("drift_tol", C.c_double)]


class SgReport(C.Structure):
    _fields_ = [("blocks", C.c_int64), ("accepted", C.c_int64), ("fallbacks", C.c_int64),
                ("max_drift", C.c_double), ("last_drift", C.c_double)]


def library_path() -> str:
    return _build.LIB


def load(build_if_missing: bool = False):
    """Load liblbfd.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    path = _build.LIB
    if not os.path.exists(path):
        if not build_if_missing:
            raise ImportError(f"{path} is missing: build it with __graft_entry__.build()")
        _build.build()
    # torch provides the workspace and the stream, so its HIP runtime must be the
    # one the library binds to: loaded first, the library's libamdhip64 dependency
    # resolves to it instead of a second runtime copy that knows neither
    import torch  # noqa: F401
    L = C.CDLL(path)
    P, vp, dp = C.POINTER, C.c_void_p, C.POINTER(C.c_double)
    L.lbfd_workspace_bytes.argtypes = [P(Params), P(C.c_size_t)]
    L.lbfd_create.argtypes = [P(Params), vp, C.c_size_t, vp, P(vp)]
    L.lbfd_init_fields.argtypes = [vp, P(Init)]
    L.lbfd_set_state.argtypes = [vp, dp, dp, dp, dp, dp, dp, dp, C.c_int64, C.c_double]
    L.lbfd_step.argtypes = [vp, C.c_int64]
    L.lbfd_observables.argtypes = [vp, P(Obs)]
    L.lbfd_read_field.argtypes = [vp, C.c_int32, dp, C.c_size_t]
    L.lbfd_read_field_noalloc.argtypes = [vp, C.c_int32, dp, C.c_size_t]
    L.lbfd_set_tuning.argtypes = [vp, P(Tuning)]
    L.lbfd_get_tuning.argtypes = [vp, P(Tuning)]
    L.lbfd_batch_set_tuning.argtypes = [vp, P(Tuning)]
    L.lbfd_profile.argtypes = [vp, C.c_int32]
    L.lbfd_profile_read.argtypes = [vp, C.c_int32, P(C.c_char_p), dp, P(C.c_int64), P(C.c_int32)]
    L.lbfd_destroy.argtypes = [vp]
    L.lbfd_destroy.restype = None
    L.lbfd_strerror.argtypes = [C.c_int]
    L.lbfd_strerror.restype = C.c_char_p
    L.lbfd_batch_workspace_bytes.argtypes = [P(Params), C.c_int32, P(C.c_size_t)]
    L.lbfd_batch_create.argtypes = [P(Params), C.c_int32, vp, C.c_size_t, vp, P(vp)]
    L.lbfd_batch_instance.argtypes = [vp, C.c_int32]
    L.lbfd_batch_instance.restype = vp
    L.lbfd_batch_step.argtypes = [vp, C.c_int64]
    L.lbfd_batch_destroy.argtypes = [vp]
    L.lbfd_batch_destroy.restype = None
    L.lbfd_set_graphs.argtypes = [vp, C.c_int32]
    L.lbfd_batch_set_graphs.argtypes = [vp, C.c_int32]
    L.lbfd_fd_substeps.argtypes = [vp, C.c_int64]
    L.lbfd_set_fd.argtypes = [vp, C.c_int32]
    L.lbfd_write_field.argtypes = [vp, C.c_int32, dp, C.c_size_t]
    i32, i64, szp = C.c_int32, C.c_int64, P(C.c_size_t)
    L.lbfd_sg_n_params.restype = i64
    L.lbfd_sg_n_params.argtypes = []
    L.lbfd_sg_workspace_bytes.argtypes = [P(SgParams), szp]
    L.lbfd_sg_create.argtypes = [P(SgParams), vp, C.c_size_t, vp, P(vp)]
    L.lbfd_sg_set_params.argtypes = [vp, P(C.c_float), i64]
    L.lbfd_sg_get_params.argtypes = [vp, P(C.c_float), i64]
    L.lbfd_sg_forward.argtypes = [vp, vp, i32, i32, i32, i32, vp]
    L.lbfd_sg_gradient.argtypes = [vp, vp, vp, i32, P(C.c_double), P(C.c_float), i64]
    L.lbfd_sg_train_step.argtypes = [vp, vp, vp, i32, P(C.c_double)]
    L.lbfd_sg_features.argtypes = [vp, vp, vp]
    L.lbfd_sg_snapshot.argtypes = [vp, vp, vp]
    L.lbfd_sg_tiles.argtypes = [vp, vp, vp, vp, P(i32), i32, vp, vp]
    L.lbfd_sg_advance.argtypes = [vp, vp, i64, P(SgReport)]
    L.lbfd_sg_destroy.argtypes = [vp]
    L.lbfd_sg_set_drift_tol.argtypes = [vp, C.c_double]
    L.lbfd_sg_set_lr.argtypes = [vp, C.c_double]
    L.lbfd_sg_destroy.restype = None
    _lib = L
    return L


def strerror(status: int) -> str:
    try:
        return load().lbfd_strerror(int(status)).decode()
    except ImportError:
        return "library not loaded"


def _check(status, what):
    if status != LBFD_OK:
        raise LbfdError(status, what)


def params_struct(p: dict) -> Params:
    s = Params()
    s.lattice = int(p["lattice"])
    s.precision = PRECISION[p.get("precision", "fp64")]
    s.nx, s.ny, s.nz = int(p["nx"]), int(p["ny"]), int(p["nz"])
    for a in range(3):
        s.bc[a] = int(p["bc"][a])
        s.gravity[a] = float(p["gravity"][a])
    for w in range(6):
        for a in range(3):
            s.wall_u[w][a] = float(p["wall_u"][w][a])
    for k in ("rhoR0", "rhoB0", "muR0", "muB0", "alphaR", "beta", "sigma0", "E0", "psi_inf",
              "sigma_min_ratio", "Ds", "Db", "ra", "rd", "sor_omega", "sor_tol", "weno_eps", "eps_n", "fd_eps", "upwind_eps"):
        setattr(s, k, float(p[k]))
    for k in ("source_mode", "sor_max_sweeps", "rescale", "fd_enable", "q_literal", "recolour_literal"):
        setattr(s, k, int(p[k]))
    s.buoyancy_ref = int(p.get("buoyancy_ref", 0))
    s.eos_mode = int(p.get("eos_mode", 0))
    return s


def init_struct(q: dict) -> Init:
    s = Init()
    s.n = len(q["drops"])
    for d, (cx, cy, cz, r) in enumerate(q["drops"]):
        s.cx[d], s.cy[d], s.cz[d], s.r[d] = cx, cy, cz, r
    s.width, s.psi0, s.phi0_out, s.phi0_in = q["width"], q["psi0"], q["phi0_out"], q["phi0_in"]
    s.shear_rate = q.get("shear_rate", 0.0)
    return s


def workspace_bytes(params: dict) -> int:
    n = C.c_size_t()
    _check(load().lbfd_workspace_bytes(C.byref(params_struct(params)), C.byref(n)), "lbfd_workspace_bytes")
    return int(n.value)


class _Instance:
    """Calls shared by a standalone solver and a member of a batch.

    Fields come back as FP64 numpy arrays of shape (nz, ny, nx), with a leading
    Q or D axis for populations and vectors."""

    def _bind(self, params: dict, h):
        self.p = dict(params)
        self.h = h
        self.Q = 19 if self.p["lattice"] == 1 else 9
        self.D = 3 if self.p["lattice"] == 1 else 2
        self.shape = (int(self.p["nz"]), int(self.p["ny"]), int(self.p["nx"]))
        self.N = int(np.prod(self.shape))

    def init_fields(self, init: dict):
        _check(load().lbfd_init_fields(self.h, C.byref(init_struct(init))), "lbfd_init_fields")
        return self

    def set_state(self, f, rhoR, rhoB, psi, phi, Sprev=None, Bprev=None, step=0, M0=0.0):
        arrs = []

        def ptr(a, count):
            if a is None:
                return None
            b = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
            assert b.size == count
            arrs.append(b)
            return b.ctypes.data_as(C.POINTER(C.c_double))
        N = self.N
        _check(load().lbfd_set_state(self.h, ptr(f, self.Q * N), ptr(rhoR, N), ptr(rhoB, N), ptr(psi, N),
                                     ptr(phi, N), ptr(Sprev, N), ptr(Bprev, N), int(step), float(M0)),
               "lbfd_set_state")
        return self

    def write_field(self, name: str, values):
        """Overwrite psi, phi (physical values) or Sprev / Bprev from FP64 host data."""
        a = np.ascontiguousarray(values, dtype=np.float64).reshape(-1)
        _check(load().lbfd_write_field(self.h, FIELDS[name], a.ctypes.data_as(C.POINTER(C.c_double)), a.size),
               f"lbfd_write_field({name})")
        return self

    def set_fd(self, enable: bool):
        """Switch the FD part of step() off (psi, phi held) or on."""
        _check(load().lbfd_set_fd(self.h, int(bool(enable))), "lbfd_set_fd")
        return self

    def fd_substeps(self, k: int):
        """k FD updates of psi and phi with the flow frozen at the current state."""
        _check(load().lbfd_fd_substeps(self.h, int(k)), "lbfd_fd_substeps")
        return self

    def observables(self, check=True) -> dict:
        o = Obs()
        st = load().lbfd_observables(self.h, C.byref(o))
        if check:
            _check(st, "lbfd_observables")
        return dict(step=o.step, mass_R=o.mass_R, mass_B=o.mass_B, total_surf=o.total_surf,
                    drift_pre=o.drift_pre, velocity=list(o.velocity), centroid=list(o.centroid),
                    second=list(o.second), wsum=o.wsum, nsum=o.nsum, psi_av=o.psi_av, psi_min=o.psi_min,
                    psi_max=o.psi_max, p_in=o.p_in, p_out=o.p_out, deformation=o.deformation,
                    sor_sweeps=list(o.sor_sweeps), status=o.status)

    def field(self, name: str) -> np.ndarray:
        c = self.Q if name == "f" else self.D if name in ("u", "force") else 1
        out = np.zeros(c * self.N, dtype=np.float64)
        _check(load().lbfd_read_field(self.h, FIELDS[name], out.ctypes.data_as(C.POINTER(C.c_double)),
                                      out.size), f"lbfd_read_field({name})")
        return out.reshape((c,) + self.shape) if c > 1 else out.reshape(self.shape)

    def field_noalloc(self, name: str) -> np.ndarray:
        """field() through lbfd_read_field_noalloc: staged in the library's fixed
        device array (no device allocation); LBFD_ESCRATCH above its capacity."""
        c = self.Q if name == "f" else self.D if name in ("u", "force") else 1
        out = np.zeros(c * self.N, dtype=np.float64)
        _check(load().lbfd_read_field_noalloc(self.h, FIELDS[name], out.ctypes.data_as(C.POINTER(C.c_double)),
                                              out.size), f"lbfd_read_field_noalloc({name})")
        return out.reshape((c,) + self.shape) if c > 1 else out.reshape(self.shape)

    KERNEL_CLASSES = ("collide", "macro", "geom", "fd", "sor", "total", "force", "other")

    def profile(self, enable: bool, only=None):
        """Per-kernel HIP-event timing; `only` limits it to some kernel classes."""
        code = 0
        if enable:
            mask = 0
            for name in (only or ()):
                mask |= 1 << self.KERNEL_CLASSES.index(name)
            code = 1 | (mask << 1)
        _check(load().lbfd_profile(self.h, code), "lbfd_profile")

    def profile_read(self) -> dict:
        names = (C.c_char_p * 16)()
        ms = np.zeros(16)
        cnt = np.zeros(16, dtype=np.int64)
        nk = C.c_int32()
        _check(load().lbfd_profile_read(self.h, 16, names, ms.ctypes.data_as(C.POINTER(C.c_double)),
                                        cnt.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(nk)), "lbfd_profile_read")
        return {names[i].decode(): (float(ms[i]), int(cnt[i])) for i in range(nk.value)}


class Solver(_Instance):
    """One solver instance on one device: ``Solver(params).init_fields(init).step(n)``.

    tuning: "auto" applies the tuned launch shape of the workload's key from
    tuning.json when there is one (else the defaults), None keeps the defaults,
    a dict sets one (rows, sor_wg_per_cu, sor_narrow). Results do not depend on it."""

    def __init__(self, params: dict, device: str = "cuda:0", stream=None, tuning="auto"):
        import torch

        self._ps = params_struct(params)
        L = load()
        nbytes = workspace_bytes(params)
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        ptr = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check(L.lbfd_create(C.byref(self._ps), C.c_void_p(ptr), C.c_size_t(nbytes),
                             C.c_void_p(self.stream.cuda_stream), C.byref(h)), "lbfd_create")
        self._bind(params, h)
        t = tuned_shape(tuning_key(params)) if tuning == "auto" else tuning
        if t:
            self.set_tuning(t)

    def set_tuning(self, t: dict):
        """Launch shape (rows, sor_wg_per_cu, sor_narrow); drops captured graphs."""
        _check(load().lbfd_set_tuning(self.h, C.byref(_tuning_struct(dict(DEFAULT_TUNING, **t)))), "lbfd_set_tuning")
        return self

    def get_tuning(self) -> dict:
        t = Tuning()
        _check(load().lbfd_get_tuning(self.h, C.byref(t)), "lbfd_get_tuning")
        return dict(rows=t.rows, sor_wg_per_cu=t.sor_wg_per_cu, sor_narrow=t.sor_narrow)

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.lbfd_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def step(self, n: int = 1):
        _check(load().lbfd_step(self.h, int(n)), "lbfd_step")
        return self

    def graphs(self, enable: bool):
        """Replay captured two-step HIP graphs in step(n >= 4) (default) or launch every kernel."""
        _check(load().lbfd_set_graphs(self.h, int(bool(enable))), "lbfd_set_graphs")
        return self


class BatchMember(_Instance):
    """Instance i of a Batch: initialised, observed and read like a Solver,
    advanced only through Batch.step (its handle belongs to the batch)."""

    def __init__(self, batch: "Batch", i: int, params: dict, h):
        self.batch = batch
        self.index = i
        self._bind(params, h)


class Batch:
    """Independent instances advanced together, one launch per kernel class:
    ``Batch([params0, params1, ...])``, then ``b[i].init_fields(...)`` and ``b.step(n)``."""

    def __init__(self, params_list, device: str = "cuda:0", stream=None, tuning="auto"):
        import torch

        plist = [dict(p) for p in params_list]
        n = len(plist)
        arr = (Params * n)(*[params_struct(p) for p in plist])
        self._arr = arr
        L = load()
        nb = C.c_size_t()
        _check(L.lbfd_batch_workspace_bytes(arr, n, C.byref(nb)), "lbfd_batch_workspace_bytes")
        nbytes = int(nb.value)
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.workspace.data_ptr() + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        b = C.c_void_p()
        _check(L.lbfd_batch_create(arr, n, C.c_void_p(ptr), C.c_size_t(nbytes), C.c_void_p(self.stream.cuda_stream),
                                   C.byref(b)), "lbfd_batch_create")
        self.b = b
        self.members = []
        for i, p in enumerate(plist):
            h = L.lbfd_batch_instance(b, i)
            if not h:
                raise LbfdError(LBFD_EINVAL, f"lbfd_batch_instance({i})")
            self.members.append(BatchMember(self, i, p, C.c_void_p(h)))
        self.nodes = sum(m.N for m in self.members)
        self.key = tuning_key(plist[0], instances=n, nodes=self.nodes)
        t = tuned_shape(self.key) if tuning == "auto" else tuning
        if t:
            self.set_tuning(t)

    def set_tuning(self, t: dict):
        """Launch shape of every instance (a batch uses only `rows`)."""
        _check(load().lbfd_batch_set_tuning(self.b, C.byref(_tuning_struct(dict(DEFAULT_TUNING, **t)))),
               "lbfd_batch_set_tuning")
        return self

    def __len__(self):
        return len(self.members)

    def __getitem__(self, i) -> BatchMember:
        return self.members[i]

    def step(self, n: int = 1):
        _check(load().lbfd_batch_step(self.b, int(n)), "lbfd_batch_step")
        return self

    def graphs(self, enable: bool):
        _check(load().lbfd_batch_set_graphs(self.b, int(bool(enable))), "lbfd_batch_set_graphs")
        return self

    def close(self):
        if getattr(self, "b", None) and _lib is not None:
            for m in self.members:
                m.h = None
            _lib.lbfd_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        self.close()


def _dptr(t):
    return C.c_void_p(t.data_ptr())


SG_NOUT = 7   # network outputs per node: flux coefficients of psi and phi along x, y, z, and the exchange


class Surrogate:
    """The learned surrogate of k frozen-flow FD substeps (weights, Adam state and
    work buffers on one device workspace). Tensors passed in are torch device
    tensors: inputs as int16/uint16-sized BF16 bit patterns (torch.bfloat16 is
    accepted as is), targets [..., 4] and outputs [..., SG_NOUT] FP32."""

    DEFAULTS = dict(tile=32, max_batch=8, field=(0, 0, 0), k=8, lr=1e-3, beta1=0.9, beta2=0.999, adam_eps=1e-8,
                    psi_inf=1.0, phi_s=0.1, u_s=0.01, dpsi_s=0.01, dphi_s=0.001, drift_tol=1e-6)

    def __init__(self, device: str = "cuda:0", stream=None, **kw):
        import torch

        cfg = dict(self.DEFAULTS)
        cfg.update(kw)
        self.cfg = cfg
        ps = SgParams()
        for k, v in cfg.items():
            if k == "field":
                for a in range(3):
                    ps.field[a] = int(v[a])
            else:
                setattr(ps, k, v)
        self._ps = ps
        L = load()
        nb = C.c_size_t()
        _check(L.lbfd_sg_workspace_bytes(C.byref(ps), C.byref(nb)), "lbfd_sg_workspace_bytes")
        self.device = torch.device(device)
        self.workspace = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.workspace.data_ptr() + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check(L.lbfd_sg_create(C.byref(ps), C.c_void_p(ptr), C.c_size_t(int(nb.value)),
                                C.c_void_p(self.stream.cuda_stream), C.byref(h)), "lbfd_sg_create")
        self.h = h
        self.n = int(L.lbfd_sg_n_params())

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.lbfd_sg_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def set_params(self, flat):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        _check(load().lbfd_sg_set_params(self.h, a.ctypes.data_as(C.POINTER(C.c_float)), a.size),
               "lbfd_sg_set_params")
        return self

    def get_params(self) -> np.ndarray:
        a = np.zeros(self.n, dtype=np.float32)
        _check(load().lbfd_sg_get_params(self.h, a.ctypes.data_as(C.POINTER(C.c_float)), a.size),
               "lbfd_sg_get_params")
        return a

    def forward(self, x, out):
        B, d, h, w, c = x.shape
        if c != 16 or not x.is_contiguous() or not out.is_contiguous():
            raise ValueError("forward: inputs [B][d][h][w][16] and outputs must be contiguous")
        if out.numel() != B * (d - 8) * (h - 8) * (w - 8) * SG_NOUT or out.element_size() != 4:
            raise ValueError(f"forward: the output must hold B (d-8)(h-8)(w-8) x {SG_NOUT} FP32 values")
        _check(load().lbfd_sg_forward(self.h, _dptr(x), B, d, h, w, _dptr(out)), "lbfd_sg_forward")
        return out

    def _check_tiles(self, x, t):
        T = self.cfg["tile"]
        if tuple(x.shape[1:]) != (T + 8, T + 8, T + 8, 16) or tuple(t.shape) != (x.shape[0], T, T, T, 4):
            raise ValueError(f"tiles: inputs [B][{T + 8}]^3[16], targets [B][{T}]^3[4]")
        if not (x.is_contiguous() and t.is_contiguous()) or t.element_size() != 4:
            raise ValueError("tiles must be contiguous, targets FP32")

    def gradient(self, x, t):
        self._check_tiles(x, t)
        g = np.zeros(self.n, dtype=np.float32)
        loss = C.c_double()
        _check(load().lbfd_sg_gradient(self.h, _dptr(x), _dptr(t), x.shape[0], C.byref(loss),
                                       g.ctypes.data_as(C.POINTER(C.c_float)), g.size), "lbfd_sg_gradient")
        return loss.value, g

    def train_step(self, x, t, want_loss=True):
        self._check_tiles(x, t)
        loss = C.c_double()
        _check(load().lbfd_sg_train_step(self.h, _dptr(x), _dptr(t), x.shape[0],
                                         C.byref(loss) if want_loss else None), "lbfd_sg_train_step")
        return loss.value if want_loss else None

    def features(self, solver, feat):
        _check(load().lbfd_sg_features(solver.h, self.h, _dptr(feat)), "lbfd_sg_features")
        return feat

    def snapshot(self, solver, snap):
        _check(load().lbfd_sg_snapshot(solver.h, self.h, _dptr(snap)), "lbfd_sg_snapshot")
        return snap

    def tiles(self, solver, feat, snap, origins, x, t):
        org = np.ascontiguousarray(np.asarray(origins, dtype=np.int32).reshape(-1))
        B = org.size // 3
        if x.shape[0] != B or t.shape[0] != B:
            raise ValueError("tiles: one input and one target tile per origin")
        self._check_tiles(x, t)
        _check(load().lbfd_sg_tiles(solver.h, self.h, _dptr(feat), _dptr(snap),
                                    org.ctypes.data_as(C.POINTER(C.c_int32)), B, _dptr(x), _dptr(t)), "lbfd_sg_tiles")
        return x, t

    def set_lr(self, lr: float):
        _check(load().lbfd_sg_set_lr(self.h, float(lr)), "lbfd_sg_set_lr")
        self.cfg["lr"] = float(lr)
        return self

    def set_drift_tol(self, tol: float):
        _check(load().lbfd_sg_set_drift_tol(self.h, float(tol)), "lbfd_sg_set_drift_tol")
        self.cfg["drift_tol"] = float(tol)
        return self

    def advance(self, solver, nblocks: int) -> dict:
        rep = SgReport()
        _check(load().lbfd_sg_advance(solver.h, self.h, int(nblocks), C.byref(rep)), "lbfd_sg_advance")
        return dict(blocks=rep.blocks, accepted=rep.accepted, fallbacks=rep.fallbacks, max_drift=rep.max_drift,
                    last_drift=rep.last_drift)
