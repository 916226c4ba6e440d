#!/usr/bin/env python3
"""Throughput of the hybrid LB colour-gradient / FD surfactant step on one MI355X.

One step = the method's whole per-step path (forces, MRT collision with
recolouring and propagation, macroscopic fields, WENO3 / Crank-Nicolson
right-hand sides, red-black SOR to tolerance, rescaling) on one batch of
synthetic input resident in HBM. The headline workload is the buoyant bubble
column: D3Q19, 128 x 128 x 384, density ratio 10, BF16-deviation population
storage with FP32 arithmetic. MLUPS = nodes x steps / wall time of the timed
region (HIP events on the solver's stream, bracketed by synchronisations).

The printed JSON line also carries:
  roofline      the dominant kernel's algorithmic bytes per launch over its
                mean launch time (HIP events around each launch, same timed
                region) against 8 TB/s; traffic = measured HBM bytes per launch
                from the rocprofv3 counter summary under profiles/ (null if the
                kernel sources changed since it was taken)
  step_bandwidth the algorithmic bytes of one whole step (every kernel, SOR
                half-sweeps counted for the sweeps that ran) x MLUPS, against
                8 TB/s
  cpu_baseline  the FP64 oracle on the host cores, on a bounded sample
  secondary     the 2-D workloads (shear 512 x 256 in FP64 / FP32 / FP16-dev,
                droplet 128 x 128 FP64), same timing method
  batched       the parameter sweep of 64 uneven 2-D bubble columns as one
                batch against the same instances run one after another
  surrogate     the learned surrogate of 8 frozen-flow FD substeps on the
                periodic multi-bubble box: training on the solver's own
                snapshots, held-out error, one whole-grid application against
                the 8 FD substeps it replaces (and its matrix-core rate), and
                surrogate mode against plain stepping
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_FILE = os.path.join(PROFILES, "traffic_bubble128x128x384_bf16dev.json")
VALU_FILE = os.path.join(PROFILES, "valu_bubble128x128x384_bf16dev.json")
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12   # wave64 VALU lane instructions per second
# A kernel is labelled issue-bound ("alu") when its VALU instructions fill at
# least this share of the issue peak. Below it the label is the HBM roof of its
# algorithmic bytes: the collision at 65 % issue ran no faster when 13 % of its
# instructions were removed, while the macro kernel at 85-90 % did.
ALU_BOUND_ISSUE = 0.8
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2311_15242_amd", "csrc", f)
                  for f in ("lbfd.hip", "lbfd_kernels.h", "lbfd_lattice_tables.h", "sg_conv.h")]
TIMED_REGIONS = 5        # the headline is the median of this many timed regions of K steps

# Minimum state a two-colour method must move per lattice update (every population
# read and written once, plus the scalar fields of the step; on-chip recomputation
# excluded), by lattice and storage: the "useful bandwidth" denominator.
USEFUL_BYTES = {(0, "fp64"): 424, (0, "fp32"): 212, (0, "fp16dev"): 148, (0, "bf16dev"): 148,
                (1, "fp64"): 768, (1, "fp32"): 384, (1, "fp16dev"): 240, (1, "bf16dev"): 240}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(kernel: str, p: dict) -> float:
    """Bytes per node one launch of `kernel` must move between HBM and the
    chip: each input and output array counted once (no halo re-reads, no
    redundant traffic). Q populations of bf bytes, scalars of br bytes."""
    three = p["lattice"] == 1
    Q, D = (19, 3) if three else (9, 2)
    prec = p["precision"]
    bf = {"fp64": 8, "fp32": 4, "fp16dev": 2, "bf16dev": 2}[prec]
    br = 8 if prec == "fp64" else 4
    dev = prec in ("fp16dev", "bf16dev")
    # descriptor written by the collision, in bytes: (a, c) in the storage real, or the
    # packed deviation-mode descriptor (a, rho FP32; c, u* FP16)
    desc_b = (8 + 4 * D) if dev else (1 + D) * br
    # state between steps: Q populations, or (deviation modes) the Q - 1 - D
    # non-conserved moments
    state = (Q - 1 - D) if dev else Q
    # the correction field qf_a exists when some colour has a non-zero
    # correction prefactor (3-D: 1 - 3 cs^2 with cs^2 = (1 - alpha)/2; 2-D: 1.8 alpha - 0.8)
    alphaB = 1.0 - (p["rhoR0"] / p["rhoB0"]) * (1.0 - p["alphaR"])
    qc = [(1.0 - 1.5 * (1.0 - al)) if three else (1.8 * al - 0.8) for al in (p["alphaR"], alphaB)]
    qf = D if any(abs(c) > 1e-15 for c in qc) else 0
    table = {
        # state in, Q populations out; rhoR rhoB, u, F, normal, qf in; descriptor out
        "collide": (state + Q) * bf + (2 + 3 * D + qf) * br + desc_b,
        # Q populations in, descriptor in, rhoR rhoB rhoN j out (+ moment state out)
        "macro": (Q + (state if dev else 0)) * bf + (3 + D) * br + desc_b,
        # rhoN in; |grad rhoN|, normal and the colour-split weights of both implicit systems out
        "geom": (4 + D) * br,
        # psi phi G rhoN u Sprev Bprev in; rhs x2, S B, psi phi guesses out
        "fd": (6 + D + 6) * br,
        # one colour half of a sweep on the colour-split arrays: psi phi and both weights in (all
        # nodes), both right-hand sides in and psi phi out (the half being updated)
        "sor": (4 + 0.5 * 2 + 0.5 * 2) * br,
        # G rhoN psi phi (colour-split) in, psi phi in node order out
        "total": 6 * br,
        # rhoN, normal, psi, rhoR rhoB j in; u, F, qf out
        "force": (4 + 2 * D) * br + (2 * D + qf) * br,
    }
    return float(table.get(kernel, 0.0))


def hbm_probe(mib=1024, reps=20):
    """Bandwidth a plain device copy and a plain fill of `mib` MiB reach on this GPU
    (torch's own copy and fill kernels, HIP events, mean of `reps` launches after
    one untimed launch): the practical ceiling of a streaming kernel, stated beside
    the published peak the rooflines use."""
    import torch

    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)

    def timed(f):
        f()
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(reps):
            f()
        e.record()
        torch.cuda.synchronize()
        return s.elapsed_time(e) / reps / 1e3

    tc = timed(lambda: b.copy_(a))
    tf = timed(lambda: b.fill_(2.0))
    out = dict(bytes=4 * n, copy_GBps=round(8 * n / tc / 1e9, 1), fill_GBps=round(4 * n / tf / 1e9, 1),
               peak=HBM_PEAK_GBS, note="copy counts bytes read and written")
    del a, b
    torch.cuda.empty_cache()
    return out


def build_solver(p, q, tuning="auto"):
    from paper_2311_15242_amd import lbfd

    return lbfd.Solver(p, tuning=tuning).init_fields(q)


def timed_run(p, q, steps, warmup, profile, only=None, regions=1, tuning="auto"):
    """Warm-up, then `regions` timed regions of `steps` steps each on the same
    solver (HIP events on its stream, synchronised on both sides). Returns the
    median region's milliseconds, the profile of all regions, the observables
    and every region's milliseconds."""
    import torch

    s = build_solver(p, q, tuning)
    s.step(warmup)
    torch.cuda.synchronize()
    ob = s.observables()
    if ob["status"] != 0:
        raise RuntimeError(f"solver status {ob['status']} after warm-up")
    timed_run.shape = s.get_tuning()
    if profile:
        s.profile(True, only=only)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    runs = []
    for _ in range(regions):
        torch.cuda.synchronize()
        a.record()
        s.step(steps)
        b.record()
        torch.cuda.synchronize()
        runs.append(a.elapsed_time(b))
    prof = s.profile_read() if profile else {}
    ob = s.observables()
    if ob["status"] != 0:
        raise RuntimeError(f"solver status {ob['status']} in the timed region")
    s.close()
    return float(np.median(runs)), prof, ob, runs


def conv_flops(d, h, w, B=1):
    """Multiply-adds x 2 of the surrogate on B grids of d x h x w input nodes, counted
    with the real channel counts (6 -> 32 -> 32 -> 32 -> 7)."""
    chans = ((6, 32), (32, 32), (32, 32), (32, 7))
    f = 0
    for l, (ci, co) in enumerate(chans):
        f += 2 * 27 * ci * co * B * (d - 2 * l - 2) * (h - 2 * l - 2) * (w - 2 * l - 2)
    return float(f)


def surrogate_bench(n, snapshots, tiles_per_snap, train_steps, blocks, lr_final=None, seed=0):
    """The learned surrogate on the multi-bubble periodic box (D3Q19 n^3, 8 bubbles
    of diameter 24, Eo 10, Bi 1, FP32 solver): snapshot tiles from the solver,
    training on the GPU, the held-out error against the FD substeps it replaces,
    the time of one whole-grid application against k = 8 FD substeps, and
    surrogate mode against FD-substep mode (the same lagged coupling with the FD
    update) and against plain stepping."""
    import torch

    import workloads as W
    from paper_2311_15242_amd import lbfd, sgtrain

    k = 8
    say = lambda *a: print("[surrogate]", *a, file=sys.stderr, flush=True)
    rng = np.random.default_rng(seed)
    p, q = W.multi_bubble(n=n, count=8, diameter=24.0, Eo=10.0, Bi=1.0, seed=seed, precision="fp32")
    # SOR launch budget as for the headline workload, with a wider margin: the first
    # frozen-flow substep starts its solve without an extrapolated guess
    p["sor_max_sweeps"] = sweep_budget(p, q, 20, margin=4)
    N = n ** 3
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        torch.cuda.synchronize()
        ev0.record()
        r = fn()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1), r

    s = lbfd.Solver(p).init_fields(q)
    s.step(100)
    dps, dph = sgtrain.change_scales(s, k)
    sg = lbfd.Surrogate(tile=32, max_batch=8, field=(n, n, n), k=k, lr=1e-3, phi_s=0.5, u_s=0.005,
                        dpsi_s=dps, dphi_s=dph, drift_tol=1e-6)
    sg.set_params(sgtrain.initial_params(seed))
    bufs = sgtrain.feature_buffers(s)
    # the training set is filled in place (at 65,536 tiles it takes 168 GB of HBM)
    T = sg.cfg["tile"]
    X = torch.empty((snapshots * tiles_per_snap, T + 8, T + 8, T + 8, 16), dtype=torch.int16, device="cuda")
    Y = torch.empty((snapshots * tiles_per_snap, T, T, T, 4), dtype=torch.float32, device="cuda")
    t0 = time.time()
    for i in range(snapshots):
        s.step(25)
        a = i * tiles_per_snap
        sgtrain.snapshot_tiles(s, sg, tiles_per_snap, rng, bufs, out=(X[a:a + tiles_per_snap], Y[a:a + tiles_per_snap]))
    s.step(25)
    Xh, Yh = sgtrain.snapshot_tiles(s, sg, 128, rng, bufs)
    torch.cuda.synchronize()
    t_data = time.time() - t0
    say(f"{X.shape[0]} training tiles in {t_data:.1f} s")
    e0, _ = sgtrain.tile_error(sg, Xh, Yh)
    ms_train, hist = timed(lambda: sgtrain.train(sg, X, Y, train_steps, 8, rng, log_every=max(1, train_steps // 4),
                                                 lr_final=lr_final))
    e1, _ = sgtrain.tile_error(sg, Xh, Yh)
    say(f"trained {train_steps} steps in {ms_train / 1e3:.1f} s: held-out error {e0:.3f} -> {e1:.3f}")
    del X, Y
    # one whole-grid application (features + network) against the k FD substeps it replaces
    feat, _ = bufs
    out = torch.empty((n, n, n, lbfd.SG_NOUT), dtype=torch.float32, device="cuda")
    x = feat.view(1, n + 8, n + 8, n + 8, 16)
    sg.features(s, feat)
    sg.forward(x, out)
    reps = 5
    ms_inf = timed(lambda: [(sg.features(s, feat), sg.forward(x, out)) for _ in range(reps)])[0] / reps
    ms_net = timed(lambda: sg.forward(x, out))[0]
    ms_fd = timed(lambda: s.fd_substeps(k))[0]
    ob = s.observables(check=False)
    if ob["status"] != 0:
        raise RuntimeError(f"FD substeps: solver status {ob['status']}")
    fd_drift = ob["drift_pre"]   # pre-rescale drift of the last FD substep
    s.close()
    del s
    # surrogate mode and its references from one warm state (deterministic runs)
    def warm():
        r = lbfd.Solver(p).init_fields(q)
        r.step(200)
        return r

    def fd_mode(r):
        for _ in range(blocks):
            r.fd_substeps(k)
            r.set_fd(False).step(k).set_fd(True)

    def ok(r, what):
        st = r.observables(check=False)["status"]
        if st != 0:
            raise RuntimeError(f"{what}: solver status {st}")

    a = warm()
    ms_strict, rep_strict = timed(lambda: sg.advance(a, blocks))
    ok(a, "surrogate mode (strict gate)")
    psi_a = a.field("psi")
    a.close()
    b = warm()
    psi0 = b.field("psi")
    ms_fdm, _ = timed(lambda: fd_mode(b))
    ok(b, "FD-substep mode")
    psi_b = b.field("psi")
    b.close()
    c = warm()
    ms_plain, _ = timed(lambda: c.step(blocks * k))
    ok(c, "plain stepping")
    psi_c = c.field("psi")
    c.close()
    nrm = lambda v: float(np.sqrt((v * v).sum()))
    say(f"mode: {rep_strict}")
    flops = conv_flops(n + 8, n + 8, n + 8)
    steps = blocks * k
    mlups = lambda ms: round(N * steps / (ms / 1e3) / 1e6, 1)
    return dict(
        workload=f"multi_bubble {n}^3 periodic D3Q19, 8 bubbles D=24, Eo=10, Bi=1, FP32 solver; k={k} substeps",
        sor_sweeps_launched=p["sor_max_sweeps"],
        tiles_train=snapshots * tiles_per_snap, tiles_heldout=int(Xh.shape[0]), data_s=round(t_data, 2),
        train_steps=train_steps, batch=8, lr=1e-3, lr_final=lr_final, train_ms=round(ms_train, 1),
        train_tiles_per_s=round(train_steps * 8 / (ms_train / 1e3), 1),
        train_tflops=round(3.0 * conv_flops(40, 40, 40, 8) * train_steps / (ms_train / 1e3) / 1e12, 2),
        loss_first=hist[0][1], loss_last=hist[-1][1],
        heldout_rel_error_untrained=round(e0, 4), heldout_rel_error=round(e1, 4),
        inference_ms=round(ms_inf, 3), network_ms=round(ms_net, 3), fd_substeps_ms=round(ms_fd, 3),
        inference_speedup=round(ms_fd / ms_inf, 3), fd_substep_drift=fd_drift,
        network_mfma=dict(bound="mfma", achieved=round(flops / (ms_net / 1e3) / 1e12, 2), peak=2500.0,
                          unit="TFLOP/s", frac=round(flops / (ms_net / 1e3) / 1e12 / 2500.0, 4)),
        mode_steps=steps,
        mode=dict(drift_tol=1e-6, range_check=True, accepted=rep_strict["accepted"],
                  fallbacks=rep_strict["fallbacks"], max_drift=rep_strict["max_drift"],
                  last_drift=rep_strict["last_drift"], mlups=mlups(ms_strict),
                  speedup_vs_plain=round(ms_plain / ms_strict, 4),
                  psi_rel_error_vs_plain=round(nrm(psi_a - psi_c) / max(nrm(psi_c - psi0), 1e-300), 4),
                  psi_rel_error_vs_fd_mode=round(nrm(psi_a - psi_b) / max(nrm(psi_b - psi0), 1e-300), 4),
                  error_norm="L2 of the psi difference over L2 of plain stepping's change of psi over the run"),
        fd_mode_mlups=mlups(ms_fdm), plain_mlups=mlups(ms_plain),
        fd_mode_psi_rel_error_vs_plain=round(nrm(psi_b - psi_c) / max(nrm(psi_c - psi0), 1e-300), 4))


def rise_validation(R, precision, max_steps, chunk, tol, cases=(0.4, 0.2, 0.1), buoyancy_ref=0):
    """Clean buoyant bubble (Eo = 1, Mo = 0.1, density and viscosity ratio 10) in
    walled channels of 2R/L_x = 0.4, 0.2 and 0.1 (L_x x L_y x L_z = 5R x 5R x 10R,
    10R x 10R x 10R, 20R x 20R x 10R, periodic in z, Sec 3.4): the rise velocity of
    eq 33 until it changes by less than tol over one chunk of steps, divided by
    the Hadamard-Rybczynski velocity of eq 35. The FD part is off (no surfactant)."""
    import workloads as W
    from paper_2311_15242_amd import lbfd

    say = lambda *a: print("[rise]", *a, file=sys.stderr, flush=True)
    out = []
    for ratio in cases:
        m = int(round(2.0 / ratio))
        p, q = W.bubble_rise(nx=m * R, ny=m * R, nz=10 * R, radius=float(R), Eo=1.0, Mo=0.1, clean=True,
                             precision=precision, fd_enable=0, buoyancy_ref=buoyancy_ref)
        g = -p["gravity"][2]
        drho = p["rhoB0"] - p["rhoR0"]
        muB, muR = p["muB0"], p["muR0"]
        u_th = (2.0 / 3.0) * g * drho * R * R / muB * (muB + muR) / (2.0 * muB + 3.0 * muR)
        s = lbfd.Solver(p).init_fields(q)
        hist = []
        steps = 0
        t0 = time.time()
        while steps < max_steps:
            s.step(chunk)
            steps += chunk
            ob = s.observables()
            u = ob["velocity"][2]
            hist.append(u / u_th)
            if len(hist) % 5 == 0:
                say(f"  2R/Lx={ratio}: {steps} steps, U/U_th={hist[-1]:.4f}")
            if len(hist) >= 3 and abs(hist[-1] - hist[-2]) <= tol * abs(hist[-1]) and \
                    abs(hist[-2] - hist[-3]) <= tol * abs(hist[-2]):
                break
        uz_mean = float(s.field("u")[2].mean())
        say(f"2R/Lx={ratio}: U/U_th={hist[-1]:.4f}, mean u_z/U_th={uz_mean / u_th:.4f} after {steps} steps "
            f"({time.time() - t0:.1f} s)")
        out.append(dict(confinement=ratio, grid=[p["nx"], p["ny"], p["nz"]], steps=steps, u_over_uth=round(hist[-1], 4),
                        mean_uz_over_uth=round(uz_mean / u_th, 4),
                        u_th=u_th, re=2.0 * p["rhoB0"] * hist[-1] * u_th * R / muB,
                        converged=len(hist) >= 3 and abs(hist[-1] - hist[-2]) <= tol * abs(hist[-1]),
                        history=[round(v, 4) for v in hist[::max(1, len(hist) // 12)]]))
        s.close()
    return dict(workload=f"clean bubble rise, R={R}, Eo=1, Mo=0.1, {precision}, buoyancy_ref={buoyancy_ref}",
                paper=[0.552, 0.811, 0.937], cases=out)


def ygb_validation(R, precision, max_steps, chunk, tol, widths=(5, 10), min_steps=0):
    """Drop migration in the imposed surfactant gradient of Sec 3.2 (linear
    tension law, psi held at the ramp of eq 31, walls in x and y, L_z = 10R):
    the migration velocity of eq 33 divided by the YGB velocity of eq 32. The
    value wobbles by a few tenths of a per cent as the drop crosses the lattice,
    so the run stops when the means over the last two windows of five chunks
    agree within tol, and the result is the mean over the last ten chunks."""
    import workloads as W
    from paper_2311_15242_amd import lbfd

    say = lambda *a: print("[ygb]", *a, file=sys.stderr, flush=True)
    out = []
    for wr in widths:
        p, q = W.ygb_migration(R=R, width=wr, precision=precision)
        # eq 32 with the outer (blue) viscosity on the 6 and the drop's on the 9, as in
        # Young, Goldstein and Block; the printed labels are the other way round, which
        # gives the same value at the equal viscosities of the test
        u_ygb = 2.0 * p["sigma0"] * p["E0"] * R / (p["nz"] * (6.0 * p["muB0"] + 9.0 * p["muR0"]))
        s = lbfd.Solver(p).init_fields(q).write_field("psi", W.migration_psi(p))
        hist = []
        steps = 0
        converged = False
        t0 = time.time()
        while steps < max_steps:
            s.step(chunk)
            steps += chunk
            ob = s.observables()
            hist.append(ob["velocity"][2] / u_ygb)
            r_eff = (3.0 * ob["nsum"] / (4.0 * np.pi)) ** (1.0 / 3.0)
            if len(hist) % 5 == 0:
                say(f"  L_x = {wr}R: {steps} steps, U/U_YGB={hist[-1]:.4f}, drop radius {r_eff:.3f}")
            converged = steps >= min_steps and len(hist) >= 10 and \
                abs(np.mean(hist[-5:]) - np.mean(hist[-10:-5])) <= tol * abs(np.mean(hist[-5:]))
            if converged:
                break
        ob = s.observables()
        uz_mean = float(s.field("u")[2].mean())
        tail = np.asarray(hist[-10:])
        say(f"L_x = {wr}R: U/U_YGB={tail.mean():.4f} +- {tail.std():.4f}, mean u_z/U_YGB={uz_mean / u_ygb:.4f} "
            f"after {steps} steps ({time.time() - t0:.1f} s)")
        out.append(dict(width=wr, grid=[p["nx"], p["ny"], p["nz"]], steps=steps, u_over_uygb=round(float(tail.mean()), 4),
                        spread=round(float(tail.std()), 4), mean_uz_over_uygb=round(uz_mean / u_ygb, 4), u_ygb=u_ygb,
                        tau=round(float(tail.mean()) * u_ygb * steps / R, 3),
                        drift_z=round(ob["centroid"][2] - q["drops"][0][2], 3), converged=bool(converged),
                        radius_end=round((3.0 * ob["nsum"] / (4.0 * np.pi)) ** (1.0 / 3.0), 3),
                        seconds=round(time.time() - t0, 1),
                        history=[round(v, 4) for v in hist[::max(1, len(hist) // 12)]]))
        s.close()
    return dict(workload=f"drop migration in an imposed surfactant gradient, R={R}, {precision}",
                paper=[0.958, 0.993], cases=out)


def adsorption_theory(t, r, R, D, ra, psi_inf, phi0, psi0=0.0):
    """Eqs 29 and 30 of Sec 3.1 (uptake onto a sphere with the source
    j = ra psi_inf phi, no desorption), with m = ra psi_inf / D, a = sqrt(pi D),
    eta = a (1 + R m) / R. Readings: D is the bulk diffusivity, and the
    denominator of eq 29 is 1 + eta sqrt(t) (the printed one lacks the 1/R that
    makes it dimensionless; with it, eq 30 is the time integral of eq 29 at
    r = R). Returns (psi / psi_inf, phi / phi0 at the radii r)."""
    from scipy.special import erfc

    m = ra * psi_inf / D
    a = np.sqrt(np.pi * D)
    eta = a * (1.0 + R * m) / R
    st = np.sqrt(t)
    psi = psi0 / psi_inf + ra * phi0 * (t - a * m / eta ** 3 * (eta ** 2 * t - 2.0 * eta * st + 2.0 * np.log1p(eta * st)))
    r = np.asarray(r, dtype=np.float64)
    if t <= 0.0:
        return psi, np.ones_like(r)
    phi = 1.0 - m * a * st / (1.0 + eta * st) * (R / r) * erfc((r - R) / (2.0 * np.sqrt(D * t)))
    return psi, phi


def adsorption_validation(R, precision, taus=(0.011, 0.022, 0.044, 0.089, 0.22, 0.55, 1.11, 3.0), samples=60):
    """Uptake of bulk surfactant onto a stationary drop (Sec 3.1, workload
    adsorption_3d): psi / psi_inf on the interface (mean over nodes with
    |rhoN| <= 0.2) against eq 30, and the radial profile of phi / phi0 at the
    paper's times tau = D_b t / R^2 against eq 29 over R + 3 <= r <= 2.5 R (the
    half-width of the periodic cell), outside the diffuse interface."""
    import workloads as W
    from paper_2311_15242_amd import lbfd

    say = lambda *a: print("[adsorption]", *a, file=sys.stderr, flush=True)
    p, q = W.adsorption_3d(R=R, precision=precision)
    D, ra, pinf, phi0 = p["Db"], p["ra"], p["psi_inf"], q["phi0_out"]
    n = p["nx"]
    c = q["drops"][0][0]
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    rr = np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2)
    edges = np.arange(R + 3.0, 2.5 * R + 1e-9, 1.0)
    mids = 0.5 * (edges[:-1] + edges[1:])
    shell = np.digitize(rr.ravel(), edges) - 1
    inb = (shell >= 0) & (shell < mids.size)
    counts = np.bincount(shell[inb], minlength=mids.size)
    s = lbfd.Solver(p).init_fields(q)
    t_end = int(round(max(taus) * R * R / D))
    marks = sorted(set([int(round(tau * R * R / D)) for tau in taus] +
                       [int(round(t_end * (i + 1) / samples)) for i in range(samples)]))
    hist, prof = [], []
    t0 = time.time()
    step = 0
    for tm in marks:
        s.step(tm - step)
        step = tm
        rN, psi = s.field("rhoN"), s.field("psi")
        band = np.abs(rN) <= 0.2
        ps = float(psi[band].mean()) / pinf
        th, _ = adsorption_theory(float(step), [R], R, D, ra, pinf, phi0)
        hist.append((step, ps, float(th)))
        tau = D * step / (R * R)
        for tt in taus:
            if int(round(tt * R * R / D)) == step:
                phi = s.field("phi").ravel()
                sim = np.bincount(shell[inb], weights=phi[inb], minlength=mids.size) / np.maximum(counts, 1) / phi0
                _, thp = adsorption_theory(float(step), mids, R, D, ra, pinf, phi0)
                prof.append(dict(tau=tt, step=step, max_abs_err=round(float(np.abs(sim - thp).max()), 5),
                                 r_over_R=[round(v, 3) for v in (mids / R)[::6]],
                                 sim=[round(float(v), 4) for v in sim[::6]],
                                 theory=[round(float(v), 4) for v in thp[::6]]))
                say(f"tau={tt}: phi* max |sim - eq 29| = {prof[-1]['max_abs_err']:.4f}")
        if len(hist) % 10 == 0:
            say(f"step {step}/{t_end} (tau {tau:.3f}): psi/psi_inf {ps:.5f}, eq 30 {float(th):.5f} "
                f"({time.time() - t0:.1f} s)")
    ob = s.observables()
    s.close()
    h = np.array(hist)
    taus_h = D * h[:, 0] / (R * R)
    sel = taus_h >= 0.1
    rel = np.abs(h[sel, 1] - h[sel, 2]) / h[sel, 2]
    pick = lambda tt: h[np.argmin(np.abs(taus_h - tt))]
    return dict(workload=f"adsorption onto a stationary drop, R={R}, periodic {n}^3 cube, {precision}",
                status=ob["status"], steps=step, seconds=round(time.time() - t0, 1),
                psi_max_rel_err_tau_ge_0p1=round(float(rel.max()), 4),
                psi=[dict(tau=tt, sim=round(float(pick(tt)[1]), 6), eq30=round(float(pick(tt)[2]), 6))
                     for tt in (0.1, 0.5, 1.0, 2.0, 3.0)],
                phi_profiles=prof)


def retardation_study(R, precision, tau_eo1=25.0, tau_eo10=40.0, buoyancy_ref=1):
    """Surfactant retardation of the rising bubble (Sec 3.4, 2R/L_x = 0.4,
    5R x 5R x 10R): Eo = 1 clean against surfactant-laden (Bi = 10), and Eo = 10
    clean against Bi = 0.5, 1 and 10, with the other groups of the paper (Mo =
    0.1, E0 = 0.5, Pe = 10, k = 1, x_in = 0). The paper prints no numbers for
    these cases, only orderings, which are checked here: the surfactant slows
    the bubble, at Eo = 1 its velocity first rises and then falls to a lower
    steady value, at Eo = 10 the Reynolds number grows with Bi and the
    retardation is weaker than at Eo = 1, the final psi_av hardly depends on
    Bi, and with growing Bi psi_min rises while psi_max falls. Times in
    tau = t / sqrt(2R/g)."""
    import workloads as W
    from paper_2311_15242_amd import lbfd

    say = lambda *a: print("[retardation]", *a, file=sys.stderr, flush=True)
    cases = [("Eo1 clean", 1.0, None, tau_eo1), ("Eo1 Bi10", 1.0, 10.0, tau_eo1),
             ("Eo10 clean", 10.0, None, tau_eo10), ("Eo10 Bi0.5", 10.0, 0.5, tau_eo10),
             ("Eo10 Bi1", 10.0, 1.0, tau_eo10), ("Eo10 Bi10", 10.0, 10.0, tau_eo10)]
    out = {}
    for name, Eo, Bi, tau_end in cases:
        p, q = W.bubble_rise(nx=5 * R, ny=5 * R, nz=10 * R, radius=float(R), Eo=Eo, Mo=0.1,
                             Bi=Bi if Bi is not None else 1.0, clean=Bi is None, precision=precision,
                             buoyancy_ref=buoyancy_ref)
        g = -p["gravity"][2]
        drho = p["rhoB0"] - p["rhoR0"]
        muB, muR = p["muB0"], p["muR0"]
        u_th = (2.0 / 3.0) * g * drho * R * R / muB * (muB + muR) / (2.0 * muB + 3.0 * muR)
        t_ref = np.sqrt(2.0 * R / g)
        n_steps = int(round(tau_end * t_ref))
        chunk = max(1, n_steps // 200)
        s = lbfd.Solver(p).init_fields(q)
        t0 = time.time()
        hist = []
        step = 0
        while step < n_steps:
            s.step(chunk)
            step += chunk
            ob = s.observables()
            hist.append((step / t_ref, ob["velocity"][2], ob["psi_av"], ob["psi_min"], ob["psi_max"]))
            if len(hist) % 40 == 0:
                say(f"{name}: tau {step / t_ref:.1f}/{tau_end}, U/U_th {ob['velocity'][2] / u_th:.4f} "
                    f"({time.time() - t0:.1f} s)")
        if s.observables()["status"] != 0:
            raise RuntimeError(f"{name}: status {s.observables()['status']}")
        s.close()
        h = np.array(hist)
        tail = h[h[:, 0] >= 0.9 * tau_end]
        u_end = float(tail[:, 1].mean())
        ipk = int(np.argmax(h[:, 1]))
        out[name] = dict(u_over_uth=round(u_end / u_th, 4), re=round(2.0 * p["rhoB0"] * u_end * R / muB, 3),
                         peak_u_over_uth=round(float(h[ipk, 1]) / u_th, 4), peak_tau=round(float(h[ipk, 0]), 2),
                         psi_av=round(float(tail[:, 2].mean()), 5), psi_min=round(float(tail[:, 3].mean()), 5),
                         psi_max=round(float(tail[:, 4].mean()), 5), steps=step, seconds=round(time.time() - t0, 1),
                         u_history=[[round(float(a), 2), round(float(b) / u_th, 4)] for a, b in h[::20, :2]])
        say(f"{name}: U/U_th {out[name]['u_over_uth']}, Re {out[name]['re']}, peak {out[name]['peak_u_over_uth']} "
            f"at tau {out[name]['peak_tau']}, psi_av {out[name]['psi_av']}")
    c1, s1 = out["Eo1 clean"], out["Eo1 Bi10"]
    c10 = out["Eo10 clean"]
    b = [out["Eo10 Bi0.5"], out["Eo10 Bi1"], out["Eo10 Bi10"]]
    ret1 = 1.0 - s1["re"] / c1["re"]
    ret10 = 1.0 - b[2]["re"] / c10["re"]
    checks = dict(
        eo1_surfactant_slower=s1["re"] < c1["re"],
        eo1_rises_then_falls=s1["peak_u_over_uth"] > s1["u_over_uth"] * 1.01,
        eo10_surfactant_slower=all(x["re"] < c10["re"] for x in b),
        eo10_re_grows_with_bi=b[0]["re"] < b[1]["re"] < b[2]["re"],
        weaker_at_eo10=ret10 < ret1,
        psi_av_spread_over_bi=round((max(x["psi_av"] for x in b) - min(x["psi_av"] for x in b)) /
                                    max(x["psi_av"] for x in b), 4),
        psi_min_grows_with_bi=b[0]["psi_min"] < b[1]["psi_min"] < b[2]["psi_min"],
        psi_max_falls_with_bi=b[0]["psi_max"] > b[1]["psi_max"] > b[2]["psi_max"])
    return dict(workload=f"surfactant retardation of the rising bubble, R={R}, 2R/L_x=0.4, {precision}, "
                         f"buoyancy_ref={buoyancy_ref}",
                retardation_eo1=round(ret1, 4), retardation_eo10_bi10=round(ret10, 4), checks=checks, cases=out)


def radial_uptake(R, R_out, D, ra, rd, psi_inf, phi0, times, source_mode=0, nr=800, dt=0.5, dt_rel=0.0):
    """Sharp-interface reference of uptake onto a circular drop (the 2-D
    analogue of eq 30): bulk diffusion d phi/dt = D r^-1 d/dr(r d phi/dr) on
    R < r < R_out with no flux at R_out, the flux D d phi/dr = j into the
    interface at r = R, and d psi/dt = j, with j of eq 22 (source_mode 0) or
    ra psi_inf phi (1). Finite volumes in r (the first cell's value stands for
    the surface value) and Crank-Nicolson in t for phi and psi together; the
    product phi (psi_inf - psi) of eq 22 is linearised about the mid-step psi,
    re-estimated three times per step. The interface takes exactly what the
    bulk loses, so R psi + sum r dr phi is conserved. Time steps of
    max(dt, dt_rel t). Returns psi at the given times and the final profile
    (r, phi)."""
    from scipy.linalg import solve_banded

    dr = (R_out - R) / nr
    rc = R + (np.arange(nr) + 0.5) * dr
    rf = R + np.arange(nr + 1) * dr
    vol = rc * dr
    cf = D * rf / dr                      # face conductances per unit angle
    cf[0] = 0.0
    cf[-1] = 0.0
    # (L phi)_i = di_i phi_i + up_i phi_{i+1} + lo_i phi_{i-1}: face fluxes into cell i
    lo = np.zeros(nr)
    up = np.zeros(nr)
    di = np.zeros(nr)
    di[:-1] -= cf[1:-1]
    up[:-1] += cf[1:-1]
    di[1:] -= cf[1:-1]
    lo[1:] += cf[1:-1]
    phi = np.full(nr, float(phi0))
    psi = 0.0
    out = []
    t = 0.0
    for target in sorted(times):
        while target - t > 1e-12:
            h = min(max(dt, dt_rel * t), target - t)
            Lphi = di * phi + np.concatenate([[0.0], lo[1:] * phi[:-1]]) + np.concatenate([up[:-1] * phi[1:], [0.0]])
            psi_mid = psi
            for _ in range(3):
                # j = (a phi_mid - rd psi^n) / (1 + c) with c = h rd / 2 and phi_mid the
                # mean of the old and new surface values (psi of eq 22 at the mid step)
                if source_mode == 1:
                    a, c, b = ra * psi_inf, 0.0, 0.0
                else:
                    a, c, b = ra * (psi_inf - psi_mid), 0.5 * h * rd, rd * psi
                alpha, beta = a / (1.0 + c), -b / (1.0 + c)
                A = np.zeros((3, nr))
                A[0, 1:] = -0.5 * up[:-1]
                A[1, :] = vol / h - 0.5 * di
                A[2, :-1] = -0.5 * lo[1:]
                A[1, 0] += 0.5 * R * alpha
                rhs = vol / h * phi + 0.5 * Lphi
                rhs[0] += -0.5 * R * alpha * phi[0] - R * beta
                new = solve_banded((1, 1), A, rhs)
                j = alpha * 0.5 * (phi[0] + new[0]) + beta
                psi_new = psi + h * j
                psi_mid = 0.5 * (psi + psi_new)
            phi, psi = new, psi_new
            t += h
        out.append(psi)
    return np.array(out), rc, phi


def uptake_validation(precision="fp64", times=(100, 250, 500, 1000, 2000, 5000, 10000, 20000, 50000, 100000)):
    """The adsorption workload (droplet128: D2Q9 128 x 128 periodic, R = 25,
    Langmuir kinetics of eq 22) against the sharp-interface reference
    radial_uptake on the disk of the box's area: the interface concentration
    psi_av = sum G psi / sum G of the solver at the given times."""
    import workloads as W
    from paper_2311_15242_amd import lbfd

    say = lambda *a: print("[uptake]", *a, file=sys.stderr, flush=True)
    p, q = W.droplet_adsorption(precision=precision)
    R = q["drops"][0][3]
    R_out = p["nx"] / np.sqrt(np.pi)
    s = lbfd.Solver(p).init_fields(q)
    t0 = time.time()
    sim = []
    step = 0
    for t in times:
        s.step(t - step)
        step = t
        sim.append(s.observables()["psi_av"])
        say(f"t={t}: psi_av {sim[-1]:.6f} ({time.time() - t0:.1f} s)")
    status = s.observables()["status"]
    s.close()
    ref, _, _ = radial_uptake(R, R_out, p["Db"], p["ra"], p["rd"], p["psi_inf"], q["phi0_out"],
                              [float(t) for t in times], source_mode=p["source_mode"], dt_rel=2e-3)
    rel = [round(float(a / b - 1.0), 4) for a, b in zip(sim, ref)]
    return dict(workload=f"uptake onto the droplet128 drop (D2Q9 128^2, R={R}), {precision}", status=status,
                seconds=round(time.time() - t0, 1), times=list(times), psi_sim=[round(float(v), 6) for v in sim],
                psi_sharp=[round(float(v), 6) for v in ref], rel_diff=rel)


def shear_study(precision="fp64", R=50, sigma0=5e-4):
    """The surfactant-covered drop in simple shear of Sec 3.3 (D2Q9, [-6R, 6R] x
    [-2R, 2R], walls moving at -/+u_w, Re = 1, Ca = 0.5, lambda = 1, Pe_s = 10,
    E0 = 0.3, x_in = 0.5, h = 0.5, Bi = 1, k = 1, sigma0 = 5e-4, so u_w follows
    from Ca and Re): soluble cases with Pe_b = 0.1, 1 and 10 and an insoluble
    one (no exchange). The paper compares shapes with another code's figures,
    which are not available here; the orderings its text states are checked:
    each soluble drop is more deformed than the insoluble one at tau = 4 and 8
    (tau = shear rate x t), deformation falls as Pe_b grows, psi is highest at
    the poles and lowest at the equator, and the insoluble case has the least
    uniform psi."""
    import workloads as W
    from paper_2311_15242_amd import lbfd

    say = lambda *a: print("[shear]", *a, file=sys.stderr, flush=True)
    # sigma0 = mu U / Ca with mu = U R / Re (rho = 1) gives U^2 = sigma0 Re Ca / R
    Re, Ca = 1.0, 0.5
    U = np.sqrt(sigma0 * Re * Ca / R)
    u_w = 2.0 * U
    cases = [("Pe_b 0.1", dict(Pe_b=0.1)), ("Pe_b 1", dict(Pe_b=1.0)), ("Pe_b 10", dict(Pe_b=10.0)),
             ("insoluble", dict(Pe_b=1.0, ra=0.0, rd=0.0))]
    out = {}
    for name, over in cases:
        extra = {kk: v for kk, v in over.items() if kk in ("ra", "rd")}
        p, q = W.shear_droplet(nx=12 * R, ny=4 * R, radius=float(R), u_w=u_w, Ca=Ca, Re=Re, Pe_s=10.0,
                               Pe_b=over["Pe_b"], Bi=1.0, E0=0.3, x_in=0.5, h=0.5, k=1.0, precision=precision,
                               **extra)
        shear = 2.0 * u_w / p["ny"]
        s = lbfd.Solver(p).init_fields(q)
        t0 = time.time()
        res = {}
        step = 0
        for tau in (4.0, 8.0):
            n_t = int(round(tau / shear))
            s.step(n_t - step)
            step = n_t
            ob = s.observables()
            rec = dict(deformation=round(ob["deformation"], 4))
            if tau == 4.0:
                # psi at the interface by angle from the major axis of the drop
                rN, psi = s.field("rhoN")[0], s.field("psi")[0]        # the one plane of the 2-D grid
                ys, xs = np.nonzero(np.abs(rN) <= 0.2)
                cx, cy = ob["centroid"][0], ob["centroid"][1]
                sxx, syy, sxy = ob["second"][0], ob["second"][1], ob["second"][3]
                ang = 0.5 * np.arctan2(2.0 * sxy, sxx - syy)           # major axis
                dx, dy = xs - cx, ys - cy
                c = np.abs(dx * np.cos(ang) + dy * np.sin(ang)) / np.maximum(np.hypot(dx, dy), 1e-12)
                pv = psi[ys, xs] / q["psi0"]
                rec.update(psi_poles=round(float(pv[c > 0.95].mean()), 4), psi_equator=round(float(pv[c < 0.3].mean()), 4),
                           psi_spread=round(float(ob["psi_max"] - ob["psi_min"]) / q["psi0"], 4),
                           incline_deg=round(float(np.degrees(ang)), 2))
            res[f"tau{int(tau)}"] = rec
            say(f"{name}: tau {tau}: {rec} ({time.time() - t0:.1f} s)")
        res["status"] = s.observables()["status"]
        s.close()
        out[name] = res
    sol = ["Pe_b 0.1", "Pe_b 1", "Pe_b 10"]
    D = lambda nm, t: out[nm][t]["deformation"]
    checks = dict(
        soluble_more_deformed=all(D(nm, t) > D("insoluble", t) for nm in sol for t in ("tau4", "tau8")),
        deformation_falls_with_pe_b=all(D(sol[0], t) > D(sol[1], t) > D(sol[2], t) for t in ("tau4", "tau8")),
        psi_highest_at_poles=all(out[nm]["tau4"]["psi_poles"] > out[nm]["tau4"]["psi_equator"] for nm in out),
        insoluble_least_uniform=all(out["insoluble"]["tau4"]["psi_spread"] > out[nm]["tau4"]["psi_spread"] for nm in sol))
    return dict(workload=f"surfactant-covered drop in simple shear, R={R}, {12 * R}x{4 * R}, Ca=0.5, {precision}",
                u_w=round(float(u_w), 6), checks=checks, cases=out)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(p, q, budget_s, warmup=0, min_steps=1):
    """Whole FP64 oracle steps of a workload after `warmup` untimed steps, as many
    as fit the time budget (at least min_steps): (MLUPS, steps, seconds)."""
    import oracle

    o = oracle.Oracle(dict(p, precision="fp64")).init(q)
    if warmup:
        o.step(warmup)
    t0 = time.perf_counter()
    o.step(min_steps)
    per = (time.perf_counter() - t0) / min_steps
    steps = min_steps + int(max(0.0, budget_s - per * min_steps) // per)
    if steps > min_steps:
        o.step(steps - min_steps)
    dt = time.perf_counter() - t0
    return o.N * steps / dt / 1e6, steps, dt


def cpu_baseline(p, q, budget_s):
    """The oracle as it stands, timed on the host cores: whole FP64 steps of the
    same workload, as many as fit the time budget, on every core the OpenMP
    runtime offers, then one step on a single thread."""
    import oracle

    cores = oracle.threads()
    mlups, steps, dt = _oracle_rate(p, q, budget_s)
    oracle.set_threads(1)
    m1, s1, d1 = _oracle_rate(p, q, 0.0)
    oracle.set_threads(cores)
    return dict(value=round(mlups, 4), unit="MLUPS", cores=cores, kind="oracle", cpu_model=cpu_model(),
                one_thread_mlups=round(m1, 4),
                sample=f"{steps} FP64 step(s) of the same {p['nx']}x{p['ny']}x{p['nz']} workload after "
                       f"initialisation on {cores} threads, {dt:.1f} s; {s1} step on 1 thread, {d1:.1f} s")


def cpu_windows():
    """The oracle over fixed windows on every host core (droplet128 2000 steps,
    shear512x256 1000 steps, bubble128x128x384 50 steps after 10) and over
    shortened windows on one thread (200, 50 and 1 after 1)."""
    import oracle

    import workloads as W

    cores = oracle.threads()
    rows = [f"CPU: {cpu_model()}, {cores} OpenMP threads (all cores) and 1 thread; FP64 oracle, whole steps"]
    rows.append(f"{'workload':22s} {'threads':>8s} {'warm-up':>8s} {'steps':>6s} {'seconds':>9s} {'MLUPS':>9s}")
    plan = [("droplet128", 2000, 0, 200, 0), ("shear512x256", 1000, 0, 50, 0), ("bubble128x128x384", 50, 10, 1, 1)]
    for name, n_all, w_all, n_one, w_one in plan:
        p, q = W.config(name, "fp64")
        for thr, n, w in ((cores, n_all, w_all), (1, n_one, w_one)):
            oracle.set_threads(thr)
            o = oracle.Oracle(p).init(q)
            if w:
                o.step(w)
            t0 = time.perf_counter()
            o.step(n)
            dt = time.perf_counter() - t0
            rows.append(f"{name:22s} {thr:8d} {w:8d} {n:6d} {dt:9.2f} {o.N * n / dt / 1e6:9.4f}")
            print(rows[-1], file=sys.stderr, flush=True)
            del o
    oracle.set_threads(cores)
    return "\n".join(rows)


KERNEL_CLASS_OF = {"k_collide<": "collide", "k_macro<": "macro", "k_geom<": "geom", "k_fd<": "fd",
                   "k_sor<": "sor", "k_total_part<": "total", "k_force<": "force"}


def kernel_class(name):
    for pat, cls in KERNEL_CLASS_OF.items():
        if pat in name:
            return cls
    return None


def _evidence(path):
    """A profile record under profiles/ if it was taken on the current kernel sources."""
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    return t if t.get("source_hash") == kernel_source_hash() else None


def traffic_for(kernel, launches_per_step=1.0):
    """Measured HBM bytes per launch of a kernel class (scaled FETCH_SIZE +
    WRITE_SIZE, from the profile record), or None."""
    t = _evidence(TRAFFIC_FILE)
    if not t:
        return None
    return t.get("bytes_per_launch", {}).get(kernel)


def _pmc_rows(path):
    import csv

    with open(path) as fh:
        for r in csv.DictReader(fh):
            yield r["Kernel_Name"], float(r["Counter_Value"]), int(r["Grid_Size"])


def pmc_summary(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv):
    """Per-kernel mean FETCH_SIZE and WRITE_SIZE (KiB per dispatch, summed over
    the counter instances of a dispatch) and the HBM bytes they imply once each
    is scaled by what the same counter reads for a plain copy of known size."""
    import collections

    def per_kernel(path):
        acc = collections.defaultdict(list)
        for name, v, _ in _pmc_rows(path):
            acc[name].append(v)
        return {k: (sum(v) / len(v), len(v)) for k, v in acc.items()}

    def copy_kib(path):
        vals = [v for name, v, _ in _pmc_rows(path) if "copy" in name.lower() or "elementwise" in name.lower()]
        return max(vals) if vals else None

    f, w = per_kernel(fetch_csv), per_kernel(write_csv)
    cf, cw = copy_kib(copy_fetch_csv), copy_kib(copy_write_csv)
    nbytes = 1024 * (1 << 20)
    sf = nbytes / (cf * 1024) if cf else float("nan")
    sw = nbytes / (cw * 1024) if cw else float("nan")
    lines = [f"copy calibration: {nbytes} B copied; FETCH_SIZE read {cf} KiB, WRITE_SIZE read {cw} KiB "
             f"-> scale fetch x{sf:.4f}, write x{sw:.4f}",
             f"{'kernel':78s} {'dispatches':>10s} {'FETCH KiB':>12s} {'WRITE KiB':>12s} {'HBM MB/launch':>14s}"]
    for k in sorted(f, key=lambda k: -(f[k][0] + w.get(k, (0, 0))[0])):
        fk, n = f[k]
        wk = w.get(k, (0.0, 0))[0]
        hbm = (fk * sf + wk * sw) * 1024 / 1e6
        lines.append(f"{k[:78]:78s} {n:10d} {fk:12.1f} {wk:12.1f} {hbm:14.2f}")
    return "\n".join(lines)


def trace_summary(stats_csv):
    """Per-kernel table of a rocprofv3 --kernel-trace --stats run (kernel_stats.csv)."""
    import csv

    rows = list(csv.DictReader(open(stats_csv)))
    lines = [f"{'kernel':60s} {'calls':>7s} {'avg us':>10s} {'min us':>10s} {'max us':>10s} {'total %':>8s}"]
    for r in rows:
        name = r["Name"].replace("void lbfd::", "").split("(")[0]
        lines.append(f"{name[:60]:60s} {int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:10.2f} "
                     f"{float(r['MinNs']) / 1e3:10.2f} {float(r['MaxNs']) / 1e3:10.2f} {float(r['Percentage']):8.2f}")
    return "\n".join(lines)


def write_traffic(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, out_path):
    """HBM bytes per launch of every kernel class of the step (scaled FETCH_SIZE +
    WRITE_SIZE), stored with the hash of the kernel sources they were measured on.
    SOR: the mean over the half-sweeps that did work (the launches that found both
    systems converged, and returned at once, move about a thousandth of that)."""
    import collections

    def mean_kib(path):
        acc = collections.defaultdict(list)
        for name, v, _ in _pmc_rows(path):
            c = kernel_class(name)
            if c and not name.split("lbfd::")[-1].startswith("kb_"):
                acc[c].append(v)
        if "sor" in acc:
            top = max(acc["sor"])
            acc["sor"] = [v for v in acc["sor"] if v > 0.1 * top]
        return {c: sum(v) / len(v) for c, v in acc.items()}

    def copy_kib(path):
        vals = [v for name, v, _ in _pmc_rows(path) if "copy" in name.lower()]
        return max(vals) if vals else None

    nbytes = 1024 * (1 << 20)
    sf = nbytes / (copy_kib(copy_fetch_csv) * 1024)
    sw = nbytes / (copy_kib(copy_write_csv) * 1024)
    fk, wk = mean_kib(fetch_csv), mean_kib(write_csv)
    rec = dict(source_hash=kernel_source_hash(), fetch_scale=round(sf, 4), write_scale=round(sw, 4),
               fetch_kib={c: round(v, 1) for c, v in fk.items()}, write_kib={c: round(v, 1) for c, v in wk.items()},
               bytes_per_launch={c: round((fk[c] * sf + wk.get(c, 0.0) * sw) * 1024) for c in fk})
    with open(out_path, "w") as fh:
        json.dump(rec, fh, indent=1)
    return rec


def write_valu(pmc_csv, out_path):
    """VALU instructions per wavefront and wavefronts per launch of every kernel
    class, from a rocprofv3 --pmc SQ_INSTS_VALU SQ_WAVES run, stored with the
    hash of the kernel sources."""
    import collections
    import csv

    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    with open(pmc_csv) as fh:
        for r in csv.DictReader(fh):
            c = kernel_class(r["Kernel_Name"])
            if c and not r["Kernel_Name"].split("lbfd::")[-1].startswith("kb_"):
                acc[c][r["Counter_Name"]].append(float(r["Counter_Value"]))
    rec = dict(source_hash=kernel_source_hash(), classes={})
    for c, d in acc.items():
        v, w = d.get("SQ_INSTS_VALU"), d.get("SQ_WAVES")
        if v and w and sum(w) > 0:
            rec["classes"][c] = dict(valu_per_wave=round(sum(v) / sum(w), 1), waves_per_launch=round(sum(w) / len(w)))
    with open(out_path, "w") as fh:
        json.dump(rec, fh, indent=1)
    return rec


def sor_half_sweeps(p, ob):
    """SOR half-sweeps that did work in a step: K sweeps and, with omega = 1 and
    no seam classes, the red half of sweep K + 1 that found the residual within
    tolerance (otherwise the whole of sweep K + 1 tested it)."""
    if not p["fd_enable"]:
        return 0
    K = max(ob["sor_sweeps"])
    exact = p["sor_omega"] == 1.0 and not any(
        p["bc"][a] == 0 and n % 2 == 1 for a, n in enumerate((p["nx"], p["ny"], p["nz"])) if a < 2 or p["lattice"] == 1)
    return 2 * K + 1 if exact else 2 * K + 2


def _valu_roof(cls, per_launch_s):
    """Issue-rate view of a kernel class from the VALU counter record: lane
    instructions per second against 256 CUs x 64 lanes x 2.4 GHz (one wave64
    VALU instruction per CU per clock; the FP32 FMA rate without packed FP32)."""
    rec = _evidence(VALU_FILE)
    if not rec or cls not in rec["classes"]:
        return None
    c = rec["classes"][cls]
    lane_ops = c["valu_per_wave"] * c["waves_per_launch"] * 64
    achieved = lane_ops / per_launch_s / 1e12
    return dict(achieved=round(achieved, 2), peak=VALU_PEAK_TOPS, unit="T lane-instr/s",
                frac=round(achieved / VALU_PEAK_TOPS, 4), valu_per_wave=c["valu_per_wave"])


def class_rooflines(p, prof, steps, sor_half):
    """Per kernel class: algorithmic bytes per step over its time per step against
    HBM peak, the measured traffic, and (from the VALU counter record) the issue
    rate; `bound` is the roof the kernel is nearer to."""
    N = p["nx"] * p["ny"] * p["nz"]
    out = {}
    for cls, (ms, launches) in prof.items():
        if cls == "other" or launches == 0 or ms <= 0:
            continue
        per_step_s = ms / steps / 1e3
        if cls == "sor":
            nbytes = sor_half * algorithmic_bytes("sor", p) * N
        else:
            # the total class launches a pass over the nodes and a one-workgroup
            # final reduction: its bytes count once per pair
            passes = launches / 2 if cls == "total" else launches
            nbytes = algorithmic_bytes(cls, p) * N * passes / steps
        ach = nbytes / per_step_s / 1e9
        r = dict(achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s", frac=round(ach / HBM_PEAK_GBS, 4),
                 ms_per_step=round(ms / steps, 4), algorithmic_bytes_per_step=nbytes)
        t = traffic_for(cls)
        r["traffic_per_launch"] = t
        v = _valu_roof(cls, ms / launches / 1e3)
        if v:
            r["valu"] = v
        r["bound"] = "alu" if v and v["frac"] >= ALU_BOUND_ISSUE else "hbm"
        r["bound_frac"] = v["frac"] if r["bound"] == "alu" else r["frac"]   # the labelled roof's fraction
        if cls == "sor":
            r["half_sweeps_with_work"] = sor_half
            r["launches_per_step"] = round(launches / steps, 2)
        out[cls] = r
    return out


def headline_roofline(p, kname, per_launch_ms, launches_per_step, share, ms_step):
    """The longest single-pass kernel, timed alone: against HBM with its
    algorithmic bytes, or against the VALU issue peak (bound "alu") where the
    VALU counters show at least ALU_BOUND_ISSUE of it; both figures are kept."""
    N = p["nx"] * p["ny"] * p["nz"]
    abytes = algorithmic_bytes(kname, p) * N
    hbm = abytes / (per_launch_ms / 1e3) / 1e9
    v = _valu_roof(kname, per_launch_ms / 1e3)
    common = dict(kernel=kname, traffic=traffic_for(kname, launches_per_step), algorithmic_bytes_per_launch=abytes,
                  mean_launch_us=round(per_launch_ms * 1e3, 2), share_of_step=round(share, 3),
                  timed_region_ms_per_step=round(ms_step, 4),
                  hbm=dict(achieved=round(hbm, 1), peak=HBM_PEAK_GBS, unit="GB/s", frac=round(hbm / HBM_PEAK_GBS, 4)))
    if v:
        common["valu"] = v
    if v and v["frac"] >= ALU_BOUND_ISSUE:
        return dict(bound="alu", achieved=v["achieved"], peak=v["peak"], unit=v["unit"], frac=v["frac"],
                    valu_per_wave=v["valu_per_wave"], **common)
    return dict(bound="hbm", achieved=round(hbm, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(hbm / HBM_PEAK_GBS, 4), **common)


def autotune(out_path, workload, precision, warmup):
    """Tune the launch shapes of the headline workload (with its measured SOR
    launch budget) and of the 64-instance batch; write the table."""
    import workloads as W
    from paper_2311_15242_amd import autotune as T

    p, q = W.config(workload, precision)
    p["sor_max_sweeps"] = sweep_budget(p, q, max(warmup, 5))
    res = [T.tune_solver(p, q)]
    print(f"[autotune] {res[-1]['key']}: {res[-1]['tuning']} {res[-1]['ms_per_step']} ms "
          f"(default {res[-1]['default_ms_per_step']} ms)", file=sys.stderr, flush=True)
    inst = W.batch_instances(W.load_manifest(), precision="bf16dev")
    plist = [dict(pp) for pp, _ in inst]
    for pp in plist:
        pp["sor_max_sweeps"] = 6
    res.append(T.tune_batch(plist, [qq for _, qq in inst]))
    print(f"[autotune] {res[-1]['key']}: {res[-1]['tuning']} {res[-1]['ms_per_step']} ms "
          f"(default {res[-1]['default_ms_per_step']} ms)", file=sys.stderr, flush=True)
    import torch

    T.write(res, out_path, device=torch.cuda.get_device_name(0))
    return dict(written=out_path, entries=[dict(key=r["key"], tuning=r["tuning"], ms_per_step=r["ms_per_step"],
                                                default_ms_per_step=r["default_ms_per_step"]) for r in res])


def column_rise_report(eos=(1.0, 10.0, 50.0), bis=(None, 0.01, 1.0, 10.0), precision="bf16dev", steps=50000,
                       sor_sweeps=16):
    """The benchmark column itself (D3Q19 128 x 128 x 384, walls in x and y,
    periodic z, bubble diameter 32, density and viscosity ratio 10, Mo = 0.1 at
    Eo = 1, C = 0.5 outside, Gamma = 0) over the configuration's 50 000 steps:
    terminal rise velocity (eq 33, mean over the last tenth of the run) of each
    Eo with a clean interface (bis entry None) and with surfactant at each Biot
    number, and its ratio to the clean run of the same Eo. buoyancy_ref = 1
    (the domain-mean density): with the printed reference the periodic column
    as a whole accelerates and no terminal velocity exists."""
    import workloads as W
    from paper_2311_15242_amd import lbfd

    say = lambda *a: print("[column]", *a, file=sys.stderr, flush=True)
    out = dict(grid=[128, 128, 384], precision=precision, steps=steps, sor_sweeps_launched=sor_sweeps,
               velocity="eq 33, mean over the last tenth; U_th of eq 35", cases={})
    for Eo in eos:
        clean_u = None
        for Bi in bis:
            name = f"Eo{Eo:g} " + ("clean" if Bi is None else f"Bi{Bi:g}")
            p, q = W.bubble_rise(Eo=Eo, Bi=Bi if Bi is not None else 1.0, clean=Bi is None, precision=precision,
                                 buoyancy_ref=1)
            p["sor_max_sweeps"] = sor_sweeps
            g = -p["gravity"][2]
            drho, muB, muR, R = p["rhoB0"] - p["rhoR0"], p["muB0"], p["muR0"], 16.0
            u_th = (2.0 / 3.0) * g * drho * R * R / muB * (muB + muR) / (2.0 * muB + 3.0 * muR)
            chunk = steps // 100
            s = lbfd.Solver(p).init_fields(q)
            t0 = time.time()
            hist = []
            try:
                for c in range(100):
                    s.step(chunk)
                    ob = s.observables()
                    hist.append((ob["velocity"][2], ob["psi_av"], ob["centroid"][2], ob["deformation"]))
                    if c % 25 == 24:
                        say(f"{name}: {(c + 1) * chunk} steps, U/U_th {ob['velocity'][2] / u_th:.4f} "
                            f"({time.time() - t0:.1f} s)")
            except lbfd.LbfdError as e:
                out["cases"][name] = dict(error=str(e), steps_done=len(hist) * chunk)
                say(f"{name}: {e}")
                s.close()
                continue
            s.close()
            h = np.array(hist)
            u_end = float(h[90:, 0].mean())
            rec = dict(u_terminal=float(f"{u_end:.6g}"), u_over_uth=round(u_end / u_th, 4),
                       re=round(2.0 * p["rhoB0"] * u_end * R / muB, 3),
                       u_change_last_tenth=float(f"{abs(h[99, 0] - h[89, 0]) / max(abs(u_end), 1e-30):.3e}"),
                       deformation=round(float(h[99, 3]), 4), seconds=round(time.time() - t0, 1))
            if Bi is None:
                clean_u = u_end
            else:
                rec["psi_av"] = round(float(h[90:, 1].mean()), 5)
                if clean_u:
                    rec["u_over_clean"] = round(u_end / clean_u, 4)
            out["cases"][name] = rec
            say(f"{name}: {json.dumps(rec)}")
    return out


def shear_precision_report(steps=20000, every=1000, field_every=5000):
    """The sheared drop (D2Q9 512 x 256, Sec 3.3 groups) at the eight corners
    Ca in {0.1, 0.4}, Bi in {0.1, 1}, E0 in {0.1, 0.5}, in the FP64, FP32 and
    FP16-deviation modes for `steps` steps. Deformation D(t) every `every` steps
    against the FP64 oracle's curve where tests/golden/make_golden.py stored one,
    and against the FP64 GPU solver (which matches the oracle to 1e-10) at every
    corner; velocity, G psi and psi on the interface band at every `field_every`
    steps against the FP64 GPU solver (max |a - b| / max |b| and RMS / max |b|)."""
    import itertools

    import workloads as W
    from paper_2311_15242_amd import lbfd

    path = os.path.join(ROOT, "tests", "golden", "shear_deformation_20k.json")
    gold = {}
    if os.path.exists(path):
        with open(path) as fh:
            for case in json.load(fh).values():
                gold[tuple(case["params"][k] for k in ("Ca", "Bi", "E0"))] = {r["step"]: r for r in case["records"]}
    def run(prec, cfg):
        p, q = W.shear_droplet(precision=prec, **cfg)
        s = lbfd.Solver(p).init_fields(q)
        D, fields = {}, {}
        for c in range(0, steps + 1, every):
            if c:
                s.step(every)
            ob = s.observables()
            if ob["status"] != 0:
                raise RuntimeError(f"shear {cfg} {prec}: status {ob['status']} at step {c}")
            D[c] = ob["deformation"]
            if c % field_every == 0:
                G, rN, psi = s.field("G"), s.field("rhoN"), s.field("psi")
                fields[c] = (s.field("u"), G * psi, np.where(np.abs(rN) <= 0.5, psi, np.nan))
        s.close()
        return D, fields

    def rel_D(D, ref):
        return max((abs(D[c] - ref[c]) / ref[c] for c in D if c in ref and ref[c] > 1e-3), default=0.0)

    out = dict(steps=steps, grid=[512, 256], D_norm="max over t of |D - D_ref| / D_ref (D_ref > 1e-3)",
               field_norm="max over checkpoints of max |a - b| / max |b| (RMS / max |b|); Gpsi: the "
                          "conserved interface density G psi; psi_band: psi where |rhoN| <= 0.5 (the band of "
                          "psi_av); MLUPS of the three modes on this grid are in the bench line's secondary block",
               corners={})
    for Ca, Bi, E0 in itertools.product((0.1, 0.4), (0.1, 1.0), (0.1, 0.5)):
        cfg = dict(Ca=Ca, Bi=Bi, E0=E0)
        name = f"ca{Ca:g}_bi{Bi:g}_e{E0:g}"
        D64, F64 = run("fp64", cfg)
        orc = gold.get((Ca, Bi, E0))
        rec = dict(D_final_fp64=round(D64[steps], 6), fp64={})
        if orc:
            rec["fp64"]["D_vs_oracle"] = float(f"{rel_D(D64, {c: r['deformation'] for c, r in orc.items()}):.3e}")
        for prec in ("fp32", "fp16dev"):
            D, F = run(prec, cfg)
            e = dict(D_vs_fp64=float(f"{rel_D(D, D64):.3e}"))
            if orc:
                e["D_vs_oracle"] = float(f"{rel_D(D, {c: r['deformation'] for c, r in orc.items()}):.3e}")
            for k, i in (("u", 0), ("Gpsi", 1), ("psi_band", 2)):
                mx = rms = 0.0
                for c in F:
                    a, b = F[c][i], F64[c][i]
                    m = np.isfinite(a) & np.isfinite(b)     # the band of the two runs can differ by a node
                    if not m.any():
                        continue
                    d = np.abs(a[m] - b[m])
                    sc = max(float(np.abs(b[m]).max()), 1e-300)
                    mx = max(mx, float(d.max()) / sc)
                    rms = max(rms, float(np.sqrt(np.mean(d ** 2))) / sc)
                e[k] = float(f"{mx:.3e}")
                e[k + "_rms"] = float(f"{rms:.3e}")
            rec[prec] = e
        out["corners"][name] = rec
        print(f"[shear] {name}: {json.dumps(rec)}", file=sys.stderr, flush=True)
    return out


def accuracy_report(workload, precision, steps):
    """The benchmarked mode and the other deviation mode against the plain FP32
    GPU solver and the FP64 GPU solver (which matches the FP64 oracle to 1e-10)
    on the same workload after the same number of steps: max-norm errors
    relative to the reference field's largest magnitude, and RMS errors."""
    import workloads as W
    from paper_2311_15242_amd import lbfd

    def fields(prec):
        pp, qq = W.config(workload, prec)
        s = lbfd.Solver(pp).init_fields(qq).step(steps)
        ob = s.observables()
        f = dict(u=s.field("u"), Gpsi=s.field("G") * s.field("psi"), rhoN=s.field("rhoN"))
        s.close()
        return f, ob

    ref, _ = fields("fp64")
    base, _ = fields("fp32")

    def errs(a, b):
        out = {}
        for k in ("u", "Gpsi", "rhoN"):
            d = np.abs(a[k] - b[k])
            if d.ndim == 4:
                d = d.max(0)
            m = float(np.abs(b[k]).max())
            out[k] = float(d.max() / m)
            out[k + "_rms"] = float(np.sqrt((d * d).mean()) / m)
        return {k: float(f"{v:.3e}") for k, v in out.items()}

    rep = dict(steps=steps, norm="max |a - b| / max |b| per field (u: over components); _rms: RMS / max |b|",
               target=1e-3, fp32=dict(vs_fp64=errs(base, ref)))
    for prec in dict.fromkeys([precision, "fp16dev", "bf16dev"]):
        if prec in ("fp32", "fp64"):
            continue
        f, _ = fields(prec)
        rep[prec] = dict(vs_fp32=errs(f, base), vs_fp64=errs(f, ref))
    return rep


def sweep_budget(p, q, warmup, margin=2):
    """SOR sweeps to launch per step: the most any warm-up step needed, plus a
    margin. Every step still checks its own convergence on the device; a step
    that does not converge within the budget sets LBFD_ESOR and fails the run."""
    from paper_2311_15242_amd import lbfd

    s = lbfd.Solver(p).init_fields(q)
    used = 0
    n = max(warmup, 1)
    for i in range(n):
        s.step(1)
        ob = s.observables()
        # the first two steps (Euler step, no extrapolated guess yet) are special;
        # the timed steps come after the warm-up
        if i >= 2 or n <= 3:
            used = max(used, *ob["sor_sweeps"])
    s.close()
    return min(used + margin, p["sor_max_sweeps"])


def batch_bench(steps, warmup, sor_sweeps, precision="bf16dev"):
    """The parameter sweep: 64 uneven 2-D bubble columns (the committed
    manifest), advanced as one batch, against the same 64 instances run one
    after another as single solvers. Both use the same SOR launch budget (the
    most any instance needed in the batched warm-up, plus a margin)."""
    import torch

    import workloads as W
    from paper_2311_15242_amd import lbfd

    inst = W.batch_instances(W.load_manifest(), precision=precision)
    nodes = sum(p["nx"] * p["ny"] * p["nz"] for p, _ in inst)

    def new_batch(tuning="auto"):
        b = lbfd.Batch([p for p, _ in inst], tuning=tuning)
        for m, (_, q) in zip(b.members, inst):
            m.init_fields(q)
        return b

    if sor_sweeps == "auto":
        b = new_batch()
        used = 0
        for i in range(max(warmup, 3)):
            b.step(1)
            if i >= 2:
                used = max([used] + [max(m.observables()["sor_sweeps"]) for m in b.members])
        b.close()
        budget = min(used + 2, inst[0][0]["sor_max_sweeps"])
    else:
        budget = int(sor_sweeps)
    for p, _ in inst:
        p["sor_max_sweeps"] = budget

    def check(objs, where):
        bad = [i for i, m in enumerate(objs) if m.observables()["status"] != 0]
        if bad:
            raise RuntimeError(f"instances {bad[:8]} report a solver error {where}")

    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b = new_batch()
    b.step(warmup)
    torch.cuda.synchronize()
    check(b.members, "after the batched warm-up")
    ev0.record()
    b.step(steps)
    ev1.record()
    torch.cuda.synchronize()
    ms_b = ev0.elapsed_time(ev1)
    check(b.members, "in the batched timed region")
    # the state each instance reached, for the comparison with its sequential run
    snap = [(m.field("u"), m.field("psi")) for m in b.members]
    bkey = b.key
    b.close()
    del b
    # the same batch in the library's default launch shape
    b = new_batch(tuning=None)
    b.step(warmup)
    torch.cuda.synchronize()
    ev0.record()
    b.step(steps)
    ev1.record()
    torch.cuda.synchronize()
    ms_bf = ev0.elapsed_time(ev1)
    check(b.members, "in the fixed-shape batched timed region")
    b.close()
    del b

    solvers = [lbfd.Solver(p).init_fields(q) for p, q in inst]
    for s in solvers:
        s.step(warmup)
    torch.cuda.synchronize()
    ev0.record()
    for s in solvers:
        s.step(steps)
    ev1.record()
    torch.cuda.synchronize()
    ms_s = ev0.elapsed_time(ev1)
    check(solvers, "in the sequential timed region")
    diff = 0.0
    for (u, ps), s in zip(snap, solvers):
        diff = max(diff, float(np.abs(s.field("u") - u).max()), float(np.abs(s.field("psi") - ps).max()))
    for s in solvers:
        s.close()
    mb = nodes * steps / (ms_b / 1e3) / 1e6
    ms = nodes * steps / (ms_s / 1e3) / 1e6
    return dict(workload="bubble_rise_batch64: 64 uneven 2-D bubble columns (D2Q9, W 128-256 x H 256-768, "
                         "Eo and Bi swept)", storage=precision, instances=len(inst), nodes=nodes, steps=steps,
                batched_mlups=round(mb, 2), sequential_mlups=round(ms, 2), speedup=round(mb / ms, 3),
                batched_ms_per_step=round(ms_b / steps, 4), sequential_ms_per_step=round(ms_s / steps, 4),
                sor_sweeps_launched=budget, max_abs_diff_vs_sequential=diff,
                tuning=dict(key=bkey, shape=lbfd.tuned_shape(bkey) or lbfd.DEFAULT_TUNING,
                            fixed_mlups=round(nodes * steps / (ms_bf / 1e3) / 1e6, 2),
                            tuned_over_fixed=round(ms_bf / ms_b, 4)),
                accuracy="u and psi of every instance after warm-up + timed steps: batched - sequential")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="bubble128x128x384")
    ap.add_argument("--precision", default=None)
    ap.add_argument("--sor-sweeps", default="auto",
                    help="SOR sweeps launched per step: an integer, or auto (warm-up maximum + 2)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-instance parameter sweep")
    ap.add_argument("--batch-steps", type=int, default=100)
    ap.add_argument("--no-surrogate", action="store_true", help="skip the learned-surrogate measurement")
    ap.add_argument("--validate-rise", type=int, default=0, metavar="R",
                    help="clean bubble terminal velocity against Hadamard-Rybczynski at three confinements (radius R)")
    ap.add_argument("--rise-precision", default="fp32")
    ap.add_argument("--rise-max-steps", type=int, default=80000)
    ap.add_argument("--rise-chunk", type=int, default=2000)
    ap.add_argument("--rise-tol", type=float, default=2e-3)
    ap.add_argument("--rise-cases", default="0.4,0.2,0.1", help="confinement ratios 2R/L_x to run")
    ap.add_argument("--rise-buoyancy-ref", type=int, default=0, help="0: rhoB0 as printed; 1: domain-mean density")
    ap.add_argument("--validate-ygb", type=int, default=0, metavar="R",
                    help="drop migration in an imposed gradient (Sec 3.2) at drop radius R, against eq 32")
    ap.add_argument("--ygb-precision", default="fp32")
    ap.add_argument("--ygb-max-steps", type=int, default=200000)
    ap.add_argument("--ygb-chunk", type=int, default=2000)
    ap.add_argument("--ygb-tol", type=float, default=1e-3)
    ap.add_argument("--ygb-widths", default="5,10", help="box widths L_x = L_y in units of R")
    ap.add_argument("--ygb-min-steps", type=int, default=0)
    ap.add_argument("--validate-adsorption", type=int, default=0, metavar="R",
                    help="uptake onto a stationary 3-D drop of radius R (Sec 3.1) against eqs 29 and 30")
    ap.add_argument("--adsorption-precision", default="fp64")
    ap.add_argument("--validate-retardation", type=int, default=0, metavar="R",
                    help="surfactant retardation of the rising bubble at radius R (Sec 3.4 orderings)")
    ap.add_argument("--retardation-precision", default="fp32")
    ap.add_argument("--validate-uptake", action="store_true",
                    help="the adsorption workload against the sharp-interface radial reference")
    ap.add_argument("--validate-shear", action="store_true",
                    help="orderings of the surfactant-covered drop in simple shear (Sec 3.3)")
    ap.add_argument("--sg-size", type=int, default=256)
    ap.add_argument("--sg-snapshots", type=int, default=16)
    ap.add_argument("--sg-tiles", type=int, default=512, help="training tiles per snapshot")
    ap.add_argument("--sg-train-steps", type=int, default=12000)
    ap.add_argument("--sg-blocks", type=int, default=4)
    ap.add_argument("--sg-lr-final", type=float, default=1e-5,
                    help="Adam step size at the end of a half-cosine decay from 1e-3 (negative: constant)")
    ap.add_argument("--omega", type=float, default=None, help="SOR relaxation factor (default: the workload's)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (scales rocprofv3 byte counters)")
    ap.add_argument("--pmc-summary", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="summarise rocprofv3 FETCH_SIZE / WRITE_SIZE counter CSVs per kernel (scaled by the "
                         "copy calibration run) and exit")
    ap.add_argument("--trace-summary", metavar="KERNEL_STATS_CSV",
                    help="print the per-kernel table of a rocprofv3 --kernel-trace --stats run and exit")
    ap.add_argument("--write-traffic", nargs=5,
                    metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV", "OUT_JSON"),
                    help="store the measured HBM bytes per launch of every kernel class and exit")
    ap.add_argument("--write-valu", nargs=2, metavar=("PMC_CSV", "OUT_JSON"),
                    help="store VALU instructions per wave of every kernel class (SQ_INSTS_VALU, SQ_WAVES) and exit")
    ap.add_argument("--no-fixed-shape", action="store_true",
                    help="skip the comparison run in the default launch shape (profiler runs: one shape per kernel)")
    ap.add_argument("--hbm-probe", action="store_true",
                    help="print the bandwidth of a plain 1 GiB device copy and fill, then exit")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the deviation modes' errors against the FP32 and FP64 GPU solvers")
    ap.add_argument("--accuracy-steps", type=int, default=500)
    ap.add_argument("--autotune", metavar="OUT_JSON",
                    help="tune the launch shapes of the headline workload and of the 64-instance batch, write "
                         "the table to OUT_JSON and exit")
    ap.add_argument("--column-report", default=None, metavar="EOS",
                    help="terminal rise velocity on the benchmark column (128x128x384, 50000 steps) at the "
                         "comma-separated Eo values, clean and at Bi 0.01, 1, 10; print JSON and exit")
    ap.add_argument("--column-precision", default="bf16dev")
    ap.add_argument("--column-bis", default="clean,0.01,1,10")
    ap.add_argument("--column-sweeps", type=int, default=16, help="SOR sweeps launched per step")
    ap.add_argument("--shear-report", action="store_true",
                    help="deformation D(t) of the sheared drop in FP64 / FP32 / FP16-dev against the stored FP64 "
                         "oracle curves (tests/golden/shear_deformation_20k.json), print JSON and exit")
    ap.add_argument("--cpu-windows", action="store_true",
                    help="time the oracle over the fixed windows (C1 2000, C2 1000, C3 10 + 50 steps) on all host "
                         "cores and a shortened window on one thread, print a table and exit")
    args = ap.parse_args()
    if args.pmc_summary:
        print(pmc_summary(*args.pmc_summary))
        return
    if args.trace_summary:
        print(trace_summary(args.trace_summary))
        return
    if args.write_traffic:
        print(json.dumps(write_traffic(*args.write_traffic)))
        return
    if args.write_valu:
        print(json.dumps(write_valu(*args.write_valu)))
        return
    if args.cpu_windows:
        print(cpu_windows(), flush=True)
        return
    if args.column_report:
        eos = tuple(float(e) for e in args.column_report.split(","))
        bis = tuple(None if b == "clean" else float(b) for b in args.column_bis.split(","))
        print(json.dumps(column_rise_report(eos, bis, args.column_precision, sor_sweeps=args.column_sweeps)),
              flush=True)
        return
    if args.shear_report:
        print(json.dumps(shear_precision_report()), flush=True)
        return
    if args.autotune:
        print(json.dumps(autotune(args.autotune, args.workload, args.precision, args.warmup)), flush=True)
        return
    if args.hbm_probe:
        print(json.dumps(hbm_probe()), flush=True)
        return
    if args.copy_calibration:
        import torch

        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps(dict(copy_calibration_bytes=n * 4, repeats=5)))
        return
    if args.validate_shear:
        print(json.dumps(shear_study()), flush=True)
        return
    if args.validate_uptake:
        print(json.dumps(uptake_validation()), flush=True)
        return
    if args.validate_retardation:
        print(json.dumps(retardation_study(args.validate_retardation, args.retardation_precision)), flush=True)
        return
    if args.validate_adsorption:
        print(json.dumps(adsorption_validation(args.validate_adsorption, args.adsorption_precision)), flush=True)
        return
    if args.validate_ygb:
        widths = tuple(float(c) for c in args.ygb_widths.split(","))
        print(json.dumps(ygb_validation(args.validate_ygb, args.ygb_precision, args.ygb_max_steps,
                                        args.ygb_chunk, args.ygb_tol, widths, args.ygb_min_steps)), flush=True)
        return
    if args.validate_rise:
        cases = tuple(float(c) for c in args.rise_cases.split(","))
        print(json.dumps(rise_validation(args.validate_rise, args.rise_precision, args.rise_max_steps,
                                         args.rise_chunk, args.rise_tol, cases, args.rise_buoyancy_ref)), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              f"(the solver runs on a single MI355X; sharding over several GPUs is not implemented).", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    p, q = W.config(args.workload, args.precision)
    if args.omega:
        p["sor_omega"] = args.omega
    p["sor_max_sweeps"] = sweep_budget(p, q, args.warmup) if args.sor_sweeps == "auto" else int(args.sor_sweeps)
    N = p["nx"] * p["ny"] * p["nz"]

    # 1) the headline: the median of TIMED_REGIONS timed regions of K steps each, in
    #    the tuned launch shape (the autotuner's table; the defaults where it has none)
    ms_plain, _, ob, runs = timed_run(p, q, args.steps, args.warmup, profile=False, regions=TIMED_REGIONS)
    value = N * args.steps / (ms_plain / 1e3) / 1e6
    shape = timed_run.shape
    from paper_2311_15242_amd import lbfd as _L
    tuning = dict(key=_L.tuning_key(p), shape=shape, tuned_table_entry=_L.tuned_shape(_L.tuning_key(p)) is not None,
                  fixed_shape=_L.DEFAULT_TUNING)
    if not args.no_fixed_shape:
        ms_fixed, _, _, _ = timed_run(p, q, args.steps, args.warmup, profile=False, regions=TIMED_REGIONS,
                                      tuning=None)
        tuning.update(fixed_mlups=round(N * args.steps / (ms_fixed / 1e3) / 1e6, 2),
                      tuned_over_fixed=round(ms_fixed / ms_plain, 4))
    # 2) every kernel class timed (breakdown; the events add some overhead)
    ms_prof, prof, _, _ = timed_run(p, q, args.steps, args.warmup, profile=True)
    # 3) the longest single-pass kernel timed alone, for the headline roofline
    kname = max((k for k in prof if k not in ("sor", "total", "other")), key=lambda k: prof[k][0])
    ms_k, prof_k, _, _ = timed_run(p, q, args.steps, args.warmup, profile=True, only=[kname])
    kms, klaunch = prof_k[kname]
    per_launch_ms = kms / max(klaunch, 1)
    launches_per_step = klaunch / args.steps
    sor_half = sor_half_sweeps(p, ob)
    rooflines = class_rooflines(p, prof, args.steps, sor_half)
    roof = headline_roofline(p, kname, per_launch_ms, launches_per_step, kms / ms_k, ms_k / args.steps)
    breakdown = {k: dict(ms_per_step=round(v[0] / args.steps, 4), launches_per_step=round(v[1] / args.steps, 2),
                         gbs=rooflines[k]["achieved"] if k in rooflines else 0.0)
                 for k, v in prof.items() if v[1] > 0}

    # whole-step bandwidth: the algorithmic bytes of every kernel of one step (SOR
    # half-sweeps counted for those that ran) x lattice updates per second
    step_bytes = sum(algorithmic_bytes(k, p) for k in ("collide", "macro", "geom", "force")) + \
        (algorithmic_bytes("fd", p) + algorithmic_bytes("total", p) + sor_half * algorithmic_bytes("sor", p)
         if p["fd_enable"] else 0.0)
    step_gbs = step_bytes * value * 1e6 / 1e9
    step_bw = dict(bytes_per_lup=round(step_bytes, 1), sor_half_sweeps_counted=sor_half,
                   achieved=round(step_gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s", frac=round(step_gbs / HBM_PEAK_GBS, 4))
    # useful bandwidth: the minimum state of a two-colour method per update x updates per second
    ub = USEFUL_BYTES[(p["lattice"], p["precision"])]
    useful = dict(bytes_per_lup=ub, achieved=round(ub * value / 1e3, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                  frac=round(ub * value / 1e3 / HBM_PEAK_GBS, 4))
    out = dict(metric="MLUPS (LBM+FD step)", value=round(value, 2), unit="MLUPS", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=round(ms_plain / args.steps, 4), higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="f32" if p["precision"] != "fp64" else "f64",
               data="synthetic",
               config=dict(workload=args.workload, lattice="D3Q19" if p["lattice"] == 1 else "D2Q9",
                           grid=[p["nx"], p["ny"], p["nz"]], storage=p["precision"],
                           sor_sweeps_launched=p["sor_max_sweeps"], sor_sweeps_used=ob["sor_sweeps"],
                           parallelism="single GPU"),
               timed_regions=dict(count=TIMED_REGIONS, statistic="median",
                                  mlups=[round(N * args.steps / (r / 1e3) / 1e6, 1) for r in runs]),
               tuning=tuning, roofline=roof, rooflines=rooflines, step_bandwidth=step_bw, useful_bandwidth=useful,
               kernels=breakdown, ms_per_step_profiled=round(ms_prof / args.steps, 4))
    out["hbm_probe"] = hbm_probe()
    out["roofline"]["frac_of_copy"] = round(out["roofline"]["hbm"]["achieved"] / out["hbm_probe"]["copy_GBps"], 4)
    if not args.no_accuracy:
        out["accuracy"] = accuracy_report(args.workload, p["precision"], args.accuracy_steps)

    if not args.no_secondary:
        sec = {}
        for name, prec in (("shear512x256", "fp64"), ("shear512x256", "fp32"), ("shear512x256", "fp16dev"),
                           ("droplet128", "fp64")):
            pp, qq = W.config(name, prec)
            pp["sor_max_sweeps"] = sweep_budget(pp, qq, 20) if args.sor_sweeps == "auto" else int(args.sor_sweeps)
            nn = pp["nx"] * pp["ny"] * pp["nz"]
            ms2, _, ob2, _ = timed_run(pp, qq, 200, 20, profile=False)
            sec[f"{name}_{prec}"] = dict(mlups=round(nn * 200 / (ms2 / 1e3) / 1e6, 2),
                                         ms_per_step=round(ms2 / 200, 4), sor_sweeps_used=ob2["sor_sweeps"],
                                         sor_sweeps_launched=pp["sor_max_sweeps"])
        out["secondary"] = sec
    if not args.no_batch:
        out["batched"] = batch_bench(args.batch_steps, args.warmup, args.sor_sweeps)
    if not args.no_surrogate:
        out["surrogate"] = surrogate_bench(args.sg_size, args.sg_snapshots, args.sg_tiles, args.sg_train_steps,
                                           args.sg_blocks, args.sg_lr_final if args.sg_lr_final > 0 else None)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, q, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
