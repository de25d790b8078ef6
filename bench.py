#!/usr/bin/env python
"""Throughput of the CRM step on one MI355X: particle-steps/s on the
single-wheel soil bin (200 x 120 x 40 soil particles at dx = 5 mm, container,
grousered wheel driven at slip 0.3 under a 100 N load), then the same step in
its other forms: the 10 km strip with active boxes around a four-wheeled
vehicle at x = 5 km with plain FP32 positions and with cell index + FP32
offset positions, and 64 batched bins in one context.

Every step is one co-simulation exchange as in the paper's FSI loop: the host
(standing in for the multibody side) sets the body states, libcrm advances one
step, and the host reads back the forces (for the wheel bins it integrates the
wheel's free vertical degree of freedom).

Prints one JSON line: the wheel bin's figures as the headline (value, roofline
of k_fluid_stage2, the oracle's CPU baseline, the reverse-mode cost) and each
further form under "forms" with its own rate, ms per step and roofline of its
dominant kernel. With --gpus N > 1 it exits: this build measures one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work of the dominant kernel (soil RHS + stage-2 update + return
# mapping), per neighbour pair and per soil particle:
#   FP32 flops per pair: kernel gradient 12, V_j grad W 4, velocity difference
#   and outer product 21, stress sum and contraction 24, artificial viscosity 19
#   (only pairs with v.r < 0 in the unilateral form; not counted) -> 61.
#   HBM bytes per particle: own y_mid 52 + own y_n 52 + y_{n+1} 52 and
#   row/count/offset words 16; per pair its 16-bit tile position (2 B).
FLOPS_PER_PAIR = 61
BYTES_PER_PARTICLE = 3 * 52 + 16
BYTES_PER_PAIR = 2
PEAK_FP32_TFLOPS = 157.3
TILE_NAMES = ("none", "small", "large")
PEAK_HBM_GBS = 8000.0
# Algorithmic bytes of the activity pass per particle (all N particles, every
# list rebuild with active domains): what decides the flag read (the 12 B of
# FP32 coordinates; in cell-offset form the 8 B of cell indices, which reject
# every particle but the few near a box), one flag byte written.
ACTIVITY_BYTES = {0: 12 + 1, 1: 8 + 1}

# HBM bytes per launch from rocprofv3 FETCH_SIZE and WRITE_SIZE (scaled by a
# plain copy of known size: fetch x2, write x1), with the digest of the kernel
# sources they were taken on; reported only while the sources are unchanged
# (summaries and commands in profiles/).
MEASURED_TRAFFIC = {
    "k_fluid_stage2 wheel bin": dict(bytes=466.16e6, source="e9246f134bbde8ee"),
    "k_activity strip pos_mode 0": dict(bytes=1923.2e6, source="e9246f134bbde8ee"),
    "k_activity strip pos_mode 1": dict(bytes=1334.5e6, source="e9246f134bbde8ee"),
    "k_fluid_stage2 batch small": dict(bytes=1914.5e6, source="e9246f134bbde8ee"),
}
KERNEL_SOURCES = ("crm_kernels.hip", "crm_device.h", "crm_internal.h")


def source_digest():
    h = hashlib.sha256()
    for n in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2507_05643_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(key):
    m = MEASURED_TRAFFIC.get(key)
    if not m or m["bytes"] is None or m["source"] != source_digest():
        return None
    return m["bytes"]


class WheelDriver:
    """Host stand-in for the multibody side: prescribed angular velocity and
    forward speed v = (1 - s) w r_g, free vertical motion under the load."""

    def __init__(self, scene):
        m = scene.meta
        self.omega = m["omega"]
        self.v = (1.0 - m["slip"]) * m["omega"] * m["r_g"]
        self.mass = m["mass"]
        self.g = 9.81
        self.bodies = scene.bodies
        self.x = np.array(scene.bodies[1].pos, dtype=np.float64)
        self.vz = 0.0
        self.theta = 0.0
        nb = len(self.bodies)
        self._pos = np.array([b.pos for b in self.bodies], dtype=np.float64)
        self._quat = np.tile([1.0, 0.0, 0.0, 0.0], (nb, 1))
        self._lin = np.zeros((nb, 3))
        self._ang = np.zeros((nb, 3))
        self._ang[1, 1] = self.omega

    def state(self):
        """Body states (reused arrays, overwritten by the next call)."""
        self._pos[1] = self.x
        h = 0.5 * self.theta
        self._quat[1, 0] = math.cos(h)
        self._quat[1, 2] = math.sin(h)
        self._lin[1, 0] = self.v
        self._lin[1, 2] = self.vz
        return self._pos, self._quat, self._lin, self._ang

    def advance(self, force, dt):
        self.vz += dt * (force[2] / self.mass - self.g)
        self.x[0] += dt * self.v
        self.x[2] += dt * self.vz
        self.theta += dt * self.omega


class BinDrivers:
    """One WheelDriver-like wheel per bin of a batched scene (bodies 2b, 2b + 1)."""

    def __init__(self, scene):
        self.bins = scene.meta["bins"]
        self.bodies = scene.bodies
        nb = len(self.bins)
        self.x = np.array([scene.bodies[2 * k + 1].pos for k in range(nb)], dtype=np.float64)
        self.v = np.array([(1.0 - b["slip"]) * b["omega"] * b["r_g"] for b in self.bins])
        self.omega = np.array([b["omega"] for b in self.bins])
        self.mass = np.array([b["mass"] for b in self.bins])
        self.vz = np.zeros(nb)
        self.theta = np.zeros(nb)

    def state(self, ks=None):
        ks = range(len(self.bins)) if ks is None else ks
        pos, quat, lin, ang = [], [], [], []
        for k in ks:
            c = self.bodies[2 * k]
            pos += [c.pos, self.x[k]]
            quat += [(1.0, 0.0, 0.0, 0.0), (math.cos(0.5 * self.theta[k]), 0.0, math.sin(0.5 * self.theta[k]), 0.0)]
            lin += [(0.0, 0.0, 0.0), (self.v[k], 0.0, self.vz[k])]
            ang += [(0.0, 0.0, 0.0), (0.0, self.omega[k], 0.0)]
        return (np.array(pos, dtype=np.float64), np.array(quat), np.array(lin), np.array(ang))

    def advance(self, fz, dt, ks=None):
        ks = np.arange(len(self.bins)) if ks is None else np.asarray(ks)
        self.vz[ks] += dt * (fz / self.mass[ks] - 9.81)
        self.x[ks, 0] += dt * self.v[ks]
        self.x[ks, 2] += dt * self.vz[ks]
        self.theta[ks] += dt * self.omega[ks]


def stage2_roofline(prof, cnt, key):
    """k_fluid_stage2 against the FP32 vector peak: 61 flops per soil pair over
    the mean launch time (HIP events around that kernel on the context's stream)."""
    st2 = prof["soil_stage2"]
    ms2 = st2["ms"] / max(st2["launches"], 1)
    pairs = prof["soil_pairs"]
    rows = cnt["soil_rows"]
    flops = FLOPS_PER_PAIR * pairs
    bytes_ = BYTES_PER_PARTICLE * rows + BYTES_PER_PAIR * pairs
    tflops = flops / (ms2 * 1e-3) / 1e12
    gbs = bytes_ / (ms2 * 1e-3) / 1e9
    return dict(bound="alu", achieved=round(tflops, 3), peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                frac=round(tflops / PEAK_FP32_TFLOPS, 4), traffic=measured_traffic(key),
                kernel="k_fluid_stage2", launch_ms=round(ms2, 5), algorithmic_flops=flops,
                hbm_view=dict(achieved=round(gbs, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                              frac=round(gbs / PEAK_HBM_GBS, 4), algorithmic_bytes=bytes_))


def activity_roofline(prof, cnt, pos_mode):
    """k_activity (flags of all N particles at each list rebuild) against HBM."""
    act = prof["activity"]
    if act["launches"] == 0:
        return None
    ms = act["ms"] / act["launches"]
    bytes_ = ACTIVITY_BYTES[pos_mode] * cnt["n_total"]
    gbs = bytes_ / (ms * 1e-3) / 1e9
    return dict(bound="hbm", achieved=round(gbs, 1), peak=PEAK_HBM_GBS, unit="GB/s", frac=round(gbs / PEAK_HBM_GBS, 4),
                traffic=measured_traffic(f"k_activity strip pos_mode {pos_mode}"), kernel="k_activity",
                launch_ms=round(ms, 5), algorithmic_bytes=bytes_)


def per_launch(prof):
    return {k: round(v["ms"] / max(v["launches"], 1), 5) for k, v in prof.items() if isinstance(v, dict)}


def timed_steps(step_fn, n_warm, n_steps):
    import torch
    for _ in range(n_warm):
        step_fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_steps):
        step_fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def run_wheel(args, crm, scenes):
    """The single-wheel soil bin, one co-simulation exchange per step (the headline)."""
    import torch
    sc = scenes.wheel_bin(seed=0, ps_freq=args.ps_freq)
    drv = WheelDriver(sc)
    sim = crm.Simulation(sc, device=0)
    dt = sc.params["dt"]

    def one_step():
        F, _ = sim.cosim_step(*drv.state())
        drv.advance(F[1], dt)

    for _ in range(args.warmup):
        one_step()
    tile = sim.autotune() if args.autotune else sim.autotune(TILE_NAMES.index(args.tile))
    torch.cuda.synchronize()
    if args.wheel_graph:
        # the per-step kernels as one graph (the profiling events below would
        # bypass it: the timed region then runs without them)
        sim.graph(True)
        wall = timed_steps(one_step, 0, args.steps)
        sim.profiling(True, classes=["soil_stage2"])
        timed_steps(one_step, 0, min(args.steps, 100))
    else:
        # events around the dominant kernel only, on the context's stream
        sim.profiling(True, classes=["soil_stage2"])
        wall = timed_steps(one_step, 0, args.steps)
    prof = sim.profile()
    # per-class breakdown (every kernel class timed) over a short untimed run
    sim.profiling(True)
    for _ in range(min(args.steps, 10 * args.ps_freq)):
        one_step()
    prof_all = sim.profile()
    sim.profiling(False)
    cnt = sim.counts()
    F, T = sim.forces()
    key = "k_fluid_stage2 wheel bin" if (args.ps_freq == 10 and tile == crm.TILE_SMALL) else None
    roofline = stage2_roofline(prof, cnt, key)
    adjoint = adjoint_cost(sim, one_step, args.adjoint_steps, args.ps_freq, sc.n_soil, len(sc.bodies)) \
        if args.adjoint_steps > 0 else None
    print(json.dumps(dict(form="wheel", profile_ms_per_launch=per_launch(prof_all), counts=cnt,
                          wheel_force=F[1].tolist(), wheel_torque=T[1].tolist(), wheel_z=float(drv.x[2]))),
          file=sys.stderr, flush=True)
    sim.close()
    return dict(value=cnt["n_proc"] * args.steps / wall, wall=wall, cnt=cnt, roofline=roofline, adjoint=adjoint,
                soil_rate=cnt["soil_rows"] * args.steps / wall, breakdown=per_launch(prof_all),
                config={"workload": "single-wheel soil bin: 200x120x40 soil particles (dx 5 mm, seeded jitter) "
                                    "+ 3-layer container + grousered wheel r 0.25 m, slip 0.3, load 100 N; "
                                    "co-simulation exchange every step",
                        "n_particles": cnt["n_total"], "n_processed": cnt["n_proc"], "ps_freq": args.ps_freq,
                        "dt": dt, "lds_tile": TILE_NAMES[tile]})


def run_wheel_trace(args, crm, scenes):
    """The single-wheel bin run for args.trace_steps co-simulation steps from
    rest (20,000 steps = 0.5 s): drawbar pull F_x, vertical force F_z and
    driving torque T_y of the wheel, their means over the last quarter of the
    run, and the wheel's sinkage. Stops at the first non-finite force (the
    library reports it as CRM_E_NONFINITE)."""
    sc = scenes.wheel_bin(seed=0, ps_freq=args.ps_freq)
    drv = WheelDriver(sc)
    sim = crm.Simulation(sc, device=0)
    dt = sc.params["dt"]
    n = args.trace_steps
    F = np.full((n, 3), np.nan)
    T = np.full((n, 3), np.nan)
    z0 = float(drv.x[2])
    t0 = time.perf_counter()
    done, err = 0, None
    try:
        for k in range(n):
            f, t = sim.cosim_step(*drv.state())
            F[k], T[k] = f[1], t[1]
            drv.advance(f[1], dt)
            done = k + 1
            if done % 5000 == 0:
                print(json.dumps(dict(trace_step=done, Fx=F[k, 0], Fz=F[k, 2], Ty=T[k, 1],
                                      wheel_z=float(drv.x[2]))), file=sys.stderr, flush=True)
    except crm.CrmError as e:
        err = str(e)
    wall = time.perf_counter() - t0
    sim.close()
    q = slice(max(done - max(done // 4, 1), 0), done)
    load = drv.mass * drv.g
    every = max(n // 40, 1)
    return dict(steps=n, steps_done=done, error=err, wall_s=round(wall, 2), ms_per_step=wall / max(done, 1) * 1e3,
                t_end=done * dt, load_N=load,
                last_quarter=dict(Fx_mean=float(np.mean(F[q, 0])), Fz_mean=float(np.mean(F[q, 2])),
                                  Fz_std=float(np.std(F[q, 2])), Ty_mean=float(np.mean(T[q, 1])),
                                  Fz_over_load=float(np.mean(F[q, 2]) / load)),
                sinkage_m=z0 - float(drv.x[2]), finite=bool(np.isfinite(F[:done]).all() and np.isfinite(T[:done]).all()),
                trace_every=every, trace=dict(Fx=F[::every, 0].round(4).tolist(), Fz=F[::every, 2].round(4).tolist(),
                                              Ty=T[::every, 1].round(5).tolist()))


def strip_at(sc, x0):
    """The strip scene with the vehicle moved so that its centre is at x = x0
    (the soil and the floor are shared, not copied)."""
    import dataclasses
    cx = 0.5 * (sc.bodies[1].pos[0] + sc.bodies[-1].pos[0])
    bodies = [sc.bodies[0]] + [dataclasses.replace(b, pos=(b.pos[0] + (x0 - cx), b.pos[1], b.pos[2]))
                               for b in sc.bodies[1:]]
    return dataclasses.replace(sc, bodies=bodies)


def strip_subpatch(sc, xc, half=0.5):
    """A 2 half x 4 m sub-patch of the strip around x = xc: its soil particles
    (stored FP32 coordinates, as the strip holds them) and the floor markers
    below them, in a domain of their own; no wheel. Settles under gravity."""
    import dataclasses
    from paper_2507_05643_amd import scenes
    p = np.asarray(sc.pos, dtype=np.float64)
    keep = (p[:, 0] >= xc - half) & (p[:, 0] < xc + half)
    fl = sc.bodies[0]
    m = np.asarray(fl.markers, dtype=np.float64)
    mk = (m[:, 0] >= xc - half - 0.2) & (m[:, 0] < xc + half + 0.2)
    dx = sc.params["dx"]
    lo = (xc - half - 0.2 - 4 * dx, sc.params["domain_lo"][1], sc.params["domain_lo"][2])
    hi = (xc + half + 0.2 + 4 * dx, sc.params["domain_hi"][1], sc.params["domain_hi"][2])
    params = dict(sc.params, domain_lo=lo, domain_hi=hi, active_domains=0, ps_freq=10)
    floor = scenes.Body(markers=np.ascontiguousarray(m[mk].astype(np.float32)), name="floor")
    return dataclasses.replace(sc, pos=np.ascontiguousarray(p[keep].astype(np.float32)), vel=None, sigma=None,
                               rho=None, bodies=[floor], params=params, name="strip_subpatch")


def subpatch_drift(sc, crm, steps=100):
    """Positions after `steps` steps of the strip's sub-patch at x ~ 9,999 m,
    GPU (plain FP32 and cell-offset positions) against the FP64 oracle: the
    displacement error max |x_gpu - x_oracle| over the largest displacement."""
    from oracle.oracle import Oracle
    orc = Oracle(sc, nbr_mode="cells")
    t0 = time.perf_counter()
    orc.step(steps)
    t_orc = time.perf_counter() - t0
    n = sc.n_soil
    x0 = np.asarray(sc.pos, dtype=np.float64)
    xr = orc.state()["pos"][:n]
    dmax = float(np.abs(xr - x0).max())
    out = dict(x_centre=round(float(x0[:, 0].mean()), 3), n_soil=n, n_particles=sc.n_total, steps=steps,
               oracle_max_displacement_m=dmax,
               oracle_particle_steps_per_s=sc.n_total * steps / t_orc)
    for mode in (0, 1):
        sim = crm.Simulation(sc, params=dict(sc.params, pos_mode=mode), device=0)
        sim.step(steps)
        xg = sim.state()["pos"][:n]
        sim.close()
        out[f"displacement_error_pos_mode_{mode}"] = float(np.abs(xg - xr).max() / dmax)
    return out


def run_strip(args, crm, scenes, pos_mode, sc=None, scan=0):
    """Long strip with four wheels carrying active boxes, positions plain FP32
    (pos_mode 0) or cell index + FP32 offset (pos_mode 1); the vehicle sits at
    x = args.strip_x and moves with the wheels' speed. Active-domain flags from
    the coarse-cell index (scan 0, the library's default) or from the test of
    all N particles (scan 1, the paper's pass; its k_activity roofline)."""
    if sc is None:
        sc = scenes.strip(seed=0, length=args.strip_length, x0=args.strip_x, ps_freq=args.ps_freq, t_delay=-1.0)
    params = dict(sc.params, pos_mode=pos_mode, activity_scan=scan)
    dt = params["dt"]
    t0 = time.perf_counter()
    sim = crm.Simulation(sc, params=params, device=0)
    t_init = time.perf_counter() - t0
    sim.graph(True)
    pos0 = np.array([b.pos for b in sc.bodies], dtype=np.float64)
    quat = np.tile([1.0, 0.0, 0.0, 0.0], (len(sc.bodies), 1))
    lin = np.array([b.linvel for b in sc.bodies])
    ang = np.array([b.angvel for b in sc.bodies])
    state = {"k": 0}

    def one_step():
        p = pos0.copy()
        p[1:, 0] += lin[1:, 0] * dt * state["k"]
        sim.cosim_step(p, quat, lin, ang)
        state["k"] += 1

    steps = args.strip_steps
    wall = timed_steps(one_step, args.form_warmup, steps)
    sim.profiling(True)
    for _ in range(2 * args.ps_freq):
        one_step()
    prof = sim.profile()
    sim.profiling(False)
    cnt = sim.counts()
    sim.close()
    roof = activity_roofline(prof, cnt, pos_mode) if scan else None
    bd = per_launch(prof)
    return dict(value=cnt["n_proc"] * steps / wall, ms_per_step=wall / steps * 1e3, steps=steps,
                warmup=args.form_warmup, soil_rate=cnt["soil_rows"] * steps / wall, roofline=roof,
                activity_flags="test of all N" if scan else "coarse-cell index",
                activity_launch_ms=bd.get("activity"), breakdown=bd, init_s=round(t_init, 1),
                config={"workload": f"strip {args.strip_length:g} m x 4 m x 0.3 m at dx 0.05 m (seeded jitter), "
                                    f"3-layer floor, 4 wheels at 5 m/s at x = {args.strip_x:g} m with 2 m active "
                                    f"boxes, {'cell index + FP32 offset' if pos_mode else 'plain FP32'} positions",
                        "pos_mode": pos_mode, "n_particles": cnt["n_total"], "n_processed": cnt["n_proc"],
                        "ps_freq": args.ps_freq, "dt": dt})


def run_batch(args, crm, scenes):
    """Batched bins: one context for all bins (the step kernels replayed as a
    hipGraph) vs one context per bin, stepped one after the other on the same
    stream."""
    sc = scenes.batch_bins(seed=0, ps_freq=args.ps_freq)
    dt = sc.params["dt"]
    nbins = len(sc.meta["bins"])
    drv = BinDrivers(sc)
    sim = crm.Simulation(sc, device=0)
    sim.set_materials(sc.meta["materials"], sc.meta["material"])
    sim.graph(True)

    def step_batched():
        F, _ = sim.cosim_step(*drv.state())
        drv.advance(F[1::2, 2], dt)

    step_batched()
    tile = sim.autotune()
    steps = args.batch_steps
    wall = timed_steps(step_batched, args.form_warmup, steps)
    sim.profiling(True, classes=["soil_stage2"])
    for _ in range(2 * args.ps_freq):
        step_batched()
    prof = sim.profile()
    sim.profiling(False)
    cnt = sim.counts()
    sim.close()
    roof = stage2_roofline(prof, cnt, f"k_fluid_stage2 batch {TILE_NAMES[tile]}" if args.ps_freq == 10 else None)
    value = cnt["n_proc"] * steps / wall

    # one context per bin
    drv2 = BinDrivers(sc)
    sims = []
    for k in range(nbins):
        one = scenes.batch_bins(seed=0, ps_freq=args.ps_freq, only=[k])
        s1 = crm.Simulation(one, device=0)
        s1.set_materials(one.meta["materials"], one.meta["material"])
        s1.graph(True)
        s1.set_bodies(*drv2.state([k]))
        s1.step(1)
        s1.autotune()
        sims.append(s1)

    def step_separate():
        fz = np.array([s1.cosim_step(*drv2.state([k]))[0][1, 2] for k, s1 in enumerate(sims)])
        drv2.advance(fz, dt)

    n_sep = max(1, steps // 4)
    wall2 = timed_steps(step_separate, max(1, args.form_warmup // 4), n_sep)
    for s1 in sims:
        s1.close()
    value2 = cnt["n_proc"] * n_sep / wall2
    return dict(value=value, ms_per_step=wall / steps * 1e3, steps=steps, warmup=args.form_warmup,
                soil_rate=cnt["soil_rows"] * steps / wall, roofline=roof,
                separate_contexts=dict(value=value2, ms_per_step=wall2 / n_sep * 1e3, steps=n_sep),
                batched_over_separate=value / value2,
                config={"workload": f"{nbins} independent single-wheel bins, sizes log-uniform 8k-250k soil "
                                    "particles (seed 0), per-bin friction 0.5-0.9, slip 0-0.6, load 50-200 N, "
                                    "one context, step kernels replayed as a hipGraph",
                        "n_bins": nbins, "n_particles": cnt["n_total"], "n_processed": cnt["n_proc"],
                        "ps_freq": args.ps_freq, "dt": dt, "lds_tile": TILE_NAMES[tile]})


def adjoint_cost(sim, one_step, k, ps_freq, n_soil, nb):
    """Wall time of k plain forward steps, of recording k steps and of the
    adjoint sweep over them (seeded weights on the end state and on every
    step's body forces), bodies frozen over the k steps as in crm_step."""
    import torch
    while sim.counts()["steps"] % ps_freq:
        one_step()
    rng = np.random.default_rng(0)
    seeds = dict(lam_pos=rng.normal(size=(n_soil, 3)), lam_vel=rng.normal(size=(n_soil, 3)),
                 lam_sigma=rng.normal(size=(n_soil, 6)), lam_rho=rng.normal(size=n_soil),
                 lam_force=rng.normal(size=(k, nb, 3)), lam_torque=rng.normal(size=(k, nb, 3)))

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3, r

    t_fwd, _ = timed(lambda: sim.step(k))
    t_rec, _ = timed(lambda: sim.record(k))
    t_adj, g = timed(lambda: sim.adjoint(**seeds))
    # a second record and sweep of the same length, with the context's buffers
    # already allocated (the steady state of a repeated optimisation loop)
    while sim.counts()["steps"] % ps_freq:
        one_step()
    t_rec2, _ = timed(lambda: sim.record(k))
    t_adj2, _ = timed(lambda: sim.adjoint(**seeds))
    return dict(steps=k, forward_ms=round(t_fwd, 3), record_ms=round(t_rec, 3), adjoint_ms=round(t_adj, 3),
                ratio=round(t_adj / t_fwd, 3), record_ms_again=round(t_rec2, 3), adjoint_ms_again=round(t_adj2, 3),
                ratio_again=round(t_adj2 / t_fwd, 3), dL_dE=float(g["params"][0]), dL_dmu_s=float(g["params"][2]),
                note="wall time of each call, host seeds and outputs included; *_again: second call")


def _oracle_rate(scene, steps):
    from oracle.oracle import Oracle
    orc = Oracle(scene, nbr_mode="cells")
    t0 = time.perf_counter()
    orc.step(steps)
    return scene.n_total * steps / (time.perf_counter() - t0)


def _oracle_rate_one_thread(workload, steps):
    """The oracle on one host thread, in a child process (OpenMP reads the
    thread count when the library starts)."""
    import subprocess
    code = ("import sys, time; sys.path.insert(0, %r)\n"
            "from paper_2507_05643_amd import scenes\n"
            "from oracle.oracle import Oracle\n"
            "sc = scenes.%s\n"
            "o = Oracle(sc, nbr_mode='cells'); t = time.perf_counter(); o.step(%d)\n"
            "print(sc.n_total * %d / (time.perf_counter() - t))\n") % (ROOT, workload, steps, steps)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    return float(r.stdout.strip().splitlines()[-1]) if r.returncode == 0 else None


def cpu_baseline(scenes, ps_freq, steps, runs, subpatch_rate=None):
    """The FP64 oracle (cell-list neighbour search, OpenMP over the host's
    threads) on the wheel bin: the median of `runs` runs of `steps` steps; then
    one thread on one step of the same workload, and the other workloads."""
    from oracle.oracle import Oracle
    sc = scenes.wheel_bin(seed=0, ps_freq=ps_freq)
    t0 = time.perf_counter()
    rates = [_oracle_rate(sc, steps) for _ in range(runs)]
    t_w = time.perf_counter() - t0
    one = _oracle_rate_one_thread(f"wheel_bin(seed=0, ps_freq={ps_freq})", 1)
    other = dict(column_16cubed_100_steps=_oracle_rate(scenes.column(seed=0, n=16, ps_freq=ps_freq), 100),
                 plate_32x32x16_200_steps=_oracle_rate(scenes.plate_patch(seed=0, ps_freq=ps_freq), 200))
    if subpatch_rate is not None:
        other["strip_subpatch_at_9999m_100_steps"] = subpatch_rate
    return dict(value=float(np.median(rates)), unit="particle-steps/s", cores=Oracle.threads(), kind="oracle",
                sample=f"median of {runs} runs of {steps} steps of the same wheel-bin workload ({sc.n_total} "
                       f"particles, all processed), FP64 C oracle with cell-list search, {t_w:.1f} s; one thread: "
                       f"1 step; other workloads: one run each",
                runs=[round(r) for r in rates], single_thread=one,
                other_workloads={k: round(v) for k, v in other.items()})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--ps-freq", type=int, default=10)
    ap.add_argument("--cpu-steps", type=int, default=10,
                    help="oracle steps per run of the CPU baseline (about 3 s on 16 cores)")
    ap.add_argument("--cpu-runs", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="strip0,strip1,batch",
                    help="further forms measured after the wheel bin, comma-separated from strip0 (10 km "
                         "strip, plain FP32 positions), strip1 (cell index + FP32 offset), batch (64 bins); "
                         "'none' for the wheel bin alone")
    ap.add_argument("--wheel-graph", action="store_true",
                    help="replay the wheel bin's per-step kernels as a hipGraph in the timed region")
    ap.add_argument("--trace-steps", type=int, default=20000,
                    help="after the forms, run the wheel bin this many steps from rest and report the drawbar "
                         "pull, vertical force and torque (20000: the 0.5 s single-wheel test)")
    ap.add_argument("--strip-length", type=float, default=10000.0)
    ap.add_argument("--strip-x", type=float, default=5000.0)
    ap.add_argument("--strip-steps", type=int, default=2000)
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--form-warmup", type=int, default=20)
    ap.add_argument("--tile", choices=TILE_NAMES, default="small",
                    help="LDS tile configuration of the soil stages")
    ap.add_argument("--autotune", action="store_true",
                    help="time the soil-stage tile configurations after the warm-up and keep the fastest "
                         "(default: the small tile)")
    ap.add_argument("--adjoint-steps", type=int, default=20,
                    help="after the timed run, cost of the reverse sweep (crm_record + crm_adjoint) "
                         "over this many steps against the plain forward steps (0: skip)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the timed steps, copy a buffer of this many MiB once (a plain copy "
                         "kernel of known size, to calibrate HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the step runs on one GPU",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2507_05643_amd import crm, scenes

    torch.cuda.set_device(0)
    t_start = time.perf_counter()
    w = run_wheel(args, crm, scenes)
    if args.copy_probe_mib > 0:
        src = torch.ones(args.copy_probe_mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    forms = {}
    wanted = [f for f in args.forms.split(",") if f and f != "none"]
    strip_scene = None
    drift = None
    for f in wanted:
        t0 = time.perf_counter()
        if f in ("strip0", "strip1"):
            if strip_scene is None:
                strip_scene = scenes.strip(seed=0, length=args.strip_length, x0=args.strip_x,
                                           ps_freq=args.ps_freq, t_delay=-1.0)
            mode = int(f[-1])
            r = run_strip(args, crm, scenes, mode, strip_scene)
            name = "strip_fp32" if f == "strip0" else "strip_cell_offset"
            # the same form with the paper's activity pass (all N particles
            # tested at every rebuild): the k_activity roofline
            q = run_strip(args, crm, scenes, mode, strip_scene, scan=1)
            r["roofline"] = q["roofline"]
            r["with_activity_scan"] = dict(value=q["value"], ms_per_step=q["ms_per_step"],
                                           activity_launch_ms=q["activity_launch_ms"],
                                           rebuild_ms=q["breakdown"].get("rebuild"))
            # the same form with the vehicle near either end of the strip
            r["along_the_strip"] = {}
            for xv in (10.0, args.strip_length - 10.0):
                q = run_strip(args, crm, scenes, mode, strip_at(strip_scene, xv))
                r["along_the_strip"][f"x={xv:g}"] = dict(value=q["value"], ms_per_step=q["ms_per_step"],
                                                         n_processed=q["config"]["n_processed"],
                                                         activity_launch_ms=q["activity_launch_ms"])
            if drift is None and args.strip_length >= 9999.5:
                drift = subpatch_drift(strip_subpatch(strip_scene, 9999.0), crm)
        elif f == "batch":
            strip_scene = None
            r = run_batch(args, crm, scenes)
            name = "batch_64_bins"
        else:
            raise SystemExit(f"unknown form {f}")
        r["seconds"] = round(time.perf_counter() - t0, 1)
        forms[name] = r
        print(json.dumps(dict(form=name, **{k: v for k, v in r.items() if k != "breakdown"},
                              breakdown=r.get("breakdown"))), file=sys.stderr, flush=True)
    strip_scene = None
    for r in forms.values():
        r["over_wheel_bin"] = round(r["value"] / w["value"], 4)

    trace = run_wheel_trace(args, crm, scenes) if args.trace_steps > 0 else None

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(scenes, args.ps_freq, args.cpu_steps, args.cpu_runs,
                           drift["oracle_particle_steps_per_s"] if drift else None)

    out = {
        "metric": "particle-steps/s",
        "value": w["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": w["wall"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": w["config"],
        "roofline": w["roofline"],
        "cpu_baseline": cpu,
        "soil_particle_steps_per_s": w["soil_rate"],
        "adjoint": w["adjoint"],
        "forms": forms,
        "strip_subpatch_drift": drift,
        "wheel_trace": trace,
        "total_seconds": round(time.perf_counter() - t_start, 1),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
