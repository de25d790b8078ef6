"""Writes tests/golden/plate_fd.json: central finite differences of the FP64
oracle for the plate-pressing calibration workload (32 x 32 x 16 soil at
dx = 1 cm, 0.1 x 0.1 m plate moving down at 0.05 m/s, 200 steps), the
reference gradients of the reverse-mode test (Sec. 2.3-2.5 differentiated).

Functional: L = mean over the 200 steps of the plate's vertical force F_z
(Sec. 2.5.1 body force). Parameters: E, nu, mu_s, mu_2 and the initial soil
velocities along one seeded direction about the workload's soil (E = 1 MPa,
nu = 0.3, mu_s = mu_2 = 0.7, no cohesion); the cohesion derivative about
100 Pa (at zero cohesion a central difference would leave the admissible
range). With cohesion the tension cut-off makes the stress jump (from
(c / mu_s) I to zero), and velocity perturbations push particles across it:
the velocity derivative is therefore taken without cohesion, where the
cut-off is continuous. The differentiated run starts from the
state after 20 oracle steps of the workload from rest (rounded to FP32, the
GPU's input). At rest itself the step is not differentiable in the initial
velocities: every pair has v_ij . r_ij = 0, the switch of the unilateral
artificial viscosity, and every stress is isotropic, where the equivalent
shear stress (a norm) has no derivative. Random initial velocities do not
help either: at 1e-6 m/s the pairs sit at the switch for many steps, at
1e-2 m/s many particles cross the cohesive tension cut-off, where the stress
jumps.

Each parameter derivative is taken with two relative steps (1e-6 and 1e-5);
where they disagree beyond 1e-4 a return-mapping or viscosity branch flipped
inside the difference and the entry is marked unusable. The velocity
derivative takes steps 1e-6, 1e-5 and 1e-4 along the 0.01 m/s direction and
is usable when the estimates converge (see below). Calls only the oracle and the
seeded scene generator:

    python tests/golden/make_plate_fd.py
"""
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.oracle import Oracle  # noqa: E402
from paper_2507_05643_amd import scenes  # noqa: E402

STEPS = 200
PS_FREQ = 20
WARM = 20
BASE = dict(E=1.0e6, nu=0.3, mu_s=0.7, mu_2=0.7, cohesion=0.0)
COHESION_BASE = 100.0
VEL_SCALE = 0.01       # m/s: the direction of the initial-velocity derivative
VEL_SEED = 11
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "plate_fd.json")


def scene():
    """The workload after WARM oracle steps from rest (soil state rounded to
    FP32; the plate keeps its initial pose: bodies are set by the caller)."""
    sc = scenes.plate_patch(seed=0, nx=32, ny=32, nz=16, ps_freq=PS_FREQ)
    p = dict(sc.params)
    p.update(BASE)
    o = Oracle(sc, nbr_mode="cells", params=p)
    o.step(WARM)
    st = o.state()
    n = sc.n_soil
    f32 = lambda a: np.asarray(a[:n], dtype=np.float32)
    return dataclasses.replace(sc, pos=f32(st["pos"]), vel=f32(st["vel"]), sigma=f32(st["sigma"]),
                               rho=f32(st["rho"]))


def functional(sc, theta, vel0):
    p = dict(sc.params)
    p.update(theta)
    o = Oracle(sc, nbr_mode="cells", params=p)
    o.set_state(vel=vel0)
    fz = 0.0
    for _ in range(STEPS):
        o.step(1)
        F, _ = o.forces()
        fz += F[1, 2]
    return fz / STEPS


def direction(n):
    return np.random.default_rng(VEL_SEED).normal(0.0, VEL_SCALE, size=(n, 3))


def main():
    sc = scene()
    t0 = time.time()
    n = sc.n_soil
    vb = np.asarray(sc.vel, dtype=np.float64)
    L0 = functional(sc, BASE, vb)
    res = dict(steps=STEPS, ps_freq=PS_FREQ, warm=WARM, base=BASE, functional="mean_k F_z(plate)", L0=L0,
               vel_seed=VEL_SEED, vel_scale=VEL_SCALE, n_soil=int(n), grads={})
    res["cohesion_base"] = COHESION_BASE
    res["L0_cohesion_base"] = functional(sc, dict(BASE, cohesion=COHESION_BASE), vb)
    for k in BASE:
        base = dict(BASE, cohesion=COHESION_BASE) if k == "cohesion" else BASE
        v = base[k]
        est = []
        for rel in (1e-6, 1e-5):
            hstep = rel * abs(v)
            lp = functional(sc, dict(base, **{k: v + hstep}), vb)
            lm = functional(sc, dict(base, **{k: v - hstep}), vb)
            est.append((lp - lm) / (2.0 * hstep))
        agree = abs(est[0] - est[1]) <= 1e-4 * max(abs(est[0]), abs(est[1]), 1e-300)
        res["grads"][k] = dict(fd=est[0], fd_coarse=est[1], usable=bool(agree))
        print(k, est, "usable" if agree else "branch flip", f"{time.time() - t0:.0f}s", flush=True)
    d = direction(n)
    est = []
    for eps in (1e-6, 1e-5, 1e-4):
        lp = functional(sc, BASE, vb + eps * d)
        lm = functional(sc, BASE, vb - eps * d)
        est.append((lp - lm) / (2.0 * eps))
    # kinks (the unilateral viscosity's switch, the yield surface) leave an
    # error linear in the step: the estimates converge, the two finest agree
    # to 2e-3 and closer than the two coarsest; a jump would make them diverge
    e01, e12 = abs(est[0] - est[1]), abs(est[1] - est[2])
    agree = e01 <= 2e-3 * abs(est[0]) and e01 < e12
    res["grads"]["vel0_dir"] = dict(fd=est[0], fd_coarse=est[1], fd_coarsest=est[2], usable=bool(agree))
    print("vel0_dir", est, "usable" if agree else "branch flip", flush=True)
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1)
    print("wrote", OUT, f"{time.time() - t0:.0f}s")


if __name__ == "__main__":
    main()
