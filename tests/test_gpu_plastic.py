"""Forward parity where every case of the return mapping fires (Sec. 2.4):
friction mu_s 0.7 rising to mu_2 0.8 with the inertial number (I0 0.08, grain
size 3 mm, the cone-penetration rheology of Sec. 3.2) and cohesion 500 Pa.

Two workloads: a grousered wheel pressed 12 mm into a small soil bin, and a
cohesive cluster pulled apart by a diverging velocity field. The oracle
reports, per particle and step, the branch of its return mapping (tension
cut-off, admissible, radial return) and the mu(I) case of the radial returns
(mu_s: no shear-rate increase; mu_2: tensile trial pressure; the interior
formula); over the two workloads each is taken at least 100 times. Both sides start
from the same FP32 state, warmed by oracle steps so that plastic flow is
under way in the first compared step.
"""
import dataclasses

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2507_05643_amd import scenes
from tests.parity_util import check_fields, normwise

pytestmark = pytest.mark.gpu

RHEOLOGY = dict(mu_s=0.7, mu_2=0.8, I0=0.08, grain_d=3.0e-3, cohesion=500.0)


@pytest.fixture(scope="module")
def crm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_05643_amd import crm as C
    return C


def _wheel():
    sc = scenes.wheel_bin(seed=3, nx=60, ny=36, nz=12, ps_freq=10)
    wb = sc.bodies[1]
    wb.pos = (wb.pos[0], wb.pos[1], wb.pos[2] - 0.012)
    sc.params.update(RHEOLOGY)
    return sc


def _cluster():
    sc = scenes.cluster(seed=3, n=10, vel_scale=0.0, sigma_scale=0.0)
    x = sc.pos.astype(np.float64)
    sc.vel = (3.0 * (x - x.mean(axis=0))).astype(np.float32)
    rng = np.random.default_rng(0)
    sig = np.zeros((sc.n_soil, 6))
    sig[:, :3] = -200.0 + rng.normal(0.0, 300.0, size=(sc.n_soil, 3))
    sig[:, 3:] = rng.normal(0.0, 200.0, size=(sc.n_soil, 3))
    sc.sigma = sig.astype(np.float32)
    sc.params.update(RHEOLOGY, ps_freq=5)
    return sc


def _warm(sc, steps):
    """The scene after `steps` oracle steps, rounded to the FP32 state both
    sides start from."""
    o = Oracle(sc, nbr_mode="cells")
    o.step(steps)
    st = o.state()
    ns = sc.n_soil
    return dataclasses.replace(sc, pos=st["pos"][:ns].astype(np.float32), vel=st["vel"][:ns].astype(np.float32),
                               sigma=st["sigma"][:ns].astype(np.float32), rho=st["rho"][:ns].astype(np.float32))


def _tally(orc, acc):
    br, mc = orc.branches()
    acc["cut_off"] += int((br == 1).sum())
    acc["admissible"] += int((br == 3).sum())
    acc["radial"] += int((br == 4).sum())
    acc["radial_mu_s"] += int(((br == 4) & (mc == 0)).sum())
    acc["radial_mu_2"] += int(((br == 4) & (mc == 1)).sum())
    acc["radial_mu_I"] += int(((br == 4) & (mc == 2)).sum())


# The pressed wheel takes every case (the interior mu(I) formula where the
# shear rate rises under compression); the pull-apart cluster is there for the
# tensile cases (cut-off, and radial returns at mu_2 under a tensile trial
# pressure). Measured over 30 steps: wheel every case >= 100; cluster cut-off
# 5341, admissible 17834, radial 6825 (mu_s 1345, mu_2 5473, interior 7).
REQUIRED = {"wheel": ("cut_off", "admissible", "radial", "radial_mu_s", "radial_mu_2", "radial_mu_I"),
            "cluster": ("cut_off", "admissible", "radial", "radial_mu_s", "radial_mu_2")}


@pytest.mark.parametrize("name,warm,steps", [("wheel", 20, 30), ("cluster", 3, 30)])
def test_return_mapping_branches_parity(crm, name, warm, steps):
    sc = _warm(_wheel() if name == "wheel" else _cluster(), warm)
    sim = crm.Simulation(sc)
    orc = Oracle(sc, nbr_mode="cells")
    acc = dict(cut_off=0, admissible=0, radial=0, radial_mu_s=0, radial_mu_2=0, radial_mu_I=0)
    sim.step(1)
    orc.step(1)
    _tally(orc, acc)
    print(name, "branches of the first step", acc, flush=True)
    assert acc["radial"] >= 100
    check_fields(sim.state(), orc.state(), sc, 1, 1e-5, f"plastic {name}")
    for _ in range(steps - 1):
        sim.step(1)
        orc.step(1)
        _tally(orc, acc)
    print(name, "branches over", steps, "steps", acc, flush=True)
    for k in REQUIRED[name]:
        assert acc[k] >= 100, (k, acc[k])
    check_fields(sim.state(), orc.state(), sc, steps, 1e-3, f"plastic {name}")
    if sc.bodies:
        F, T = sim.forces()
        Fr, Tr = orc.forces()
        print("forces", F[1], Fr[1], flush=True)
        assert normwise(F[1], Fr[1]) <= 1e-3
    sim.close()


def test_whole_cell_translation_is_bit_identical(crm):
    """A scene and its grid translated by whole cells (to ~10 km along x, every
    coordinate an exact binary fraction): with cell-index + FP32-offset
    positions the run is bit-identical (positions up to the shift); plain FP32
    positions lose the motion there."""
    H = 2.0 ** -7
    S = 2.0 * H

    def scene(shift_cells, pos_mode, move_grid=True):
        sh = np.array([shift_cells * S, 0.0, 0.0])
        sc = scenes.column(seed=3, n=10, dx=H / 1.2)
        lo, hi = np.full(3, -3 * S), np.full(3, 10 * S) + sh
        if move_grid:
            lo = lo + sh
        sc.params.update(h=H, pos_mode=pos_mode, domain_lo=tuple(lo), domain_hi=tuple(hi))
        sc.pos = sc.pos.astype(np.float64) + sh
        b = sc.bodies[0]
        b.pos = tuple(np.asarray(b.pos, dtype=np.float64) + sh)
        return sc, sh

    runs = {}
    for shift, move, modes in ((0, True, (0, 1)), (640000, True, (0, 1)), (64000, False, (1,))):
        for mode in modes:
            sc, sh = scene(shift, mode, move)
            sim = crm.Simulation(sc)
            sim.step(40)
            st = sim.state()
            st["pos"] = st["pos"] - sh
            runs[(shift, mode)] = (st, sim.forces())
            if not move:
                print("grid cells", sim.counts()["cells"], flush=True)
            sim.close()
    near = runs[(0, 1)]
    for key in ((640000, 1), (64000, 1)):      # grid moved along; grid fixed, cells 64,000 apart
        far = runs[key]
        for k in ("pos", "vel", "sigma", "rho"):
            assert np.array_equal(near[0][k], far[0][k]), (key, k)
        assert np.array_equal(near[1][0], far[1][0]) and np.array_equal(near[1][1], far[1][1]), key
    # plain FP32 positions at 10 km: the spacing there (~1 mm) swallows the motion
    assert not np.array_equal(runs[(0, 0)][0]["pos"], runs[(640000, 0)][0]["pos"])
