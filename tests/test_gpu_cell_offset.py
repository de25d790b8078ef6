"""Cell-index + FP32-offset positions (pos_mode 1) against the FP64 oracle.

Far from the coordinate origin (a column placed at x = 9,999 m, where the FP32
spacing is 0.98 mm, larger than the motion of a step) the cell-offset form
keeps the motion: displacements, velocities, stresses and densities match the
oracle to the same bars as the plain form near the origin, while the plain
FP32 form loses the displacements there. Integer decisions (cells, neighbour
lists) are bit-exact, taken on the stored representation on both sides.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from oracle.oracle import Oracle
from paper_2507_05643_amd import scenes
from tests.parity_util import check_cell_sort, check_fields, csr_rows, normwise, world_positions

pytestmark = pytest.mark.gpu
FAR = (9999.0, 0.0, 0.0)


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def crm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_05643_amd import crm as C
    return C


@pytest.mark.parametrize("origin", [None, FAR])
def test_cell_offset_lists_bit_exact(crm, origin):
    sc = scenes.column(seed=2, origin=origin, pos_mode=1)
    sim = crm.Simulation(sc)
    sim.step(1)
    ex = sim.export()
    x = world_positions(sc)
    sid, skey, cs, ce = O.sort_cells(sc.params, x)
    check_cell_sort(ex["sorted_ids"], sid, cs, ce, x)
    assert np.array_equal(ex["cell_start"][:-1].astype(np.int64), cs)
    off, nbr = O.neighbors(sc.params, x, mode="cells")
    ref = csr_rows(off, nbr)
    got = csr_rows(ex["off"], ex["nbr"], ex["rows"])
    for i in range(sc.n_total):
        want = ref[i] if i < sc.n_soil else ref[i][ref[i] < sc.n_soil]
        assert np.array_equal(got[i], want), i
    sim.close()


@pytest.mark.parametrize("steps,tol", [(1, 1e-5), (100, 1e-3)])
def test_cell_offset_parity_far_from_origin(crm, steps, tol):
    sc = scenes.column(seed=0, origin=FAR, pos_mode=1)
    sim = crm.Simulation(sc)
    orc = Oracle(sc, nbr_mode="cells")
    sim.step(steps)
    orc.step(steps)
    check_fields(sim.state(), orc.state(), sc, steps, tol, "cell-offset at 9999 m")
    F, _ = sim.forces()
    Fr, _ = orc.forces()
    assert normwise(F, Fr) <= tol
    sim.close()


@pytest.mark.parametrize("steps", [50, 100])
def test_both_forms_near_origin_against_oracle(crm, steps):
    """Near the origin both forms resolve the motion. Plain FP32 positions round
    every step's update at the coordinates' magnitude (half an ulp at 0.15 m is
    7.5e-9 m against ~1e-7 m of motion per step); the cell-offset form rounds
    it at the magnitude of the offset inside a cell (half an ulp at 0.024 m is
    0.9e-9 m), so its displacements hold a bar eight times tighter."""
    errs = {}
    for mode in (0, 1):
        sc = scenes.column(seed=1, pos_mode=mode)
        sim = crm.Simulation(sc)
        orc = Oracle(sc, nbr_mode="cells")
        sim.step(steps)
        orc.step(steps)
        rep = check_fields(sim.state(), orc.state(), sc, steps, 1e-3, f"near origin, pos_mode {mode}")
        errs[mode] = rep["disp"]
        sim.close()
    say("displacement error: plain", errs[0], "cell-offset", errs[1])
    assert errs[1] <= errs[0]


def test_plain_fp32_loses_motion_far_from_origin(crm):
    """The reason for the cell-offset form: at 9,999 m the FP32 spacing (0.98 mm)
    exceeds the per-step motion, so plain FP32 positions stop moving, while the
    cell-offset form tracks the oracle's displacements."""
    errs = {}
    for mode in (0, 1):
        sc = scenes.column(seed=0, origin=FAR, pos_mode=mode)
        x0 = world_positions(sc)
        sim = crm.Simulation(sc)
        orc = Oracle(sc, nbr_mode="cells")
        sim.step(40)
        orc.step(40)
        g, r = sim.state(), orc.state()
        n = sc.n_soil
        disp_ref = r["pos"][:n] - x0[:n]
        assert np.abs(disp_ref[:, 2]).max() > 1e-7
        errs[mode] = normwise(g["pos"][:n] - x0[:n], disp_ref)
        sim.close()
    say("displacement error after 40 steps at 9999 m: plain", errs[0], "cell-offset", errs[1])
    assert errs[0] > 0.5
    assert errs[1] < 1e-2


@pytest.mark.parametrize("pos_mode", [0, 1])
def test_lists_with_particles_outside_the_grid(crm, pos_mode):
    """Particles (soil and markers) below the grid's lower corner along x and y
    share its edge cells with particles of other stored cells; inside such a
    cell the slots are still in x order, and the lists equal the brute-force
    definition |x_i - x_j| < 2h."""
    sc = scenes.column(seed=4, n=10, pos_mode=pos_mode)
    sc.params.update(domain_lo=(0.045, 0.045, -0.04))
    x = world_positions(sc)
    assert (x[:, 0] < 0.045).sum() > 300
    sim = crm.Simulation(sc)
    sim.step(1)
    ex = sim.export()
    sid, skey, cs, ce = O.sort_cells(sc.params, x)
    check_cell_sort(ex["sorted_ids"], sid, cs, ce, x)
    off, nbr = O.neighbors(sc.params, x, mode="brute")
    ref = csr_rows(off, nbr)
    got = csr_rows(ex["off"], ex["nbr"], ex["rows"])
    for i in range(sc.n_total):
        want = ref[i] if i < sc.n_soil else ref[i][ref[i] < sc.n_soil]
        assert np.array_equal(got[i], want), i
    sim.close()
