"""Batched soil bins: many independent bins in one context.

A bin inside the batch is bit-identical (state and body forces) to the same bin
run alone with the same grid, since its neighbour lists, their order and its
bodies' marker ranges are the same (on an 8-bin batch, and on the full 64-bin
batch under graph replay); a small batch with per-bin friction matches the
FP64 oracle with per-particle materials.
"""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2507_05643_amd import scenes
from tests.parity_util import check_fields, normwise

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def crm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_05643_amd import crm as C
    return C


def _sim(crm, sc):
    sim = crm.Simulation(sc)
    sim.set_materials(sc.meta["materials"], sc.meta["material"])
    return sim


def _bin_slices(sc):
    """Soil and marker id ranges of each kept bin (bins in order, two bodies each)."""
    out, s0, m0 = [], 0, sc.n_soil
    for k, b in enumerate(sc.meta["bins"]):
        nm = sc.bodies[2 * k].markers.shape[0] + sc.bodies[2 * k + 1].markers.shape[0]
        out.append((slice(s0, s0 + b["n"]), slice(m0, m0 + nm)))
        s0 += b["n"]
        m0 += nm
    return out


def test_bin_in_batch_equals_bin_alone(crm):
    kw = dict(seed=3, n_bins=8, n_min=4.0e3, n_max=2.0e4, ps_freq=5)
    full = scenes.batch_bins(**kw)
    sim = _sim(crm, full)
    sim.step(12)
    gf = sim.state()
    Ff, Tf = sim.forces()
    sl_full = _bin_slices(full)
    sim.close()
    for b in (2, 5):
        alone = scenes.batch_bins(only=[b], **kw)
        s1 = _sim(crm, alone)
        s1.step(12)
        g1 = s1.state()
        F1, T1 = s1.forces()
        (ss, ms), = _bin_slices(alone)
        fs, fm = sl_full[b]
        for k in ("pos", "vel", "sigma", "rho"):
            assert np.array_equal(g1[k][ss], gf[k][fs]), (b, k)
            assert np.array_equal(g1[k][ms], gf[k][fm]), (b, k, "markers")
        assert np.array_equal(F1, Ff[2 * b:2 * b + 2]) and np.array_equal(T1, Tf[2 * b:2 * b + 2])
        s1.close()


def test_full_batch_bins_equal_bins_alone(crm):
    """The 64-bin batch at full size (seed 0: 6,923,164 particles, the bench's
    workload), stepped as a graph replay over two list rebuilds: its smallest
    and largest bins are bit-identical to the same bins alone."""
    kw = dict(seed=0, ps_freq=10)
    full = scenes.batch_bins(**kw)
    assert full.n_total == 6923164
    sizes = [b["n"] for b in full.meta["bins"]]
    pick = (int(np.argmin(sizes)), int(np.argmax(sizes)))
    sim = _sim(crm, full)
    sim.graph(True)
    sim.step(25)
    gf = sim.state()
    Ff, Tf = sim.forces()
    sl_full = _bin_slices(full)
    sim.close()
    for b in pick:
        alone = scenes.batch_bins(only=[b], **kw)
        s1 = _sim(crm, alone)
        s1.graph(True)
        s1.step(25)
        g1 = s1.state()
        F1, T1 = s1.forces()
        (ss, ms), = _bin_slices(alone)
        fs, fm = sl_full[b]
        print("bin", b, "soil", sizes[b], flush=True)
        for k in ("pos", "vel", "sigma", "rho"):
            assert np.array_equal(g1[k][ss], gf[k][fs]), (b, k)
            assert np.array_equal(g1[k][ms], gf[k][fm]), (b, k, "markers")
        assert np.array_equal(F1, Ff[2 * b:2 * b + 2]) and np.array_equal(T1, Tf[2 * b:2 * b + 2])
        s1.close()


def test_small_batch_matches_oracle_with_materials(crm):
    sc = scenes.batch_bins(seed=1, n_bins=4, n_min=3.0e3, n_max=6.0e3, ps_freq=5)
    # put the wheels into the soil so that friction matters
    for k in range(len(sc.meta["bins"])):
        w = sc.bodies[2 * k + 1]
        w.pos = (w.pos[0], w.pos[1], w.pos[2] - 0.015)
    sim = _sim(crm, sc)
    orc = Oracle(sc, nbr_mode="cells")
    orc.set_materials(sc.meta["materials"], sc.meta["material"])
    sim.step(20)
    orc.step(20)
    check_fields(sim.state(), orc.state(), sc, 20, 1e-3, "batch vs oracle")
    F, _ = sim.forces()
    Fr, _ = orc.forces()
    assert normwise(F, Fr) <= 1e-3
    sim.close()
