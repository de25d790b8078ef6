"""Reverse mode (crm_record + crm_adjoint) against the FP64 autograd replay of
the oracle run (``oracle/adjoint.py``), through the C ABI.

The functional is L = w . y_K + sum_k (wF . F_k + wT . T_k) with seeded random
weights; the library returns dL/dy_0 and dL/d(E, nu, mu_s, mu_2, cohesion).
Tolerance: the adjoint runs in FP32 around the FP32 trajectory, the oracle in
FP64 around its own, so each field's gradient agrees normwise (max error over
max magnitude) to the 1e-3 bar of the forward fields after many steps; on
smooth settings (bilateral viscosity, no yield) the agreement is far tighter,
and the bar there is 1e-4.
"""
import dataclasses

import numpy as np
import pytest

from oracle import adjoint as A
from oracle.oracle import Oracle
from paper_2507_05643_amd import scenes
from tests.parity_util import normwise

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def crm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_05643_amd import crm as C
    return C


def _warm(sc, steps):
    """The scene after `steps` oracle steps (non-zero velocity and stress)."""
    o = Oracle(sc, nbr_mode="cells")
    o.step(steps)
    st = o.state()
    ns = sc.n_soil
    return dataclasses.replace(sc, pos=st["pos"][:ns].copy(), vel=st["vel"][:ns].copy(),
                               sigma=st["sigma"][:ns].copy(), rho=st["rho"][:ns].copy())


def _run(crm, sc, K, seed=5, materials=None):
    ns, nb = sc.n_soil, len(sc.bodies)
    w = A.loss_weights(seed, ns, K, nb)
    rec = A.Recording(sc, K, materials=materials)
    ref = A.gradient(rec, w, materials=materials)
    sim = crm.Simulation(sc)
    if materials is not None:
        sim.set_materials(*materials)
    sim.record(K)
    got = sim.adjoint(lam_pos=w["x"], lam_vel=w["u"], lam_sigma=w["s"], lam_rho=w["rho"],
                      lam_force=w["F"] if nb else None, lam_torque=w["T"] if nb else None)
    rep = dict(x=normwise(got["pos"], ref["x"]), u=normwise(got["vel"], ref["u"]),
               s=normwise(got["sigma"], ref["s"]), rho=normwise(got["rho"], ref["rho"]))
    pref = np.concatenate([[ref["E"], ref["nu"]], ref["mat"].reshape(-1)])
    rep["params"] = float(np.max(np.abs(got["params"] - pref) / np.maximum(np.abs(pref), 1e-300)))
    return sim, got, ref, rep


@pytest.mark.parametrize("smooth", [True, False])
def test_adjoint_matches_autograd_column(crm, smooth):
    sc = scenes.column(seed=0, n=8, ps_freq=2)
    if smooth:
        p = dict(sc.params, av_mode=1, mu_s=100.0, mu_2=100.0, cohesion=1.0e3)
        sc = dataclasses.replace(sc, params=p)
    sc = _warm(sc, 30)
    sim, got, ref, rep = _run(crm, sc, 4)
    say("column adjoint vs oracle", "smooth" if smooth else "plastic", rep)
    tol = 1e-4 if smooth else 1e-3
    for k in ("x", "u", "s", "rho"):
        assert rep[k] <= tol, (k, rep[k])
    assert rep["params"] <= 10 * tol, rep["params"]
    sim.close()


def test_adjoint_matches_autograd_moving_plate(crm):
    """A plate moving into the soil: body-force seeds on every step, two list
    rebuilds inside the record."""
    sc = scenes.plate_patch(seed=0, nx=16, ny=16, nz=8, ps_freq=3)
    sc = _warm(sc, 20)
    sim, got, ref, rep = _run(crm, sc, 6, seed=7)
    say("plate adjoint vs oracle", rep)
    for k in ("x", "u", "s", "rho"):
        assert rep[k] <= 1e-3, (k, rep[k])
    assert rep["params"] <= 1e-2, rep["params"]
    sim.close()


def test_adjoint_cell_offset_positions(crm):
    sc = scenes.column(seed=1, n=8, ps_freq=2, pos_mode=1)
    sc = _warm(sc, 30)
    sim, got, ref, rep = _run(crm, sc, 4, seed=9)
    say("cell-offset adjoint vs oracle", rep)
    for k in ("x", "u", "s", "rho"):
        assert rep[k] <= 1e-3, (k, rep[k])
    assert rep["params"] <= 1e-2, rep["params"]
    sim.close()


def test_adjoint_two_materials(crm):
    sc = _warm(scenes.column(seed=2, n=8, ps_freq=2), 30)
    ns = sc.n_soil
    mat = (np.arange(ns) % 2).astype(np.uint16)
    table = np.array([[0.7, 0.7, 0.0], [0.4, 0.9, 20.0]])
    sim, got, ref, rep = _run(crm, sc, 4, seed=11, materials=(table, mat))
    say("two-material adjoint vs oracle", rep, got["params"])
    for k in ("x", "u", "s", "rho"):
        assert rep[k] <= 1e-3, (k, rep[k])
    # friction and cohesion of both materials (what a calibration needs)
    assert rep["params"] <= 1e-2, rep["params"]
    sim.close()


def test_adjoint_leaves_the_run_unchanged(crm):
    """After the sweep the context holds the recorded end state, bit for bit,
    and later steps equal those of a context that never ran it."""
    sc = _warm(scenes.column(seed=3, n=8, ps_freq=3), 10)
    a, b = crm.Simulation(sc), crm.Simulation(sc)
    a.record(7)
    b.step(7)
    s0 = a.state()
    w = A.loss_weights(1, sc.n_soil, 7, len(sc.bodies))
    a.adjoint(lam_pos=w["x"], lam_force=w["F"], lam_torque=w["T"])
    s1 = a.state()
    for k in ("pos", "vel", "sigma", "rho"):
        assert np.array_equal(s0[k], s1[k]), k
    a.step(5)
    b.step(5)
    sa, sb = a.state(), b.state()
    for k in ("pos", "vel", "sigma", "rho"):
        assert np.array_equal(sa[k][:sc.n_soil], sb[k][:sc.n_soil]), k
    a.close()
    b.close()


def test_adjoint_error_paths(crm):
    sc = scenes.column(seed=0, n=6, ps_freq=4)
    sim = crm.Simulation(sc)
    with pytest.raises(crm.CrmError):
        sim.adjoint()                       # nothing recorded
    sim.step(1)
    with pytest.raises(crm.CrmError):
        sim.record(2)                       # not at a list rebuild
    sim.step(3)
    sim.record(2)
    sim.step(1)
    with pytest.raises(crm.CrmError):
        sim.adjoint()                       # stepped since the record
    sim.close()
    p = dict(sc.params, active_domains=1)
    s2 = crm.Simulation(sc, params=p)
    with pytest.raises(crm.CrmError):
        s2.record(1)
    s2.close()


def test_adjoint_wendland_kernel(crm):
    sc = scenes.column(seed=4, n=8, ps_freq=2)
    sc.params["kernel"] = 1
    sc = _warm(sc, 30)
    sim, got, ref, rep = _run(crm, sc, 4, seed=13)
    say("wendland adjoint vs oracle", rep)
    for k in ("x", "u", "s", "rho"):
        assert rep[k] <= 1e-3, (k, rep[k])
    assert rep["params"] <= 1e-2, rep["params"]
    sim.close()
