"""crm_step_noalloc: the step for callers that cannot allocate, through the C
ABI, against crm_step on twin contexts (bit for bit: the same kernels, only
the transient buffers live in the library's static scratch array).

Two calls in a row share the device's scratch array, the second on a smaller
context; a rebuild that needs more memory than the context holds returns
CRM_E_NOMEM and leaves the run as it was.
"""
import numpy as np
import pytest

from paper_2507_05643_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def crm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_05643_amd import crm as C
    return C


def _strip():
    # active domains (flags + compaction) and a list rebuild every other step
    return scenes.strip(seed=1, length=3.0, width=1.2, depth=0.2, dx=0.05, half=0.3, wheelbase=1.2, track=0.6,
                        t_delay=-1.0, ps_freq=2, x0=0.0)


def _moved(sc, dx):
    pos = np.array([b.pos for b in sc.bodies], dtype=np.float64)
    pos[1:, 0] += dx
    nb = len(sc.bodies)
    return (pos, np.tile([1.0, 0.0, 0.0, 0.0], (nb, 1)), np.array([b.linvel for b in sc.bodies]),
            np.array([b.angvel for b in sc.bodies]))


def _same(a, b):
    return all(np.array_equal(a[k], b[k]) for k in ("pos", "vel", "sigma", "rho"))


def _twins(crm, sc):
    a, b = crm.Simulation(sc), crm.Simulation(sc)
    a.step(1)                     # the first step allocates the working set and the lists
    b.step(1)
    return a, b


def test_noalloc_step_equals_step_two_calls(crm):
    big, small = _strip(), scenes.column(seed=3, n=8, ps_freq=3)
    assert small.n_total < big.n_total
    a1, b1 = _twins(crm, big)
    a2, b2 = _twins(crm, small)
    for (a, b, k, name) in ((a1, b1, 7, "strip"), (a2, b2, 5, "column")):
        a.step(k)
        crm.crm_step_noalloc(b.ctx, k)
        sa, sb = a.state(), b.state()
        Fa, Ta = a.forces()
        Fb, Tb = b.forces()
        print(name, "steps", b.counts()["steps"], "rebuilds", b.counts()["rebuilds"], flush=True)
        assert b.counts()["steps"] == k + 1, name
        assert _same(sa, sb), name
        assert np.array_equal(Fa, Fb) and np.array_equal(Ta, Tb), name
        assert np.isfinite(Fb).all(), name
    # the larger context again, after the smaller one used the same array
    a1.step(3)
    crm.crm_step_noalloc(b1.ctx, 3)
    assert _same(a1.state(), b1.state())
    assert np.array_equal(a1.forces()[0], b1.forces()[0])
    for s in (a1, b1, a2, b2):
        s.close()


def test_noalloc_step_needs_no_growth(crm):
    sc = _strip()
    ref, sim = _twins(crm, sc)
    ref.step(1)
    sim.step(1)
    ref.set_bodies(*_moved(sc, 1.5))      # the boxes move over more soil: the working set must grow
    sim.set_bodies(*_moved(sc, 1.5))
    before, c0 = sim.state(), sim.counts()
    with pytest.raises(crm.CrmError) as e:
        crm.crm_step_noalloc(sim.ctx, 1)
    assert e.value.status == -2                                  # CRM_E_NOMEM
    assert _same(before, sim.state())
    assert sim.counts()["steps"] == c0["steps"]
    ref.step(4)
    sim.step(1)                                                  # may allocate: grows
    crm.crm_step_noalloc(sim.ctx, 3)
    assert _same(ref.state(), sim.state())
    assert np.array_equal(ref.forces()[0], sim.forces()[0])
    ref.close()
    sim.close()


def test_noalloc_step_before_the_first_step(crm):
    sim = crm.Simulation(scenes.column(seed=0, n=6))
    with pytest.raises(crm.CrmError) as e:
        crm.crm_step_noalloc(sim.ctx, 1)
    assert e.value.status == -2
    assert sim.counts()["steps"] == 0
    sim.step(1)
    crm.crm_step_noalloc(sim.ctx, 2)
    assert sim.counts()["steps"] == 3
    sim.close()
