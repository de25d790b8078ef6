"""Failure handling and restart through the C ABI, all forced from the host (no
kernel is made to fail):

* an allocation that fails while the working set or the neighbour lists grow
  returns CRM_E_NOMEM and leaves the context as it was: the state reads back
  bit-identically and, once memory is available again, the run continues bit
  for bit as one where the allocation never failed;
* a non-finite stress set through crm_set_state surfaces as CRM_E_NONFINITE at
  the next force read, and poisons the context;
* a checkpoint taken at a list rebuild (crm_save_checkpoint) restores into a
  new context that continues bit-identically (FP32 and cell-offset positions,
  active domains, per-particle materials); so does the soil state read with
  crm_get_state and written with crm_set_state at a list rebuild (FP32
  positions).
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


class FailingAllocator:
    """torch's caching allocator, made to refuse allocations on demand: after
    `grant` more allocations every further one fails (grant None: never)."""

    def __init__(self, crm, device=0):
        self.inner = crm._TorchAllocator(device)
        self.grant = None
        self.calls = 0

        def _alloc(nbytes, user, stream):
            self.calls += 1
            if self.grant is not None:
                if self.grant <= 0:
                    return None
                self.grant -= 1
            return self.inner.alloc(nbytes, user, stream)

        def _free(ptr, user, stream):
            self.inner.free(ptr, user, stream)

        self.alloc = crm.ALLOC_FN(_alloc)
        self.free = crm.FREE_FN(_free)


def _strip():
    return scenes.strip(seed=1, length=3.0, width=1.2, depth=0.2, dx=0.05, half=0.3, wheelbase=1.2, track=0.6,
                        t_delay=-1.0, ps_freq=2, x0=0.0)


def _bodies(sc, dx):
    pos = np.array([b.pos for b in sc.bodies], dtype=np.float64)
    pos[1:, 0] += dx
    nb = len(sc.bodies)
    return (pos, np.tile([1.0, 0.0, 0.0, 0.0], (nb, 1)), np.array([b.linvel for b in sc.bodies]),
            np.array([b.angvel for b in sc.bodies]))


def _same(a, b):
    return all(np.array_equal(a[k], b[k]) for k in ("pos", "vel", "sigma", "rho"))


def test_failed_growth_leaves_the_context_unchanged(crm):
    sc = _strip()
    # how many allocations the growth step makes (a counting allocator)
    probe_alloc = FailingAllocator(crm)
    probe = crm.Simulation(sc, allocator=probe_alloc)
    probe.step(2)
    probe.set_bodies(*_bodies(sc, 1.5))       # the boxes move over the soil: more particles
    cap0 = probe.counts()["capacity"]
    n0 = probe_alloc.calls
    probe.step(1)
    grown = probe.counts()["capacity"]
    n_growth = probe_alloc.calls - n0
    probe.close()
    print("capacity", cap0, "->", grown, "allocations in the growth step", n_growth, flush=True)
    assert grown > cap0 and n_growth >= 20
    ref = crm.Simulation(sc)
    ref.step(2)
    ref.set_bodies(*_bodies(sc, 1.5))
    ref.step(4)
    want, Fw = ref.state(), ref.forces()
    ref.close()
    for grant in (0, n_growth // 2, n_growth - 1):
        fa = FailingAllocator(crm)
        sim = crm.Simulation(sc, allocator=fa)
        sim.step(2)
        sim.set_bodies(*_bodies(sc, 1.5))
        before, c0 = sim.state(), sim.counts()
        fa.grant = grant
        with pytest.raises(crm.CrmError) as e:
            sim.step(1)
        assert e.value.status == -2, e.value            # CRM_E_NOMEM
        after, c1 = sim.state(), sim.counts()
        assert _same(before, after), grant
        assert c1["steps"] == c0["steps"]
        fa.grant = None
        sim.step(4)
        got, Fg = sim.state(), sim.forces()
        assert _same(got, want), grant
        assert np.array_equal(Fg[0], Fw[0]) and np.array_equal(Fg[1], Fw[1]), grant
        sim.close()


def test_nonfinite_state_surfaces_at_the_force_read(crm):
    sc = scenes.column(seed=1, n=6)
    sim = crm.Simulation(sc)
    sim.step(1)
    sig = np.zeros((sc.n_soil, 6), dtype=np.float32)
    sig[:, 2] = np.nan
    sim.set_state(sigma=sig)
    sim.step(1)
    with pytest.raises(crm.CrmError) as e:
        sim.forces()
    assert e.value.status == -5                          # CRM_E_NONFINITE
    with pytest.raises(crm.CrmError) as e:
        sim.step(1)
    assert e.value.status == -4                          # poisoned: CRM_E_STATE
    sim.close()


def _checkpoint_cases():
    a = scenes.plate_patch(seed=2, nx=16, ny=16, nz=8, ps_freq=4)
    b = scenes.column(seed=0, n=10, origin=(9999.0, 0.0, 0.0), pos_mode=1, ps_freq=3)
    c = _strip()
    return [("plate", a, 8), ("cell-offset at 9999 m", b, 6), ("active domains", c, 4)]


@pytest.mark.parametrize("case", [0, 1, 2])
def test_checkpoint_restart_is_bit_identical(crm, case):
    name, sc, at = _checkpoint_cases()[case]
    mats = None
    if case == 0:
        mats = (np.array([[0.7, 0.7, 0.0], [0.5, 0.8, 200.0]]), (np.arange(sc.n_soil) % 2).astype(np.uint16))
    a = crm.Simulation(sc)
    if mats:
        a.set_materials(*mats)
    a.step(at)
    blob = a.save_checkpoint()
    a.step(7)
    want, Fw = a.state(), a.forces()
    b = crm.Simulation(sc)                               # materials come with the checkpoint
    b.load_checkpoint(blob)
    assert b.counts()["steps"] == at
    b.step(7)
    got, Fg = b.state(), b.forces()
    print(name, "checkpoint bytes", len(blob), flush=True)
    assert _same(got, want), name
    assert np.array_equal(Fg[0], Fw[0]) and np.array_equal(Fg[1], Fw[1]), name
    a.close()
    b.close()


def test_checkpoint_errors(crm):
    sc = scenes.plate_patch(seed=2, nx=16, ny=16, nz=8, ps_freq=4)
    a = crm.Simulation(sc)
    a.step(4)
    blob = a.save_checkpoint()
    a.step(1)
    with pytest.raises(crm.CrmError) as e:
        a.save_checkpoint()                              # inside a list segment
    assert e.value.status == -4
    other = crm.Simulation(scenes.plate_patch(seed=2, nx=12, ny=16, nz=8, ps_freq=4))
    st0 = other.state()
    with pytest.raises(crm.CrmError) as e:
        other.load_checkpoint(blob)                      # another particle count
    assert e.value.status == -1
    assert _same(other.state(), st0)
    with pytest.raises(crm.CrmError) as e:
        other.load_checkpoint(b"not a checkpoint at all, really not" * 4)
    assert e.value.status == -1
    bad = bytearray(blob)
    bad[-1:] = b""
    with pytest.raises(crm.CrmError):
        a.load_checkpoint(bytes(bad))                    # truncated
    a.close()
    other.close()


def test_state_round_trip_restart_is_bit_identical(crm):
    """FP32 positions: the soil state read at a list rebuild and written into a
    new context (with the same bodies) continues bit for bit."""
    sc = scenes.plate_patch(seed=5, nx=16, ny=16, nz=8, ps_freq=5)
    a = crm.Simulation(sc)
    a.step(10)
    st = a.state()
    n = sc.n_soil
    a.step(6)
    want, Fw = a.state(), a.forces()
    b = crm.Simulation(sc)
    b.set_state(pos=st["pos"][:n], vel=st["vel"][:n], sigma=st["sigma"][:n], rho=st["rho"][:n])
    b.step(6)
    got, Fg = b.state(), b.forces()
    assert _same(got, want)
    assert np.array_equal(Fg[1], Fw[1])
    a.close()
    b.close()


def test_state_read_between_set_bodies_and_step_changes_nothing(crm):
    """crm_get_state after crm_set_bodies (bodies moved) places the markers at
    the new poses without losing them to the working set's records of the
    previous poses: the run continues as one where the state was not read."""
    sc = _strip()
    runs = []
    for read in (False, True):
        sim = crm.Simulation(sc)
        sim.step(2)
        sim.set_bodies(*_bodies(sc, 1.5))
        if read:
            sim.state()
        sim.step(3)
        runs.append((sim.state(), sim.forces()))
        sim.close()
    (a, Fa), (b, Fb) = runs
    assert _same(a, b)
    assert np.array_equal(Fa[0], Fb[0]) and np.array_equal(Fa[1], Fb[1])
