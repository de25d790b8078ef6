"""Host-side checks of libcrm without a GPU: every symbol declared in
include/crm.h is exported, the struct layouts match, the capacity policy
(Sec. 4.2 item 3) follows the hand-computed sequence, and invalid input is
rejected with CRM_E_INVALID before any device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def crm():
    from paper_2507_05643_amd import crm as m
    return m


def _declared():
    txt = open(os.path.join(ROOT, "include", "crm.h")).read()
    return sorted(set(re.findall(r"^\s*(?:crm_status|int64_t|const char\*|void)\s+(crm_\w+)\(", txt, re.M)))


def test_every_declared_symbol_is_exported(crm):
    names = _declared()
    assert len(names) >= 13
    L = crm.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(crm.EXPORTED)


def test_params_layout(crm):
    # two uint32, 3 + 3 doubles, 8 + 2 doubles, 6 doubles, 2 uint32, 3 doubles, 2 uint32, 1 double, 1 int64
    assert C.sizeof(crm.crm_params) == 8 + 8 * 6 + 8 * 10 + 8 * 6 + 8 + 8 * 3 + 8 + 8 + 8 + 8 + 8
    assert crm.crm_params.moved_cap.offset == C.sizeof(crm.crm_params) - 8
    assert crm.crm_params.ps_freq.offset == 8 + 8 * 6 + 8 * 10 + 8 * 6
    assert C.sizeof(crm.crm_body_desc) == 40


def test_capacity_policy(crm):
    f = crm.crm_capacity_next
    assert f(0, 100, 1) == 120
    assert f(120, 110, 1) == 120
    assert f(120, 121, 7) == 146
    assert f(146, 100, 49) == 146
    assert f(146, 100, 50) == 100
    assert f(146, 110, 50) == 146
    assert f(1000, 10, 150) == 10


def _raw_init(crm, p, pos):
    out = C.c_void_p()
    P = crm.make_params(p)
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    st = crm.lib().crm_init(C.byref(P), pos.shape[0], pos.ctypes.data_as(C.POINTER(C.c_double)), None, None, None,
                            0, None, crm.ALLOC_FN(), crm.FREE_FN(), None, None, C.byref(out))
    return st, out.value


@pytest.mark.parametrize("key,val", [("dx", 0.0), ("h", -1.0), ("dt", float("nan")), ("nu", 0.5),
                                     ("mu_s", 0.0), ("av_mode", 3), ("ps_freq", 0), ("grow_G", 0.9),
                                     ("shrink_S", 1.5), ("shrink_interval", 0), ("cohesion", -1.0),
                                     ("kernel", 2), ("pos_mode", 2), ("skin", -1.0)])
def test_invalid_params_rejected(crm, key, val):
    from paper_2507_05643_amd import scenes
    p = dict(scenes.DEFAULT_PARAMS)
    p[key] = val
    st, ctx = _raw_init(crm, p, np.zeros((4, 3)))
    assert st == -1 and not ctx
    assert len(crm.crm_last_error(None)) > 0


def test_invalid_inputs_rejected(crm):
    from paper_2507_05643_amd import scenes
    p = dict(scenes.DEFAULT_PARAMS)
    st, ctx = _raw_init(crm, p, np.full((3, 3), np.inf))
    assert st == -1 and "position" in crm.crm_last_error(None)
    p2 = dict(p, domain_lo=(0.0, 0.0, 0.0), domain_hi=(-1.0, 1.0, 1.0))
    st, _ = _raw_init(crm, p2, np.zeros((3, 3)))
    assert st == -1
    p3 = dict(p, domain_lo=(0.0, 0.0, 0.0), domain_hi=(1e6, 1e6, 1e6))
    st, _ = _raw_init(crm, p3, np.zeros((3, 3)))
    assert st == -6          # cell grid beyond 2^32 cells
    st, _ = _raw_init(crm, p, np.zeros((0, 3)))
    assert st == -1          # no particles at all
