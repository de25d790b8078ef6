"""The comparison helpers of the GPU parity tests, on hand-made inputs (CPU)."""
import numpy as np
import pytest

from tests.parity_util import check_cell_sort, csr_rows, normwise

# three cells: ids 0..5; cell 0 holds {3, 0}, cell 1 is empty, cell 2 holds {1, 4, 2}, cell 3 holds {5}
X = np.array([[0.30, 0, 0], [0.70, 0, 0], [0.90, 0, 0], [0.10, 0, 0], [0.80, 0, 0], [1.50, 0, 0]])
SID = np.array([0, 3, 1, 2, 4, 5])          # oracle: cell order, ids ascending in a cell
CS = np.array([0, 2, 2, 5])
CE = np.array([2, 2, 5, 6])


def test_accepts_x_order_inside_cells():
    check_cell_sort(np.array([3, 0, 1, 4, 2, 5]), SID, CS, CE, X)


def test_accepts_the_oracle_order_when_it_ascends_in_x():
    x = X.copy()
    x[3, 0] = 0.35                      # id 3 now right of id 0, id 2 right of 4 already
    x[2, 0] = 0.95
    check_cell_sort(np.array([0, 3, 1, 4, 2, 5]), SID, CS, CE, x)


def test_rejects_id_order_against_x():
    with pytest.raises(AssertionError):
        check_cell_sort(SID, SID, CS, CE, X)        # id 0 (x 0.30) before id 3 (x 0.10)


def test_rejects_a_particle_in_the_wrong_cell():
    with pytest.raises(AssertionError):
        check_cell_sort(np.array([3, 1, 0, 4, 2, 5]), SID, CS, CE, X)


def test_rejects_a_missing_particle():
    with pytest.raises(AssertionError):
        check_cell_sort(np.array([3, 0, 1, 4, 4, 5]), SID, CS, CE, X)


def test_csr_rows_sorts_each_row_and_maps_row_ids():
    off = np.array([0, 2, 2, 5])
    nbr = np.array([7, 3, 9, 1, 4])
    got = csr_rows(off, nbr, rows=np.array([10, 11, 12]))
    assert list(got) == [10, 11, 12]
    assert got[10].tolist() == [3, 7] and got[11].tolist() == [] and got[12].tolist() == [1, 4, 9]


def test_normwise():
    assert normwise([1.0, 2.0], [1.0, 2.0]) == 0.0
    assert normwise([1.0, 2.5], [1.0, 2.0]) == pytest.approx(0.25)
    assert normwise([0.5], [0.0]) == 0.5


def test_displacement_bar():
    from tests.parity_util import displacement_bar, half_ulp32
    assert half_ulp32(1.0) == 2.0 ** -24
    assert half_ulp32(0.16) == 2.0 ** -27          # 0.16 lies in [0.125, 0.25)
    # 100 steps near 0.16 m with 3e-5 m of motion: 1e-3 + 101 * 7.45e-9 / 3e-5
    b = displacement_bar(100, 1e-3, 0.16, 3.0e-5)
    assert abs(b - (1e-3 + 101 * 2.0 ** -27 / 3.0e-5)) < 1e-15
    assert displacement_bar(5, 1e-3, 0.16, 0.0) == 0.0


def test_check_fields_catches_a_frozen_position():
    """A path that never moves its particles passes a position check normalised
    by the coordinates, but not the displacement check."""
    import types
    from tests.parity_util import check_fields
    rng = np.random.default_rng(0)
    x0 = rng.uniform(0.0, 0.16, size=(500, 3)).astype(np.float32).astype(np.float64)
    ref = dict(pos=x0 + rng.normal(0.0, 3e-5, size=x0.shape), vel=np.ones((500, 3)), sigma=np.ones((500, 6)),
               rho=np.ones(500))
    got = dict(ref, pos=x0.copy())
    sc = types.SimpleNamespace(n_soil=500, pos=x0, params=dict(pos_mode=0, h=0.012))
    import pytest
    with pytest.raises(AssertionError):
        check_fields(got, ref, sc, 100, 1e-3)
    check_fields(ref, ref, sc, 100, 1e-3)
