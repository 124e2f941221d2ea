"""The allocation-free G1 query (wp_lattice_resolvent_noalloc) against the allocating one
(wp_lattice_resolvent), through the C ABI: bit-identical results on two calls in a row, the second
on a smaller lattice than the first (the shared scratch array still holds the first call's
values), and no device allocation through the lattice's allocator during either call."""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    import paper_1404_5253_amd as wp


def _lattice(M, two_J, j_max, swave):
    L = wp.Lattice(M, M, two_J=two_J, j_max=j_max, swave_only=swave)
    L.pseudostates(kind="mt", V_R=1438.72)
    L.build_perm("fp64")   # device tables resident
    return L


def test_noalloc_resolvent_matches_allocating_entry_point():
    big = _lattice(40, 1, 2, False)      # 18 channels, 10 pair waves
    small = _lattice(12, 1, 1, True)     # 2 channels
    for L, E_lab, chans in ((big, 22.7, (0, 7, 17)), (small, 3.0, (0, 1))):
        ref = {a: L.resolvent(E_lab, a) for a in chans}
        n0 = L.alloc.n_alloc
        got = {a: L.resolvent_noalloc(E_lab, a) for a in chans}
        assert L.alloc.n_alloc == n0
        for a in chans:
            assert np.array_equal(got[a], ref[a]), (L.M, a)
    # the scratch array keeps the last call's contents: the big lattice again after the small one
    assert np.array_equal(big.resolvent_noalloc(14.1, 3), big.resolvent(14.1, 3))


def test_noalloc_resolvent_energy_weights():
    """The same with energy-weight packets (the closed-form G1 kernel, no work list), after a
    unit-weight call has left its values in the scratch array."""
    unit = _lattice(16, 3, 1, True)
    L = wp.Lattice(20, 20, two_J=1, j_max=1, swave_only=False, weights="energy")
    L.pseudostates(kind="mt", V_R=1438.72)
    L.build_perm("fp64")
    ref_unit = unit.resolvent(3.0, 0)   # makes the G1 tables resident (a documented precondition)
    assert np.array_equal(unit.resolvent_noalloc(3.0, 0), ref_unit)
    L.resolvent(3.0, 0)
    for E_lab in (3.0, 22.7):
        for a in (0, 4, 9):
            n0 = L.alloc.n_alloc
            got = L.resolvent_noalloc(E_lab, a)
            assert L.alloc.n_alloc == n0
            assert np.array_equal(got, L.resolvent(E_lab, a)), (E_lab, a)
