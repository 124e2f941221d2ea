"""Failure paths forced from the host, every kernel exiting normally: a one-byte device-memory
budget (WP_EBUDGET), a solve cut off before its series converges (WP_ENOCONV, the solution still
returned), non-finite or out-of-lattice energies (WP_EINVAL before any launch), and the call order
(WP_ENOTREADY)."""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    import paper_1404_5253_amd as wp


def _lat():
    L = wp.Lattice(12, 12, two_J=1)
    L.pseudostates(kind="mt", V_R=1438.72)
    L.build_perm("fp64")
    return L


def test_one_byte_budget_is_rejected():
    import ctypes as C
    L = _lat()
    for mode in (wp.WP_SOLVE_FP64, wp.WP_SOLVE_MIXED_SPLIT):
        o = wp._SolveOpts(mode=mode, tol=1e-10, accept=1e-6, max_iter=200)
        b = C.c_void_p()
        st = wp._lib.faddeev_batch_create(L.h, 4, 1, C.byref(o), C.byref(b))
        assert st == wp.WP_EBUDGET and not b.value
        assert b"budget" in wp._lib.wp_last_error()


def test_cut_off_series_reports_no_convergence():
    L = _lat()
    with pytest.raises(wp.WpError) as e:
        L.solve([14.1], "fp64", tol=1e-14, accept=1e-14, max_iter=6)
    assert e.value.status == wp.WP_ENOCONV
    sol = L.solve([14.1], "fp64", tol=1e-14, accept=1e-14, max_iter=6, allow_noconv=True)
    assert not sol.converged
    assert np.all(np.isfinite(sol.amplitude(0)["A"]))
    with pytest.raises(wp.WpError) as e:
        L.solve([14.1], "fp64", max_iter=3)   # fewer than four terms: not a valid request
    assert e.value.status == wp.WP_EINVAL


@pytest.mark.parametrize("E", [float("nan"), float("inf"), -1.0, 1e6])
def test_bad_energies_are_rejected(E):
    L = _lat()
    with pytest.raises(wp.WpError) as e:
        L.solve([14.1, E], "fp64")
    assert e.value.status == wp.WP_EINVAL


def test_call_order():
    L = wp.Lattice(8, 8, two_J=3)
    with pytest.raises(wp.WpError) as e:
        L.build_perm("fp64")
        L.solve([3.0], "fp64")
    assert e.value.status == wp.WP_ENOTREADY
