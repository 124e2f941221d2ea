"""CPU tests of libwpcd: symbol exports, argument checking, call order and the host FP64 steps
(channels, pseudostates, strength tuning) against the oracle. No GPU work is started."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_1404_5253_amd as wp
from oracle import channels, pipeline

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "wpcd.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(\w+)\s*\(", txt, flags=re.M)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert "perm_matrix_build" in names and "faddeev_solve" in names and "amplitude" in names
    lib = C.CDLL(wp.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(wp.exported_symbols())


def test_argument_errors_and_call_order():
    with pytest.raises(wp.WpError) as e:
        wp.wp_lattice_build(1, 10)
    assert e.value.status == wp.WP_EINVAL
    with pytest.raises(wp.WpError):
        wp.wp_lattice_build(10, 10, n_x=40)
    with pytest.raises(wp.WpError):
        wp.wp_lattice_build(10, 10, p_edges=np.array([0.0] + [1.0] * 10), q_edges=np.linspace(0, 1, 11))
    L = wp.Lattice(8, 8, two_J=3, torch_alloc=False)
    with pytest.raises(wp.WpError) as e:
        L.solve([10.0])
    assert e.value.status == wp.WP_ENOTREADY
    with pytest.raises(wp.WpError) as e:
        L.resolvent(10.0, 0)
    assert e.value.status == wp.WP_ENOTREADY
    assert wp._lib.perm_matrix_export(L.h, None, None, None) == wp.WP_ENOTREADY
    assert b"perm_matrix_build" in wp._lib.wp_last_error()


@pytest.mark.parametrize("two_J,j_max,swave", [(1, 2, False), (1, 1, True), (3, 1, True), (3, 2, False)])
def test_channels_match_oracle(two_J, j_max, swave):
    L = wp.Lattice(6, 6, two_J=two_J, j_max=j_max, swave_only=swave, torch_alloc=False)
    ref = channels.enumerate_channels(two_J, +1, j_max)
    if swave:
        ref = [c for c in ref if c[0] == 0 and c[3] == 0]
    assert L.channels == ref


@pytest.mark.parametrize("pot,two_J", [("yamaguchi", 3), ("mt", 1)])
def test_pseudostates_match_oracle(pot, two_J):
    M = 20
    L = wp.Lattice(M, M, two_J=two_J, torch_alloc=False)
    eps0, strength = L.pseudostates(kind=pot)
    s = pipeline.build_system(pipeline.Spec(M=M, N=M, two_J=two_J, pot=pot))
    assert strength == pytest.approx(s.strength, rel=1e-12)
    assert eps0 == pytest.approx(-2.2246, abs=1e-12)
    pe, qe = L.edges()
    assert np.allclose(pe, s.p_edges, rtol=1e-15, atol=0) and np.allclose(qe, s.q_edges, rtol=1e-15, atol=0)
    for a, ch in enumerate(L.channels):
        nb, eps, O, bins = L.pseudostate_data(a)
        d = s.pair[(ch[0], ch[1])]
        assert nb == d["nb"]
        assert np.allclose(eps, d["eps"], rtol=1e-11, atol=1e-11)
        # signs fixed by the same convention on both sides (largest component positive)
        assert np.allclose(O, d["O"], atol=1e-10)
        assert np.allclose(O @ O.T, np.eye(M), atol=1e-13)
        assert np.allclose(bins, d["bins"], rtol=1e-12)


def test_noalloc_resolvent_host_checks():
    """wp_lattice_resolvent_noalloc rejects, before any device work, a lattice whose scratch need
    exceeds the fixed array (WP_EINVAL) and a lattice whose device tables are not resident yet
    (WP_ENOTREADY)."""
    L = wp.Lattice(12, 12, two_J=1, torch_alloc=False)
    L.pseudostates(kind="mt", V_R=1438.72)
    G = np.zeros(2 * 12 * 12)
    st = wp._lib.wp_lattice_resolvent_noalloc(L.h, 14.1, 0, G.ctypes.data_as(C.POINTER(C.c_double)))
    assert st == wp.WP_ENOTREADY and b"not resident" in wp._lib.wp_last_error()
    big = wp.Lattice(600, 600, two_J=1, torch_alloc=False)
    big.pseudostates(kind="mt", V_R=1438.72)
    G = np.zeros(2 * 600 * 600)
    st = wp._lib.wp_lattice_resolvent_noalloc(big.h, 14.1, 0, G.ctypes.data_as(C.POINTER(C.c_double)))
    assert st == wp.WP_EINVAL and b"scratch" in wp._lib.wp_last_error()


def test_lattice_info_matches_the_oracle_rule():
    """Moment count of the P0 rule and stored values per block: the oracle's distinct moment keys,
    and the channel pairs with a nonzero recoupling coefficient (all n_ch^2 for <= 4 channels)."""
    for spec in (pipeline.Spec(M=6, N=7, two_J=1, j_max=2, swave_only=False, pot="mt"),
                 pipeline.Spec(M=6, N=6, two_J=1, pot="mt")):
        s = pipeline.build_system(spec)
        L = wp.Lattice(spec.M, spec.N, two_J=spec.two_J, j_max=spec.j_max, swave_only=spec.swave_only,
                       torch_alloc=False)
        assert L.nmom == len(s.P0geo.keys)
        nz = int(np.any(s.C != 0.0, axis=2).sum())
        assert L.n_stored == (nz if L.nch > 4 else L.nch ** 2), (L.n_stored, nz)


@pytest.mark.parametrize("pot,two_J", [("yamaguchi", 3), ("mt", 1)])
def test_energy_weight_pseudostates_match_oracle(pot, two_J):
    """Energy-weight packets (Sec. III.B footnote): h0, potential, strength tuning, pseudostates and
    the energy bins against the oracle."""
    M = 16
    L = wp.Lattice(M, M, two_J=two_J, torch_alloc=False, weights="energy")
    eps0, strength = L.pseudostates(kind=pot)
    s = pipeline.build_system(pipeline.Spec(M=M, N=M, two_J=two_J, pot=pot, weights="energy"))
    assert strength == pytest.approx(s.strength, rel=1e-11)
    assert eps0 == pytest.approx(-2.2246, abs=1e-12)
    for a, ch in enumerate(L.channels):
        nb, eps, O, bins = L.pseudostate_data(a)
        d = s.pair[(ch[0], ch[1])]
        assert nb == d["nb"]
        assert np.allclose(eps, d["eps"], rtol=1e-10, atol=1e-10)
        assert np.allclose(O, d["O"], atol=1e-9)
        assert np.allclose(bins, d["bins"], rtol=1e-11)


def test_weights_call_order():
    L = wp.Lattice(8, 8, two_J=3, torch_alloc=False)
    assert wp._lib.wp_lattice_weights(L.h, 7) == wp.WP_EINVAL
    assert wp._lib.wp_lattice_weights(L.h, wp.WP_WEIGHTS_ENERGY) == wp.WP_OK
    L.pseudostates(kind="yamaguchi")
    assert wp._lib.wp_lattice_weights(L.h, wp.WP_WEIGHTS_UNIT) == wp.WP_EINVAL
    assert b"before twobody_pseudostates" in wp._lib.wp_last_error()
    with pytest.raises(ValueError):
        wp.Lattice(8, 8, torch_alloc=False, weights="momentum")


def test_rule_size_limits():
    """n_x, n_phi in [1, 64] with at most 256 nodes per cell pair (the per-box kernels' limit)."""
    wp.Lattice(6, 6, n_x=64, n_phi=4, torch_alloc=False)
    wp.Lattice(6, 6, n_x=16, n_phi=16, torch_alloc=False)
    for nx, nphi in ((65, 1), (20, 20), (0, 8)):
        with pytest.raises(wp.WpError) as e:
            wp.Lattice(6, 6, n_x=nx, n_phi=nphi, torch_alloc=False)
        assert e.value.status == wp.WP_EINVAL
