"""CPU tests of the library's elastic-observable calls (host FP64, no GPU work) against the oracle:
channel-spin S, eigenphases, dsigma/dOmega and A_y over J^pi blocks with random symmetric S
(unitary and not), and the argument checks."""
import numpy as np
import pytest

import paper_1404_5253_amd as wp
from oracle import channels
from oracle import observables as ob


def _blocks(seed, unitary=True, twoJs=(1, 3, 5, 7, 9)):
    rng = np.random.default_rng(seed)
    out = []
    for two_J in twoJs:
        for par in (1, -1):
            chans = wp.open_channels(channels.enumerate_channels(two_J, par, 1))
            n = len(chans)
            O, _ = np.linalg.qr(rng.normal(size=(n, n)))
            d = np.exp(2j * rng.uniform(-1.5, 1.5, n)) * (1.0 if unitary else rng.uniform(0.4, 1.0, n))
            out.append((two_J, chans, O @ np.diag(d) @ O.T))
    return out


@pytest.mark.parametrize("unitary", [True, False])
def test_observables_match_oracle(unitary):
    blocks = _blocks(5, unitary)
    th = np.linspace(0.0, np.pi, 13)
    for k in (0.2, 0.9):
        ds, ay = wp.nd_elastic_observables(blocks, k, th)
        ds0, ay0 = ob.observables(blocks, k, th)
        assert np.max(np.abs(ds - ds0) / ds0) <= 1e-13
        assert np.max(np.abs(ay - ay0)) <= 1e-13


def test_sigma_rep_and_eigenphases_match_oracle():
    for two_J, chans, S in _blocks(6):
        sig, Ss = wp.nd_sigma_rep(two_J, chans, S)
        sig0, Ss0 = ob.to_sigma(two_J, chans, S)
        assert sig == sig0
        assert np.max(np.abs(Ss - Ss0)) <= 1e-14
        d, O = wp.nd_eigenphases(Ss)
        assert np.allclose(O @ np.diag(np.exp(2j * d)) @ O.T, Ss, atol=1e-13)
        d0, _ = ob.eigenphases(Ss)
        assert np.allclose(np.sort(np.mod(d, np.pi)), np.sort(np.mod(d0, np.pi)), atol=1e-12)


def test_observable_argument_checks():
    S = np.eye(2, dtype=complex)
    with pytest.raises(wp.WpError):
        wp.nd_sigma_rep(1, [(0, 1), (2, 5)], S)     # lam = 2 shell incomplete for J = 1/2
    with pytest.raises(wp.WpError):
        wp.nd_elastic_observables([(1, [(0, 1), (2, 3)], S)], -1.0, [0.5])
    with pytest.raises(wp.WpError):
        wp.nd_eigenphases(np.eye(9, dtype=complex))


def test_spin_free_scattering_matches_the_spinless_formula():
    from test_oracle_observables import _spin_free_blocks, spinless_cross_section
    rng = np.random.default_rng(8)
    # lam <= 3 scatter: up to J = 9/2 every (lam, Sigma, J) of these lam is present; higher lam
    # (incomplete shells) do not scatter
    s_lam = np.ones(8, dtype=complex)
    s_lam[:4] = np.exp(2j * rng.uniform(-1.2, 1.2, 4)) * rng.uniform(0.6, 1.0, 4)
    blocks = [(tJ, [tuple(c) for c in ch], S) for tJ, ch, S in _spin_free_blocks(s_lam)]
    th = np.linspace(0.0, np.pi, 11)
    ds, ay = wp.nd_elastic_observables(blocks, 0.8, th)
    assert np.max(np.abs(ay)) <= 1e-12
    assert np.allclose(ds, spinless_cross_section(s_lam, 0.8, th), rtol=1e-11)
