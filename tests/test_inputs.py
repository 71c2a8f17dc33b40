"""The seeded input generators (no method arithmetic): the paper's LES start
(Sec. 6) is divergence-free on the staggered grid, vanishes on the walls, has
the flattened laminar mean and the stated perturbation rms."""
import numpy as np
import pytest

import oracle
from paper_1511_07800_amd import inputs, workloads


def test_les_curl_state_is_divergence_free_with_stated_mean():
    wl = workloads.params("les_channel_paper_240x140x120")
    nx, ny, nz = 48, 28, 24  # the paper's box at a fifth of its resolution
    u, v, w = inputs.les_curl_state(nx, ny, nz, wl["lx"], wl["ly"], wl["lz"], wl["nu"], wl["dpdx"],
                                    a=wl["curl_a"], modes=wl["curl_modes"], seed=wl["seed"])
    P = oracle.make_params(nx, ny, nz, wl["lx"], wl["ly"], wl["lz"])
    scale = np.abs(u).max() * nx / wl["lx"]
    assert np.abs(oracle.divergence(P, u, v, w)).max() <= 1e-14 * scale
    assert not w[0].any() and not w[nz].any()
    base = inputs.laminar_profile(nz, wl["lz"], wl["nu"], wl["dpdx"])
    # every mode has kx, ky >= 1: the perturbation has no x-y mean
    np.testing.assert_allclose(u.mean(axis=(1, 2)), base / 3, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(v.mean(axis=(1, 2)), 0.0, atol=1e-12)
    du = u - base[:, None, None] / 3
    rms = np.sqrt((np.sum(du**2) + np.sum(v**2) + np.sum(w**2)) / (du.size + v.size + w.size))
    assert rms == pytest.approx(0.1 * base.max() / 3, rel=2e-3)  # a tenth of the flattened centreline speed
    # seeded: the same seed gives the same field, another seed another one
    u2, _, _ = inputs.les_curl_state(nx, ny, nz, wl["lx"], wl["ly"], wl["lz"], wl["nu"], wl["dpdx"], seed=wl["seed"])
    u3, _, _ = inputs.les_curl_state(nx, ny, nz, wl["lx"], wl["ly"], wl["lz"], wl["nu"], wl["dpdx"], seed=7)
    assert np.array_equal(u, u2) and not np.array_equal(u, u3)
