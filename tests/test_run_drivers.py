"""Host-side measurement code of the two validation drivers, on signals whose
answers are known in closed form: the Orr-Sommerfeld growth-rate and period
fits (Sec. 4.2) and the LES bulk statistics (Sec. 6)."""
import math

import numpy as np
import pytest

from paper_1511_07800_amd import os_validation
from paper_1511_07800_amd.les import bulk


def test_growth_rate_and_period_of_a_damped_oscillation():
    """L2^w = A e^{sigma t} and W_m = e^{sigma t} cos(omega t + phi): the fit
    returns sigma exactly and the crossings 2 pi / omega to the sampling step."""
    sigma, omega, dt = 1.8056, 33.873, 1e-3
    ts = np.arange(1, 1001) * dt
    l2 = 3e-5 * np.exp(sigma * ts)
    wm = np.exp(sigma * ts) * np.cos(omega * ts + 0.3)
    assert os_validation.growth_rate(ts, l2, 0.05) == pytest.approx(sigma, rel=1e-12)
    t_osc = os_validation.period(ts, wm, 0.05)
    # each crossing lands within one sample of the true one, and 2 x the mean
    # of the N - 1 >= 9 spacings after t = 0.05 is then within 2 dt / 9
    assert abs(t_osc - 2 * math.pi / omega) <= 2 * dt / 9
    # too few crossings
    assert os_validation.period(ts[:20], wm[:20], 0.0) is None


def test_growth_rate_ignores_samples_before_the_window():
    ts = np.linspace(0.0, 1.0, 201)
    l2 = np.where(ts < 0.5, np.exp(5 * ts), math.exp(2.5) * np.exp(-1.0 * (ts - 0.5)))
    assert os_validation.growth_rate(ts, l2, 0.5) == pytest.approx(-1.0, rel=1e-12)


@pytest.mark.parametrize("nz", [16, 15])
def test_bulk_statistics_of_the_laminar_profile(nz):
    """<u> = z(1 - z)/nu sampled at the cell centres (G = -2, H = 1): U_mean =
    (1 + dz^2/2)/(6 nu) (the midpoint rule exceeds the integral 1/6 by
    dz^2/12 for a parabola of curvature -2), U_cl and U_max at the
    centre plane(s), C_f = 2/U_mean^2, and the wall shear from the odd ghost
    nu 2 <u>_0 / dz = 1 - dz/2."""
    nu = 1.0 / 360.0
    wl = {"nz": nz, "lz": 1.0, "nu": nu}
    dz = 1.0 / nz
    zc = (np.arange(nz) + 0.5) * dz
    prof = zc * (1 - zc) / nu
    st = bulk(prof, wl)
    u_mean = (1 + dz * dz / 2) / (6 * nu)
    assert st["U_mean"] == pytest.approx(u_mean, rel=1e-13)
    assert st["Re_mean"] == pytest.approx(u_mean / nu, rel=1e-13)
    if nz % 2 == 0:
        u_cl = 0.5 * (prof[nz // 2 - 1] + prof[nz // 2])
    else:
        u_cl = 0.25 / nu
    assert st["U_cl"] == pytest.approx(u_cl, rel=1e-13)
    assert st["U_max"] == pytest.approx(prof.max(), rel=0)
    assert st["C_f"] == pytest.approx(2 / u_mean**2, rel=1e-13)
    assert st["wall_shear"] == pytest.approx(1 - dz / 2, rel=1e-12)
