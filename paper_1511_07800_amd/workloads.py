"""The five channel workloads, as physical parameters.

The paper non-dimensionalises with the channel height (walls at z = 0 and 1)
and the friction velocity U = sqrt(L_z |dp/dx| / 2) (Sec. 2.1).  These
workloads are stated with walls at z = 0 and 2 (half-height 1):
  * laminar cases by a centreline Reynolds number Re = U_cl / nu with the
    laminar centreline speed U_cl = |G| / (2 nu) = 1, so nu = 1/Re, G = -2/Re;
  * LES cases by Re_tau = u_tau / nu with u_tau = sqrt(L_z |G| / 2) = 1, so
    G = -1, nu = 1/Re_tau.
dt of the LES cases follows the paper's rule U_max dt <= 0.1 dx (Sec. 3.2)
for the laminar start (U_cl = |G|/(2 nu) = 90) plus its 10% noise.
srj_reduction of the LES cases is the bound on one FP32 defect-correction
pass's reduction (the adaptive cycles never aim lower): 1e-4 is about what an
FP32 pass attains, so two passes reach 1e-8 from the previous pressure.
"""
import math

WORKLOADS = {
    "laminar_poiseuille_32x16x16": dict(
        nx=32, ny=16, nz=16, lx=2 * math.pi, ly=math.pi, lz=2.0, nu=1.0 / 100, dpdx=-2.0 / 100, dt=1e-3,
        les=0, steps=200, precision="fp64", poisson_rtol=1e-10, init="rest"),
    "linear_instability_256x8x128": dict(
        nx=256, ny=8, nz=128, lx=2 * math.pi, ly=0.5, lz=2.0, nu=1.0 / 7500, dpdx=-2.0 / 7500, dt=5e-4,
        les=0, steps=4000, precision="fp64", poisson_rtol=1e-10, init="ts_wave", ts_alpha=1.0,
        ts_amplitude=1e-5, noise=1e-7, seed=1511),
    "les_channel_256x128x128": dict(
        nx=256, ny=128, nz=128, lx=4 * math.pi, ly=2 * math.pi, lz=2.0, nu=1.0 / 180, dpdx=-1.0, dt=4e-5,
        les=1, cs=0.1, vd_a=25.0, steps=500, precision="mixed", poisson_rtol=1e-8, srj_reduction=1e-4,
        init="laminar_noise",
        noise=0.1, seed=7800),
    "les_channel_512x256x192": dict(
        nx=512, ny=256, nz=192, lx=4 * math.pi, ly=2 * math.pi, lz=2.0, nu=1.0 / 180, dpdx=-1.0, dt=2e-5,
        les=1, cs=0.1, vd_a=25.0, steps=500, precision="mixed", poisson_rtol=1e-8, srj_reduction=1e-4,
        init="laminar_noise",
        noise=0.1, seed=7801),
    "les_channel_1024x512x384": dict(
        nx=1024, ny=512, nz=384, lx=4 * math.pi, ly=2 * math.pi, lz=2.0, nu=1.0 / 180, dpdx=-1.0, dt=1e-5,
        les=1, cs=0.1, vd_a=25.0, steps=500, precision="mixed", poisson_rtol=1e-8, srj_reduction=1e-4,
        init="laminar_noise",
        noise=0.1, seed=7802),
    # the paper's LES (Sec. 6 and its LES parameter table): height 1, friction
    # velocity 1 (|G| = 2), Re_* = 360; the start is a U0 + curl[f A] with 5^3
    # random Fourier modes (a = 1/3), statistics averaged over t in [20, 53]
    "les_channel_paper_240x140x120": dict(
        nx=240, ny=140, nz=120, lx=8.0, ly=4.0, lz=1.0, nu=1.0 / 360, dpdx=-2.0, dt=1e-4,
        les=1, cs=0.1, vd_a=25.0, steps=530000, precision="mixed", poisson_rtol=1e-8, srj_reduction=1e-4,
        init="curl_random_modes", curl_a=1.0 / 3.0, curl_modes=5, seed=360, t_stats=(20.0, 53.0)),
}


def params(name):
    return dict(WORKLOADS[name])
