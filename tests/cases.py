"""Workload parameter sets shared by the tests: each side (oracle, library) builds
its own objects from these plain dictionaries."""
from paper_2405_04229_amd import workload as W

LINSLEY = dict(a=W.LINSLEY_A, b=W.LINSLEY_B, c=W.LINSLEY_C, hb=W.LINSLEY_HB_M, kappa=W.KAPPA)

# straight rays, Rayleigh only, continuous wavelength (tiny vertical workload)
ATMO_STRAIGHT = dict(profile="linsley5", h_top=25000.0, step=1.0, rayleigh400=2974.0, **LINSLEY)
# 100 layers of 250 m, Rayleigh + aerosol tables on 64 wavelength bins (telescope workload)
ATMO_LAYERED = dict(profile="linsley5", h_top=25000.0, step=1.0, rayleigh400=2974.0, aer_tau350=0.05,
                    aer_H=1200.0, aer_angstrom=1.0, n_layers=100, n_lam=64, **LINSLEY)

RUN_TINY = dict(transport="straight", detector="grid", spectrum="uniform", bunch=1, h_obs=2200.0,
                nx=100, ny=100, cell=10.0)
RUN_TELESCOPE = dict(transport="layered", detector="spheres", spectrum="frank_tamm", bunch=5, h_obs=2200.0,
                     snx=10, sny=10, pitch=150.0, radius=6.0, n_t=512, dt=1.0)
