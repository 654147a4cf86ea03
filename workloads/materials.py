"""Optical constants of silver and the LSPR wavelength grid.

The table is the paper's printed excerpt of Johnson and Christy's silver
data (Sec. 6.3, Benchmark II, table "Optical constants of silver"): wavelength in nm,
refractive index n and extinction coefficient kappa, with
eps_r = (n + i kappa)^2.  Between table rows n and kappa are interpolated
linearly in the wavelength (the paper only says that the permittivity is
interpolated; this reading reproduces its quoted eps_r = -10.15 + 0.32i at
506 nm).  Outside the table range the functions raise.
"""
from __future__ import annotations

import numpy as np

# (lambda [nm], n, kappa), increasing lambda
JC_SILVER = np.array([
    (300.9, 1.34, 0.964), (310.7, 1.13, 0.616), (320.4, 0.81, 0.392),
    (331.5, 0.17, 0.829), (342.5, 0.14, 1.142), (354.2, 0.10, 1.419),
    (367.9, 0.07, 1.657), (381.5, 0.05, 1.864), (397.4, 0.05, 2.070),
    (413.3, 0.05, 2.275), (430.5, 0.04, 2.462), (450.9, 0.04, 2.657),
    (471.4, 0.05, 2.869), (495.9, 0.05, 3.093), (520.9, 0.05, 3.324),
    (548.6, 0.06, 3.586), (582.1, 0.05, 3.858), (616.8, 0.06, 4.152),
    (659.5, 0.05, 4.483), (704.5, 0.04, 4.838), (756.0, 0.03, 5.242),
    (821.1, 0.04, 5.727),
], dtype=np.float64)


def silver_eps(lam_nm) -> np.ndarray:
    """Relative permittivity of silver at the given vacuum wavelengths [nm]."""
    lam = np.atleast_1d(np.asarray(lam_nm, dtype=np.float64))
    lo, hi = JC_SILVER[0, 0], JC_SILVER[-1, 0]
    if np.any(lam < lo) or np.any(lam > hi):
        raise ValueError(f"wavelength outside the table range [{lo}, {hi}] nm")
    n = np.interp(lam, JC_SILVER[:, 0], JC_SILVER[:, 1])
    kap = np.interp(lam, JC_SILVER[:, 0], JC_SILVER[:, 2])
    return (n + 1j * kap) ** 2


def lspr_wavelengths() -> np.ndarray:
    """The spectrum grid of the silver-spheroid benchmark: 350-800 nm, 1 nm
    steps over 475-525 nm and 5 nm steps elsewhere (131 wavelengths)."""
    return np.concatenate([np.arange(350.0, 475.0, 5.0), np.arange(475.0, 526.0, 1.0),
                           np.arange(530.0, 801.0, 5.0)])
