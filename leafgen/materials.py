"""Per-label complex refractive indices n + ik as functions of vacuum wavelength.

Input recipes only: these tables feed both the oracle and the GPU library, and
hold none of the method's arithmetic (the map (n, k) -> (eps_r, sigma) -> update
coefficients lives separately in each of them).

Values follow the paper's tissue classes (Sec. 2.8: cuticle, cell wall,
pigment, water) with synthetic stand-ins where the paper takes data from
PROSPECT-PRO or from figures that are not available:
  * cuticle n = 1.50 (the synthetic-leaf workloads' value; the paper uses 1.45),
  * cell walls n = 1.42-1.52 (paper: 1.52),
  * cytoplasm/water n = 1.33 + B (1/lambda^2 - 1/0.55^2), B = 0.003 um^2, with a
    synthetic water-absorption k: Gaussian bands at 970, 1200, 1450 and
    1940 nm and a rise towards 2500 nm, of the magnitudes liquid water has
    there (k ~ 4e-6, 1e-5, 3e-4, 2e-3, 1e-3); k < 1e-7 below 900 nm,
  * chloroplast n = 1.36 (paper's pigment n) with
    k = 1e-5 + 0.02 [G(430 nm, 25 nm) + G(662 nm, 15 nm)], G a unit Gaussian,
  * melanised hypha n = 1.7, k = 0.3 (0.05/0.3)^((lambda - 400 nm)/600 nm).
Wavelengths are in metres.
"""
from __future__ import annotations

import numpy as np


def _um(lam_m: float) -> float:
    return lam_m * 1e6


def gaussian(lam_nm: float, centre_nm: float, width_nm: float) -> float:
    return float(np.exp(-0.5 * ((lam_nm - centre_nm) / width_nm) ** 2))


def air(lam):
    return 1.0, 0.0


def cuticle(lam):
    return 1.50, 0.0


def wall(n):
    return lambda lam: (n, 0.0)


def water_k(lam):
    ln = lam * 1e9
    k = (4e-6 * gaussian(ln, 970.0, 30.0) + 1e-5 * gaussian(ln, 1200.0, 40.0)
         + 3e-4 * gaussian(ln, 1450.0, 60.0) + 2e-3 * gaussian(ln, 1940.0, 70.0)
         + 1e-3 * gaussian(ln, 2600.0, 150.0))
    return k if k >= 1e-12 else 0.0


def cytoplasm(lam):
    lu = _um(lam)
    return 1.33 + 0.003 * (1.0 / lu ** 2 - 1.0 / 0.55 ** 2), water_k(lam)


def chloroplast(lam):
    ln = lam * 1e9
    return 1.36, 1e-5 + 0.02 * (gaussian(ln, 430.0, 25.0) + gaussian(ln, 662.0, 15.0))


def hypha(lam):
    ln = lam * 1e9
    return 1.7, 0.3 * (0.05 / 0.3) ** ((ln - 400.0) / 600.0)


def vascular(lam):
    return 1.45, 0.0


# Label tables.  Index = label value in the uint8 map.
DICOT_LABELS = ["air", "cuticle", "wall_epidermis", "wall_palisade", "wall_spongy",
                "cytoplasm", "chloroplast", "hypha"]
_DICOT_FUNCS = [air, cuticle, wall(1.52), wall(1.47), wall(1.42), cytoplasm, chloroplast, hypha]

MONOCOT_LABELS = ["air", "cuticle", "wall", "epidermal_cytoplasm", "mesophyll_cytoplasm",
                  "chloroplast", "vascular"]
_MONOCOT_FUNCS = [air, cuticle, wall(1.52), cytoplasm, cytoplasm, chloroplast, vascular]


def dicot_nk(lam: float) -> np.ndarray:
    """(8, 2) table of (n, k) for the dicot label set at wavelength lam (m)."""
    return np.array([f(lam) for f in _DICOT_FUNCS], dtype=np.float64)


def monocot_nk(lam: float) -> np.ndarray:
    """(7, 2) table of (n, k) for the monocot label set at wavelength lam (m)."""
    return np.array([f(lam) for f in _MONOCOT_FUNCS], dtype=np.float64)


def slab_nk(n: float = 1.45, k: float = 0.01) -> np.ndarray:
    return np.array([[1.0, 0.0], [n, k]], dtype=np.float64)


# ---------------------------------------------------------------------------
# Dispersive (Lorentz-Drude) stand-ins for broadband runs
# ---------------------------------------------------------------------------
# eps(w) = eps_inf + i sigma/(w eps0) + sum_p a_p/(w_p^2 - w^2 - i g_p w), a row
# per label: eps_inf, sigma (S/m), then (a_p, w_p, g_p) per pole, two poles.
#   * cuticle, walls: eps_inf = n^2 of the monochromatic table, no dispersion;
#   * cytoplasm/water: one undamped ultraviolet pole (126 nm, d_eps 0.5) on
#     eps_inf = 1.2425, which reproduces the Cauchy n of the table within 0.002
#     over 400-1000 nm (the weak water bands above 900 nm are left out);
#   * chloroplast: Lorentz absorption lines at 430 and 662 nm whose peak k
#     (0.020) and widths match the table's Gaussians, on eps_inf = 1.8392 and a
#     conductivity that gives the table's background k = 1e-5 at 700 nm; the
#     Lorentzian wings absorb more between the lines (k ~ 2-4e-3) than the table;
#   * melanised hypha: one broad ultraviolet pole (330 nm, d_eps 0.8224,
#     damping 0.7736 w_p) on eps_inf = 2.0559, a least-squares fit to the
#     table's n = 1.7 and falling k (n 1.63-1.71, k 0.32 -> 0.07 over 400-1000 nm).
_C0 = 299792458.0
_EPS0 = 1.0 / (1.25663706212e-6 * _C0 * _C0)
MODEL_POLES = 2


def _pole(d_eps: float, lam_p: float, gamma_rel: float):
    wp = 2.0 * np.pi * _C0 / lam_p
    return [d_eps * wp * wp, wp, gamma_rel * wp]


def _chl_gamma(lam_c: float, sigma_nm: float) -> float:
    """Damping (in units of w_p) whose Lorentzian FWHM equals the Gaussian's."""
    fwhm = 2.3548 * sigma_nm * 1e-9
    return fwhm / lam_c


def dicot_model() -> np.ndarray:
    """(8, 2 + 3*2) Lorentz-Drude table for the dicot label set (see above)."""
    none = [0.0, 0.0, 0.0]
    g1, g2 = _chl_gamma(430e-9, 25.0), _chl_gamma(662e-9, 15.0)
    im_peak = 2.0 * 1.36 * 0.02
    d1, d2 = im_peak * g1, im_peak * g2
    sigma_chl = 2.0 * 1.36 * 1e-5 * (2.0 * np.pi * _C0 / 700e-9) * _EPS0
    rows = [
        [1.0, 0.0] + none + none,                                   # air
        [1.50 ** 2, 0.0] + none + none,                             # cuticle
        [1.52 ** 2, 0.0] + none + none,                             # epidermis wall
        [1.47 ** 2, 0.0] + none + none,                             # palisade wall
        [1.42 ** 2, 0.0] + none + none,                             # spongy wall
        [1.2425, 0.0] + _pole(0.5, 126e-9, 0.0) + none,             # cytoplasm
        [1.36 ** 2 - d1 - d2, sigma_chl] + _pole(d1, 430e-9, g1) + _pole(d2, 662e-9, g2),   # chloroplast
        [2.0559, 0.0] + _pole(0.8224, 330e-9, 0.7736) + none,      # hypha
    ]
    return np.array(rows, dtype=np.float64)


def model_nk(model: np.ndarray, lam: float) -> np.ndarray:
    """(n, k) per label of a Lorentz-Drude table at the wavelength lam: the
    monochromatic equivalent of the broadband material."""
    w = 2.0 * np.pi * _C0 / lam
    n_poles = (model.shape[1] - 2) // 3
    eps = model[:, 0] + 1j * model[:, 1] / (w * _EPS0)
    for p in range(n_poles):
        a, wp, g = model[:, 2 + 3 * p], model[:, 3 + 3 * p], model[:, 4 + 3 * p]
        eps = eps + a / (wp * wp - w * w - 1j * g * w)
    nk = np.sqrt(eps)
    return np.stack([nk.real, np.abs(nk.imag)], axis=1)
