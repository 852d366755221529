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
