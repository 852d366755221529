"""Closed forms used to pin the oracle (test code; independent of the oracle).

* Continuous slab transfer matrix (Fresnel + Fabry-Perot, e^{-i w t} convention,
  n~ = n + i k as in eqs. 1-2).
* Discrete transfer matrix: the exact time-harmonic steady state of the Yee
  recurrence (eqs. 18-20) for an x-invariant stack between semi-infinite
  vacuum.  A polarisation current adds (u - 1/u) Cb P/dt to the E update's
  left side, P = pchi E being its steady-state response.  With E^{n+1/2}_j = Re(E_j e^{-i w (n+1/2) dt}), H^n_j = Re(H_j e^{-i w n dt})
  and u = e^{-i w dt/2}, eliminating H gives
      E_{j+1} - (2 - q_j) E_j + E_{j-1} = 0,
      q_j = -(u - Ce_j/u)(u - 1/u) mu0 h^2 / (Cb_j dt).
  In vacuum q = 4 sin^2(w dt/2)/S1^2 and the outgoing waves are e^{-+i kappa j},
  sin(kappa/2) = sin(w dt/2)/S1.
* Full-column frequency-domain solve: the same steady state on the finite
  column, including the convolutional PML recursions (psi phasor
  = c dF/(h (1 - b e^{i w dt}))), the magnetic walls at both ends and the TF/SF
  line, solved as one banded linear system.
All formulas here are in SI units and take the per-row coefficients as inputs.
"""
from __future__ import annotations

import numpy as np

C0 = 299792458.0
MU0 = 1.25663706212e-6
EPS0 = 1.0 / (MU0 * C0 * C0)


def slab_rt(n: float, k: float, d: float, lam: float):
    """Continuous R, T of a slab of thickness d in vacuum at normal incidence."""
    nn = n + 1j * k
    k0 = 2 * np.pi / lam
    r12 = (1 - nn) / (1 + nn)
    t12 = 2 / (1 + nn)
    t21 = 2 * nn / (1 + nn)
    r21 = -r12
    ph = k0 * nn * d
    den = 1 - r21 ** 2 * np.exp(2j * ph)
    r = r12 + t12 * t21 * r21 * np.exp(2j * ph) / den
    t = t12 * t21 * np.exp(1j * ph) / den
    return abs(r) ** 2, abs(t) ** 2


def _q(ce, cb, h, dt, omega, pchi=0.0):
    """pchi: P/E of the polarisation update at this frequency (SI, eps0 chi),
    which enters the E update as -(P^{n+1/2} - P^{n-1/2})/dt."""
    u = np.exp(-1j * omega * dt / 2)
    return -((u - ce / u) + cb * (u - 1 / u) * pchi / dt) * (u - 1 / u) * MU0 * h * h / (cb * dt)


def discrete_stack_rt(ce_col, cb_col, h, dt, omega, pchi_col=None):
    """Exact steady-state R, T of the Yee recurrence for an x-invariant stack
    (rows given by ce_col, cb_col and optionally the polarisation response
    pchi_col; rows equal to vacuum are the exterior)."""
    ce_col = np.asarray(ce_col, float)
    cb_col = np.asarray(cb_col, float)
    pchi = 0.0 if pchi_col is None else np.asarray(pchi_col, complex)
    q = _q(ce_col, cb_col, h, dt, omega, pchi)
    qv = _q(1.0, dt / EPS0, h, dt, omega)
    kap = 2 * np.arcsin(np.sqrt(qv.real) / 2)
    idx = np.nonzero(np.abs(q - qv) > 1e-12 * abs(qv))[0]
    if len(idx) == 0:
        return 0.0, 1.0
    lo, hi = idx.min(), idx.max() + 1
    e_prev, e_cur = np.exp(-1j * kap * (lo - 1)), np.exp(-1j * kap * lo)
    for j in range(lo, hi):
        e_prev, e_cur = e_cur, (2 - q[j]) * e_cur - e_prev
    L = hi
    M = np.array([[np.exp(-1j * kap * (L - 1)), np.exp(1j * kap * (L - 1))],
                  [np.exp(-1j * kap * L), np.exp(1j * kap * L)]])
    A, B = np.linalg.solve(M, np.array([e_prev, e_cur]))
    return abs(B / A) ** 2, abs(1 / A) ** 2


def column_steady_state(ce_col, cb_col, prof_e, prof_h, h, dt, omega, j_src):
    """Steady-state phasors (E_j, H_j) of the whole finite column, with the
    absorbing layers given as per-row {b, c, 1/kappa} profiles (prof_e for Ez
    rows, prof_h for Hx edges) and a unit-amplitude incident wave injected on
    the TF/SF line below row j_src+1.  Returns E (ny,) complex."""
    from scipy.sparse import lil_matrix
    from scipy.sparse.linalg import spsolve

    ny = len(ce_col)
    u = np.exp(-1j * omega * dt / 2)
    d = u - 1 / u
    z1 = np.exp(1j * omega * dt)
    qv = _q(1.0, dt / EPS0, h, dt, omega)
    kap = 2 * np.arcsin(np.sqrt(qv.real) / 2)

    def S(prof, j):
        b, c, ik = prof[j]
        return ik + (c / (1 - b * z1) if c != 0.0 else 0.0)

    # unknowns: E_0..E_{ny-1}, then H_1..H_{ny-1}
    nE, nH = ny, ny - 1
    A = lil_matrix((nE + nH, nE + nH), dtype=complex)
    rhs = np.zeros(nE + nH, complex)
    hidx = lambda j: nE + j - 1
    for j in range(ny):
        A[j, j] = u - ce_col[j] / u
        s = S(prof_e, j) * cb_col[j] / h
        if j + 1 <= ny - 1:
            A[j, hidx(j + 1)] += s
        if j >= 1:
            A[j, hidx(j)] -= s
    for j in range(1, ny):
        r = hidx(j)
        A[r, r] = d
        s = S(prof_h, j) * dt / (MU0 * h)
        A[r, j] += s
        A[r, j - 1] -= s
    e_inc = np.exp(-1j * kap * j_src)
    h_inc = -(dt / (MU0 * h * d)) * (np.exp(-1j * kap * (j_src + 1)) - np.exp(-1j * kap * j_src))
    rhs[j_src] = -cb_col[j_src] / h * h_inc
    rhs[hidx(j_src + 1)] = -(dt / (MU0 * h)) * e_inc
    x = spsolve(A.tocsc(), rhs)
    return x[:nE]
