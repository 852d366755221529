"""Shared helpers of the GPU parity tests: run the oracle on a leafgen
instance, run the HIP library on the same instance, compare."""
import numpy as np

import oracle as O


def problem_for(inst, n_steps=None, dft_start=-1, literal=0):
    return O.Problem(nx=inst.nx, ny=inst.ny, h=inst.dx, lambda0=inst.lambda0,
                     n_steps=n_steps or inst.n_steps, n_pml=inst.n_pml, j_src=inst.j_src,
                     j_ref=inst.j_ref, j_trn=inst.j_trn, courant=inst.courant,
                     dft_start=dft_start, ramp_periods=inst.ramp_periods, literal_orders=literal)


def oracle_run(inst, n_steps=None, literal=0):
    prob = problem_for(inst, n_steps, literal=literal)
    return prob, O.simulate(prob, inst.labels, inst.nk)


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a - b))


def oracle_fields_normalised(res):
    """Oracle fields in the library's units (H~ = eta0 H)."""
    st = res["state"]
    return st.ez, st.hx * O.ETA0, st.hy * O.ETA0
