"""Physical properties of whole synthetic-leaf runs on the GPU, where no
closed form exists: reflectance and transmittance are non-negative, energy is
not created (R + T <= 1 up to the steady-state error of the window), a
nearly transparent leaf in the near infrared (k ~ 1e-5) absorbs almost
nothing, and the same leaf absorbs strongly at the chlorophyll peak."""
import numpy as np
import pytest

import leafgen as LG

pytestmark = pytest.mark.gpu


def _run(fdtd, inst, steps):
    with fdtd.Simulation([inst], fdtd.Options(n_steps=steps)) as s:
        s.run()
        R, T, A = s.spectra()
    return R[0], T[0], A[0]


def test_monocot_leaf_spectra_are_physical(gpu_lib):
    """R, T >= 0 and R + T <= 1 (up to the window's steady-state error) at a
    near-infrared and a chlorophyll-band wavelength; the chlorophyll band
    absorbs strongly and several times more than the near infrared, where the
    only loss is k ~ 1e-5 in the chloroplasts.  (The near-infrared run is not
    converged to A ~ 0 in 30000 steps: near-grazing Bloch orders of this wide
    lossless structure leave the domain slowly.)"""
    base = LG.configs.monocot_config(512, 1024, 30000)[0]
    out = {}
    for lam_nm in (850, 430):
        inst = LG.configs.Instance(base.labels, LG.materials.monocot_nk(lam_nm * 1e-9), base.dx, lam_nm * 1e-9,
                                   base.n_pml, 30000, name="monocot_%dnm" % lam_nm)
        R, T, A = _run(gpu_lib, inst, inst.n_steps)
        print(lam_nm, "nm: R %.5f T %.5f A %.5f" % (R, T, A))
        assert R >= 0 and T >= 0
        assert R + T <= 1 + 2e-3
        out[lam_nm] = A
    assert out[430] > 0.05
    assert out[430] > 3 * out[850]
