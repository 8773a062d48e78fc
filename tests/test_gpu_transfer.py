"""The GPU driver's macro tangent B^T Abar B against the literal FE-HMM transfer
(eqs. k-mac-element-5..7): after GPU load steps, every macro element stiffness
built from the GPU's transferred tangents equals, to 1e-8, the oracle's T^T K T
from the micro responses to the element's unit nodal displacement states."""
import numpy as np
import pytest

import oracle
from paper_1908_08292_amd import fehmm, rve

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("bc", ["periodic", "kubc"])
def test_gpu_macro_tangent_against_literal_transfer(bc):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print(f"case literal transfer vs GPU Abar, 4x4 plate, RVE 8x8, {bc}", flush=True)
    n, r = 8, 0.25
    gbc = rve.BC_PERIODIC if bc == "periodic" else rve.BC_LINEAR
    obc = oracle.BC_PERIODIC if bc == "periodic" else oracle.BC_LINEAR
    mesh = rve.Mesh(2, n, rve.two_phase_lame(10.0), radius=r, bc=gbc)
    drv = fehmm.Driver(mesh, 4, 4, bc=fehmm.BC_CLAMPED_PULL, stretch=1.1, nsteps=10)
    with oracle.bc(obc):
        orc = oracle.Macro(4, 4, n, oracle.phase_by_centroid(2, n, r), oracle.two_phase_lame(10.0), bc=0,
                           stretch=1.1, nsteps=10)
        for k in (1, 2, 3):
            assert drv.step(k)["status"] == 0 and orc.step(k)["status"] == 0
        Fg, Pg, Ag = drv.qp()
        Fo, _, _ = orc.qp()
        assert Fg.shape == Fo.shape
        # same quadrature-point order on both sides
        assert np.abs(Fg - Fo).max() <= 1e-8
        lit = [orc.element_stiffness(e, literal=True) for e in range(orc.nelem())]
        orc.set_qp(A=Ag)
        for e in range(orc.nelem()):
            kc = orc.element_stiffness(e, literal=False)  # from the GPU's Abar
            assert np.abs(kc - lit[e]).max() <= 1e-8 * np.abs(lit[e]).max(), e
    drv.destroy()
    orc.close()
