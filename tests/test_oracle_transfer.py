"""Pins of the literal FE-HMM stiffness transfer (eqs. k-mac-element-5..7 with
the linear constrained problem of eq. Lagrange-Functional-for-StiffnessTransfer):
the macro element stiffness built from the micro responses to the element's
N_node x d unit nodal displacement states, T^T K T / |K_delta| summed over the
Gauss points, against B^T Abar B from the condensed tangent -- two routes the
paper's transfer and its FE^2 form take to the same matrix."""
import numpy as np
import pytest

import oracle

LAME = oracle.two_phase_lame(10.0)


@pytest.mark.parametrize("bc", [oracle.BC_PERIODIC, oracle.BC_LINEAR])
@pytest.mark.parametrize("scheme", [0, 1])
def test_literal_transfer_equals_condensed_tangent(bc, scheme):
    n = 4
    with oracle.bc(bc):
        m = oracle.Macro(3, 3, n, oracle.phase_by_centroid(2, n, 0.3), LAME, bc=0, stretch=1.1, nsteps=2,
                         scheme=scheme)
        for k in (1, 2):
            assert m.step(k)["status"] == 0
        for e in range(m.nelem()):
            kl = m.element_stiffness(e, literal=True)
            kc = m.element_stiffness(e, literal=False)
            assert np.abs(kl - kc).max() <= 1e-11 * np.abs(kc).max()
            assert np.abs(kl - kl.T).max() <= 1e-12 * np.abs(kl).max()
            # macro rigid translations carry no energy
            for i in range(2):
                t = np.zeros(8); t[i::2] = 1.0
                assert np.abs(kl @ t).max() <= 1e-11 * np.abs(kl).max()
        m.close()


def test_unit_gradient_states_give_the_tangent_and_translations_no_energy():
    d, n = 2, 6
    ph = oracle.phase_by_centroid(d, n, 0.25)
    F = np.array([[1.06, 0.03], [-0.02, 0.95]])
    r = oracle.rve_solve(d, n, ph, LAME, F, w=np.zeros(d * n * n))
    G = np.eye(d * d).reshape(d * d, d, d)
    st, kT = oracle.transfer_states(d, n, ph, LAME, F, r["w"], G)
    assert st == 0
    assert np.abs(kT - r["A"]).max() <= 1e-11 * np.abs(r["A"]).max()
    t = np.array([[1.0, 0.0], [0.0, 1.0], [0.7, -0.2]])
    st, k0 = oracle.transfer_states(d, n, ph, LAME, F, r["w"], np.zeros((3, d, d)), t)
    assert st == 0 and np.abs(k0).max() <= 1e-12 * np.abs(r["A"]).max()
