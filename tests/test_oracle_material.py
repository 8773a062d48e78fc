"""Pins of the oracle's constitutive law (neo-Hookean, Sec. 6) and Lame table."""
import json
import os

import numpy as np
import pytest

import oracle
from tests import fe_ref

HERE = os.path.dirname(__file__)


def rand_F(rng, d, amp=0.3):
    while True:
        F = np.eye(d) + rng.uniform(-amp, amp, (d, d))
        if np.linalg.det(F) > 0.3:
            return F


def test_lame_table_matches_paper():
    tab = json.load(open(os.path.join(HERE, "golden", "lame_table.json")))
    for row in tab["rows"]:
        lam, mu = oracle.lame(row["E"], row["nu"])
        assert round(lam, 2) == pytest.approx(row["lambda"], abs=1e-9)
        assert round(mu, 2) == pytest.approx(row["mu"], abs=1e-9)


@pytest.mark.parametrize("d", [2, 3])
def test_reference_state(d):
    lam, mu = 1.3, 0.7
    st, S, Cm, psi = oracle.nh_sc(d, lam, mu, np.eye(d))
    assert st == 0
    assert abs(psi) < 1e-15 and np.abs(S).max() < 1e-15
    I = np.eye(d)
    C_lin = lam * np.einsum("IJ,KL->IJKL", I, I) + mu * (np.einsum("IK,JL->IJKL", I, I) + np.einsum("IL,JK->IJKL", I, I))
    assert np.abs(Cm - C_lin).max() < 1e-14


@pytest.mark.parametrize("d", [2, 3])
def test_S_and_C_are_derivatives_of_psi(d):
    """S = 2 dpsi/dC and C = 4 d^2psi/dCdC (the definitions of Sec. 6), by central
    differences of psi along symmetric perturbations of C (through F = U)."""
    rng = np.random.default_rng(1)
    lam, mu = 0.8, 0.45
    for _ in range(5):
        F = rand_F(rng, d)
        Cc = F.T @ F
        def psi_of_C(Cq):
            # any F with F^T F = Cq: take the symmetric square root
            ev, V = np.linalg.eigh(Cq)
            U = V @ np.diag(np.sqrt(ev)) @ V.T
            return oracle.nh_sc(d, lam, mu, U)[3]
        st, S, Cm, _ = oracle.nh_sc(d, lam, mu, F)
        h = 1e-6
        for I in range(d):
            for J in range(I, d):
                E = np.zeros((d, d)); E[I, J] = E[J, I] = 1.0
                dpsi = (psi_of_C(Cc + h * E) - psi_of_C(Cc - h * E)) / (2 * h)
                # dpsi along symmetric direction E = S : E / 2
                assert dpsi == pytest.approx(0.5 * np.sum(S * E), rel=1e-7, abs=1e-9)
        h = 1e-4
        for I in range(d):
            for J in range(I, d):
                E1 = np.zeros((d, d)); E1[I, J] = E1[J, I] = 1.0
                Sp = oracle.nh_sc(d, lam, mu, _sqrt_spd(Cc + h * E1))[1]
                Sm = oracle.nh_sc(d, lam, mu, _sqrt_spd(Cc - h * E1))[1]
                dS = (Sp - Sm) / (2 * h)
                # dS = C : (dC/2)
                pred = 0.5 * np.einsum("IJKL,KL->IJ", Cm, E1)
                assert np.abs(dS - pred).max() < 1e-7 * max(1.0, np.abs(pred).max())


def _sqrt_spd(C):
    ev, V = np.linalg.eigh(C)
    return V @ np.diag(np.sqrt(ev)) @ V.T


@pytest.mark.parametrize("d", [2, 3])
def test_first_piola_matches_hand_derived_closed_form(d):
    """P = F S from the oracle equals the hand-derived dpsi/dF; the material
    tangent pushed to A_iJkL = d_ik S_JL + F_iM C_MJNL F_kN equals d^2psi/dF^2."""
    rng = np.random.default_rng(2)
    lam, mu = 2.0, 0.6
    for _ in range(10):
        F = rand_F(rng, d)
        st, S, Cm, psi = oracle.nh_sc(d, lam, mu, F)
        assert psi == pytest.approx(float(fe_ref.psi(F, lam, mu)), rel=1e-13, abs=1e-15)
        assert np.abs(F @ S - fe_ref.P_closed(F, lam, mu)).max() < 1e-13
        A = np.einsum("ik,JL->iJkL", np.eye(d), S) + np.einsum("iM,MJNL,kN->iJkL", F, Cm, F)
        assert np.abs(A.reshape(d * d, d * d) - fe_ref.A_closed(F, lam, mu)).max() < 1e-12


def test_plane_strain_is_3d_law_with_unit_stretch():
    """2D reading (plane strain): the in-plane S and C equal those of the 3D law
    at F = diag(F_2D, 1)."""
    rng = np.random.default_rng(3)
    for _ in range(5):
        F2 = rand_F(rng, 2)
        F3 = np.eye(3); F3[:2, :2] = F2
        _, S2, C2, psi2 = oracle.nh_sc(2, 1.1, 0.4, F2)
        _, S3, C3, psi3 = oracle.nh_sc(3, 1.1, 0.4, F3)
        assert np.abs(S2 - S3[:2, :2]).max() < 1e-14
        assert np.abs(C2 - C3[:2, :2, :2, :2]).max() < 1e-13
        assert psi2 == pytest.approx(psi3, rel=1e-14, abs=1e-15)


def test_detF_guard():
    st, *_ = oracle.nh_sc(2, 1.0, 1.0, np.array([[1.0, 0.0], [0.0, -0.5]]))
    assert st == oracle.DETF
