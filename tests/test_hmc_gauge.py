"""The host gauge part of the twisted-mass molecular dynamics (CPU only).

The Wilson plaquette force must be the derivative of the plaquette action
along U_mu(y) -> exp(i w T^a) U_mu(y) (central finite differences), and the
link update exp(i dt P) must stay in SU(3).
"""

import math

import numpy as np
import pytest

from lattice_inputs import gauge_field
from oracle import force as OF

hmc = pytest.importorskip("paper_1411_5219_amd.hmc")

L4 = (4, 2, 2, 2)
BETA = 5.6


@pytest.fixture(scope="module")
def case():
    U = gauge_field(L4, "haar", seed=51)
    return U, hmc.plaquette_force(U, L4, BETA)


@pytest.mark.parametrize("lmu,y,a", [(0, 0, 0), (1, 5, 3), (2, 9, 7), (3, 15, 2), (3, 6, 5)])
def test_plaquette_force_finite_differences(case, lmu, y, a):
    U, Fg = case
    T = OF.gellmann_generators()

    def S(w):
        return hmc.plaquette_action(OF.rotate_link(U, lmu, y, a, w), L4, BETA)

    h = 1e-4
    fd = (8 * (S(h) - S(-h)) - (S(2 * h) - S(-2 * h))) / (12 * h)
    an = 2.0 * np.trace(T[a] @ Fg[lmu, y]).real
    assert abs(fd - an) <= 1e-8 * max(1.0, abs(an)), (fd, an)


def test_plaquette_force_hermitian_traceless(case):
    _, Fg = case
    assert np.allclose(Fg, np.conj(np.swapaxes(Fg, -1, -2)), atol=1e-14)
    assert np.allclose(np.trace(Fg, axis1=-2, axis2=-1), 0, atol=1e-14)


def test_unit_links_action_and_force_vanish():
    U = gauge_field(L4, "unit")
    assert hmc.plaquette_action(U, L4, BETA) == 0.0
    assert np.max(np.abs(hmc.plaquette_force(U, L4, BETA))) == 0.0


def test_link_update_stays_su3():
    U = gauge_field(L4, "haar", seed=52)
    P = hmc.gaussian_momenta(L4, np.random.default_rng(53))
    assert np.allclose(P, np.conj(np.swapaxes(P, -1, -2)))
    assert np.allclose(np.trace(P, axis1=-2, axis2=-1), 0)
    U1 = hmc.expi(P, 0.3) @ U
    eye = np.eye(3)
    assert np.allclose(U1 @ np.conj(np.swapaxes(U1, -1, -2)), eye, atol=1e-13)
    assert np.allclose(np.linalg.det(U1), 1.0, atol=1e-13)


def test_momentum_heatbath_normalisation():
    """<tr P^2> = 8 / 2 per link for P = sum_a p_a T^a, p_a ~ N(0, 1)."""
    P = hmc.gaussian_momenta((8, 8, 8, 8), np.random.default_rng(54))
    k = np.trace(P @ P, axis1=-2, axis2=-1).real.mean()
    assert abs(k - 4.0) < 0.05
