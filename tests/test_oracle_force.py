"""The oracle's twisted-mass pseudo-fermion force against its definition (CPU only).

F_mu(y) = sum_a (dS_f / dw^a) T^a for S_f = || M^-1 phi ||^2 and the link
rotation U_mu(y) -> exp(i w T^a) U_mu(y): the closed form in oracle/force.py
is checked against central finite differences of S_f computed with dense
solves, on links in the bulk and links that cross twisted boundaries, and
for its algebraic properties (Hermitian, traceless, gauge covariant).
"""

import math

import numpy as np
import pytest

from lattice_inputs import gauge_field, gauge_transform, gaussian_spinor
from oracle import force as F

L4 = (4, 2, 2, 2)
THETA = (0.3, 0.0, 0.7, math.pi)
KAPPA, MU = 0.13, 0.2


@pytest.fixture(scope="module")
def case():
    U = gauge_field(L4, "haar", seed=5)
    phi = gaussian_spinor(L4, seed=6)
    X, Z = F.solve_pair(U, phi, L4, THETA, KAPPA, MU)
    return U, phi, F.force(U, X, Z, L4, THETA, KAPPA)


# (mu, site, generator): bulk links and links across the x, z and t boundaries
LINKS = [(0, 0, 0), (0, 3, 2), (1, 1, 1), (2, 5, 7), (2, 9, 4), (3, 7, 4), (3, 12, 5), (3, 15, 3), (1, 14, 6)]


@pytest.mark.parametrize("lmu,y,a", LINKS)
def test_force_matches_finite_differences(case, lmu, y, a):
    U, phi, Fa = case
    T = F.gellmann_generators()
    fd = F.force_fd(U, phi, L4, THETA, KAPPA, MU, lmu, y, a)
    an = 2.0 * np.trace(T[a] @ Fa[lmu, y]).real  # F = sum_a f_a T^a, tr(T^a T^b) = delta_ab / 2
    assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


def test_force_is_hermitian_traceless(case):
    _, _, Fa = case
    assert np.allclose(Fa, np.conj(np.swapaxes(Fa, -1, -2)), atol=1e-15)
    assert np.allclose(np.trace(Fa, axis1=-2, axis2=-1), 0, atol=1e-15)


def test_force_gauge_covariant(case):
    """U'_mu(y) = G(y) U_mu(y) G(y+mu)^+, phi' = G phi  =>  F'_mu(y) = G(y) F_mu(y) G(y)^+."""
    U, phi, Fa = case
    G = gauge_transform(L4, seed=7)
    Up = np.empty_like(U)
    for mu in range(4):
        Up[mu] = G @ U[mu] @ np.conj(np.swapaxes(G[F._neighbour(L4, mu, +1)], 1, 2))
    phip = np.einsum("vab,vsb->vsa", G, phi)
    X, Z = F.solve_pair(Up, phip, L4, THETA, KAPPA, MU)
    Fp = F.force(Up, X, Z, L4, THETA, KAPPA)
    expect = G[None] @ Fa @ np.conj(np.swapaxes(G, 1, 2))[None]
    assert np.allclose(Fp, expect, atol=1e-12)


def test_generators():
    T = F.gellmann_generators()
    for a in range(8):
        assert np.allclose(T[a], T[a].conj().T) and abs(np.trace(T[a])) < 1e-15
        for b in range(8):
            assert abs(np.trace(T[a] @ T[b]) - 0.5 * (a == b)) < 1e-15
