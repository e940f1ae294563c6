"""The oracle's hopping term and fermion matrix against closed forms and
exact identities (free field, gamma_5-hermiticity, adjointness, gauge
covariance, norm bound, boundary-phase convention, twisted-mass normal
equation)."""

import numpy as np
import pytest

import pins
from oracle import wilson as W


def test_gammas_follow_chiral_basis():
    g, g5 = W.gammas()
    ref = pins.chiral_gammas()
    assert np.array_equal(g, ref)
    for m in range(4):
        assert np.allclose(g[m], g[m].conj().T)
        for n in range(4):
            assert np.allclose(g[m] @ g[n] + g[n] @ g[m], 2 * np.eye(4) * (m == n))
    assert np.allclose(g5, np.diag([1, 1, -1, -1]))


@pytest.mark.parametrize("name,err", sorted(pins.all_pins(
    lambda U, p, L, th, d: W.hop(U, p, L, th, d),
    lambda U, p, L, th, k, m, d: W.apply_M(U, p, L, th, k, m, d)).items()))
def test_operator_pin(name, err):
    assert err < 1e-12, (name, err)


def test_free_field_noncubic_sizes():
    for L in [(4, 6, 8, 2), (6, 4, 4, 8), (2, 2, 2, 2)]:
        for th in [(0, 0, 0, np.pi), (0.5, 0.0, 1.5, np.pi + 0.3)]:
            e = pins.free_field_closed_form(W.apply_M, L, th, 0.12, 0.005, (1, 1, 0, 1))
            assert e < 1e-13, (L, th, e)


def test_schur_blocks_recombine():
    """M x = b for x built from the Schur pieces: solve the even system
    densely on 2x2x2x2, reconstruct the odd sites, check the full residual."""
    L, th, kappa, mu = (2, 2, 2, 2), (0, 0, 0, np.pi), 0.15, 0.1
    from lattice_inputs import gauge_field, gaussian_spinor
    U = gauge_field(L, "haar", seed=5)
    b = gaussian_spinor(L, seed=6)
    even = W.parity(L) == 0
    n = int(even.sum()) * 12
    cols = []
    for j in range(n):
        e = np.zeros((int(np.prod(L)), 4, 3), complex)
        e[even] = np.eye(n)[j].reshape(-1, 4, 3)
        cols.append(W.schur(U, e, L, th, kappa, mu)[even].ravel())
    Mhat = np.array(cols).T
    bhat = W.eo_source(U, b, L, th, kappa, mu)
    xe = np.zeros_like(b)
    xe[even] = np.linalg.solve(Mhat, bhat[even].ravel()).reshape(-1, 4, 3)
    x = W.eo_reconstruct(U, xe, b, L, th, kappa, mu)
    assert W.true_residual(U, x, b, L, th, kappa, mu) < 1e-13
