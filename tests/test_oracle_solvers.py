"""The oracle's solvers against a dense LU solve (2^4 lattice) and against
the free-field closed-form inverse of M on a larger lattice."""

import numpy as np
import pytest

import pins
from lattice_inputs import gauge_field, gaussian_spinor, unit_gauge
from oracle import solvers as S
from oracle import wilson as W


@pytest.mark.parametrize("method", ["cgnr", "bicgstab", "bicgstab_l"])
@pytest.mark.parametrize("eo", [True, False])
@pytest.mark.parametrize("mu", [0.0, 0.05])
def test_dense_lu_2x2x2x2(method, eo, mu):
    L, th, kappa = (2, 2, 2, 2), (0, 0, 0, np.pi), 0.12
    U = gauge_field(L, "haar", seed=1000)
    b = gaussian_spinor(L, seed=2000)
    M = W.dense_M(U, L, th, kappa, mu)
    x_ref = np.linalg.solve(M, b.ravel()).reshape(b.shape)
    x, info = S.solve(U, b, L, th, kappa, mu, tol=1e-13, method=method, eo=eo)
    assert info.status == S.OK
    assert info.true_resid <= 1e-13
    assert np.linalg.norm((x - x_ref).ravel()) / np.linalg.norm(x_ref.ravel()) < 1e-11


def test_dense_matches_operator_4x2x2x2_twisted():
    L, th, kappa, mu = (4, 2, 2, 2), (0.2, 0, 0, np.pi), 0.16, 0.005
    U = gauge_field(L, "exp", eps=0.4, seed=1001)
    b = gaussian_spinor(L, seed=2001)
    M = W.dense_M(U, L, th, kappa, mu)
    x_ref = np.linalg.solve(M, b.ravel()).reshape(b.shape)
    x, info = S.solve(U, b, L, th, kappa, mu, tol=1e-12, method="cgnr", eo=True)
    cond = np.linalg.cond(M)
    err = np.linalg.norm((x - x_ref).ravel()) / np.linalg.norm(x_ref.ravel())
    assert info.true_resid <= 1e-12
    assert err <= cond * 1e-12


@pytest.mark.parametrize("method", ["cgnr", "bicgstab", "bicgstab_l"])
def test_free_field_inverse(method):
    """U = 1, b = exp(ipx) u: x = exp(ipx) M(p)^-1 u with
    M(p)^-1 = (a - i b.gamma - i c gamma_5) / (a^2 + b.b + c^2)."""
    L, th, kappa, mu = (6, 4, 4, 8), (0, 0, 0, np.pi), 0.12, 0.05
    n = (1, 0, 1, 2)
    rng = np.random.default_rng(3)
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    b, p = pins.plane_wave(L, n, th, u)
    g = pins.chiral_gammas()
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    a = 1 - 2 * kappa * np.cos(p).sum()
    bv = 2 * kappa * np.sin(p)
    c = 2 * kappa * mu
    Minv = (a * np.eye(4) - 1j * sum(bv[m] * g[m] for m in range(4)) - 1j * c * g5) / (a * a + bv @ bv + c * c)
    x_ref, _ = pins.plane_wave(L, n, th, Minv @ u)
    x, info = S.solve(unit_gauge(L), b, L, th, kappa, mu, tol=1e-12, method=method, eo=True)
    assert info.status == S.OK and info.true_resid <= 1e-12
    assert np.linalg.norm((x - x_ref).ravel()) / np.linalg.norm(x_ref.ravel()) < 1e-10


def test_zero_source_and_nonfinite():
    L, th = (2, 2, 2, 2), (0, 0, 0, np.pi)
    U = unit_gauge(L)
    b = np.zeros((16, 4, 3), complex)
    x, info = S.solve(U, b, L, th, 0.1, 0.0, tol=1e-10)
    assert info.iters == 0 and not x.any()
    b[3, 1, 2] = np.nan
    _, info = S.solve(U, b, L, th, 0.1, 0.0, tol=1e-10, eo=False)
    assert info.status == S.ENONFINITE


def test_maxiter_reports_noconv():
    L, th = (4, 4, 4, 4), (0, 0, 0, np.pi)
    U = gauge_field(L, "haar", seed=1000)
    b = gaussian_spinor(L, seed=2000)
    x, info = S.solve(U, b, L, th, 0.12, 0.0, tol=1e-12, maxiter=3)
    assert info.status == S.ENOCONV and info.iters == 3
    assert 0 < info.true_resid < 1


@pytest.mark.parametrize("kappa,mu,kind,steps", [(0.12, 0.05, "haar", (1, 2, 3, 7, 12, 20)),
                                                  (0.16, 0.005, "exp", (1, 2, 3))])
def test_bicgstab_l_of_degree_one_is_bicgstab(kappa, mu, kind, steps):
    """BiCGStab(1) is BiCGStab: after the same number of steps (no stop) the
    iterates agree to rounding on twisted-mass Schur complements.  (On the
    kappa = 0.16 system BiCGStab's residual oscillates, which amplifies
    rounding differences after a few steps, so only the first are compared.)"""
    L, th = (4, 4, 4, 4), (0, 0, 0, np.pi)
    U = gauge_field(L, kind, eps=0.4, seed=1001)
    b = gaussian_spinor(L, seed=2001)
    bhat = W.eo_source(U, b, L, th, kappa, mu)
    A = lambda v: W.schur(U, v, L, th, kappa, mu)  # noqa: E731
    for k in steps:
        x1, i1 = S.bicgstab(A, bhat, 1e-30, k)
        xl, il = S.bicgstab_l(A, bhat, 1e-30, k, ell=1)
        assert i1.status == il.status == S.ENOCONV and i1.iters == il.iters == k
        assert np.linalg.norm((x1 - xl).ravel()) <= 1e-13 * np.linalg.norm(x1.ravel()), k


@pytest.mark.parametrize("ell", [2, 4])
def test_bicgstab_l_dense_and_minimal_residual(ell):
    """BiCGStab(2) and (4) on 2^4 against a dense LU solve (twisted
    boundaries, twisted mass)."""
    L, th, kappa, mu = (2, 2, 2, 2), (0.3, 0, 0, np.pi), 0.12, 0.05
    U = gauge_field(L, "haar", seed=1002)
    b = gaussian_spinor(L, seed=2002)
    M = W.dense_M(U, L, th, kappa, mu)
    x_ref = np.linalg.solve(M, b.ravel()).reshape(b.shape)
    x, info = S.solve(U, b, L, th, kappa, mu, tol=1e-13, method="bicgstab_l", eo=True, ell=ell)
    assert info.status == S.OK and info.true_resid <= 1e-13
    assert np.linalg.norm((x - x_ref).ravel()) / np.linalg.norm(x_ref.ravel()) < 1e-11


def test_bicgstab_l_converges_where_bicgstab_needs_more():
    """On the 8^3 x 4 twisted-mass Schur complement at kappa = 0.16 (the
    spectrum has eigenvalue pairs left of the imaginary axis) BiCGStab(2)
    reaches 1e-10 in fewer steps than BiCGStab, and both agree with CGNR's
    solution within cond * tol."""
    L, th, kappa, mu = (8, 8, 8, 4), (0, 0, 0, np.pi), 0.16, 0.005
    U = gauge_field(L, "exp", eps=0.4, seed=1001)
    b = gaussian_spinor(L, seed=2001)
    xc, ic = S.solve(U, b, L, th, kappa, mu, tol=1e-10, method="cgnr")
    x2, i2 = S.solve(U, b, L, th, kappa, mu, tol=1e-10, method="bicgstab_l", ell=2)
    x1, i1 = S.solve(U, b, L, th, kappa, mu, tol=1e-10, method="bicgstab")
    assert ic.status == i2.status == i1.status == S.OK
    assert i2.true_resid <= 1e-10 and i2.iters < i1.iters
    for x in (x1, x2):
        assert np.linalg.norm((x - xc).ravel()) / np.linalg.norm(xc.ravel()) < 1e-6
