"""The staggered oracle against what the mathematics fixes (CPU only).

Operator: free-field closed forms of D and of M^+ M, anti-Hermiticity, the
mass term, gauge covariance, the norm bound, the even-odd structure and the
boundary-convention equivalence (tests/pins_staggered.py).  Solvers: dense
LU on small lattices, the free-field inverse in closed form, the per-shift
closed form and dense solves for the multi-shift CG, and edge cases.
"""

import math

import numpy as np
import pytest

import pins_staggered as PS
from lattice_inputs import gauge_field, site_coords, unit_gauge
from oracle import solvers as SV
from oracle import staggered as S


def test_operator_pins():
    errs = PS.all_stag_pins(S.hop, S.apply_M)
    bad = {k: v for k, v in errs.items() if v > 1e-12}
    assert not bad, bad


def test_eta_matches_definition():
    L = (4, 2, 6, 2)
    X = site_coords(L)
    e = S.eta_phases(L)
    assert np.array_equal(e[0], np.ones(X.shape[1]))
    assert np.array_equal(e[1], (-1.0) ** X[0])
    assert np.array_equal(e[2], (-1.0) ** (X[0] + X[1]))
    assert np.array_equal(e[3], (-1.0) ** (X[0] + X[1] + X[2]))


def test_eo_blocks_recombine():
    """D = D_eo + D_oe on the full lattice, and N = m^2 - D_eo D_oe equals
    the even block of M^+ M."""
    L, th, m = (4, 2, 2, 4), (0.0, 0.4, 0.0, math.pi), 0.3
    U = gauge_field(L, "haar", seed=3)
    phi = PS.colour_field(L, 4)
    full = S.hop(U, phi, L, th)
    assert np.allclose(S.hop_eo(U, phi, L, th, 0) + S.hop_eo(U, phi, L, th, 1), full, atol=1e-13)
    pe = S.mask(phi, L, 0)
    MtM = S.apply_M(U, S.apply_M(U, pe, L, th, m), L, th, m, dagger=True)
    assert np.allclose(S.normal_e(U, pe, L, th, m), S.mask(MtM, L, 0), atol=1e-13)
    assert np.allclose(S.mask(MtM, L, 1), 0, atol=1e-13)


@pytest.mark.parametrize("L,theta,mass", [((2, 4, 2, 2), (0.0, 0.0, 0.0, math.pi), 0.2),
                                          ((4, 2, 2, 4), (0.3, -0.7, 1.1, math.pi), 0.05)])
def test_eo_cg_matches_dense_lu(L, theta, mass):
    U = gauge_field(L, "haar", seed=17)
    b = PS.colour_field(L, 18)
    x, info = SV.stag_solve(U, b, L, theta, mass, 1e-12)
    assert info.status == SV.OK and info.true_resid <= 1e-12
    xd = np.linalg.solve(S.dense_M(U, L, theta, mass), b.ravel()).reshape(b.shape)
    M = S.dense_M(U, L, theta, mass)
    cond = np.linalg.cond(M)
    assert np.linalg.norm((x - xd).ravel()) / np.linalg.norm(xd.ravel()) <= 10 * cond * 1e-12


def test_free_field_inverse_closed_form():
    """U = 1, b = exp(i p.x) c: M^+ M is (m^2 + s^2) on b, so
    x = M^+ b / (m^2 + s^2) = (m - i sum eta_mu sin p_mu) b / (m^2 + s^2)."""
    L, th, m = (4, 6, 4, 8), (0.0, 0.0, 0.0, math.pi), 0.1
    c = np.array([1.0 + 0.5j, -0.3j, 0.7])
    b, p = PS.plane_wave(L, (1, 2, 0, 3), th, c)
    s2 = float(np.sum(np.sin(p) ** 2))
    f = m - 1j * np.tensordot(np.sin(p), PS.eta(L), axes=(0, 0))
    expect = f[:, None] * b / (m * m + s2)
    x, info = SV.stag_solve(unit_gauge(L), b, L, th, m, 1e-12)
    assert info.status == SV.OK
    assert np.linalg.norm((x - expect).ravel()) / np.linalg.norm(expect.ravel()) < 1e-10


def test_cg_zero_source_and_nonfinite():
    L, th = (2, 2, 2, 2), (0.0, 0.0, 0.0, math.pi)
    U = gauge_field(L, "haar", seed=1)
    x, info = SV.stag_solve(U, np.zeros((16, 3), complex), L, th, 0.1, 1e-10)
    assert info.status == SV.OK and not np.any(x)
    b = PS.colour_field(L, 2)
    b[3, 1] = np.nan
    A = lambda v: S.normal_e(U, v, L, th, 0.1)  # noqa: E731
    _, info = SV.cg(A, S.mask(b, L, 0) + 0 * b, 1e-10, 100)
    assert info.status == SV.ENONFINITE


def test_multishift_free_field_closed_form():
    """U = 1, b = P_e exp(i p.x) c: N b = (m^2 + s^2) b, so each shifted
    solution is b / (m^2 + s^2 + sigma)."""
    L, th, m = (4, 4, 6, 8), (0.0, 0.0, 0.0, math.pi), 0.08
    c = np.array([0.2 - 1j, 1.0, 0.4j])
    pw, p = PS.plane_wave(L, (1, 1, 2, 3), th, c)
    b = S.mask(pw, L, 0)
    s2 = float(np.sum(np.sin(p) ** 2))
    shifts = [0.0, 0.003, 0.05, 0.4, 2.0]
    A = lambda v: S.normal_e(unit_gauge(L), v, L, th, m)  # noqa: E731
    xs, out = SV.multishift_cg(A, b, shifts, 1e-12, 1000)
    for x, s, (it, res) in zip(xs, shifts, out):
        expect = b / (m * m + s2 + s)
        assert np.linalg.norm((x - expect).ravel()) / np.linalg.norm(expect.ravel()) < 1e-10
        assert res <= 1e-12


def _dense_normal(U, L, th, m):
    V = int(np.prod(L))
    even = np.flatnonzero(S.mask(np.ones((V, 3)), L, 0)[:, 0] != 0)
    idx = (even[:, None] * 3 + np.arange(3)[None, :]).ravel()
    n = idx.size
    N = np.empty((n, n), dtype=np.complex128)
    e = np.zeros((V, 3), dtype=np.complex128)
    for j, k in enumerate(idx):
        e.reshape(-1)[:] = 0
        e.reshape(-1)[k] = 1
        N[:, j] = S.normal_e(U, e, L, th, m).reshape(-1)[idx]
    return N, idx


def test_multishift_matches_dense_per_shift():
    L, th, m = (4, 4, 2, 2), (0.0, 0.6, 0.0, math.pi), 0.07
    U = gauge_field(L, "exp", eps=0.5, seed=27)
    b = S.mask(PS.colour_field(L, 28), L, 0)
    N, idx = _dense_normal(U, L, th, m)
    shifts = [0.5, 0.0, 0.02, 0.02, 0.11]  # unsorted, with a repeat
    A = lambda v: S.normal_e(U, v, L, th, m)  # noqa: E731
    xs, out = SV.multishift_cg(A, b, shifts, 1e-11, 2000)
    for x, s, (it, res) in zip(xs, shifts, out):
        xd = np.linalg.solve(N + s * np.eye(N.shape[0]), b.reshape(-1)[idx])
        cond = np.linalg.cond(N + s * np.eye(N.shape[0]))
        assert np.linalg.norm(x.reshape(-1)[idx] - xd) / np.linalg.norm(xd) <= 10 * cond * 1e-11
        assert res <= 1e-11
        assert np.all(x.reshape(-1)[np.setdiff1d(np.arange(x.size), idx)] == 0)
    # larger shifts converge no later than the base system
    its = [it for it, _ in out]
    assert its[1] == max(its)


def test_multishift_single_shift_equals_cg():
    L, th, m = (4, 2, 4, 2), (0.0, 0.0, 0.0, math.pi), 0.2
    U = gauge_field(L, "haar", seed=33)
    b = S.mask(PS.colour_field(L, 34), L, 0)
    A = lambda v: S.normal_e(U, v, L, th, m)  # noqa: E731
    xs, out = SV.multishift_cg(A, b, [0.0], 1e-12, 1000)
    x, info = SV.cg(A, b, 1e-12, 1000)
    assert out[0][0] == info.iters
    assert np.linalg.norm((xs[0] - x).ravel()) / np.linalg.norm(x.ravel()) < 1e-13
