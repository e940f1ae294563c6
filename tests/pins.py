"""Checks that pin the oracle's operator to facts fixed by the mathematics.

Each check takes the operator under test as callables

    hop(U, psi, L, theta, dagger) -> H psi or H^+ psi
    apply_M(U, psi, L, theta, kappa, mu, dagger) -> M psi or M^+ psi

and returns a relative error that must be at rounding level.  The same
checks run against the real oracle (tests/test_oracle_pins.py) and against
copies of it with planted mistakes (tests/test_oracle_mutants.py), which
shows that each plausible mistake is caught by at least one of them.

Nothing here computes the operator itself, except the free-field closed
form (plane waves diagonalise the hopping term when all links are 1).
"""

from __future__ import annotations

import numpy as np

from lattice_inputs import gauge_field, gauge_transform, gaussian_spinor, site_coords, unit_gauge


def chiral_gammas():
    """Chiral basis from its definition: gamma_k = [[0, -i s_k], [i s_k, 0]],
    gamma_4 = [[0, 1], [1, 0]], built from the Pauli matrices."""
    s = [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]]),
         np.array([[1, 0], [0, -1]], complex)]
    z = np.zeros((2, 2), complex)
    one = np.eye(2, dtype=complex)
    g = [np.block([[z, -1j * sk], [1j * sk, z]]) for sk in s]
    g.append(np.block([[z, one], [one, z]]))
    return np.array(g)


def _rel(a, b):
    den = max(np.linalg.norm(b.ravel()), 1e-300)
    return float(np.linalg.norm((a - b).ravel()) / den)


def _inner(a, b):
    return complex(np.vdot(a.ravel(), b.ravel()))


def plane_wave(L, n, theta, u):
    """psi(x) = exp(i p.x) u with p_mu = (2 pi n_mu + theta_mu) / L_mu, which
    obeys psi(x + L_mu mu-hat) = exp(i theta_mu) psi(x)."""
    X = site_coords(L)
    p = np.array([(2 * np.pi * n[m] + theta[m]) / L[m] for m in range(4)])
    phase = np.exp(1j * np.tensordot(p, X, axes=(0, 0)))
    return phase[:, None, None] * u[None, :, :], p


def free_field_closed_form(apply_M, L, theta, kappa, mu, n, seed=7, dagger=False):
    """U = 1: M(p) = 1 - 2 kappa sum cos p + 2 i kappa sum gamma sin p
    + 2 i kappa mu gamma_5 acting on the constant spinor u; for M^+ the
    sin and mu terms change sign."""
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    psi, p = plane_wave(L, n, theta, u)
    g = chiral_gammas()
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    sgn = -1.0 if dagger else 1.0
    Mp = (1 - 2 * kappa * np.cos(p).sum()) * np.eye(4) \
        + sgn * 2j * kappa * sum(g[m] * np.sin(p[m]) for m in range(4)) \
        + sgn * 2j * kappa * mu * g5
    expect, _ = plane_wave(L, n, theta, Mp @ u)
    got = apply_M(unit_gauge(L), psi, L, theta, kappa, mu, dagger)
    return _rel(got, expect)


def gamma5_hermiticity(hop, apply_M, L, theta, kappa, mu, seed=11):
    """<chi, H psi> = <g5 H g5 chi, psi> and M(mu)^+ = g5 M(-mu) g5."""
    U = gauge_field(L, "haar", seed=seed)
    psi = gaussian_spinor(L, seed=seed + 1)
    chi = gaussian_spinor(L, seed=seed + 2)
    g = chiral_gammas()
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    G5 = lambda v: np.einsum("ab,vbc->vac", g5, v)  # noqa: E731
    lhs = _inner(chi, hop(U, psi, L, theta, False))
    rhs = _inner(G5(hop(U, G5(chi), L, theta, False)), psi)
    e1 = abs(lhs - rhs) / abs(lhs)
    lhs = _inner(chi, apply_M(U, psi, L, theta, kappa, mu, False))
    rhs = _inner(G5(apply_M(U, G5(chi), L, theta, kappa, -mu, False)), psi)
    e2 = abs(lhs - rhs) / abs(lhs)
    return max(e1, e2)


def adjoint_consistency(hop, apply_M, L, theta, kappa, mu, seed=21):
    """The dagger kernels are the adjoints: <chi, H psi> = <H^+ chi, psi>
    and <chi, M psi> = <M^+ chi, psi>."""
    U = gauge_field(L, "haar", seed=seed)
    psi = gaussian_spinor(L, seed=seed + 1)
    chi = gaussian_spinor(L, seed=seed + 2)
    a = _inner(chi, hop(U, psi, L, theta, False))
    b = _inner(hop(U, chi, L, theta, True), psi)
    c = _inner(chi, apply_M(U, psi, L, theta, kappa, mu, False))
    d = _inner(apply_M(U, chi, L, theta, kappa, mu, True), psi)
    return max(abs(a - b) / abs(a), abs(c - d) / abs(c))


def _shift_index(L, mu, step):
    X = site_coords(L)
    X[mu] = (X[mu] + step) % L[mu]
    return X[0] + L[0] * (X[1] + L[1] * (X[2] + L[2] * X[3]))


def gauge_covariance(hop, L, theta, seed=31, dagger=False):
    """U'_mu(x) = G(x) U_mu(x) G(x+mu)^+, psi' = G psi  =>  H' psi' = G H psi."""
    U = gauge_field(L, "haar", seed=seed)
    psi = gaussian_spinor(L, seed=seed + 1)
    G = gauge_transform(L, seed=seed + 2)
    Up = np.empty_like(U)
    for mu in range(4):
        fwd = _shift_index(L, mu, +1)
        Up[mu] = G @ U[mu] @ np.conj(np.swapaxes(G[fwd], 1, 2))
    psip = np.einsum("vab,vsb->vsa", G, psi)
    lhs = hop(Up, psip, L, theta, dagger)
    rhs = np.einsum("vab,vsb->vsa", G, hop(U, psi, L, theta, dagger))
    return _rel(lhs, rhs)


def norm_bound(hop, L, theta, seed=41):
    """Each direction contributes (1 -+ gamma) times a unitary hop, and
    (1 -+ gamma)/2 are orthogonal projectors, so ||H psi|| <= 8 ||psi||;
    with U = 1, theta = 0 and a constant spinor the bound is attained."""
    U = gauge_field(L, "haar", seed=seed)
    psi = gaussian_spinor(L, seed=seed + 1)
    ratio = np.linalg.norm(hop(U, psi, L, theta, False).ravel()) / np.linalg.norm(psi.ravel())
    const = np.broadcast_to(gaussian_spinor((1, 1, 1, 1), seed=seed + 2), psi.shape).copy()
    sat = _rel(hop(unit_gauge(L), const, L, (0, 0, 0, 0), False), 8 * const)
    return ratio, sat


def boundary_convention_equivalence(hop, L, theta, seed=51):
    """Boundary phases applied only on hops that cross the boundary equal
    phases spread as exp(i theta_mu / L_mu) on every link (periodic BC),
    conjugated by psi(x) -> exp(i sum theta_mu x_mu / L_mu) psi(x)."""
    U = gauge_field(L, "haar", seed=seed)
    psi = gaussian_spinor(L, seed=seed + 1)
    X = site_coords(L)
    w = sum(theta[m] * X[m] / L[m] for m in range(4))
    T = np.exp(1j * w)[:, None, None]
    Us = U * np.exp(1j * np.array([theta[m] / L[m] for m in range(4)]))[:, None, None, None]
    lhs = hop(U, psi, L, theta, False)
    rhs = T * hop(Us, psi / T, L, (0, 0, 0, 0), False)
    return _rel(lhs, rhs)


def twisted_mass_normal(apply_M, L, theta, kappa, mu, seed=61):
    """M = D_W + 2 i kappa mu gamma_5 with gamma_5-Hermitian D_W, so
    ||M psi||^2 = ||D_W psi||^2 + (2 kappa mu)^2 ||psi||^2."""
    U = gauge_field(L, "haar", seed=seed)
    psi = gaussian_spinor(L, seed=seed + 1)
    lhs = np.linalg.norm(apply_M(U, psi, L, theta, kappa, mu, False).ravel()) ** 2
    rhs = np.linalg.norm(apply_M(U, psi, L, theta, kappa, 0.0, False).ravel()) ** 2 \
        + (2 * kappa * mu) ** 2 * np.linalg.norm(psi.ravel()) ** 2
    return abs(lhs - rhs) / rhs


def all_pins(hop, apply_M):
    """Run every operator pin on a few lattices; returns {name: error}."""
    errs = {}
    cases = [((2, 4, 2, 4), (0.0, 0.0, 0.0, np.pi)), ((4, 2, 6, 2), (0.3, -1.1, 0.7, 2.0))]
    kappa, mu = 0.13, 0.21
    for k, (L, th) in enumerate(cases):
        for n in [(0, 0, 0, 0), (1, 0, 1, 1), (0, 1, 2, 1)]:
            for dag in (False, True):
                errs[f"free{k}{n}{dag}"] = free_field_closed_form(apply_M, L, th, kappa, mu, n, dagger=dag)
        errs[f"g5herm{k}"] = gamma5_hermiticity(hop, apply_M, L, th, kappa, mu)
        errs[f"adjoint{k}"] = adjoint_consistency(hop, apply_M, L, th, kappa, mu)
        errs[f"covariance{k}"] = gauge_covariance(hop, L, th)
        errs[f"covariance_dag{k}"] = gauge_covariance(hop, L, th, dagger=True)
        errs[f"bc{k}"] = boundary_convention_equivalence(hop, L, th)
        errs[f"tmnormal{k}"] = twisted_mass_normal(apply_M, L, th, kappa, mu)
        ratio, sat = norm_bound(hop, L, th)
        errs[f"normbound{k}"] = max(0.0, ratio - 8.0)
        errs[f"normsat{k}"] = sat
    return errs
