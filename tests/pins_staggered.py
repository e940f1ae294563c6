"""Checks that pin the staggered oracle to facts fixed by the mathematics.

Each check takes the operator under test as callables

    hop(U, phi, L, theta) -> D phi
    apply_M(U, phi, L, theta, mass, dagger) -> (m + D) phi or (m - D) phi

and returns a relative error that must be at rounding level.  The same
checks run against the real oracle (tests/test_oracle_staggered.py) and
against copies of it with planted mistakes (tests/test_oracle_mutants.py).

Nothing here computes the operator itself, except the free-field closed
form: with all links 1 a plane wave exp(i p.x) c is mapped by the hop in
direction mu to 1/2 eta_mu(x) (exp(i p_mu) - exp(-i p_mu)) = i eta_mu(x)
sin(p_mu) times itself, and the staggered phases eta are computed here from
their definition.
"""

from __future__ import annotations

import numpy as np

from lattice_inputs import gauge_field, gauge_transform, site_coords, unit_gauge


def _rel(a, b):
    den = max(np.linalg.norm(b.ravel()), 1e-300)
    return float(np.linalg.norm((a - b).ravel()) / den)


def _inner(a, b):
    return complex(np.vdot(a.ravel(), b.ravel()))


def colour_field(L, seed):
    """Gaussian colour vectors (V, 3), each component CN(0, 1)."""
    rng = np.random.default_rng(seed)
    V = int(np.prod(L))
    return (rng.standard_normal((V, 3)) + 1j * rng.standard_normal((V, 3))) / np.sqrt(2.0)


def eta(L):
    """eta[mu, site] = (-1)^(x_0 + ... + x_{mu-1})."""
    X = site_coords(L)
    out = np.ones((4, X.shape[1]))
    acc = np.zeros(X.shape[1], dtype=np.int64)
    for mu in range(4):
        out[mu] = 1.0 - 2.0 * (acc % 2)
        acc = acc + X[mu]
    return out


def plane_wave(L, n, theta, c):
    """phi(x) = exp(i p.x) c, p_mu = (2 pi n_mu + theta_mu) / L_mu."""
    X = site_coords(L)
    p = np.array([(2 * np.pi * n[m] + theta[m]) / L[m] for m in range(4)])
    phase = np.exp(1j * np.tensordot(p, X, axes=(0, 0)))
    return phase[:, None] * c[None, :], p


def free_field_hop(hop, L, theta, n, seed=7):
    """U = 1: (D phi)(x) = i sum_mu eta_mu(x) sin(p_mu) phi(x)."""
    rng = np.random.default_rng(seed)
    c = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    phi, p = plane_wave(L, n, theta, c)
    f = 1j * np.tensordot(np.sin(p), eta(L), axes=(0, 0))
    return _rel(hop(unit_gauge(L), phi, L, theta), f[:, None] * phi)


def free_field_normal(apply_M, L, theta, mass, n, seed=8):
    """U = 1: M^+ M phi = (m^2 + sum_mu sin^2 p_mu) phi (the cross terms
    of D^2 cancel because eta_mu(x) eta_nu(x + mu) = -eta_nu(x) eta_mu(x + nu))."""
    rng = np.random.default_rng(seed)
    c = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    phi, p = plane_wave(L, n, theta, c)
    U = unit_gauge(L)
    got = apply_M(U, apply_M(U, phi, L, theta, mass, False), L, theta, mass, True)
    return _rel(got, (mass * mass + np.sum(np.sin(p) ** 2)) * phi)


def anti_hermiticity(hop, apply_M, L, theta, mass, seed=11):
    """<chi, D phi> = -<D chi, phi> and <chi, M phi> = <M^+ chi, phi>."""
    U = gauge_field(L, "haar", seed=seed)
    phi = colour_field(L, seed + 1)
    chi = colour_field(L, seed + 2)
    lhs = _inner(chi, hop(U, phi, L, theta))
    rhs = -_inner(hop(U, chi, L, theta), phi)
    e1 = abs(lhs - rhs) / abs(lhs)
    lhs = _inner(chi, apply_M(U, phi, L, theta, mass, False))
    rhs = _inner(apply_M(U, chi, L, theta, mass, True), phi)
    e2 = abs(lhs - rhs) / abs(lhs)
    return max(e1, e2)


def mass_term(hop, apply_M, L, theta, mass, seed=15):
    """M phi - D phi = m phi and M^+ phi + D phi = m phi."""
    U = gauge_field(L, "haar", seed=seed)
    phi = colour_field(L, seed + 1)
    d = hop(U, phi, L, theta)
    e1 = _rel(apply_M(U, phi, L, theta, mass, False) - d, mass * phi)
    e2 = _rel(apply_M(U, phi, L, theta, mass, True) + d, mass * phi)
    return max(e1, e2)


def _shift_index(L, mu, step):
    X = site_coords(L)
    X[mu] = (X[mu] + step) % L[mu]
    return X[0] + L[0] * (X[1] + L[1] * (X[2] + L[2] * X[3]))


def gauge_covariance(hop, L, theta, seed=31):
    """U'_mu(x) = G(x) U_mu(x) G(x+mu)^+, phi' = G phi  =>  D' phi' = G D phi."""
    U = gauge_field(L, "haar", seed=seed)
    phi = colour_field(L, seed + 1)
    G = gauge_transform(L, seed=seed + 2)
    Up = np.empty_like(U)
    for mu in range(4):
        fwd = _shift_index(L, mu, +1)
        Up[mu] = G @ U[mu] @ np.conj(np.swapaxes(G[fwd], 1, 2))
    lhs = hop(Up, np.einsum("vab,vb->va", G, phi), L, theta)
    rhs = np.einsum("vab,vb->va", G, hop(U, phi, L, theta))
    return _rel(lhs, rhs)


def norm_bound(hop, L, theta, seed=41):
    """Each direction is 1/2 (a unitary shift minus another), so ||D phi|| <= 4 ||phi||."""
    U = gauge_field(L, "haar", seed=seed)
    phi = colour_field(L, seed + 1)
    return float(np.linalg.norm(hop(U, phi, L, theta).ravel()) / np.linalg.norm(phi.ravel()))


def parity_structure(hop, L, theta, seed=45):
    """D maps fields on even sites to fields on odd sites and back."""
    U = gauge_field(L, "haar", seed=seed)
    phi = colour_field(L, seed + 1)
    X = site_coords(L)
    par = X.sum(axis=0) % 2
    out = 0.0
    for p in (0, 1):
        src = np.where((par == p)[:, None], phi, 0)
        d = hop(U, src, L, theta)
        out = max(out, float(np.linalg.norm(d[par == p].ravel()) / np.linalg.norm(d.ravel())))
    return out


def boundary_convention_equivalence(hop, L, theta, seed=51):
    """Phases on boundary hops only equal phases exp(i theta_mu / L_mu) spread
    on every link, conjugated by phi(x) -> exp(i sum theta_mu x_mu / L_mu) phi(x)."""
    U = gauge_field(L, "haar", seed=seed)
    phi = colour_field(L, seed + 1)
    X = site_coords(L)
    T = np.exp(1j * sum(theta[m] * X[m] / L[m] for m in range(4)))[:, None]
    Us = U * np.exp(1j * np.array([theta[m] / L[m] for m in range(4)]))[:, None, None, None]
    return _rel(hop(U, phi, L, theta), T * hop(Us, phi / T, L, (0, 0, 0, 0)))


def all_stag_pins(hop, apply_M):
    """Run every staggered operator pin on a few lattices; returns {name: error}."""
    errs = {}
    cases = [((2, 4, 2, 4), (0.0, 0.0, 0.0, np.pi)), ((4, 2, 6, 2), (0.3, -1.1, 0.7, 2.0))]
    mass = 0.17
    for k, (L, th) in enumerate(cases):
        for n in [(0, 0, 0, 0), (1, 0, 1, 1), (0, 1, 2, 1)]:
            errs[f"free_hop{k}{n}"] = free_field_hop(hop, L, th, n)
            errs[f"free_normal{k}{n}"] = free_field_normal(apply_M, L, th, mass, n)
        errs[f"antiherm{k}"] = anti_hermiticity(hop, apply_M, L, th, mass)
        errs[f"mass{k}"] = mass_term(hop, apply_M, L, th, mass)
        errs[f"covariance{k}"] = gauge_covariance(hop, L, th)
        errs[f"parity{k}"] = parity_structure(hop, L, th)
        errs[f"bc{k}"] = boundary_convention_equivalence(hop, L, th)
        errs[f"normbound{k}"] = max(0.0, norm_bound(hop, L, th) - 4.0)
    return errs
