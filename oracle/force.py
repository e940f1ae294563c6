"""FP64 oracle of the twisted-mass pseudo-fermion action and its force.

TEST INFRASTRUCTURE ONLY (see ``oracle/wilson.py``).

The paper (sections 1 and 3) generates gauge fields for N_f = 2 twisted-mass
Wilson fermions with HMC, the determinant entering through pseudo-fermions
phi that need the inverse of the fermion matrix.  Reading used here (the
paper prints no formulas): the pseudo-fermion action

    S_f(U) = || M(U)^-1 phi ||^2 = phi^+ (M M^+)^-1 phi

and its derivative along a left rotation of one link,
U_mu(y) -> exp(i w T^a) U_mu(y) with T^a = lambda_a / 2:

    F_mu(y) = sum_a (dS_f / dw^a) T^a            (Hermitian, traceless)

With X = M^-1 phi and Z = (M^+)^-1 X, dS_f = -2 Re <Z, dM X>, dM = -kappa dH,
and collecting the two hops in H that carry U_mu(y) (forward from y, backward
from y + mu) into the colour matrix

    W = sum_s [ f+ U (1 - gamma_mu) X(y + mu) ]_s Z_s(y)^+
      - f- sum_s X_s(y) [ U (1 + gamma_mu) Z(y + mu) ]_s^+

(f+- the boundary phases of the two hops), one finds
dS_f / dw^a = i kappa tr(T^a (W - W^+)) and, with sum_a T^a tr(T^a A) =
(A - tr(A)/3) / 2 for traceless-projecting,

    F_mu(y) = (i kappa / 2) [ (W - W^+) - tr(W - W^+) / 3 ].

``action`` and ``force_fd`` compute S_f and its derivative directly from
the definition (dense solves, central finite differences), so they pin
``force`` without using this derivation.
"""

from __future__ import annotations

import numpy as np

from lattice_inputs import site_coords
from . import wilson as W


def gellmann_generators():
    """T^a = lambda_a / 2, a = 1..8, built from the Gell-Mann matrices."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7] = np.diag([1, 1, -2]) / np.sqrt(3)
    return lam / 2


def _neighbour(L, mu, step):
    X = site_coords(L)
    X[mu] = (X[mu] + step) % L[mu]
    return X[0] + L[0] * (X[1] + L[1] * (X[2] + L[2] * X[3]))


def force_link(U, X, Z, L, theta, kappa, mu, y):
    """F_mu(y) (3x3 Hermitian traceless) of the link U_mu(y), from X = M^-1 phi
    and Z = (M^+)^-1 X."""
    g, _ = W.gammas()
    one = np.eye(4)
    c = [y % L[0], (y // L[0]) % L[1], (y // (L[0] * L[1])) % L[2], y // (L[0] * L[1] * L[2])]
    edge = c[mu] == L[mu] - 1                         # the link crosses the boundary
    c[mu] = (c[mu] + 1) % L[mu]
    fwd = c[0] + L[0] * (c[1] + L[1] * (c[2] + L[2] * c[3]))
    fp = np.exp(1j * theta[mu]) if edge else 1.0      # forward hop phase
    fm = np.conj(fp)                                  # backward hop phase (from y + mu)
    u = U[mu, y]
    v = (u @ ((one - g[mu]) @ X[fwd]).T).T * fp       # [s, colour] = f+ U (1 - gamma) X(y+mu)
    w1 = sum(np.outer(v[s], np.conj(Z[y, s])) for s in range(4))
    r = (u @ ((one + g[mu]) @ Z[fwd]).T).T            # U (1 + gamma) Z(y+mu)
    w2 = fm * sum(np.outer(X[y, s], np.conj(r[s])) for s in range(4))
    Wm = w1 - w2
    A = Wm - Wm.conj().T
    return 0.5j * kappa * (A - np.trace(A) / 3 * np.eye(3))


def force(U, X, Z, L, theta, kappa):
    """F[mu, site] for every link (force_link on each)."""
    V = int(np.prod(L))
    F = np.zeros((4, V, 3, 3), dtype=np.complex128)
    for mu in range(4):
        for y in range(V):
            F[mu, y] = force_link(U, X, Z, L, theta, kappa, mu, y)
    return F


def solve_pair(U, phi, L, theta, kappa, mu, dense=None):
    """X = M^-1 phi and Z = (M^+)^-1 X by dense LU (tiny lattices)."""
    M = W.dense_M(U, L, theta, kappa, mu) if dense is None else dense
    X = np.linalg.solve(M, phi.reshape(-1)).reshape(phi.shape)
    Z = np.linalg.solve(M.conj().T, X.reshape(-1)).reshape(phi.shape)
    return X, Z


def action(U, phi, L, theta, kappa, mu):
    """S_f = || M^-1 phi ||^2 by a dense solve."""
    M = W.dense_M(U, L, theta, kappa, mu)
    x = np.linalg.solve(M, phi.reshape(-1))
    return float(np.vdot(x, x).real)


def rotate_link(U, mu, y, a, w):
    """U with U_mu(y) replaced by exp(i w T^a) U_mu(y)."""
    T = gellmann_generators()[a]
    ev, vec = np.linalg.eigh(T)
    R = vec @ np.diag(np.exp(1j * w * ev)) @ vec.conj().T
    out = U.copy()
    out[mu, y] = R @ U[mu, y]
    return out


def force_fd(U, phi, L, theta, kappa, mu, link_mu, y, a, h=1e-5):
    """dS_f / dw^a at link (link_mu, y) by a central difference (fourth-order)."""
    def S(w):
        return action(rotate_link(U, link_mu, y, a, w), phi, L, theta, kappa, mu)
    return (8 * (S(h) - S(-h)) - (S(2 * h) - S(-2 * h))) / (12 * h)
