"""Molecular dynamics of the N_f = 2 twisted-mass HMC.

The fermion part runs on the GPU through the C ABI: the pseudo-fermion
heatbath phi = M eta, the action S_f = ||M^-1 phi||^2 and its force (two
even-odd CGNR solves and the force kernel).  The gauge part stays on the
host (numpy): the Wilson plaquette action S_g = beta sum_P (1 - Re tr U_P / 3),
its force, the momenta and the link updates U <- exp(i dt P) U.

Conventions: momenta P_mu(x) are Hermitian traceless 3x3 matrices, the
kinetic energy is sum tr P^2 (= 1/2 sum_a p_a^2 for P = sum_a p_a T^a,
T^a = lambda_a / 2), the force of an action S is F = sum_a (dS / dw^a) T^a
for the link rotation U -> exp(i w T^a) U, and the equations of motion are
dU/dt = i P U, dP/dt = -F, which conserve H = sum tr P^2 + S_g + S_f.

Scope: this module exists to check the GPU force end to end (the leapfrog
energy violation must fall as dt^2, which fails for any wrong term of the
force).  The host-side gauge action, momenta and the Metropolis step are the
minimum that check needs; a production HMC (integrator hierarchies,
observables, gauge updates on the device) is not part of this library.
"""

from __future__ import annotations

import math

import numpy as np
import torch

from . import fields
from . import lqcd as L


def _dag(A):
    return np.conj(np.swapaxes(A, -1, -2))


def traceless_antihermitian(G):
    """(G - G^+) - tr(G - G^+) / 3 for every 3x3 matrix of G."""
    A = G - _dag(G)
    tr = np.trace(A, axis1=-2, axis2=-1)[..., None, None]
    return A - tr / 3.0 * np.eye(3)


def _shift(L4, mu, step):
    """Canonical index of site x + step * mu for every site x."""
    Lx, Ly, Lz, Lt = L4
    i = np.arange(Lx * Ly * Lz * Lt)
    c = [i % Lx, (i // Lx) % Ly, (i // (Lx * Ly)) % Lz, i // (Lx * Ly * Lz)]
    c[mu] = (c[mu] + step) % L4[mu]
    return c[0] + Lx * (c[1] + Ly * (c[2] + Lz * c[3]))


def plaquette_action(U, L4, beta):
    """S_g = beta sum_{x, mu < nu} (1 - Re tr U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+ / 3)."""
    s = 0.0
    for mu in range(4):
        fm = _shift(L4, mu, 1)
        for nu in range(mu + 1, 4):
            fn = _shift(L4, nu, 1)
            P = U[mu] @ U[nu][fm] @ _dag(U[mu][fn]) @ _dag(U[nu])
            s += np.sum(1.0 - np.trace(P, axis1=-2, axis2=-1).real / 3.0)
    return float(beta * s)


def plaquette_force(U, L4, beta):
    """F_mu(x) = -(i beta / 12) TA(U_mu(x) Sigma_mu(x)), Sigma the sum of the
    six staples (upper U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+, lower
    U_nu(x+mu-nu)^+ U_mu(x-nu)^+ U_nu(x-nu))."""
    F = np.empty_like(U)
    for mu in range(4):
        fm = _shift(L4, mu, 1)
        sig = np.zeros_like(U[mu])
        for nu in range(4):
            if nu == mu:
                continue
            fn = _shift(L4, nu, 1)
            bn = _shift(L4, nu, -1)
            fm_bn = _shift(L4, nu, -1)[fm]  # x + mu - nu
            sig += U[nu][fm] @ _dag(U[mu][fn]) @ _dag(U[nu])
            sig += _dag(U[nu][fm_bn]) @ _dag(U[mu][bn]) @ U[nu][bn]
        F[mu] = -1j * beta / 12.0 * traceless_antihermitian(U[mu] @ sig)
    return F


def expi(P, dt):
    """exp(i dt P) for Hermitian P (batched)."""
    w, v = np.linalg.eigh(P)
    return (v * np.exp(1j * dt * w)[..., None, :]) @ _dag(v)


def gaussian_momenta(L4, rng):
    """P = sum_a p_a T^a with p_a ~ N(0, 1) on every link."""
    V = int(np.prod(L4))
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7] = np.diag([1, 1, -2]) / math.sqrt(3)
    p = rng.standard_normal((4, V, 8))
    return np.einsum("xva,aij->xvij", p, lam / 2)


class TwistedMassHMC:
    """N_f = 2 twisted-mass molecular dynamics on one GPU (fermion part) and
    the host (gauge part).  Solves run to a relative true residual ``tol``."""

    def __init__(self, L4, theta, kappa, mu, beta, tol=1e-12, device="cuda:0", stream=None):
        self.L4 = tuple(int(v) for v in L4)
        self.theta = tuple(float(t) for t in theta)
        self.kappa, self.mu, self.beta, self.tol = float(kappa), float(mu), float(beta), float(tol)
        self.stream = stream
        self.lat = fields.Lattice(self.L4, self.theta, device)
        self.op = L.op(self.kappa, self.mu)
        self.op_m = L.op(self.kappa, -self.mu)  # M(-mu): (M^+)^-1 = gamma_5 M(-mu)^-1 gamma_5
        self.params = L.solve_params(tol=self.tol, maxiter=100000, eo=1, inner_prec=64)
        self.ws = self.lat.workspace(self.op, self.params)
        V = self.lat.V
        self.X = self.lat.zeros(L.FIELD_SPINOR_FULL, 64)
        self.Wf = self.lat.zeros(L.FIELD_SPINOR_FULL, 64)
        self.tmp = self.lat.zeros(L.FIELD_SPINOR_FULL, 64)
        self.F = torch.zeros((4, V, 3, 3), dtype=torch.complex128, device=self.lat.device)
        self.solves = 0
        self.iters = 0

    def _gauge(self, U):
        return self.lat.gauge(U, 64, 18, self.stream)

    def _solve(self, op, Ud, b, x):
        rc, info = L.cg_solve(self.lat.g, op, Ud, b, x, self.params, self.ws, self.stream)
        if rc != L.OK:
            raise RuntimeError(f"pseudo-fermion solve failed: {L.ERROR_NAMES.get(rc, rc)} {info}")
        self.solves += 1
        self.iters += info[0]["iters"]

    def heatbath(self, U, eta):
        """phi = M eta for a Gaussian eta (canonical (V, 4, 3)): S_f(phi) = ||eta||^2."""
        Ud = self._gauge(U)
        phi = self.lat.empty(L.FIELD_SPINOR_FULL, 64)
        L.dslash_apply(self.lat.g, self.op, Ud, self.lat.spinor(eta, 64, self.stream), phi, stream=self.stream)
        return phi

    def fermion_action(self, U, phi):
        """S_f = ||M^-1 phi||^2."""
        self._solve(self.op, self._gauge(U), phi, self.X)
        x = self.lat.unpack(self.X, 64, stream=self.stream)
        return float(np.vdot(x.ravel(), x.ravel()).real)

    def fermion_force(self, U, phi):
        """F of S_f: X = M^-1 phi, Wf = M(-mu)^-1 gamma_5 X, then the force kernel."""
        Ud = self._gauge(U)
        self._solve(self.op, Ud, phi, self.X)
        L.lqcd_gamma5(self.lat.g, self.X, self.tmp, stream=self.stream)
        self._solve(self.op_m, Ud, self.tmp, self.Wf)
        L.tm_force(self.lat.g, self.op, Ud, self.X, self.Wf, self.F, stream=self.stream)
        torch.cuda.synchronize(self.lat.device)
        return self.F.cpu().numpy()

    def force(self, U, phi):
        return plaquette_force(U, self.L4, self.beta) + self.fermion_force(U, phi)

    def hamiltonian(self, U, P, phi):
        kin = float(np.sum(np.trace(P @ P, axis1=-2, axis2=-1).real))
        return kin + plaquette_action(U, self.L4, self.beta) + self.fermion_action(U, phi)

    def leapfrog(self, U, P, phi, dt, nsteps):
        """nsteps leapfrog steps of size dt: P half step, (U step, P step)*, P half step."""
        U = U.copy()
        P = P - 0.5 * dt * self.force(U, phi)
        for k in range(nsteps):
            U = expi(P, dt) @ U
            P = P - (dt if k < nsteps - 1 else 0.5 * dt) * self.force(U, phi)
        return U, P

    def trajectory(self, U, rng, tau=1.0, nsteps=10):
        """One HMC trajectory from U: momentum and pseudo-fermion heatbath,
        leapfrog, Metropolis.  Returns (U', accepted, dH)."""
        V = int(np.prod(self.L4))
        P = gaussian_momenta(self.L4, rng)
        eta = (rng.standard_normal((V, 4, 3)) + 1j * rng.standard_normal((V, 4, 3))) / math.sqrt(2.0)
        phi = self.heatbath(U, eta)
        H0 = self.hamiltonian(U, P, phi)
        U1, P1 = self.leapfrog(U, P, phi, tau / nsteps, nsteps)
        dH = self.hamiltonian(U1, P1, phi) - H0
        accept = dH <= 0 or rng.random() < math.exp(-dH)
        return (U1 if accept else U), accept, dH
