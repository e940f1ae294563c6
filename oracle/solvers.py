"""FP64 Krylov solvers of the oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/wilson.py``).

The paper (section 1) names the inversion D phi = psi with Krylov methods,
conjugate gradient in particular, as the most expensive part of the
simulation, and (section 3) lists standard inversion algorithms.  The two
solvers here are the textbook methods:

* CGNR: conjugate gradient on the normal equations M^+ M x = M^+ b that
  tracks the residual r = b - M x of the original system (Saad, "Iterative
  Methods for Sparse Linear Systems", the CGNR algorithm);
* BiCGStab (van der Vorst 1992) on the non-Hermitian M directly;
* BiCGStab(l) (Sleijpen and Fokkema 1993): l BiCG steps, then a minimal
  residual polynomial of degree l instead of BiCGStab's degree 1, which
  handles the complex eigenvalue pairs near the imaginary axis on which
  BiCGStab's one-dimensional minimisation stalls; l = 1 is BiCGStab.

Both stop when the tracked residual satisfies ||r|| <= tol * ||b_ref||, then
recompute the true residual in FP64; if that misses the tolerance they
restart from the recomputed residual.  ``b_ref`` is the right-hand side of
the full, unpreconditioned system, so the even-odd solve stops on the same
criterion as the full-lattice one.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import wilson as W

OK = 0
ENOCONV = -3
EBREAKDOWN = -4
ENONFINITE = -5


@dataclass
class SolveInfo:
    status: int = OK
    iters: int = 0
    restarts: int = 0
    true_resid: float = float("nan")
    eo_resid: float = float("nan")


def _dot(a, b):
    return complex(np.vdot(a.ravel(), b.ravel()))


def _nrm2(a):
    return float(np.vdot(a.ravel(), a.ravel()).real)


def cgnr(A, Ah, b, tol, maxiter, b_ref_norm=None, residual=None, x0=None):
    """Solve A x = b by CG on A^+ A, tracking r = b - A x.

    ``residual(x)`` returns the true relative residual used to confirm
    convergence (defaults to ||b - A x|| / b_ref_norm).
    """
    info = SolveInfo()
    bn = float(np.sqrt(_nrm2(b))) if b_ref_norm is None else float(b_ref_norm)
    if residual is None:
        residual = lambda x: float(np.sqrt(_nrm2(b - A(x)))) / bn  # noqa: E731
    x = np.zeros_like(b) if x0 is None else x0.copy()
    if bn == 0.0:
        info.true_resid = 0.0
        return x, info
    if not np.all(np.isfinite(b)):
        info.status = ENONFINITE
        return x, info
    r = b - A(x)
    z = Ah(r)
    p = z.copy()
    zz = _nrm2(z)
    k = 0
    while True:
        if np.sqrt(_nrm2(r)) <= tol * bn:
            tr = residual(x)
            if tr <= tol:
                info.true_resid = tr
                break
            # recursion drifted: restart from the true residual
            info.restarts += 1
            r = b - A(x)
            z = Ah(r)
            p = z.copy()
            zz = _nrm2(z)
        if k >= maxiter:
            info.status = ENOCONV
            info.true_resid = residual(x)
            break
        w = A(p)
        alpha = zz / _nrm2(w)
        x = x + alpha * p
        r = r - alpha * w
        z = Ah(r)
        zz_new = _nrm2(z)
        beta = zz_new / zz
        zz = zz_new
        p = z + beta * p
        k += 1
        if not np.isfinite(zz):
            info.status = ENONFINITE
            break
    info.iters = k
    return x, info


def bicgstab(A, b, tol, maxiter, b_ref_norm=None, residual=None, x0=None):
    """BiCGStab (van der Vorst 1992) on A x = b."""
    info = SolveInfo()
    bn = float(np.sqrt(_nrm2(b))) if b_ref_norm is None else float(b_ref_norm)
    if residual is None:
        residual = lambda x: float(np.sqrt(_nrm2(b - A(x)))) / bn  # noqa: E731
    x = np.zeros_like(b) if x0 is None else x0.copy()
    if bn == 0.0:
        info.true_resid = 0.0
        return x, info
    if not np.all(np.isfinite(b)):
        info.status = ENONFINITE
        return x, info

    def start(x):
        r = b - A(x)
        return r, r.copy(), 1.0 + 0j, 1.0 + 0j, 1.0 + 0j, np.zeros_like(b), np.zeros_like(b)

    r, r0, rho, alpha, omega, v, p = start(x)
    k = 0
    while True:
        if np.sqrt(_nrm2(r)) <= tol * bn:
            tr = residual(x)
            if tr <= tol:
                info.true_resid = tr
                break
            info.restarts += 1
            r, r0, rho, alpha, omega, v, p = start(x)
        if k >= maxiter:
            info.status = ENOCONV
            info.true_resid = residual(x)
            break
        rho_new = _dot(r0, r)
        if rho_new == 0 or omega == 0:
            info.status = EBREAKDOWN
            info.true_resid = residual(x)
            break
        beta = (rho_new / rho) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = A(p)
        alpha = rho_new / _dot(r0, v)
        s = r - alpha * v
        t = A(s)
        tt = _nrm2(t)
        if tt == 0.0:
            # s is already the exact residual of x + alpha p
            x = x + alpha * p
            r = s
            k += 1
            continue
        omega = _dot(t, s) / tt
        x = x + alpha * p + omega * s
        r = s - omega * t
        rho = rho_new
        k += 1
        if not np.isfinite(_nrm2(r)):
            info.status = ENONFINITE
            break
    info.iters = k
    return x, info


def bicgstab_l(A, b, tol, maxiter, ell=2, b_ref_norm=None, residual=None, x0=None):
    """BiCGStab(ell) (Sleijpen and Fokkema 1993) on A x = b.

    Each cycle takes ell BiCG steps that build r_0..r_ell with r_{j+1} =
    A r_j (and u_0..u_ell likewise), then chooses the polynomial of degree
    ell that minimises ||r_0 - sum_j g_j r_j|| by modified Gram-Schmidt on
    r_1..r_ell.  maxiter and info.iters count BiCG steps (ell per cycle,
    2 applications of A each).  Stopping and restarts as for bicgstab."""
    info = SolveInfo()
    bn = float(np.sqrt(_nrm2(b))) if b_ref_norm is None else float(b_ref_norm)
    if residual is None:
        residual = lambda x: float(np.sqrt(_nrm2(b - A(x)))) / bn  # noqa: E731
    x = np.zeros_like(b) if x0 is None else x0.copy()
    if bn == 0.0:
        info.true_resid = 0.0
        return x, info
    if not np.all(np.isfinite(b)):
        info.status = ENONFINITE
        return x, info

    def start(x):
        r = [b - A(x)] + [None] * ell
        u = [np.zeros_like(b)] + [None] * ell
        return r, u, r[0].copy(), 1.0 + 0j, 0.0 + 0j, 1.0 + 0j

    r, u, rt, rho0, alpha, omega = start(x)
    k = 0
    while True:
        if np.sqrt(_nrm2(r[0])) <= tol * bn:
            tr = residual(x)
            if tr <= tol:
                info.true_resid = tr
                break
            info.restarts += 1
            r, u, rt, rho0, alpha, omega = start(x)
        if k >= maxiter:
            info.status = ENOCONV
            info.true_resid = residual(x)
            break
        rho0 = -omega * rho0
        broke = False
        # the BiCG part: ell steps, each extending the r and u sequences by one
        for j in range(ell):
            rho1 = _dot(rt, r[j])
            if rho0 == 0:
                broke = True
                break
            beta = alpha * rho1 / rho0
            rho0 = rho1
            for i in range(j + 1):
                u[i] = r[i] - beta * u[i]
            u[j + 1] = A(u[j])
            gamma = _dot(rt, u[j + 1])
            if gamma == 0:
                broke = True
                break
            alpha = rho0 / gamma
            for i in range(j + 1):
                r[i] = r[i] - alpha * u[i + 1]
            r[j + 1] = A(r[j])
            x = x + alpha * u[0]
        if broke:
            info.status = EBREAKDOWN
            info.true_resid = residual(x)
            break
        # the minimal residual part: modified Gram-Schmidt on r_1..r_ell
        tau = np.zeros((ell + 1, ell + 1), dtype=complex)
        sigma = np.zeros(ell + 1)
        gp = np.zeros(ell + 1, dtype=complex)
        for j in range(1, ell + 1):
            for i in range(1, j):
                tau[i, j] = _dot(r[i], r[j]) / sigma[i]
                r[j] = r[j] - tau[i, j] * r[i]
            sigma[j] = _nrm2(r[j])
            if sigma[j] == 0.0:
                broke = True
                break
            gp[j] = _dot(r[j], r[0]) / sigma[j]
        if broke:
            # r_j = 0 for some j: x already solves the system to rounding
            k += ell
            continue
        g = np.zeros(ell + 1, dtype=complex)
        g[ell] = gp[ell]
        omega = g[ell]
        for j in range(ell - 1, 0, -1):
            g[j] = gp[j] - sum(tau[j, i] * g[i] for i in range(j + 1, ell + 1))
        gpp = np.zeros(ell + 1, dtype=complex)
        for j in range(1, ell):
            gpp[j] = g[j + 1] + sum(tau[j, i] * g[i + 1] for i in range(j + 1, ell))
        x = x + g[1] * r[0]
        r[0] = r[0] - gp[ell] * r[ell]
        u[0] = u[0] - g[ell] * u[ell]
        for j in range(1, ell):
            u[0] = u[0] - g[j] * u[j]
            x = x + gpp[j] * r[j]
            r[0] = r[0] - gp[j] * r[j]
        k += ell
        if not np.isfinite(_nrm2(r[0])):
            info.status = ENONFINITE
            info.true_resid = residual(x)
            break
    info.iters = k
    return x, info


def solve(U, b, L, theta, kappa, mu, tol, maxiter=100000, method="cgnr", eo=True, ell=2):
    """x = M^-1 b with the chosen method ("cgnr", "bicgstab" or "bicgstab_l"
    with degree ell), on the full lattice or through the even-odd Schur
    complement (prepare, solve on even sites, reconstruct)."""
    bn = float(np.sqrt(_nrm2(b)))
    if not eo:
        A = lambda v: W.apply_M(U, v, L, theta, kappa, mu)  # noqa: E731
        Ah = lambda v: W.apply_M(U, v, L, theta, kappa, mu, dagger=True)  # noqa: E731
        res = lambda x: W.true_residual(U, x, b, L, theta, kappa, mu)  # noqa: E731
        if method == "cgnr":
            x, info = cgnr(A, Ah, b, tol, maxiter, bn, res)
        elif method == "bicgstab_l":
            x, info = bicgstab_l(A, b, tol, maxiter, ell, bn, res)
        else:
            x, info = bicgstab(A, b, tol, maxiter, bn, res)
        return x, info

    bhat = W.eo_source(U, b, L, theta, kappa, mu)
    A = lambda v: W.schur(U, v, L, theta, kappa, mu)  # noqa: E731
    Ah = lambda v: W.schur(U, v, L, theta, kappa, mu, dagger=True)  # noqa: E731

    def res(x_e):
        x = W.eo_reconstruct(U, x_e, b, L, theta, kappa, mu)
        return W.true_residual(U, x, b, L, theta, kappa, mu)

    if method == "cgnr":
        x_e, info = cgnr(A, Ah, bhat, tol, maxiter, bn, res)
    elif method == "bicgstab_l":
        x_e, info = bicgstab_l(A, bhat, tol, maxiter, ell, bn, res)
    else:
        x_e, info = bicgstab(A, bhat, tol, maxiter, bn, res)
    x = W.eo_reconstruct(U, x_e, b, L, theta, kappa, mu)
    info.true_resid = W.true_residual(U, x, b, L, theta, kappa, mu)
    r_eo = bhat - A(x_e)
    nbh = np.sqrt(_nrm2(bhat))
    info.eo_resid = float(np.sqrt(_nrm2(r_eo)) / nbh) if nbh > 0 else 0.0
    return x, info


# ---------------------------------------------------------------------------
# Staggered fermions: CG on the even-site normal operator, multi-shift CG


def cg(A, b, tol, maxiter, stop_norm=None, residual=None, x0=None):
    """Conjugate gradient (Hestenes-Stiefel) on a Hermitian positive definite A.

    Stops when ||b - A x|| <= tol * stop_norm on the recursion, then confirms
    with ``residual(x)`` (a relative true residual) and restarts from the
    recomputed residual if that misses ``tol``.
    """
    info = SolveInfo()
    sn = float(np.sqrt(_nrm2(b))) if stop_norm is None else float(stop_norm)
    if residual is None:
        residual = lambda x: float(np.sqrt(_nrm2(b - A(x)))) / sn  # noqa: E731
    x = np.zeros_like(b) if x0 is None else x0.copy()
    if sn == 0.0:
        info.true_resid = 0.0
        return x, info
    if not np.all(np.isfinite(b)):
        info.status = ENONFINITE
        return x, info
    r = b - A(x)
    p = r.copy()
    rr = _nrm2(r)
    k = 0
    while True:
        if np.sqrt(rr) <= tol * sn:
            tr = residual(x)
            if tr <= tol:
                info.true_resid = tr
                break
            info.restarts += 1
            r = b - A(x)
            p = r.copy()
            rr = _nrm2(r)
        if k >= maxiter:
            info.status = ENOCONV
            info.true_resid = residual(x)
            break
        w = A(p)
        pw = _dot(p, w).real
        alpha = rr / pw
        x = x + alpha * p
        r = r - alpha * w
        rr_new = _nrm2(r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        k += 1
        if not np.isfinite(rr):
            info.status = ENONFINITE
            break
    info.iters = k
    return x, info


def multishift_cg(A, b, shifts, tol, maxiter):
    """Solve (A + s_i) x_i = b for every shift s_i at once (A Hermitian
    positive definite, every A + s_i too) with one Krylov space.

    The base system is the smallest shift s0; the residuals of the other
    systems stay collinear with the base residual, r_i = zeta_i r, and the
    CG three-term recurrence gives (shift d = s_i - s0, CG coefficients
    alpha_k, beta_k of the base system, zeta_{-1} = zeta_0 = 1,
    alpha_{-1} = 1, beta_{-1} = 0):

      zeta_{k+1} = zeta_k zeta_{k-1} alpha_{k-1}
                   / (alpha_k beta_{k-1} (zeta_{k-1} - zeta_k) + zeta_{k-1} alpha_{k-1} (1 + d alpha_k))
      alpha^i_k = alpha_k zeta_{k+1} / zeta_k,   beta^i_k = beta_k (zeta_{k+1} / zeta_k)^2
      x_i += alpha^i_k p_i,   p_i = zeta_{k+1} r_{k+1} + beta^i_k p_i

    (Jegerlehner, "Krylov space solvers for shifted linear systems", 1996;
    written here with the shift added to A).  System i is done when
    |zeta_i| ||r|| <= tol ||b||; its x_i and p_i are then frozen.
    Returns the solutions and per-shift (iterations, true relative residual).
    """
    shifts = [float(s) for s in shifts]
    n = len(shifts)
    base = int(np.argmin(shifts))
    s0 = shifts[base]
    bn = float(np.sqrt(_nrm2(b)))
    xs = [np.zeros_like(b) for _ in range(n)]
    if bn == 0.0:
        return xs, [(0, 0.0)] * n
    r = b.copy()
    ps = [b.copy() for _ in range(n)]
    rr = _nrm2(r)
    zeta_prev = np.ones(n)
    zeta = np.ones(n)
    alpha_prev, beta_prev = 1.0, 0.0
    active = np.ones(n, dtype=bool)
    iters = np.zeros(n, dtype=int)
    k = 0
    while active.any() and k < maxiter:
        w = A(ps[base]) + s0 * ps[base]
        alpha = rr / _dot(ps[base], w).real
        zeta_new = np.ones(n)
        for i in range(n):
            if not active[i]:
                continue
            d = shifts[i] - s0
            den = alpha * beta_prev * (zeta_prev[i] - zeta[i]) + zeta_prev[i] * alpha_prev * (1.0 + d * alpha)
            zeta_new[i] = zeta[i] * zeta_prev[i] * alpha_prev / den
            xs[i] = xs[i] + (alpha * zeta_new[i] / zeta[i]) * ps[i]
        r = r - alpha * w
        rr_new = _nrm2(r)
        beta = rr_new / rr
        k += 1
        for i in range(n):
            if not active[i]:
                continue
            bi = beta * (zeta_new[i] / zeta[i]) ** 2
            ps[i] = zeta_new[i] * r + bi * ps[i]
            iters[i] = k
            if abs(zeta_new[i]) * np.sqrt(rr_new) <= tol * bn:
                active[i] = False
        zeta_prev, zeta = zeta, zeta_new
        alpha_prev, beta_prev = alpha, beta
        rr = rr_new
    out = []
    for i in range(n):
        ri = b - A(xs[i]) - shifts[i] * xs[i]
        out.append((int(iters[i]), float(np.sqrt(_nrm2(ri)) / bn)))
    return xs, out


def stag_solve(U, b, L, theta, mass, tol, maxiter=100000):
    """x = M^-1 b for M = m + D (staggered): CG on N = m^2 - D_eo D_oe for
    x_e, then x_o = (b_o - D_oe x_e) / m.  The recursion residual r_e of N
    relates to the full one by ||b - M x|| = ||r_e|| / m, so CG stops at
    ||r_e|| <= tol * m * ||b||."""
    from . import staggered as S

    bn = float(np.sqrt(_nrm2(b)))
    rhs = S.eo_source(U, b, L, theta, mass)
    A = lambda v: S.normal_e(U, v, L, theta, mass)  # noqa: E731

    def res(x_e):
        return S.true_residual(U, S.eo_reconstruct(U, x_e, b, L, theta, mass), b, L, theta, mass)

    x_e, info = cg(A, rhs, tol, maxiter, stop_norm=mass * bn, residual=res)
    x = S.eo_reconstruct(U, x_e, b, L, theta, mass)
    info.true_resid = S.true_residual(U, x, b, L, theta, mass)
    return x, info
