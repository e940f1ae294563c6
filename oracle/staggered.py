"""FP64 oracle of the staggered fermion matrix, its even-odd blocks and solvers.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
benchmark's CPU baseline, never by the product library.  It shares no code
with the GPU path.

The derivative part D (the paper's D_KS, sections 1 and 3) and M = m + D
come from the plain C loops in ``staggered_oracle.c``.  D only connects
sites of opposite parity, so with P_p keeping the sites of parity p

* D_pq = P_p D P_q, M = [[m, D_eo], [D_oe, m]];
* D is anti-Hermitian, hence M^+ M = m^2 - D^2 is block diagonal and its
  even block N = m^2 - D_eo D_oe is Hermitian positive definite;
* the even-odd solve of M x = b: N x_e = (M^+ b)_e = m b_e - D_eo b_o,
  then x_o = (b_o - D_oe x_e) / m;
* the full residual of the reconstructed x is b - M x = (r_e / m) on even
  sites and zero on odd sites, where r_e = m b_e - D_eo b_o - N x_e.

Arrays: gauge (4, V, 3, 3), colour field (V, 3), complex128, canonical site
order x fastest.  Parity of a site is (x + y + z + t) mod 2; even = 0.
"""

from __future__ import annotations

import ctypes
import functools

import numpy as np

from .build import STAG_LIB, STAG_SRC, build_oracle
from .wilson import parity


@functools.lru_cache(maxsize=None)
def _lib():
    lib = ctypes.CDLL(build_oracle(src=STAG_SRC, out=STAG_LIB))
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lib.stag_oracle_hop.argtypes = [ip, dp, dp, dp, dp]
    lib.stag_oracle_hop.restype = None
    lib.stag_oracle_apply_M.argtypes = [ip, dp, ctypes.c_double, dp, dp, dp, ctypes.c_int]
    lib.stag_oracle_apply_M.restype = None
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _geom(L, theta):
    Li = (ctypes.c_int * 4)(*[int(v) for v in L])
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(4))
    return Li, th


def _check(U, phi, L):
    V = int(np.prod(L))
    if U.shape != (4, V, 3, 3) or U.dtype != np.complex128:
        raise ValueError(f"gauge must be complex128 (4,{V},3,3), got {U.dtype} {U.shape}")
    if phi.shape != (V, 3) or phi.dtype != np.complex128:
        raise ValueError(f"colour field must be complex128 ({V},3), got {phi.dtype} {phi.shape}")


def hop(U, phi, L, theta):
    """D phi on the full lattice."""
    U = np.ascontiguousarray(U)
    phi = np.ascontiguousarray(phi)
    _check(U, phi, L)
    out = np.empty_like(phi)
    Li, th = _geom(L, theta)
    _lib().stag_oracle_hop(Li, _dptr(th), _dptr(U), _dptr(phi), _dptr(out))
    return out


def apply_M(U, phi, L, theta, mass, dagger=False):
    """M phi = m phi + D phi (or M^+ phi = m phi - D phi)."""
    U = np.ascontiguousarray(U)
    phi = np.ascontiguousarray(phi)
    _check(U, phi, L)
    out = np.empty_like(phi)
    Li, th = _geom(L, theta)
    _lib().stag_oracle_apply_M(Li, _dptr(th), float(mass), _dptr(U), _dptr(phi), _dptr(out), int(bool(dagger)))
    return out


def mask(phi, L, p):
    """P_p phi: keep the sites of parity p, zero the others."""
    keep = (parity(L) == p)[:, None]
    return np.where(keep, phi, 0)


def hop_eo(U, phi, L, theta, out_parity):
    """D_{p,1-p} phi = P_p D P_{1-p} phi."""
    return mask(hop(U, mask(phi, L, 1 - out_parity), L, theta), L, out_parity)


def normal_e(U, v, L, theta, mass):
    """N v = m^2 v - D_eo D_oe v on even sites."""
    return mass * mass * mask(v, L, 0) - hop_eo(U, hop_eo(U, v, L, theta, 1), L, theta, 0)


def eo_source(U, b, L, theta, mass):
    """(M^+ b)_e = m b_e - D_eo b_o."""
    return mass * mask(b, L, 0) - hop_eo(U, mask(b, L, 1), L, theta, 0)


def eo_reconstruct(U, x_e, b, L, theta, mass):
    """x = x_e + x_o with x_o = (b_o - D_oe x_e) / m."""
    x_e = mask(x_e, L, 0)
    x_o = (mask(b, L, 1) - hop_eo(U, x_e, L, theta, 1)) / mass
    return x_e + mask(x_o, L, 1)


def true_residual(U, x, b, L, theta, mass):
    """||b - M x||_2 / ||b||_2 on the full system."""
    r = b - apply_M(U, x, L, theta, mass)
    nb = np.linalg.norm(b.ravel())
    return float(np.linalg.norm(r.ravel()) / nb) if nb > 0 else float(np.linalg.norm(r.ravel()))


def dense_M(U, L, theta, mass):
    """M as a dense (3V x 3V) matrix from unit vectors (tiny lattices only)."""
    V = int(np.prod(L))
    n = 3 * V
    cols = np.empty((n, n), dtype=np.complex128)
    e = np.zeros((V, 3), dtype=np.complex128)
    flat = e.reshape(-1)
    for j in range(n):
        flat[:] = 0
        flat[j] = 1
        cols[:, j] = apply_M(U, e, L, theta, mass).reshape(-1)
    return cols


def eta_phases(L) -> np.ndarray:
    """eta[mu, site] = (-1)^(x_0 + ... + x_{mu-1}) (the staggered phases)."""
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    i = np.arange(Lx * Ly * Lz * Lt)
    c = [i % Lx, (i // Lx) % Ly, (i // (Lx * Ly)) % Lz, i // (Lx * Ly * Lz)]
    out = np.ones((4, i.size))
    for mu in range(4):
        s = sum(c[nu] for nu in range(mu)) if mu else np.zeros_like(i)
        out[mu] = np.where(s % 2 == 1, -1.0, 1.0)
    return out
