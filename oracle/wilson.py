"""FP64 oracle of the Wilson / twisted-mass fermion matrix and its even-odd blocks.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
benchmark's CPU baseline, never by the product library.  It shares no code
with the GPU path.

The hopping term H and the full matrix M = 1 + 2 i kappa mu gamma_5 - kappa H
come from the plain C loops in ``wilson_oracle.c`` (section 1 of the paper:
D is applied many times inside a Krylov inversion; section 3: twisted-mass
Wilson fermions).  The even-odd blocks below are written on full-lattice
arrays with parity masks, the definition itself:

* ``H_pq = P_p H P_q`` (P_p keeps the sites of parity p), so
  M = [[A, -kappa H_eo], [-kappa H_oe, A]] with A = 1 + 2 i kappa mu gamma_5;
* Schur complement on even sites: Mhat = A - kappa^2 H_eo A^-1 H_oe;
* prepared source: bhat = b_e + kappa H_eo A^-1 b_o;
* odd reconstruction: x_o = A^-1 (b_o + kappa H_oe x_e).

Arrays: gauge (4, V, 3, 3), spinor (V, 4, 3), complex128, canonical site
order x fastest.  Parity of a site is (x + y + z + t) mod 2; even = 0.
"""

from __future__ import annotations

import ctypes
import functools

import numpy as np

from .build import build_oracle


@functools.lru_cache(maxsize=None)
def _lib():
    lib = ctypes.CDLL(build_oracle())
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lib.oracle_hop.argtypes = [ip, dp, dp, dp, dp, ctypes.c_int]
    lib.oracle_hop.restype = None
    lib.oracle_apply_M.argtypes = [ip, dp, ctypes.c_double, ctypes.c_double, dp, dp, dp, ctypes.c_int]
    lib.oracle_apply_M.restype = None
    lib.oracle_gammas.argtypes = [dp]
    lib.oracle_gammas.restype = None
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = ctypes.c_int
    return lib


def num_threads() -> int:
    return int(_lib().oracle_num_threads())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _geom(L, theta):
    Li = (ctypes.c_int * 4)(*[int(v) for v in L])
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(4))
    return Li, th


def _check(U, psi, L):
    V = int(np.prod(L))
    if U.shape != (4, V, 3, 3) or U.dtype != np.complex128:
        raise ValueError(f"gauge must be complex128 (4,{V},3,3), got {U.dtype} {U.shape}")
    if psi.shape != (V, 4, 3) or psi.dtype != np.complex128:
        raise ValueError(f"spinor must be complex128 ({V},4,3), got {psi.dtype} {psi.shape}")


@functools.lru_cache(maxsize=None)
def gammas():
    """(gamma[4,4,4], gamma5[4,4]) exactly as the C oracle builds them."""
    buf = np.zeros(5 * 16, dtype=np.complex128)
    _lib().oracle_gammas(_dptr(buf))
    g = buf[:64].reshape(4, 4, 4).copy()
    g5 = buf[64:].reshape(4, 4).copy()
    return g, g5


def hop(U, psi, L, theta, dagger=False):
    """H psi (or H^+ psi): the Wilson hopping term on the full lattice."""
    U = np.ascontiguousarray(U)
    psi = np.ascontiguousarray(psi)
    _check(U, psi, L)
    out = np.empty_like(psi)
    Li, th = _geom(L, theta)
    _lib().oracle_hop(Li, _dptr(th), _dptr(U), _dptr(psi), _dptr(out), int(bool(dagger)))
    return out


def apply_M(U, psi, L, theta, kappa, mu, dagger=False):
    """M psi (or M^+ psi), M = 1 + 2 i kappa mu gamma_5 - kappa H."""
    U = np.ascontiguousarray(U)
    psi = np.ascontiguousarray(psi)
    _check(U, psi, L)
    out = np.empty_like(psi)
    Li, th = _geom(L, theta)
    _lib().oracle_apply_M(Li, _dptr(th), float(kappa), float(mu), _dptr(U), _dptr(psi),
                          _dptr(out), int(bool(dagger)))
    return out


def parity(L) -> np.ndarray:
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    i = np.arange(Lx * Ly * Lz * Lt)
    x = i % Lx
    y = (i // Lx) % Ly
    z = (i // (Lx * Ly)) % Lz
    t = i // (Lx * Ly * Lz)
    return (x + y + z + t) % 2


def mask(psi, L, p):
    """P_p psi: keep the sites of parity p, zero the others."""
    keep = (parity(L) == p)[:, None, None]
    return np.where(keep, psi, 0)


def apply_gamma5(psi):
    _, g5 = gammas()
    return np.einsum("ab,vbc->vac", g5, psi)


def apply_A(psi, kappa, mu, dagger=False, inverse=False):
    """A psi with A = 1 + 2 i kappa mu gamma_5 (site-diagonal), A^+ for
    dagger; the inverse uses A^-1 = (1 - 2 i kappa mu gamma_5) / (1 + 4 kappa^2 mu^2)
    (gamma_5 squares to one)."""
    sign = -1.0 if dagger else 1.0
    tw = 2j * kappa * mu * sign
    if inverse:
        return (psi - tw * apply_gamma5(psi)) / (1.0 + 4.0 * kappa * kappa * mu * mu)
    return psi + tw * apply_gamma5(psi)


def hop_eo(U, psi, L, theta, out_parity, dagger=False):
    """H_{p,1-p} psi = P_p H P_{1-p} psi."""
    return mask(hop(U, mask(psi, L, 1 - out_parity), L, theta, dagger), L, out_parity)


def schur(U, v, L, theta, kappa, mu, dagger=False):
    """Mhat v = A v - kappa^2 H_eo A^-1 H_oe v on even sites; for dagger,
    Mhat^+ = A^+ - kappa^2 H^+_eo (A^-1)^+ H^+_oe."""
    t = apply_A(hop_eo(U, v, L, theta, 1, dagger), kappa, mu, dagger, inverse=True)
    return mask(apply_A(v, kappa, mu, dagger), L, 0) - kappa * kappa * hop_eo(U, t, L, theta, 0, dagger)


def eo_source(U, b, L, theta, kappa, mu):
    """bhat = b_e + kappa H_eo A^-1 b_o."""
    b_o = mask(b, L, 1)
    return mask(b, L, 0) + kappa * hop_eo(U, apply_A(b_o, kappa, mu, inverse=True), L, theta, 0)


def eo_reconstruct(U, x_e, b, L, theta, kappa, mu):
    """x = x_e + x_o with x_o = A^-1 (b_o + kappa H_oe x_e)."""
    x_e = mask(x_e, L, 0)
    x_o = apply_A(mask(b, L, 1) + kappa * hop_eo(U, x_e, L, theta, 1), kappa, mu, inverse=True)
    return x_e + mask(x_o, L, 1)


def true_residual(U, x, b, L, theta, kappa, mu):
    """||b - M x||_2 / ||b||_2 on the full, unpreconditioned system."""
    r = b - apply_M(U, x, L, theta, kappa, mu)
    nb = np.linalg.norm(b.ravel())
    return float(np.linalg.norm(r.ravel()) / nb) if nb > 0 else float(np.linalg.norm(r.ravel()))


def dense_M(U, L, theta, kappa, mu):
    """M as a dense (12V x 12V) matrix, built column by column from unit
    vectors.  Only for tiny lattices."""
    V = int(np.prod(L))
    n = 12 * V
    cols = np.empty((n, n), dtype=np.complex128)
    e = np.zeros((V, 4, 3), dtype=np.complex128)
    flat = e.reshape(-1)
    for j in range(n):
        flat[:] = 0
        flat[j] = 1
        cols[:, j] = apply_M(U, e, L, theta, kappa, mu).reshape(-1)
    return cols
