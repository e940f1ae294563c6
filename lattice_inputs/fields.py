"""Seeded generators for gauge fields, spinor sources and gauge transforms.

Canonical host layout (complex128, C order):

* lattice extents ``L = (Lx, Ly, Lz, Lt)``; direction mu = 0, 1, 2, 3 is
  x, y, z, t; site index ``i = x + Lx*(y + Ly*(z + Lz*t))`` (x fastest,
  t slowest);
* gauge field ``U[mu, i, a, b]`` of shape ``(4, V, 3, 3)``: the SU(3) link
  from site i to site i + mu-hat, row a, column b;
* spinor field ``psi[i, s, c]`` of shape ``(V, 4, 3)``: spin s, colour c;
  a batch of right-hand sides is stacked in front, ``(nrhs, V, 4, 3)``.

Boundary phases are never folded into the stored links (links must stay in
SU(3) so that two rows determine the third).

Random numbers come from numpy's ``Generator(PCG64(seed))``.  Draws happen
in a fixed sequential order; the expensive per-matrix linear algebra that
follows is split over a thread pool, which cannot change the result because
each matrix is computed independently of every other.
"""

from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

# Seed scheme: gauge 1000 + config, source 2000 + config, gauge transform
# 3000 + config; lattices of one uneven batch add 10 * (lattice index).
SEEDS = {"gauge": 1000, "source": 2000, "transform": 3000}


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def lattice_volume(L) -> int:
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    return Lx * Ly * Lz * Lt


def canonical_shapes(L, nrhs: int | None = None):
    V = lattice_volume(L)
    spin = (V, 4, 3) if nrhs is None else (nrhs, V, 4, 3)
    return {"gauge": (4, V, 3, 3), "spinor": spin, "transform": (V, 3, 3)}


def site_coords(L):
    """Integer coordinates (x, y, z, t) of every canonical site index."""
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    i = np.arange(Lx * Ly * Lz * Lt, dtype=np.int64)
    x = i % Lx
    y = (i // Lx) % Ly
    z = (i // (Lx * Ly)) % Lz
    t = i // (Lx * Ly * Lz)
    return np.stack([x, y, z, t], axis=0)


# The eight Gell-Mann matrices, the usual basis of su(3): Hermitian,
# traceless, tr(lambda_a lambda_b) = 2 delta_ab.
GELL_MANN = np.zeros((8, 3, 3), dtype=np.complex128)
GELL_MANN[0][0, 1] = GELL_MANN[0][1, 0] = 1
GELL_MANN[1][0, 1] = -1j
GELL_MANN[1][1, 0] = 1j
GELL_MANN[2][0, 0] = 1
GELL_MANN[2][1, 1] = -1
GELL_MANN[3][0, 2] = GELL_MANN[3][2, 0] = 1
GELL_MANN[4][0, 2] = -1j
GELL_MANN[4][2, 0] = 1j
GELL_MANN[5][1, 2] = GELL_MANN[5][2, 1] = 1
GELL_MANN[6][1, 2] = -1j
GELL_MANN[6][2, 1] = 1j
GELL_MANN[7][0, 0] = GELL_MANN[7][1, 1] = 1 / np.sqrt(3)
GELL_MANN[7][2, 2] = -2 / np.sqrt(3)

_CHUNK = 1 << 16


def _pool_workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _chunked(fn, n: int, *arrays):
    """Apply ``fn`` to row chunks of ``arrays`` on a thread pool, in order."""
    if n <= _CHUNK:
        return fn(*arrays)
    starts = list(range(0, n, _CHUNK))
    with ThreadPoolExecutor(_pool_workers()) as ex:
        parts = list(ex.map(lambda s: fn(*(a[s:s + _CHUNK] for a in arrays)), starts))
    return np.concatenate(parts, axis=0)


def _complex_gaussian(rng, shape):
    """Components with Re, Im ~ N(0, 1/2) (unit variance complex normal)."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) * np.sqrt(0.5)


def _haar_from_gaussian(Z):
    Q, R = np.linalg.qr(Z)
    d = np.diagonal(R, axis1=-2, axis2=-1)
    Q = Q * (d / np.abs(d))[..., None, :]
    det = np.linalg.det(Q)
    # principal cube root of the determinant phase: det(Q) has modulus 1
    root = np.exp(1j * np.angle(det) / 3.0)
    return Q / root[..., None, None]


def haar_su3(rng, n: int) -> np.ndarray:
    """n Haar-random SU(3) matrices: QR of a complex Gaussian, phases of
    R's diagonal moved into Q (Haar on U(3)), then the determinant divided
    out with its principal cube root (the result stays Haar on SU(3) since
    multiplying by a scalar phase commutes with the group action)."""
    Z = _complex_gaussian(rng, (n, 3, 3))
    return _chunked(_haar_from_gaussian, n, Z)


def _exp_from_coeffs(c, eps):
    H = np.einsum("na,aij->nij", c, GELL_MANN * 0.5)
    w, V = np.linalg.eigh(H)
    ph = np.exp(1j * eps * w)
    return np.einsum("nij,nj,nkj->nik", V, ph, np.conj(V))


def su3_exp_ieps_h(rng, n: int, eps: float) -> np.ndarray:
    """n links U = exp(i eps H), H = sum_a c_a lambda_a / 2 with c_a ~ N(0,1).

    The exponential is taken through the eigendecomposition of the Hermitian
    H, so U is unitary with det 1 to rounding.
    """
    c = rng.standard_normal((n, 8))
    return _chunked(lambda cc: _exp_from_coeffs(cc, eps), n, c)


def unit_gauge(L) -> np.ndarray:
    V = lattice_volume(L)
    U = np.zeros((4, V, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U


def gauge_field(L, kind: str = "exp", eps: float = 0.4, seed: int = 1000) -> np.ndarray:
    """Gauge field of shape (4, V, 3, 3): ``kind`` is 'haar', 'exp' or 'unit'."""
    V = lattice_volume(L)
    if kind == "unit":
        return unit_gauge(L)
    rng = rng_for(seed)
    if kind == "haar":
        U = haar_su3(rng, 4 * V)
    elif kind == "exp":
        U = su3_exp_ieps_h(rng, 4 * V, eps)
    else:
        raise ValueError(f"unknown gauge kind {kind!r}")
    return np.ascontiguousarray(U.reshape(4, V, 3, 3))


def gaussian_spinor(L, seed: int = 2000, nrhs: int | None = None) -> np.ndarray:
    """Spinor with every component ~ CN(0, 1); shape (V,4,3) or (nrhs,V,4,3)."""
    rng = rng_for(seed)
    return np.ascontiguousarray(_complex_gaussian(rng, canonical_shapes(L, nrhs)["spinor"]))


def point_source(L, spin: int, colour: int, site=(0, 0, 0, 0)) -> np.ndarray:
    """Unit source: 1 at one site, one spin and one colour component."""
    Lx, Ly, Lz, _ = (int(v) for v in L)
    V = lattice_volume(L)
    b = np.zeros((V, 4, 3), dtype=np.complex128)
    x, y, z, t = site
    b[x + Lx * (y + Ly * (z + Lz * t)), spin, colour] = 1.0
    return b


def gauge_transform(L, seed: int = 3000) -> np.ndarray:
    """One Haar-random SU(3) matrix per site, shape (V, 3, 3)."""
    return haar_su3(rng_for(seed), lattice_volume(L))
