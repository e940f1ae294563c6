"""The seeded generators produce what they promise: SU(3) links, the stated
distributions, deterministic output for a seed."""

import numpy as np

from lattice_inputs import (gauge_field, gauge_transform, gaussian_spinor, point_source,
                            site_coords)


def _su3_err(U):
    U = U.reshape(-1, 3, 3)
    uu = U @ np.conj(np.swapaxes(U, 1, 2))
    return np.abs(uu - np.eye(3)).max(), np.abs(np.linalg.det(U) - 1).max()


def test_haar_links_are_su3():
    U = gauge_field((4, 4, 4, 4), "haar", seed=1000)
    a, b = _su3_err(U)
    assert a < 1e-14 and b < 1e-14
    # Haar: E[tr U] = 0 and E|tr U|^2 = 1
    tr = np.trace(U.reshape(-1, 3, 3), axis1=1, axis2=2)
    assert abs(tr.mean()) < 0.05 and abs((np.abs(tr) ** 2).mean() - 1) < 0.08


def test_exp_links_are_su3_and_near_unit():
    U = gauge_field((8, 8, 8, 8), "exp", eps=0.4, seed=1001)
    a, b = _su3_err(U)
    assert a < 1e-14 and b < 1e-14
    plaq_like = np.trace(U.reshape(-1, 3, 3), axis1=1, axis2=2).real.mean() / 3
    # 1 - eps^2 <tr H^2> / 6 = 1 - 0.16 * 4 / 6 to leading order
    assert 0.88 < plaq_like < 0.91


def test_determinism_and_chunking():
    a = gauge_field((4, 4, 8, 8), "exp", eps=0.3, seed=9)
    b = gauge_field((4, 4, 8, 8), "exp", eps=0.3, seed=9)
    assert np.array_equal(a, b)
    big = gauge_field((16, 16, 16, 8), "exp", eps=0.3, seed=9)  # spans several chunks
    assert _su3_err(big)[0] < 1e-14


def test_spinor_and_point_source():
    s = gaussian_spinor((4, 4, 4, 4), seed=2000)
    assert s.shape == (256, 4, 3)
    assert abs(np.mean(np.abs(s) ** 2) - 1) < 0.1
    ms = gaussian_spinor((2, 2, 2, 2), seed=1, nrhs=3)
    assert ms.shape == (3, 16, 4, 3)
    p = point_source((4, 4, 4, 4), 2, 1)
    assert p[0, 2, 1] == 1 and np.count_nonzero(p) == 1
    X = site_coords((2, 4, 6, 8))
    assert X[:, 1 + 2 * (3 + 4 * (5 + 6 * 7))].tolist() == [1, 3, 5, 7]
    G = gauge_transform((2, 2, 2, 2), seed=3)
    assert _su3_err(G)[0] < 1e-14
