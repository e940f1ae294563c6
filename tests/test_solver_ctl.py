"""CPU tests of the solvers' scalar steps (the device control block of
``csrc/solver_ctl.h``, compiled here for the host).

The library runs every Krylov scalar on the device: each reduction's
finalize calls ``finalize_totals`` on the grand totals.  These tests drive
the same function from numpy:

* the launch sequences of the library's CGNR, BiCGStab and multi-shift CG are
  replayed with numpy vectors on small dense systems, taking every scalar
  from the control block, and must reproduce the oracle's solvers
  (``oracle/solvers.py``: the textbook methods) to rounding;
* the mixed-precision triggers (reliable update, stagnation window, FP64
  residual that did not fall, outer step at tol_inner, fall back from FP16
  to FP32 storage) and the BiCGStab breakdown / ||t|| = 0 cases are checked
  on hand-made sequences of totals.
"""

from __future__ import annotations

import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import solvers as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ENOCONV, EBREAKDOWN, ENONFINITE = -3, -4, -5


@pytest.fixture(scope="module")
def H(tmp_path_factory):
    cxx = shutil.which("g++")
    if not cxx:
        pytest.skip("no host C++ compiler")
    out = str(tmp_path_factory.mktemp("ctl") / "libctl.so")
    subprocess.run([cxx, "-O1", "-std=c++17", "-shared", "-fPIC", "-I", os.path.join(ROOT, "include"), "-I",
                    os.path.join(ROOT, "paper_1411_5219_amd", "csrc"), os.path.join(ROOT, "tests", "ctl_harness.cpp"),
                    "-o", out], check=True)
    lib = ctypes.CDLL(out)
    lib.ctl_size.restype = ctypes.c_size_t
    lib.ctl_init.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                             ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.ctl_fin.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                            ctypes.c_double]
    lib.ctl_get.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_char_p]
    lib.ctl_get.restype = ctypes.c_double
    lib.ctl_set.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_char_p, ctypes.c_double]
    lib.ctl_fin_code.argtypes = [ctypes.c_char_p]
    lib.ctl_fin_v.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                              ctypes.c_int]
    lib.chunk_iterations_left.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                          ctypes.c_double]
    lib.chunk_next.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
    return lib


class Ctl:
    """A family of n control blocks in host memory."""

    def __init__(self, lib, n=1, tol=1e-10, delta=0.0, tol_inner=0.0, iter_limit=10000, stag_window=0,
                 max_stag=0, fallback_ok=0, shifts=None):
        self.lib = lib
        self.buf = ctypes.create_string_buffer(lib.ctl_size() * n)
        sh = (ctypes.c_double * n)(*shifts) if shifts is not None else None
        lib.ctl_init(self.buf, n, tol, delta, tol_inner, iter_limit, stag_window, max_stag, fallback_ok, sh)

    def fin(self, name, v0=0.0, v1=0.0, v2=0.0, idx=0):
        code = self.lib.ctl_fin_code(name.encode())
        assert code >= 0, name
        self.lib.ctl_fin(self.buf, idx, code, float(v0), float(v1), float(v2))

    def fin_v(self, name, *vals, idx=0):
        code = self.lib.ctl_fin_code(name.encode())
        assert code >= 0, name
        arr = (ctypes.c_double * len(vals))(*[float(v) for v in vals])
        self.lib.ctl_fin_v(self.buf, idx, code, arr, len(vals))

    def __getitem__(self, name):
        return self.get(name)

    def get(self, name, idx=0):
        v = self.lib.ctl_get(self.buf, idx, name.encode())
        assert v != -1e300, name
        return v

    def cplx(self, name, idx=0):
        return complex(self.get(name + "_re", idx), self.get(name + "_im", idx))

    def set(self, name, v, idx=0):
        assert self.lib.ctl_set(self.buf, idx, name.encode(), float(v)) == 0


def nrm2(v):
    return float(np.vdot(v, v).real)


def dense_system(n, seed, hermitian=False, shift=0.0):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    A = np.eye(n) * 3.0 + 0.4 * A / np.sqrt(n)
    if hermitian:
        A = A.conj().T @ A
    b = rng.normal(size=n) + 1j * rng.normal(size=n)
    return A + shift * np.eye(n), b


# ---------------------------------------------------------------------------
# The library's launch sequences replayed on dense systems


def cgnr_by_ctl(H, A, b, tol, maxiter=1000):
    """The FP64 CGNR of the library: start r = b - A x, z = A^+ r (FIN_CG_ZZ),
    p = z; iteration w = A p (FIN_CG_ALPHA), x += alpha p, r -= alpha w
    (FIN_CG_RR), z = A^+ r (FIN_CG_BETA), p = z + beta p."""
    c = Ctl(H, tol=tol, iter_limit=maxiter)
    c.fin("BB_FULL", nrm2(b))
    x = np.zeros_like(b)
    r = b - A @ x
    z = A.conj().T @ r
    c.fin("CG_ZZ", nrm2(z))
    p = z.copy()
    while not c["done"]:
        w = A @ p
        c.fin("CG_ALPHA", nrm2(w))
        if c["done"]:
            break
        x = x + c["alpha"] * p
        r = r - c["alpha"] * w
        c.fin("CG_RR", nrm2(r))
        if c["done"]:
            break
        z = A.conj().T @ r
        c.fin("CG_BETA", nrm2(z))
        if c["done"]:
            break
        p = z + c["beta"] * p
    return x, c


def test_cgnr_sequence_matches_oracle(H):
    A, b = dense_system(24, 1)
    x, c = cgnr_by_ctl(H, A, b, 1e-12)
    assert c["status"] == 0 and c["done"] == 1
    xo, info = S.cgnr(lambda v: A @ v, lambda v: A.conj().T @ v, b, 1e-12, 1000)
    assert info.status == 0
    # the oracle counts the same iterations (its loop confirms the true residual, which holds here)
    assert int(c["iter"]) == info.iters
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) < 1e-13
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) <= 1e-12


def bicgstab_by_ctl(H, A, b, tol, maxiter=1000):
    """The library's BiCGStab launch sequence: start r = b - A x, r0 = r
    (FIN_BI_INIT), p = v = 0; iteration p = r + beta (p - omega v), v = A p
    (FIN_BI_ALPHA), s = r - alpha v, t = A s (FIN_BI_OMEGA),
    x += alpha p + omega_step s, r = s - omega_step t (FIN_BI_RHO)."""
    c = Ctl(H, tol=tol, iter_limit=maxiter)
    c.fin("BB_FULL", nrm2(b))
    x = np.zeros_like(b)
    r = b - A @ x
    r0 = r.copy()
    d = np.vdot(r0, r)
    c.fin("BI_INIT", nrm2(r), d.real, d.imag)
    p = np.zeros_like(b)
    v = np.zeros_like(b)
    while not c["done"]:
        beta = (c.cplx("rho") / c.cplx("rho_old")) * (c.cplx("balpha") / c.cplx("omega"))
        p = r + beta * (p - c.cplx("omega") * v)
        v = A @ p
        d = np.vdot(r0, v)
        c.fin("BI_ALPHA", d.real, d.imag)
        if c["done"]:
            break
        s = r - c.cplx("balpha") * v
        t = A @ s
        d = np.vdot(t, s)
        c.fin("BI_OMEGA", nrm2(t), d.real, d.imag)
        if c["done"]:
            break
        om = c.cplx("omega_step")
        x = x + c.cplx("balpha") * p + om * s
        r = s - om * t
        d = np.vdot(r0, r)
        c.fin("BI_RHO", nrm2(r), d.real, d.imag)
    return x, c


def test_bicgstab_sequence_matches_oracle(H):
    A, b = dense_system(24, 2)
    x, c = bicgstab_by_ctl(H, A, b, 1e-12)
    assert c["status"] == 0
    xo, info = S.bicgstab(lambda v: A @ v, b, 1e-12, 1000)
    assert info.status == 0 and int(c["iter"]) == info.iters
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) < 1e-12
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) <= 1e-12


def test_bicgstab_zero_t_is_not_a_breakdown(H):
    """||t|| = 0: s is the exact residual of x + alpha p.  The step takes
    omega = 0 for the update only; rho_old and omega of the recursion are kept
    (as the oracle does) and the solve goes on."""
    c = Ctl(H, tol=1e-10)
    c.fin("BB_FULL", 1.0)
    c.fin("BI_INIT", 1.0, 0.7, 0.1)
    c.fin("BI_ALPHA", 0.5, 0.2)
    c.fin("BI_OMEGA", 0.0, 0.0, 0.0)
    assert c["lucky"] == 1 and c.cplx("omega_step") == 0
    c.fin("BI_RHO", 0.3, 0.2, -0.05)
    assert c["done"] == 0 and c["status"] == 0
    assert c.cplx("omega") == 1.0 and c.cplx("rho_old") == 1.0     # kept from the start
    assert c.cplx("rho") == complex(0.2, -0.05)
    # the next step with ||t|| > 0 moves them on
    c.fin("BI_ALPHA", 0.5, 0.0)
    c.fin("BI_OMEGA", 2.0, 0.5, 0.25)
    assert c["lucky"] == 0 and c.cplx("omega_step") == complex(0.25, 0.125)
    c.fin("BI_RHO", 0.1, 0.3, 0.0)
    assert c.cplx("omega") == complex(0.25, 0.125) and c.cplx("rho_old") == complex(0.2, -0.05)
    # ||t|| = 0 with s = 0: converged
    c.fin("BI_OMEGA", 0.0, 0.0, 0.0)
    c.fin("BI_RHO", 0.0, 0.0, 0.0)
    assert c["done"] == 1 and c["status"] == 0


def test_bicgstab_breakdowns(H):
    c = Ctl(H, tol=1e-10)
    c.fin("BB_FULL", 1.0)
    c.fin("BI_INIT", 1.0, 1.0, 0.0)
    c.fin("BI_ALPHA", 0.0, 0.0)                 # <r0, v> = 0
    assert c["status"] == EBREAKDOWN and c["done"] == 1
    c = Ctl(H, tol=1e-10)
    c.fin("BB_FULL", 1.0)
    c.fin("BI_INIT", 1.0, 1.0, 0.0)
    c.fin("BI_ALPHA", 1.0, 0.0)
    c.fin("BI_RHO", 0.5, 0.0, 0.0)              # rho = <r0, r> = 0, not converged
    assert c["status"] == EBREAKDOWN
    c = Ctl(H, tol=1e-10)
    c.fin("BB_FULL", 1.0)
    c.fin("BI_INIT", 1.0, 1.0, 0.0)
    c.fin("BI_ALPHA", 1.0, 0.0)
    c.fin("BI_OMEGA", 1.0, 0.0, 0.0)            # omega = <t, s> / ||t||^2 = 0
    c.fin("BI_RHO", 0.5, 0.3, 0.0)
    assert c["status"] == EBREAKDOWN
    c = Ctl(H, tol=1e-10)                        # convergence wins over breakdown
    c.fin("BB_FULL", 1.0)
    c.fin("BI_INIT", 1.0, 1.0, 0.0)
    c.fin("BI_ALPHA", 1.0, 0.0)
    c.fin("BI_OMEGA", 1.0, 0.0, 0.0)
    c.fin("BI_RHO", 1e-22, 0.0, 0.0)
    assert c["status"] == 0 and c["done"] == 1


def bicgstab2_by_ctl(H, A, b, tol, maxiter=1000):
    """The library's BiCGStab(2) launch sequence: start r_0 = b - A x,
    rt = r_0 (FIN_BL_INIT), u_0 = u_1 = u_2 = 0; cycle u_0 = r_0 - beta (u_0 -
    g1 u_1 - g2 u_2), u_1 = A u_0 (FIN_BL_ALPHA), x += alpha u_0, r_0 -= alpha
    u_1, r_1 = A r_0 (FIN_BL_BETA), u_0 = r_0 - beta u_0, u_1 = r_1 - beta u_1,
    u_2 = A u_1 (FIN_BL_ALPHA), x += alpha u_0, r_0 -= alpha u_1, r_1 -= alpha
    u_2, r_2 = A r_1, Gram totals (FIN_BL_TAU), r_2 -= tau r_1 (FIN_BL_OMEGA),
    x += g1 r_0 + g2 r_1, r_0 -= gp1 r_1 + gp2 r_2 (FIN_BL_RES)."""
    c = Ctl(H, tol=tol, iter_limit=maxiter)
    c.fin("BB_FULL", nrm2(b))
    x = np.zeros_like(b)
    r0 = b - A @ x
    rt = r0.copy()
    d = np.vdot(rt, r0)
    c.fin("BL_INIT", nrm2(r0), d.real, d.imag)
    u0, u1, u2 = (np.zeros_like(b) for _ in range(3))
    while not c["done"]:
        be, g1, g2 = c.cplx("bl_beta"), c.cplx("bl_g1"), c.cplx("bl_g2")
        u0 = r0 - be * (u0 - g1 * u1 - g2 * u2)
        u1 = A @ u0
        d = np.vdot(rt, u1)
        c.fin("BL_ALPHA", d.real, d.imag)
        if c["done"]:
            break
        al = c.cplx("balpha")
        x = x + al * u0
        r0 = r0 - al * u1
        r1 = A @ r0
        d = np.vdot(rt, r1)
        c.fin("BL_BETA", d.real, d.imag)
        if c["done"]:
            break
        be = c.cplx("bl_beta")
        u0 = r0 - be * u0
        u1 = r1 - be * u1
        u2 = A @ u1
        d = np.vdot(rt, u2)
        c.fin("BL_ALPHA", d.real, d.imag)
        if c["done"]:
            break
        al = c.cplx("balpha")
        x = x + al * u0
        r0 = r0 - al * u1
        r1 = r1 - al * u2
        r2 = A @ r1
        d12, d10 = np.vdot(r1, r2), np.vdot(r1, r0)
        c.fin_v("BL_TAU", nrm2(r1), d12.real, d12.imag, d10.real, d10.imag)
        if c["done"]:
            break
        r2 = r2 - c.cplx("bl_tau") * r1
        d = np.vdot(r2, r0)
        c.fin("BL_OMEGA", nrm2(r2), d.real, d.imag)
        if c["done"]:
            break
        g1, g2, gp1, gp2 = (c.cplx(n) for n in ("bl_g1", "bl_g2", "bl_gp1", "bl_gp2"))
        x = x + g1 * r0 + g2 * r1
        r0 = r0 - gp1 * r1 - gp2 * r2
        d = np.vdot(rt, r0)
        c.fin("BL_RES", nrm2(r0), d.real, d.imag)
    return x, c


@pytest.mark.parametrize("n,seed,shift", [(24, 2, 0.0), (40, 5, -2.0)])
def test_bicgstab2_sequence_matches_oracle(H, n, seed, shift):
    """The fused launch sequence (the polynomial step's u_0 update folded into
    the next cycle) against the oracle's BiCGStab(ell = 2): the same BiCG step
    count and the same solution to rounding."""
    A, b = dense_system(n, seed, shift=shift)
    x, c = bicgstab2_by_ctl(H, A, b, 1e-12)
    assert c["status"] == 0
    xo, info = S.bicgstab_l(lambda v: A @ v, b, 1e-12, 1000, ell=2)
    assert info.status == 0 and int(c["iter"]) == info.iters
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) < 1e-12
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) <= 1e-12


def test_bicgstab2_sequence_first_cycles_near_singular(H):
    """On a shifted system whose spectrum reaches within 0.012 of the origin
    the iteration amplifies rounding (a 1e-15 change of b moves the oracle's
    own iterate by 4e-8 after 10 steps), so only the first cycles are compared,
    each within a few times that self-sensitivity."""
    A, b = dense_system(40, 5, shift=-3.0)
    for k, bound in ((2, 1e-14), (4, 1e-13), (6, 1e-10)):
        x, c = bicgstab2_by_ctl(H, A, b, 1e-30, maxiter=k)
        xo, info = S.bicgstab_l(lambda v: A @ v, b, 1e-30, k, ell=2)
        assert c["status"] == info.status == ENOCONV and int(c["iter"]) == info.iters == k
        assert np.linalg.norm(x - xo) / np.linalg.norm(xo) < bound, k


def test_bicgstab2_first_cycle_scalars(H):
    """FIN_BL_INIT and the first BiCG step by hand: beta = 0 in the first
    cycle (alpha = 0), alpha = rho / gamma, beta = alpha rho1 / rho0."""
    c = Ctl(H, tol=1e-10)
    c.fin("BB_FULL", 1.0)
    c.fin("BL_INIT", 1.0, 0.8, 0.2)
    assert c.cplx("bl_beta") == 0 and c.cplx("rho_old") == complex(0.8, 0.2)
    assert c.cplx("bl_g1") == 0 and c.cplx("bl_g2") == 0 and c["done"] == 0
    c.fin("BL_ALPHA", 0.4, -0.2)
    al = complex(0.8, 0.2) / complex(0.4, -0.2)
    assert abs(c.cplx("balpha") - al) < 1e-15
    c.fin("BL_BETA", 0.3, 0.1)
    assert abs(c.cplx("bl_beta") - al * complex(0.3, 0.1) / complex(0.8, 0.2)) < 1e-15
    assert c.cplx("rho_old") == complex(0.3, 0.1)
    c.fin("BL_ALPHA", 0.5, 0.0)
    c.fin_v("BL_TAU", 2.0, 0.4, 0.2, 1.0, -0.6)
    assert c.cplx("bl_tau") == complex(0.2, 0.1) and c.cplx("bl_gp1") == complex(0.5, -0.3)
    c.fin("BL_OMEGA", 4.0, 1.0, 2.0)
    assert c.cplx("bl_gp2") == complex(0.25, 0.5) and c.cplx("omega") == complex(0.25, 0.5)
    assert abs(c.cplx("bl_g1") - (complex(0.5, -0.3) - complex(0.2, 0.1) * complex(0.25, 0.5))) < 1e-15
    c.fin("BL_RES", 0.5, 0.1, 0.0)
    assert c["iter"] == 2 and c["done"] == 0
    # next cycle: rho0 = -omega rho0, beta = alpha rho1 / rho0
    rho0 = -complex(0.25, 0.5) * complex(0.3, 0.1)
    assert abs(c.cplx("bl_beta") - c.cplx("balpha") * complex(0.1, 0.0) / rho0) < 1e-15


def test_bicgstab2_degenerate_cycles(H):
    """r_1 = 0 or r_2' = 0 ends the cycle without the polynomial step
    (omega kept, g = 0); gamma = 0 and omega = 0 are breakdowns; a NaN total
    is reported; convergence wins over a breakdown."""
    def cycle(c, tau_totals, omega_totals):
        c.fin("BL_ALPHA", 1.0, 0.0)
        c.fin("BL_BETA", 0.5, 0.0)
        c.fin("BL_ALPHA", 1.0, 0.0)
        c.fin_v("BL_TAU", *tau_totals)
        c.fin("BL_OMEGA", *omega_totals)

    for tau_totals, omega_totals in [((0.0, 0.0, 0.0, 0.0, 0.0), (1.0, 0.5, 0.0)),
                                     ((1.0, 0.2, 0.0, 0.3, 0.0), (0.0, 0.0, 0.0))]:
        c = Ctl(H, tol=1e-10)
        c.fin("BB_FULL", 1.0)
        c.fin("BL_INIT", 1.0, 1.0, 0.0)
        cycle(c, tau_totals, omega_totals)
        assert c["bl_skip"] == 1 and c["status"] == 0
        assert c.cplx("omega") == 1.0 and c.cplx("bl_g1") == 0 and c.cplx("bl_g2") == 0
        assert c.cplx("bl_gp1") == 0 and c.cplx("bl_gp2") == 0
        c.fin("BL_RES", 0.5, 0.2, 0.0)
        assert c["done"] == 0 and c["iter"] == 2
        cycle(c, (1.0, 0.2, 0.0, 0.3, 0.0), (2.0, 1.0, 0.0))     # an ordinary cycle clears the skip
        assert c["bl_skip"] == 0 and c.cplx("omega") == 0.5
    c = Ctl(H, tol=1e-10)
    c.fin("BB_FULL", 1.0)
    c.fin("BL_INIT", 1.0, 1.0, 0.0)
    c.fin("BL_ALPHA", 0.0, 0.0)                                  # gamma = <rt, u_1> = 0
    assert c["status"] == EBREAKDOWN and c["done"] == 1
    c = Ctl(H, tol=1e-10)
    c.fin("BB_FULL", 1.0)
    c.fin("BL_INIT", 1.0, 1.0, 0.0)
    cycle(c, (1.0, 0.2, 0.0, 0.3, 0.0), (2.0, 0.0, 0.0))         # omega = gp2 = 0
    c.fin("BL_RES", 0.5, 0.2, 0.0)
    assert c["status"] == EBREAKDOWN
    c = Ctl(H, tol=1e-10)
    c.fin("BB_FULL", 1.0)
    c.fin("BL_INIT", 1.0, 1.0, 0.0)
    cycle(c, (1.0, 0.2, 0.0, 0.3, 0.0), (2.0, 0.0, 0.0))
    c.fin("BL_RES", 1e-22, 0.0, 0.0)
    assert c["status"] == 0 and c["done"] == 1
    c = Ctl(H, tol=1e-10)
    c.fin("BB_FULL", 1.0)
    c.fin("BL_INIT", 1.0, 1.0, 0.0)
    c.fin("BL_ALPHA", 1.0, 0.0)
    c.fin("BL_BETA", 0.5, 0.0)
    c.fin("BL_ALPHA", 1.0, 0.0)
    c.fin_v("BL_TAU", 1.0, 0.2, 0.0, float("nan"), 0.0)
    assert c["status"] == ENONFINITE and c["done"] == 1
    c = Ctl(H, tol=1e-10, iter_limit=2)
    c.fin("BB_FULL", 1.0)
    c.fin("BL_INIT", 1.0, 1.0, 0.0)
    cycle(c, (1.0, 0.2, 0.0, 0.3, 0.0), (2.0, 1.0, 0.0))
    c.fin("BL_RES", 0.5, 0.2, 0.0)
    assert c["status"] == ENOCONV and c["iter"] == 2


def test_eo_residual_scalars_leave_the_solve_alone(H):
    """FIN_BBHAT and FIN_EO_RR only record ||bhat||^2 and the even half of
    ||b - M x||^2: no other field of the control block changes."""
    c = Ctl(H, tol=1e-10)
    c.fin("BB_FULL", 4.0)
    c.fin("CG_ZZ", 1.0)
    before = {n: c[n] for n in ("bb", "thresh", "rr", "zz", "iter", "done", "status", "true_rr")}
    c.fin("BBHAT", 2.5)
    c.fin("TRUE_RR", 3e-20)
    c.fin("EO_RR", 2e-20)
    assert c["bbh"] == 2.5 and c["eo_rr"] == 2e-20 and c["true_rr"] == 3e-20
    before["true_rr"] = 3e-20
    assert {n: c[n] for n in before} == before


def test_multishift_sequence_matches_oracle(H):
    """The library's multi-shift iteration (w = (A + s0) p_base with
    <p, w> -> FIN_MS_ALPHA; x_i += alpha_i p_i; r -= alpha w -> FIN_MS_BETA;
    p_i = zeta_i r + beta_i p_i) against the oracle's multishift_cg."""
    A, b = dense_system(20, 3, hermitian=True)
    shifts = [0.3, 0.0, 0.05, 1.0, 0.05]
    n = len(shifts)
    base = int(np.argmin(shifts))
    c = Ctl(H, n=n, tol=1e-11, shifts=shifts)
    c.fin("MS_INIT", nrm2(b), idx=base)
    xs = [np.zeros_like(b) for _ in range(n)]
    ps = [b.copy() for _ in range(n)]
    r = b.copy()
    while not all(c.get("done", i) for i in range(n)):
        w = A @ ps[base] + shifts[base] * ps[base]
        c.fin("MS_ALPHA", nrm2(w), np.vdot(w, ps[base]).real, 0.0, idx=base)
        for i in range(n):
            if not c.get("done", i):
                xs[i] = xs[i] + c.get("alpha", i) * ps[i]
        r = r - c.get("alpha", base) * w
        c.fin("MS_BETA", nrm2(r), idx=base)
        for i in range(n):
            if not c.get("done", i) or c.get("iter", i) == c.get("iter", base):
                # p_i of a system finished in this iteration is no longer used
                ps[i] = c.get("zeta", i) * r + c.get("beta", i) * ps[i]
        assert c.get("iter", base) < 500
    xo, out = S.multishift_cg(lambda v: A @ v, b, shifts, 1e-11, 500)
    for i in range(n):
        assert c.get("status", i) == 0
        assert int(c.get("iter", i)) == out[i][0]
        assert np.linalg.norm(xs[i] - xo[i]) / np.linalg.norm(xo[i]) < 1e-12
        res = np.linalg.norm(b - A @ xs[i] - shifts[i] * xs[i]) / np.linalg.norm(b)
        assert res < 1e-10


# ---------------------------------------------------------------------------
# Mixed precision: reliable updates, stagnation, outer steps, fall back


def mixed_start(c, rr=1.0):
    c.fin("BB_FULL", 1.0)
    c.fin("RR_INIT", rr)
    c.fin("CG_ZZ", 1.0)


def test_reliable_update_trigger(H):
    c = Ctl(H, tol=1e-10, delta=0.1)
    mixed_start(c)
    c.fin("CG_ALPHA", 2.0)
    c.fin("CG_RR", 0.5)                       # not below delta^2 * max
    assert c["update"] == 0 and c["rr_max"] == 1.0
    c.fin("CG_BETA", 0.6)
    c.fin("CG_RR", 0.009)                     # below 0.01 * rr_max: update
    assert c["update"] == 1 and c["reset_p"] == 0
    c.fin("RU_RR", 0.0095)                    # FP64 residual after the update
    assert c["nupdates"] == 1 and c["rr_max"] == 0.0095 and c["last_upd_iter"] == 2
    assert c["nstag"] == 0 and c["done"] == 0
    c.fin("CG_BETA", 0.3)
    assert c["update"] == 0 and abs(c["beta"] - 0.3 / 0.6) < 1e-15
    # the recursion reaching tol also asks for an update; only the FP64 residual stops
    c.fin("CG_RR", 1e-21)
    assert c["update"] == 1 and c["done"] == 0
    c.fin("RU_RR", 5e-21)
    assert c["done"] == 1 and c["status"] == 0


def test_stagnation_window_restarts_direction(H):
    c = Ctl(H, tol=1e-10, delta=0.1, stag_window=3)
    mixed_start(c)
    for rr in (0.9, 0.85):
        c.fin("CG_RR", rr)
        assert c["update"] == 0
        c.fin("CG_BETA", 0.5)
    c.fin("CG_RR", 0.8)                       # three iterations without an update
    assert c["update"] == 1 and c["reset_p"] == 1 and c["nstag"] == 1
    c.fin("RU_RR", 0.79)
    assert c["nstag"] == 1                    # not counted twice
    c.fin("CG_BETA", 0.5)
    assert c["beta"] == 0.0 and c["reset_p"] == 0 and c["update"] == 0
    c.fin("CG_RR", 0.7)
    c.fin("CG_BETA", 0.4)
    assert c["beta"] > 0.0


def test_fp64_residual_not_falling_is_a_stagnation(H):
    c = Ctl(H, tol=1e-10, delta=0.1)
    mixed_start(c, rr=1.0)
    c.fin("CG_RR", 0.005)
    c.fin("RU_RR", 0.004)
    assert c["nstag"] == 0
    c.fin("CG_BETA", 0.5)
    c.fin("CG_RR", 1e-5)
    c.fin("RU_RR", 0.0041)                    # FP64 residual above the previous update's
    assert c["nstag"] == 1 and c["reset_p"] == 1
    c.fin("CG_BETA", 0.5)
    assert c["beta"] == 0.0


@pytest.mark.parametrize("fallback_ok", [0, 1])
def test_fall_back_after_max_stagnations(H, fallback_ok):
    c = Ctl(H, tol=1e-10, delta=0.1, stag_window=1, max_stag=2, fallback_ok=fallback_ok)
    mixed_start(c)
    c.fin("CG_RR", 0.5)                       # stagnation 1 (window of one iteration)
    c.fin("RU_RR", 0.5)
    assert c["nstag"] == 1 and c["done"] == 0
    c.fin("CG_BETA", 0.5)
    c.fin("CG_RR", 0.3)                       # stagnation 2
    c.fin("RU_RR", 0.3)
    assert c["nstag"] == 2
    if fallback_ok:
        assert c["done"] == 1 and c["status"] == H.ctl_status_fallback()
    else:
        assert c["done"] == 0 and c["status"] == 0


def test_outer_step_at_tol_inner(H):
    c = Ctl(H, tol=1e-12, delta=1e-3, tol_inner=1e-2)
    mixed_start(c, rr=4.0)
    c.fin("CG_RR", 5e-4)                      # above tol_inner^2 * 4 = 4e-4 and delta^2 * 4
    assert c["update"] == 0
    c.fin("CG_BETA", 0.5)
    c.fin("CG_RR", 3e-5)                      # below 4e-4 (above delta^2 * 4): the outer step ends
    assert c["update"] == 1 and c["outer_req"] == 1 and c["reset_p"] == 1
    c.fin("RU_RR", 3.5e-5)
    assert c["nouter"] == 1 and c["rr_outer"] == 3.5e-5 and c["outer_req"] == 0 and c["nstag"] == 0
    c.fin("CG_BETA", 0.5)
    assert c["beta"] == 0.0


def test_iteration_limit_and_nonfinite(H):
    c = Ctl(H, tol=1e-10, delta=0.1, iter_limit=2)
    mixed_start(c)
    c.fin("CG_RR", 0.9)
    c.fin("CG_BETA", 0.5)
    c.fin("CG_RR", 0.8)
    assert c["status"] == ENOCONV and c["done"] == 1
    c = Ctl(H, tol=1e-10, delta=0.1)
    mixed_start(c)
    c.fin("CG_RR", float("nan"))
    assert c["status"] == ENONFINITE


def test_mixed_cgnr_with_float32_inner_converges(H):
    """The mixed launch sequence with the inner vectors rounded to FP32
    (x_low, r_low, p_low, w_low, z_low) and FP64 reliable updates (x += x_low,
    r = b - A x in FP64, r_low = r): the control block alone drives it to
    the FP64 tolerance."""
    A, b = dense_system(32, 4)
    A32 = A.astype(np.complex64)
    lo = lambda v: v.astype(np.complex64)  # noqa: E731
    c = Ctl(H, tol=1e-12, delta=0.1)
    c.fin("BB_FULL", nrm2(b))
    x = np.zeros_like(b)
    r = b - A @ x
    c.fin("RR_INIT", nrm2(r))
    rl, xl = lo(r), np.zeros(b.shape, np.complex64)
    zl = A32.conj().T @ rl
    c.fin("CG_ZZ", nrm2(zl))
    pl = zl.copy()
    while not c["done"]:
        wl = A32 @ pl
        c.fin("CG_ALPHA", nrm2(wl))
        a = np.float32(c["alpha"])
        xl = xl + a * pl
        rl = rl - a * wl
        c.fin("CG_RR", nrm2(rl))
        if c["done"]:
            break
        if c["update"]:
            x = x + xl
            xl[:] = 0
            r = b - A @ x
            c.fin("RU_RR", nrm2(r))
            if c["done"]:
                break
            rl = lo(r)
        zl = A32.conj().T @ rl
        c.fin("CG_BETA", nrm2(zl))
        pl = zl + np.float32(c["beta"]) * pl
        assert c["iter"] < 500
    assert c["status"] == 0 and c["nupdates"] >= 2
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) <= 1e-12


def test_chunk_sizing(H):
    """The host loop's estimate of the iterations left: ||r||^2 falling by
    0.8 per iteration from 1 to 1e-20 needs ceil(log(1e-20 / rr) / log 0.8)
    more; no estimate without a decrease or a second read-back; 0 once below
    the threshold; the next chunk covers what the chunk in flight does not,
    between 1 and the full chunk."""
    left = H.chunk_iterations_left
    rr_prev, rr = 0.8 ** 10, 0.8 ** 18
    assert left(rr_prev, 10, rr, 18, 1e-20) == int(np.ceil(np.log(1e-20 / rr) / np.log(0.8)))
    assert left(rr_prev, 10, rr, 18, 1e-20) == 189
    assert left(rr, 18, rr_prev, 26, 1e-20) == -1        # increasing
    assert left(rr, 18, rr, 26, 1e-20) == -1             # stalled
    assert left(-1.0, -1, rr, 18, 1e-20) == -1           # first read-back
    assert left(rr_prev, 10, rr, 10, 1e-20) == -1        # no iteration in between
    assert left(rr_prev, 10, 1e-21, 18, 1e-20) == 0      # already below
    assert left(rr_prev, 10, rr, 18, 0.0) == -1          # b = 0 has no threshold to reach
    nxt = H.chunk_next
    assert nxt(-1, 8, 8) == 8
    assert nxt(100, 8, 8) == 8
    assert nxt(10, 8, 8) == 3
    assert nxt(3, 8, 8) == 1
    assert nxt(0, 0, 8) == 1
