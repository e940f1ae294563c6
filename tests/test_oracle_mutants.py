"""Planted mistakes in a copy of the oracle's C source are caught by the pins.

Each case compiles a mutated copy of oracle/wilson_oracle.c (CPU only) and
runs the operator pins of tests/pins.py against it; at least one pin must
fail.  This shows the pins constrain every part of the operator: projector
signs, link direction and adjoint, link site, boundary phase, a dropped
direction, the gamma matrices, the twisted-mass term and kappa.  The
staggered oracle (oracle/staggered_oracle.c) gets the same treatment with
tests/pins_staggered.py: staggered phases, the 1/2, the backward sign, link
adjoint and site, boundary phases, a dropped direction and the mass term.
"""

import ctypes
import os
import subprocess

import numpy as np
import pytest

import pins
from oracle.build import SRC

MUTANTS = {
    "fwd_projector_sign": ("const double sg = dir == 0 ? -s : s;", "const double sg = dir == 0 ? s : s;"),
    "bwd_projector_sign": ("const double sg = dir == 0 ? -s : s;", "const double sg = dir == 0 ? -s : -s;"),
    "bwd_link_not_adjoint": ("conj(link[3 * b + a])", "link[3 * a + b]"),
    "bwd_link_no_conj": ("conj(link[3 * b + a])", "link[3 * b + a]"),
    "fwd_link_transposed": ("? link[3 * a + b] :", "? link[3 * b + a] :"),
    "fwd_link_wrong_site": ("link = U + ((int64_t)mu * V + i) * 9;",
                            "link = U + ((int64_t)mu * V + site_index(cn, L)) * 9;"),
    "bwd_link_wrong_site": ("link = U + ((int64_t)mu * V + site_index(cn, L)) * 9;",
                            "link = U + ((int64_t)mu * V + i) * 9;"),
    "bwd_phase_not_conj": ("phase = conj(ph[mu]);", "phase = ph[mu];"),
    "fwd_phase_wrong_edge": ("if (c[mu] == L[mu] - 1) phase = ph[mu];", "if (c[mu] == 0) phase = ph[mu];"),
    "dropped_t_direction": ("for (int mu = 0; mu < 4; ++mu) {\n            for (int dir",
                            "for (int mu = 0; mu < 3; ++mu) {\n            for (int dir"),
    "gamma_lower_block_sign": ("g[k - 1][2 + a][b] = I * s[a][b];", "g[k - 1][2 + a][b] = -I * s[a][b];"),
    "twisted_mass_sign": ("(dagger ? -1.0 : 1.0) * 2.0 * I", "(dagger ? 1.0 : -1.0) * 2.0 * I"),
    "twisted_mass_no_dagger_flip": ("(dagger ? -1.0 : 1.0) * 2.0 * I", "(1.0) * 2.0 * I"),
    "missing_kappa": ("- kappa * o[3 * a + col]", "- o[3 * a + col]"),
    "spin_colour_swap": ("t += u * pn[3 * sp + b];", "t += u * pn[3 * b + (sp % 3)];"),
}


def _build_mutant(tmp_path, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique: {old!r}"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-fopenmp", "-fPIC", "-shared", str(path), "-o", str(lib), "-lm"],
                   check=True)
    return ctypes.CDLL(str(lib))


def _bind(lib):
    dp = ctypes.POINTER(ctypes.c_double)

    def ptr(a):
        return a.ctypes.data_as(dp)

    def geom(L, th):
        return (ctypes.c_int * 4)(*L), np.ascontiguousarray(np.asarray(th, float))

    def hop(U, psi, L, th, dag):
        U, psi = np.ascontiguousarray(U), np.ascontiguousarray(psi)
        out = np.empty_like(psi)
        Li, t = geom(L, th)
        lib.oracle_hop(Li, ptr(t), ptr(U), ptr(psi), ptr(out), ctypes.c_int(int(dag)))
        return out

    def apply_M(U, psi, L, th, k, m, dag):
        U, psi = np.ascontiguousarray(U), np.ascontiguousarray(psi)
        out = np.empty_like(psi)
        Li, t = geom(L, th)
        lib.oracle_apply_M(Li, ptr(t), ctypes.c_double(k), ctypes.c_double(m), ptr(U), ptr(psi), ptr(out),
                           ctypes.c_int(int(dag)))
        return out

    return hop, apply_M


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    hop, apply_M = _bind(_build_mutant(tmp_path, old, new))
    errs = pins.all_pins(hop, apply_M)
    worst = max(errs.values())
    assert worst > 1e-6, f"mutant {name} passed every pin: {errs}"


# ---------------------------------------------------------------------------
# The staggered oracle (oracle/staggered_oracle.c) against tests/pins_staggered.py

import pins_staggered  # noqa: E402
from oracle.build import STAG_SRC  # noqa: E402

STAG_MUTANTS = {
    "eta_includes_own_direction": ("for (int nu = 0; nu < mu; ++nu) s += c[nu];",
                                   "for (int nu = 0; nu <= mu; ++nu) s += c[nu];"),
    "eta_from_later_directions": ("for (int nu = 0; nu < mu; ++nu) s += c[nu];",
                                  "for (int nu = mu + 1; nu < 4; ++nu) s += c[nu];"),
    "missing_half": ("acc[a] += 0.5 * e * f * t;", "acc[a] += e * f * t;"),
    "bwd_sign": ("acc[a] -= 0.5 * e * f * t;", "acc[a] += 0.5 * e * f * t;"),
    "eta_on_bwd_only": ("acc[a] += 0.5 * e * f * t;", "acc[a] += 0.5 * f * t;"),
    "bwd_link_not_adjoint": ("conj(u[3 * b + a])", "u[3 * a + b]"),
    "bwd_link_no_conj": ("conj(u[3 * b + a])", "u[3 * b + a]"),
    "fwd_link_transposed": ("t += u[3 * a + b] * pn[b];", "t += u[3 * b + a] * pn[b];"),
    "fwd_link_wrong_site": ("const cplx *u = U + ((int64_t)mu * V + i) * 9;",
                            "const cplx *u = U + ((int64_t)mu * V + site_index(cn, L)) * 9;"),
    "bwd_link_wrong_site": ("const cplx *u = U + ((int64_t)mu * V + j) * 9;",
                            "const cplx *u = U + ((int64_t)mu * V + i) * 9;"),
    "bwd_phase_not_conj": ("c[mu] == 0 ? conj(ph[mu]) : 1.0", "c[mu] == 0 ? ph[mu] : 1.0"),
    "fwd_phase_wrong_edge": ("c[mu] == L[mu] - 1 ? ph[mu] : 1.0", "c[mu] == 0 ? ph[mu] : 1.0"),
    "dropped_t_direction": ("for (int mu = 0; mu < 4; ++mu) {\n            const double e",
                            "for (int mu = 0; mu < 3; ++mu) {\n            const double e"),
    "mass_no_dagger_flip": ("const double sd = dagger ? -1.0 : 1.0;", "const double sd = 1.0;"),
    "missing_mass": ("out[k] = mass * in[k] + sd * out[k];", "out[k] = in[k] + sd * out[k];"),
}


def _build_stag_mutant(tmp_path, old, new):
    src = open(STAG_SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique: {old!r}"
    path = tmp_path / "stag_mutant.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / "libstagmutant.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-fopenmp", "-fPIC", "-shared", str(path), "-o", str(lib), "-lm"],
                   check=True)
    return ctypes.CDLL(str(lib))


def _bind_stag(lib):
    dp = ctypes.POINTER(ctypes.c_double)

    def ptr(a):
        return a.ctypes.data_as(dp)

    def geom(L, th):
        return (ctypes.c_int * 4)(*L), np.ascontiguousarray(np.asarray(th, float))

    def hop(U, phi, L, th):
        U, phi = np.ascontiguousarray(U), np.ascontiguousarray(phi)
        out = np.empty_like(phi)
        Li, t = geom(L, th)
        lib.stag_oracle_hop(Li, ptr(t), ptr(U), ptr(phi), ptr(out))
        return out

    def apply_M(U, phi, L, th, m, dag):
        U, phi = np.ascontiguousarray(U), np.ascontiguousarray(phi)
        out = np.empty_like(phi)
        Li, t = geom(L, th)
        lib.stag_oracle_apply_M(Li, ptr(t), ctypes.c_double(m), ptr(U), ptr(phi), ptr(out), ctypes.c_int(int(dag)))
        return out

    return hop, apply_M


@pytest.mark.parametrize("name", sorted(STAG_MUTANTS))
def test_staggered_mutant_is_caught(name, tmp_path):
    old, new = STAG_MUTANTS[name]
    hop, apply_M = _bind_stag(_build_stag_mutant(tmp_path, old, new))
    errs = pins_staggered.all_stag_pins(hop, apply_M)
    worst = max(errs.values())
    assert worst > 1e-6, f"mutant {name} passed every pin: {errs}"
