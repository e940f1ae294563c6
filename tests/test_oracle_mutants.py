"""Planted mistakes in a copy of the oracle's C source are caught by the pins.

Each case compiles a mutated copy of oracle/wilson_oracle.c (CPU only) and
runs the operator pins of tests/pins.py against it; at least one pin must
fail.  This shows the pins constrain every part of the operator: projector
signs, link direction and adjoint, link site, boundary phase, a dropped
direction, the gamma matrices, the twisted-mass term and kappa.
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
