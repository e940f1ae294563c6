"""GPU parity of the staggered operator and its solvers against the FP64 oracle.

The HIP kernels run through the C ABI on seeded inputs; the operator is
compared site by site with the oracle (FP64 1e-13, FP32 1e-5, FP16 1e-2 per
site, relative with an RMS floor); the solvers are certified by the
oracle's operator (true residual) and compared with the oracle's solves.
"""

import math

import numpy as np
import pytest

import pins_staggered as PS
from gpu_util import site_rel_err
from lattice_inputs import gauge_field
from oracle import solvers as SV
from oracle import staggered as S

pytestmark = pytest.mark.gpu

TOL = {64: 1e-13, 32: 1e-5, 16: 1e-2}
PRECS = [(64, 18), (64, 12), (32, 18), (32, 12), (16, 12)]
LATTICES = [
    ((2, 2, 2, 2), (0.0, 0.0, 0.0, math.pi)),
    ((4, 6, 8, 2), (0.0, 0.0, 0.0, math.pi)),
    ((6, 4, 6, 10), (0.3, -0.7, 1.1, math.pi + 0.2)),
    ((8, 8, 6, 6), (0.0, 0.0, 0.0, math.pi)),
]
LAUNCHES = [dict(block=128, swizzle=1, order=0), dict(block=64, swizzle=0, order=0),
            dict(block=192, swizzle=1, order=1), dict(block=256, swizzle=1, order=4)]


@pytest.fixture(scope="module")
def mods():
    import torch
    from paper_1411_5219_amd import fields, lqcd
    assert torch.cuda.is_available()
    return torch, fields, lqcd


def _setup(L4, seed=0, kind="haar", eps=0.4):
    U = gauge_field(L4, kind, eps=eps, seed=1000 + seed)
    chi = PS.colour_field(L4, 2000 + seed)
    return U, chi


@pytest.mark.parametrize("L4,theta", LATTICES)
@pytest.mark.parametrize("prec,recon", PRECS)
@pytest.mark.parametrize("dagger", [0, 1])
def test_full_M(mods, L4, theta, prec, recon, dagger):
    torch, fields, lqcd = mods
    mass = 0.13
    U, chi = _setup(L4)
    print(f"\n[case] stag full M L={L4} prec={prec} recon={recon} dagger={dagger}", flush=True)
    lat = fields.Lattice(L4, theta)
    Ud = lat.gauge(U, prec, recon)
    inp = lat.colour(chi, prec)
    ref = S.apply_M(U, chi, L4, theta, mass, dagger=bool(dagger))
    saved = lqcd.lqcd_get_launch(lqcd.KERNEL_STAG, prec)
    try:
        for cfg in LAUNCHES:
            lqcd.lqcd_set_launch(lqcd.KERNEL_STAG, prec, **cfg)
            out = lat.empty(lqcd.FIELD_COLOUR_FULL, prec)
            lqcd.stag_apply(lat.g, lqcd.stag_op(mass, prec, recon), Ud, inp, out, dagger=dagger)
            err = site_rel_err(lat.unpack_colour(out, prec), ref, 3)
            assert err <= TOL[prec], (cfg, err)
    finally:
        lqcd.lqcd_set_launch(lqcd.KERNEL_STAG, prec, **saved)


@pytest.mark.parametrize("L4,theta", LATTICES[1:3])
@pytest.mark.parametrize("parity", [0, 1])
@pytest.mark.parametrize("prec,recon", [(64, 18), (32, 12), (16, 12)])
def test_eo_hop_and_normal(mods, L4, theta, parity, prec, recon):
    torch, fields, lqcd = mods
    mass = 0.21
    U, chi = _setup(L4, seed=1, kind="exp")
    print(f"\n[case] stag eo hop L={L4} parity={parity} prec={prec}", flush=True)
    lat = fields.Lattice(L4, theta)
    o = lqcd.stag_op(mass, prec, recon)
    Ud = lat.gauge(U, prec, recon)
    full = lat.colour(chi, prec)
    src = lat.colour_parity(full, 1 - parity, prec)
    out = lat.zeros(lqcd.FIELD_COLOUR_FULL, prec)
    pb = lat.nbytes(lqcd.FIELD_COLOUR_PARITY, prec)
    lqcd.stag_eo_apply(lat.g, o, Ud, src, out[parity * pb:(parity + 1) * pb], parity)
    ref = S.hop_eo(U, chi, L4, theta, parity)
    assert site_rel_err(lat.unpack_colour(out, prec), ref, 3) <= TOL[prec]
    if parity == 0:
        even = lat.colour_parity(full, 0, prec)
        outn = lat.zeros(lqcd.FIELD_COLOUR_FULL, prec)
        ws = lat.empty(lqcd.FIELD_COLOUR_PARITY, prec)
        lqcd.stag_eo_apply(lat.g, o, Ud, even, outn[:pb], 0, lqcd.OP_NORMAL, ws=ws)
        refn = S.normal_e(U, S.mask(chi, L4, 0), L4, theta, mass)
        assert site_rel_err(lat.unpack_colour(outn, prec), refn, 3) <= TOL[prec] * 10


@pytest.mark.parametrize("prec", [64, 32, 16])
def test_pack_roundtrip(mods, prec):
    torch, fields, lqcd = mods
    L4 = (6, 4, 6, 10)
    lat = fields.Lattice(L4)
    chi = PS.colour_field(L4, 5)
    back = lat.unpack_colour(lat.colour(chi, prec), prec)
    assert site_rel_err(back, chi, 3) <= {64: 0.0, 32: 1e-7, 16: 1e-3}[prec]


@pytest.mark.parametrize("L4,theta", [((48, 48, 48, 12), (0.0, 0.0, 0.0, math.pi))])
def test_full_size_hop(mods, L4, theta):
    """The bench shape in full: the FP64/18 even hop of every site against
    the oracle (the oracle's C loops take about a second here)."""
    torch, fields, lqcd = mods
    U = gauge_field(L4, "exp", eps=0.4, seed=1002)
    chi = PS.colour_field(L4, 2002)
    print(f"\n[case] stag full-size hop L={L4}", flush=True)
    lat = fields.Lattice(L4, theta)
    Ud = lat.gauge(U)
    full = lat.colour(chi)
    pb = lat.nbytes(lqcd.FIELD_COLOUR_PARITY, 64)
    out = lat.zeros(lqcd.FIELD_COLOUR_FULL, 64)
    lqcd.stag_eo_apply(lat.g, lqcd.stag_op(0.1), Ud, lat.colour_parity(full, 1), out[:pb], 0)
    ref = S.hop_eo(U, chi, L4, theta, 0)
    assert site_rel_err(lat.unpack_colour(out), ref, 3) <= 1e-13


SOLVE_CASES = [((4, 4, 4, 4), "haar", 0.2, 1e-12), ((8, 8, 8, 4), "exp", 0.05, 1e-10)]


@pytest.mark.parametrize("L4,kind,mass,tol", SOLVE_CASES)
@pytest.mark.parametrize("use_graph", [0, 1])
def test_cg_solve(mods, L4, kind, mass, tol, use_graph):
    torch, fields, lqcd = mods
    theta = (0.0, 0.0, 0.0, math.pi)
    U, b = _setup(L4, seed=3, kind=kind)
    print(f"\n[case] stag cg L={L4} mass={mass} graph={use_graph}", flush=True)
    lat = fields.Lattice(L4, theta)
    o = lqcd.stag_op(mass)
    Ud = lat.gauge(U)
    bd = lat.colour(b)
    xd = lat.zeros(lqcd.FIELD_COLOUR_FULL, 64)
    p = lqcd.solve_params(tol=tol, maxiter=20000, eo=1, inner_prec=64, use_graph=use_graph)
    ws = lat.stag_workspace(o)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        rc, info = lqcd.stag_cg_solve(lat.g, o, Ud, bd, xd, p, ws, stream=s)
    torch.cuda.synchronize()
    assert rc == 0, info
    x = lat.unpack_colour(xd)
    tr = S.true_residual(U, x, b, L4, theta, mass)
    assert tr <= tol, (tr, info)
    assert abs(tr - info["true_resid"]) <= 1e-3 * tol + 1e-15
    assert math.isnan(info["eo_resid"])  # reported for the Wilson even-odd solves only
    xo, oinfo = SV.stag_solve(U, b, L4, theta, mass, tol)
    assert np.linalg.norm((x - xo).ravel()) / np.linalg.norm(xo.ravel()) < 1e3 * tol / mass
    assert abs(info["iters"] - oinfo.iters) <= 2


def test_cg_zero_source(mods):
    torch, fields, lqcd = mods
    L4 = (4, 4, 4, 4)
    lat = fields.Lattice(L4)
    U, _ = _setup(L4)
    o = lqcd.stag_op(0.1)
    xd = lat.empty(lqcd.FIELD_COLOUR_FULL, 64).fill_(7)
    rc, info = lqcd.stag_cg_solve(lat.g, o, lat.gauge(U), lat.zeros(lqcd.FIELD_COLOUR_FULL, 64), xd,
                                  lqcd.solve_params(tol=1e-10), lat.stag_workspace(o))
    assert rc == 0 and info["iters"] == 0
    assert not np.any(lat.unpack_colour(xd))


@pytest.mark.parametrize("shifts", [[0.0, 0.01, 0.1, 1.0], [0.3, 0.0, 0.02, 0.02, 2.5]])
@pytest.mark.parametrize("use_graph", [0, 1])
def test_multishift(mods, shifts, use_graph):
    torch, fields, lqcd = mods
    L4, theta, mass, tol = (8, 8, 8, 4), (0.0, 0.0, 0.0, math.pi), 0.05, 1e-10
    U, chi = _setup(L4, seed=7, kind="exp")
    b = S.mask(chi, L4, 0)
    print(f"\n[case] stag multishift shifts={shifts} graph={use_graph}", flush=True)
    lat = fields.Lattice(L4, theta)
    o = lqcd.stag_op(mass)
    Ud = lat.gauge(U)
    be = lat.colour_parity(lat.colour(b), 0)
    pb = lat.nbytes(lqcd.FIELD_COLOUR_PARITY, 64)
    n = len(shifts)
    xd = lat.zeros(lqcd.FIELD_COLOUR_PARITY, 64, nrhs=n)
    p = lqcd.solve_params(tol=tol, maxiter=20000, eo=1, inner_prec=64, use_graph=use_graph)
    ws = lat.stag_workspace(o, n)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        rc, infos = lqcd.stag_multishift_solve(lat.g, o, Ud, be, xd, shifts, p, ws, stream=s)
    torch.cuda.synchronize()
    assert rc == 0, infos
    A = lambda v: S.normal_e(U, v, L4, theta, mass)  # noqa: E731
    xs_ref, out_ref = SV.multishift_cg(A, b, shifts, tol, 20000)
    for i, sh in enumerate(shifts):
        full = torch.zeros(2 * pb, dtype=torch.uint8, device="cuda")
        full[:pb] = xd[i * pb:(i + 1) * pb]
        x = lat.unpack_colour(full)
        res = np.linalg.norm((b - A(x) - sh * x).ravel()) / np.linalg.norm(b.ravel())
        assert res <= tol, (i, sh, res, infos[i])
        assert abs(res - infos[i]["true_resid"]) <= 1e-3 * tol + 1e-15
        rel = np.linalg.norm((x - xs_ref[i]).ravel()) / np.linalg.norm(xs_ref[i].ravel())
        assert rel < 1e-6, (i, rel)
        if infos[i]["restarts"] == 0:  # no refinement: the shared recursion alone
            assert abs(infos[i]["iters"] - out_ref[i][0]) <= 2, (infos[i], out_ref[i])


def test_launch_shapes_bitwise_and_autotune(mods):
    """Every launch shape of the staggered hop gives the same bits (the
    per-site arithmetic does not depend on the shape); the autotuner keeps
    one of them."""
    torch, fields, lqcd = mods
    L4, theta = (8, 6, 10, 4), (0.0, 0.0, 0.0, math.pi)
    U, chi = _setup(L4, seed=9, kind="exp")
    lat = fields.Lattice(L4, theta)
    o = lqcd.stag_op(0.1)
    Ud = lat.gauge(U)
    src = lat.colour_parity(lat.colour(chi), 1)
    saved = lqcd.lqcd_get_launch(lqcd.KERNEL_STAG, 64)
    try:
        outs = []
        for order in (0, 1, 3):
            for sw in (0, 1):
                for blk in (64, 128, 192, 256):
                    lqcd.lqcd_set_launch(lqcd.KERNEL_STAG, 64, blk, sw, order)
                    out = lat.zeros(lqcd.FIELD_COLOUR_PARITY, 64)
                    lqcd.stag_eo_apply(lat.g, o, Ud, src, out, 0)
                    outs.append(out)
        torch.cuda.synchronize()
        for out in outs[1:]:
            assert torch.equal(out, outs[0])
        scratch = lat.zeros(lqcd.FIELD_COLOUR_PARITY, 64)
        best, us = lqcd.lqcd_autotune_stag(lat.g, o, Ud, src, scratch, reps=3)
        assert lqcd.lqcd_get_launch(lqcd.KERNEL_STAG, 64) == best and us > 0
        assert lqcd.lqcd_tune_cache_get(lqcd.KERNEL_STAG, 64, 18, lat.g, 1)[::2] == (best, True)
    finally:
        lqcd.lqcd_set_launch(lqcd.KERNEL_STAG, 64, **saved)
        lqcd.lqcd_tune_cache_clear()
