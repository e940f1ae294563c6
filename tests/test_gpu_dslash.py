"""GPU parity of the Dslash family against the FP64 oracle.

Every case runs the HIP kernels through the C ABI on seeded inputs and
compares, site by site, with the oracle on the same inputs.  FP64 must agree
to 1e-13 per site (relative, with an RMS floor); FP32 and FP16 storage are
held to 1e-5 and 1e-2.
"""

import math

import numpy as np
import pytest

from gpu_util import site_rel_err
from lattice_inputs import gauge_field, gaussian_spinor
from oracle import wilson as W

pytestmark = pytest.mark.gpu

TOL = {64: 1e-13, 32: 1e-5, 16: 1e-2}

# several tiles (128 sites per block) plus ragged tails; non-cubic shapes; 2^4
LATTICES = [
    ((2, 2, 2, 2), (0.0, 0.0, 0.0, math.pi)),
    ((4, 6, 8, 2), (0.0, 0.0, 0.0, math.pi)),
    ((6, 4, 6, 10), (0.3, -0.7, 1.1, math.pi + 0.2)),
    ((8, 8, 6, 6), (0.0, 0.0, 0.0, math.pi)),
    # rows of 16 sites: row tiles of 4 or 6 x-rows, 2 or 3 y-chunks (y-chunk groups)
    ((32, 12, 4, 6), (0.0, 0.4, 0.0, math.pi)),
]


# launch configurations every full-M case is checked in: memory order with
# and without the XCD remap, and row tiles in t-fastest order
LAUNCHES = [dict(block=128, swizzle=1, order=0), dict(block=64, swizzle=0, order=0),
            dict(block=192, swizzle=1, order=1), dict(block=64, swizzle=0, order=1),
            dict(block=256, swizzle=1, order=4), dict(block=128, swizzle=0, order=3),
            dict(block=64, swizzle=1, order=1, ygroup=3), dict(block=128, swizzle=0, order=1, ygroup=2)]


@pytest.fixture(scope="module")
def mods():
    import torch
    from paper_1411_5219_amd import fields, lqcd
    assert torch.cuda.is_available()
    return torch, fields, lqcd


def _setup(L4, theta, seed=0, kind="haar", eps=0.4, nrhs=None):
    U = gauge_field(L4, kind, eps=eps, seed=1000 + seed)
    psi = gaussian_spinor(L4, seed=2000 + seed, nrhs=nrhs)
    return U, psi


@pytest.mark.parametrize("L4,theta", LATTICES)
@pytest.mark.parametrize("prec,recon", [(64, 18), (64, 12), (32, 18), (32, 12), (16, 12)])
@pytest.mark.parametrize("dagger", [0, 1])
def test_full_M(mods, L4, theta, prec, recon, dagger):
    torch, fields, lqcd = mods
    kappa, mu = 0.13, 0.05
    U, psi = _setup(L4, theta)
    print(f"\n[case] full M L={L4} prec={prec} recon={recon} dagger={dagger}", flush=True)
    lat = fields.Lattice(L4, theta)
    Ud = lat.gauge(U, prec, recon)
    inp = lat.spinor(psi, prec)
    ref = W.apply_M(U, psi, L4, theta, kappa, mu, dagger=bool(dagger))
    saved = lqcd.lqcd_get_launch(lqcd.KERNEL_DSLASH, prec)
    try:
        for cfg in LAUNCHES:
            lqcd.lqcd_set_launch(lqcd.KERNEL_DSLASH, prec, **cfg)
            out = lat.empty(lqcd.FIELD_SPINOR_FULL, prec)
            lqcd.dslash_apply(lat.g, lqcd.op(kappa, mu, prec, recon), Ud, inp, out, dagger=dagger)
            err = site_rel_err(lat.unpack(out, prec), ref)
            assert err <= TOL[prec], (cfg, err)
    finally:
        lqcd.lqcd_set_launch(lqcd.KERNEL_DSLASH, prec, **saved)


@pytest.mark.parametrize("L4,theta", LATTICES[1:3])
@pytest.mark.parametrize("parity", [0, 1])
@pytest.mark.parametrize("dagger", [0, 1])
def test_eo_hop(mods, L4, theta, parity, dagger):
    torch, fields, lqcd = mods
    U, psi = _setup(L4, theta, seed=1, kind="exp")
    print(f"\n[case] hop L={L4} parity={parity} dagger={dagger}", flush=True)
    lat = fields.Lattice(L4, theta)
    Ud = lat.gauge(U, 64, 18)
    full = lat.spinor(psi, 64)
    src = lat.parity_view(full, 1 - parity)
    out = lat.empty(lqcd.FIELD_SPINOR_PARITY, 64)
    lqcd.dslash_eo_apply(lat.g, lqcd.op(0.16, 0.0), Ud, src, out, parity, lqcd.OP_HOP, dagger)
    # place the parity result into a full field to unpack it
    both = lat.zeros(lqcd.FIELD_SPINOR_FULL, 64)
    pb = lat.nbytes(lqcd.FIELD_SPINOR_PARITY, 64)
    both.view(2, pb)[parity].copy_(out)
    got = W.mask(lat.unpack(both, 64), L4, parity)
    ref = W.hop_eo(U, psi, L4, theta, parity, dagger=bool(dagger))
    assert site_rel_err(got[W.parity(L4) == parity], ref[W.parity(L4) == parity]) <= 1e-13


@pytest.mark.parametrize("L4,theta", LATTICES)
@pytest.mark.parametrize("dagger", [0, 1])
@pytest.mark.parametrize("prec,recon", [(64, 18), (32, 12), (16, 12)])
def test_schur(mods, L4, theta, dagger, prec, recon):
    torch, fields, lqcd = mods
    kappa, mu = 0.16, 0.005
    U, psi = _setup(L4, theta, seed=2, kind="exp")
    print(f"\n[case] schur L={L4} prec={prec} dagger={dagger}", flush=True)
    lat = fields.Lattice(L4, theta)
    o = lqcd.op(kappa, mu, prec, recon)
    Ud = lat.gauge(U, prec, recon)
    full = lat.spinor(W.mask(psi, L4, 0), prec)
    src = lat.parity_view(full, 0, prec)
    out = lat.empty(lqcd.FIELD_SPINOR_PARITY, prec)
    ws = lat.workspace(o)
    lqcd.dslash_eo_apply(lat.g, o, Ud, src, out, 0, lqcd.OP_SCHUR, dagger, ws=ws)
    both = lat.zeros(lqcd.FIELD_SPINOR_FULL, prec)
    pb = lat.nbytes(lqcd.FIELD_SPINOR_PARITY, prec)
    both.view(2, pb)[0].copy_(out)
    got = lat.unpack(both, prec)
    ref = W.schur(U, W.mask(psi, L4, 0), L4, theta, kappa, mu, dagger=bool(dagger))
    ev = W.parity(L4) == 0
    assert site_rel_err(got[ev], ref[ev]) <= TOL[prec]


@pytest.mark.parametrize("prec,recon", [(64, 18), (32, 12), (16, 12)])
@pytest.mark.parametrize("tile,group,lanes", [(1, 0, 1), (2, 0, 1), (4, 0, 1), (1, 4, 1), (2, 2, 1), (4, 2, 1),
                                              (1, 16, 1), (1, 0, 4), (1, 0, 8), (1, 0, 16)])
def test_multi_rhs_equals_single(mods, prec, recon, tile, group, lanes):
    """A right-hand-side tile applies each link to several right-hand sides
    with the same per-RHS operations, so every RHS of a batch (5 RHS: full
    tiles plus a ragged one) equals its single-RHS application to rounding:
    different template instances may contract multiply-adds differently, which
    can flip the last bit of an FP32 result or the rounding of a stored half.
    With the right-hand sides across lanes (4 lanes: two tiles, the second
    ragged; 8 or 16 requested: one tile of 8 lanes, 3 of them idle) each lane
    runs the one-right-hand-side code on its own field."""
    torch, fields, lqcd = mods
    L4, theta = (6, 4, 6, 10), (0.0, 0.0, 0.0, math.pi)
    U, psi = _setup(L4, theta, seed=3, kind="exp", nrhs=5)
    print(f"\n[case] multi-rhs full M nrhs=5 prec={prec} tile={tile} group={group} lanes={lanes}", flush=True)
    lat = fields.Lattice(L4, theta)
    o = lqcd.op(0.16, 0.005, prec, recon)
    Ud = lat.gauge(U, prec, recon)
    inp = lat.spinor(psi, prec)
    saved = lqcd.lqcd_get_launch(lqcd.KERNEL_DSLASH_RHS, prec)
    try:
        lqcd.lqcd_set_launch(lqcd.KERNEL_DSLASH_RHS, prec,
                             **dict(saved, order=1, rhs_tile=tile, rhs_group=group, rhs_lanes=lanes))
        out = lat.empty(lqcd.FIELD_SPINOR_FULL, prec, nrhs=5)
        lqcd.dslash_apply(lat.g, o, Ud, inp, out, nrhs=5)
        got = lat.unpack(out, prec, nrhs=5)
        for k in range(5):
            one = lat.spinor(psi[k], prec)
            o1 = lat.empty(lqcd.FIELD_SPINOR_FULL, prec)
            lqcd.dslash_apply(lat.g, o, Ud, one, o1)
            err = site_rel_err(got[k], lat.unpack(o1, prec))
            assert err <= {64: 1e-15, 32: 1e-6, 16: 2e-3}[prec], (k, err)
    finally:
        lqcd.lqcd_set_launch(lqcd.KERNEL_DSLASH_RHS, prec, **saved)
        lqcd.lqcd_tune_cache_clear()


@pytest.mark.parametrize("prec,recon", [(64, 18), (32, 12), (16, 12)])
@pytest.mark.parametrize("dagger", [0, 1])
def test_rhs_lanes_16_against_oracle(mods, prec, recon, dagger):
    """16 right-hand sides across 16 lanes (blocks of two x-rows of 8 sites:
    256 lanes, every wave full) on the even-odd hop and the Schur complement,
    each right-hand side against the oracle."""
    torch, fields, lqcd = mods
    L4, theta = (16, 8, 4, 6), (0.2, 0.0, 0.0, math.pi)
    U, psi = _setup(L4, theta, seed=8, kind="exp", nrhs=16)
    print(f"\n[case] 16 rhs across lanes prec={prec} dagger={dagger}", flush=True)
    lat = fields.Lattice(L4, theta)
    kappa, mu = 0.16, 0.005
    o = lqcd.op(kappa, mu, prec, recon)
    Ud = lat.gauge(U, prec, recon)
    full = lat.spinor(psi, prec)
    even = lat.parity_view(full, 0, prec, nrhs=16)
    odd = lat.parity_view(full, 1, prec, nrhs=16)
    pb = lat.nbytes(lqcd.FIELD_SPINOR_PARITY, prec)
    saved = lqcd.lqcd_get_launch(lqcd.KERNEL_DSLASH_RHS, prec)
    try:
        lqcd.lqcd_set_launch(lqcd.KERNEL_DSLASH_RHS, prec, 256, 1, 1, 1, 0, 1, 16)
        hop = lat.zeros(lqcd.FIELD_SPINOR_PARITY, prec, nrhs=16)
        lqcd.dslash_eo_apply(lat.g, o, Ud, odd, hop, 0, lqcd.OP_HOP, dagger, nrhs=16)
        sch = lat.zeros(lqcd.FIELD_SPINOR_PARITY, prec, nrhs=16)
        lqcd.dslash_eo_apply(lat.g, o, Ud, even, sch, 0, lqcd.OP_SCHUR, dagger, nrhs=16, ws=lat.workspace(o))
        ev = W.parity(L4) == 0
        for name, buf in (("hop", hop), ("schur", sch)):
            f = lat.zeros(lqcd.FIELD_SPINOR_FULL, prec, nrhs=16)
            f.view(16, 2, pb)[:, 0, :] = buf.view(16, pb)
            got = lat.unpack(f, prec, nrhs=16)
            for k in range(16):
                if name == "hop":
                    ref = W.hop_eo(U, psi[k], L4, theta, 0, dagger=bool(dagger))
                else:
                    ref = W.schur(U, W.mask(psi[k], L4, 0), L4, theta, kappa, mu, dagger=bool(dagger))
                assert site_rel_err(got[k][ev], ref[ev]) <= TOL[prec], (name, k)
    finally:
        lqcd.lqcd_set_launch(lqcd.KERNEL_DSLASH_RHS, prec, **saved)


@pytest.mark.parametrize("prec,recon", [(64, 18), (32, 12), (16, 12)])
def test_rhs_autotune(mods, prec, recon):
    """The right-hand-side autotuner keeps the XCD remap and block order,
    installs one of the block requests and compiled tiles and groups in the
    several-right-hand-side slot (the single-RHS slot untouched), and the
    tuned even-odd hop of 6 right-hand sides still equals the oracle's hop of
    each."""
    torch, fields, lqcd = mods
    L4, theta = (8, 6, 10, 4), (0.0, 0.0, 0.0, math.pi)
    U, psi = _setup(L4, theta, seed=4, kind="exp", nrhs=6)
    print(f"\n[case] rhs autotune prec={prec}", flush=True)
    lat = fields.Lattice(L4, theta)
    o = lqcd.op(0.16, 0.005, prec, recon)
    Ud = lat.gauge(U, prec, recon)
    src = lat.parity_view(lat.spinor(psi, prec), 1, prec, nrhs=6)
    saved = lqcd.lqcd_get_launch(lqcd.KERNEL_DSLASH_RHS, prec)
    single = lqcd.lqcd_get_launch(lqcd.KERNEL_DSLASH, prec)
    try:
        scratch = lat.empty(lqcd.FIELD_SPINOR_PARITY, prec, nrhs=6)
        best, us = lqcd.lqcd_autotune_dslash_rhs(lat.g, o, Ud, src, scratch, 6, reps=3)
        now = lqcd.lqcd_get_launch(lqcd.KERNEL_DSLASH_RHS, prec)
        assert now == best and us > 0
        cached, cus, found = lqcd.lqcd_tune_cache_get(lqcd.KERNEL_DSLASH_RHS, prec, recon, lat.g, 6)
        assert found and cached == best and cus > 0  # kept for this lattice and nrhs
        assert lqcd.lqcd_get_launch(lqcd.KERNEL_DSLASH, prec) == single
        assert {k: now[k] for k in ("swizzle", "order")} == {k: saved[k] for k in ("swizzle", "order")}
        assert now["block"] in (128, 192, 256)
        assert now["rhs_tile"] in ((1, 2) if prec == 64 else (1, 2, 4)) and now["rhs_group"] in (0, 2, 4, 8, 16)
        assert now["rhs_lanes"] in (1, 2, 4, 8, 16)
        out = lat.zeros(lqcd.FIELD_SPINOR_FULL, prec, nrhs=6)
        pb = lat.nbytes(lqcd.FIELD_SPINOR_PARITY, prec)
        even = lat.zeros(lqcd.FIELD_SPINOR_PARITY, prec, nrhs=6)
        lqcd.dslash_eo_apply(lat.g, o, Ud, src, even, 0, nrhs=6)
        out.view(6, 2, pb)[:, 0, :] = even.view(6, pb)
        got = lat.unpack(out, prec, nrhs=6)
        for k in range(6):
            ref = W.hop_eo(U, psi[k], L4, theta, 0)
            assert site_rel_err(got[k], ref) <= TOL[prec], k
    finally:
        lqcd.lqcd_set_launch(lqcd.KERNEL_DSLASH_RHS, prec, **saved)


def test_pack_roundtrip(mods):
    torch, fields, lqcd = mods
    L4 = (6, 4, 6, 10)
    psi = gaussian_spinor(L4, seed=5, nrhs=2)
    lat = fields.Lattice(L4)
    for prec, tol in [(64, 0.0), (32, 1e-7), (16, 1e-3)]:
        back = lat.unpack(lat.spinor(psi, prec), prec, nrhs=2)
        assert site_rel_err(back, psi) <= tol, prec


def test_deterministic(mods):
    torch, fields, lqcd = mods
    L4, theta = (8, 8, 6, 6), (0.0, 0.0, 0.0, math.pi)
    U, psi = _setup(L4, theta, seed=4, kind="exp")
    lat = fields.Lattice(L4, theta)
    Ud = lat.gauge(U)
    inp = lat.spinor(psi)
    # zero-filled so the padding sites past V/2 compare equal too
    a = lat.zeros(lqcd.FIELD_SPINOR_FULL, 64)
    b = lat.zeros(lqcd.FIELD_SPINOR_FULL, 64)
    o = lqcd.op(0.16, 0.005)
    lqcd.dslash_apply(lat.g, o, Ud, inp, a)
    lqcd.dslash_apply(lat.g, o, Ud, inp, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("L4", [(24, 24, 24, 8), (48, 48, 48, 12)])
def test_full_size_fp64(mods, L4):
    """The production shapes (24^3x8 and 48^3x12), exp(i eps H) links at
    eps = 0.4: the whole FP64 full-lattice M against the oracle, and FP32/12,
    FP16/12 against their bounds."""
    torch, fields, lqcd = mods
    theta = (0.0, 0.0, 0.0, math.pi)
    kappa, mu = 0.16, 0.005
    print(f"\n[case] full-size M L={L4}", flush=True)
    U = gauge_field(L4, "exp", eps=0.4, seed=1002)
    psi = gaussian_spinor(L4, seed=2002)
    ref = W.apply_M(U, psi, L4, theta, kappa, mu)
    lat = fields.Lattice(L4, theta)
    for prec, recon in [(64, 18), (64, 12), (32, 12), (16, 12)]:
        Ud = lat.gauge(U, prec, recon)
        inp = lat.spinor(psi, prec)
        out = lat.empty(lqcd.FIELD_SPINOR_FULL, prec)
        lqcd.dslash_apply(lat.g, lqcd.op(kappa, mu, prec, recon), Ud, inp, out)
        err = site_rel_err(lat.unpack(out, prec), ref)
        print(f"  prec={prec} recon={recon} max site err={err:.3e}", flush=True)
        assert err <= TOL[prec]
        del Ud, inp, out
        torch.cuda.empty_cache()


def test_autotune_configs_agree(mods):
    """Every launch configuration computes each site with the same code, so
    the FP64 results of all 16 configurations are bitwise identical; the
    autotuner installs one of them."""
    torch, fields, lqcd = mods
    saved = lqcd.lqcd_get_launch(lqcd.KERNEL_DSLASH, 64)
    try:
        for L4 in ((8, 6, 10, 4), (32, 12, 4, 6)):
            theta = (0.0, 0.0, 0.0, math.pi)
            U, psi = _setup(L4, theta, seed=9, kind="exp")
            lat = fields.Lattice(L4, theta)
            o = lqcd.op(0.16, 0.005)
            Ud = lat.gauge(U)
            src = lat.parity_view(lat.spinor(psi), 1)
            outs = []
            for order, yg in ((0, 1), (1, 1), (1, 2), (1, 3), (2, 1), (5, 1)):
                for sw in (0, 1):
                    for blk in (64, 128, 192, 256):
                        lqcd.lqcd_set_launch(lqcd.KERNEL_DSLASH, 64, blk, sw, order, ygroup=yg)
                        out = lat.zeros(lqcd.FIELD_SPINOR_PARITY, 64)
                        lqcd.dslash_eo_apply(lat.g, o, Ud, src, out, 0)
                        outs.append(out)
            torch.cuda.synchronize()
            for out in outs[1:]:
                assert torch.equal(out, outs[0]), L4
            scratch = lat.zeros(lqcd.FIELD_SPINOR_PARITY, 64)
            best, us = lqcd.lqcd_autotune_dslash(lat.g, o, Ud, src, scratch, reps=3)
            assert lqcd.lqcd_get_launch(lqcd.KERNEL_DSLASH, 64) == best and us > 0
            cached, _, found = lqcd.lqcd_tune_cache_get(lqcd.KERNEL_DSLASH, 64, 18, lat.g, 1)
            assert found and cached == best
            # the cached shape is what launches on this lattice use, whatever the table says
            lqcd.lqcd_set_launch(lqcd.KERNEL_DSLASH, 64, 64, 0, 0)
            assert lqcd.lqcd_tune_cache_get(lqcd.KERNEL_DSLASH, 64, 18, lat.g, 1)[0] == best
            out = lat.zeros(lqcd.FIELD_SPINOR_PARITY, 64)
            lqcd.dslash_eo_apply(lat.g, o, Ud, src, out, 0)
            torch.cuda.synchronize()
            assert torch.equal(out, outs[0]), L4
            lqcd.lqcd_tune_cache_clear()
    finally:
        lqcd.lqcd_set_launch(lqcd.KERNEL_DSLASH, 64, **saved)
        lqcd.lqcd_tune_cache_clear()


def test_tune_cache_file_round_trip(mods, tmp_path):
    """An autotuner run on the GPU is written to the cache file under this
    device's architecture and read back after a clear."""
    import json
    torch, fields, lqcd = mods
    L4, theta = (8, 6, 10, 4), (0.0, 0.0, 0.0, math.pi)
    U, psi = _setup(L4, theta, seed=9, kind="exp")
    lat = fields.Lattice(L4, theta)
    o = lqcd.op(0.16, 0.005, 32, 12)
    Ud = lat.gauge(U, 32, 12)
    src = lat.parity_view(lat.spinor(psi, 32), 1, 32)
    saved = lqcd.lqcd_get_launch(lqcd.KERNEL_DSLASH, 32)
    print("\n[case] tune cache round trip", flush=True)
    try:
        lqcd.lqcd_tune_cache_clear()
        best, us = lqcd.lqcd_autotune_dslash(lat.g, o, Ud, src, lat.zeros(lqcd.FIELD_SPINOR_PARITY, 32), reps=3)
        path = str(tmp_path / "tune.json")
        lqcd.lqcd_tune_cache_save(path)
        entries = json.load(open(path))
        assert len(entries) == 1
        e = entries[0]
        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
        assert e["arch"] == arch and e["L"] == list(L4) and e["prec"] == 32 and e["recon"] == 12 and e["nrhs"] == 1
        assert {k: e[k] for k in best} == best and abs(e["us"] - us) < 1e-2
        lqcd.lqcd_tune_cache_clear()
        lqcd.lqcd_tune_cache_load(path)
        assert lqcd.lqcd_tune_cache_get(lqcd.KERNEL_DSLASH, 32, 12, lat.g, 1)[0] == best
    finally:
        lqcd.lqcd_set_launch(lqcd.KERNEL_DSLASH, 32, **saved)
        lqcd.lqcd_tune_cache_clear()


def test_device_memory(mods):
    torch, fields, lqcd = mods
    clock_khz, bus_bits = lqcd.lqcd_device_memory(0)
    assert clock_khz > 0 and bus_bits > 0
    with pytest.raises(lqcd.LqcdError):
        lqcd.lqcd_device_memory(torch.cuda.device_count())
    # the failed query leaves nothing behind for the next launch
    lat = fields.Lattice((4, 4, 4, 4))
    out = lat.empty(lqcd.FIELD_SPINOR_FULL, 64)
    lqcd.lqcd_pack_spinor(lat.g, 64, 1, torch.zeros((lat.V, 4, 3), dtype=torch.complex128, device="cuda"), out)
    torch.cuda.synchronize()
