"""Parity at the benchmark's full sizes, in the launch configuration bench.py times.

Solves are certified by the oracle's operator on the returned x (FP64 true
residual, per right-hand side and per system); the force kernel is compared
with the oracle on sampled links (bulk and every boundary); the staggered
solvers by the oracle's staggered operator.  Inputs follow the benchmark's
recipes and seeds.
"""

import math

import numpy as np
import pytest

from gpu_util import site_rel_err
from lattice_inputs import gauge_field, gaussian_spinor, point_source
from oracle import force as OF
from oracle import staggered as OS
from oracle import wilson as W

pytestmark = pytest.mark.gpu

THETA = (0.0, 0.0, 0.0, math.pi)
KAPPA, MU, TOL = 0.16, 0.005, 1e-10
DELTA = {64: 0.1, 32: 0.001, 16: 0.05}  # the reliable-update thresholds bench.py uses
L48 = (48, 48, 48, 12)
L32 = (32, 32, 32, 8)


@pytest.fixture(scope="module")
def mods():
    import torch
    from paper_1411_5219_amd import fields, lqcd
    assert torch.cuda.is_available()
    return torch, fields, lqcd


@pytest.fixture(scope="module")
def big(mods):
    """48^3 x 12, exp(i eps H) links at eps = 0.4, one Gaussian source (the
    benchmark's single-source workload), with the device copies."""
    torch, fields, lqcd = mods
    print("\n[setup] 48^3x12 inputs", flush=True)
    U = gauge_field(L48, "exp", eps=0.4, seed=1002)
    b = gaussian_spinor(L48, seed=2002)
    lat = fields.Lattice(L48, THETA)
    return U, b, lat, lat.gauge(U), lat.spinor(b)


@pytest.mark.parametrize("inner", [(64, 18), (32, 12), (16, 12)])
def test_single_source_48x12_certified(mods, big, inner):
    torch, fields, lqcd = mods
    U, b, lat, Ud, bd = big
    print(f"\n[case] 48^3x12 solve inner={inner}", flush=True)
    o = lqcd.op(KAPPA, MU)
    p = lqcd.solve_params(tol=TOL, maxiter=100000, eo=1, inner_prec=inner[0], inner_recon=inner[1],
                          delta_reliable=DELTA[inner[0]])
    xd = lat.zeros(lqcd.FIELD_SPINOR_FULL, 64)
    rc, info = lqcd.cg_solve(lat.g, o, Ud, bd, xd, p, lat.workspace(o, p))
    assert rc == lqcd.OK, info
    x = lat.unpack(xd)
    tr = W.true_residual(U, x, b, L48, THETA, KAPPA, MU)
    print(f"  iters={info[0]['iters']} updates={info[0]['reliable_updates']} true={tr:.3e}", flush=True)
    assert tr <= TOL
    assert abs(tr - info[0]["true_resid"]) <= 1e-3 * TOL


def test_fp64_links12_48x12_certified(mods, big):
    """The FP64 solve on 12-real FP64 links (third row rebuilt in FP64)."""
    torch, fields, lqcd = mods
    U, b, lat, Ud, bd = big
    print("\n[case] 48^3x12 fp64 solve, 12-real links", flush=True)
    o = lqcd.op(KAPPA, MU, 64, 12)
    p = lqcd.solve_params(tol=TOL, maxiter=100000, eo=1, inner_prec=64)
    xd = lat.zeros(lqcd.FIELD_SPINOR_FULL, 64)
    rc, info = lqcd.cg_solve(lat.g, o, lat.gauge(U, 64, 12), bd, xd, p, lat.workspace(o, p))
    assert rc == lqcd.OK, info
    tr = W.true_residual(U, lat.unpack(xd), b, L48, THETA, KAPPA, MU)
    assert tr <= TOL and abs(tr - info[0]["true_resid"]) <= 1e-3 * TOL


def test_force_48x12_sampled(mods, big):
    """The force kernel on the full lattice (Gaussian X and Z) against the
    oracle's per-link force on sampled links: random bulk links and links on
    every boundary face."""
    torch, fields, lqcd = mods
    U, b, lat, Ud, bd = big
    print("\n[case] 48^3x12 force sampled", flush=True)
    X = gaussian_spinor(L48, seed=2102)
    Z = gaussian_spinor(L48, seed=2103)
    _, g5 = W.gammas()
    Wf = np.einsum("st,vtc->vsc", g5, Z)
    V = lat.V
    Fd = torch.full((4, V, 3, 3), float("nan"), dtype=torch.complex128, device=lat.device)
    lqcd.tm_force(lat.g, lqcd.op(KAPPA, MU), Ud, lat.spinor(X), lat.spinor(Wf), Fd)
    torch.cuda.synchronize()
    F = Fd.cpu().numpy()
    assert np.all(np.isfinite(F))
    rng = np.random.default_rng(7)
    Lx, Ly, Lz, Lt = L48
    sites = list(rng.integers(0, V, 48))
    for mu in range(4):  # a site on the last slice of each direction (the link crosses the boundary)
        c = [int(v) for v in rng.integers(0, 12, 4)]
        c[mu] = L48[mu] - 1
        sites.append(c[0] + Lx * (c[1] + Ly * (c[2] + Lz * c[3])))
    sites.append(V - 1)
    for mu in range(4):
        got = np.stack([F[mu, y] for y in sites])
        ref = np.stack([OF.force_link(U, X, Z, L48, THETA, KAPPA, mu, y) for y in sites])
        assert site_rel_err(got, ref, ncomp=9) <= 1e-12, mu


@pytest.mark.parametrize("inner", [(64, 18), (32, 12), (16, 12)])
def test_single_source_32x8_certified(mods, inner):
    """32^3 x 8 (the smaller mixed-precision lattice), one Gaussian source:
    plain FP64 and FP32 / FP16-storage inner solves with FP64 reliable
    updates, each certified by the oracle's M, in bench.py's configuration."""
    torch, fields, lqcd = mods
    print(f"\n[case] 32^3x8 solve inner={inner}", flush=True)
    U = gauge_field(L32, "exp", eps=0.4, seed=1002)
    b = gaussian_spinor(L32, seed=2002)
    lat = fields.Lattice(L32, THETA)
    o = lqcd.op(KAPPA, MU)
    p = lqcd.solve_params(tol=TOL, maxiter=100000, eo=1, inner_prec=inner[0], inner_recon=inner[1],
                          delta_reliable=DELTA[inner[0]])
    xd = lat.zeros(lqcd.FIELD_SPINOR_FULL, 64)
    rc, info = lqcd.cg_solve(lat.g, o, lat.gauge(U), lat.spinor(b), xd, p, lat.workspace(o, p))
    assert rc == lqcd.OK, info
    tr = W.true_residual(U, lat.unpack(xd), b, L32, THETA, KAPPA, MU)
    print(f"  iters={info[0]['iters']} updates={info[0]['reliable_updates']} true={tr:.3e}", flush=True)
    assert tr <= TOL and abs(tr - info[0]["true_resid"]) <= 1e-3 * TOL


def test_bicgstab2_32x8_certified(mods):
    """BiCGStab(2) on the same 32^3 x 8 system (where BiCGStab stalls):
    converges to 1e-10 (about 5300 BiCG steps), certified by the oracle's M,
    with the even-odd residual it reports equal to the oracle's."""
    torch, fields, lqcd = mods
    print("\n[case] 32^3x8 bicgstab2", flush=True)
    U = gauge_field(L32, "exp", eps=0.4, seed=1002)
    b = gaussian_spinor(L32, seed=2002)
    lat = fields.Lattice(L32, THETA)
    o = lqcd.op(KAPPA, MU)
    p = lqcd.solve_params(tol=TOL, maxiter=20000, eo=1, bicgstab_ell=2)
    xd = lat.zeros(lqcd.FIELD_SPINOR_FULL, 64)
    rc, info = lqcd.bicgstab_solve(lat.g, o, lat.gauge(U), lat.spinor(b), xd, p, lat.workspace(o, p))
    print(f"  rc={rc} steps={info[0]['iters']} t={info[0]['seconds']:.2f}s", flush=True)
    assert rc == lqcd.OK, info
    x = lat.unpack(xd)
    tr = W.true_residual(U, x, b, L32, THETA, KAPPA, MU)
    assert tr <= TOL and abs(tr - info[0]["true_resid"]) <= 1e-3 * TOL
    bhat = W.eo_source(U, b, L32, THETA, KAPPA, MU)
    r = bhat - W.schur(U, W.mask(x, L32, 0), L32, THETA, KAPPA, MU)
    eo = float(np.linalg.norm(r.ravel()) / np.linalg.norm(bhat.ravel()))
    assert abs(info[0]["eo_resid"] - eo) <= 1e-3 * eo


@pytest.mark.parametrize("sc", [(0, 0), (2, 1)])
def test_fp16_point_source_32x8_certified(mods, sc):
    """FP16-storage inner solve on a unit point source at the origin (the
    multi-right-hand-side workload's parameters, 32^3 x 8): the per-site
    FP16 scale carries the source's dynamic range; certified by the oracle."""
    torch, fields, lqcd = mods
    print(f"\n[case] 32^3x8 fp16 point source spin/colour={sc}", flush=True)
    U = gauge_field(L32, "exp", eps=0.4, seed=1003)
    b = point_source(L32, *sc)
    lat = fields.Lattice(L32, THETA)
    o = lqcd.op(KAPPA, MU)
    p = lqcd.solve_params(tol=TOL, maxiter=100000, eo=1, inner_prec=16, inner_recon=12, delta_reliable=DELTA[16])
    xd = lat.zeros(lqcd.FIELD_SPINOR_FULL, 64)
    rc, info = lqcd.cg_solve(lat.g, o, lat.gauge(U), lat.spinor(b), xd, p, lat.workspace(o, p))
    assert rc == lqcd.OK, info
    tr = W.true_residual(U, lat.unpack(xd), b, L32, THETA, KAPPA, MU)
    print(f"  iters={info[0]['iters']} updates={info[0]['reliable_updates']} stag={info[0]['stagnations']} "
          f"fallbacks={info[0]['fallbacks']} true={tr:.3e}", flush=True)
    assert tr <= TOL


def test_multi_rhs_32x8_certified(mods):
    """16 right-hand sides (12 unit point sources at the origin, one per spin
    and colour, and 4 Gaussian) on 32^3 x 8, FP32/12 inner: each certified."""
    torch, fields, lqcd = mods
    print("\n[case] 32^3x8 16-rhs solve", flush=True)
    U = gauge_field(L32, "exp", eps=0.4, seed=1003)
    b = np.concatenate([np.stack([point_source(L32, s, c) for s in range(4) for c in range(3)]),
                        gaussian_spinor(L32, seed=2003, nrhs=4)])
    n = b.shape[0]
    lat = fields.Lattice(L32, THETA)
    o = lqcd.op(KAPPA, MU)
    p = lqcd.solve_params(tol=TOL, maxiter=100000, eo=1, inner_prec=32, inner_recon=12, nrhs=n,
                          delta_reliable=DELTA[32])
    xd = lat.zeros(lqcd.FIELD_SPINOR_FULL, 64, nrhs=n)
    rc, infos = lqcd.cg_solve(lat.g, o, lat.gauge(U), lat.spinor(b), xd, p, lat.workspace(o, p))
    assert rc == lqcd.OK, infos
    x = lat.unpack(xd, nrhs=n)
    for k in range(n):
        tr = W.true_residual(U, x[k], b[k], L32, THETA, KAPPA, MU)
        assert tr <= TOL, (k, tr)


@pytest.mark.parametrize("persistent", [0, 1])
def test_uneven_batch_full_size_certified(mods, persistent):
    """The benchmark's uneven batch: 16^3, 20^3, 24^3 and 32^3 x 8 with their
    own eps and kappa, 4 Gaussian sources each, one batched CGNR (replayed
    from a HIP graph, or one cooperative persistent launch); all 16 solutions
    certified."""
    torch, fields, lqcd = mods
    print(f"\n[case] uneven batch full size persistent={persistent}", flush=True)
    systems = [((16, 16, 16, 8), 0.3, 0.15), ((20, 20, 20, 8), 0.4, 0.16), ((24, 24, 24, 8), 0.5, 0.155),
               ((32, 32, 32, 8), 0.4, 0.16)]
    nrhs = 4
    s = torch.cuda.Stream()
    geoms, ops, Us, bs, xs, host = [], [], [], [], [], []
    for i, (L4, eps, kappa) in enumerate(systems):
        U = gauge_field(L4, "exp", eps=eps, seed=1004 + 10 * i)
        b = gaussian_spinor(L4, seed=2004 + 10 * i, nrhs=nrhs)
        lat = fields.Lattice(L4, THETA)
        geoms.append(lat.g)
        ops.append(lqcd.op(kappa, MU))
        Us.append(lat.gauge(U))
        bs.append(lat.spinor(b))
        xs.append(lat.zeros(lqcd.FIELD_SPINOR_FULL, 64, nrhs=nrhs))
        host.append((L4, kappa, U, b, lat))
    p = lqcd.solve_params(tol=TOL, maxiter=100000, eo=1, inner_prec=32, inner_recon=12, nrhs=nrhs, use_graph=1,
                          delta_reliable=DELTA[32], persistent=persistent)
    ws = torch.empty(lqcd.lqcd_workspace_bytes_batch(geoms, ops, p), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        rc, infos = lqcd.cg_solve_batch(geoms, ops, Us, bs, xs, p, ws, stream=s)
    torch.cuda.synchronize()
    assert rc == lqcd.OK, infos
    if persistent:
        launches = [i["persistent_launches"] for inf in infos for i in inf]
        print(f"  launches={max(launches)} iters={[max(i['iters'] for i in inf) for inf in infos]}", flush=True)
        assert min(launches) >= 1
    for i, (L4, kappa, U, b, lat) in enumerate(host):
        x = lat.unpack(xs[i], 64, nrhs=nrhs)
        for k in range(nrhs):
            tr = W.true_residual(U, x[k], b[k], L4, THETA, kappa, MU)
            assert tr <= TOL, (i, k, tr)


def test_staggered_48x12_certified(mods, big):
    """Staggered CG at m = 0.1 and the 8-shift multi-shift CG on the
    benchmark's 48^3 x 12 links and source (the first spin component of the
    Wilson source as the colour vector), certified by the oracle's operators."""
    torch, fields, lqcd = mods
    U, b, lat, Ud, bd = big
    print("\n[case] 48^3x12 staggered cg + multishift", flush=True)
    mass = 0.1
    chi = np.ascontiguousarray(b[:, 0, :])
    o = lqcd.stag_op(mass)
    p = lqcd.solve_params(tol=TOL, maxiter=100000, eo=1, inner_prec=64, use_graph=1)
    cd = lat.colour(chi)
    xd = lat.zeros(lqcd.FIELD_COLOUR_FULL, 64)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        rc, info = lqcd.stag_cg_solve(lat.g, o, Ud, cd, xd, p, lat.stag_workspace(o), stream=s)
    torch.cuda.synchronize()
    assert rc == lqcd.OK, info
    x = lat.unpack_colour(xd)
    tr = OS.true_residual(U, x, chi, L48, THETA, mass)
    assert tr <= TOL, tr

    shifts = [0.0, 1e-4, 4.6e-4, 2.2e-3, 1e-2, 4.6e-2, 0.22, 1.0]
    n = len(shifts)
    be = lat.colour_parity(cd, 0)
    xs = lat.zeros(lqcd.FIELD_COLOUR_PARITY, 64, nrhs=n)
    with torch.cuda.stream(s):
        rc, infos = lqcd.stag_multishift_solve(lat.g, o, Ud, be, xs, shifts, p, lat.stag_workspace(o, n), stream=s)
    torch.cuda.synchronize()
    assert rc == lqcd.OK, infos
    pb = lat.nbytes(lqcd.FIELD_COLOUR_PARITY, 64)
    e_sites = OS.mask(np.ones((lat.V, 3)), L48, 0)[:, 0] != 0
    b_e = OS.mask(chi, L48, 0)
    bn = np.linalg.norm(b_e.ravel())
    for i, sh in enumerate(shifts):
        # the even-parity solution as a full-lattice field (odd half zero)
        full = torch.zeros(2 * pb, dtype=torch.uint8, device=lat.device)
        full[:pb] = xs[i * pb:(i + 1) * pb]
        xi = lat.unpack_colour(full)
        assert np.all(xi[~e_sites] == 0)
        r = b_e - (OS.normal_e(U, xi, L48, THETA, mass) + sh * xi)
        res = np.linalg.norm(r.ravel()) / bn
        assert res <= TOL, (i, sh, res, infos[i])
        assert abs(res - infos[i]["true_resid"]) <= 1e-3 * TOL, (i, res, infos[i])
