"""GPU solvers certified by the FP64 oracle.

The solution of M x = b is unique, so every solver variant (FP64 CGNR and
BiCGStab, full lattice or even-odd, mixed FP32 / FP16-storage with reliable
updates, several right-hand sides, graph replay) must return an x whose
true residual ||b - M x|| / ||b||, computed with the oracle's M, meets the
tolerance; on small lattices x is also compared with the oracle's solve.
"""

import math

import numpy as np
import pytest

from lattice_inputs import gauge_field, gaussian_spinor, point_source
from oracle import solvers as S
from oracle import wilson as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    import torch
    from paper_1411_5219_amd import fields, lqcd
    assert torch.cuda.is_available()
    return torch, fields, lqcd


def run_solve(mods, L4, theta, U, b, kappa, mu, method="cg", nrhs=1, stream=None, outer_recon=18, **kw):
    torch, fields, lqcd = mods
    lat = fields.Lattice(L4, theta)
    o = lqcd.op(kappa, mu, 64, outer_recon)
    if method == "bicgstab2":
        kw = dict(kw, bicgstab_ell=2)
    p = lqcd.solve_params(nrhs=nrhs, **kw)
    Ud = lat.gauge(U, 64, outer_recon)
    bd = lat.spinor(b)
    xd = lat.zeros(lqcd.FIELD_SPINOR_FULL, 64, nrhs=nrhs)
    ws = lat.workspace(o, p)
    fn = lqcd.cg_solve if method == "cg" else lqcd.bicgstab_solve
    rc, infos = fn(lat.g, o, Ud, bd, xd, p, ws, stream=stream)
    x = lat.unpack(xd, 64, nrhs=nrhs)
    return rc, infos, x


def true_res(U, x, b, L4, theta, kappa, mu):
    return W.true_residual(U, x, b, L4, theta, kappa, mu)


def eo_res(U, x, b, L4, theta, kappa, mu):
    """||bhat - Mhat x_e|| / ||bhat|| by the oracle on the returned x."""
    bhat = W.eo_source(U, b, L4, theta, kappa, mu)
    r = bhat - W.schur(U, W.mask(x, L4, 0), L4, theta, kappa, mu)
    return float(np.linalg.norm(r.ravel()) / np.linalg.norm(bhat.ravel()))


def check_eo_resid(info, U, x, b, L4, theta, kappa, mu):
    """The reported even-odd residual equals the oracle's on the returned x
    (both are rounding-limited near 1e-10: 1e-3 relative)."""
    ref = eo_res(U, x, b, L4, theta, kappa, mu)
    assert abs(info["eo_resid"] - ref) <= 1e-3 * ref + 1e-15, (info["eo_resid"], ref)


@pytest.mark.parametrize("method", ["cg", "bicgstab", "bicgstab2"])
@pytest.mark.parametrize("eo", [0, 1])
def test_config0_like_4x4x4x4(mods, method, eo):
    """Plain Wilson, Haar links, kappa = 0.12, full tolerance 1e-12."""
    L4, theta, kappa, mu = (4, 4, 4, 4), (0, 0, 0, math.pi), 0.12, 0.0
    U = gauge_field(L4, "haar", seed=1000)
    b = gaussian_spinor(L4, seed=2000)
    print(f"\n[case] 4^4 {method} eo={eo}", flush=True)
    rc, info, x = run_solve(mods, L4, theta, U, b, kappa, mu, method, tol=1e-12, maxiter=2000, eo=eo)
    assert rc == 0, info
    tr = true_res(U, x, b, L4, theta, kappa, mu)
    assert tr <= 1e-12 and abs(tr - info[0]["true_resid"]) < 1e-13
    if eo:
        check_eo_resid(info[0], U, x, b, L4, theta, kappa, mu)
    else:
        assert math.isnan(info[0]["eo_resid"])
    x_ref, _ = S.solve(U, b, L4, theta, kappa, mu, tol=1e-13, method="cgnr", eo=True)
    assert np.linalg.norm((x - x_ref).ravel()) / np.linalg.norm(x_ref.ravel()) < 1e-10


def test_dense_lu_2x2x2x2(mods):
    L4, theta, kappa, mu = (2, 2, 2, 2), (0, 0, 0, math.pi), 0.15, 0.1
    U = gauge_field(L4, "haar", seed=7)
    b = gaussian_spinor(L4, seed=8)
    x_ref = np.linalg.solve(W.dense_M(U, L4, theta, kappa, mu), b.ravel()).reshape(b.shape)
    for method in ["cg", "bicgstab", "bicgstab2"]:
        rc, info, x = run_solve(mods, L4, theta, U, b, kappa, mu, method, tol=1e-13, maxiter=500)
        assert rc == 0
        assert np.linalg.norm((x - x_ref).ravel()) / np.linalg.norm(x_ref.ravel()) < 1e-11


@pytest.mark.parametrize("inner", [(64, 18), (32, 12), (32, 18), (16, 12)])
def test_twisted_mass_eo_mixed(mods, inner):
    """Twisted mass at kappa = 0.16, mu = 0.005 on exp(i eps H) links,
    eps = 0.4 (the production parameters) on 8^3 x 4; tol 1e-10."""
    L4, theta, kappa, mu = (8, 8, 8, 4), (0, 0, 0, math.pi), 0.16, 0.005
    U = gauge_field(L4, "exp", eps=0.4, seed=1001)
    b = gaussian_spinor(L4, seed=2001)
    print(f"\n[case] 8^3x4 tm inner={inner}", flush=True)
    rc, info, x = run_solve(mods, L4, theta, U, b, kappa, mu, "cg", tol=1e-10, maxiter=20000,
                            inner_prec=inner[0], inner_recon=inner[1])
    assert rc == 0, info
    tr = true_res(U, x, b, L4, theta, kappa, mu)
    print(f"  iters={info[0]['iters']} updates={info[0]['reliable_updates']} true={tr:.2e}", flush=True)
    assert tr <= 1e-10
    check_eo_resid(info[0], U, x, b, L4, theta, kappa, mu)


@pytest.mark.parametrize("inner", [(64, 18), (32, 12), (32, 18), (16, 12)])
def test_mixed_on_12_real_fp64_links(mods, inner):
    """The FP64 system on 12-real links (third row rebuilt in FP64), plain and
    with every inner precision (the inner links are built from the 12-real
    field): certified by the oracle's M on the original 18-real links, the
    difference being rounding of the rebuilt row."""
    L4, theta, kappa, mu = (8, 8, 8, 4), (0, 0, 0, math.pi), 0.16, 0.005
    U = gauge_field(L4, "exp", eps=0.4, seed=1001)
    b = gaussian_spinor(L4, seed=2001)
    print(f"\n[case] 8^3x4 tm on FP64/12 links, inner={inner}", flush=True)
    rc, info, x = run_solve(mods, L4, theta, U, b, kappa, mu, "cg", outer_recon=12, tol=1e-10, maxiter=20000,
                            inner_prec=inner[0], inner_recon=inner[1])
    assert rc == 0, info
    tr = true_res(U, x, b, L4, theta, kappa, mu)
    assert tr <= 1e-10 and abs(tr - info[0]["true_resid"]) <= 1e-13


@pytest.mark.parametrize("use_graph", [0, 1])
def test_bicgstab_twisted_eo(mods, use_graph):
    """BiCGStab on the twisted-mass Schur complement at the production
    parameters (8^3 x 4): it must converge (the oracle's BiCGStab takes 398
    iterations here), be certified by the oracle's M and agree with the
    oracle's solve.  Two solutions with residuals r1, r2 differ by at most
    cond(M) (r1 + r2); the oracle's BiCGStab at 1e-10 and CGNR at 1e-12
    differ by 2.5e-10 on this system, so 2e-9 leaves a factor 8."""
    torch = mods[0]
    L4, theta, kappa, mu = (8, 8, 8, 4), (0, 0, 0, math.pi), 0.16, 0.005
    U = gauge_field(L4, "exp", eps=0.4, seed=1001)
    b = gaussian_spinor(L4, seed=2001)
    print(f"\n[case] 8^3x4 tm bicgstab graph={use_graph}", flush=True)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        rc, info, x = run_solve(mods, L4, theta, U, b, kappa, mu, "bicgstab", tol=1e-10, maxiter=20000,
                                stream=s, use_graph=use_graph)
    print(f"  rc={rc} iters={info[0]['iters']} restarts={info[0]['restarts']}", flush=True)
    assert rc == 0, info
    tr = true_res(U, x, b, L4, theta, kappa, mu)
    assert tr <= 1e-10 and abs(tr - info[0]["true_resid"]) <= 1e-13
    x_ref, ref_info = S.solve(U, b, L4, theta, kappa, mu, tol=1e-12, method="cgnr", eo=True)
    assert ref_info.status == 0
    assert np.linalg.norm((x - x_ref).ravel()) / np.linalg.norm(x_ref.ravel()) <= 2e-9


@pytest.mark.parametrize("eo", [0, 1])
def test_bicgstab2_iterates_match_oracle(mods, eo):
    """BiCGStab(2) stopped after k BiCG steps (ENOCONV) returns the oracle's
    BiCGStab(ell = 2) iterate after the same steps (then reconstructed, with
    eo): the device's fused launch sequence takes the published algorithm's
    steps.  Twisted mass and twisted boundaries on 4^4, where rounding is
    not amplified over a few cycles."""
    L4, theta, kappa, mu = (4, 4, 4, 4), (0.3, 0, 0, math.pi), 0.12, 0.05
    U = gauge_field(L4, "haar", seed=1002)
    b = gaussian_spinor(L4, seed=2002)
    for k in (2, 4, 8):
        print(f"\n[case] 4^4 bicgstab2 eo={eo} after {k} steps", flush=True)
        rc, info, x = run_solve(mods, L4, theta, U, b, kappa, mu, "bicgstab2", tol=1e-14, maxiter=k, eo=eo)
        x_ref, ref = S.solve(U, b, L4, theta, kappa, mu, tol=1e-14, maxiter=k, method="bicgstab_l", eo=bool(eo),
                             ell=2)
        assert ref.status == S.ENOCONV and ref.iters == k
        assert info[0]["status"] == S.ENOCONV and info[0]["iters"] == k
        err = np.linalg.norm((x - x_ref).ravel()) / np.linalg.norm(x_ref.ravel())
        print(f"  rel diff {err:.2e}", flush=True)
        assert err < 1e-12
        # x agrees to 1e-12 relative, so the residuals agree to about ||M|| times that
        assert abs(info[0]["true_resid"] - ref.true_resid) <= 1e-11


@pytest.mark.parametrize("use_graph", [0, 1])
def test_bicgstab2_twisted_eo(mods, use_graph):
    """BiCGStab(2) at the production parameters on 8^3 x 4 (where BiCGStab
    needs 398 iterations): certified by the oracle's M and within 2e-9 of the
    oracle's CGNR solution (the bound of the BiCGStab test)."""
    torch = mods[0]
    L4, theta, kappa, mu = (8, 8, 8, 4), (0, 0, 0, math.pi), 0.16, 0.005
    U = gauge_field(L4, "exp", eps=0.4, seed=1001)
    b = gaussian_spinor(L4, seed=2001)
    print(f"\n[case] 8^3x4 tm bicgstab2 graph={use_graph}", flush=True)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        rc, info, x = run_solve(mods, L4, theta, U, b, kappa, mu, "bicgstab2", tol=1e-10, maxiter=20000,
                                stream=s, use_graph=use_graph)
    print(f"  rc={rc} iters={info[0]['iters']} restarts={info[0]['restarts']}", flush=True)
    assert rc == 0, info
    tr = true_res(U, x, b, L4, theta, kappa, mu)
    assert tr <= 1e-10 and abs(tr - info[0]["true_resid"]) <= 1e-13
    check_eo_resid(info[0], U, x, b, L4, theta, kappa, mu)
    x_ref, ref_info = S.solve(U, b, L4, theta, kappa, mu, tol=1e-12, method="cgnr", eo=True)
    assert ref_info.status == 0
    assert np.linalg.norm((x - x_ref).ravel()) / np.linalg.norm(x_ref.ravel()) <= 2e-9


def test_bicgstab2_multi_rhs(mods):
    """Three right-hand sides (a point source and two Gaussians) solved
    together by BiCGStab(2): each has its own scalars and stops on its own;
    each solution is certified by the oracle's M."""
    L4, theta, kappa, mu = (8, 8, 8, 4), (0, 0, 0, math.pi), 0.16, 0.005
    U = gauge_field(L4, "exp", eps=0.4, seed=1003)
    b = np.concatenate([point_source(L4, 1, 2)[None], gaussian_spinor(L4, seed=2003, nrhs=2)])
    print("\n[case] 8^3x4 tm bicgstab2 nrhs=3", flush=True)
    rc, info, x = run_solve(mods, L4, theta, U, b, kappa, mu, "bicgstab2", nrhs=3, tol=1e-10, maxiter=20000)
    print(f"  rc={rc} iters={[i['iters'] for i in info]}", flush=True)
    assert rc == 0, info
    for i in range(3):
        tr = true_res(U, x[i], b[i], L4, theta, kappa, mu)
        assert tr <= 1e-10 and abs(tr - info[i]["true_resid"]) <= 1e-13


def test_multi_rhs_point_and_gaussian(mods):
    """12 point sources at the origin (one per spin-colour) plus 4 Gaussian
    sources, solved together; each must meet the tolerance."""
    L4, theta, kappa, mu = (8, 8, 8, 4), (0, 0, 0, math.pi), 0.16, 0.005
    U = gauge_field(L4, "exp", eps=0.4, seed=1003)
    b = np.concatenate([np.stack([point_source(L4, s, c) for s in range(4) for c in range(3)]),
                        gaussian_spinor(L4, seed=2003, nrhs=4)])
    print("\n[case] 16 rhs mixed fp32", flush=True)
    rc, info, x = run_solve(mods, L4, theta, U, b, kappa, mu, "cg", nrhs=16, tol=1e-10, maxiter=20000,
                            inner_prec=32, inner_recon=12)
    assert rc == 0, info
    for k in range(16):
        assert true_res(U, x[k], b[k], L4, theta, kappa, mu) <= 1e-10, k


@pytest.mark.parametrize("nrhs", [2, 3, 5])
@pytest.mark.parametrize("inner", [(32, 12), (16, 12)])
def test_mixed_several_rhs_counts(mods, nrhs, inner):
    """Mixed solves of 2, 3 and 5 right-hand sides (tiles of the inner
    Dslash partly filled for 3 and 5) at FP32 and FP16 inner storage: every
    solution certified by the oracle's M, and a graph-replayed solve equal to
    the direct one."""
    torch = mods[0]
    L4, theta, kappa, mu = (6, 6, 6, 4), (0.2, 0, 0, math.pi), 0.155, 0.01
    U = gauge_field(L4, "exp", eps=0.4, seed=1010 + nrhs)
    b = np.concatenate([point_source(L4, 2, 1)[None], gaussian_spinor(L4, seed=2010 + nrhs, nrhs=nrhs - 1)])
    print(f"\n[case] 6^3x4 mixed nrhs={nrhs} inner={inner}", flush=True)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        rc, info, x = run_solve(mods, L4, theta, U, b, kappa, mu, "cg", nrhs=nrhs, tol=1e-10, maxiter=20000,
                                inner_prec=inner[0], inner_recon=inner[1], stream=s)
        rcg, infog, xg = run_solve(mods, L4, theta, U, b, kappa, mu, "cg", nrhs=nrhs, tol=1e-10, maxiter=20000,
                                   inner_prec=inner[0], inner_recon=inner[1], stream=s, use_graph=1)
    print(f"  rc={rc} iters={[i['iters'] for i in info]}", flush=True)
    assert rc == 0 and rcg == 0, info
    for k in range(nrhs):
        tr = true_res(U, x[k], b[k], L4, theta, kappa, mu)
        assert tr <= 1e-10 and abs(tr - info[k]["true_resid"]) <= 1e-13, k
        check_eo_resid(info[k], U, x[k], b[k], L4, theta, kappa, mu)
    assert [i["iters"] for i in info] == [i["iters"] for i in infog]
    assert np.array_equal(x, xg)


def test_multi_rhs_matches_single(mods):
    L4, theta, kappa, mu = (4, 4, 4, 4), (0, 0, 0, math.pi), 0.16, 0.005
    U = gauge_field(L4, "exp", eps=0.4, seed=1)
    b = gaussian_spinor(L4, seed=2, nrhs=3)
    rc, info, x = run_solve(mods, L4, theta, U, b, kappa, mu, "cg", nrhs=3, tol=1e-11, maxiter=5000)
    assert rc == 0
    # the batched Dslash applies each link to a tile of right-hand sides with
    # the same per-RHS operations; the results agree to rounding
    for k in range(3):
        rc1, info1, x1 = run_solve(mods, L4, theta, U, b[k], kappa, mu, "cg", tol=1e-11, maxiter=5000)
        assert info1[0]["iters"] == info[k]["iters"]
        assert np.linalg.norm((x1 - x[k]).ravel()) / np.linalg.norm(x1.ravel()) < 1e-12


def test_graph_replay_matches_direct(mods):
    torch = mods[0]
    L4, theta, kappa, mu = (8, 8, 8, 4), (0, 0, 0, math.pi), 0.16, 0.005
    U = gauge_field(L4, "exp", eps=0.4, seed=1001)
    b = gaussian_spinor(L4, seed=2001)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        rc0, i0, x0 = run_solve(mods, L4, theta, U, b, kappa, mu, "cg", tol=1e-10, maxiter=20000,
                                inner_prec=32, inner_recon=12, stream=s)
        rc1, i1, x1 = run_solve(mods, L4, theta, U, b, kappa, mu, "cg", tol=1e-10, maxiter=20000,
                                inner_prec=32, inner_recon=12, stream=s, use_graph=1)
    assert rc0 == 0 and rc1 == 0
    assert i0[0]["iters"] == i1[0]["iters"]
    assert np.array_equal(x0, x1)


def test_edge_cases(mods):
    torch, fields, lqcd = mods
    L4, theta = (4, 4, 4, 4), (0, 0, 0, math.pi)
    U = gauge_field(L4, "haar", seed=3)
    zero = np.zeros((256, 4, 3), complex)
    rc, info, x = run_solve(mods, L4, theta, U, zero, 0.12, 0.0, "cg", tol=1e-10)
    assert rc == 0 and info[0]["iters"] == 0 and not x.any()
    bad = gaussian_spinor(L4, seed=4)
    bad[5, 1, 1] = np.nan
    rc, info, x = run_solve(mods, L4, theta, U, bad, 0.12, 0.0, "cg", tol=1e-10)
    assert rc == lqcd.ENONFINITE
    b = gaussian_spinor(L4, seed=5)
    rc, info, x = run_solve(mods, L4, theta, U, b, 0.12, 0.0, "cg", tol=1e-12, maxiter=3)
    assert rc == lqcd.ENOCONV and info[0]["iters"] == 3
    assert 0 < true_res(U, x, b, L4, theta, 0.12, 0.0) < 1


@pytest.mark.parametrize("method", ["bicgstab", "bicgstab2"])
@pytest.mark.parametrize("eo", [0, 1])
def test_edge_cases_bicgstab(mods, method, eo):
    """b = 0 returns x = 0 after no iteration; a NaN in b is ENONFINITE; a
    maxiter below what the solve needs is ENOCONV after maxiter iterations
    (BiCGStab(2) counts BiCG steps and tests once per cycle of two, so 3
    becomes 4, as in the oracle), with an x that lowered the residual."""
    torch, fields, lqcd = mods
    L4, theta = (4, 4, 4, 4), (0, 0, 0, math.pi)
    U = gauge_field(L4, "haar", seed=3)
    zero = np.zeros((256, 4, 3), complex)
    rc, info, x = run_solve(mods, L4, theta, U, zero, 0.12, 0.05, method, tol=1e-10, eo=eo)
    assert rc == 0 and info[0]["iters"] == 0 and not x.any()
    bad = gaussian_spinor(L4, seed=4)
    bad[5, 1, 1] = np.nan
    rc, info, x = run_solve(mods, L4, theta, U, bad, 0.12, 0.05, method, tol=1e-10, eo=eo)
    assert rc == lqcd.ENONFINITE
    b = gaussian_spinor(L4, seed=5)
    rc, info, x = run_solve(mods, L4, theta, U, b, 0.12, 0.05, method, tol=1e-12, maxiter=3, eo=eo)
    want = 4 if method == "bicgstab2" else 3
    assert rc == lqcd.ENOCONV and info[0]["iters"] == want
    _, ref = S.solve(U, b, L4, theta, 0.12, 0.05, tol=1e-12, maxiter=3, eo=bool(eo),
                     method="bicgstab_l" if method == "bicgstab2" else "bicgstab", ell=2)
    assert ref.status == S.ENOCONV and ref.iters == want
    assert 0 < true_res(U, x, b, L4, theta, 0.12, 0.05) < 1


def test_config1_full_size_certified(mods):
    """24^3 x 8, exp(i eps H) links at eps = 0.4, kappa = 0.16, a mu = 0.005,
    FP64 even-odd CGNR to 1e-10: the returned x is certified by the oracle's M."""
    L4, theta, kappa, mu = (24, 24, 24, 8), (0, 0, 0, math.pi), 0.16, 0.005
    U = gauge_field(L4, "exp", eps=0.4, seed=1001)
    b = gaussian_spinor(L4, seed=2001)
    print("\n[case] 24^3x8 fp64 eo cg", flush=True)
    rc, info, x = run_solve(mods, L4, theta, U, b, kappa, mu, "cg", tol=1e-10, maxiter=50000)
    tr = true_res(U, x, b, L4, theta, kappa, mu)
    print(f"  rc={rc} iters={info[0]['iters']} t={info[0]['seconds']:.3f}s true={tr:.2e}", flush=True)
    assert rc == 0 and tr <= 1e-10, info
    assert abs(tr - info[0]["true_resid"]) <= 1e-13


def test_config1_bicgstab_reports_what_it_reached(mods):
    """BiCGStab (van der Vorst) on the same 24^3 x 8 system does not reach
    1e-10: at kappa = 0.16 the Schur complement has eigenvalues on both sides
    of the imaginary axis, and the oracle's own BiCGStab stalls near 2e-2
    (1550 iterations).  Whatever the library stops with, it must say so
    truthfully: a converged status only with a certified x, otherwise
    ENOCONV or EBREAKDOWN with info.true_resid equal to the oracle's true
    residual of the returned x."""
    torch, fields, lqcd = mods
    L4, theta, kappa, mu = (24, 24, 24, 8), (0, 0, 0, math.pi), 0.16, 0.005
    U = gauge_field(L4, "exp", eps=0.4, seed=1001)
    b = gaussian_spinor(L4, seed=2001)
    print("\n[case] 24^3x8 fp64 eo bicgstab, 3000 iterations", flush=True)
    rc, info, x = run_solve(mods, L4, theta, U, b, kappa, mu, "bicgstab", tol=1e-10, maxiter=3000)
    tr = true_res(U, x, b, L4, theta, kappa, mu)
    print(f"  rc={rc} iters={info[0]['iters']} t={info[0]['seconds']:.3f}s true={tr:.2e}", flush=True)
    assert np.all(np.isfinite(x))
    assert rc == info[0]["status"]
    assert abs(tr - info[0]["true_resid"]) <= 1e-12 * max(1.0, tr)
    if rc == 0:
        assert tr <= 1e-10
    else:
        assert rc in (lqcd.ENOCONV, lqcd.EBREAKDOWN) and tr > 1e-10


def test_config1_bicgstab2(mods):
    """BiCGStab(2) on the 24^3 x 8 system where BiCGStab stalls (near 2e-2)
    must converge to 1e-10 within 10000 BiCG steps (about 4600 are needed),
    certified by the oracle's M."""
    L4, theta, kappa, mu = (24, 24, 24, 8), (0, 0, 0, math.pi), 0.16, 0.005
    U = gauge_field(L4, "exp", eps=0.4, seed=1001)
    b = gaussian_spinor(L4, seed=2001)
    print("\n[case] 24^3x8 fp64 eo bicgstab2, 10000 steps", flush=True)
    rc, info, x = run_solve(mods, L4, theta, U, b, kappa, mu, "bicgstab2", tol=1e-10, maxiter=10000)
    tr = true_res(U, x, b, L4, theta, kappa, mu)
    print(f"  rc={rc} iters={info[0]['iters']} t={info[0]['seconds']:.3f}s true={tr:.2e}", flush=True)
    assert rc == 0, info
    assert tr <= 1e-10 and abs(tr - info[0]["true_resid"]) <= 1e-13


@pytest.mark.parametrize("use_graph", [0, 1])
@pytest.mark.parametrize("inner", [(64, 18), (32, 12)])
def test_uneven_batch(mods, use_graph, inner):
    """Three lattices of different volumes, each with its own kappa, eps and
    links and two Gaussian right-hand sides, solved by one batched CGNR whose
    kernels each cover all systems; every solution is certified by the
    oracle's M and agrees with the system's own single solve."""
    torch, fields, lqcd = mods
    systems = [((6, 6, 6, 4), 0.3, 0.15), ((8, 8, 8, 4), 0.4, 0.16), ((4, 6, 8, 4), 0.5, 0.155)]
    theta, mu, nrhs = (0, 0, 0, math.pi), 0.005, 2
    s = torch.cuda.Stream()
    geoms, ops, Us, bs, xs, host = [], [], [], [], [], []
    for i, (L4, eps, kappa) in enumerate(systems):
        U = gauge_field(L4, "exp", eps=eps, seed=1004 + 10 * i)
        b = gaussian_spinor(L4, seed=2004 + 10 * i, nrhs=nrhs)
        lat = fields.Lattice(L4, theta)
        geoms.append(lat.g)
        ops.append(lqcd.op(kappa, mu))
        Us.append(lat.gauge(U))
        bs.append(lat.spinor(b))
        xs.append(lat.zeros(lqcd.FIELD_SPINOR_FULL, 64, nrhs=nrhs))
        host.append((L4, kappa, U, b, lat))
    p = lqcd.solve_params(tol=1e-10, maxiter=20000, nrhs=nrhs, inner_prec=inner[0], inner_recon=inner[1],
                          use_graph=use_graph)
    ws = torch.empty(lqcd.lqcd_workspace_bytes_batch(geoms, ops, p), dtype=torch.uint8, device="cuda")
    print(f"\n[case] uneven batch graph={use_graph} inner={inner}", flush=True)
    with torch.cuda.stream(s):
        rc, infos = lqcd.cg_solve_batch(geoms, ops, Us, bs, xs, p, ws, stream=s)
    torch.cuda.synchronize()
    assert rc == 0, infos
    for i, (L4, kappa, U, b, lat) in enumerate(host):
        x = lat.unpack(xs[i], 64, nrhs=nrhs)
        for k in range(nrhs):
            assert true_res(U, x[k], b[k], L4, theta, kappa, mu) <= 1e-10, (i, k)
            assert abs(infos[i][k]["true_resid"] - true_res(U, x[k], b[k], L4, theta, kappa, mu)) < 1e-12
            check_eo_resid(infos[i][k], U, x[k], b[k], L4, theta, kappa, mu)
        rc1, info1, x1 = run_solve(mods, L4, theta, U, b, kappa, mu, "cg", nrhs=nrhs, tol=1e-10, maxiter=20000,
                                   inner_prec=inner[0], inner_recon=inner[1])
        assert rc1 == 0
        for k in range(nrhs):
            assert info1[k]["iters"] == infos[i][k]["iters"], (i, k)
            err = np.linalg.norm((x1[k] - x[k]).ravel()) / np.linalg.norm(x1[k].ravel())
            assert err < 1e-9, (i, k, err)


def test_mixed_outer_steps_tol_inner(mods):
    """FP32 inner solve inside an outer defect correction (tol_inner = 1e-3:
    each outer step ends when the low-precision residual fell by 1e3, then
    restarts from the FP64 residual with a fresh direction): certified, with
    several outer steps."""
    L4, theta, kappa, mu = (8, 8, 8, 4), (0, 0, 0, math.pi), 0.16, 0.005
    U = gauge_field(L4, "exp", eps=0.4, seed=1001)
    b = gaussian_spinor(L4, seed=2001)
    print("\n[case] 8^3x4 fp32 inner, tol_inner 1e-3", flush=True)
    rc, info, x = run_solve(mods, L4, theta, U, b, kappa, mu, "cg", tol=1e-10, maxiter=20000, inner_prec=32,
                            inner_recon=12, delta_reliable=1e-4, tol_inner=1e-3)
    print(f"  iters={info[0]['iters']} outer={info[0]['outer_iters']} updates={info[0]['reliable_updates']}",
          flush=True)
    assert rc == 0, info
    assert info[0]["outer_iters"] >= 3 and info[0]["stagnations"] == 0
    assert true_res(U, x, b, L4, theta, kappa, mu) <= 1e-10


def test_fp16_stagnation_falls_back_to_fp32(mods):
    """The fall back from FP16 to FP32 inner storage, forced from the host:
    delta = 1e-6 lets no reliable update happen on its own, so every window of
    10 iterations is a stagnation; after the first (max_stagnations = 1) the
    solve continues from its x at FP32 storage.  The result is certified."""
    L4, theta, kappa, mu = (8, 8, 8, 4), (0, 0, 0, math.pi), 0.16, 0.005
    U = gauge_field(L4, "exp", eps=0.4, seed=1001)
    b = gaussian_spinor(L4, seed=2001)
    print("\n[case] 8^3x4 fp16 inner, forced fall back", flush=True)
    rc, info, x = run_solve(mods, L4, theta, U, b, kappa, mu, "cg", tol=1e-10, maxiter=20000, inner_prec=16,
                            inner_recon=12, delta_reliable=1e-6, stag_window=10, max_stagnations=1)
    print(f"  iters={info[0]['iters']} stag={info[0]['stagnations']} fallbacks={info[0]['fallbacks']}", flush=True)
    assert rc == 0, info
    assert info[0]["fallbacks"] == 1 and info[0]["stagnations"] >= 1
    assert true_res(U, x, b, L4, theta, kappa, mu) <= 1e-10


def test_fp16_no_fall_back_when_disabled(mods):
    """max_stagnations < 0: stagnations restart the search direction but the
    solve stays at FP16 storage."""
    L4, theta, kappa, mu = (8, 8, 8, 4), (0, 0, 0, math.pi), 0.16, 0.005
    U = gauge_field(L4, "exp", eps=0.4, seed=1001)
    b = gaussian_spinor(L4, seed=2001)
    print("\n[case] 8^3x4 fp16 inner, stagnation windows, no fall back", flush=True)
    rc, info, x = run_solve(mods, L4, theta, U, b, kappa, mu, "cg", tol=1e-10, maxiter=20000, inner_prec=16,
                            inner_recon=12, delta_reliable=1e-6, stag_window=10, max_stagnations=-1)
    assert rc == 0, info
    assert info[0]["fallbacks"] == 0 and info[0]["stagnations"] >= 1
    assert true_res(U, x, b, L4, theta, kappa, mu) <= 1e-10


@pytest.mark.parametrize("inner", [(64, 18), (32, 12), (16, 12)])
def test_multi_rhs_lanes_solve(mods, inner):
    """The 16-source solve (12 point + 4 Gaussian) with the right-hand sides
    across 16 lanes in every hop (per-right-hand-side reductions inside the
    blocks): each solution certified by the oracle's M."""
    torch, fields, lqcd = mods
    L4, theta, kappa, mu = (8, 8, 8, 4), (0, 0, 0, math.pi), 0.16, 0.005
    U = gauge_field(L4, "exp", eps=0.4, seed=1003)
    b = np.concatenate([np.stack([point_source(L4, s, c) for s in range(4) for c in range(3)]),
                        gaussian_spinor(L4, seed=2003, nrhs=4)])
    saved = {p: lqcd.lqcd_get_launch(lqcd.KERNEL_DSLASH_RHS, p) for p in (64, 32, 16)}
    print(f"\n[case] 16 rhs across lanes, inner={inner}", flush=True)
    try:
        for p in (64, 32, 16):
            lqcd.lqcd_set_launch(lqcd.KERNEL_DSLASH_RHS, p, 256, 1, 1, 1, 0, 1, 16)
        rc, info, x = run_solve(mods, L4, theta, U, b, kappa, mu, "cg", nrhs=16, tol=1e-10, maxiter=20000,
                                inner_prec=inner[0], inner_recon=inner[1])
    finally:
        for p, cfg in saved.items():
            lqcd.lqcd_set_launch(lqcd.KERNEL_DSLASH_RHS, p, **cfg)
    assert rc == 0, info
    for k in range(16):
        assert true_res(U, x[k], b[k], L4, theta, kappa, mu) <= 1e-10, k


def _uneven_batch(mods, nrhs=2):
    torch, fields, lqcd = mods
    systems = [((6, 6, 6, 4), 0.3, 0.15), ((8, 8, 8, 4), 0.4, 0.16), ((4, 6, 8, 4), 0.5, 0.155)]
    theta, mu = (0, 0, 0, math.pi), 0.005
    geoms, ops, Us, bs, xs, host = [], [], [], [], [], []
    for i, (L4, eps, kappa) in enumerate(systems):
        U = gauge_field(L4, "exp", eps=eps, seed=1004 + 10 * i)
        b = gaussian_spinor(L4, seed=2004 + 10 * i, nrhs=nrhs)
        lat = fields.Lattice(L4, theta)
        geoms.append(lat.g)
        ops.append(lqcd.op(kappa, mu))
        Us.append(lat.gauge(U))
        bs.append(lat.spinor(b))
        xs.append(lat.zeros(lqcd.FIELD_SPINOR_FULL, 64, nrhs=nrhs))
        host.append((L4, kappa, U, b, lat))
    return geoms, ops, Us, bs, xs, host, theta, mu


@pytest.mark.parametrize("use_graph", [0, 1])
def test_uneven_batch_persistent(mods, use_graph):
    """The uneven batch in one persistent cooperative launch per start (grid
    barriers between the steps of the iteration), launched directly or
    replayed from a captured graph: every solution certified by the oracle's
    M and equal, within cond(M) tol, to the batched-launch solve of the same
    systems."""
    torch, fields, lqcd = mods
    nrhs = 2
    geoms, ops, Us, bs, xs, host, theta, mu = _uneven_batch(mods, nrhs)
    p = lqcd.solve_params(tol=1e-10, maxiter=20000, nrhs=nrhs, inner_prec=32, inner_recon=12, persistent=1,
                          use_graph=use_graph)
    ws = torch.empty(lqcd.lqcd_workspace_bytes_batch(geoms, ops, p), dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    print(f"\n[case] uneven batch, persistent launch use_graph={use_graph}", flush=True)
    with torch.cuda.stream(s):
        rc, infos = lqcd.cg_solve_batch(geoms, ops, Us, bs, xs, p, ws, stream=s)
    torch.cuda.synchronize()
    print(f"  rc={rc} iters={[i[0]['iters'] for i in infos]} launches={infos[0][0]['persistent_launches']}",
          flush=True)
    assert rc == 0, infos
    assert infos[0][0]["persistent_launches"] >= 1
    xs_p = [lat.unpack(xs[i], 64, nrhs=nrhs) for i, (_, _, _, _, lat) in enumerate(host)]
    p0 = lqcd.solve_params(tol=1e-10, maxiter=20000, nrhs=nrhs, inner_prec=32, inner_recon=12)
    xs0 = [lat.zeros(lqcd.FIELD_SPINOR_FULL, 64, nrhs=nrhs) for (_, _, _, _, lat) in host]
    ws0 = torch.empty(lqcd.lqcd_workspace_bytes_batch(geoms, ops, p0), dtype=torch.uint8, device="cuda")
    rc0, infos0 = lqcd.cg_solve_batch(geoms, ops, Us, bs, xs0, p0, ws0)
    assert rc0 == 0
    for i, (L4, kappa, U, b, lat) in enumerate(host):
        x0 = lat.unpack(xs0[i], 64, nrhs=nrhs)
        for k in range(nrhs):
            tr = true_res(U, xs_p[i][k], b[k], L4, theta, kappa, mu)
            assert tr <= 1e-10, (i, k, tr)
            assert abs(tr - infos[i][k]["true_resid"]) < 1e-12
            err = np.linalg.norm((xs_p[i][k] - x0[k]).ravel()) / np.linalg.norm(x0[k].ravel())
            assert err < 1e-8, (i, k, err)


@pytest.mark.parametrize("nrhs,inner", [(2, (32, 12)), (1, (64, 18))])
def test_uneven_batch_autotune(mods, nrhs, inner):
    """lqcd_autotune_batch on the uneven batch: it returns one of the shapes
    it sweeps, installs it for the inner hop family (the right-hand-side
    family when nrhs > 1) and the batched solve that follows, with that
    shape, certifies every solution.  The process-wide table is restored
    afterwards."""
    torch, fields, lqcd = mods
    geoms, ops, Us, bs, xs, host, theta, mu = _uneven_batch(mods, nrhs)
    p = lqcd.solve_params(tol=1e-10, maxiter=20000, nrhs=nrhs, inner_prec=inner[0], inner_recon=inner[1])
    ws = torch.empty(lqcd.lqcd_workspace_bytes_batch(geoms, ops, p), dtype=torch.uint8, device="cuda")
    family = lqcd.KERNEL_DSLASH_RHS if nrhs > 1 else lqcd.KERNEL_DSLASH
    before = lqcd.lqcd_get_launch(family, inner[0])
    s = torch.cuda.Stream()
    print(f"\n[case] uneven batch autotune nrhs={nrhs} inner={inner}", flush=True)
    try:
        best, us = lqcd.lqcd_autotune_batch(geoms, ops, Us, bs, xs, p, ws, iters=4, stream=s)
        print(f"  best={best} us/iter={us:.1f}", flush=True)
        assert best["block"] in (128, 192, 256) and us > 0
        if nrhs > 1:
            assert (best["rhs_tile"], best["rhs_group"]) in [(1, 0), (1, 2), (1, 4), (1, 8), (2, 0), (2, 2), (2, 4)]
        else:
            assert best["order"] in (0, 1) and best["swizzle"] in (0, 1)
        assert lqcd.lqcd_get_launch(family, inner[0]) == best
        with torch.cuda.stream(s):
            rc, infos = lqcd.cg_solve_batch(geoms, ops, Us, bs, xs, p, ws, stream=s)
        torch.cuda.synchronize()
        assert rc == 0, infos
        for i, (L4, kappa, U, b, lat) in enumerate(host):
            x = lat.unpack(xs[i], 64, nrhs=nrhs)
            if nrhs == 1:  # one right-hand side comes without the leading axis
                x, b = x[None], b[None]
            for k in range(nrhs):
                assert true_res(U, x[k], b[k], L4, theta, kappa, mu) <= 1e-10, (i, k)
    finally:
        lqcd.lqcd_set_launch(family, inner[0], **before)


@pytest.mark.parametrize("persistent", [0, 1])
def test_batch_of_sixteen_systems(mods, persistent):
    """The largest batch (16 systems): tiny lattices of eight different
    shapes (extents 2..8, ragged against every block and row tile), each with
    its own kappa, 2 right-hand sides, FP32/12 inner; all 32 solutions
    certified by the oracle's M, as batched launches and as one persistent
    launch."""
    torch, fields, lqcd = mods
    shapes = [(2, 2, 2, 2), (4, 2, 2, 2), (2, 4, 2, 4), (4, 4, 4, 2), (6, 2, 4, 2), (2, 6, 2, 6), (4, 4, 2, 6),
              (8, 2, 2, 4)] * 2
    theta, mu, nrhs = (0, 0, 0, math.pi), 0.005, 2
    geoms, ops, Us, bs, xs, host = [], [], [], [], [], []
    for i, L4 in enumerate(shapes):
        kappa = 0.12 + 0.002 * i
        U = gauge_field(L4, "exp", eps=0.4, seed=1300 + i)
        b = gaussian_spinor(L4, seed=2300 + i, nrhs=nrhs)
        lat = fields.Lattice(L4, theta)
        geoms.append(lat.g)
        ops.append(lqcd.op(kappa, mu))
        Us.append(lat.gauge(U))
        bs.append(lat.spinor(b))
        xs.append(lat.zeros(lqcd.FIELD_SPINOR_FULL, 64, nrhs=nrhs))
        host.append((L4, kappa, U, b, lat))
    p = lqcd.solve_params(tol=1e-10, maxiter=20000, nrhs=nrhs, inner_prec=32, inner_recon=12, use_graph=1,
                          persistent=persistent)
    ws = torch.empty(lqcd.lqcd_workspace_bytes_batch(geoms, ops, p), dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    print(f"\n[case] 16-system batch persistent={persistent}", flush=True)
    with torch.cuda.stream(s):
        rc, infos = lqcd.cg_solve_batch(geoms, ops, Us, bs, xs, p, ws, stream=s)
    torch.cuda.synchronize()
    assert rc == 0, infos
    assert len(infos) == 16 and all(len(i) == nrhs for i in infos)
    for i, (L4, kappa, U, b, lat) in enumerate(host):
        x = lat.unpack(xs[i], 64, nrhs=nrhs)
        for k in range(nrhs):
            tr = true_res(U, x[k], b[k], L4, theta, kappa, mu)
            assert tr <= 1e-10, (i, L4, k, tr)


@pytest.mark.parametrize("use_graph", [0, 1])
def test_uneven_batch_persistent_give_up(mods, use_graph):
    """The persistent kernel's failure path, forced from the host: with the
    give-up word set at launch (persistent = 2) every block leaves at its
    first grid barrier, the kernel ends and the call fails with EHIP (also
    when the launch is replayed from a graph); the device then runs the same
    batch normally."""
    torch, fields, lqcd = mods
    nrhs = 2
    geoms, ops, Us, bs, xs, host, theta, mu = _uneven_batch(mods, nrhs)
    p2 = lqcd.solve_params(tol=1e-10, maxiter=20000, nrhs=nrhs, inner_prec=32, inner_recon=12, persistent=2,
                           use_graph=use_graph)
    ws = torch.empty(lqcd.lqcd_workspace_bytes_batch(geoms, ops, p2), dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    print(f"\n[case] uneven batch, persistent give-up use_graph={use_graph}", flush=True)
    with pytest.raises(lqcd.LqcdError) as e:
        lqcd.cg_solve_batch(geoms, ops, Us, bs, xs, p2, ws, stream=s)
    assert e.value.code == lqcd.EHIP and "gave up" in str(e.value)
    torch.cuda.synchronize()
    p1 = lqcd.solve_params(tol=1e-10, maxiter=20000, nrhs=nrhs, inner_prec=32, inner_recon=12, persistent=1,
                           use_graph=use_graph)
    rc, infos = lqcd.cg_solve_batch(geoms, ops, Us, bs, xs, p1, ws, stream=s)
    assert rc == 0, infos
    for i, (L4, kappa, U, b, lat) in enumerate(host):
        x = lat.unpack(xs[i], 64, nrhs=nrhs)
        for k in range(nrhs):
            assert true_res(U, x[k], b[k], L4, theta, kappa, mu) <= 1e-10, (i, k)


def test_persistent_refuses_unsupported(mods):
    """The persistent launch runs the FP32/12-inner batched CGNR on several
    right-hand sides; anything else is refused with EUNSUPPORTED."""
    torch, fields, lqcd = mods
    geoms, ops, Us, bs, xs, host, theta, mu = _uneven_batch(mods, 1)
    for prm in (lqcd.solve_params(nrhs=1, inner_prec=32, inner_recon=12, persistent=1),
                lqcd.solve_params(nrhs=1, inner_prec=64, persistent=1)):
        ws = torch.empty(lqcd.lqcd_workspace_bytes_batch(geoms, ops, prm), dtype=torch.uint8, device="cuda")
        with pytest.raises(lqcd.LqcdError) as e:
            lqcd.cg_solve_batch(geoms, ops, Us, bs, xs, prm, ws)
        assert e.value.code == lqcd.EUNSUPPORTED
