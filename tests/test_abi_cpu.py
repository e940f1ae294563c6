"""The C-ABI library loads on the host, exports every symbol include/lqcd.h
declares, and validates arguments before touching the GPU."""

import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lqcd.h")).read()
    return sorted(set(re.findall(r"LQCD_API\s+(?:const\s+char\s*\*|int)\s+([a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["dslash_apply", "dslash_eo_apply", "cg_solve", "bicgstab_solve"]:
        assert n in names


def test_binding_structs_match_the_header(tmp_path):
    """Every argument struct of the binding has the C header's size and
    field offsets (a host C compiler lays the header's structs out)."""
    import ctypes
    import shutil
    import subprocess

    from paper_1411_5219_amd import lqcd as L
    cc = shutil.which("gcc")
    if not cc:
        pytest.skip("no host C compiler")
    pairs = {"lqcd_geom": L.Geom, "lqcd_op": L.Op, "lqcd_stag_op": L.StagOp, "lqcd_solve_params": L.SolveParams,
             "lqcd_launch": L.Launch, "lqcd_solve_info": L.SolveInfo}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "lqcd.h"', "int main(void) {"]
    for c, py in pairs.items():
        lines.append(f'    printf("{c} size %zu\\n", sizeof({c}));')
        for f, _ in py._fields_:
            lines.append(f'    printf("{c} {f} %zu\\n", offsetof({c}, {f}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for ln in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        c, f, v = ln.split()
        got[(c, f)] = int(v)
    for c, py in pairs.items():
        assert got[(c, "size")] == ctypes.sizeof(py), c
        for f, _ in py._fields_:
            assert got[(c, f)] == getattr(py, f).offset, (c, f)


def test_library_exports_every_declared_symbol():
    from paper_1411_5219_amd import lqcd as L
    names = _declared()
    assert sorted(L.SYMBOLS) == names
    for n in names:
        assert hasattr(L._lib, n), n


def test_field_sizes():
    from paper_1411_5219_amd import lqcd as L
    g = L.geom((4, 4, 4, 4))
    # 128 sites per parity; the plane stride is an odd multiple of 16 sites
    S = 144
    assert L.lqcd_field_bytes(g, L.FIELD_SPINOR_PARITY, 64) == 192 * S
    assert L.lqcd_field_bytes(g, L.FIELD_SPINOR_FULL, 32) == 2 * 96 * S
    assert L.lqcd_field_bytes(g, L.FIELD_SPINOR_PARITY, 16) == 52 * S
    assert L.lqcd_field_bytes(g, L.FIELD_GAUGE, 64, 18) == 8 * 144 * S
    assert L.lqcd_field_bytes(g, L.FIELD_GAUGE, 32, 12) == 8 * 48 * S
    assert L.lqcd_field_bytes(g, L.FIELD_GAUGE, 16, 12) == 8 * 24 * S


@pytest.mark.parametrize("L4", [(3, 4, 4, 4), (4, 4, 4, 0), (4, 4, 5, 4), (1, 2, 2, 2)])
def test_bad_extents_rejected(L4):
    from paper_1411_5219_amd import lqcd as L
    with pytest.raises(L.LqcdError) as e:
        L.lqcd_field_bytes(L.geom(L4), L.FIELD_SPINOR_FULL, 64)
    assert e.value.code == L.EINVAL


def test_bad_arguments_rejected_before_device_work():
    from paper_1411_5219_amd import lqcd as L
    g = L.geom((4, 4, 4, 4))
    with pytest.raises(L.LqcdError) as e:
        L.lqcd_field_bytes(g, L.FIELD_GAUGE, 16, 18)
    assert e.value.code == L.EUNSUPPORTED
    with pytest.raises(L.LqcdError) as e:
        L.dslash_apply(g, L.op(0.1), 0, 0, 0, stream=0)
    assert e.value.code == L.EINVAL
    with pytest.raises(L.LqcdError) as e:
        L.dslash_eo_apply(g, L.op(0.1), 16, 32, 48, out_parity=2, stream=0)
    assert e.value.code == L.EINVAL
    with pytest.raises(L.LqcdError) as e:
        L.dslash_eo_apply(g, L.op(0.1), 16, 32, 48, out_parity=1, op_kind=L.OP_SCHUR, stream=0, ws=64)
    assert e.value.code == L.EINVAL
    with pytest.raises(L.LqcdError) as e:
        L.dslash_apply(g, L.op(0.1, prec=48), 16, 32, 48, stream=0)
    assert e.value.code == L.EINVAL
    with pytest.raises(L.LqcdError) as e:
        L.lqcd_workspace_bytes(g, L.op(0.1), L.solve_params(nrhs=17))
    assert e.value.code == L.EINVAL
    with pytest.raises(L.LqcdError) as e:
        L.lqcd_workspace_bytes(g, L.op(0.1), L.solve_params(inner_prec=16, inner_recon=18))
    assert e.value.code == L.EUNSUPPORTED
    with pytest.raises(L.LqcdError) as e:
        L.lqcd_workspace_bytes(g, L.op(0.1), L.solve_params(tol=-1))
    assert e.value.code == L.EINVAL
    with pytest.raises(L.LqcdError) as e:
        L.lqcd_workspace_bytes(L.geom((4, 4, 4, 4), (0, 0, 0, math.inf)), L.op(0.1))
    assert e.value.code == L.EINVAL


def test_workspace_grows_with_rhs_and_mixed():
    from paper_1411_5219_amd import lqcd as L
    g = L.geom((8, 8, 8, 8))
    o = L.op(0.16, 0.005)
    a = L.lqcd_workspace_bytes(g, o, L.solve_params(nrhs=1))
    b = L.lqcd_workspace_bytes(g, o, L.solve_params(nrhs=4))
    c = L.lqcd_workspace_bytes(g, o, L.solve_params(inner_prec=32))
    assert b > 3 * a > 0 and c > 0


def test_bicgstab_ell_parameter():
    """params.bicgstab_ell: 0, 1 or 2 (anything else EINVAL before any device
    work); with 2 the workspace holds BiCGStab(2)'s 9 FP64 vectors per
    right-hand side against BiCGStab's 8 (even-odd)."""
    from paper_1411_5219_amd import lqcd as L
    g = L.geom((8, 8, 8, 8))
    o = L.op(0.16, 0.005)
    for bad in (-1, 3):
        with pytest.raises(L.LqcdError) as e:
            L.lqcd_workspace_bytes(g, o, L.solve_params(bicgstab_ell=bad))
        assert e.value.code == L.EINVAL
    pb = 8 * 8 * 8 * 8 // 2 * 24 * 8            # one parity field, without the layout's padding sites
    w0 = L.lqcd_workspace_bytes(g, o, L.solve_params(nrhs=2))
    w2 = L.lqcd_workspace_bytes(g, o, L.solve_params(nrhs=2, bicgstab_ell=2))
    assert 2 * pb <= w2 - w0 <= 2 * pb * 1.1
    with pytest.raises(L.LqcdError) as e:
        L.bicgstab_solve(g, o, 16, 32, 48, L.solve_params(bicgstab_ell=2, inner_prec=32), 64, stream=0)
    assert e.value.code == L.EUNSUPPORTED


def test_batch_workspace_query_validates():
    from paper_1411_5219_amd import lqcd as L
    g = [L.geom((4, 4, 4, 4)), L.geom((6, 6, 6, 4))]
    o = [L.op(0.15, 0.005), L.op(0.16, 0.005)]
    p = L.solve_params(nrhs=4, inner_prec=32)
    n2 = L.lqcd_workspace_bytes_batch(g, o, p)
    n1 = L.lqcd_workspace_bytes_batch(g[:1], o[:1], p)
    assert n2 > n1 > 0
    with pytest.raises(L.LqcdError) as e:
        L.lqcd_workspace_bytes_batch([], [], p)
    assert e.value.code == L.EINVAL
    with pytest.raises(L.LqcdError) as e:
        L.lqcd_workspace_bytes_batch([L.geom((4, 4, 5, 4))], o[:1], p)
    assert e.value.code == L.EINVAL
    with pytest.raises(L.LqcdError) as e:
        L.lqcd_workspace_bytes_batch(g * 9, o * 9, p)
    assert e.value.code == L.EINVAL


def test_launch_validation():
    """Launch shapes outside the documented ranges are refused before any
    device work; the z-slab orders (2..64) apply to the Dslash only."""
    from paper_1411_5219_amd import lqcd as L
    for kernel, prec, cfg in [(L.KERNEL_DSLASH, 64, dict(block=96)), (L.KERNEL_DSLASH, 64, dict(block=256, order=65)),
                              (L.KERNEL_DSLASH, 64, dict(block=256, order=-1)),
                              (L.KERNEL_BLAS, 64, dict(block=256, order=2)),
                              (L.KERNEL_DSLASH, 64, dict(block=256, rhs_tile=3)),
                              (L.KERNEL_DSLASH, 64, dict(block=256, rhs_group=17)),
                              (L.KERNEL_DSLASH, 64, dict(block=256, order=1, ygroup=65)),
                              (L.KERNEL_DSLASH, 64, dict(block=256, order=1, ygroup=-1))]:
        with pytest.raises(L.LqcdError) as e:
            L.lqcd_set_launch(kernel, prec, **cfg)
        assert e.value.code == L.EINVAL, cfg
    with pytest.raises(L.LqcdError) as e:
        L.lqcd_set_launch(4, 64, 256)
    assert e.value.code == L.EINVAL
    saved = L.lqcd_get_launch(L.KERNEL_DSLASH, 32)
    saved_rhs = L.lqcd_get_launch(L.KERNEL_DSLASH_RHS, 32)
    try:
        L.lqcd_set_launch(L.KERNEL_DSLASH, 32, 256, 1, 6, 1, 4)
        assert L.lqcd_get_launch(L.KERNEL_DSLASH, 32)["order"] == 6
        assert L.lqcd_get_launch(L.KERNEL_DSLASH_RHS, 32) == saved_rhs  # separate slots
        L.lqcd_set_launch(L.KERNEL_DSLASH_RHS, 32, 128, 1, 1, 2, 8)
        assert L.lqcd_get_launch(L.KERNEL_DSLASH_RHS, 32) == dict(block=128, swizzle=1, order=1, rhs_tile=2,
                                                                   rhs_group=8, ygroup=1, rhs_lanes=1)
        L.lqcd_set_launch(L.KERNEL_DSLASH, 32, 256, 1, 1, 1, 0, 3)
        assert L.lqcd_get_launch(L.KERNEL_DSLASH, 32)["ygroup"] == 3
        L.lqcd_set_launch(L.KERNEL_DSLASH, 32, 256, 1, 1, 1, 0, 0)   # 0 means none
        assert L.lqcd_get_launch(L.KERNEL_DSLASH, 32)["ygroup"] == 1
    finally:
        L.lqcd_set_launch(L.KERNEL_DSLASH, 32, **saved)
        L.lqcd_set_launch(L.KERNEL_DSLASH_RHS, 32, **saved_rhs)



def test_staggered_sizes_and_validation():
    """Colour-field sizes follow the layout (FP64 48 B, FP32 24 B, FP16 16 B
    per site and parity at stride S); the staggered entry points refuse bad
    arguments before any device work."""
    from paper_1411_5219_amd import lqcd as L
    g = L.geom((4, 4, 4, 4))
    S = 144
    assert L.lqcd_field_bytes(g, L.FIELD_COLOUR_PARITY, 64) == 48 * S
    assert L.lqcd_field_bytes(g, L.FIELD_COLOUR_FULL, 32) == 2 * 24 * S
    assert L.lqcd_field_bytes(g, L.FIELD_COLOUR_PARITY, 16) == 16 * S
    o = L.stag_op(0.1)
    w0 = L.lqcd_workspace_bytes_stag(g, o, 0)
    w8 = L.lqcd_workspace_bytes_stag(g, o, 8)
    assert w8 > w0 > 0
    with pytest.raises(L.LqcdError) as e:
        L.lqcd_workspace_bytes_stag(g, o, 33)
    assert e.value.code == L.EINVAL
    with pytest.raises(L.LqcdError) as e:
        L.stag_apply(g, L.stag_op(0.1, prec=16, recon=18), 16, 32, 48, stream=0)
    assert e.value.code == L.EUNSUPPORTED
    with pytest.raises(L.LqcdError) as e:
        L.stag_eo_apply(g, o, 16, 32, 48, out_parity=1, op_kind=L.OP_NORMAL, ws=64, stream=0)
    assert e.value.code == L.EINVAL
    with pytest.raises(L.LqcdError) as e:
        L.stag_eo_apply(g, o, 16, 32, 48, out_parity=0, op_kind=L.OP_SCHUR, stream=0)
    assert e.value.code == L.EINVAL
    p = L.solve_params(tol=1e-10, eo=1, inner_prec=64)
    for bad_op, bad_p in [(L.stag_op(0.0), p), (L.stag_op(0.1, prec=32), p),
                          (o, L.solve_params(tol=1e-10, eo=0)), (o, L.solve_params(tol=1e-10, nrhs=2))]:
        with pytest.raises(L.LqcdError) as e:
            L.stag_cg_solve(g, bad_op, 16, 32, 48, bad_p, None, stream=0)
        assert e.value.code in (L.EINVAL, L.EUNSUPPORTED)
    for shifts in ([], [0.1] * 33, [-0.1], [float("nan")]):
        with pytest.raises(L.LqcdError) as e:
            L.stag_multishift_solve(g, o, 16, 32, 48, shifts, p, 64, stream=0)
        assert e.value.code == L.EINVAL


def test_force_and_gamma5_validation():
    """The force and gamma_5 entry points refuse bad arguments before any
    device work: FP32 operators, a bad accumulate flag, a non-finite scale,
    NULL fields, lattices whose fields would pass 2 GiB, bad nrhs; the device
    query refuses NULL outputs."""
    from paper_1411_5219_amd import lqcd as L
    g = L.geom((4, 4, 4, 4))
    o = L.op(0.13, 0.1)
    cases = [dict(o=L.op(0.13, 0.1, prec=32, recon=12)), dict(accumulate=2), dict(scale=float("nan")),
             dict(U=None), dict(F=None)]
    for c in cases:
        args = dict(g=g, o=o, U=16, X=32, Wf=48, F=64, scale=1.0, accumulate=0)
        args.update(c)
        with pytest.raises(L.LqcdError) as e:
            L.tm_force(args["g"], args["o"], args["U"], args["X"], args["Wf"], args["F"], scale=args["scale"],
                       accumulate=args["accumulate"], stream=0)
        assert e.value.code == L.EINVAL, c
    with pytest.raises(L.LqcdError) as e:  # 64^3 x 48: a full-lattice FP64 spinor field is 2.4 GB
        L.tm_force(L.geom((64, 64, 64, 48)), o, 16, 32, 48, 64, stream=0)
    assert e.value.code == L.EINVAL
    for nrhs, inp in ((0, 16), (1, None)):
        with pytest.raises(L.LqcdError) as e:
            L.lqcd_gamma5(g, inp, 32, nrhs=nrhs, stream=0)
        assert e.value.code == L.EINVAL
    assert L._lib.lqcd_device_memory(0, None, None) == L.EINVAL


def test_rhs_launch_slot_validation():
    """The several-right-hand-side launch family takes the Dslash's shape
    rules, and its autotuner refuses bad arguments before any device work."""
    from paper_1411_5219_amd import lqcd as L
    for cfg in (dict(block=96), dict(block=256, rhs_tile=3), dict(block=256, rhs_group=17),
                dict(block=256, order=65)):
        with pytest.raises(L.LqcdError) as e:
            L.lqcd_set_launch(L.KERNEL_DSLASH_RHS, 32, **cfg)
        assert e.value.code == L.EINVAL, cfg
    g = L.geom((4, 4, 4, 4))
    o = L.op(0.16, 0.005, 32, 12)
    for nrhs, reps, inp, out in ((1, 3, 16, 32), (17, 3, 16, 32), (4, 0, 16, 32), (4, 3, None, 32), (4, 3, 16, 16)):
        with pytest.raises(L.LqcdError) as e:
            L.lqcd_autotune_dslash_rhs(g, o, 48, inp, out, nrhs, reps=reps, stream=0)
        assert e.value.code == L.EINVAL, (nrhs, reps, inp, out)


def test_persistent_parameter_checks():
    """params.persistent: 0, 1 or 2 (anything else EINVAL before any device
    work); the single-system solvers refuse it (EUNSUPPORTED): the persistent
    launch runs batched solves."""
    from paper_1411_5219_amd import lqcd as L
    g = L.geom((4, 4, 4, 4))
    o = L.op(0.13, 0.1)
    for bad in (-1, 3):
        with pytest.raises(L.LqcdError) as e:
            L.lqcd_workspace_bytes(g, o, L.solve_params(persistent=bad))
        assert e.value.code == L.EINVAL
    for fn in (L.cg_solve, L.bicgstab_solve):
        with pytest.raises(L.LqcdError) as e:
            fn(g, o, 16, 32, 48, L.solve_params(persistent=1), 64, stream=0)
        assert e.value.code == L.EUNSUPPORTED


def test_batch_autotune_validation():
    """lqcd_autotune_batch refuses before any device work: iters outside
    1..1000, the persistent launch, a workspace smaller than the batch needs,
    and a bad lattice among the systems."""
    from paper_1411_5219_amd import lqcd as L
    gs = [L.geom((4, 4, 4, 4)), L.geom((6, 4, 4, 4))]
    os_ = [L.op(0.13, 0.1), L.op(0.12, 0.0)]
    p = L.solve_params(nrhs=2, inner_prec=32, inner_recon=12)
    for iters in (0, 1001):
        with pytest.raises(L.LqcdError) as e:
            L.lqcd_autotune_batch(gs, os_, [16, 16], [32, 32], [48, 48], p, 64, iters=iters, stream=0)
        assert e.value.code == L.EINVAL
    with pytest.raises(L.LqcdError) as e:
        L.lqcd_autotune_batch(gs, os_, [16, 16], [32, 32], [48, 48], L.solve_params(nrhs=2, persistent=1), 64,
                              stream=0)
    assert e.value.code == L.EINVAL
    with pytest.raises(L.LqcdError) as e:  # ws_bytes 0: too small
        L.lqcd_autotune_batch(gs, os_, [16, 16], [32, 32], [48, 48], p, 64, stream=0)
    assert e.value.code == L.EINVAL and "workspace" in str(e.value)
    with pytest.raises(L.LqcdError) as e:
        L.lqcd_autotune_batch([L.geom((4, 4, 4, 4)), L.geom((5, 4, 4, 4))], os_, [16, 16], [32, 32], [48, 48], p, 64,
                              stream=0)
    assert e.value.code == L.EINVAL


def test_tune_cache_put_get_save_load(tmp_path):
    """The autotune cache: an entry put for a key is what a launch on that
    key uses (found), other keys fall back to the table (not found); save
    writes a JSON array that load merges back after a clear.  Arch here is
    "host" (no device in this process)."""
    import json
    from paper_1411_5219_amd import lqcd as L
    L.lqcd_tune_cache_clear()
    g = L.geom((8, 8, 8, 4))
    shape = {"block": 128, "swizzle": 0, "order": 1, "rhs_tile": 1, "rhs_group": 0, "ygroup": 2, "rhs_lanes": 1}
    try:
        L.lqcd_tune_cache_put(L.KERNEL_DSLASH, 32, 12, g, 1, shape, 12.5)
        got, us, found = L.lqcd_tune_cache_get(L.KERNEL_DSLASH, 32, 12, g, 1)
        assert found and got == shape and us == 12.5
        # another precision, reconstruction, extent or nrhs is another key
        for key in [(L.KERNEL_DSLASH, 64, 12, g, 1), (L.KERNEL_DSLASH, 32, 18, g, 1),
                    (L.KERNEL_DSLASH, 32, 12, L.geom((8, 8, 8, 6)), 1), (L.KERNEL_DSLASH_RHS, 32, 12, g, 2)]:
            got2, _, found2 = L.lqcd_tune_cache_get(*key)
            assert not found2 and got2 == L.lqcd_get_launch(key[0], key[1])
        path = str(tmp_path / "tune.json")
        L.lqcd_tune_cache_save(path)
        entries = json.load(open(path))
        assert len(entries) == 1 and entries[0]["L"] == [8, 8, 8, 4] and entries[0]["arch"] == "host"
        assert entries[0]["block"] == 128 and entries[0]["ygroup"] == 2 and entries[0]["us"] == 12.5
        L.lqcd_tune_cache_clear()
        assert not L.lqcd_tune_cache_get(L.KERNEL_DSLASH, 32, 12, g, 1)[2]
        L.lqcd_tune_cache_load(path)
        assert L.lqcd_tune_cache_get(L.KERNEL_DSLASH, 32, 12, g, 1)[:2] == (shape, 12.5)
    finally:
        L.lqcd_tune_cache_clear()


def test_tune_cache_rejects_bad_files_and_arguments(tmp_path):
    """A malformed line fails the whole load (EINVAL naming the line, nothing
    merged); an entry for another architecture is kept but never used here;
    kernel families without cached shapes and invalid shapes are refused."""
    from paper_1411_5219_amd import lqcd as L
    L.lqcd_tune_cache_clear()
    g = L.geom((8, 8, 8, 4))
    good = ('{"arch": "host", "kernel": 0, "prec": 64, "recon": 18, "L": [8, 8, 8, 4], "nrhs": 1, "block": 192, '
            '"swizzle": 1, "order": 1, "rhs_tile": 1, "rhs_group": 0, "ygroup": 1, "rhs_lanes": 1, "us": 3.0}')
    other = good.replace('"host"', '"gfx1100"').replace('"prec": 64', '"prec": 32')
    try:
        bad = tmp_path / "bad.json"
        bad.write_text("[\n" + good + ",\n" + good.replace('"block": 192', '"block": 100') + "\n]\n")
        with pytest.raises(L.LqcdError) as e:
            L.lqcd_tune_cache_load(str(bad))
        assert e.value.code == L.EINVAL and "line 3" in str(e.value)
        assert not L.lqcd_tune_cache_get(L.KERNEL_DSLASH, 64, 18, g, 1)[2]
        bad.write_text("[\nnot json\n]\n")
        with pytest.raises(L.LqcdError) as e:
            L.lqcd_tune_cache_load(str(bad))
        assert "line 2" in str(e.value)
        with pytest.raises(L.LqcdError):
            L.lqcd_tune_cache_load(str(tmp_path / "missing.json"))
        ok = tmp_path / "ok.json"
        ok.write_text("[\n" + good + ",\n" + other + "\n]\n")
        L.lqcd_tune_cache_load(str(ok))
        assert L.lqcd_tune_cache_get(L.KERNEL_DSLASH, 64, 18, g, 1)[2]
        assert not L.lqcd_tune_cache_get(L.KERNEL_DSLASH, 32, 18, g, 1)[2]  # the gfx1100 entry
        shape = L.lqcd_get_launch(L.KERNEL_DSLASH, 64)
        for args in [(L.KERNEL_BLAS, 64, 18, g, 1, shape), (L.KERNEL_DSLASH, 48, 18, g, 1, shape),
                     (L.KERNEL_DSLASH, 64, 10, g, 1, shape), (L.KERNEL_DSLASH, 64, 18, g, 0, shape),
                     (L.KERNEL_DSLASH, 64, 18, g, 1, dict(shape, rhs_lanes=3))]:
            with pytest.raises(L.LqcdError) as e:
                L.lqcd_tune_cache_put(*args)
            assert e.value.code == L.EINVAL
    finally:
        L.lqcd_tune_cache_clear()


def test_tune_cache_read_from_environment(tmp_path):
    """LQCD_TUNE_CACHE: a fresh process reads the file on first use of the
    cache (a missing file is an empty cache)."""
    import subprocess, sys, textwrap
    path = tmp_path / "env.json"
    path.write_text('[\n{"arch": "host", "kernel": 2, "prec": 32, "recon": 12, "L": [4, 4, 4, 4], "nrhs": 1, '
                    '"block": 64, "swizzle": 0, "order": 0, "rhs_tile": 1, "rhs_group": 0, "ygroup": 1, '
                    '"rhs_lanes": 1, "us": 1.0}\n]\n')
    code = textwrap.dedent("""
        import sys
        sys.path.insert(0, %r)
        from paper_1411_5219_amd import lqcd as L
        got, us, found = L.lqcd_tune_cache_get(L.KERNEL_STAG, 32, 12, L.geom((4, 4, 4, 4)), 1)
        print(found, got["block"], us)
    """ % ROOT)
    import os
    for p, want in [(path, "True 64 1.0"), (tmp_path / "none.json", "False")]:
        env = dict(os.environ, LQCD_TUNE_CACHE=str(p))
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
        assert r.returncode == 0, r.stderr
        assert r.stdout.strip().startswith(want), r.stdout
