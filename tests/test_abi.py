"""The C ABI without a GPU: the library loads, exports what include/fmm.h
declares, agrees with the header on struct layouts, and rejects bad
arguments on the host before touching the device."""
import ctypes
import math
import os
import re
import subprocess

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "fmm.h")


@pytest.fixture(scope="module")
def fmm():
    from paper_1502_07303_amd import fmm as m
    m.load_library()
    return m


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fmm_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(fmm):
    names = declared_functions()
    assert {"fmm_solve", "fmm_workspace_bytes", "fmm_get_stats", "fmm_strerror", "fmm_default_opts",
            "fmm_eval_godunov", "fmm_solve_batch", "fmm_batch_workspace_bytes", "fmm_get_batch_stats",
            "fmm_tune_batch"} <= set(names)
    out = subprocess.run(["nm", "-D", "--defined-only", fmm.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (fmm_\w+)", out))
    for n in names:
        assert n in exported, n
        assert hasattr(fmm.load_library(), n)


def test_struct_layout_matches_header(fmm, tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include "fmm.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(fmm_opts), sizeof(fmm_stats),'
                   ' offsetof(fmm_stats, max_abs_T), offsetof(fmm_stats, n_workgroups), offsetof(fmm_opts, stride_h),'
                   ' sizeof(fmm_problem), offsetof(fmm_problem, status_out));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert vals == [ctypes.sizeof(fmm.FmmOpts), ctypes.sizeof(fmm.FmmStats),
                    fmm.FmmStats.max_abs_T.offset, fmm.FmmStats.n_workgroups.offset, fmm.FmmOpts.stride_h.offset,
                    ctypes.sizeof(fmm.FmmProblem), fmm.FmmProblem.status_out.offset]


def test_default_opts(fmm):
    o = fmm.FmmOpts()
    fmm.load_library().fmm_default_opts(ctypes.byref(o))
    assert math.isinf(o.band_width) and o.stride == 0.0 and o.tile_edge == 8
    assert o.max_restarts == 0 and o.flags == 0


def test_workspace_bytes(fmm):
    lib = fmm.load_library()
    F64, F32 = fmm.FMM_F64, fmm.FMM_F32
    w8 = lib.fmm_workspace_bytes(64, 64, 64, 1, F64, None)
    assert w8 > 0 and w8 % 256 == 0
    assert lib.fmm_workspace_bytes(64, 64, 64, 1, F32, None) < w8  # FP32 tiled speeds
    o = fmm.make_opts(tile_edge=4)
    w4 = lib.fmm_workspace_bytes(64, 64, 64, 1, F64, ctypes.byref(o))
    assert w4 > w8  # more tiles, more bookkeeping
    # ragged grids round up to whole tiles
    assert lib.fmm_workspace_bytes(65, 64, 64, 1, F64, None) > w8
    # invalid
    assert lib.fmm_workspace_bytes(0, 64, 64, 1, F64, None) == 0
    assert lib.fmm_workspace_bytes(64, 64, 64, -1, F64, None) == 0
    assert lib.fmm_workspace_bytes(64, 64, 64, 1, 9, None) == 0
    bad = fmm.make_opts(tile_edge=5)
    assert lib.fmm_workspace_bytes(64, 64, 64, 1, F64, ctypes.byref(bad)) == 0
    # 1024^3 FP32: tiled T (8 B) + tiled F (4 B) + axis-2 faces (2 B) per point + bookkeeping
    big = lib.fmm_workspace_bytes(1024, 1024, 1024, 4, F32, None)
    assert 14 * 2 ** 30 < big < 15 * 2 ** 30


def _call(fmm, **kw):
    lib = fmm.load_library()
    fake = ctypes.c_void_p(0x100000)  # never dereferenced: host validation fails first
    args = dict(n0=8, n1=8, n2=8, h=0.1, F=fake, dt=fmm.FMM_F64, idx=fake, val=fake, ns=1, opts=None,
                T=fake, st=None, ws=fake, wsb=1 << 30, stream=None)
    args.update(kw)
    o = args["opts"]
    return lib.fmm_solve(args["n0"], args["n1"], args["n2"], args["h"], args["F"], args["dt"], args["idx"],
                         args["val"], args["ns"], ctypes.byref(o) if o is not None else None, args["T"],
                         args["st"], args["ws"], args["wsb"], args["stream"])


@pytest.mark.parametrize("kw", [
    {"n0": 0}, {"n2": -3}, {"h": 0.0}, {"h": -1.0}, {"h": math.nan}, {"h": math.inf},
    {"F": None}, {"T": None}, {"ws": None}, {"dt": 7}, {"ns": -1}, {"idx": None}, {"val": None},
    {"ws": ctypes.c_void_p(0x100010)},  # misaligned workspace
])
def test_host_rejects_bad_arguments(fmm, kw):
    assert _call(fmm, **kw) == fmm.FMM_EINVAL


@pytest.mark.parametrize("opt", [dict(band_width=-1.0), dict(band_width=math.nan), dict(stride=math.nan),
                                 dict(tile_edge=6), dict(max_restarts=-2), dict(axis_scale=(1.0, -2.0, 1.0)),
                                 dict(axis_scale=(math.nan, 1.0, 1.0)), dict(axis_scale=(1.0, 1.0, math.inf))])
def test_host_rejects_bad_options(fmm, opt):
    o = fmm.make_opts()
    for k, v in opt.items():
        if k == "axis_scale":
            for a in range(3):
                o.axis_scale[a] = v[a]
        else:
            setattr(o, k, v)
    assert _call(fmm, opts=o) == fmm.FMM_EINVAL


def test_host_reports_small_workspace(fmm):
    assert _call(fmm, wsb=64) == fmm.FMM_ENOMEM


def test_strerror(fmm):
    assert fmm.strerror(fmm.FMM_OK) == "ok"
    assert "workspace" in fmm.strerror(fmm.FMM_ENOMEM)
    assert fmm.strerror(12345) == "unknown status"


def test_eval_godunov_rejects_null(fmm):
    assert fmm.load_library().fmm_eval_godunov(None, None, None, 5, None) == fmm.FMM_EINVAL
    assert fmm.load_library().fmm_eval_godunov(None, None, None, 0, None) == fmm.FMM_OK


# --------------------------------------------------------------------------
# batches (host side)

def _problems(fmm, shapes, h=0.1, ns=1):
    fake = 0x100000  # never dereferenced: host validation or sizing only
    arr = (fmm.FmmProblem * len(shapes))()
    for p, sh in zip(arr, shapes):
        p.n0, p.n1, p.n2 = sh
        p.h = h
        p.F = p.seed_idx = p.seed_val = p.T_out = fake
        p.n_seeds = ns
    return arr


def test_batch_workspace_bytes(fmm):
    lib = fmm.load_library()
    one = lib.fmm_batch_workspace_bytes(1, _problems(fmm, [(40, 33, 47)]), fmm.FMM_F64, None)
    assert one == lib.fmm_workspace_bytes(40, 33, 47, 1, fmm.FMM_F64, None) > 0
    a = lib.fmm_workspace_bytes(32, 32, 32, 1, fmm.FMM_F64, None)
    b = lib.fmm_workspace_bytes(96, 64, 40, 1, fmm.FMM_F64, None)
    both = lib.fmm_batch_workspace_bytes(2, _problems(fmm, [(32, 32, 32), (96, 64, 40)]), fmm.FMM_F64, None)
    # the per-tile arrays add up; the control block is shared
    assert max(a, b) < both <= a + b
    assert lib.fmm_batch_workspace_bytes(0, _problems(fmm, [(8, 8, 8)]), fmm.FMM_F64, None) == 0
    assert lib.fmm_batch_workspace_bytes(2, _problems(fmm, [(8, 8, 8), (0, 8, 8)]), fmm.FMM_F64, None) == 0
    assert lib.fmm_batch_workspace_bytes(1, None, fmm.FMM_F64, None) == 0


def test_batch_rejects_bad_problems(fmm):
    lib = fmm.load_library()
    ws = ctypes.c_void_p(0x100000)
    good = _problems(fmm, [(8, 8, 8), (9, 10, 11)])
    assert lib.fmm_solve_batch(2, good, fmm.FMM_F64, None, ws, 64, None) == fmm.FMM_ENOMEM
    for field, val in [("h", 0.0), ("F", None), ("T_out", None), ("n_seeds", -1), ("seed_idx", None), ("n1", 0)]:
        bad = _problems(fmm, [(8, 8, 8), (9, 10, 11)])
        setattr(bad[1], field, val)
        assert lib.fmm_solve_batch(2, bad, fmm.FMM_F64, None, ws, 1 << 30, None) == fmm.FMM_EINVAL, field
    assert lib.fmm_solve_batch(0, good, fmm.FMM_F64, None, ws, 1 << 30, None) == fmm.FMM_EINVAL
    o = fmm.make_opts(stride_h=math.nan)
    assert lib.fmm_solve_batch(2, good, fmm.FMM_F64, ctypes.byref(o), ws, 1 << 30, None) == fmm.FMM_EINVAL


def test_tune_rejects_bad_candidates(fmm):
    lib = fmm.load_library()
    ws = ctypes.c_void_p(0x100000)
    good = _problems(fmm, [(16, 16, 16)])
    best = fmm.FmmOpts()
    strides = (ctypes.c_double * 2)(1.0, 2.0)
    for edges, wsb in [([5], 1 << 30), ([4, 8], 64)]:
        e = (ctypes.c_int32 * len(edges))(*edges)
        rc = lib.fmm_tune_batch(1, good, fmm.FMM_F64, None, e, len(edges), strides, 2, 1, ws, wsb, None,
                                ctypes.byref(best), None)
        assert rc == (fmm.FMM_EINVAL if wsb > 64 else fmm.FMM_ENOMEM)
    e = (ctypes.c_int32 * 1)(8)
    bad_s = (ctypes.c_double * 1)(0.0)
    assert lib.fmm_tune_batch(1, good, fmm.FMM_F64, None, e, 1, bad_s, 1, 1, ws, 1 << 30, None,
                              ctypes.byref(best), None) == fmm.FMM_EINVAL


# --------------------------------------------------------------------------
# adjoint (host side)

def test_adjoint_struct_layout(fmm, tmp_path):
    src = tmp_path / "adj.c"
    src.write_text('#include "fmm.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                   'int main(void){printf("%zu %zu %zu\\n", sizeof(fmm_adjoint_problem),'
                   ' offsetof(fmm_adjoint_problem, dL_dF), sizeof(fmm_adjoint_stats));return 0;}\n')
    exe = tmp_path / "adj"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert vals == [ctypes.sizeof(fmm.FmmAdjointProblem), fmm.FmmAdjointProblem.dL_dF.offset,
                    ctypes.sizeof(fmm.FmmAdjointStats)]


def _adj_problems(fmm, shapes):
    fake = 0x100000
    arr = (fmm.FmmAdjointProblem * len(shapes))()
    for p, sh in zip(arr, shapes):
        p.n0, p.n1, p.n2 = sh
        p.h = 0.1
        p.F = p.T = p.status = p.dL_dT = p.dL_dF = fake
    return arr


def test_adjoint_workspace_and_rejects(fmm):
    lib = fmm.load_library()
    one = lib.fmm_adjoint_workspace_bytes(1, _adj_problems(fmm, [(10, 11, 12)]))
    two = lib.fmm_adjoint_workspace_bytes(2, _adj_problems(fmm, [(10, 11, 12), (10, 11, 12)]))
    assert one >= 29 * 1320 and two > one
    assert lib.fmm_adjoint_workspace_bytes(1, _adj_problems(fmm, [(0, 4, 4)])) == 0
    ws = ctypes.c_void_p(0x100000)
    good = _adj_problems(fmm, [(8, 8, 8)])
    assert lib.fmm_adjoint_batch(1, good, fmm.FMM_F64, ws, 64, None) == fmm.FMM_ENOMEM
    for field, val in [("h", -1.0), ("T", None), ("status", None), ("dL_dT", None), ("dL_dF", None), ("F", None)]:
        bad = _adj_problems(fmm, [(8, 8, 8)])
        setattr(bad[0], field, val)
        assert lib.fmm_adjoint_batch(1, bad, fmm.FMM_F64, ws, 1 << 30, None) == fmm.FMM_EINVAL, field
    assert lib.fmm_adjoint_batch(1, good, 5, ws, 1 << 30, None) == fmm.FMM_EINVAL


# --------------------------------------------------------------------------
# the entry point that allocates nothing (host side)

def _call_noalloc(fmm, **kw):
    lib = fmm.load_library()
    fake = ctypes.c_void_p(0x100000)  # never dereferenced: host validation fails first
    args = dict(n0=8, n1=8, n2=8, h=0.1, F=fake, dt=fmm.FMM_F64, idx=fake, val=fake, ns=1, opts=None,
                T=fake, st=None, err=None, stream=None)
    args.update(kw)
    o = args["opts"]
    return lib.fmm_solve_noalloc(args["n0"], args["n1"], args["n2"], args["h"], args["F"], args["dt"],
                                 args["idx"], args["val"], args["ns"], ctypes.byref(o) if o is not None else None,
                                 args["T"], args["st"], args["err"], args["stream"])


@pytest.mark.parametrize("kw", [{"n0": 0}, {"h": 0.0}, {"F": None}, {"T": None}, {"dt": 3}, {"ns": -1},
                                {"idx": None}])
def test_noalloc_rejects_bad_arguments(fmm, kw):
    assert _call_noalloc(fmm, **kw) == fmm.FMM_EINVAL


def test_noalloc_rejects_grids_beyond_its_array(fmm):
    """Grids whose workspace exceeds the fixed array are refused on the host
    (FMM_ENOMEM) before anything is enqueued; the limit is the header's."""
    lib = fmm.load_library()
    limit = fmm.NOALLOC_MAX_BYTES
    text = open(HEADER).read()
    assert re.search(r"#define FMM_NOALLOC_MAX_BYTES \(64u << 20\)", text)
    for n, dt in ((161, fmm.FMM_F32), (153, fmm.FMM_F64), (1024, fmm.FMM_F32)):
        assert lib.fmm_workspace_bytes(n, n, n, 1, dt, None) > limit
        assert _call_noalloc(fmm, n0=n, n1=n, n2=n, dt=dt) == fmm.FMM_ENOMEM
    for n, dt in ((160, fmm.FMM_F32), (152, fmm.FMM_F64)):
        assert lib.fmm_workspace_bytes(n, n, n, 1, dt, None) <= limit


def test_binding_rejects_host_tensors(fmm):
    """Tensors on the host never reach the library: the binding raises
    FMM_EINVAL before any launch (a host pointer in a kernel would fault)."""
    import torch
    F = torch.ones((8, 8, 8), dtype=torch.float64)
    idx = torch.zeros(1, dtype=torch.int64)
    val = torch.zeros(1, dtype=torch.float64)
    T = torch.empty((8, 8, 8), dtype=torch.float64)
    with pytest.raises(fmm.FmmError) as ei:
        fmm.solve_noalloc_into(F, 0.1, idx, val, T)
    assert ei.value.code == fmm.FMM_EINVAL
    with pytest.raises(fmm.FmmError) as ei:
        fmm.BatchSolver([{"F": F, "h": 0.1, "seed_idx": idx, "seed_val": val}])
    assert ei.value.code == fmm.FMM_EINVAL
    with pytest.raises(fmm.FmmError) as ei:
        fmm.AdjointSolver([{"F": F, "h": 0.1, "T": T, "status": torch.zeros((8, 8, 8), dtype=torch.uint8),
                            "dL_dT": T, "dL_dF": T}])
    assert ei.value.code == fmm.FMM_EINVAL
    with pytest.raises(fmm.FmmError):
        fmm._check_cuda("seed_idx", idx, torch.device("cuda:0"))
