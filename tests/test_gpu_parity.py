"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bar (from the method's own accuracy claim, Sec. 5.2): identical status bytes
(accepted set, band, seeds, sides) and max |T_gpu - T_oracle| <= 1e-12 max|T|
over the accepted points.  Floating point never decides the accepted set in
these cases except at the band edge, which the two-sided cases check
explicitly."""
import math
import os

import numpy as np
import pytest
import torch

from helpers import accepted_mask, backward_error, load_golden, parity_report, seed_mask
from paper_1502_07303_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-12
# the paper's strides (Sec. 5.1) and the ones the benchmark's autotuner tries
STRIDES_H = (0.5, 1.5, 2.0, 3.0, 3.5, 4.0, 4.5, 5.0, math.inf)


@pytest.fixture(scope="module")
def fmm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1502_07303_amd import fmm as m
    m.load_library()
    return m


def gpu_solve(fmm, w, **kw):
    dev = torch.device("cuda:0")
    kw.setdefault("time_limit_s", 30)
    T, st, stats = fmm.solve(w.F.to(dev), w.h, w.seed_idx.to(dev), w.seed_val.to(dev),
                             band_width=w.width, **kw)
    return T.cpu().numpy(), st.cpu().numpy(), stats


def oracle_solve(oracle_mod, w):
    F, idx, val = w.numpy()
    T, st, stats, _ = oracle_mod.solve(F, w.h, idx, val, width=w.width)
    return T, st, stats


def assert_parity(Tg, sg, To, so, tol=TOL, allow_edge=None):
    """Identical status bytes and values within tol * max|T|.  With a finite
    band (allow_edge = width), a point may change status only if the solver
    that accepted it holds a value within rounding of the width: the other
    solver, whose value differs by rounding, may then have left it in the
    band.  Every such flip is checked against the accepting side's value, and
    the flips must keep their side bit."""
    rep = parity_report(Tg, sg, To, so)
    if not rep["same_status"]:
        diff = np.flatnonzero(sg.reshape(-1) != so.reshape(-1))
        if allow_edge is None:
            raise AssertionError(f"status differs at {len(diff)} points, first {diff[:5]}: "
                                 f"gpu {sg.reshape(-1)[diff[:5]]} oracle {so.reshape(-1)[diff[:5]]}")
        tg, to = Tg.reshape(-1)[diff], To.reshape(-1)[diff]
        # the oracle writes +inf where it did not accept; take the accepting side's value
        ref = np.where(np.isinf(to), np.abs(tg), np.abs(to))
        assert np.all(np.isfinite(ref)), rep
        # exactly one of the two accepted each flipped point
        acc_g = (sg.reshape(-1)[diff] & 3) == 2
        acc_o = (so.reshape(-1)[diff] & 3) == 2
        assert np.all(acc_g != acc_o), rep
        edge = np.abs(ref - allow_edge) <= 1e-12 * allow_edge
        n_edge = int(np.count_nonzero(edge))
        print(f"band-edge flips: {rep['n_status_diff']} status differences, {n_edge} within rounding of the "
              f"width", flush=True)
        assert rep["n_status_diff"] == n_edge, rep
    assert rep["rel"] <= tol, rep
    return rep


# --------------------------------------------------------------------------

def test_device_local_solver_bitwise(fmm, oracle_mod):
    """Device G against the oracle's G on random arguments: identical bits
    (correctly rounded sqrt and division, no contraction on either side)."""
    rng = np.random.default_rng(0)
    n = 1 << 20
    r = rng.uniform(1e-4, 1.0, size=n)
    base = rng.uniform(0, 50, size=(n, 1))
    a = base + rng.uniform(0, 1.5, size=(n, 3)) * r[:, None]
    a[rng.random(n) < 0.2, 2] = np.inf
    a[rng.random(n) < 0.1, 1] = np.inf
    tie = rng.random(n) < 0.1
    a[tie, 1] = a[tie, 0]
    expect = oracle_mod.godunov_batch(a, r)
    got = fmm.eval_godunov(torch.from_numpy(a).cuda(), torch.from_numpy(r).cuda()).cpu().numpy()
    assert np.array_equal(got.view(np.uint64), expect.view(np.uint64))


def test_device_local_solver_bitwise_edges(fmm, oracle_mod):
    """Device G against the oracle's G where the square roots and the division
    by 3 leave their usual range: discriminants that are exactly zero, tiny or
    subnormal, r = 0 and r = +inf (a zero speed), equal upwind values, and
    values near the top of the double range, where 2 r^2, 3 r^2, the squared
    differences or a root's numerator overflow."""
    rng = np.random.default_rng(1)
    rows, rs = [], []
    # D2 = 2 r^2 - (a2 - a1)^2 exactly zero: a1 = 0, a2 = d with RN(d d) = RN(2 r r)
    for r in rng.uniform(1e-3, 10.0, size=20000):
        d0 = r * math.sqrt(2.0)
        for k in range(-3, 4):
            d = d0 + k * math.ulp(d0)
            if d * d == 2.0 * r * r:
                rows.append((0.0, d, math.inf))
                rs.append(r)
                rows.append((0.0, d, d))
                rs.append(r)
    assert len(rows) > 10
    # r near the square root of the largest double, where 2 r^2 or 3 r^2
    # overflows, and values near the top of the range, where the sum of a
    # third root's numerator or the squared differences overflow
    for r in (0.0, 1e-300, 1e-200, 1e-160, 1e-155, 1e-120, 1e-100, 5e-324, math.inf, 1e150,
              9e153, 1.1e154, 1.4e154, 1e200, 1e300):
        for base in (0.0, 1e-300, 1e-160, 1.0, 1e150, 1e200, 5e307):
            for spread in (0.0, 0.5, 1.0, 2.0):
                d = spread * (r if math.isfinite(r) else 1.0)
                rows += [(base, base, base), (base, base + d, base + 2 * d), (base, base + d, math.inf),
                         (base, math.inf, math.inf), (base + d, base, base + 0.5 * d)]
                rs += [r] * 5
    a = np.array(rows, dtype=np.float64)
    r = np.array(rs, dtype=np.float64)
    expect = oracle_mod.godunov_batch(a, r)
    got = fmm.eval_godunov(torch.from_numpy(a).cuda(), torch.from_numpy(r).cuda()).cpu().numpy()
    bad = np.nonzero(got.view(np.uint64) != expect.view(np.uint64))[0]
    assert bad.size == 0, [(a[i].tolist(), r[i], got[i], expect[i]) for i in bad[:5]]


def test_single_tile_infinite_stride_two_restarts(fmm, oracle_mod):
    """Sec. 5.3: one subdomain with an infinite stride finishes in 2 restarts."""
    (row,) = load_golden("restarts_single_subdomain.txt")
    assert math.isinf(row[0]) and row[1] == 1
    w = inputs.random_small((8, 8, 8), n_sources=2, seed=3)
    Tg, sg, st = gpu_solve(fmm, w, stride=math.inf, tile_edge=8)
    To, so, _ = oracle_solve(oracle_mod, w)
    assert st.n_restarts == int(row[2])
    assert_parity(Tg, sg, To, so)


@pytest.mark.parametrize("edge", [8, 16])
@pytest.mark.parametrize("stride_h", [2.0, math.inf, 0.5])
def test_point_source_64(fmm, oracle_mod, stride_h, edge):
    w = inputs.point_source(64)
    Tg, sg, st = gpu_solve(fmm, w, stride=stride_h * w.h, tile_edge=edge)
    To, so, sto = oracle_solve(oracle_mod, w)
    assert st.n_accepted == sto.n_accepted == 64 ** 3 - 1
    assert_parity(Tg, sg, To, so)


@pytest.mark.parametrize("edge", [4, 8, 16])
@pytest.mark.parametrize("shape,seed,nsrc,dtype,zero", [
    ((16, 16, 16), 0, 1, torch.float64, 0.0),
    ((37, 29, 45), 1, 3, torch.float32, 0.0),
    ((33, 40, 18), 2, 2, torch.float64, 0.08),
])
def test_random_speed_parity(fmm, oracle_mod, edge, shape, seed, nsrc, dtype, zero):
    w = inputs.random_small(shape, n_sources=nsrc, seed=seed, dtype=dtype, zero_frac=zero)
    To, so, _ = oracle_solve(oracle_mod, w)
    for stride_h in STRIDES_H:
        Tg, sg, st = gpu_solve(fmm, w, stride=stride_h * w.h, tile_edge=edge)
        assert_parity(Tg, sg, To, so)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_extreme_speeds_parity(fmm, oracle_mod, dtype):
    """Speeds at the ends of their range: +inf (r = 0: a point takes its
    smallest upwind value), the largest and the smallest normal FP32 values,
    a subnormal FP32 value, speeds so small that squared values overflow, and
    impassable points (zero, negative and NaN speeds), mixed into a random
    grid."""
    w = inputs.random_small((37, 29, 41), n_sources=3, seed=41, dtype=torch.float64, zero_frac=0.05)
    F = w.F.numpy().copy()
    rng = np.random.default_rng(5)
    src = set(w.seed_idx.tolist())
    # NaN, zero and negative speeds are impassable (no FMM_VALIDATE here);
    # 1e-300 and 1e-160 (FP64 only; 0 in FP32) give values whose squares
    # overflow
    extremes = [np.inf, 3.402823466e38, 1.1754944e-38, 1e-40, 1e30, 1e-30, np.nan, -1.0, -np.inf, -0.0,
                1e-300, 1e-160]
    for k, v in enumerate(extremes):
        cells = rng.choice(F.size, size=200, replace=False)
        for c in cells:
            if int(c) not in src:
                F.reshape(-1)[c] = v
    F = torch.from_numpy(F).to(dtype)
    w = type(w)(w.name, F, w.h, w.seed_idx, w.seed_val, w.width, w.meta)
    To, so, _ = oracle_solve(oracle_mod, w)
    fin = np.isfinite(To)
    # tiny speeds give values near 1e38 at their own points; the others stay
    # of order 1, so the bar is relative per point (1e-12 of max(1, |T|))
    big = np.abs(To) > 1e3
    assert np.any(big) and np.any(fin & ~big)
    for edge in (4, 8, 16):
        for stride_h in (2.0, 3.5, math.inf):
            Tg, sg, st = gpu_solve(fmm, w, stride=stride_h * w.h, tile_edge=edge)
            assert np.array_equal(sg, so), (edge, stride_h, int(np.count_nonzero(sg != so)))
            assert np.array_equal(np.isfinite(Tg), fin)
            err = np.abs(Tg[fin] - To[fin]) / np.maximum(1.0, np.abs(To[fin]))
            assert float(err.max()) <= TOL, (edge, stride_h, float(err.max()))


@pytest.mark.parametrize("edge", [8, 16])
def test_many_tiles_parity(fmm, oracle_mod, edge):
    """A grid of several hundred 16^3 (or thousands of 8^3) tiles with a
    ragged tail on every axis, FP32 speeds and impassable cells."""
    w = inputs.random_small((101, 87, 118), n_sources=5, seed=31, dtype=torch.float32, zero_frac=0.03)
    To, so, _ = oracle_solve(oracle_mod, w)
    for stride_h in (1.5, 4.0, 8.0):
        Tg, sg, st = gpu_solve(fmm, w, stride=stride_h * w.h, tile_edge=edge)
        assert_parity(Tg, sg, To, so)


@pytest.mark.parametrize("width", [0.1, math.inf])
def test_two_sided_spheres(fmm, oracle_mod, width):
    w = inputs.spheres(n=48, n_spheres=5, seed=1, width=width)
    To, so, _ = oracle_solve(oracle_mod, w)
    assert np.any(so & 0x80)
    for edge in (8, 16):
        for stride_h in (2.0, 4.0):
            Tg, sg, st = gpu_solve(fmm, w, stride=stride_h * w.h, tile_edge=edge)
            assert_parity(Tg, sg, To, so, allow_edge=width if math.isfinite(width) else None)


def test_sphere_reinit_256(fmm, oracle_mod):
    """The 256^3 signed-distance reinitialisation workload (8 spheres, band
    0.1) at the paper's stride and at the tuned one, and the run-to-run spread
    of two solves at the same stride (ulps of the larger magnitude)."""
    w = inputs.spheres(n=256)
    To, so, sto = oracle_solve(oracle_mod, w)
    runs = {}
    for stride_h in (2.0, 4.0):
        Tg, sg, st = gpu_solve(fmm, w, stride=stride_h * w.h)
        rep = assert_parity(Tg, sg, To, so, allow_edge=w.width)
        print(f"spheres_256 stride {stride_h}h", rep, st.as_dict(), flush=True)
        runs[stride_h] = (Tg, sg)
    Tg, sg, st = gpu_solve(fmm, w, stride=4.0 * w.h, tile_edge=16)
    rep = assert_parity(Tg, sg, To, so, allow_edge=w.width)
    print("spheres_256 stride 4h, 16^3 tiles", rep, st.as_dict(), flush=True)
    T2, s2, _ = gpu_solve(fmm, w, stride=4.0 * w.h)
    T1, s1 = runs[4.0]
    both = ((s1 & 3) >= 2) & ((s2 & 3) >= 2)
    spread = run_to_run_ulps(T1[both], T2[both])
    print(f"spheres_256 run-to-run at 4h: {spread}", flush=True)
    assert parity_report(T1, s1, T2, s2)["rel"] <= TOL


def run_to_run_ulps(a, b):
    """Largest and mean |a - b| in ulps of max(|a|, |b|), and the share of
    points that differ at all."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    u = np.spacing(np.maximum(np.abs(a), np.abs(b)))
    d = np.abs(a - b) / np.where(u > 0, u, 1.0)
    return {"max_ulps": float(d.max()) if d.size else 0.0, "mean_ulps": float(d.mean()) if d.size else 0.0,
            "frac_differing": float(np.count_nonzero(a != b) / max(1, a.size))}


def test_repeatable(fmm):
    """Two solves of the same input: tiles are claimed dynamically, so a march
    may see a neighbour's halo before or after that neighbour's concurrent
    update, and the local solver's upwind set depends on the point's current
    value.  Valid schedules agree up to rounding (several results are correct
    at the ulp level); the accepted set is identical and the values agree to
    the parity bar."""
    w = inputs.random_small((40, 33, 47), n_sources=3, seed=9)
    T1, s1, _ = gpu_solve(fmm, w, stride=2 * w.h)
    T2, s2, _ = gpu_solve(fmm, w, stride=2 * w.h)
    assert np.array_equal(s1, s2)
    rep = parity_report(T1, s1, T2, s2)
    assert rep["rel"] <= TOL, rep


def test_solver_rejects_host_tensors(fmm):
    """Seeds or outputs on the host raise FMM_EINVAL in the binding, before
    any launch."""
    dev = torch.device("cuda:0")
    s = fmm.Solver((8, 8, 8), 1, 0.1, device=dev)
    F = torch.ones((8, 8, 8), dtype=torch.float64, device=dev)
    idx = torch.zeros(1, dtype=torch.int64, device=dev)
    val = torch.zeros(1, dtype=torch.float64, device=dev)
    T = torch.empty((8, 8, 8), dtype=torch.float64, device=dev)
    for args in ((F, idx.cpu(), val, T), (F, idx, val.cpu(), T), (F, idx, val, T.cpu()),
                 (F, idx, val, T, torch.empty((8, 8, 8), dtype=torch.uint8))):
        with pytest.raises(fmm.FmmError) as ei:
            s.solve_into(*args)
        assert ei.value.code == fmm.FMM_EINVAL


def test_no_seeds(fmm):
    dev = torch.device("cuda:0")
    F = torch.ones((9, 10, 11), dtype=torch.float64, device=dev)
    e = torch.empty(0, dtype=torch.int64, device=dev)
    T, st, stats = fmm.solve(F, 0.1, e, e.to(torch.float64), time_limit_s=30)
    assert torch.all(torch.isinf(T)) and torch.all(st == 0) and stats.n_accepted == 0


def test_residual_and_seeds_verbatim(fmm):
    w = inputs.random_small((30, 31, 29), n_sources=4, seed=12)
    w.seed_val[:] = torch.tensor([0.0, -0.0, 0.01, 0.02], dtype=torch.float64)
    Tg, sg, st = gpu_solve(fmm, w)
    F, idx, val = w.numpy()
    acc = accepted_mask(sg)
    err = backward_error(Tg, F, w.h, acc)
    assert np.max(np.abs(err[acc])) <= 1e-13 * np.max(np.abs(Tg[acc]))
    got = Tg.reshape(-1)[idx]
    assert np.array_equal(got.view(np.uint64), val.view(np.uint64))
    assert np.all(sg.reshape(-1)[idx] == 3)


@pytest.mark.parametrize("bad", ["dup", "range", "nan_seed", "nan_speed"])
def test_device_input_errors(fmm, bad):
    dev = torch.device("cuda:0")
    F = torch.ones((12, 12, 12), dtype=torch.float64, device=dev)
    idx = torch.tensor([5, 700], dtype=torch.int64, device=dev)
    val = torch.zeros(2, dtype=torch.float64, device=dev)
    if bad == "dup":
        idx[1] = 5
    elif bad == "range":
        idx[1] = 12 ** 3
    elif bad == "nan_seed":
        val[1] = math.nan
    else:
        F[3, 4, 5] = math.nan
    with pytest.raises(fmm.FmmError) as ei:
        fmm.solve(F, 0.1, idx, val, validate=True, time_limit_s=30)
    assert ei.value.code == fmm.FMM_EDEVICE


def test_restart_limit(fmm):
    w = inputs.point_source(32)
    dev = torch.device("cuda:0")
    with pytest.raises(fmm.FmmError) as ei:
        fmm.solve(w.F.to(dev), w.h, w.seed_idx.to(dev), w.seed_val.to(dev), max_restarts=1, time_limit_s=30)
    assert ei.value.code == fmm.FMM_ENOCONV


@pytest.mark.parametrize("edge", [8, 16])
@pytest.mark.parametrize("shape,seed", [((37, 29, 45), 1), ((33, 40, 18), 2)])
def test_one_march_per_restart_parity(fmm, oracle_mod, shape, seed, edge):
    """FMM_ONE_MARCH defers the second march of Alg. 16 to the next restart;
    the solution must not change."""
    w = inputs.random_small(shape, n_sources=2, seed=seed, zero_frac=0.05)
    To, so, _ = oracle_solve(oracle_mod, w)
    for stride_h in (0.5, 2.0, 4.0, math.inf):
        Tg, sg, st = gpu_solve(fmm, w, stride=stride_h * w.h, one_march=True, tile_edge=edge)
        assert_parity(Tg, sg, To, so)
    w2 = inputs.spheres(n=40, n_spheres=4, seed=3, width=0.12)
    To, so, _ = oracle_solve(oracle_mod, w2)
    Tg, sg, st = gpu_solve(fmm, w2, one_march=True, tile_edge=edge)
    assert_parity(Tg, sg, To, so, allow_edge=w2.width)


def test_stats_of_unused_workspace(fmm):
    """A workspace no solve has initialised reports FMM_EINVAL, not garbage."""
    s = fmm.Solver((16, 16, 16), 1, 0.1, device=torch.device("cuda:0"))
    s.workspace.zero_()
    with pytest.raises(fmm.FmmError) as ei:
        s.stats()
    assert ei.value.code == fmm.FMM_EINVAL
    a_ws = torch.zeros(4096, dtype=torch.uint8, device=torch.device("cuda:0"))
    st = fmm.FmmAdjointStats()
    rc = fmm.load_library().fmm_get_adjoint_stats(fmm._ptr(a_ws), fmm.ctypes.byref(st), fmm._stream_handle())
    assert rc == fmm.FMM_EINVAL


@pytest.mark.parametrize("stride_h", [0.5, 4.0, math.inf])
def test_stats_consistent(fmm, stride_h):
    """The solve counters obey bounds every correct run meets: each accepted
    non-seed point was solved at least once, a reopened value is a solve that
    improved a released value, every march does at least one round of work or
    none, and a solve needs at least the two restarts that start and end the
    loop."""
    w = inputs.random_small((37, 29, 45), n_sources=3, seed=1, dtype=torch.float32)
    Tg, sg, st = gpu_solve(fmm, w, stride=stride_h * w.h)
    assert st.n_accepted == int(np.sum((sg & 3) == 2))
    assert st.n_solves >= st.n_accepted
    assert 0 <= st.n_reopened <= st.n_solves
    tiles = math.ceil(37 / 8) * math.ceil(29 / 8) * math.ceil(45 / 8)
    assert st.n_tile_marches >= tiles
    assert st.n_rounds <= st.n_solves
    assert st.n_restarts >= 2
    assert st.max_abs_T == float(np.max(np.abs(Tg[(sg & 3) >= 2])))
