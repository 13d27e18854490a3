"""The 1024^3 random-speed workload at full size, in the launch configuration
bench.py times (8^3 tiles, FP32 speeds, stride 3.5h: the stride its autotuner
picks from 3h, 3.5h, 4h and 4.5h).  The oracle cannot march 1.07e9 points in a test,
so the GPU result is checked by properties that hold at any size: every
accepted value satisfies its discrete upwind equation (backward error
<= 1e-13 max|T|), every point is reached (F >= 0.25 everywhere), on the band
|T| <= 0.06 the full solve equals the oracle's banded solve of the same grid
(a banded solve is the full solve restricted to the band), and solves at the
paper's stride 2h, at 4h and again at 3.5h give the same accepted set and values within
the parity bar (the run-to-run spread is printed in ulps).  Full oracle parity
on the same generator at 512^3 is in test_gpu_full512.py."""
import math

import numpy as np
import pytest
import torch

from paper_1502_07303_amd import inputs

pytestmark = pytest.mark.gpu

N1D = 1024
BAND = 0.06
STRIDE_H = 3.5


@pytest.fixture(scope="module")
def full_solve():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1502_07303_amd import fmm
    dev = torch.device("cuda:0")
    w = inputs.random_speed(n=N1D, seed=0, device=dev)
    T, st, stats = fmm.solve(w.F, w.h, w.seed_idx, w.seed_val, stride=STRIDE_H * w.h, tile_edge=8,
                             time_limit_s=100)
    print(f"full solve at {STRIDE_H}h: F {inputs.fingerprint(w.F)}, {stats.as_dict()}", flush=True)
    return w, T, st, stats


def residual_max(T, F, h, seed_mask, slab=64):
    """max over accepted non-seed points of |backward error|, computed with
    torch on the GPU one slab of planes at a time."""
    n0, n1, n2 = T.shape
    inf = math.inf
    worst = 0.0
    for a in range(0, n0, slab):
        b = min(n0, a + slab)
        lo, hi = max(0, a - 1), min(n0, b + 1)
        V = T[lo:hi].abs()
        plane = torch.full((1, n1, n2), inf, dtype=V.dtype, device=V.device)
        if a == 0:
            V = torch.cat([plane, V])
        if b == n0:
            V = torch.cat([V, plane])
        P = torch.nn.functional.pad(V, (1, 1, 1, 1), value=inf)
        u = P[1:-1, 1:-1, 1:-1]
        m = (torch.minimum(P[:-2, 1:-1, 1:-1], P[2:, 1:-1, 1:-1]),
             torch.minimum(P[1:-1, :-2, 1:-1], P[1:-1, 2:, 1:-1]),
             torch.minimum(P[1:-1, 1:-1, :-2], P[1:-1, 1:-1, 2:]))
        d = [torch.clamp(u - mi, min=0.0) for mi in m]
        r = h / F[a:b].to(torch.float64)
        s1 = d[0] + d[1] + d[2]
        e = (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] - r * r) / (2.0 * s1)
        mask = torch.isfinite(u) & (s1 > 0) & ~seed_mask[a:b]
        if bool(mask.any()):
            worst = max(worst, float(e[mask].abs().max()))
        del P, V, d, e, m
    return worst


def test_all_points_accepted(full_solve):
    w, T, st, stats = full_solve
    assert stats.n_accepted == w.F.numel() - w.seed_idx.numel()
    assert bool(torch.all(torch.isfinite(T)))


def test_residual_full(full_solve):
    w, T, st, stats = full_solve
    seeds = torch.zeros(T.numel(), dtype=torch.bool, device=T.device)
    seeds[w.seed_idx] = True
    res = residual_max(T, w.F, w.h, seeds.view(T.shape))
    assert res <= 1e-13 * float(T.abs().max()), res


def test_band_parity_against_oracle(full_solve, oracle_mod):
    w, T, st, stats = full_solve
    F, idx, val = w.numpy()
    To, so, sto, _ = oracle_mod.solve(F, w.h, idx, val, width=BAND)
    Tg = T.cpu().numpy()
    acc_o = ((so & 3) == 2) | ((so & 3) == 3)
    assert sto.n_accepted > 1_000_000
    inband_g = np.abs(Tg) <= BAND
    diff = np.flatnonzero((inband_g != acc_o).reshape(-1))
    if diff.size:
        edge = np.abs(np.abs(Tg.reshape(-1)[diff]) - BAND) <= 1e-12 * BAND
        assert np.all(edge), diff[:10]
    both = acc_o & inband_g
    err = float(np.max(np.abs(Tg[both] - To[both])))
    assert err <= 1e-12 * float(np.max(np.abs(To[both]))), err


def test_other_stride_and_rerun_agree(full_solve):
    """The paper's stride 2h, 4h and a second solve at 3.5h: identical status
    bytes and values within 1e-12 max|T| of the first 3.5h solve; the run-to-run
    spread (tiles are claimed dynamically) is printed in ulps."""
    from paper_1502_07303_amd import fmm
    w, T, st, stats = full_solve
    maxT = float(T.abs().max())
    for sh in (2.0, 4.0, STRIDE_H):
        T2, st2, s2 = fmm.solve(w.F, w.h, w.seed_idx, w.seed_val, stride=sh * w.h, tile_edge=8, time_limit_s=100)
        assert bool(torch.equal(st, st2)), sh
        d = (T2 - T).abs()
        ulps = d / torch.maximum(T.abs(), T2.abs()).clamp(min=1e-300) / 2.0 ** -52
        print(f"stride {sh}h vs {STRIDE_H}h: max|dT| {float(d.max()):.3e} ({float(d.max()) / maxT:.3e} "
              f"relative), max {float(ulps.max()):.1f} ulps, mean {float(ulps.mean()):.4f} ulps, "
              f"{float((d > 0).double().mean()):.4f} of points differ; restarts {s2.n_restarts}", flush=True)
        assert float(d.max()) <= 1e-12 * maxT
        del T2, st2, d, ulps
