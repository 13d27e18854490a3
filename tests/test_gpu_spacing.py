"""Per-axis grid spacing (the paper's Delta x, Delta y, Delta z, Sec. 2.1) on
the GPU: the weighted local solver in the march, batches and the adjoint,
against the oracle run with the same spacing.  Bars as for uniform grids."""
import math

import numpy as np
import pytest
import torch

from helpers import parity_report
from oracle import adjoint as oadj
from paper_1502_07303_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-12
SCALES = [(1.0, 1.7, 0.6), (0.5, 1.0, 1.0), (2.0, 0.8, 1.3)]


@pytest.fixture(scope="module")
def fmm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1502_07303_amd import fmm as m
    m.load_library()
    return m


@pytest.mark.parametrize("sc", SCALES)
@pytest.mark.parametrize("edge", [4, 8])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_spacing_parity(fmm, oracle_mod, sc, edge, dtype):
    """FP64 and FP32 speeds take different march instantiations (FP64 tiles
    hold r = h/F in LDS, FP32 tiles divide per solve)."""
    dev = torch.device("cuda:0")
    for shape, seed, zero in (((37, 29, 45), 1, 0.0), ((33, 40, 18), 2, 0.08)):
        w = inputs.random_small(shape, n_sources=2, seed=seed, zero_frac=zero, dtype=dtype)
        F, idx, val = w.numpy()
        To, so, _, _ = oracle_mod.solve(F, w.h, idx, val, axis_scale=sc)
        for stride_h in (0.5, 2.0, 3.0, 3.5, 4.0, 4.5, 5.0, math.inf):
            T, st, _ = fmm.solve(w.F.to(dev), w.h, w.seed_idx.to(dev), w.seed_val.to(dev),
                                 stride=stride_h * w.h, tile_edge=edge, axis_scale=sc, time_limit_s=30)
            rep = parity_report(T.cpu().numpy(), st.cpu().numpy(), To, so)
            assert rep["same_status"] and rep["rel"] <= TOL, (shape, stride_h, rep)


def test_spacing_on_axis_sums(fmm):
    """Point source, F = 1: on each axis T is the running sum of h s_a."""
    dev = torch.device("cuda:0")
    sc, h, n = (0.7, 1.0, 2.3), 0.03, 31
    c = n // 2
    idx = torch.tensor([(c * n + c) * n + c], dtype=torch.int64, device=dev)
    T, _, _ = fmm.solve(torch.ones((n, n, n), dtype=torch.float64, device=dev), h, idx,
                        torch.zeros(1, dtype=torch.float64, device=dev), axis_scale=sc)
    T = T.cpu().numpy()
    for ax in range(3):
        acc = 0.0
        for m in range(1, n - c):
            acc = acc + h * sc[ax]
            pos = [c, c, c]
            pos[ax] = c + m
            assert T[tuple(pos)] == acc, (ax, m)


def test_spacing_batch(fmm, oracle_mod):
    dev = torch.device("cuda:0")
    sc = SCALES[0]
    ws = [inputs.random_small((20, 17, 23), n_sources=2, seed=s) for s in (3, 4, 5)]
    b = fmm.BatchSolver([{"F": w.F.to(dev), "h": w.h, "seed_idx": w.seed_idx.to(dev),
                          "seed_val": w.seed_val.to(dev)} for w in ws], axis_scale=sc, time_limit_s=30)
    b.solve()
    b.stats()
    for i, w in enumerate(ws):
        F, idx, val = w.numpy()
        To, so, _, _ = oracle_mod.solve(F, w.h, idx, val, axis_scale=sc)
        rep = parity_report(b.T[i].cpu().numpy(), b.status[i].cpu().numpy(), To, so)
        assert rep["same_status"] and rep["rel"] <= TOL, rep


@pytest.mark.parametrize("sc", SCALES)
def test_spacing_adjoint_against_dense_oracle(fmm, oracle_mod, sc):
    dev = torch.device("cuda:0")
    w = inputs.random_small((14, 16, 13), n_sources=2, seed=7)
    F, idx, val = w.numpy()
    To, so, _, _ = oracle_mod.solve(F, w.h, idx, val, axis_scale=sc)
    rng = np.random.default_rng(3)
    rec = rng.choice(np.flatnonzero((so.reshape(-1) & 3) == 2), size=40, replace=False)
    gT = np.zeros(To.size)
    np.add.at(gT, rec, 2.0 * (To.reshape(-1)[rec] - 0.9 * To.reshape(-1)[rec]))
    gT = gT.reshape(To.shape)
    g_or = oadj.dense_adjoint(F, w.h, To, so, gT, axis_scale=sc)
    Fd = w.F.to(dev)
    g1 = fmm.adjoint(Fd, w.h, torch.from_numpy(To).to(dev), torch.from_numpy(so).to(dev),
                     torch.from_numpy(gT).to(dev), axis_scale=sc).cpu().numpy()
    assert np.max(np.abs(g1 - g_or)) <= 1e-12 * np.max(np.abs(g_or))
    # through autograd: GPU forward with the spacing, then the GPU adjoint
    Fg = Fd.clone().requires_grad_(True)
    T, st = fmm.Eikonal.apply(Fg, w.h, w.seed_idx.to(dev), w.seed_val.to(dev), math.inf, None, sc)
    r = torch.from_numpy(rec).to(dev)
    L = ((T.reshape(-1)[r] - 0.9 * torch.from_numpy(To.reshape(-1)[rec]).to(dev)) ** 2).sum()
    L.backward()
    assert np.max(np.abs(Fg.grad.cpu().numpy() - g_or)) <= 1e-9 * np.max(np.abs(g_or))
