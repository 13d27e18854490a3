"""GPU batches: many problems in one persistent launch, each with its own
restart loop (Alg. 16 per problem), through the C ABI.

Bar: every problem of a batch has the oracle's accepted set and status bytes
and max |T - T_oracle| <= 1e-12 max |T| (the same bar as single solves), and
its own restart count equals that of the same problem solved alone."""
import math

import numpy as np
import pytest
import torch

from helpers import parity_report
from paper_1502_07303_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def fmm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1502_07303_amd import fmm as m
    m.load_library()
    return m


def as_problem(w, dev):
    return {"F": w.F.to(dev).contiguous(), "h": w.h, "seed_idx": w.seed_idx.to(dev), "seed_val": w.seed_val.to(dev)}


def oracle_of(oracle_mod, w, width=math.inf):
    F, idx, val = w.numpy()
    T, st, stats, _ = oracle_mod.solve(F, w.h, idx, val, width=width)
    return T, st, stats


def check(Tg, sg, To, so, tol=TOL):
    rep = parity_report(Tg, sg, To, so)
    assert rep["same_status"], rep
    assert rep["rel"] <= tol, rep
    return rep


def mixed_batch(dtype=torch.float64):
    """Uneven shapes (ragged tile counts), speeds, spacings and seed counts,
    including a single-tile problem and one without seeds."""
    ws = [inputs.random_small((37, 29, 45), n_sources=3, seed=1, dtype=dtype),
          inputs.random_small((8, 8, 8), n_sources=2, seed=3, dtype=dtype),
          inputs.random_small((16, 16, 16), n_sources=1, seed=0, dtype=dtype, zero_frac=0.05),
          inputs.random_small((33, 40, 18), n_sources=2, seed=2, dtype=dtype, zero_frac=0.08),
          inputs.random_small((5, 70, 9), n_sources=4, seed=5, dtype=dtype)]
    empty = inputs.random_small((12, 13, 14), n_sources=1, seed=6, dtype=dtype)
    empty.seed_idx = empty.seed_idx[:0]
    empty.seed_val = empty.seed_val[:0]
    ws.append(empty)
    return ws


@pytest.mark.parametrize("edge", [4, 8, 16])
@pytest.mark.parametrize("stride_h", [0.5, 2.0, 3.0, 3.5, 4.0, 4.5, 5.0, math.inf])
def test_batch_parity_mixed(fmm, oracle_mod, edge, stride_h):
    dev = torch.device("cuda:0")
    ws = mixed_batch()
    kw = {"stride_h": stride_h} if math.isfinite(stride_h) else {"stride": math.inf}
    b = fmm.BatchSolver([as_problem(w, dev) for w in ws], tile_edge=edge, time_limit_s=30, **kw)
    b.solve()
    st = b.stats()
    for i, w in enumerate(ws):
        To, so, sto = oracle_of(oracle_mod, w)
        check(b.T[i].cpu().numpy(), b.status[i].cpu().numpy(), To, so)
        assert st[i].n_accepted == sto.n_accepted
    assert st[5].n_accepted == 0 and st[5].n_restarts == 1
    assert bool(torch.all(torch.isinf(b.T[5])))


def test_batch_matches_single_solves(fmm):
    """Each problem's solution and restart count are those of a solve of that
    problem alone: the batch couples nothing but the work list."""
    dev = torch.device("cuda:0")
    ws = mixed_batch(torch.float32)
    b = fmm.BatchSolver([as_problem(w, dev) for w in ws], time_limit_s=30)
    b.solve()
    st = b.stats()
    for i, w in enumerate(ws):
        T, s, one = fmm.solve(w.F.to(dev), w.h, w.seed_idx.to(dev), w.seed_val.to(dev), time_limit_s=30)
        check(b.T[i].cpu().numpy(), b.status[i].cpu().numpy(), T.cpu().numpy(), s.cpu().numpy())
        assert st[i].n_restarts == one.n_restarts, (i, st[i].n_restarts, one.n_restarts)
        assert st[i].n_accepted == one.n_accepted


def test_batch_single_tile_exits_on_its_own(fmm):
    """Sec. 5.3: one subdomain with an infinite stride needs 2 restarts; in a
    batch with a large problem that needs many, it still reports 2."""
    dev = torch.device("cuda:0")
    small = inputs.random_small((8, 8, 8), n_sources=2, seed=3)
    big = inputs.point_source(64)
    b = fmm.BatchSolver([as_problem(small, dev), as_problem(big, dev)], stride=math.inf, tile_edge=8,
                        time_limit_s=30)
    b.solve()
    st = b.stats()
    assert st[0].n_restarts == 2
    b2 = fmm.BatchSolver([as_problem(small, dev), as_problem(big, dev)], stride_h=0.5, tile_edge=8,
                         time_limit_s=30)
    b2.solve()
    st2 = b2.stats()
    assert st2[1].n_restarts > st2[0].n_restarts


def test_batch_two_sided_band(fmm, oracle_mod):
    dev = torch.device("cuda:0")
    ws = [inputs.spheres(n=40, n_spheres=4, seed=3, width=0.12), inputs.spheres(n=48, n_spheres=5, seed=1,
                                                                               width=0.12)]
    b = fmm.BatchSolver([as_problem(w, dev) for w in ws], band_width=0.12, time_limit_s=30)
    b.solve()
    b.stats()
    for i, w in enumerate(ws):
        To, so, _ = oracle_of(oracle_mod, w, width=0.12)
        sg = b.status[i].cpu().numpy()
        diff = np.flatnonzero(sg.reshape(-1) != so.reshape(-1))
        edge = np.abs(np.abs(To.reshape(-1)[diff]) - 0.12) <= 1e-12 * 0.12
        assert np.all(edge | np.isinf(To.reshape(-1)[diff]))
        rep = parity_report(b.T[i].cpu().numpy(), sg, To, so)
        assert rep["rel"] <= TOL, rep


def test_batch_graph_replay(fmm):
    """The launch sequence captured into a HIP graph and replayed: every replay
    equals the eager solve of the inputs current at replay time (speeds
    changed in place between replays, eager work in between)."""
    dev = torch.device("cuda:0")
    ws = mixed_batch()
    probs = [as_problem(w, dev) for w in ws]
    b = fmm.BatchSolver(probs, time_limit_s=30)
    b.solve()
    b.stats()
    ref = [t.clone() for t in b.T]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            b.solve(stream=s)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        scale = 2.0 ** rep
        for p, w in zip(probs, ws):
            p["F"].copy_(w.F.to(dev) * scale)  # F -> cF gives T -> T/c, bitwise for c = 2^k
        junk = torch.randn(1 << 20, device=dev).sum()  # unrelated eager work between replays
        torch.cuda.synchronize()
        for t in b.T:
            t.fill_(-7.0)
        g.replay()
        torch.cuda.synchronize()
        st = b.stats()
        assert st[0].device_error == 0
        for i in range(len(ws)):
            # F -> 2^k F scales T by 2^-k exactly; schedules differ only by rounding
            got = b.T[i].cpu().numpy()
            exp = ref[i].cpu().numpy() / scale
            assert np.array_equal(np.isinf(got), np.isinf(exp)), (rep, i)
            fin = np.isfinite(exp)
            if fin.any():
                err = np.max(np.abs(got[fin] - exp[fin]))
                assert err <= TOL * np.max(np.abs(exp[fin])), (rep, i, err)
        del junk


def test_autotune_picks_a_candidate_and_stays_exact(fmm, oracle_mod):
    dev = torch.device("cuda:0")
    ws = inputs.batch_problems(6, seed=1, edge_range=(16, 40))
    b = fmm.BatchSolver([as_problem(w, dev) for w in ws], time_limit_s=30, workspace_edges=[4, 8, 16])
    times = b.tune(edges=(4, 8, 16), strides_h=(1.0, 2.0, 4.0), reps=1)
    assert len(times) == 9 and all(v > 0 for v in times.values())
    best = min(times, key=times.get)
    assert (b.opts.tile_edge, b.opts.stride_h) == best
    b.solve()
    b.stats()
    for i, w in enumerate(ws):
        To, so, _ = oracle_of(oracle_mod, w)
        check(b.T[i].cpu().numpy(), b.status[i].cpu().numpy(), To, so)


def test_batch_64_full_config(fmm, oracle_mod):
    """The 64-problem batch (cube edges 32-192, smooth speeds in (0.5, 2),
    1-4 sources): all points accepted in every problem, and the eight smallest
    problems equal their oracle solutions."""
    dev = torch.device("cuda:0")
    ws = inputs.batch_problems(64, seed=0, device=dev)
    b = fmm.BatchSolver([as_problem(w, dev) for w in ws], time_limit_s=60, with_status=True)
    b.solve()
    st = b.stats()
    for i, w in enumerate(ws):
        n = w.F.numel()
        assert st[i].n_accepted + w.seed_idx.numel() == n, i
    order = sorted(range(64), key=lambda i: ws[i].F.numel())[:8]
    for i in order:
        To, so, _ = oracle_of(oracle_mod, ws[i].to("cpu"))
        check(b.T[i].cpu().numpy(), b.status[i].cpu().numpy(), To, so)
