"""Pins of the dense reference adjoint (oracle/adjoint.py), CPU only.

The adjoint is pinned to things other than itself: a closed form on a 1-D
line of points, and central finite differences of the oracle's own forward
solve (an independent route to the same derivative)."""
import numpy as np
import pytest

from oracle import adjoint as oadj
from paper_1502_07303_amd import inputs


def test_line_closed_form(oracle_mod):
    """On an n-point line from a seed at index 0, T_i = sum_{j=1..i} h/F_j, so
    dT_i/dF_j = -h/F_j^2 for 1 <= j <= i; with L = sum_i c_i T_i,
    dL/dF_j = -(h/F_j^2) sum_{i>=j} c_i."""
    rng = np.random.default_rng(4)
    n, h = 23, 0.05
    F = rng.uniform(0.5, 2.0, size=(1, 1, n))
    T, st, _, _ = oracle_mod.solve(F, h, np.array([0], dtype=np.int64), np.zeros(1))
    c = rng.normal(size=(1, 1, n))
    g = oadj.dense_adjoint(F, h, T, st, c)
    f = F.reshape(-1)
    tail = np.cumsum(c.reshape(-1)[::-1])[::-1]
    expect = -(h / f ** 2) * tail
    expect[0] = 0.0  # the seed does not depend on F
    np.testing.assert_allclose(g.reshape(-1), expect, rtol=1e-13, atol=1e-15)


def loss_and_grad(T, rec, d):
    Tr = T.reshape(-1)[rec]
    L = float(np.sum((Tr - d) ** 2))
    dL = np.zeros(T.size)
    np.add.at(dL, rec, 2.0 * (Tr - d))
    return L, dL.reshape(T.shape)


def fd_check(oracle_mod, F, h, idx, val, rec, d, cells, eps=1e-6):
    """Central differences of L(F) at ``cells``; cells where the one-sided
    slopes disagree (a kink of the piecewise-smooth solution map within eps)
    are reported as None."""
    out = []
    for c in cells:
        vals = []
        for s in (-1.0, 0.0, 1.0):
            Fp = F.copy()
            Fp.reshape(-1)[c] += s * eps
            T, _, _, _ = oracle_mod.solve(Fp, h, idx, val)
            vals.append(loss_and_grad(T, rec, d)[0])
        lo, mid, hi = vals
        back, fwd = (mid - lo) / eps, (hi - mid) / eps
        central = (hi - lo) / (2 * eps)
        kink = abs(fwd - back) > 1e-4 * max(abs(central), 1e-12)
        out.append(None if kink else central)
    return out


@pytest.mark.parametrize("seed", [0, 1])
def test_finite_differences_random_speed(oracle_mod, seed):
    w = inputs.random_small((10, 11, 12), n_sources=2, seed=seed)
    F, idx, val = w.numpy()
    T, st, _, _ = oracle_mod.solve(F, w.h, idx, val)
    rng = np.random.default_rng(100 + seed)
    rec = rng.choice(T.size, size=30, replace=False)
    d = T.reshape(-1)[rec] * (1.0 + 0.05 * rng.normal(size=30))
    _, dL = loss_and_grad(T, rec, d)
    g = oadj.dense_adjoint(F, w.h, T, st, dL)
    # cells with a gradient well above the finite-difference noise floor
    gm = np.abs(g.reshape(-1))
    cand = np.flatnonzero(gm > 1e-3 * gm.max())
    cells = rng.choice(cand, size=min(20, cand.size), replace=False)
    fd = fd_check(oracle_mod, F, w.h, idx, val, rec, d, cells)
    used = 0
    for c, v in zip(cells, fd):
        if v is None:
            continue
        used += 1
        assert abs(g.reshape(-1)[c] - v) <= 1e-6 * abs(v), (c, g.reshape(-1)[c], v)
    assert used >= 15


def test_finite_differences_two_sided(oracle_mod):
    """Signed distance from spheres (both sides, full march): the sign of T
    enters through d|T|.  Receivers and checked cells are drawn from both
    sides."""
    n = 16
    h = 1.0 / (n - 1)
    x = np.arange(n) * h
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    phi = np.sqrt((X - 0.47) ** 2 + (Y - 0.52) ** 2 + (Z - 0.5) ** 2) - 0.36
    # seeds: points next to a sign change of phi, with value phi
    s = np.sign(phi)
    adj = np.zeros(phi.shape, dtype=bool)
    for ax in range(3):
        a = [slice(None)] * 3
        b = [slice(None)] * 3
        a[ax], b[ax] = slice(0, -1), slice(1, None)
        ch = s[tuple(a)] != s[tuple(b)]
        adj[tuple(a)] |= ch
        adj[tuple(b)] |= ch
    idx = np.flatnonzero(adj.reshape(-1)).astype(np.int64)
    val = phi.reshape(-1)[idx].copy()
    F = np.random.default_rng(5).uniform(0.7, 1.4, size=phi.shape)
    T, st, _, _ = oracle_mod.solve(F, h, idx, val)
    rng = np.random.default_rng(7)
    acc = (st.reshape(-1) & 3) == 2
    neg = T.reshape(-1) < 0
    inside, outside = np.flatnonzero(acc & neg), np.flatnonzero(acc & ~neg)
    assert inside.size >= 30 and outside.size >= 30
    rec = np.concatenate([rng.choice(inside, 12, replace=False), rng.choice(outside, 12, replace=False)])
    d = T.reshape(-1)[rec] + 0.01 * rng.normal(size=rec.size)
    _, dL = loss_and_grad(T, rec, d)
    g = oadj.dense_adjoint(F, h, T, st, dL)
    gm = np.abs(g.reshape(-1))
    big = gm > 1e-3 * gm.max()
    cells = np.concatenate([rng.choice(np.flatnonzero(big & neg), 6, replace=False),
                            rng.choice(np.flatnonzero(big & ~neg), 6, replace=False)])
    fd = fd_check(oracle_mod, F, h, idx, val, rec, d, cells)
    used = {True: 0, False: 0}
    for c, v in zip(cells, fd):
        if v is None:
            continue
        used[bool(neg[c])] += 1
        assert abs(g.reshape(-1)[c] - v) <= 1e-6 * abs(v), (c, g.reshape(-1)[c], v)
    assert used[True] >= 4 and used[False] >= 4


def test_zero_outside_the_system(oracle_mod):
    w = inputs.random_small((9, 8, 7), n_sources=2, seed=3, zero_frac=0.1)
    F, idx, val = w.numpy()
    T, st, _, _ = oracle_mod.solve(F, w.h, idx, val)
    g = oadj.dense_adjoint(F, w.h, T, st, np.ones(T.shape))
    assert np.all(g.reshape(-1)[idx] == 0.0)
    assert np.all(g[F <= 0] == 0.0)
    # every solved point's travel time decreases when its speed grows
    acc = (st & 3) == 2
    assert np.all(g[acc] < 0.0)


def test_line_closed_form_with_spacing(oracle_mod):
    """The 1-D closed form on a line along axis 1 with spacing h s: dL/dF_j =
    -(h s / F_j^2) sum_{i>=j} c_i."""
    rng = np.random.default_rng(9)
    n, h, s = 17, 0.05, 2.5
    F = rng.uniform(0.5, 2.0, size=(1, n, 1))
    sc = (0.7, s, 1.3)
    T, st, _, _ = oracle_mod.solve(F, h, np.array([0], dtype=np.int64), np.zeros(1), axis_scale=sc)
    c = rng.normal(size=(1, n, 1))
    g = oadj.dense_adjoint(F, h, T, st, c, axis_scale=sc)
    f = F.reshape(-1)
    expect = -(h * s / f ** 2) * np.cumsum(c.reshape(-1)[::-1])[::-1]
    expect[0] = 0.0
    np.testing.assert_allclose(g.reshape(-1), expect, rtol=1e-13, atol=1e-15)


def test_finite_differences_with_spacing(oracle_mod):
    w = inputs.random_small((9, 10, 11), n_sources=2, seed=5)
    F, idx, val = w.numpy()
    sc = (0.6, 1.4, 1.0)
    T, st, _, _ = oracle_mod.solve(F, w.h, idx, val, axis_scale=sc)
    rng = np.random.default_rng(55)
    rec = rng.choice(T.size, size=30, replace=False)
    d = T.reshape(-1)[rec] * (1.0 + 0.05 * rng.normal(size=30))
    _, dL = loss_and_grad(T, rec, d)
    g = oadj.dense_adjoint(F, w.h, T, st, dL, axis_scale=sc)
    gm = np.abs(g.reshape(-1))
    cells = rng.choice(np.flatnonzero(gm > 1e-3 * gm.max()), size=16, replace=False)
    used = 0
    for c in cells:
        vals = []
        for s_ in (-1.0, 0.0, 1.0):
            Fp = F.copy()
            Fp.reshape(-1)[c] += s_ * 1e-6
            Tp, _, _, _ = oracle_mod.solve(Fp, w.h, idx, val, axis_scale=sc)
            vals.append(loss_and_grad(Tp, rec, d)[0])
        lo, mid, hi = vals
        if abs((hi - mid) - (mid - lo)) > 1e-4 * abs(hi - lo) / 2:
            continue
        used += 1
        central = (hi - lo) / 2e-6
        assert abs(g.reshape(-1)[c] - central) <= 1e-6 * abs(central), c
    assert used >= 12
