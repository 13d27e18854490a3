"""Dense reference adjoint of the discrete Eikonal solve -- TEST INFRASTRUCTURE.

Only the test suite may import this module; the product path never does.

The paper solves the first-order Godunov discretisation (Sec. 2.1, Eqs. 2-3)
and does not differentiate it; the gradient of a loss with respect to the
speed is an extension built on that discretisation.  At a solution T, every
accepted non-seed point p with F_p > 0 satisfies, with u = |T| (the march
works on magnitudes, Sec. 3) and U_p its upwind set,

    sum_{q in U_p} (u_p - u_q)^2 = (h / F_p)^2 .

U_p holds, for the k axes whose values the root of the local solver used
(Alg. 11: the k smallest per-axis upwind values), the neighbour on that axis
with the smaller value.  Differentiating,

    S_p du_p - sum_{q in U_p} (u_p - u_q) du_q = -(h^2 / F_p^3) dF_p,
    S_p = sum_{q in U_p} (u_p - u_q),

while seeds and points outside the accepted set do not move (du = 0).  Written
as A du = B dF, the gradient of a loss L(T) is dL/dF = B^T A^-T (dL/du),
with dL/du_p = sign(T_p) dL/dT_p.  This module builds A as a dense N x N
matrix and solves the transposed system by LU (numpy.linalg.solve): plain and
slow, for grids of a few thousand points.

Per-axis spacing h s_a (the paper allows Delta x, Delta y, Delta z to
differ, Sec. 2.1) weights each term by w = 1 / s_a^2, in the equation and in
its linearisation alike.

Readings this module fixes:
  - the upwind candidates of p are the accepted or seed neighbours on p's side
    with |T_q| < |T_p| (the final values; Alg. 11's filter);
  - on an axis whose two neighbours tie, the lower-index one is taken (the
    derivative has a kink there; either side is a valid one-sided choice);
  - the k axes are those of the sorted per-axis values, ties in axis order.
"""
import numpy as np

from . import ST_ACCEPTED, ST_NEG, ST_SEED, _load, godunov_k, godunov_w


def upwind_sets(F, h, T, status, axis_scale=None):
    """Per accepted non-seed point: list of (neighbour linear index) in U_p.

    ``axis_scale``: per-axis spacing factors (grid spacing h * s_a), or None.
    Returns a dict {p: [q, ...]} over linear indices (C order)."""
    _load()
    n0, n1, n2 = T.shape
    strides = (n1 * n2, n2, 1)
    Tf = T.reshape(-1)
    sf = status.reshape(-1)
    Ff = F.reshape(-1).astype(np.float64)
    out = {}
    for p in range(Tf.size):
        if (sf[p] & 3) != ST_ACCEPTED or not (Ff[p] > 0.0):
            continue
        c = np.unravel_index(p, T.shape)
        up = abs(Tf[p])
        side = sf[p] & ST_NEG
        per_axis = []
        for ax in range(3):
            best_q, best_v = -1, np.inf
            for d in (-1, 1):
                cc = c[ax] + d
                if cc < 0 or cc >= T.shape[ax]:
                    continue
                q = p + d * strides[ax]
                if (sf[q] & 3) not in (ST_ACCEPTED, ST_SEED) or (sf[q] & ST_NEG) != side:
                    continue
                v = abs(Tf[q])
                if v < up and v < best_v:
                    best_q, best_v = q, v
            per_axis.append((best_v, ax, best_q))
        if axis_scale is None:
            u, k = godunov_k(per_axis[0][0], per_axis[1][0], per_axis[2][0], h / Ff[p])
        else:
            u, k = godunov_w(per_axis[0][0], per_axis[1][0], per_axis[2][0], *axis_scale, h / Ff[p])
        chosen = sorted(per_axis, key=lambda t: (t[0], t[1]))[:k]
        out[p] = [(q, ax) for _, ax, q in chosen]
    return out


def dense_adjoint(F, h, T, status, dL_dT, axis_scale=None):
    """dL/dF for a loss whose gradient with respect to T is ``dL_dT``.

    With per-axis spacing h s_a the equation of p is sum_{q in U_p} w_q
    (u_p - u_q)^2 = (h / F_p)^2, w = 1 / s_a^2 for the axis of q, and its
    linearisation carries the same weights.  Zero at seeds, at points
    outside the accepted set and where F <= 0."""
    F = np.asarray(F)
    T = np.asarray(T, dtype=np.float64)
    N = T.size
    sets = upwind_sets(F, h, T, status, axis_scale)
    w = [1.0, 1.0, 1.0] if axis_scale is None else [1.0 / (s * s) for s in axis_scale]
    Tf = np.abs(T.reshape(-1))
    Ff = F.reshape(-1).astype(np.float64)
    A = np.eye(N)
    B = np.zeros(N)
    for p, U in sets.items():
        S = sum(w[ax] * (Tf[p] - Tf[q]) for q, ax in U)
        A[p, p] = S
        for q, ax in U:
            A[p, q] = -w[ax] * (Tf[p] - Tf[q])
        B[p] = -(h * h) / (Ff[p] ** 3)
    sign = np.where(T.reshape(-1) < 0.0, -1.0, 1.0)
    g = np.zeros(N)
    mask = np.zeros(N, dtype=bool)
    mask[list(sets.keys())] = True
    g[mask] = sign[mask] * dL_dT.reshape(-1)[mask]
    lam = np.linalg.solve(A.T, g)
    return (B * lam).reshape(T.shape)
