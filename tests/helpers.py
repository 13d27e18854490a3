"""Test-side checks shared by the CPU and GPU suites (numpy only)."""
import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([float(x) for x in line.split()])
    return rows


def axis_upwind(T, side_mask=None):
    """Per-axis minima of the neighbours' values, +inf beyond the array ends.

    ``side_mask`` (bool array) restricts neighbours to the masked points."""
    V = np.where(np.isfinite(T), np.abs(T), np.inf)
    if side_mask is not None:
        V = np.where(side_mask, V, np.inf)
    P = np.pad(V, 1, constant_values=np.inf)
    out = []
    for ax in range(3):
        lo = [slice(1, -1)] * 3
        hi = [slice(1, -1)] * 3
        lo[ax] = slice(0, -2)
        hi[ax] = slice(2, None)
        out.append(np.minimum(P[tuple(lo)], P[tuple(hi)]))
    return out


def backward_error(T, F, h, check_mask):
    """Backward error of the discrete Godunov equation at the masked points.

    For u = |T_p| and the same-side per-axis neighbour minima a_i it returns
    (sum max(u - a_i, 0)^2 - r^2) / (2 sum max(u - a_i, 0)), r = h / F_p: the
    shift of u that would satisfy the equation to first order."""
    neg = T < 0
    err = np.zeros(T.shape)
    u = np.abs(T)
    for side in (False, True):
        sm = neg == side
        a = axis_upwind(T, sm)
        d = [np.maximum(u - ai, 0.0) for ai in a]
        with np.errstate(invalid="ignore", divide="ignore"):
            r = h / F.astype(np.float64)
            s2 = d[0] ** 2 + d[1] ** 2 + d[2] ** 2
            s1 = d[0] + d[1] + d[2]
            e = (s2 - r * r) / (2.0 * s1)
        m = check_mask & sm
        err[m] = e[m]
    return err


def accepted_mask(status):
    return (status & 3) == 2


def seed_mask(status):
    return (status & 3) == 3


def parity_report(T_a, st_a, T_b, st_b):
    """Compare two solves: status bytes, and max |dT| over accepted points."""
    same_status = np.array_equal(st_a, st_b)
    acc = accepted_mask(st_a) | seed_mask(st_a)
    both = acc & (accepted_mask(st_b) | seed_mask(st_b))
    maxT = float(np.max(np.abs(T_b[both]))) if both.any() else 0.0
    dmax = float(np.max(np.abs(T_a[both] - T_b[both]))) if both.any() else 0.0
    return {"same_status": same_status, "n_status_diff": int(np.count_nonzero(st_a != st_b)),
            "max_abs_diff": dmax, "max_T": maxT,
            "rel": dmax / maxT if maxT > 0 else 0.0}


def ulp(x):
    return math.ulp(x)
