"""Seeded synthetic inputs for the Eikonal workloads.

This module only builds inputs.  It holds none of the solver's arithmetic, and
both the product path and the CPU oracle's tests take their inputs from it.

All grids are node grids on the unit cube: ``n`` points per axis, spacing
``h = 1 / (n - 1)``, point ``(i0, i1, i2)`` at ``(i0 h, i1 h, i2 h)``.  Arrays
are C-contiguous with axis 2 fastest, so the linear index is
``(i0 * n1 + i1) * n2 + i2``.

The workloads mirror the paper's test problems (Sec. 5.1): analytic
interfaces and point sources with prescribed speed functions.  The paper
publishes no dataset, so nothing here stands in for external data.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
import torch


@dataclasses.dataclass
class Workload:
    """One solve: speed field, seeds (linear index + value), band width."""
    name: str
    F: torch.Tensor            # (n0, n1, n2), float32 or float64
    h: float
    seed_idx: torch.Tensor     # int64, on the same device as F
    seed_val: torch.Tensor     # float64
    width: float = math.inf
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def shape(self):
        return tuple(self.F.shape)

    def to(self, device) -> "Workload":
        return dataclasses.replace(self, F=self.F.to(device), seed_idx=self.seed_idx.to(device),
                                   seed_val=self.seed_val.to(device))

    def numpy(self):
        """(F, seed_idx, seed_val) as host numpy arrays."""
        return (self.F.detach().cpu().numpy(), self.seed_idx.detach().cpu().numpy(),
                self.seed_val.detach().cpu().numpy())


def linear_index(shape, i0, i1, i2):
    n0, n1, n2 = shape
    return (np.asarray(i0, dtype=np.int64) * n1 + np.asarray(i1, dtype=np.int64)) * n2 + np.asarray(i2, dtype=np.int64)


def point_source(n: int = 64, speed: float = 1.0, dtype=torch.float64, device="cpu",
                 width: float = math.inf, center: Optional[tuple] = None) -> Workload:
    """Uniform speed, one source with T = 0 at the centre point ``n // 2`` per axis
    (paper case 3, Eq. 13, on a node grid)."""
    c = center if center is not None else (n // 2, n // 2, n // 2)
    F = torch.full((n, n, n), float(speed), dtype=dtype, device=device)
    idx = torch.tensor([int(linear_index((n, n, n), *c))], dtype=torch.int64, device=device)
    val = torch.zeros(1, dtype=torch.float64, device=device)
    return Workload(f"point_source_{n}", F, 1.0 / (n - 1), idx, val, width, {"center": c})


def spheres(n: int = 256, n_spheres: int = 8, seed: int = 0, width: float = 0.1,
            device="cpu") -> Workload:
    """Signed-distance reinitialisation of a union of spheres (cf. case 1).

    Centres ~ U[0.2, 0.8]^3 and radii ~ U[0.05, 0.2] from
    ``numpy.random.default_rng(seed)``; phi(x) = min_k (|x - c_k| - r_k),
    negative inside.  Seeds are the points adjacent to the interface: phi = 0,
    or a 6-neighbour with the opposite sign (negative means phi < 0).  Each seed
    keeps its own phi value.  F = 1 in FP64; both sides march out to |T| <= width.
    """
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.2, 0.8, size=(n_spheres, 3))
    radii = rng.uniform(0.05, 0.2, size=n_spheres)
    h = 1.0 / (n - 1)
    x = np.arange(n, dtype=np.float64) * h
    phi = np.full((n, n, n), np.inf)
    for c, r in zip(centres, radii):
        d = np.sqrt((x[:, None, None] - c[0]) ** 2 + (x[None, :, None] - c[1]) ** 2
                    + (x[None, None, :] - c[2]) ** 2) - r
        np.minimum(phi, d, out=phi)
    neg = phi < 0
    adj = phi == 0
    for ax in range(3):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, n - 1)
        hi[ax] = slice(1, n)
        flip = neg[tuple(lo)] != neg[tuple(hi)]
        adj[tuple(lo)] |= flip
        adj[tuple(hi)] |= flip
    idx = np.flatnonzero(adj.reshape(-1)).astype(np.int64)
    val = phi.reshape(-1)[idx].astype(np.float64)
    F = torch.ones((n, n, n), dtype=torch.float64, device=device)
    return Workload(f"spheres_{n}", F, h, torch.from_numpy(idx).to(device),
                    torch.from_numpy(val).to(device), width,
                    {"seed": seed, "centres": centres.tolist(), "radii": radii.tolist()})


def gaussian_field(n: int, seed: int, corr_len: float = 0.05, device="cpu",
                   shape: Optional[tuple] = None) -> torch.Tensor:
    """Periodic Gaussian random field with unit variance and correlation
    exp(-r^2 / (2 l^2)), l = ``corr_len`` in unit-cube lengths (grid spacing
    1/(n-1)); returned in FP64.

    White noise (FP32 normals from a seeded torch generator on ``device``) is
    convolved, one axis after the other and periodically, with a Gaussian
    kernel of standard deviation l / sqrt(2) truncated at 4 standard
    deviations (the convolution of two such kernels gives the correlation
    above), then shifted and scaled to zero mean and unit variance.  Every
    step is an elementwise FP64 operation in a fixed order, so the same seed,
    shape and device give the same bits on every run (no FFT library whose
    kernel choice could change between runs)."""
    shape = tuple(shape or (n, n, n))
    h = 1.0 / (n - 1)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    g = torch.randn(shape, generator=gen, device=device, dtype=torch.float32).to(torch.float64)
    s = corr_len / math.sqrt(2.0) / h  # kernel standard deviation in grid spacings
    R = max(1, int(math.ceil(4.0 * s)))
    taps = [math.exp(-0.5 * (j / s) ** 2) for j in range(-R, R + 1)]
    tot = math.fsum(taps)
    taps = [t / tot for t in taps]
    for ax in range(3):
        m = shape[ax]
        # periodic extension by R on both sides (tiled as often as needed)
        reps = (R + m - 1) // m
        ext = torch.cat([g] * (2 * reps + 1), dim=ax)
        P = ext.narrow(ax, reps * m - R, m + 2 * R)
        del ext
        out = torch.zeros_like(g)
        for j, wj in enumerate(taps):
            out.add_(P.narrow(ax, j, m), alpha=wj)
        del P
        g = out
    g -= g.mean()
    g /= g.std()
    return g


def fingerprint(t: torch.Tensor) -> str:
    """CRC-32 of a tensor's bytes (copied to the host in chunks), to tie a
    measurement to the exact input it ran on."""
    import zlib
    flat = t.detach().contiguous().reshape(-1)
    crc = 0
    step = 1 << 26
    for a in range(0, flat.numel(), step):
        crc = zlib.crc32(flat[a:a + step].cpu().numpy().tobytes(), crc)
    return f"crc32:{crc:08x}"


def random_speed(n: int = 1024, n_sources: int = 4, seed: int = 0, corr_len: float = 0.05,
                 log_std: float = 0.5, clip=(0.25, 4.0), device="cpu",
                 width: float = math.inf) -> Workload:
    """Speed F = clip(exp(log_std * g), 0.25, 4) stored as FP32, g a seeded
    Gaussian field (correlation length 0.05), and ``n_sources`` distinct point
    sources with T = 0 at uniformly drawn grid points (cf. cases 4-5)."""
    g = gaussian_field(n, seed, corr_len, device=device)
    F = torch.clamp(torch.exp(log_std * g), clip[0], clip[1]).to(torch.float32).contiguous()
    del g
    rng = np.random.default_rng(seed + 7919)
    pts = set()
    while len(pts) < n_sources:
        pts.add(tuple(int(v) for v in rng.integers(0, n, size=3)))
    pts = sorted(pts)
    idx = np.array([linear_index((n, n, n), *p) for p in pts], dtype=np.int64)
    return Workload(f"random_speed_{n}", F, 1.0 / (n - 1), torch.from_numpy(idx).to(device),
                    torch.zeros(len(idx), dtype=torch.float64, device=device), width,
                    {"seed": seed, "sources": pts})


def random_small(shape=(16, 16, 16), n_sources: int = 2, seed: int = 0, fmin: float = 0.5,
                 fmax: float = 2.0, dtype=torch.float64, device="cpu",
                 width: float = math.inf, zero_frac: float = 0.0) -> Workload:
    """Small grids with i.i.d. uniform speed in [fmin, fmax] (optionally a
    fraction of impassable F = 0 points) and random point sources; for parity
    tests over ragged tile counts."""
    rng = np.random.default_rng(seed)
    Fn = rng.uniform(fmin, fmax, size=shape)
    if zero_frac > 0:
        Fn[rng.random(size=shape) < zero_frac] = 0.0
    N = int(np.prod(shape))
    idx = np.sort(rng.choice(N, size=n_sources, replace=False)).astype(np.int64)
    Fn.reshape(-1)[idx] = np.maximum(Fn.reshape(-1)[idx], fmin)
    F = torch.from_numpy(Fn).to(dtype).to(device)
    h = 1.0 / (max(shape) - 1)
    return Workload(f"random_small_{'x'.join(map(str, shape))}", F, h,
                    torch.from_numpy(idx).to(device),
                    torch.zeros(len(idx), dtype=torch.float64, device=device), width,
                    {"seed": seed})


def batch_problems(n_problems: int = 64, seed: int = 0, edge_range=(32, 192), corr_len: float = 0.1,
                   dtype=torch.float64, device="cpu") -> list:
    """A batch of independent full-domain point-source problems of uneven
    size: cube edges drawn uniformly from ``edge_range`` (inclusive), each
    with its own smooth speed field F = 2^tanh(g) in (0.5, 2) (g a seeded
    Gaussian field, correlation length ``corr_len``) stored as ``dtype``, and
    1-4 distinct point sources with T = 0 at uniformly drawn grid points."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_problems):
        n = int(rng.integers(edge_range[0], edge_range[1] + 1))
        ns = int(rng.integers(1, 5))
        g = gaussian_field(n, seed * 100003 + i, corr_len, device=device)
        F = torch.exp(math.log(2.0) * torch.tanh(g.to(torch.float64))).to(dtype).contiguous()
        del g
        pts = set()
        while len(pts) < ns:
            pts.add(tuple(int(v) for v in rng.integers(0, n, size=3)))
        pts = sorted(pts)
        idx = np.array([linear_index((n, n, n), *p) for p in pts], dtype=np.int64)
        out.append(Workload(f"batch_{i}_{n}", F, 1.0 / (n - 1), torch.from_numpy(idx).to(device),
                            torch.zeros(len(idx), dtype=torch.float64, device=device), math.inf,
                            {"seed": seed, "index": i, "sources": pts}))
    return out


def tomography(n: int = 256, n_shots: int = 16, n_receivers: int = 1024, seed: int = 0, corr_len: float = 0.1,
               amp: float = 0.3, perturb: float = 0.03, f_floor: float = 0.1, device="cpu") -> dict:
    """A travel-time tomography setup on the n^3 unit cube (FP64): speed
    F = max(1 + amp g, f_floor) with g a seeded Gaussian field; "observed"
    travel times come from the perturbed model F_obs = max(1 + amp g +
    perturb g', f_floor) with an independent field g'.  ``n_shots`` point
    sources (T = 0) at distinct random points of the z = 0 face (axis 2
    index 0), ``n_receivers`` distinct random points of the z = 1 face (axis 2
    index n - 1), shared by all shots."""
    g = gaussian_field(n, seed, corr_len, device=device).to(torch.float64)
    g2 = gaussian_field(n, seed + 1, corr_len, device=device).to(torch.float64)
    F = torch.clamp(1.0 + amp * g, min=f_floor).contiguous()
    F_obs = torch.clamp(1.0 + amp * g + perturb * g2, min=f_floor).contiguous()
    del g, g2
    rng = np.random.default_rng(seed + 31337)
    face = rng.choice(n * n, size=n_shots, replace=False)
    shots = []
    for f in face:
        i0, i1 = divmod(int(f), n)
        idx = torch.tensor([int(linear_index((n, n, n), i0, i1, 0))], dtype=torch.int64, device=device)
        shots.append((idx, torch.zeros(1, dtype=torch.float64, device=device)))
    rf = rng.choice(n * n, size=n_receivers, replace=False)
    rec = np.array([linear_index((n, n, n), int(f) // n, int(f) % n, n - 1) for f in rf], dtype=np.int64)
    return {"n": n, "h": 1.0 / (n - 1), "F": F, "F_obs": F_obs, "shots": shots,
            "receivers": torch.from_numpy(rec).to(device), "seed": seed}


def _signed_seeds(phi: np.ndarray):
    """Seeds of an interface given by the sign of phi: the points with phi = 0
    or with a 6-neighbour of the opposite sign, valued phi (Alg. 1/8)."""
    s = np.sign(phi)
    adj = s == 0
    for ax in range(3):
        a = [slice(None)] * 3
        b = [slice(None)] * 3
        a[ax], b[ax] = slice(0, -1), slice(1, None)
        ch = s[tuple(a)] * s[tuple(b)] < 0
        adj[tuple(a)] |= ch
        adj[tuple(b)] |= ch
    idx = np.flatnonzero(adj.reshape(-1)).astype(np.int64)
    return idx, phi.reshape(-1)[idx].astype(np.float64).copy()


def paper_case(case: int, n: int = 64, device="cpu") -> Workload:
    """The paper's six test problems (Sec. 5.1) on an n^3 node grid over its
    domain [-0.5, 0.5]^3 (h = 1/(n-1)), FP64, full march:

    1. sphere of radius 0.25 at the centre, interior negative (two-sided);
    2. plane 100x + y + 2z = 0, positive where 100x + y + 2z > 0 (two-sided);
    3-5. point source at the centre with F from Eqs. 13, 14, 15;
    6. point source at the centre, F = 0 inside the four perforated spherical
       shells of Eq. 16 (w = 1/24) and 1 elsewhere.

    Interfaces are seeded with their exact signed distance at the points next
    to a sign change; the point source is the grid point nearest the centre
    (index n // 2 per axis), T = 0."""
    h = 1.0 / (n - 1)
    x = -0.5 + np.arange(n) * h
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    F = np.ones((n, n, n))
    if case == 1:
        idx, val = _signed_seeds(np.sqrt(X ** 2 + Y ** 2 + Z ** 2) - 0.25)
    elif case == 2:
        idx, val = _signed_seeds((100.0 * X + Y + 2.0 * Z) / math.sqrt(100.0 ** 2 + 1.0 + 4.0))
    elif case in (3, 4, 5, 6):
        c = n // 2
        idx = np.array([linear_index((n, n, n), c, c, c)], dtype=np.int64)
        val = np.zeros(1)
        if case == 4:
            F = 1.0 + 0.50 * np.sin(20 * np.pi * X) * np.sin(20 * np.pi * Y) * np.sin(20 * np.pi * Z)
        elif case == 5:
            F = 1.0 - 0.99 * np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y) * np.sin(2 * np.pi * Z)
        elif case == 6:
            w = 1.0 / 24.0
            R = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
            r = np.sqrt(X ** 2 + Y ** 2)
            shells = [(0.15, 0.05, Z < 0), (0.25, 0.10, Z > 0), (0.35, 0.10, Z < 0), (0.45, 0.10, Z > 0)]
            for r0, hole, side in shells:
                F[(R > r0) & (R < r0 + w) & ~((r < hole) & side)] = 0.0
            F.reshape(-1)[idx] = 1.0
    else:
        raise ValueError("case must be 1..6")
    return Workload(f"paper_case{case}_{n}", torch.from_numpy(np.ascontiguousarray(F)).to(device), h,
                    torch.from_numpy(idx).to(device), torch.from_numpy(val).to(device), math.inf,
                    {"case": case})
