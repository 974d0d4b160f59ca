"""Seeded synthetic inputs for the recursive multi-scale PCG solver.

This module only draws permeability fields, sources and request streams. It
holds none of the solver's arithmetic (no transmissibilities, no operators), so
the GPU path and the CPU oracle can both consume what it produces without
sharing any of the method.

The paper's own fields (random log-normal permeability with power-law
auto-correlation, Section 4) are not available, so these generators stand in
for them with the same sizes (10^3 to 10^6 unknowns), contrasts (10^2 to 10^9)
and channelised structure.

Array layout: every cell array is float64 with x fastest, i.e. numpy shape
(nz, ny, nx) in C order, flattened to idx = i + nx*(j + ny*k).

Random draws: one ``numpy.random.Generator(PCG64(seed))`` per problem, drawing
uniforms first, then integers, then normals.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

NEUMANN = 0
DIRICHLET = 1


@dataclass
class Problem:
    """One solve: grid, cell-centred permeability per axis, source, boundary data."""

    name: str
    dim: int
    n: tuple  # (nx, ny, nz); nz == 1 in 2-D
    kx: np.ndarray
    ky: np.ndarray
    kz: np.ndarray | None
    f: np.ndarray
    bc_type: list = field(default_factory=lambda: [DIRICHLET, DIRICHLET, NEUMANN, NEUMANN, NEUMANN, NEUMANN])
    bc_value: list = field(default_factory=lambda: [0.0, 1.0, 0.0, 0.0, 0.0, 0.0])
    length: tuple = (1.0, 1.0, 1.0)
    tol: float = 1e-10

    @property
    def N(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _box3_mean(a: np.ndarray) -> np.ndarray:
    """3x3 moving average in the (y, x) plane, window truncated at the edges."""
    ny, nx = a.shape
    s = np.zeros_like(a)
    c = np.zeros_like(a)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            ys = slice(max(0, dy), ny + min(0, dy))
            yd = slice(max(0, -dy), ny + min(0, -dy))
            xs = slice(max(0, dx), nx + min(0, dx))
            xd = slice(max(0, -dx), nx + min(0, -dx))
            s[yd, xd] += a[ys, xs]
            c[yd, xd] += 1.0
    return s / c


def smoothed_lognormal_2d(seed: int, nx: int, ny: int | None = None, lo: float = -1.0, hi: float = 1.0,
                          tol: float = 1e-10, bc_value=(0.0, 1.0), name: str | None = None) -> Problem:
    """log10 k ~ U[lo, hi] i.i.d. per cell, 3x3 box-smoothed; f ~ N(0, 1).

    Dirichlet p = bc_value[0] on x = 0 and bc_value[1] on x = 1, no flow on the
    y boundaries.  lo, hi = -1, 1 is the 32x32 small case; -3, 3 is the
    serving stream's contrast-1e6 field.
    """
    ny = nx if ny is None else ny
    rng = _rng(seed)
    u = rng.uniform(lo, hi, size=(ny, nx))
    f = rng.standard_normal(size=(ny, nx))
    k = 10.0 ** _box3_mean(u)
    k = k.reshape(-1)
    return Problem(name=name or f"smoothed{nx}x{ny}_s{seed}", dim=2, n=(nx, ny, 1), kx=k, ky=k.copy(), kz=None,
                   f=f.reshape(-1).copy(), bc_value=[bc_value[0], bc_value[1], 0.0, 0.0, 0.0, 0.0], tol=tol)


def channelised_2d(seed: int, nx: int = 1024, ny: int | None = None, block: int = 8, amp: float = 4.5,
                   n_channels: int = 5, width: int = 4, tol: float = 1e-10, bc_value=(0.0, 1.0),
                   name: str | None = None) -> Problem:
    """Blocky field with high-permeability channels (contrast 10^(2*amp)).

    log10 k is drawn per block x block cell block from U[-amp, amp]; then
    n_channels horizontal channels, each `width` rows tall across the full x
    extent, are set to log10 k = +amp.  Channel rows y0 ~ UniformInt[0, ny-width]
    (overlaps allowed).  f ~ N(0, 1).
    """
    ny = nx if ny is None else ny
    if nx % block or ny % block:
        raise ValueError("grid sides must be multiples of the block size")
    rng = _rng(seed)
    u = rng.uniform(-amp, amp, size=(ny // block, nx // block))
    y0 = rng.integers(0, ny - width, size=n_channels, endpoint=True)
    f = rng.standard_normal(size=(ny, nx))
    logk = np.repeat(np.repeat(u, block, axis=0), block, axis=1)
    for y in y0:
        logk[y:y + width, :] = amp
    k = (10.0 ** logk).reshape(-1)
    return Problem(name=name or f"channel{nx}x{ny}_s{seed}", dim=2, n=(nx, ny, 1), kx=k, ky=k.copy(), kz=None,
                   f=f.reshape(-1).copy(), bc_value=[bc_value[0], bc_value[1], 0.0, 0.0, 0.0, 0.0], tol=tol)


def layered_3d(seed: int, n: int = 128, ny: int | None = None, nz: int | None = None, n_layers: int = 16,
               amp: float = 3.0, kz_ratio: float = 0.01, tol: float = 1e-10, bc_value=(0.0, 1.0),
               name: str | None = None) -> Problem:
    """Horizontal layers with a diagonal anisotropic permeability tensor.

    The z extent is split into n_layers equal slabs; each slab has
    log10 kx = log10 ky ~ U[-amp, amp] and kz = kz_ratio * kx.  Dirichlet on
    the two x faces (p = 0 at x = 0, p = 1 at x = 1), no flow elsewhere.
    f ~ N(0, 1).
    """
    nx = n
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    if nz % n_layers:
        raise ValueError("nz must be a multiple of n_layers")
    rng = _rng(seed)
    lk = rng.uniform(-amp, amp, size=n_layers)
    f = rng.standard_normal(size=(nz, ny, nx))
    thick = nz // n_layers
    logk = np.repeat(lk, thick)[:, None, None] * np.ones((1, ny, nx))
    kx = (10.0 ** logk).reshape(-1)
    return Problem(name=name or f"layered{nx}x{ny}x{nz}_s{seed}", dim=3, n=(nx, ny, nz), kx=kx, ky=kx.copy(),
                   kz=kx * kz_ratio, f=f.reshape(-1).copy(),
                   bc_value=[bc_value[0], bc_value[1], 0.0, 0.0, 0.0, 0.0], tol=tol)


def anisotropic_strip_2d(seed: int, nx: int = 512, ny: int = 128, ratio: float = 100.0, lo: float = -1.0,
                         hi: float = 1.0, tol: float = 1e-10, name: str | None = None) -> Problem:
    """A strip nx/ny times longer than wide (square cells) with ky = ratio * kx.

    log10 kx ~ U[lo, hi] i.i.d., 3x3 box-smoothed; ky = ratio * kx; Dirichlet
    p = 0 / 1 on the two short (x) ends, no flow on the long sides; f ~ N(0, 1).
    The stand-in for the paper's flow in a narrow channel (Section 5).
    """
    rng = _rng(seed)
    u = rng.uniform(lo, hi, size=(ny, nx))
    f = rng.standard_normal(size=(ny, nx))
    k = (10.0 ** _box3_mean(u)).reshape(-1)
    return Problem(name=name or f"strip{nx}x{ny}_s{seed}", dim=2, n=(nx, ny, 1), kx=k, ky=k * ratio, kz=None,
                   f=f.reshape(-1).copy(), length=(nx / ny, 1.0, 1.0), tol=tol)


def small_case(seed: int = 0) -> Problem:
    """32x32, log10 k ~ U[-1, 1] box-smoothed, FP64, tolerance 1e-10."""
    return smoothed_lognormal_2d(seed, 32, lo=-1.0, hi=1.0, tol=1e-10, name=f"small32_s{seed}")


def channel_1024(seed: int = 0) -> Problem:
    """1024x1024, 8x8 blocks of log10 k ~ U[-4.5, 4.5] plus 5 channels (contrast 1e9)."""
    return channelised_2d(seed, 1024, tol=1e-10, name=f"channel1024_s{seed}")


def layered_128(seed: int = 0) -> Problem:
    """128^3, 16 layers of log10 kx = log10 ky ~ U[-3, 3], kz = kx / 100."""
    return layered_3d(seed, 128, tol=1e-10, name=f"layered128_s{seed}")


@dataclass
class Request:
    idx: int
    arrival_s: float
    side: int
    seed: int


def request_stream(count: int = 4096, rate_per_s: float = 1000.0, sides=(64, 128, 256, 512), arrival_seed: int = 7,
                   first_seed: int = 1000) -> list:
    """Poisson arrivals at a fixed rate; side ~ U{sides}; request i uses seed first_seed + i."""
    rng = _rng(arrival_seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    side_idx = rng.integers(0, len(sides), size=count)
    t = np.cumsum(gaps) - gaps[0]
    return [Request(i, float(t[i]), int(sides[side_idx[i]]), first_seed + i) for i in range(count)]


def request_problem(req: Request, tol: float = 1e-8) -> Problem:
    """The serving stream's field: smoothed log-normal with log10 k ~ U[-3, 3] (contrast 1e6)."""
    return smoothed_lognormal_2d(req.seed, req.side, lo=-3.0, hi=3.0, tol=tol, name=f"req{req.idx}_{req.side}")


def request_fields_torch(req: Request, device, lo: float = -3.0, hi: float = 3.0, stream=None):
    """The serving stream's request drawn on the GPU from the request's seed.

    Same recipe as `smoothed_lognormal_2d` (log10 k ~ U[lo, hi] i.i.d., 3x3
    box mean with the window truncated at the edges, f ~ N(0, 1)), drawn by a
    seeded torch generator on `device` so a request's inputs appear in HBM
    without a host round trip.  Returns (k, f) as flat float64 device tensors.
    """
    import torch
    import torch.nn.functional as F
    n = req.side
    g = torch.Generator(device=device)
    g.manual_seed(req.seed)
    with torch.cuda.stream(stream) if stream is not None else _null():
        u = torch.rand((1, 1, n, n), generator=g, device=device, dtype=torch.float64) * (hi - lo) + lo
        f = torch.randn((n * n,), generator=g, device=device, dtype=torch.float64)
        logk = F.avg_pool2d(u, 3, stride=1, padding=1, count_include_pad=False)
        k = torch.pow(10.0, logk).reshape(-1).contiguous()
    return k, f


class _null:
    def __enter__(self):
        return None

    def __exit__(self, *a):
        return False
