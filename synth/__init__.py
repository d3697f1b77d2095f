"""Seeded synthetic inputs shared by the oracle-side tests and the HIP path.

This module draws the inputs of a shot simulation: the Earth model V
(velocity, m/s), the source time function f, and the source/receiver
positions.  It holds none of the method's arithmetic: no stencil, no
time-step update, no damping profile, no (V*dt)^2 scaling.  Both sides of
every parity check take their inputs from here and compute everything else
themselves.

The paper fixes the model only as "wavefield u, Earth model V, source f"
(Sec. III-A, Eq. 1); it names no velocity model or wavelet.  The recipes
below are synthetic stand-ins with the paper's workload shape: a total grid
that includes the damping layer (Table III is reproduced by a 1000^3 grid
with a 27-cell layer around a 946^3 inner box), a layered sedimentary
velocity model, one point source, 1000 time steps (Sec. V-B).
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

__all__ = [
    "Shot",
    "layered_velocity",
    "constant_velocity",
    "ricker",
    "receiver_line",
    "config_c1",
    "config_c2",
    "config_c3",
    "config_small_layered",
    "batch_shapes",
    "serve_requests",
    "CFL",
    "H",
]

H = 10.0      # grid spacing (m), all axes
CFL = 0.4     # dt = CFL * h / v_max
F0 = 15.0     # Ricker peak frequency (Hz)


@dataclass
class Shot:
    """One shot simulation: grid, model, source, receivers, step count.

    Arrays are [nz][ny][nx] with x fastest (Sec. IV, flat 1-D array with x
    innermost).  `w` is the damping-layer width in cells per face; the inner
    box is [w, n-w) on every axis (the grid size includes the layer).
    """
    name: str
    nx: int
    ny: int
    nz: int
    w: int
    dx: float
    dy: float
    dz: float
    dt: float
    vel: np.ndarray                      # float32 [nz][ny][nx], m/s
    steps: int
    src: List[Tuple[int, int, int]] = field(default_factory=list)   # (i, j, k)
    wavelet: Optional[np.ndarray] = None  # float32 [nsrc][steps]
    rec: Optional[np.ndarray] = None      # int32 [nrec][3] (i, j, k)
    seed: int = 0

    @property
    def vmax(self) -> float:
        return float(np.max(self.vel))

    @property
    def points(self) -> int:
        return self.nx * self.ny * self.nz


def ricker(nsamples: int, dt: float, f0: float = F0, t0: Optional[float] = None) -> np.ndarray:
    """Ricker wavelet f(t) = (1 - 2 pi^2 f0^2 tau^2) exp(-pi^2 f0^2 tau^2),
    tau = t - t0, sampled at t = n dt, n = 0..nsamples-1 (a harness constant;
    the library only sees the samples)."""
    if t0 is None:
        t0 = 1.5 / f0
    t = np.arange(nsamples, dtype=np.float64) * dt - t0
    a = (math.pi * f0 * t) ** 2
    return ((1.0 - 2.0 * a) * np.exp(-a)).astype(np.float32)


def _filter_axis(p: np.ndarray, sigma: float, ax: int, threads: int) -> np.ndarray:
    """gaussian_filter1d of p along axis `ax`, computed in slabs cut along
    another axis by a thread pool (each slab's lines are filtered exactly as
    in one call, so the result is the same)."""
    from scipy.ndimage import gaussian_filter1d
    cut = 1 if ax == 0 else 0
    n = p.shape[cut]
    if threads <= 1 or n < 2 * threads:
        return gaussian_filter1d(p, sigma, axis=ax, mode="reflect")
    out = np.empty_like(p)
    bounds = np.linspace(0, n, threads + 1).astype(int)

    def work(k):
        sl = [slice(None)] * 3
        sl[cut] = slice(bounds[k], bounds[k + 1])
        sl = tuple(sl)
        out[sl] = gaussian_filter1d(p[sl], sigma, axis=ax, mode="reflect")

    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(work, range(threads)))
    return out


def _smooth_noise(rng: np.random.Generator, shape, sigma: float) -> np.ndarray:
    p = rng.standard_normal(shape, dtype=np.float32)
    threads = min(16, os.cpu_count() or 1) if p.size >= 1 << 22 else 1
    for ax in range(3):
        p = _filter_axis(p, sigma, ax, threads)
    sd = float(p.std())
    if sd > 0:
        p /= sd
    return p


def layered_velocity(nx: int, ny: int, nz: int, w: int, seed: int,
                     nlayers: int = 8, vlo: float = 1500.0, vhi: float = 4500.0,
                     pert: float = 0.05, sigma_cells: float = 4.0) -> np.ndarray:
    """Seeded layered model: `nlayers` flat layers along z (depth) with
    interfaces at sorted uniform depths inside the inner box, velocities
    sorted uniform(vlo, vhi) increasing with depth, times (1 + pert * p)
    where p is unit-std Gaussian-smoothed noise, clipped to
    [0.9 vlo, 1.1 vhi]."""
    rng = np.random.default_rng(seed)
    lo, hi = w, max(w + 1, nz - w)
    iface = np.sort(rng.integers(lo, hi, size=nlayers - 1))
    vel_layers = np.sort(rng.uniform(vlo, vhi, size=nlayers))
    k = np.arange(nz)
    layer_of_k = np.searchsorted(iface, k, side="right")
    vz = vel_layers[layer_of_k].astype(np.float32)
    v = np.broadcast_to(vz[:, None, None], (nz, ny, nx)).astype(np.float32)
    if pert > 0:
        p = _smooth_noise(rng, (nz, ny, nx), sigma_cells)
        v *= (1.0 + pert * p)
    np.clip(v, 0.9 * vlo, 1.1 * vhi, out=v)
    return np.ascontiguousarray(v, dtype=np.float32)


def constant_velocity(nx: int, ny: int, nz: int, v: float) -> np.ndarray:
    return np.full((nz, ny, nx), v, dtype=np.float32)


def receiver_line(nx: int, j: int, k: int) -> np.ndarray:
    """A line of receivers along x at (j, k): one per grid column."""
    r = np.zeros((nx, 3), dtype=np.int32)
    r[:, 0] = np.arange(nx)
    r[:, 1] = j
    r[:, 2] = k
    return r


def _dt_for(vmax: float, h: float = H) -> float:
    return CFL * h / vmax


def config_c1(steps: int = 100) -> Shot:
    """64^3 grid, h = 10 m, V = 2000 m/s, 16-cell layer, 15 Hz Ricker at the
    grid centre, dt from Courant 0.4, a receiver line 5 cells below the top of
    the inner box (k = w + 5) through the centre (j = 32)."""
    n, w = 64, 16
    vel = constant_velocity(n, n, n, 2000.0)
    dt = _dt_for(2000.0)
    return Shot("c1_64cube", n, n, n, w, H, H, H, dt, vel, steps,
                src=[(32, 32, 32)], wavelet=ricker(steps, dt)[None, :],
                rec=receiver_line(n, 32, w + 5), seed=1001)


def config_c2(steps: int = 1000, n: int = 512, w: int = 20, seed: int = 1002) -> Shot:
    """512^3 grid, 20-cell layer, seeded 8-layer model with a 5 % smoothed
    perturbation, Ricker source near the surface (5 cells below the layer),
    receivers along x at the source depth."""
    vel = layered_velocity(n, n, n, w, seed)
    vmax = float(vel.max())
    dt = _dt_for(vmax)
    c = n // 2
    return Shot(f"c2_{n}cube", n, n, n, w, H, H, H, dt, vel, steps,
                src=[(c, c, w + 5)], wavelet=ricker(steps, dt)[None, :],
                rec=receiver_line(n, c, w + 5), seed=seed)


def config_c3(steps: int = 500) -> Shot:
    """1024^3 grid, 32-cell layer, same generator (another seed)."""
    return config_c2(steps=steps, n=1024, w=32, seed=1003)


def config_small_layered(nx: int, ny: int, nz: int, w: int, steps: int, seed: int,
                         nsrc: int = 1) -> Shot:
    """A small non-cubic layered shot for parity tests (ragged tiles)."""
    vel = layered_velocity(nx, ny, nz, w, seed)
    dt = _dt_for(float(vel.max()))
    rng = np.random.default_rng(seed + 7)
    src = []
    for s in range(nsrc):
        src.append((int(rng.integers(0, nx)), int(rng.integers(0, ny)), int(rng.integers(0, nz))))
    wav = np.stack([ricker(steps, dt, t0=(1.5 + 0.3 * s) / F0) for s in range(nsrc)])
    rec = np.stack([rng.integers(0, nx, 16), rng.integers(0, ny, 16),
                    rng.integers(0, nz, 16)], axis=1).astype(np.int32)
    return Shot(f"small_{nx}x{ny}x{nz}_w{w}", nx, ny, nz, w, H, H, H, dt, vel, steps,
                src=src, wavelet=wav, rec=rec, seed=seed)


def shot_from_shape(nx: int, ny: int, nz: int, steps: int, seed: int, w: int = 20,
                    pert: float = 0.05) -> Shot:
    """A layered-model shot of the given shape: Ricker source 5 cells below the
    layer at the xy centre, a receiver line along x at the source depth."""
    vel = layered_velocity(nx, ny, nz, w, seed, pert=pert)
    dt = _dt_for(float(vel.max()))
    k = min(nz - 1, w + 5)
    return Shot(f"shot_{nx}x{ny}x{nz}", nx, ny, nz, w, H, H, H, dt, vel, steps,
                src=[(nx // 2, ny // 2, k)], wavelet=ricker(steps, dt)[None, :],
                rec=receiver_line(nx, ny // 2, k), seed=seed)


def batch_shapes(count: int = 64, seed: int = 4000, lo: int = 128, hi: int = 384,
                 step: int = 16, smin: int = 200, smax: int = 1000):
    """Seeded shot shapes for the many-shot workload: each axis uniform over
    {lo, lo+step, ..., hi}, steps uniform in [smin, smax]."""
    rng = np.random.default_rng(seed)
    choices = np.arange(lo, hi + 1, step)
    out = []
    for s in range(count):
        nx, ny, nz = (int(v) for v in rng.choice(choices, 3))
        out.append((nx, ny, nz, int(rng.integers(smin, smax + 1)), 1_000_000 * 4 + s))
    return out


def serve_requests(count: int = 256, rate: float = 20.0, seed: int = 5000,
                   lo: int = 96, hi: int = 512, smin: int = 200, smax: int = 2000):
    """Seeded Poisson request stream: arrival time (s), grid shape (multiples
    of 16 in [lo, hi]), step count, storage kind (0 f32, 1 bf16, 2 f16)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, count))
    choices = np.arange(lo, hi + 1, 16)
    out = []
    for s in range(count):
        nx, ny, nz = (int(v) for v in rng.choice(choices, 3))
        out.append(dict(t=float(t[s]), nx=nx, ny=ny, nz=nz,
                        steps=int(rng.integers(smin, smax + 1)),
                        storage=int(rng.integers(0, 3)), seed=1_000_000 * 5 + s))
    return out
