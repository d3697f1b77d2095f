"""CPU oracle for the acoustic wave time stepping (test infrastructure).

TEST INFRASTRUCTURE ONLY: only `tests/`, `__graft_entry__.smoke()` and the
CPU-baseline leg of `bench.py` may import this package.  It shares no code
with the HIP library and never imports it.

The arithmetic lives in `oracle.c` (plain loops, FP64 truth and an FP32 mode
with a fixed operation order); this module only builds that file with gcc and
marshals numpy arrays.  Every function cites what it follows:

* `coefficients`   -- Sec. III-A, Eq. 3 (weights are a reading: standard
  8th-order central second-difference weights).
* `vp`             -- Eq. 2, the dt^2 V^2 factor.
* `eta_default`    -- the damping profile (a reading; the paper defers the
  PML to a cited report).
* `run`            -- Alg. 1 with Eq. 2 in the inner region and the layer
  update in the surrounding region.
* `energy`         -- discrete energy of Eq. 2 with damping off (a closed
  form of the scheme, used by the pins).
* `regions`        -- Sec. III-B, the third decomposition (inner + 6 slabs).

Each of these is pinned to something other than itself in
`tests/test_oracle_pins.py` (P1-P14 and closed forms).  The layer is a
reading: its update is pinned by the dense matrix form, the eta = 0
reduction, energy decay and symmetry; its absorption by P14 against a rigid
box, with bounds of the test's own (the paper prints no reflection figure).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

STORAGE = {"f32": 0, "bf16": 1, "f16": 2, "bf16sr": 3}


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (no fused multiply-add beyond explicit fmaf)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
    if force or not os.path.exists(_LIB_PATH):
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if (not os.path.exists(_LIB_PATH)
                or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
            build(force=True)
        lib = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        i32, f64 = C.c_int, C.c_double
        lib.ora_coefficients.argtypes = [f64, f64, f64, P]
        lib.ora_coefficients.restype = None
        lib.ora_stability.argtypes = [f64] * 5
        lib.ora_stability.restype = f64
        lib.ora_is_inner.argtypes = [i32] * 7
        lib.ora_is_inner.restype = i32
        lib.ora_vp.argtypes = [P, C.c_size_t, f64, P, P]
        lib.ora_vp.restype = None
        lib.ora_eta_default.argtypes = [i32, i32, i32, i32, f64, f64, f64, f64, f64, f64, P, P]
        lib.ora_eta_default.restype = None
        lib.ora_eta_axis_tables.argtypes = [i32, i32, i32, i32, f64, f64, f64, f64, f64, P, P, P]
        lib.ora_eta_axis_tables.restype = None
        lib.ora_round_bf16.argtypes = [C.c_float]
        lib.ora_round_bf16.restype = C.c_float
        lib.ora_round_f16.argtypes = [C.c_float]
        lib.ora_round_f16.restype = C.c_float
        lib.ora_round_array.argtypes = [P, C.c_longlong, i32]
        lib.ora_round_array.restype = None
        lib.ora_pcg_hash.argtypes = [C.c_uint32]
        lib.ora_pcg_hash.restype = C.c_uint32
        lib.ora_sr_bits.argtypes = [i32] * 7
        lib.ora_sr_bits.restype = C.c_uint
        lib.ora_round_bf16_sr.argtypes = [C.c_float, C.c_uint]
        lib.ora_round_bf16_sr.restype = C.c_float
        lib.ora_run_f64.argtypes = [i32, i32, i32, i32, f64, f64, f64, P, P, P, f64,
                                    i32, P, P, i32, i32, P, P, i32, i32, P, P, P]
        lib.ora_run_f64.restype = i32
        lib.ora_run_f32.argtypes = [i32, i32, i32, i32, f64, f64, f64, P, P, P, f64, i32,
                                    i32, P, P, i32, i32, P, P, i32, i32, P, P, P]
        lib.ora_run_f32.restype = i32
        lib.ora_energy.argtypes = [i32, i32, i32, f64, f64, f64, P, P, P]
        lib.ora_energy.restype = f64
        lib.ora_regions.argtypes = [i32, i32, i32, i32, i32, P]
        lib.ora_regions.restype = None
        _lib = lib
        return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def set_threads(n: int) -> None:
    """OpenMP thread count for the sweep (the oracle's only parallelism)."""
    os.environ["OMP_NUM_THREADS"] = str(int(n))


def coefficients(dx: float, dy: float, dz: float) -> np.ndarray:
    """[c_xyz, c_x1..4, c_y1..4, c_z1..4] in float64 (Eq. 3)."""
    c = np.zeros(13, dtype=np.float64)
    _load().ora_coefficients(dx, dy, dz, _ptr(c))
    return c


def stability(dx: float, dy: float, dz: float, dt: float, vmax: float) -> float:
    """Stability number of the scheme (<= 1 is stable)."""
    return float(_load().ora_stability(dx, dy, dz, dt, vmax))


def is_inner(nx, ny, nz, w, i, j, k) -> bool:
    return bool(_load().ora_is_inner(nx, ny, nz, w, i, j, k))


def vp(vel: np.ndarray, dt: float):
    """(V dt)^2 as (float64 array, float32 array rounded once from it)."""
    vel = np.ascontiguousarray(vel, dtype=np.float32)
    v64 = np.empty(vel.shape, np.float64)
    v32 = np.empty(vel.shape, np.float32)
    _load().ora_vp(_ptr(vel), vel.size, float(dt), _ptr(v64), _ptr(v32))
    return v64, v32


def eta_default(nx, ny, nz, w, dx, dy, dz, dt, vmax, refl=1e-3):
    """Default damping profile as (float64, float32) arrays [nz][ny][nx]."""
    e64 = np.empty((nz, ny, nx), np.float64)
    e32 = np.empty((nz, ny, nx), np.float32)
    _load().ora_eta_default(nx, ny, nz, w, dx, dy, dz, dt, vmax, refl, _ptr(e64), _ptr(e32))
    return e64, e32


def eta_axis_tables(nx, ny, nz, w, dx, dy, dz, vmax, refl=1e-3):
    """Axis terms (t_x, t_y, t_z) of the default profile, float64 arrays of
    n_a + 2 entries for i = -1..n_a; eta = dt ((t_x + t_y) + t_z)."""
    t = [np.empty(n + 2, np.float64) for n in (nx, ny, nz)]
    _load().ora_eta_axis_tables(nx, ny, nz, w, dx, dy, dz, vmax, refl,
                                _ptr(t[0]), _ptr(t[1]), _ptr(t[2]))
    return tuple(t)


def round_bf16(x: float) -> float:
    return float(_load().ora_round_bf16(float(x)))


def round_f16(x: float) -> float:
    return float(_load().ora_round_f16(float(x)))


def pcg_hash(v: int) -> int:
    """The 32-bit "pcg" hash (PCG step and RXS-M-XS permutation) of v."""
    return int(_load().ora_pcg_hash(v & 0xFFFFFFFF))


def sr_bits(n: int, nx: int, ny: int, nz: int, i: int, j: int, k: int) -> int:
    """The 16 random bits of point (i, j, k) at step n (stochastic rounding)."""
    return int(_load().ora_sr_bits(n, nx, ny, nz, i, j, k))


def round_bf16_sr(x: float, r: int) -> float:
    """Stochastic rounding of float32 x to bfloat16 with 16 random bits r."""
    return float(_load().ora_round_bf16_sr(float(x), int(r)))


def regions(nx, ny, nz, w, order: int = 0) -> np.ndarray:
    """7 boxes (x0, y0, z0, ex, ey, ez): inner, then the six layer slabs."""
    out = np.zeros((7, 6), dtype=np.int32)
    _load().ora_regions(nx, ny, nz, w, order, _ptr(out))
    return out


def energy(vp64: np.ndarray, u_next, u_now, dx, dy, dz) -> float:
    """E^{n+1/2} of Eq. 2 with damping off (float64 accumulation)."""
    nz, ny, nx = vp64.shape
    a = np.ascontiguousarray(u_next, dtype=np.float64)
    b = np.ascontiguousarray(u_now, dtype=np.float64)
    v = np.ascontiguousarray(vp64, dtype=np.float64)
    return float(_load().ora_energy(nx, ny, nz, dx, dy, dz, _ptr(v), _ptr(a), _ptr(b)))


def run(nx, ny, nz, w, dx, dy, dz, dt, vel, steps, *,
        src=(), wavelet=None, rec=None, precision="f64", storage="f32",
        eta="default", refl=1e-3, state=None, n0=0, damping=True):
    """Advance `steps` steps of Alg. 1 from `state` (default: all zero).

    vel      float32 [nz][ny][nx] velocity (m/s); vp = (V dt)^2 is derived here.
    src      sequence of (i, j, k); wavelet float32 [nsrc][nsamp] (w[n]).
    rec      int32 [nrec][3] receiver (i, j, k) or None.
    eta      "default" (the profile from vmax, its gradient from the axis
             terms), "default-array" (the same profile as a plain array:
             gradient from differences of the array, zero beyond the faces),
             an explicit array (array semantics), or None.
    damping  False runs Eq. 2 on every point (no layer formula).
    state    dict(u=u^n, u_prev=u^{n-1}, phi=phi^n) or None (zeros).
    Returns dict(u, u_prev, phi, traces[steps][nrec] float64, vp, eta).
    """
    lib = _load()
    shape = (nz, ny, nx)
    vel = np.ascontiguousarray(vel, dtype=np.float32)
    assert vel.shape == shape
    vp64, vp32 = vp(vel, dt)
    etab = None
    if not damping:
        e64 = e32 = None
    elif isinstance(eta, str) and eta in ("default", "default-array"):
        e64, e32 = eta_default(nx, ny, nz, w, dx, dy, dz, dt, float(vel.max()), refl)
        if eta == "default":
            etab = np.ascontiguousarray(np.concatenate(
                eta_axis_tables(nx, ny, nz, w, dx, dy, dz, float(vel.max()), refl)))
    elif eta is None:
        e64 = e32 = None
    else:
        e64 = np.ascontiguousarray(eta, dtype=np.float64)
        e32 = np.ascontiguousarray(eta, dtype=np.float32)
    src = list(src)
    nsrc = len(src)
    src_a = np.ascontiguousarray(np.array(src, dtype=np.int32).reshape(nsrc, 3))
    if nsrc:
        wav = np.ascontiguousarray(np.asarray(wavelet, dtype=np.float32).reshape(nsrc, -1))
        nsamp = wav.shape[1]
    else:
        wav = np.zeros((0, 1), np.float32)
        nsamp = 0
    if rec is None:
        rec_a = np.zeros((0, 3), np.int32)
    else:
        rec_a = np.ascontiguousarray(np.asarray(rec, dtype=np.int32).reshape(-1, 3))
    nrec = rec_a.shape[0]
    traces = np.zeros((steps, nrec), np.float64)
    dt_np = np.float64 if precision == "f64" else np.float32
    if state is None:
        u = np.zeros(shape, dt_np)
        up = np.zeros(shape, dt_np)
        ph = np.zeros(shape, dt_np)
    else:
        u = np.array(state["u"], dtype=dt_np, order="C", copy=True)
        up = np.array(state["u_prev"], dtype=dt_np, order="C", copy=True)
        ph = np.array(state.get("phi", np.zeros(shape)), dtype=dt_np, order="C", copy=True)
    if precision == "f64":
        rc = lib.ora_run_f64(nx, ny, nz, w, dx, dy, dz, _ptr(vp64), _ptr(e64), _ptr(etab), dt,
                             nsrc, _ptr(src_a), _ptr(wav), nsamp, nrec, _ptr(rec_a),
                             _ptr(traces), n0, steps, _ptr(u), _ptr(up), _ptr(ph))
        vpo, eo = vp64, e64
    elif precision == "f32":
        if storage != "f32" and state is not None:
            for arr in (u, up):   # the state as stored (each element rounded)
                lib.ora_round_array(_ptr(arr), arr.size, STORAGE[storage])
        rc = lib.ora_run_f32(nx, ny, nz, w, dx, dy, dz, _ptr(vp32), _ptr(e32), _ptr(etab), dt,
                             STORAGE[storage],
                             nsrc, _ptr(src_a), _ptr(wav), nsamp, nrec, _ptr(rec_a),
                             _ptr(traces), n0, steps, _ptr(u), _ptr(up), _ptr(ph))
        vpo, eo = vp32, e32
    else:
        raise ValueError(precision)
    if rc != 0:
        raise RuntimeError("oracle run failed")
    return dict(u=u, u_prev=up, phi=ph, traces=traces, vp=vpo, eta=eo)


def run_shot(shot, steps=None, **kw):
    """`run` on a synth.Shot."""
    s = shot
    return run(s.nx, s.ny, s.nz, s.w, s.dx, s.dy, s.dz, s.dt, s.vel,
               s.steps if steps is None else steps,
               src=s.src, wavelet=s.wavelet, rec=s.rec, **kw)
