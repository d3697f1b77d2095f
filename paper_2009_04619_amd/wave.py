"""ctypes binding of the C ABI in include/wave.h (argument marshalling only).

Every function of the header is exposed under the same name and returns the
same status codes (a non-zero status raises `WaveError` in the `Shot`
convenience class; the plain functions return it).  All computation runs in
the HIP kernels of `libwave.so`; there is no fallback: importing this module
fails loudly when the library is missing.

PyTorch serves only as the device allocator (the arena is a torch uint8
tensor) and as the source of the HIP stream.  torch is imported before the
library is loaded so that both share one HIP runtime.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library binds to)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwave.so")

WAVE_OK, WAVE_EINVAL, WAVE_ENOMEM, WAVE_EUNSTABLE = 0, -1, -2, -3
WAVE_EDEVICE, WAVE_ESTATE, WAVE_EBUDGET = -4, -5, -6
WAVE_F32, WAVE_BF16, WAVE_F16 = 0, 1, 2
WAVE_DAMPING_OFF = 1
WAVE_ETA_ARRAY = 2
WAVE_TWO_STEP = 4
WAVE_STOCH_ROUND = 8
WAVE_FIELD_U, WAVE_FIELD_UPREV, WAVE_FIELD_PHI, WAVE_FIELD_VP, WAVE_FIELD_ETA = 0, 1, 2, 3, 4
WAVE_KERNEL_DIRECT, WAVE_KERNEL_STREAM, WAVE_KERNEL_STREAM2 = 0, 1, 2
WAVE_KERNEL_GMEM, WAVE_KERNEL_RING, WAVE_KERNEL_SHIFT, WAVE_KERNEL_PAIR = 3, 4, 5, 6
WAVE_KERNEL_SEMI, WAVE_KERNEL_PERSIST, WAVE_KERNEL_SHUFFLE = 7, 8, 9
STORAGE = {"f32": WAVE_F32, "bf16": WAVE_BF16, "f16": WAVE_F16}

EXPORTED = [
    "wave_bytes_required", "wave_admit", "wave_coefficients", "wave_stability", "wave_eta_default",
    "wave_alloc", "wave_free", "wave_inject", "wave_record", "wave_step", "wave_sync",
    "wave_step_count", "wave_read_field", "wave_write_field", "wave_read_traces",
    "wave_energy", "wave_energy_noalloc", "wave_set_kernel", "wave_set_timing", "wave_read_timing",
    "wave_sweep_bytes", "wave_stream_copy", "wave_stream_mix", "wave_strerror", "wave_last_error",
    "wave_batch_bytes_required", "wave_batch_create", "wave_batch_add", "wave_batch_remove",
    "wave_batch_run", "wave_batch_remaining", "wave_batch_set_kernel", "wave_batch_set_graph",
    "wave_batch_free", "wave_tune", "wave_batch_tune",
]


class wave_desc(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("w", C.c_int32),
        ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double), ("dt", C.c_double),
        ("storage", C.c_int32), ("flags", C.c_int32), ("refl", C.c_double),
        ("max_src", C.c_int32), ("max_rec", C.c_int32), ("max_steps", C.c_int32),
        ("reserved", C.c_int32),
    ]


class WaveError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {wave_strerror(status)} ({status}): {wave_last_error()}")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2009_04619_amd.build` "
            "(there is no fallback path)")
    lib = C.CDLL(LIB_PATH)
    P, i32, i64, f64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
    D = C.POINTER(wave_desc)
    sig = {
        "wave_bytes_required": (sz, [D]),
        "wave_admit": (C.c_int, [D, sz, sz, C.POINTER(sz), C.POINTER(i32)]),
        "wave_coefficients": (C.c_int, [D, P]),
        "wave_stability": (f64, [D, f64]),
        "wave_eta_default": (C.c_int, [D, f64, P]),
        "wave_alloc": (C.c_int, [D, P, P, P, sz, P, C.POINTER(P)]),
        "wave_free": (C.c_int, [P]),
        "wave_inject": (C.c_int, [P, i32, i32, i32, P, i32]),
        "wave_record": (C.c_int, [P, P, i32]),
        "wave_step": (C.c_int, [P, i32]),
        "wave_sync": (C.c_int, [P]),
        "wave_step_count": (i64, [P]),
        "wave_read_field": (C.c_int, [P, i32, P]),
        "wave_write_field": (C.c_int, [P, i32, P]),
        "wave_read_traces": (C.c_int, [P, P, C.POINTER(i32)]),
        "wave_energy": (C.c_int, [P, C.POINTER(f64)]),
        "wave_energy_noalloc": (C.c_int, [P, P]),
        "wave_set_kernel": (C.c_int, [P, i32, i32, i32, i32]),
        "wave_set_timing": (C.c_int, [P, i32]),
        "wave_read_timing": (C.c_int, [P, C.POINTER(f64), C.POINTER(i64)]),
        "wave_sweep_bytes": (f64, [P]),
        "wave_stream_copy": (C.c_int, [P, P, sz, P]),
        "wave_stream_mix": (C.c_int, [i32, P, P, P, P, sz, P]),
        "wave_batch_bytes_required": (sz, [i32]),
        "wave_batch_create": (C.c_int, [i32, i32, P, sz, P, C.POINTER(P)]),
        "wave_batch_add": (C.c_int, [P, P, i32]),
        "wave_batch_remove": (C.c_int, [P, P]),
        "wave_batch_run": (C.c_int, [P, i32]),
        "wave_batch_remaining": (C.c_int, [P, P, C.POINTER(i32)]),
        "wave_batch_set_kernel": (C.c_int, [P, i32, i32]),
        "wave_batch_set_graph": (C.c_int, [P, i32]),
        "wave_batch_free": (C.c_int, [P]),
        "wave_tune": (C.c_int, [P, i32, P]),
        "wave_batch_tune": (C.c_int, [P, i32, P]),
        "wave_strerror": (C.c_char_p, [C.c_int]),
        "wave_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# ---- the C functions under their own names ---------------------------------
def wave_bytes_required(d: wave_desc) -> int:
    return int(_lib.wave_bytes_required(C.byref(d)))


def wave_admit(d: wave_desc, budget_bytes: int, in_use_bytes: int):
    """(status, bytes needed, fits now) of a request under a memory budget."""
    need = C.c_size_t(0)
    fits = C.c_int32(0)
    rc = _lib.wave_admit(C.byref(d), C.c_size_t(int(budget_bytes)), C.c_size_t(int(in_use_bytes)),
                         C.byref(need), C.byref(fits))
    return int(rc), int(need.value), bool(fits.value)


def wave_coefficients(d: wave_desc):
    out = np.zeros(13, np.float32)
    return int(_lib.wave_coefficients(C.byref(d), _p(out))), out


def wave_stability(d: wave_desc, vmax: float) -> float:
    return float(_lib.wave_stability(C.byref(d), float(vmax)))


def wave_eta_default(d: wave_desc, vmax: float):
    out = np.zeros((d.nz, d.ny, d.nx), np.float32)
    return int(_lib.wave_eta_default(C.byref(d), float(vmax), _p(out))), out


def wave_alloc(d: wave_desc, vel: np.ndarray, eta: Optional[np.ndarray], arena_ptr: int,
               arena_bytes: int, stream_ptr: int):
    ctx = C.c_void_p()
    rc = _lib.wave_alloc(C.byref(d), _p(vel), _p(eta), C.c_void_p(arena_ptr), arena_bytes,
                         C.c_void_p(stream_ptr), C.byref(ctx))
    return int(rc), ctx


def wave_free(ctx) -> int:
    return int(_lib.wave_free(ctx))


def wave_inject(ctx, i: int, j: int, k: int, samples: np.ndarray) -> int:
    s = np.ascontiguousarray(samples, dtype=np.float32)
    return int(_lib.wave_inject(ctx, i, j, k, _p(s), s.size))


def wave_record(ctx, ijk: np.ndarray) -> int:
    a = np.ascontiguousarray(np.asarray(ijk, dtype=np.int32).reshape(-1, 3))
    return int(_lib.wave_record(ctx, _p(a), a.shape[0]))


def wave_step(ctx, n: int) -> int:
    return int(_lib.wave_step(ctx, int(n)))


def wave_sync(ctx) -> int:
    return int(_lib.wave_sync(ctx))


def wave_step_count(ctx) -> int:
    return int(_lib.wave_step_count(ctx))


def wave_read_field(ctx, which: int, out: np.ndarray) -> int:
    assert out.dtype == np.float32 and out.flags.c_contiguous
    return int(_lib.wave_read_field(ctx, which, _p(out)))


def wave_write_field(ctx, which: int, data: np.ndarray) -> int:
    a = np.ascontiguousarray(data, dtype=np.float32)
    return int(_lib.wave_write_field(ctx, which, _p(a)))


def wave_read_traces(ctx, out: Optional[np.ndarray]):
    n = C.c_int32()
    rc = _lib.wave_read_traces(ctx, _p(out), C.byref(n))
    return int(rc), int(n.value)


def wave_energy(ctx):
    e = C.c_double()
    rc = _lib.wave_energy(ctx, C.byref(e))
    return int(rc), float(e.value)


def wave_energy_noalloc(ctx, dev_out_ptr: int) -> int:
    """Enqueue the energy into 2 doubles of device memory at dev_out_ptr
    (kinetic, potential); no allocation, no wait."""
    return int(_lib.wave_energy_noalloc(ctx, dev_out_ptr))


def wave_set_kernel(ctx, variant: int, rows_per_wave: int = 1, waves_per_group: int = 16,
                    zchunk: int = 0) -> int:
    return int(_lib.wave_set_kernel(ctx, variant, rows_per_wave, waves_per_group, zchunk))


def wave_set_timing(ctx, on: bool) -> int:
    return int(_lib.wave_set_timing(ctx, 1 if on else 0))


def wave_read_timing(ctx):
    ms, n = C.c_double(), C.c_int64()
    rc = _lib.wave_read_timing(ctx, C.byref(ms), C.byref(n))
    return int(rc), float(ms.value), int(n.value)


def wave_sweep_bytes(ctx) -> float:
    return float(_lib.wave_sweep_bytes(ctx))


def wave_stream_mix(kind: int, dst_ptr: int, a_ptr: int, b_ptr: int, c_ptr: int, nbytes: int,
                    stream_ptr: int) -> int:
    return int(_lib.wave_stream_mix(kind, C.c_void_p(dst_ptr), C.c_void_p(a_ptr),
                                    C.c_void_p(b_ptr), C.c_void_p(c_ptr), nbytes,
                                    C.c_void_p(stream_ptr)))


def wave_stream_copy(dst_ptr: int, src_ptr: int, nbytes: int, stream_ptr: int) -> int:
    return int(_lib.wave_stream_copy(C.c_void_p(dst_ptr), C.c_void_p(src_ptr), nbytes,
                                     C.c_void_p(stream_ptr)))


def wave_batch_bytes_required(max_shots: int) -> int:
    return int(_lib.wave_batch_bytes_required(int(max_shots)))


def wave_batch_create(storage: int, max_shots: int, arena_ptr: int, arena_bytes: int,
                      stream_ptr: int):
    b = C.c_void_p()
    rc = _lib.wave_batch_create(int(storage), int(max_shots), C.c_void_p(arena_ptr), arena_bytes,
                                C.c_void_p(stream_ptr), C.byref(b))
    return int(rc), b


def wave_batch_add(b, ctx, nsteps: int) -> int:
    return int(_lib.wave_batch_add(b, ctx, int(nsteps)))


def wave_batch_remove(b, ctx) -> int:
    return int(_lib.wave_batch_remove(b, ctx))


def wave_batch_run(b, n: int) -> int:
    return int(_lib.wave_batch_run(b, int(n)))


def wave_batch_remaining(b, ctx):
    r = C.c_int32()
    rc = _lib.wave_batch_remaining(b, ctx, C.byref(r))
    return int(rc), int(r.value)


def wave_batch_set_kernel(b, rows_per_wave: int, waves_per_group: int) -> int:
    return int(_lib.wave_batch_set_kernel(b, int(rows_per_wave), int(waves_per_group)))


def wave_batch_set_graph(b, steps_per_graph: int) -> int:
    return int(_lib.wave_batch_set_graph(b, int(steps_per_graph)))


def wave_batch_free(b) -> int:
    return int(_lib.wave_batch_free(b))


def wave_tune(ctx, trial_steps: int):
    out = np.zeros(4, np.int32)
    rc = _lib.wave_tune(ctx, int(trial_steps), _p(out))
    return int(rc), tuple(int(v) for v in out)


def wave_batch_tune(b, trial_steps: int):
    out = np.zeros(2, np.int32)
    rc = _lib.wave_batch_tune(b, int(trial_steps), _p(out))
    return int(rc), tuple(int(v) for v in out)


def wave_strerror(status: int) -> str:
    return _lib.wave_strerror(int(status)).decode()


def wave_last_error() -> str:
    return _lib.wave_last_error().decode()


def make_desc(nx, ny, nz, w, dx, dy, dz, dt, storage="f32", damping=True, refl=1e-3,
              max_src=4, max_rec=0, max_steps=0, eta_array=False, two_step=False,
              stochastic_round=False) -> wave_desc:
    d = wave_desc()
    d.nx, d.ny, d.nz, d.w = int(nx), int(ny), int(nz), int(w)
    d.dx, d.dy, d.dz, d.dt = float(dx), float(dy), float(dz), float(dt)
    d.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    d.flags = ((0 if damping else WAVE_DAMPING_OFF) | (WAVE_ETA_ARRAY if (eta_array and damping) else 0)
               | (WAVE_TWO_STEP if two_step else 0) | (WAVE_STOCH_ROUND if stochastic_round else 0))
    d.refl = float(refl)
    d.max_src, d.max_rec, d.max_steps = int(max_src), int(max_rec), int(max_steps)
    d.reserved = 0
    return d


def _check(rc: int, what: str):
    if rc != WAVE_OK:
        raise WaveError(rc, what)


class Shot:
    """One simulation context on a GPU: owns its torch arena and the ctx.

    Arguments mirror `wave_desc`; `vel` is float32 [nz][ny][nx] (m/s) and
    `eta` an explicit damping array or None for the default profile."""

    def __init__(self, nx, ny, nz, w, dx, dy, dz, dt, vel, *, eta=None, storage="f32",
                 damping=True, refl=1e-3, max_src=4, max_rec=0, max_steps=0,
                 device="cuda:0", stream=None, two_step=False, stochastic_round=False):
        self.device = torch.device(device)
        self.desc = make_desc(nx, ny, nz, w, dx, dy, dz, dt, storage, damping, refl,
                              max_src, max_rec, max_steps,
                              eta_array=eta is not None and damping, two_step=two_step,
                              stochastic_round=stochastic_round)
        nbytes = wave_bytes_required(self.desc)
        if nbytes == 0:
            raise WaveError(WAVE_EINVAL, "wave_bytes_required")
        self.nbytes = nbytes
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        # the arena belongs to the context's stream (the caching allocator
        # reuses it there only after the context has waited for its work)
        with torch.cuda.stream(self.stream):
            self.arena = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        vel = np.ascontiguousarray(vel, dtype=np.float32)
        assert vel.shape == (nz, ny, nx)
        eta_a = None if (eta is None or not damping) else np.ascontiguousarray(eta, dtype=np.float32)
        rc, self.ctx = wave_alloc(self.desc, vel, eta_a, self.arena.data_ptr(), nbytes,
                                  self.stream.cuda_stream)
        _check(rc, "wave_alloc")
        self.shape = (nz, ny, nx)
        self.nrec = 0

    def inject(self, i, j, k, samples):
        _check(wave_inject(self.ctx, i, j, k, samples), "wave_inject")

    def record(self, ijk):
        a = np.asarray(ijk, dtype=np.int32).reshape(-1, 3)
        _check(wave_record(self.ctx, a), "wave_record")
        self.nrec = a.shape[0]

    def step(self, n):
        _check(wave_step(self.ctx, n), "wave_step")

    def sync(self):
        _check(wave_sync(self.ctx), "wave_sync")

    def read(self, which=WAVE_FIELD_U) -> np.ndarray:
        out = np.empty(self.shape, np.float32)
        _check(wave_read_field(self.ctx, which, out), "wave_read_field")
        return out

    def write(self, which, data):
        _check(wave_write_field(self.ctx, which, data), "wave_write_field")

    def traces(self) -> np.ndarray:
        rc, n = wave_read_traces(self.ctx, None)
        _check(rc, "wave_read_traces")
        out = np.zeros((n, self.nrec), np.float64)
        if n and self.nrec:
            rc, _ = wave_read_traces(self.ctx, out)
            _check(rc, "wave_read_traces")
        return out

    def energy(self) -> float:
        rc, e = wave_energy(self.ctx)
        _check(rc, "wave_energy")
        return e

    def set_kernel(self, variant, rows_per_wave=1, waves_per_group=16, zchunk=0):
        _check(wave_set_kernel(self.ctx, variant, rows_per_wave, waves_per_group, zchunk),
               "wave_set_kernel")

    def set_timing(self, on):
        _check(wave_set_timing(self.ctx, on), "wave_set_timing")

    def read_timing(self):
        rc, ms, n = wave_read_timing(self.ctx)
        _check(rc, "wave_read_timing")
        return ms, n

    def sweep_bytes(self) -> float:
        return wave_sweep_bytes(self.ctx)

    def tune(self, trial_steps: int):
        """Advance trial_steps steps per candidate tile and keep the fastest."""
        rc, cfg = wave_tune(self.ctx, trial_steps)
        _check(rc, "wave_tune")
        return cfg

    @property
    def step_count(self) -> int:
        return wave_step_count(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            wave_free(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def shot_from_synth(s, storage="f32", damping=True, device="cuda:0", max_steps=None, eta=None,
                    stream=None, two_step=False, stochastic_round=False):
    """A `Shot` for a synth.Shot (sources injected, receivers set)."""
    steps = s.steps if max_steps is None else max_steps
    nrec = 0 if s.rec is None else len(s.rec)
    sh = Shot(s.nx, s.ny, s.nz, s.w, s.dx, s.dy, s.dz, s.dt, s.vel, eta=eta, storage=storage,
              damping=damping, max_src=max(1, len(s.src)), max_rec=nrec,
              max_steps=max(steps, s.wavelet.shape[1] if s.wavelet is not None else 0),
              device=device, stream=stream, two_step=two_step, stochastic_round=stochastic_round)
    for q, (i, j, k) in enumerate(s.src):
        sh.inject(i, j, k, s.wavelet[q])
    if nrec:
        sh.record(s.rec)
    return sh


class Batch:
    """Several `Shot`s advanced together (one sweep launch per step for all).

    All members share the batch's storage type; their streams may differ
    from the batch's (the library orders them with events)."""

    def __init__(self, storage="f32", max_shots=64, device="cuda:0", stream=None):
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        n = wave_batch_bytes_required(max_shots)
        if n == 0:
            raise WaveError(WAVE_EINVAL, "wave_batch_bytes_required")
        self.arena = torch.empty(n, dtype=torch.uint8, device=self.device)
        st = STORAGE[storage] if isinstance(storage, str) else int(storage)
        rc, self.b = wave_batch_create(st, max_shots, self.arena.data_ptr(), n,
                                       self.stream.cuda_stream)
        _check(rc, "wave_batch_create")
        self.members = []

    def add(self, shot: "Shot", nsteps: int):
        _check(wave_batch_add(self.b, shot.ctx, nsteps), "wave_batch_add")
        self.members.append(shot)

    def remove(self, shot: "Shot"):
        _check(wave_batch_remove(self.b, shot.ctx), "wave_batch_remove")
        self.members.remove(shot)

    def run(self, n: int):
        _check(wave_batch_run(self.b, n), "wave_batch_run")

    def remaining(self, shot: "Shot") -> int:
        rc, r = wave_batch_remaining(self.b, shot.ctx)
        _check(rc, "wave_batch_remaining")
        return r

    def set_kernel(self, rows_per_wave=1, waves_per_group=16):
        _check(wave_batch_set_kernel(self.b, rows_per_wave, waves_per_group), "wave_batch_set_kernel")

    def tune(self, trial_steps: int):
        rc, cfg = wave_batch_tune(self.b, trial_steps)
        _check(rc, "wave_batch_tune")
        return cfg

    def set_graph(self, steps_per_graph: int):
        _check(wave_batch_set_graph(self.b, steps_per_graph), "wave_batch_set_graph")

    def close(self):
        if getattr(self, "b", None):
            wave_batch_free(self.b)
            self.b = None
            self.members = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
