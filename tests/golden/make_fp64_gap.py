#!/usr/bin/env python3
"""Write the float32-vs-float64 goldens of a benchmark-sized shot.

Calls only the oracle (`oracle/`) and the seeded input generator (`synth/`):
it runs the oracle's float64 mode (the truth) and its float32 mode (the fixed
per-point operation order the GPU reproduces bit for bit) on the same shot,
side by side in segments, and records after every segment the relative L2
distance of the float32 wavefield u^n from the float64 one, and of the
receiver traces so far.  At the end it stores, for tests and the benchmark,
a sample of both final fields (one xz plane through the source, every 4th
point) and the traces of every 16th receiver, in both precisions.

The workload is the paper's timing protocol, 1000 steps (Sec. V-B, Table II),
on the synthetic 512^3 stand-in with a 20-cell layer:

    OMP_NUM_THREADS=8 python tests/golden/make_fp64_gap.py --config c2

Outputs `tests/golden/<config>_fp64_gap.json` (scalars, per checkpoint) and
`tests/golden/<config>_fp64_gap.npz` (the samples).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402


def rel_l2(a: np.ndarray, b: np.ndarray) -> float:
    """||a - b|| / ||b|| in float64."""
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    nb = float(np.sqrt(np.dot(b, b)))
    d = a - b
    return float(np.sqrt(np.dot(d, d))) / nb if nb > 0 else float("nan")


def sample_plane(u: np.ndarray, j: int, stride: int) -> np.ndarray:
    """u[k, j, i] for k, i multiples of `stride` (an xz plane through j)."""
    return np.ascontiguousarray(u[::stride, j, ::stride])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="c2", choices=["c2", "c3"])
    ap.add_argument("--segment", type=int, default=100, help="steps between checkpoints")
    ap.add_argument("--steps", type=int, default=None, help="override the config's steps")
    args = ap.parse_args()

    steps = args.steps or (1000 if args.config == "c2" else 500)
    shot = synth.config_c2(steps=steps) if args.config == "c2" else synth.config_c3(steps=steps)
    s = shot
    print(f"{args.config}: {s.nx}x{s.ny}x{s.nz} w{s.w} {steps} steps, "
          f"OMP_NUM_THREADS={os.environ.get('OMP_NUM_THREADS')}", flush=True)
    rec_stride = 16
    plane_stride = 4
    jsrc = s.src[0][1]

    st64 = st32 = None
    tr64 = np.zeros((0, s.rec.shape[0]))
    tr32 = np.zeros((0, s.rec.shape[0]))
    checkpoints = []
    t_start = time.time()
    n = 0
    while n < steps:
        k = min(args.segment, steps - n)
        t0 = time.time()
        r64 = oracle.run_shot(s, steps=k, precision="f64", state=st64, n0=n)
        t1 = time.time()
        r32 = oracle.run_shot(s, steps=k, precision="f32", state=st32, n0=n)
        t2 = time.time()
        n += k
        st64 = dict(u=r64["u"], u_prev=r64["u_prev"], phi=r64["phi"])
        st32 = dict(u=r32["u"], u_prev=r32["u_prev"], phi=r32["phi"])
        tr64 = np.concatenate([tr64, r64["traces"]])
        tr32 = np.concatenate([tr32, r32["traces"]])
        cp = {"step": n, "field_rel_l2": rel_l2(st32["u"], st64["u"]),
              "traces_rel_l2": rel_l2(tr32, tr64),
              "field_l2_f64": float(np.sqrt(np.sum(st64["u"] ** 2))),
              "field_max_abs_f64": float(np.max(np.abs(st64["u"])))}
        checkpoints.append(cp)
        print(f"step {n}: field {cp['field_rel_l2']:.3e} traces {cp['traces_rel_l2']:.3e} "
              f"(f64 {t1 - t0:.0f} s, f32 {t2 - t1:.0f} s)", flush=True)
        del r64, r32

    out = {
        "config": args.config,
        "grid": [s.nx, s.ny, s.nz], "layer": s.w, "steps": steps, "seed": s.seed,
        "dt": s.dt, "h": s.dx, "source": list(s.src[0]),
        "receivers": int(s.rec.shape[0]),
        "what": "oracle float32 mode vs oracle float64 mode on the same seeded shot",
        "checkpoints": checkpoints,
        "field_rel_l2": checkpoints[-1]["field_rel_l2"],
        "traces_rel_l2": checkpoints[-1]["traces_rel_l2"],
        "sample": {"plane_j": jsrc, "plane_stride": plane_stride,
                   "receiver_stride": rec_stride},
        "oracle_threads": int(os.environ.get("OMP_NUM_THREADS", "0") or 0),
        "oracle_seconds": round(time.time() - t_start, 1),
    }
    base = os.path.join(HERE, f"{args.config}_fp64_gap")
    with open(base + ".json", "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    np.savez_compressed(
        base + ".npz",
        plane_f64=sample_plane(st64["u"], jsrc, plane_stride),
        plane_f32=sample_plane(st32["u"], jsrc, plane_stride).astype(np.float32),
        traces_f64=np.ascontiguousarray(tr64[:, ::rec_stride]),
        traces_f32=np.ascontiguousarray(tr32[:, ::rec_stride]).astype(np.float32))
    print(f"wrote {base}.json and .npz ({out['oracle_seconds']} s)", flush=True)


if __name__ == "__main__":
    main()
