#!/usr/bin/env python3
"""Write the float64 goldens of the benchmark workloads (calls only `oracle/`).

Calls only the oracle (`oracle/`) and the seeded input generator (`synth/`).
Four workloads, one per `--config`:

c2     The 512^3 grid with a 20-cell layer, 1000 steps (the paper's timing
       protocol, Sec. V-B, Table II).  The oracle's float64 mode (the truth)
       and its float32-arithmetic mode with the given wavefield storage
       (`--storage f32|bf16|f16`; f32 is the fixed per-point operation order
       the GPU reproduces bit for bit) run side by side in segments; after
       every segment the relative L2 distance of u^n and of the traces so far
       is recorded.  At the end a sample of both final fields (one xz plane
       through the source, every 4th point) and the traces of every 16th
       receiver are stored in both precisions.
c3     The 1024^3 grid with a 32-cell layer, 500 steps, float32 storage.  The
       two modes do not fit in host memory together, so the float64 run goes
       first and leaves its final u^n in a scratch file (`--scratch`), then
       the float32 run is compared with it.
batch  A subset of the 64-shot batch workload (each axis in {128, .., 384},
       200-1000 steps, 5 % perturbed layered models): the shot with the most
       point-steps, the one with the largest grid and the two with the fewest
       point-steps.  Float64 only: the final u^n sampled on the xz plane
       through the source (every 8th point) and the traces of every 8th
       receiver, stored as float32 (rounding the truth to float32 adds at
       most 6e-8 relative).  The benchmark compares its batched results
       (float32 and bf16 storage) against these.
serve  A subset of the Poisson serving workload: the request with the
       largest grid and, for each storage type, the five requests with the
       most steps among grids of at most 5e6 points (a type with fewer such
       requests takes the ones of fewest point-steps next); float64 samples
       as for `batch`.

`--reuse` keeps the stored entries of a `batch` or `serve` golden whose
request, grid, step count and seed are unchanged (results of an earlier run
of this script) and runs the oracle only for the others.

    OMP_NUM_THREADS=8 python tests/golden/make_fp64_gap.py --config c2
    OMP_NUM_THREADS=8 python tests/golden/make_fp64_gap.py --config c2 --storage bf16
    OMP_NUM_THREADS=8 python tests/golden/make_fp64_gap.py --config batch
    OMP_NUM_THREADS=8 python tests/golden/make_fp64_gap.py --config serve [--reuse]
    OMP_NUM_THREADS=8 python tests/golden/make_fp64_gap.py --config c3 --scratch /big/dir

Outputs `tests/golden/<name>_fp64_gap.json` (scalars) and `.npz` (samples),
<name> = c2, c2_bf16, c2_f16, c3, batch, serve.
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


def threads() -> int:
    return int(os.environ.get("OMP_NUM_THREADS", "0") or 0)


def write(name: str, meta: dict, arrays: dict):
    base = os.path.join(HERE, f"{name}_fp64_gap")
    with open(base + ".json", "w") as f:
        json.dump(meta, f, indent=1)
        f.write("\n")
    np.savez_compressed(base + ".npz", **arrays)
    print(f"wrote {base}.json and .npz", flush=True)


def side_by_side(s, steps: int, storage: str, segment: int):
    """float64 and float32-arithmetic (given storage) runs of one shot in
    lockstep; returns the final states, traces and per-segment distances."""
    st64 = st32 = None
    tr64 = np.zeros((0, s.rec.shape[0]))
    tr32 = np.zeros((0, s.rec.shape[0]))
    checkpoints = []
    n = 0
    while n < steps:
        k = min(segment, steps - n)
        t0 = time.time()
        r64 = oracle.run_shot(s, steps=k, precision="f64", state=st64, n0=n)
        t1 = time.time()
        r32 = oracle.run_shot(s, steps=k, precision="f32", storage=storage, state=st32, n0=n)
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
              f"(f64 {t1 - t0:.0f} s, {storage} {t2 - t1:.0f} s)", flush=True)
        del r64, r32
    return st64, st32, tr64, tr32, checkpoints


def config_c2(args):
    steps = args.steps or 1000
    s = synth.config_c2(steps=steps)
    print(f"c2: {s.nx}x{s.ny}x{s.nz} w{s.w} {steps} steps, storage {args.storage}, "
          f"OMP_NUM_THREADS={threads()}", flush=True)
    rec_stride, plane_stride = 16, 4
    jsrc = s.src[0][1]
    t_start = time.time()
    st64, st32, tr64, tr32, checkpoints = side_by_side(s, steps, args.storage, args.segment)
    name = "c2" if args.storage == "f32" else f"c2_{args.storage}"
    meta = {
        "config": "c2",
        "grid": [s.nx, s.ny, s.nz], "layer": s.w, "steps": steps, "seed": s.seed,
        "dt": s.dt, "h": s.dx, "source": list(s.src[0]),
        "receivers": int(s.rec.shape[0]),
        "what": "oracle float32 mode vs oracle float64 mode on the same seeded shot"
                if args.storage == "f32" else
                f"oracle float32-arithmetic mode with {args.storage} storage vs oracle float64 "
                "mode on the same seeded shot",
        "checkpoints": checkpoints,
        "field_rel_l2": checkpoints[-1]["field_rel_l2"],
        "traces_rel_l2": checkpoints[-1]["traces_rel_l2"],
        "sample": {"plane_j": jsrc, "plane_stride": plane_stride,
                   "receiver_stride": rec_stride},
        "oracle_threads": threads(),
        "oracle_seconds": round(time.time() - t_start, 1),
    }
    arrays = dict(
        plane_f64=sample_plane(st64["u"], jsrc, plane_stride),
        plane_f32=sample_plane(st32["u"], jsrc, plane_stride).astype(np.float32),
        traces_f64=np.ascontiguousarray(tr64[:, ::rec_stride]),
        traces_f32=np.ascontiguousarray(tr32[:, ::rec_stride]).astype(np.float32))
    write(name, meta, arrays)


def config_c3(args):
    steps = args.steps or 500
    s = synth.config_c3(steps=steps)
    if not args.scratch:
        sys.exit("--config c3 needs --scratch DIR (about 9 GB for the float64 field)")
    os.makedirs(args.scratch, exist_ok=True)
    print(f"c3: {s.nx}x{s.ny}x{s.nz} w{s.w} {steps} steps, OMP_NUM_THREADS={threads()}", flush=True)
    rec_stride, plane_stride = 32, 8
    jsrc = s.src[0][1]
    t0 = time.time()
    r = oracle.run_shot(s, steps=steps, precision="f64")
    t64 = time.time() - t0
    f64_path = os.path.join(args.scratch, "c3_u_f64.npy")
    np.save(f64_path, r["u"])
    tr64 = r["traces"].copy()
    plane64 = sample_plane(r["u"], jsrc, plane_stride)
    del r
    print(f"float64 done ({t64:.0f} s)", flush=True)
    t1 = time.time()
    r = oracle.run_shot(s, steps=steps, precision="f32")
    t32 = time.time() - t1
    u64 = np.load(f64_path, mmap_mode="r")
    field = rel_l2(r["u"], u64)
    meta = {
        "config": "c3",
        "grid": [s.nx, s.ny, s.nz], "layer": s.w, "steps": steps, "seed": s.seed,
        "dt": s.dt, "h": s.dx, "source": list(s.src[0]),
        "receivers": int(s.rec.shape[0]),
        "storage": "f32",
        "what": "oracle float32 mode vs oracle float64 mode on the same seeded shot "
                "(run one after the other)",
        "field_rel_l2": field,
        "traces_rel_l2": rel_l2(r["traces"], tr64),
        "field_l2_f64": float(np.sqrt(np.sum(np.square(u64, dtype=np.float64)))),
        "sample": {"plane_j": jsrc, "plane_stride": plane_stride,
                   "receiver_stride": rec_stride},
        "oracle_threads": threads(),
        "oracle_seconds": {"f64": round(t64, 1), "f32": round(t32, 1)},
    }
    arrays = dict(plane_f64=plane64,
                  plane_f32=sample_plane(r["u"], jsrc, plane_stride).astype(np.float32),
                  traces_f64=np.ascontiguousarray(tr64[:, ::rec_stride]),
                  traces_f32=np.ascontiguousarray(r["traces"][:, ::rec_stride]).astype(np.float32))
    print(f"c3: field {field:.3e} traces {meta['traces_rel_l2']:.3e}", flush=True)
    write("c3", meta, arrays)
    os.remove(f64_path)


def stored(name: str):
    """The entries and arrays of a stored golden by key ({} when absent)."""
    base = os.path.join(HERE, f"{name}_fp64_gap")
    if not (os.path.exists(base + ".json") and os.path.exists(base + ".npz")):
        return {}, {}
    meta = json.load(open(base + ".json"))
    arr = np.load(base + ".npz")
    return {e["key"]: e for e in meta["members"]}, {k: arr[k] for k in arr.files}


def sampled_f64(name: str, items, what: str, reuse: bool = False):
    """float64 runs of a list of (key, shot, extra) and their samples;
    with `reuse`, a stored entry of the same key, grid, steps and seed is
    kept instead of run again."""
    plane_stride, rec_stride = 8, 8
    entries, arrays = [], {}
    old_entries, old_arrays = stored(name) if reuse else ({}, {})
    t_start = time.time()
    for key, s, extra in items:
        t0 = time.time()
        e = old_entries.get(key)
        if e and e["grid"] == [s.nx, s.ny, s.nz] and e["steps"] == s.steps \
                and e["seed"] == s.seed and all(e.get(k) == v for k, v in extra.items()):
            entries.append(e)
            for part in ("plane", "traces"):
                arrays[f"{key}_{part}"] = old_arrays[f"{key}_{part}"]
            print(f"{key}: kept", flush=True)
            continue
        r = oracle.run_shot(s, precision="f64")
        jsrc = s.src[0][1]
        arrays[f"{key}_plane"] = sample_plane(r["u"], jsrc, plane_stride).astype(np.float32)
        arrays[f"{key}_traces"] = np.ascontiguousarray(r["traces"][:, ::rec_stride]).astype(np.float32)
        e = {"key": key, "grid": [s.nx, s.ny, s.nz], "steps": s.steps, "seed": s.seed,
             "plane_j": jsrc, "oracle_seconds": round(time.time() - t0, 1)}
        e.update(extra)
        entries.append(e)
        print(f"{key}: {s.nx}x{s.ny}x{s.nz} {s.steps} steps ({time.time() - t0:.0f} s)", flush=True)
        del r
    meta = {"config": name, "what": what, "members": entries,
            "sample": {"plane_stride": plane_stride, "receiver_stride": rec_stride,
                       "dtype": "float32 (the float64 result rounded once)"},
            "oracle_threads": threads(),
            "oracle_seconds": round(time.time() - t_start, 1)}
    write(name, meta, arrays)


def config_batch(args):
    shapes = synth.batch_shapes()
    work = [nx * ny * nz * st for (nx, ny, nz, st, _) in shapes]
    grid = [nx * ny * nz for (nx, ny, nz, _, _) in shapes]
    order = np.argsort(work, kind="stable")
    pick = []
    for i in (int(np.argmax(work)), int(np.argmax(grid)), int(order[0]), int(order[1])):
        if i not in pick:
            pick.append(i)
    items = []
    for i in pick:
        nx, ny, nz, st, seed = shapes[i]
        items.append((f"b{i}", synth.shot_from_shape(nx, ny, nz, st, seed), {"index": i}))
    sampled_f64("batch", items, "float64 oracle results of a subset of the 64-shot batch "
                "(synth.batch_shapes, 5 % perturbed layered models)", reuse=args.reuse)


def config_serve(args):
    reqs = synth.serve_requests()
    grid = [r["nx"] * r["ny"] * r["nz"] for r in reqs]
    pick = [int(np.argmax(grid))]
    for kind in range(3):
        small = [i for i, r in enumerate(reqs) if r["storage"] == kind and grid[i] <= 5_000_000]
        small.sort(key=lambda i: (-reqs[i]["steps"], i))
        more = [i for i, r in enumerate(reqs) if r["storage"] == kind and i not in small]
        more.sort(key=lambda i: (grid[i] * reqs[i]["steps"], i))
        take = [i for i in small + more if i not in pick][:5]
        pick += take
    items = []
    for i in pick:
        r = reqs[i]
        items.append((f"r{i}", synth.shot_from_shape(r["nx"], r["ny"], r["nz"], r["steps"], r["seed"]),
                      {"index": i, "storage": ["f32", "bf16", "f16"][r["storage"]]}))
    sampled_f64("serve", items, "float64 oracle results of a subset of the serving requests "
                "(synth.serve_requests, 5 % perturbed layered models)", reuse=args.reuse)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="c2", choices=["c2", "c3", "batch", "serve"])
    ap.add_argument("--reuse", action="store_true",
                    help="batch/serve: keep stored entries whose request is unchanged")
    ap.add_argument("--storage", default="f32", choices=["f32", "bf16", "f16"])
    ap.add_argument("--segment", type=int, default=100, help="steps between checkpoints")
    ap.add_argument("--steps", type=int, default=None, help="override the config's steps")
    ap.add_argument("--scratch", default=None, help="directory for the c3 float64 field")
    args = ap.parse_args()
    {"c2": config_c2, "c3": config_c3, "batch": config_batch, "serve": config_serve}[args.config](args)


if __name__ == "__main__":
    main()
