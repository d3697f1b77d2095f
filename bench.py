#!/usr/bin/env python3
"""Benchmark: time stepping of the 3-D acoustic wave equation on one MI355X.

Workload (default): 512^3 total grid with a 20-cell damping layer, seeded
8-layer velocity model with a 5 % smoothed perturbation, 15 Hz Ricker source
5 cells below the layer, a line of 512 receivers, float32 fields.  One bench
"step" is one full time step of the hot path: the sweep over every point
(inner region and damping layer), the source add, the receiver sample and the
rotation of the time levels.

Prints one JSON line: throughput in Gpoints/s (grid points x steps / time),
the sweep kernel against the HBM roofline (algorithmic bytes / measured
kernel time), and the float64 CPU oracle timed on a bounded sample of the
same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0   # MI355X HBM3E nameplate
GOLD = os.path.join(ROOT, "tests", "golden")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# sweep kernel of each variant: name, profile prefix, sources it is built from
KERNELS = {0: ("k_sweep_direct", "direct", ("wave_kernels.hip", "wave_direct.h", "wave_point.h")),
           1: ("k_sweep_stream", "sweep", ("wave_kernels.hip", "wave_point.h")),
           2: ("k_sweep2", "sweep2", ("wave_kernels2.hip", "wave_point.h")),
           3: ("k_sweep_gmem", "gmem", ("wave_shapes.hip", "wave_direct.h", "wave_point.h")),
           4: ("k_sweep_ring", "ring", ("wave_shapes.hip", "wave_direct.h", "wave_point.h")),
           5: ("k_sweep_shift", "shift", ("wave_shapes.hip", "wave_direct.h", "wave_point.h")),
           6: ("k_sweep_pair", "pair", ("wave_kernels_pair.hip", "wave_point.h")),
           7: ("k_sweep_stream", "semi", ("wave_kernels.hip", "wave_point.h")),
           8: ("k_sweep_persist", "persist", ("wave_kernels.hip", "wave_point.h")),
           9: ("k_sweep_stream", "shuffle", ("wave_kernels.hip", "wave_point.h"))}


def kernel_source_sha(variant: int = 1) -> str:
    h = hashlib.sha256()
    for f in KERNELS[variant][2]:
        h.update(open(os.path.join(ROOT, "paper_2009_04619_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def describe(cfg) -> str:
    v, ry, nw, zc = cfg
    if v == 2:
        return f"two-step (3.5-D) zchunk={zc}"
    if v == 0:
        return "direct"
    if v == 3:
        return f"3-D tile {ry}x{nw}x{zc}, all operands from memory"
    if v == 6:
        return f"stream, two points per lane, 128x{nw} zchunk={zc}"
    if v == 7:
        return f"stream, z semi-stencil, 64x{nw} zchunk={zc}"
    if v == 8:
        return f"stream, persistent (one workgroup per CU), 64x{nw} zchunk={zc}"
    if v == 9:
        return f"stream, x neighbours by wavefront shuffles, 64x{nw} zchunk={zc}"
    if v in (4, 5):
        return f"2.5-D {'ring of 9 LDS planes' if v == 4 else 'LDS plane + shifted registers'} " \
               f"64x{nw} zchunk={zc}"
    return f"stream rows_per_wave={ry} waves_per_group={nw} zchunk={zc}"


def measured_traffic(workload: str, launches_bytes: float, variant: int = 1, tile=None):
    """HBM bytes per sweep launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source; else None.  `tile`
    (rows_per_wave, waves_per_group) selects the kernel instance the run used
    when the summary lists it."""
    name, prefix, _ = KERNELS[variant]
    p = os.path.join(ROOT, "profiles", f"traffic_{prefix}_{workload}.json")
    if not os.path.exists(p):
        return None
    try:
        t = json.load(open(p))
    except Exception:
        return None
    if t.get("kernel_sha") != kernel_source_sha(variant):
        return None
    inst = t.get("instances", {}).get(f"{tile[0]},{tile[1]}") if tile else None
    if inst:
        return float(inst["hbm_bytes_per_launch"])
    return float(t["hbm_bytes_per_launch"])


# ---- error against float64 ------------------------------------------------------
# The float64 results come from goldens written by tests/golden/make_fp64_gap.py
# (the CPU oracle's float64 mode on the same seeded shots); the GPU results are
# compared on the samples stored there: an xz plane through the source (every
# few points) and the traces of every few receivers.

def load_golden(name):
    base = os.path.join(GOLD, f"{name}_fp64_gap")
    if not (os.path.exists(base + ".json") and os.path.exists(base + ".npz")):
        return None
    import numpy as np
    return json.load(open(base + ".json")), np.load(base + ".npz")


def rel_l2(a, b) -> float:
    import numpy as np
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float("nan")


def c2_accuracy(W, shot, storage, kernel, sr=False):
    """The benchmark shot run for the golden's step count (1000, the paper's
    protocol) on the GPU with the given launch, against the float64 oracle on
    the golden's samples, and whether it equals the oracle's own
    float32-arithmetic mode there bit for bit (not with stochastically
    rounded bf16 storage, `sr`, whose golden holds the float64 samples only)."""
    import dataclasses
    import numpy as np
    import synth
    base = {(512, 20): "c2", (1024, 32): "c3"}.get((shot.nx, shot.w))
    if base is None:
        return None
    g = load_golden(base if storage == "f32" or sr else f"{base}_{storage}")
    if g is None or [shot.nx, shot.ny, shot.nz] != g[0]["grid"] or shot.w != g[0]["layer"] \
            or shot.seed != g[0]["seed"]:
        return None
    meta, arr = g
    steps = meta["steps"]
    s = dataclasses.replace(shot, steps=steps, wavelet=synth.ricker(steps, shot.dt)[None, :])
    sh = W.shot_from_synth(s, storage=storage, max_steps=steps, stochastic_round=sr)
    sh.set_kernel(*kernel)
    sh.step(steps)
    u = sh.read(W.WAVE_FIELD_U)
    tr = sh.traces()
    sh.close()
    sm = meta["sample"]
    plane = np.ascontiguousarray(u[::sm["plane_stride"], sm["plane_j"], ::sm["plane_stride"]])
    trs = np.ascontiguousarray(tr[:, ::sm["receiver_stride"]])
    same = None if sr else bool(np.array_equal(plane, arr["plane_f32"]) and
                                np.array_equal(trs.astype(np.float32), arr["traces_f32"]))
    out = {"steps": steps,
           "rel_l2_vs_fp64": {"field_sample": round(rel_l2(plane, arr["plane_f64"]), 10),
                              "traces_sample": round(rel_l2(trs, arr["traces_f64"]), 10)},
           "equals_oracle_same_arithmetic_on_sample": same}
    if not sr:
        out.update({
           "oracle_whole_field_rel_l2_vs_fp64": meta["field_rel_l2"],
           "oracle_traces_rel_l2_vs_fp64": meta["traces_rel_l2"]})
    out.update({
           "sample": f"xz plane j={sm['plane_j']} every {sm['plane_stride']}th point, "
                     f"every {sm['receiver_stride']}th receiver trace"})
    log(f"[bench] {storage} {shot.nx}^3 x {steps} steps vs fp64: {out['rel_l2_vs_fp64']} "
        f"(equals oracle: {same})")
    return out


def sampled_error(golden_entry, arr, u, traces):
    """rel L2 of a GPU result against a float64 golden entry's samples: the
    final field on a plane through the source, the traces of every few
    receivers over the whole run, and how far the final field has decayed
    (its sampled maximum over the traces' peak; a long run ends on the small
    remainder the layer has not absorbed yet, whose relative error is large
    for 16-bit storage although its absolute error is not)."""
    import numpy as np
    key = golden_entry["key"]
    ps = 8
    plane = u[::ps, golden_entry["plane_j"], ::ps]
    g_plane, g_tr = arr[f"{key}_plane"], arr[f"{key}_traces"]
    return {"field": round(rel_l2(plane, g_plane), 9),
            "traces": round(rel_l2(traces[:, ::8], g_tr), 9),
            "final_over_peak": float(f"{np.abs(g_plane).max() / max(np.abs(g_tr).max(), 1e-30):.3g}")}


def error_summary(errs):
    """Largest field and trace errors over a set of sampled_error results."""
    return {"max_field_rel_l2": max(e["field"] for e in errs),
            "max_traces_rel_l2": max(e["traces"] for e in errs),
            "min_final_over_peak": min(e["final_over_peak"] for e in errs)}


def build_shots(specs, threads=8):
    """synth shots for (nx, ny, nz, steps, seed) on a thread pool (the
    velocity models are the bulk of the host time)."""
    import synth
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(threads) as ex:
        return list(ex.map(lambda t: synth.shot_from_shape(*t), specs))


def copy_bandwidth(W, torch, nbytes=2 << 30, reps=10):
    """Plain streams (the measured-bandwidth references): copy (1 read, 1
    write), read only, and three reads with one write (the access mix of an
    inner point of the sweep); GB/s moved."""
    a = torch.zeros(nbytes, dtype=torch.uint8, device="cuda:0")
    b, c, d = torch.zeros_like(a), torch.zeros_like(a), torch.zeros_like(a)
    s = torch.cuda.current_stream()
    P = (a.data_ptr(), b.data_ptr(), c.data_ptr(), d.data_ptr())
    legs = {"copy": (lambda: W.wave_stream_copy(P[3], P[0], nbytes, s.cuda_stream), 2.0),
            "read": (lambda: W.wave_stream_mix(0, P[3], P[0], 0, 0, nbytes, s.cuda_stream), 1.0),
            "read3_write1": (lambda: W.wave_stream_mix(1, P[3], P[0], P[1], P[2], nbytes,
                                                       s.cuda_stream), 4.0)}
    out = {}
    for name, (fn, moved) in legs.items():
        for _ in range(2):
            assert fn() == 0
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            fn()
        e1.record(s)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = round(moved * nbytes / (ms / 1e3) / 1e9, 1)
    del a, b, c, d
    torch.cuda.empty_cache()
    return out


def plain_rate(W, torch, n, w, storage, steps, seed=1002, accuracy=True, sr=False):
    """One shot, plain launches, given storage (`sr`: bf16 rounded
    stochastically): Gpoints/s, the sweep kernel's algorithmic GB/s, and
    (with a golden for the grid) the error of a 1000-step run against
    float64."""
    import synth
    shot = synth.config_c2(steps=steps + 20 + 256, n=n, w=w, seed=seed)
    sh = W.shot_from_synth(shot, storage=storage, max_steps=steps + 20 + 50 + 256,
                           two_step=not sr, stochastic_round=sr)
    cfg = sh.tune(2)
    sh.step(max(0, 20 - sh.step_count))
    sh.sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(sh.stream)
    sh.step(steps)
    e1.record(sh.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    sh.set_timing(True)
    sh.step(50)
    kms, k = sh.read_timing()
    gbs = sh.sweep_bytes() / (kms / k / 1e3) / 1e9
    sh.close()
    log(f"[bench] {storage} {n}^3: {shot.points * steps / ms / 1e6:.1f} Gpt/s, sweep {gbs:.0f} GB/s")
    out = {"value": round(shot.points * steps / ms / 1e6, 3), "unit": "Gpoints/s",
           "storage": storage + (" stochastic rounding" if sr else ""), "steps": steps,
           "kernel": describe(cfg),
           "sweep_ms": round(kms / k, 5),
           "sweep_gbps_algorithmic": round(gbs, 1), "frac": round(gbs / PEAK_HBM_GBS, 4)}
    if accuracy:
        out["accuracy"] = c2_accuracy(W, shot, storage, cfg, sr=sr)
    return out


# the paper's code shapes (Sec. IV, Table II) on this GPU: wave_set_kernel
# arguments and a label
SHAPES = [((1, 1, 16, 0), "2.5-D stream, LDS plane + register ring, prefetch (default)"),
          ((0, 0, 0, 0), "3-D 64x4x1, all operands from memory (direct)"),
          ((3, 8, 8, 8), "gmem 8x8x8"), ((3, 4, 4, 4), "gmem 4x4x4"),
          ((3, 16, 16, 4), "gmem 16x16x4"), ((3, 32, 32, 1), "gmem 32x32x1"),
          ((3, 64, 4, 4), "gmem 64x4x4"),
          ((4, 1, 8, 0), "st_smem 64x8 (ring of 9 LDS planes)"),
          ((4, 1, 16, 0), "st_smem 64x16 (ring of 9 LDS planes)"),
          ((5, 1, 8, 0), "st_reg_shft 64x8 (LDS plane + 9 shifted registers)"),
          ((5, 1, 16, 0), "st_reg_shft 64x16 (LDS plane + 9 shifted registers)")]


def shapes_rate(W, torch, n, w, steps=20):
    """Sweep-kernel time of each code shape on one shot (kernel time from HIP
    events on the shot's stream; identical results by construction)."""
    import synth
    shot = synth.config_c2(steps=len(SHAPES) * (steps + 2) + 8, n=n, w=w)
    sh = W.shot_from_synth(shot, max_steps=len(SHAPES) * (steps + 2) + 8)
    out = []
    for cfg, label in SHAPES:
        sh.set_kernel(*cfg)
        sh.step(2)
        sh.set_timing(True)
        sh.step(steps)
        kms, k = sh.read_timing()
        sh.set_timing(False)
        avg = kms / max(k, 1)
        gbs = sh.sweep_bytes() / (avg / 1e3) / 1e9
        log(f"[bench] shape {label}: {avg:.3f} ms, {shot.points / avg / 1e6:.1f} Gpt/s")
        out.append({"shape": label, "args": list(cfg), "ms": round(avg, 4),
                    "gpoints_per_s": round(shot.points / avg / 1e6, 2),
                    "frac": round(gbs / PEAK_HBM_GBS, 4)})
    sh.close()
    return out


def batched_rate(W, torch, count):
    """`count` seeded shots (each axis uniform in {128, 144, .., 384}, 200-1000
    steps, 20-cell layer, 5 % perturbed layered models) advanced together with
    captured step blocks and a tuned tile, against the same shots run one at
    a time; the error against float64 of the shots the batch golden holds."""
    import synth
    shapes = synth.batch_shapes(count=count)
    log(f"[bench] batched: building {count} shots")
    shots = build_shots([(nx, ny, nz, st, seed) for (nx, ny, nz, st, seed) in shapes])
    work = sum(s.points * s.steps for s in shots)
    gold = load_golden("batch")
    check = [e for e in gold[0]["members"] if e["index"] < count] if gold else []
    out = {"shots": count, "points_x_steps": work}
    for storage in ("f32", "bf16", "f16"):
        members = [W.shot_from_synth(s, storage=storage) for s in shots]
        alg = sum(m.sweep_bytes() * s.steps for m, s in zip(members, shots))
        b = W.Batch(storage=storage, max_shots=count)
        for s, m in zip(shots, members):
            b.add(m, s.steps)
        b.set_graph(10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cfg = b.tune(2)
        b.run(max(s.steps for s in shots))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        b.close()
        errs = {}
        for e in check:
            m = members[e["index"]]
            errs[e["key"]] = sampled_error(e, gold[1], m.read(W.WAVE_FIELD_U), m.traces())
        for m in members:
            m.close()
        out[f"batched_{storage}"] = {"value": round(work / dt / 1e9, 3), "unit": "Gpoints/s",
                                     "seconds": round(dt, 3), "tile": list(cfg),
                                     "sweep_bytes_algorithmic": alg,
                                     "gbps_algorithmic_incl_tuning": round(alg / dt / 1e9, 1)}
        if errs:
            out[f"batched_{storage}"]["error_vs_fp64"] = error_summary(list(errs.values()))
            out[f"batched_{storage}"]["error_vs_fp64_per_shot"] = errs
        log(f"[bench] batched {storage}: {work / dt / 1e9:.1f} Gpt/s ({dt:.2f} s), errors {errs}")
    # the same shots one at a time, plain float32 launches (set-up untimed,
    # like the batched leg's)
    solo = 0.0
    for s in shots:
        m = W.shot_from_synth(s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.step(s.steps)
        m.sync()
        solo += time.perf_counter() - t0
        m.close()
    solo = max(solo, 1e-9)
    out["one_at_a_time_f32"] = {"value": round(work / solo / 1e9, 3), "unit": "Gpoints/s",
                                "seconds": round(solo, 3)}
    out["batched_f32_over_one_at_a_time"] = round(out["batched_f32"]["value"] /
                                                  out["one_at_a_time_f32"]["value"], 4)
    if gold:
        out["error_sample"] = (f"shots {[e['index'] for e in check]}: rel L2 vs the float64 "
                               "oracle of the final field on an xz plane through the source "
                               "(every 8th point) and of every 8th receiver's trace")
    log(f"[bench] one at a time f32: {work / solo / 1e9:.1f} Gpt/s ({solo:.2f} s)")
    return out


def serve_run(W, torch, count, rate=20.0, check_errors=True):
    """Seeded Poisson stream (20 requests/s and 256 requests by default) of
    shots 96-512 per axis, 200-2000 steps, storage uniform over
    f32/bf16/f16, 5 % perturbed layered models, 240 GB budget.  Offered and
    served load are both reported: above capacity, latency includes
    queueing.  The requests the serve golden holds keep their wavefield and
    are compared with float64 (max rel L2 per storage type)."""
    import synth
    from paper_2009_04619_amd.serve import GpuExecutor, Request, Server, summarize
    specs = synth.serve_requests(count=count, rate=rate)
    log(f"[bench] serve: building {count} requests")
    shots = build_shots([(r["nx"], r["ny"], r["nz"], r["steps"], r["seed"]) for r in specs])
    reqs = [Request(rid=q, arrival=r["t"], shot=shot, storage=["f32", "bf16", "f16"][r["storage"]])
            for q, (r, shot) in enumerate(zip(specs, shots))]
    offered = sum(r.points * r.shot.steps for r in reqs) / max(reqs[-1].arrival, 1e-9)
    gold = load_golden("serve") if check_errors else None
    check = {e["index"]: e for e in gold[0]["members"] if e["index"] < count} if gold else {}
    ex = GpuExecutor(graph_steps=10)
    srv = Server(ex, budget_bytes=240 * 10 ** 9, block_steps=50)
    t0 = time.perf_counter()
    done = srv.run(reqs)
    wall = time.perf_counter() - t0
    ex.close()
    out = summarize(done, wall)
    out["offered_gpoints_per_s"] = round(offered / 1e9, 3)
    out["arrival_rate_per_s"] = rate
    if check:
        # errors from a second, untimed pass over the golden's requests (all
        # arriving at once), so that reading whole fields back does not slow
        # the timed loop; a served result does not depend on the batch it
        # ran in (bit for bit, tested), so these are the timed pass's values
        again = [Request(rid=q, arrival=0.0, shot=reqs[q].shot, storage=reqs[q].storage)
                 for q in sorted(check)]
        ex2 = GpuExecutor(graph_steps=10)
        done2 = Server(ex2, budget_bytes=240 * 10 ** 9, block_steps=50).run(
            again, keep_fields=set(check))
        ex2.close()
        errs = {}
        for r in done2:
            if r.error is None:
                errs.setdefault(r.storage, []).append(
                    sampled_error(check[r.rid], gold[1], r.field, r.traces))
        out["error_vs_fp64"] = {k: dict(error_summary(v), requests=len(v)) for k, v in errs.items()}
    log(f"[bench] serve: {out}")
    return out


def cpu_baseline(shot, budget_s: float):
    """The float64 oracle as it stands on the host cores, on a bounded number
    of steps of the same grid (calibrated to about `budget_s` seconds)."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    s = shot
    t0 = time.perf_counter()
    st = oracle.run_shot(s, steps=1, precision="f64")
    t1 = time.perf_counter()
    # one step includes set-up (vp, damping profile); time the rest alone
    state = dict(u=st["u"], u_prev=st["u_prev"], phi=st["phi"])
    del st
    n = 2
    t2 = time.perf_counter()
    oracle.run_shot(s, steps=n, precision="f64", state=state, n0=1)
    per = (time.perf_counter() - t2) / n
    steps = max(1, min(40, int(budget_s / max(per, 1e-3))))
    t3 = time.perf_counter()
    oracle.run_shot(s, steps=steps, precision="f64", state=state, n0=1)
    dt = time.perf_counter() - t3
    gpts = s.points * steps / dt / 1e9
    return {"value": round(gpts, 5), "unit": "Gpoints/s", "cores": threads, "kind": "oracle",
            "sample": f"float64 oracle, same {s.nx}x{s.ny}x{s.nz} w{s.w} grid and model, "
                      f"{steps} steps after 1 set-up step ({t1 - t0:.1f} s incl. set-up), "
                      f"{threads} OpenMP threads"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--n", type=int, default=512, help="grid extent per axis")
    ap.add_argument("--w", type=int, default=20, help="damping layer width")
    ap.add_argument("--storage", default="f32", choices=["f32", "bf16", "f16"])
    ap.add_argument("--kernel", default="tune",
                    help="'tune' (autotune during warmup) or variant,rows_per_wave,waves_per_group,zchunk")
    ap.add_argument("--roofline-steps", type=int, default=200)
    ap.add_argument("--single-step", action="store_true",
                    help="do not offer the two-step kernel to the tuner")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-copy", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the bf16, batched and serving measurements")
    ap.add_argument("--batch-shots", type=int, default=64)
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--extras", default="bf16,bf16_sr,batched,serve,serve_low,shapes,large",
                    help="comma-separated measurements beside the headline: bf16, batched, "
                         "serve, serve_low, shapes, large (1024^3)")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the 1000-step runs compared with the float64 goldens")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the library has no "
              "multi-GPU path (a z-slab decomposition is described, not implemented)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    from paper_2009_04619_amd import wave as W

    log(f"[bench] building workload {args.n}^3 w{args.w}")
    total = args.warmup + args.steps
    shot = synth.config_c2(steps=total + 256, n=args.n, w=args.w)
    torch.cuda.synchronize()
    s0 = time.perf_counter()
    sh = W.shot_from_synth(shot, storage=args.storage,
                           max_steps=total + 256 + args.roofline_steps,
                           two_step=not args.single_step)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - s0          # host-to-device set-up (vel over PCIe)
    stream = sh.stream
    log(f"[bench] warmup {args.warmup} steps")
    if args.kernel == "tune":
        # the tuner's trials are ordinary steps of this run (every tile shape
        # computes identical results); they count toward the warmup
        cfg = sh.tune(max(1, min(4, args.warmup // 16)))
        kernel = describe(cfg) + " (tuned)"
        log(f"[bench] tuned: {kernel} after {sh.step_count} steps")
    else:
        k = [int(v) for v in args.kernel.split(",")]
        sh.set_kernel(*k)
        cfg = tuple(k)
        kernel = describe(cfg)
    sh.step(max(0, args.warmup - sh.step_count))
    sh.sync()

    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    e0.record(stream)
    sh.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = e0.elapsed_time(e1)
    log(f"[bench] timed {args.steps} steps: {ms:.2f} ms (wall {wall * 1e3:.2f} ms)")
    pts = shot.points
    gpts = pts * args.steps / (ms / 1e3) / 1e9

    # roofline of the sweep kernel: its own launches bracketed by HIP events
    # on the stream it runs on
    sh.set_timing(True)
    sh.step(args.roofline_steps)
    kms, launches = sh.read_timing()
    sh.set_timing(False)
    avg_ms = kms / max(launches, 1)
    alg_bytes = sh.sweep_bytes()
    achieved = alg_bytes / (avg_ms / 1e3) / 1e9
    workload = f"{args.n}cube_w{args.w}_{args.storage}"
    variant = cfg[0] if cfg[0] in KERNELS else 1
    traffic = measured_traffic(workload, alg_bytes, variant,
                               tile=(cfg[1], cfg[2]) if variant in (1, 6, 8) else None)
    log(f"[bench] sweep kernel avg {avg_ms:.4f} ms over {launches} launches, "
        f"{alg_bytes / pts:.2f} B/pt algorithmic -> {achieved:.0f} GB/s")
    r0 = time.perf_counter()
    tr = sh.traces()
    readout_s = time.perf_counter() - r0        # receiver traces back to the host
    assert np.isfinite(tr).all()
    log(f"[bench] set-up {setup_s * 1e3:.1f} ms, trace read-out {readout_s * 1e3:.1f} ms")
    sh.close()
    del sh
    # the same launch run for the paper's 1000 steps, against float64
    accuracy = None if args.no_accuracy else c2_accuracy(W, shot, args.storage, cfg)

    extras = None
    legs = [] if args.no_extras else args.extras.split(",")
    if legs:
        extras = {}
        if "bf16" in legs:
            extras["bf16_plain"] = plain_rate(W, torch, args.n, args.w, "bf16", 200)
        if "bf16_sr" in legs:
            extras["bf16_sr_plain"] = plain_rate(W, torch, args.n, args.w, "bf16", 200, sr=True)
        if "batched" in legs:
            extras["batched"] = batched_rate(W, torch, args.batch_shots)
        if "serve" in legs:
            extras["serve"] = serve_run(W, torch, args.serve_requests)
        if "serve_low" in legs:
            # the same stream at a quarter of the arrival rate, below
            # capacity: latency is then service time, not backlog
            extras["serve_below_capacity"] = serve_run(W, torch, args.serve_requests // 4,
                                                       rate=5.0, check_errors=False)
        if "shapes" in legs:
            extras["code_shapes"] = shapes_rate(W, torch, args.n, args.w)
        if "large" in legs and args.n == 512 and args.w == 20:
            # the large-domain configuration: 1024^3 with a 32-cell layer
            extras["large_1024cube_w32_f32"] = plain_rate(W, torch, 1024, 32, "f32", 100,
                                                          seed=1003)

    streams = None if args.no_copy else copy_bandwidth(W, torch)
    copy_gbs = None if streams is None else streams["copy"]
    if streams:
        log(f"[bench] plain streams GB/s: {streams}")

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (float64 oracle)")
        cpu = cpu_baseline(synth.config_c2(steps=64, n=args.n, w=args.w), args.cpu_budget)

    line = {
        "metric": "Gpoints/s & % HBM roofline (plain vs batched/BF16); shots/s + p50/p99 latency",
        "value": round(gpts, 3),
        "unit": "Gpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage == "f32" else f"f32 math, {args.storage} storage",
        "data": "synthetic (seeded layered velocity model, Ricker source)",
        "config": {"workload": f"acoustic 25-pt leapfrog, {args.n}^3 grid incl. {args.w}-cell "
                               f"damping layer, 1 source, {args.n} receivers",
                   "grid": [args.n, args.n, args.n], "layer": args.w,
                   "storage": args.storage, "kernel": kernel},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": None if traffic is None else round(traffic / 1e9, 4),
                     "traffic_unit": "GB per launch (FETCH_SIZE + WRITE_SIZE, calibrated)",
                     "kernel": KERNELS[variant][0], "algorithmic_bytes_per_launch": alg_bytes,
                     "avg_kernel_ms": round(avg_ms, 5)},
        "accuracy": accuracy,
        "copy_gbps": copy_gbs,
        "empirical_roofline": None if streams is None else {
            "unit": "GB/s", **streams,
            "sweep_traffic_gbps": None if traffic is None else round(traffic / (avg_ms / 1e3) / 1e9, 1),
            "note": "plain streams on this GPU (copy; read only; three reads and one write, the "
                    "mix of an inner point); sweep_traffic_gbps = the sweep's measured HBM "
                    "bytes (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated) per launch over its "
                    "average launch time"},
        "host_io": {"setup_s": round(setup_s, 4), "trace_readout_s": round(readout_s, 4),
                    "value_incl_host_io": round(pts * args.steps / (ms / 1e3 + setup_s + readout_s) / 1e9, 3),
                    "note": "value with the set-up (velocity upload, vp) and the trace read-out "
                            "added to the timed steps"},
        "extras": extras,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
