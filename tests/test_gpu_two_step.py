"""Two time steps per launch (WAVE_KERNEL_STREAM2) against the oracle.

The two-step sweep evaluates every point with the same operations as two
single steps, so its fields, phi and traces must equal the float32 oracle bit
for bit: ragged grids, every storage type, damping on and off, chunkings
that cut the z caps into pieces, grids that are all layer, sources on tile
and chunk edges, odd step counts (the last step runs the single-step kernel),
and contexts that move between two-step stepping and a batch.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def W():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU (run with -m 'not gpu' on CPU)")
    from paper_2009_04619_amd import wave
    return wave


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def read_all(W, sh):
    return dict(u=sh.read(W.WAVE_FIELD_U), u_prev=sh.read(W.WAVE_FIELD_UPREV),
                phi=sh.read(W.WAVE_FIELD_PHI), traces=sh.traces())


def assert_same(a, b, what):
    for key in ("u", "u_prev", "phi", "traces"):
        x, y = a[key], b[key]
        assert x.shape == y.shape, (what, key)
        if not np.array_equal(x, y):
            bad = np.argwhere(x != y)
            i = tuple(bad[0])
            raise AssertionError(f"{what}: {key} differs at {len(bad)} points, first {i}: "
                                 f"{x[i]!r} vs {y[i]!r}")


def run_two_step(W, shot, steps, storage, damping, zc2):
    sh = W.shot_from_synth(shot, storage=storage, damping=damping, max_steps=max(steps, 1),
                           two_step=True)
    sh.set_kernel(W.WAVE_KERNEL_STREAM2, 1, 16, zc2)
    sh.step(steps)
    out = read_all(W, sh)
    sh.close()
    return out


def oracle_ref(shot, steps, storage, damping):
    r = oracle.run_shot(shot, steps=steps, precision="f32", storage=storage, damping=damping)
    if not damping:
        r["phi"] = np.zeros_like(r["u"])
    return r


CASES = [  # nx, ny, nz, w, steps, storage, damping, two-step zchunk
    (70, 45, 37, 5, 23, "f32", True, 64),
    (70, 45, 37, 5, 24, "bf16", True, 8),
    (130, 33, 11, 4, 10, "f32", True, 64),      # 2 (w + 4) >= nz: every plane a cap plane
    (65, 17, 130, 3, 12, "f16", True, 16),
    (113, 65, 60, 9, 14, "f32", False, 16),
    (9, 200, 21, 3, 9, "f32", True, 64),
    (64, 64, 64, 16, 30, "f32", True, 0),
    (120, 40, 90, 6, 16, "bf16", True, 32),
    (1, 1, 1, 0, 6, "f32", True, 64),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}_w{c[3]}_{c[5]}_"
                         f"{'damp' if c[6] else 'nodamp'}_zc{c[7]}")
def test_two_step_equals_oracle(W, case):
    nx, ny, nz, w, steps, storage, damping, zc2 = case
    shot = synth.config_small_layered(nx, ny, nz, w, steps, seed=nx + ny + nz, nsrc=2)
    say(f"case two-step {case}")
    got = run_two_step(W, shot, steps, storage, damping, zc2)
    assert_same(got, oracle_ref(shot, steps, storage, damping), f"two-step {case}")


def test_sources_on_tile_and_chunk_edges(W):
    """Sources where the first step's region of several tiles overlaps (x on
    a tile edge, y on a row-band edge, z on a chunk edge): every tile that
    recomputes the point adds the source identically."""
    nx, ny, nz, w, steps = 130, 50, 70, 6, 20
    shot = synth.config_small_layered(nx, ny, nz, w, steps, seed=31, nsrc=1)
    pts = [(56, 16, 32), (55, 15, 31), (59, 20, 33), (112, 48, 10), (60, 3, 64), (3, 33, 6)]
    shot.src = pts
    shot.wavelet = np.stack([synth.ricker(steps, shot.dt, t0=(0.2 + 0.1 * s) / 15.0)
                             for s in range(len(pts))])
    shot.rec = np.array([[i, j, k] for (i, j, k) in pts] + [[0, 0, 0], [129, 49, 69]], np.int32)
    say("case two-step sources on edges")
    ref = oracle_ref(shot, steps, "f32", True)
    for zc2 in (32, 64):
        got = run_two_step(W, shot, steps, "f32", True, zc2)
        assert_same(got, ref, f"two-step sources zc={zc2}")


def test_two_step_and_batch_and_single_steps_mix(W):
    """A two-step context stepped in pairs, then inside a batch (single-step
    kernels on its current buffers), then in pairs again, ends where a
    single-step run ends."""
    shot = synth.config_small_layered(96, 70, 50, 8, 40, seed=77, nsrc=1)
    say("case two-step mixed with batch")
    ref = oracle_ref(shot, 40, "f32", True)
    sh = W.shot_from_synth(shot, max_steps=40, two_step=True)
    sh.set_kernel(W.WAVE_KERNEL_STREAM2, 1, 16, 0)
    sh.step(11)                       # 5 pairs + 1 single step
    b = W.Batch(max_shots=2)
    other = W.shot_from_synth(synth.config_small_layered(40, 40, 40, 4, 20, seed=5))
    b.add(sh, 13)
    b.add(other, 20)
    b.run(20)
    b.remove(sh)
    b.close()
    other.close()
    sh.step(16)
    assert_same(read_all(W, sh), ref, "two-step / batch / two-step")
    sh.close()


def test_two_step_tuner_and_errors(W):
    n = 120                           # room for every candidate's trial steps
    shot = synth.config_small_layered(100, 60, 80, 8, n, seed=9, nsrc=1)
    say("case two-step tuner")
    ref = oracle_ref(shot, n, "f32", True)
    sh = W.shot_from_synth(shot, max_steps=n, two_step=True)
    cfg = sh.tune(2)
    assert len(cfg) == 4 and 1 <= cfg[0] <= 6
    assert sh.step_count < n
    sh.step(n - sh.step_count)
    assert_same(read_all(W, sh), ref, "tuned two-step context")
    sh.close()
    # the variant needs WAVE_TWO_STEP; the flag refuses an eta array
    plain = W.shot_from_synth(shot, max_steps=60)
    assert W.wave_set_kernel(plain.ctx, W.WAVE_KERNEL_STREAM2, 1, 16, 0) == W.WAVE_EINVAL
    plain.close()
    d = W.make_desc(shot.nx, shot.ny, shot.nz, shot.w, shot.dx, shot.dy, shot.dz, shot.dt,
                    eta_array=True, two_step=True, max_steps=10)
    assert W.wave_bytes_required(d) == 0


@pytest.mark.parametrize("count", [20, 40])
def test_many_sources_in_one_tile(W, count):
    """20 sources in one tile (two on the same cell, added in list order) go
    through the kernel's per-tile list; 40 exceed it, and the context then
    takes single steps. Both end where the oracle ends."""
    nx, ny, nz, w, steps = 100, 40, 30, 4, 12
    shot = synth.config_small_layered(nx, ny, nz, w, steps, seed=61, nsrc=1)
    rng = np.random.default_rng(count)
    pts = [(int(rng.integers(8, 60)), int(rng.integers(4, 20)), int(rng.integers(2, 28)))
           for _ in range(count - 1)]
    pts.append(pts[3])
    shot.src = pts
    shot.wavelet = np.stack([synth.ricker(steps, shot.dt, t0=(0.1 + 0.02 * s) / 15.0)
                             for s in range(count)])
    shot.rec = np.array([list(p) for p in pts[:6]], np.int32)
    say(f"case two-step {count} sources in one tile")
    got = run_two_step(W, shot, steps, "f32", True, 16)
    assert_same(got, oracle_ref(shot, steps, "f32", True), f"two-step {count} sources")
