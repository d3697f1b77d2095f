"""The paper's other code shapes (3-D tiles reading every operand from memory,
the 2.5-D ring of 9 staged planes, the 2.5-D staged plane with a shifted
register queue) against the float32 oracle: every point is evaluated with the
same operations in the same order, so fields, phi and traces are equal bit
for bit on ragged grids, with 16-bit storage, damping off, an explicit eta
array, and chunkings that cut z into short pieces."""
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


def run(W, shot, steps, kernel, storage="f32", damping=True, eta=None):
    sh = W.shot_from_synth(shot, storage=storage, damping=damping, max_steps=max(steps, 1),
                           eta=eta)
    sh.set_kernel(*kernel)
    sh.step(steps)
    out = dict(u=sh.read(W.WAVE_FIELD_U), u_prev=sh.read(W.WAVE_FIELD_UPREV),
               phi=sh.read(W.WAVE_FIELD_PHI), traces=sh.traces())
    sh.close()
    return out


def assert_same(a, b, what):
    for key in ("u", "u_prev", "phi", "traces"):
        x, y = a[key], b[key]
        assert x.shape == y.shape, (what, key)
        if not np.array_equal(x, y):
            bad = np.argwhere(x != y)
            i = tuple(bad[0])
            raise AssertionError(f"{what}: {key} differs at {len(bad)} points, first {i}: "
                                 f"{x[i]!r} vs {y[i]!r}")


def ref(shot, steps, storage="f32", damping=True, eta=None):
    r = oracle.run_shot(shot, steps=steps, precision="f32", storage=storage, damping=damping,
                        **({} if eta is None else {"eta": eta}))
    if not damping:
        r["phi"] = np.zeros_like(r["u"])
    return r


SHAPES = [(3, 8, 8, 8), (3, 4, 4, 4), (3, 16, 16, 4), (3, 32, 32, 1), (3, 64, 4, 1),
          (3, 64, 4, 4), (4, 1, 8, 0), (4, 1, 16, 0), (4, 1, 16, 5), (5, 1, 8, 0),
          (5, 1, 16, 0), (5, 1, 8, 7)]

GRIDS = [  # nx, ny, nz, w, steps, storage, damping
    (70, 45, 37, 5, 14, "f32", True),
    (130, 19, 22, 3, 9, "bf16", True),
    (65, 33, 17, 4, 8, "f16", True),
    (45, 70, 30, 6, 10, "f32", False),
    (6, 6, 7, 3, 6, "f32", True),       # smaller than every tile and chunk, all layer
    (1, 1, 1, 0, 4, "bf16", True),      # one point, no layer
]


@pytest.mark.parametrize("grid", GRIDS, ids=lambda g: f"{g[0]}x{g[1]}x{g[2]}_w{g[3]}_{g[5]}_"
                         f"{'damp' if g[6] else 'nodamp'}")
def test_shapes_equal_oracle(W, grid):
    nx, ny, nz, w, steps, storage, damping = grid
    shot = synth.config_small_layered(nx, ny, nz, w, steps, seed=nx * 7 + ny, nsrc=2)
    expect = ref(shot, steps, storage, damping)
    for k in SHAPES:
        say(f"case shape {k} grid {grid}")
        assert_same(run(W, shot, steps, k, storage, damping), expect, f"shape {k} {grid}")


def test_shapes_with_eta_array(W):
    nx, ny, nz, w, steps = 70, 45, 37, 5, 12
    shot = synth.config_small_layered(nx, ny, nz, w, steps, seed=78, nsrc=2)
    _, e32 = oracle.eta_default(nx, ny, nz, w, shot.dx, shot.dy, shot.dz, shot.dt,
                                float(shot.vel.max()))
    rng = np.random.default_rng(6)
    eta = (e32 * (1.0 + 0.5 * rng.random(e32.shape))).astype(np.float32)
    expect = ref(shot, steps, eta=eta)
    for k in [(3, 8, 8, 8), (3, 64, 4, 1), (4, 1, 16, 0), (5, 1, 8, 3)]:
        say(f"case shape {k} eta array")
        assert_same(run(W, shot, steps, k, eta=eta), expect, f"shape {k} eta array")


def test_shape_arguments_are_checked(W):
    shot = synth.config_small_layered(20, 20, 20, 3, 4, seed=3)
    sh = W.shot_from_synth(shot)
    for bad in [(3, 8, 8, 4), (3, 2, 2, 2), (4, 2, 8, 0), (4, 1, 12, 0), (5, 1, 16, -1)]:
        assert W.wave_set_kernel(sh.ctx, *bad) == W.WAVE_EINVAL, bad
    sh.close()
