"""Tiles that hold an x wall of the damping layer lay their lanes out as half
rows (32 columns x 2 rows per wavefront in the one-point sweep, 64 columns
x 2 rows in the two-points-per-lane sweep).  Against the float32 oracle, bit
for bit: walls wider than half a tile (the wall then reaches into the other
half's wavefronts), both walls in one tile, a right wall that starts in one
tile and ends in the next, walls of three cells, every tile shape of both
kernels, and an eta array (the one-point sweep's array mode)."""
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


def random_state(shot, storage, seed):
    """u, u_prev random and representable in the storage type; phi random on
    the layer points, 0 elsewhere: every wall point carries data from the
    first step on."""
    rng = np.random.default_rng(seed)
    shape = (shot.nz, shot.ny, shot.nx)
    w = shot.w
    k = np.arange(shot.nz)[:, None, None]
    j = np.arange(shot.ny)[None, :, None]
    i = np.arange(shot.nx)[None, None, :]
    lay = ((i < w) | (i >= shot.nx - w) | (j < w) | (j >= shot.ny - w) | (k < w)
           | (k >= shot.nz - w))

    def store(a):
        a = a.astype(np.float32)
        if storage == "f16":
            return a.astype(np.float16).astype(np.float32)
        if storage == "bf16":
            b = a.view(np.uint32)
            b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
            return b.view(np.float32)
        return a
    return {"u": store(rng.standard_normal(shape, dtype=np.float32) * np.float32(1e-2)),
            "u_prev": store(rng.standard_normal(shape, dtype=np.float32) * np.float32(1e-2)),
            "phi": np.where(lay, rng.standard_normal(shape, dtype=np.float32) * np.float32(1e-3),
                            np.float32(0)).astype(np.float32)}


def run(W, shot, steps, kernel, storage="f32", eta=None, state=None):
    sh = W.shot_from_synth(shot, storage=storage, max_steps=max(steps, 1), eta=eta)
    if state is not None:
        sh.write(W.WAVE_FIELD_U, state["u"])
        sh.write(W.WAVE_FIELD_UPREV, state["u_prev"])
        sh.write(W.WAVE_FIELD_PHI, state["phi"])
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


STREAM_EA = [(1, 1, 16, 0), (1, 1, 8, 0), (1, 2, 8, 0), (1, 2, 4, 0), (1, 1, 8, 3)]
# 64 x 32 tiles and the persistent launch take the default profile's tables only
STREAM = STREAM_EA + [(1, 2, 16, 0), (8, 1, 16, 0), (8, 1, 8, 0), (9, 1, 16, 0), (9, 1, 8, 0)]
PAIR = [(6, 1, 16, 0), (6, 1, 8, 0), (6, 1, 8, 5)]

GRIDS = [  # nx, ny, nz, w, steps, storage
    (70, 24, 22, 9, 10, "f32"),       # one-point tile 0 holds both walls
    (150, 90, 80, 37, 8, "f32"),      # wall wider than a 32-column half
    (100, 30, 26, 3, 10, "bf16"),     # three-cell walls (thinner ones amplify a random state)
    (140, 50, 44, 20, 8, "f16"),      # right wall x = 120..139 over two 64-wide tiles
    (200, 140, 140, 66, 4, "f32"),    # wall wider than a 64-column half
]


@pytest.mark.parametrize("grid", GRIDS, ids=lambda g: f"{g[0]}x{g[1]}x{g[2]}_w{g[3]}_{g[5]}")
def test_wall_tiles_equal_oracle(W, grid):
    nx, ny, nz, w, steps, storage = grid
    shot = synth.config_small_layered(nx, ny, nz, w, steps, seed=nx + 5 * w, nsrc=2)
    st = random_state(shot, storage, seed=nx * ny + w)
    expect = oracle.run_shot(shot, steps=steps, precision="f32", storage=storage, state=st)
    for k in STREAM + PAIR:
        say(f"case walls {k} grid {grid}")
        assert_same(run(W, shot, steps, k, storage, state=st), expect, f"walls {k} {grid}")


def test_wall_tiles_with_eta_array(W):
    nx, ny, nz, w, steps = 150, 90, 80, 37, 6
    shot = synth.config_small_layered(nx, ny, nz, w, steps, seed=11, nsrc=1)
    _, e32 = oracle.eta_default(nx, ny, nz, w, shot.dx, shot.dy, shot.dz, shot.dt,
                                float(shot.vel.max()))
    rng = np.random.default_rng(3)
    eta = (e32 * (1.0 + 0.5 * rng.random(e32.shape))).astype(np.float32)
    st = random_state(shot, "f32", seed=4)
    expect = oracle.run_shot(shot, steps=steps, precision="f32", eta=eta, state=st)
    for k in STREAM_EA + [(8, 1, 16, 0), (8, 1, 8, 3), (9, 1, 16, 0), (9, 1, 8, 3)]:
        say(f"case walls {k} eta array")
        assert_same(run(W, shot, steps, k, eta=eta, state=st), expect, f"walls {k} eta array")
