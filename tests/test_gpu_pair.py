"""The streaming sweep with two points per lane (WAVE_KERNEL_PAIR) against the
float32 oracle, bit for bit: odd widths whose last 128-wide tile reaches past
the padded row, every storage type, damping on and off, odd layer widths,
chunkings that cut z into short pieces, grids smaller than a tile; and the
variant's refusal of an eta array."""
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


def run(W, shot, steps, kernel, storage="f32", damping=True):
    sh = W.shot_from_synth(shot, storage=storage, damping=damping, max_steps=max(steps, 1))
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


GRIDS = [  # nx, ny, nz, w, steps, storage, damping
    (70, 45, 37, 5, 14, "f32", True),
    (129, 33, 20, 7, 10, "bf16", True),      # last tile past the padded row
    (257, 19, 13, 3, 8, "f16", True),
    (257, 40, 22, 9, 9, "f32", True),
    (130, 70, 30, 6, 10, "f32", False),
    (200, 48, 44, 20, 8, "bf16", True),      # layer wider than half a tile row
    (6, 6, 7, 3, 6, "f32", True),        # all layer, smaller than every tile
    (1, 1, 1, 0, 4, "f16", True),
]
KERNELS = [(6, 1, 16, 0), (6, 1, 8, 0), (6, 1, 16, 5), (6, 1, 8, 3)]


@pytest.mark.parametrize("grid", GRIDS, ids=lambda g: f"{g[0]}x{g[1]}x{g[2]}_w{g[3]}_{g[5]}_"
                         f"{'damp' if g[6] else 'nodamp'}")
def test_pair_equals_oracle(W, grid):
    nx, ny, nz, w, steps, storage, damping = grid
    shot = synth.config_small_layered(nx, ny, nz, w, steps, seed=nx * 3 + nz, nsrc=2)
    expect = oracle.run_shot(shot, steps=steps, precision="f32", storage=storage, damping=damping)
    if not damping:
        expect["phi"] = np.zeros_like(expect["u"])
    for k in KERNELS:
        say(f"case pair {k} grid {grid}")
        assert_same(run(W, shot, steps, k, storage, damping), expect, f"pair {k} {grid}")


def test_pair_refuses_eta_array_and_bad_tiles(W):
    nx, ny, nz, w = 40, 30, 20, 4
    shot = synth.config_small_layered(nx, ny, nz, w, 4, seed=5)
    _, e32 = oracle.eta_default(nx, ny, nz, w, shot.dx, shot.dy, shot.dz, shot.dt,
                                float(shot.vel.max()))
    sh = W.shot_from_synth(shot, eta=e32)
    assert W.wave_set_kernel(sh.ctx, W.WAVE_KERNEL_PAIR, 1, 16, 0) == W.WAVE_EINVAL
    sh.close()
    sh = W.shot_from_synth(shot)
    for bad in [(6, 2, 16, 0), (6, 1, 4, 0), (6, 1, 16, -2)]:
        assert W.wave_set_kernel(sh.ctx, *bad) == W.WAVE_EINVAL, bad
    assert W.wave_set_kernel(sh.ctx, W.WAVE_KERNEL_PAIR, 1, 8, 0) == W.WAVE_OK
    sh.close()


def test_pair_full_size_bf16_bitwise(W):
    """512^3, 20-cell layer, layered model, bf16 storage, from a random
    state: the launches the benchmark's bf16 leg can pick (two points per
    lane, both tile heights), 2 steps against the oracle's bf16 mode on
    every point."""
    shot = synth.config_c2(steps=2)
    rng = np.random.default_rng(21)
    shape = (shot.nz, shot.ny, shot.nx)
    w = shot.w
    k = np.arange(shot.nz)[:, None, None]
    j = np.arange(shot.ny)[None, :, None]
    i = np.arange(shot.nx)[None, None, :]
    lay = (i < w) | (i >= shot.nx - w) | (j < w) | (j >= shot.ny - w) | (k < w) | (k >= shot.nz - w)
    # u values representable in bf16 (the state is stored in the storage type)
    def bf16(a):
        b = a.astype(np.float32).view(np.uint32)
        b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
        return b.view(np.float32)
    st = {"u": bf16(rng.standard_normal(shape, dtype=np.float32) * np.float32(1e-2)),
          "u_prev": bf16(rng.standard_normal(shape, dtype=np.float32) * np.float32(1e-2)),
          "phi": np.where(lay, rng.standard_normal(shape, dtype=np.float32) * np.float32(1e-3),
                          np.float32(0)).astype(np.float32)}
    say("case pair 512^3 bf16: oracle")
    o = oracle.run_shot(shot, precision="f32", storage="bf16", state=st)
    for kern in [(6, 1, 8, 128), (6, 1, 16, 64)]:
        say(f"case pair 512^3 bf16 kernel {kern}")
        sh = W.shot_from_synth(shot, storage="bf16", max_steps=2)
        sh.write(W.WAVE_FIELD_U, st["u"])
        sh.write(W.WAVE_FIELD_UPREV, st["u_prev"])
        sh.write(W.WAVE_FIELD_PHI, st["phi"])
        sh.set_kernel(*kern)
        sh.step(2)
        g = dict(u=sh.read(W.WAVE_FIELD_U), u_prev=sh.read(W.WAVE_FIELD_UPREV),
                 phi=sh.read(W.WAVE_FIELD_PHI), traces=sh.traces())
        sh.close()
        assert_same(g, o, f"pair 512^3 bf16 {kern}")
