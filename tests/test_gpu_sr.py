"""bf16 storage with stochastic rounding (WAVE_STOCH_ROUND) against the
oracle's stochastically rounded bf16 mode, bit for bit: every launch shape
that supports it on ragged grids (odd widths, tiles past the padded row, a
layer wider than half a tile, a grid smaller than every tile), the per-point
eta array, and batches, whose members equal their solo runs.  The random
bits of a point depend on its grid position and step only, so every shape
draws the same ones."""
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


def run(W, shot, steps, kernel, eta=None):
    sh = W.shot_from_synth(shot, storage="bf16", stochastic_round=True, max_steps=max(steps, 1),
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


GRIDS = [  # nx, ny, nz, w, steps
    (70, 45, 37, 5, 14),
    (129, 33, 20, 7, 10),     # the last 128-wide pair tile reaches past the padded row
    (200, 48, 44, 20, 8),     # a layer wider than half a tile row
    (6, 6, 7, 3, 6),          # all layer, smaller than every tile
]
KERNELS = [(0, 0, 0, 0), (1, 1, 16, 0), (1, 1, 8, 5), (1, 2, 8, 0), (1, 2, 4, 3), (1, 2, 16, 0),
           (8, 1, 16, 0), (8, 1, 8, 0), (6, 1, 16, 0), (6, 1, 8, 3), (9, 1, 16, 0),
           (3, 8, 8, 8), (4, 1, 16, 0), (5, 1, 16, 0)]


@pytest.mark.parametrize("grid", GRIDS, ids=lambda g: f"{g[0]}x{g[1]}x{g[2]}_w{g[3]}")
def test_stochastic_rounding_equals_oracle_every_shape(W, grid):
    nx, ny, nz, w, steps = grid
    shot = synth.config_small_layered(nx, ny, nz, w, steps, seed=nx + 7 * nz, nsrc=2)
    expect = oracle.run_shot(shot, steps=steps, precision="f32", storage="bf16sr")
    plain = oracle.run_shot(shot, steps=steps, precision="f32", storage="bf16")
    assert not np.array_equal(expect["u"], plain["u"])   # the rounding is really different
    for k in KERNELS:
        say(f"case sr {k} grid {grid}")
        assert_same(run(W, shot, steps, k), expect, f"sr {k} {grid}")


def test_stochastic_rounding_with_an_eta_array(W):
    nx, ny, nz, w = 70, 45, 37, 5
    shot = synth.config_small_layered(nx, ny, nz, w, 20, seed=78, nsrc=2)
    _, e32 = oracle.eta_default(nx, ny, nz, w, shot.dx, shot.dy, shot.dz, shot.dt,
                                float(shot.vel.max()))
    eta = (e32 * (1.0 + 0.5 * np.random.default_rng(6).random(e32.shape))).astype(np.float32)
    expect = oracle.run_shot(shot, precision="f32", storage="bf16sr", eta=eta)
    for k in [(0, 0, 0, 0), (1, 1, 16, 0), (1, 1, 8, 0), (8, 1, 16, 0), (9, 1, 8, 0)]:
        say(f"case sr eta array {k}")
        assert_same(run(W, shot, 20, k, eta=eta), expect, f"sr eta array {k}")


def test_batched_members_equal_solo_runs_and_rounding_must_agree(W):
    shots = [synth.config_small_layered(nx, ny, nz, 5, st, seed=900 + nx, nsrc=1)
             for (nx, ny, nz, st) in [(70, 45, 37, 20), (96, 40, 30, 13), (33, 65, 41, 17)]]
    solo = [oracle.run_shot(s, precision="f32", storage="bf16sr") for s in shots]
    for tile in [(1, 16), (1, 8), (0, 16), (0, 8)]:
        say(f"case sr batch tile {tile}")
        members = [W.shot_from_synth(s, storage="bf16", stochastic_round=True) for s in shots]
        b = W.Batch(storage="bf16", max_shots=8)
        for s, m in zip(shots, members):
            b.add(m, s.steps)
        b.set_kernel(*tile)
        b.set_graph(4)
        b.run(max(s.steps for s in shots))
        b.close()
        for s, m, ref in zip(shots, members, solo):
            got = dict(u=m.read(W.WAVE_FIELD_U), u_prev=m.read(W.WAVE_FIELD_UPREV),
                       phi=m.read(W.WAVE_FIELD_PHI), traces=m.traces())
            assert_same(got, ref, f"sr batch {tile} {s.nx}x{s.ny}x{s.nz}")
            m.close()
    # a batch runs one kernel instance: members must agree on the rounding
    a = W.shot_from_synth(shots[0], storage="bf16", stochastic_round=True)
    c = W.shot_from_synth(shots[1], storage="bf16")
    b = W.Batch(storage="bf16", max_shots=4)
    b.add(a, 2)
    assert W.wave_batch_add(b.b, c.ctx, 2) == W.WAVE_EINVAL
    b.close()
    a.close()
    c.close()


def _random_state(shot, seed):
    rng = np.random.default_rng(seed)
    shape = (shot.nz, shot.ny, shot.nx)
    u = rng.standard_normal(shape, dtype=np.float32) * np.float32(1e-2)
    up = rng.standard_normal(shape, dtype=np.float32) * np.float32(1e-2)
    w = shot.w
    k = np.arange(shot.nz)[:, None, None]
    j = np.arange(shot.ny)[None, :, None]
    i = np.arange(shot.nx)[None, None, :]
    lay = (i < w) | (i >= shot.nx - w) | (j < w) | (j >= shot.ny - w) | (k < w) | (k >= shot.nz - w)
    phi = np.where(lay, rng.standard_normal(shape, dtype=np.float32) * np.float32(1e-3),
                   np.float32(0)).astype(np.float32)
    return {"u": u, "u_prev": up, "phi": phi}


@pytest.fixture(scope="module")
def c2_sr_case():
    """The 512^3 benchmark grid (20-cell layer, layered model) from a random
    state, and the oracle's stochastically rounded bf16 result after 3 steps."""
    shot = synth.config_c2(steps=3)
    st = _random_state(shot, 21)
    say("case sr 512^3: oracle, 3 steps")
    return shot, st, oracle.run_shot(shot, precision="f32", storage="bf16sr", state=st)


@pytest.mark.parametrize("k", [(1, 2, 4, 64), (1, 1, 16, 64), (8, 1, 16, 32), (6, 1, 16, 64),
                               (6, 1, 8, 64)], ids=lambda k: "v{}_{}x{}_z{}".format(*k))
def test_stochastic_rounding_full_size_bitwise(W, c2_sr_case, k):
    """The launches the tuner can pick for the benchmark's stochastically
    rounded bf16 leg, 3 steps at 512^3 against the oracle on every point."""
    shot, st, expect = c2_sr_case
    say(f"case sr 512^3 3 steps kernel {k}")
    sh = W.shot_from_synth(shot, storage="bf16", stochastic_round=True, max_steps=3)
    sh.set_kernel(*k)
    sh.write(W.WAVE_FIELD_U, st["u"])
    sh.write(W.WAVE_FIELD_UPREV, st["u_prev"])
    sh.write(W.WAVE_FIELD_PHI, st["phi"])
    sh.step(3)
    got = dict(u=sh.read(W.WAVE_FIELD_U), u_prev=sh.read(W.WAVE_FIELD_UPREV),
               phi=sh.read(W.WAVE_FIELD_PHI), traces=sh.traces())
    sh.close()
    assert_same(got, expect, f"sr 512^3 {k}")
