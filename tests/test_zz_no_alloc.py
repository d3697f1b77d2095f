"""wave_energy_noalloc (the entry point for callers that cannot allocate)
against wave_energy: the same value bit for bit, on two calls in a row, the
second with a smaller grid (the static workspace keeps the first call's
partial sums beyond the second grid's rows, which must not leak in), and
the refusal of grids with more rows than the workspace holds."""
import sys

import numpy as np
import pytest

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


def shot_with_state(W, nx, ny, nz, seed, steps=3):
    shot = synth.config_small_layered(nx, ny, nz, 4, steps, seed=seed)
    sh = W.shot_from_synth(shot, max_steps=steps)
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    sh.write(W.WAVE_FIELD_U, rng.standard_normal(shape, dtype=np.float32) * np.float32(1e-2))
    sh.write(W.WAVE_FIELD_UPREV, rng.standard_normal(shape, dtype=np.float32) * np.float32(1e-2))
    sh.step(steps)
    return sh


def noalloc_energy(W, sh):
    import torch
    out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda:0")
    assert W.wave_energy_noalloc(sh.ctx, out.data_ptr()) == W.WAVE_OK
    sh.sync()
    r = out.cpu().numpy()
    return float(r[0] - r[1])


def test_noalloc_energy_equals_wave_energy_twice_second_smaller(W):
    for (nx, ny, nz, seed) in [(96, 80, 72, 1), (40, 30, 20, 2)]:
        say(f"case noalloc energy {nx}x{ny}x{nz}")
        sh = shot_with_state(W, nx, ny, nz, seed)
        ref = sh.energy()
        got = noalloc_energy(W, sh)
        sh.close()
        say(f"  wave_energy {ref!r} noalloc {got!r}")
        assert np.isfinite(ref) and ref != 0.0
        assert got == ref


def test_noalloc_energy_rejects_grids_beyond_the_workspace(W):
    import torch
    nx, ny, nz = 1, 1025, 1024          # 1049600 rows > 1048576
    vel = synth.constant_velocity(nx, ny, nz, 2000.0)
    sh = W.Shot(nx, ny, nz, 0, 10.0, 10.0, 10.0, 0.002, vel, damping=False, max_steps=1)
    out = torch.zeros(2, dtype=torch.float64, device="cuda:0")
    assert W.wave_energy_noalloc(sh.ctx, out.data_ptr()) == W.WAVE_EINVAL
    assert W.wave_energy_noalloc(sh.ctx, 0) == W.WAVE_EINVAL
    sh.close()
