"""GPU parity: the HIP path through the C ABI against the CPU oracle.

The kernels evaluate every point with the same float32 operations in the same
order as the oracle's float32 mode, so the comparison with it is exact
(value equality of every field element and trace sample).  Against the
float64 oracle the bar is 1e-5 relative L2 after N steps (float32 storage).
16-bit storage is exact against the oracle's 16-bit mode and its distance
from float64 is reported and bounded.
"""
import os
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


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


def gpu_run(W, shot, steps, storage="f32", damping=True, kernel=None, state=None, eta=None,
            two_step=False):
    sh = W.shot_from_synth(shot, storage=storage, damping=damping, max_steps=max(steps, 1),
                           eta=eta, two_step=two_step)
    if kernel is not None:
        sh.set_kernel(*kernel)
    if state is not None:
        sh.write(W.WAVE_FIELD_U, state["u"])
        sh.write(W.WAVE_FIELD_UPREV, state["u_prev"])
        if damping and "phi" in state:
            sh.write(W.WAVE_FIELD_PHI, state["phi"])
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


def rel_l2(a, b):
    n = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / n) if n > 0 else float(np.linalg.norm(a))


# --------------------------------------------------------------------------
def test_c1_plain_fp32_vs_oracle(W):
    """64^3, 16-cell layer, 2000 m/s, Ricker at the centre, 100 steps."""
    shot = synth.config_c1(steps=100)
    say("case c1 64^3 w16 100 steps")
    g = gpu_run(W, shot, 100)
    o32 = oracle.run_shot(shot, precision="f32")
    o32["traces"] = o32["traces"]
    assert_same(g, o32, "c1 vs fp32 oracle")
    o64 = oracle.run_shot(shot, precision="f64")
    eu, et = rel_l2(g["u"], o64["u"]), rel_l2(g["traces"], o64["traces"])
    say(f"c1 rel L2 vs fp64: field {eu:.3e} traces {et:.3e}")
    assert eu <= 1e-5 and et <= 1e-5
    assert np.abs(g["phi"]).max() > 0          # the layer update ran
    assert np.abs(g["traces"]).max() > 0


RAGGED = [
    (70, 45, 37, 5, 2),     # partial x tile, partial y tiles
    (65, 17, 130, 3, 1),    # 1 lane in the last x tile; long z
    (130, 33, 11, 4, 3),
    (9, 200, 21, 3, 1),     # narrow x (3 inner columns)
    (1, 1, 1, 0, 1),        # a single point
    (64, 16, 8, 0, 1),      # no layer
    (40, 40, 40, 20, 1),    # all layer (2w = n)
]

KERNELS = [(W_, ry, nw, zc) for (W_, ry, nw, zc) in [
    (0, 1, 16, 0), (1, 1, 16, 0), (1, 1, 8, 0), (1, 2, 8, 0), (1, 2, 4, 0),
    (1, 1, 16, 5), (1, 2, 8, 7), (1, 1, 8, 1), (1, 2, 4, 3),
    # 64 x 32 tiles (two rows per wavefront, 16 wavefronts)
    (1, 2, 16, 0), (1, 2, 16, 3),
    # the persistent launch of the same tiles
    (8, 1, 16, 0), (8, 1, 8, 0), (8, 1, 16, 5), (8, 1, 8, 1),
    # x neighbours by wavefront shuffles
    (9, 1, 16, 0), (9, 1, 8, 3)]]


@pytest.mark.parametrize("case", RAGGED, ids=lambda c: "x".join(map(str, c[:3])) + f"_w{c[3]}")
def test_ragged_grids_every_kernel_bitwise(W, case):
    nx, ny, nz, w, nsrc = case
    steps = 25
    shot = synth.config_small_layered(nx, ny, nz, w, steps, seed=nx * 7 + ny, nsrc=nsrc)
    say(f"case ragged {case}")
    ref = oracle.run_shot(shot, precision="f32")
    for k in KERNELS:
        g = gpu_run(W, shot, steps, kernel=k)
        assert_same(g, ref, f"{case} kernel {k}")


def test_eta_array_mode_and_table_mode(W):
    """An explicit per-point eta (array mode) against the oracle with the same
    eta; the default profile held as tables against the oracle's table mode
    (and the same profile passed as an array against the oracle's array
    mode).  The two modes differ only in how the eta differences round, and
    on the outermost cells, where the tables continue the profile past the
    face: tight agreement in between."""
    nx, ny, nz, w = 70, 45, 37, 5
    shot = synth.config_small_layered(nx, ny, nz, w, 25, seed=77, nsrc=2)
    e64, e32 = oracle.eta_default(nx, ny, nz, w, shot.dx, shot.dy, shot.dz, shot.dt,
                                  float(shot.vel.max()))
    rng = np.random.default_rng(5)
    eta = (e32 * (1.0 + 0.5 * rng.random(e32.shape))).astype(np.float32)
    say("case eta array mode")
    ref = oracle.run_shot(shot, precision="f32", eta=eta)
    for k in [(0, 1, 16, 0), (1, 1, 16, 0), (1, 1, 8, 5), (1, 2, 8, 0), (1, 2, 4, 3),
              (8, 1, 16, 0), (9, 1, 16, 0), (9, 1, 8, 4)]:
        assert_same(gpu_run(W, shot, 25, kernel=k, eta=eta), ref, f"array mode {k}")
    # 64 x 32 tiles take the default profile's tables only
    sh = W.shot_from_synth(shot, eta=eta, max_steps=1)
    assert W.wave_set_kernel(sh.ctx, 1, 2, 16, 0) == W.WAVE_EINVAL
    sh.close()
    tab = gpu_run(W, shot, 25)
    arr = gpu_run(W, shot, 25, eta=e32)
    assert_same(tab, oracle.run_shot(shot, precision="f32"), "table mode vs oracle")
    assert_same(arr, oracle.run_shot(shot, precision="f32", eta="default-array"),
                "default profile as an array vs oracle")
    assert rel_l2(tab["u"], arr["u"]) < 1e-5 and rel_l2(tab["traces"], arr["traces"]) < 1e-5


# Bound vs float64 from the storage rounding unit u (2^-8 bf16, 2^-11 f16):
# one rounding per stored value and step, accumulating like a random walk over
# N steps with a modest amplification, 2 sqrt(N) u.
@pytest.mark.parametrize("storage,unit", [("bf16", 2.0 ** -8), ("f16", 2.0 ** -11)])
def test_16bit_storage_exact_vs_oracle_and_bounded_vs_fp64(W, storage, unit):
    bound = 2.0 * np.sqrt(150.0) * unit
    shot = synth.config_small_layered(96, 80, 72, 12, 150, seed=21)
    say(f"case storage {storage}")
    g = gpu_run(W, shot, 150, storage=storage)
    o = oracle.run_shot(shot, precision="f32", storage=storage)
    assert_same(g, o, storage)
    for k in [(0, 1, 16, 0), (1, 2, 8, 9)]:
        assert_same(gpu_run(W, shot, 150, storage=storage, kernel=k), o, f"{storage} {k}")
    o64 = oracle.run_shot(shot, precision="f64")
    eu, et = rel_l2(g["u"], o64["u"]), rel_l2(g["traces"], o64["traces"])
    say(f"{storage} rel L2 vs fp64 after 150 steps: field {eu:.3e} traces {et:.3e} "
        f"(bound {bound:.3e})")
    assert eu < bound and et < bound


def test_energy_conserved_with_damping_off(W):
    nx, ny, nz = 80, 72, 64
    shot = synth.config_small_layered(nx, ny, nz, 0, 1, seed=31)
    shot.src, shot.wavelet, shot.rec = [], np.zeros((0, 1), np.float32), None
    k_, j_, i_ = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    bump = np.exp(-(((i_ - 40) / 4.0) ** 2 + ((j_ - 30) / 3.0) ** 2
                    + ((k_ - 33) / 5.0) ** 2)).astype(np.float32)
    say("case energy damping off")
    sh = W.shot_from_synth(shot, damping=False, max_steps=1)
    sh.write(W.WAVE_FIELD_U, bump)
    sh.write(W.WAVE_FIELD_UPREV, bump)
    e = [sh.energy()]
    # the device energy equals the oracle's float64 energy of the same fields
    # with the float32 vp the scheme runs with (sum order differs: 1e-11)
    _, vp32 = oracle.vp(shot.vel, shot.dt)
    vp64 = vp32.astype(np.float64)
    for _ in range(5):
        sh.step(60)
        e.append(sh.energy())
    u, up = sh.read(W.WAVE_FIELD_U), sh.read(W.WAVE_FIELD_UPREV)
    eo = oracle.energy(vp64, u, up, shot.dx, shot.dy, shot.dz)
    assert abs(e[-1] - eo) <= 1e-11 * abs(eo)
    e = np.array(e)
    drift = np.abs(e - e[0]).max() / e[0]
    say(f"float32 fields, float64 energy: max relative drift over 300 steps {drift:.3e}")
    assert e[0] > 0 and drift < 1e-5
    sh.close()


def random_state(shot, seed):
    """u^n, u^{n-1} random everywhere and phi random in the layer (zero
    elsewhere): every point of the grid then carries a nonzero value, so a
    tile that is skipped, doubled or misplaced shows up."""
    rng = np.random.default_rng(seed)
    shape = (shot.nz, shot.ny, shot.nx)
    u = (rng.standard_normal(shape, dtype=np.float32) * np.float32(1e-2))
    up = (rng.standard_normal(shape, dtype=np.float32) * np.float32(1e-2))
    w = shot.w
    k = np.arange(shot.nz)[:, None, None]
    j = np.arange(shot.ny)[None, :, None]
    i = np.arange(shot.nx)[None, None, :]
    lay = ((i < w) | (i >= shot.nx - w) | (j < w) | (j >= shot.ny - w) | (k < w) | (k >= shot.nz - w))
    phi = np.where(lay, rng.standard_normal(shape, dtype=np.float32) * np.float32(1e-3),
                   np.float32(0)).astype(np.float32)
    return {"u": u, "u_prev": up, "phi": phi}


# wave_tune's candidates at 512^3: every compiled tile at the automatic chunk
# (64 planes; 32 for the 64 x 32 tile), half and double; the persistent
# launch at the automatic chunk and half; two steps per launch at 64, 32,
# 128; two points per lane (16 rows: 32 and 64 planes, 8 rows: 64 and 128);
# the four code shapes it times
C2_CANDIDATES = (
    [(1, ry, nw, z) for (ry, nw) in [(1, 16), (1, 8), (2, 8), (2, 4)] for z in (64, 32, 128)]
    + [(1, 2, 16, z) for z in (32, 16, 64)]
    + [(8, 1, 16, 64), (8, 1, 16, 32), (8, 1, 8, 64), (8, 1, 8, 32),
       (2, 1, 16, 64), (2, 1, 16, 32), (2, 1, 16, 128),
       (6, 1, 16, 32), (6, 1, 16, 64), (6, 1, 8, 64), (6, 1, 8, 128),
       (9, 1, 16, 64), (9, 1, 8, 64),
       (3, 8, 8, 8), (3, 64, 4, 4), (4, 1, 16, 0), (5, 1, 16, 0)])


@pytest.fixture(scope="module")
def c2_case():
    """512^3, 20-cell layer, layered model, from a random state, and the
    float32 oracle's result after 4 steps."""
    shot = synth.config_c2(steps=4)
    st = random_state(shot, 11)
    say("case c2 512^3: oracle, 4 steps")
    return shot, st, oracle.run_shot(shot, precision="f32", state=st)


@pytest.mark.parametrize("k", C2_CANDIDATES, ids=lambda k: "v{}_{}x{}_z{}".format(*k))
def test_c2_full_size_few_steps_bitwise(W, c2_case, k):
    """Every launch configuration the benchmark's tuner can pick at 512^3
    (the streaming tiles at their z-chunk lengths, the persistent launch,
    two steps per launch, two points per lane, and the paper's other code
    shapes it times: 3-D 8x8x8 and 64x4x4, the LDS plane ring, the shifted
    register queue), 4 steps against the float32 oracle on every point."""
    shot, st, o = c2_case
    say(f"case c2 512^3 4 steps kernel {k}")
    assert_same(gpu_run(W, shot, 4, kernel=k, state=st, two_step=k[0] == 2), o, f"c2 512^3 {k}")


def test_c3_size_few_steps_bitwise(W):
    """1024^3 with a 32-cell layer (the large-domain configuration's grid and
    layer; constant velocity so that the model is quick to build), from a
    random state: one step of the default launch against the float32 oracle
    on every point."""
    n, w = 1024, 32
    vel = synth.constant_velocity(n, n, n, 3000.0)
    dt = synth._dt_for(3000.0)
    c = n // 2
    shot = synth.Shot("c3_size", n, n, n, w, synth.H, synth.H, synth.H, dt, vel, 1,
                      src=[(c, c, w + 5), (w + 2, 9, n - 3)],
                      wavelet=np.stack([synth.ricker(1, dt, t0=0.0), synth.ricker(1, dt, t0=0.0)]),
                      rec=synth.receiver_line(n, c, w + 5), seed=0)
    say("case c3-size 1024^3 1 step: random state")
    st = random_state(shot, 12)
    say("case c3-size 1024^3 1 step: oracle")
    o = oracle.run_shot(shot, steps=1, precision="f32", state=st)
    for k in (None, (8, 1, 16, 64)):
        say(f"case c3-size 1024^3 1 step: GPU kernel {k or 'default'}")
        g = gpu_run(W, shot, 1, state=st, kernel=k)
        assert_same(g, o, f"1024^3 {k}")
        del g


def test_paper_shape_one_step_bitwise(W):
    """The paper's 1000^3 grid with a 27-cell layer (Sec. V-B, Table III):
    its width is not a multiple of the 64-column tiles, so the last tile
    column holds 40 columns and lanes past the grid.  From a random state,
    one step of the default launch (persistent) and of the per-tile launch
    against the float32 oracle on every point."""
    n, w = 1000, 27
    vel = synth.constant_velocity(n, n, n, 3000.0)
    dt = synth._dt_for(3000.0)
    c = n // 2
    shot = synth.Shot("paper_shape", n, n, n, w, synth.H, synth.H, synth.H, dt, vel, 1,
                      src=[(c, c, w + 5), (n - 3, n - 5, 2)],
                      wavelet=np.stack([synth.ricker(1, dt, t0=0.0), synth.ricker(1, dt, t0=0.0)]),
                      rec=synth.receiver_line(n, c, w + 5), seed=0)
    say("case paper shape 1000^3 1 step: random state")
    st = random_state(shot, 13)
    say("case paper shape 1000^3 1 step: oracle")
    o = oracle.run_shot(shot, steps=1, precision="f32", state=st)
    for k in (None, (1, 1, 8, 0)):
        say(f"case paper shape 1000^3 1 step: GPU kernel {k or 'default'}")
        g = gpu_run(W, shot, 1, state=st, kernel=k)
        assert_same(g, o, f"1000^3 {k}")
        del g


def test_long_run_medium_grid_vs_oracles(W):
    """500 steps in 100-step segments: exact against the float32 oracle, and
    within 1e-5 relative L2 of the float64 oracle at every checkpoint."""
    shot = synth.config_small_layered(128, 112, 96, 20, 500, seed=41)
    c = (64, 56, 25)
    shot.src = [c]
    shot.wavelet = synth.ricker(500, shot.dt)[None, :]
    shot.rec = synth.receiver_line(128, 56, 25)
    say("case long run 128x112x96 500 steps")
    sh = W.shot_from_synth(shot, max_steps=500)
    st64 = None
    peak = 0.0
    rows = []
    for seg in range(5):
        sh.step(100)
        g = sh.read(W.WAVE_FIELD_U)
        o = oracle.run_shot(shot, steps=100, precision="f64", state=st64, n0=100 * seg)
        st64 = dict(u=o["u"], u_prev=o["u_prev"], phi=o["phi"])
        nrm = float(np.linalg.norm(o["u"]))
        peak = max(peak, nrm)
        err = float(np.linalg.norm(g - o["u"]))
        rows.append((100 * (seg + 1), nrm, err))
        say(f"  step {100 * (seg + 1)}: |u| {nrm:.3e} rel L2 {err / nrm:.3e} "
            f"err/peak {err / peak:.3e}")
    traces = sh.traces()
    gu = sh.read(W.WAVE_FIELD_U)
    sh.close()
    o32 = oracle.run_shot(shot, precision="f32")
    assert np.array_equal(gu, o32["u"]) and np.array_equal(traces, o32["traces"])
    o64 = oracle.run_shot(shot, precision="f64")
    et = rel_l2(traces, o64["traces"])
    say(f"500 steps traces rel L2 vs fp64 {et:.3e}")
    assert et <= 1e-5
    for step, nrm, err in rows:
        assert err <= 1e-5 * nrm, step


def test_deterministic_and_restartable(W):
    shot = synth.config_small_layered(72, 66, 60, 8, 60, seed=51)
    say("case determinism/restart")
    a = gpu_run(W, shot, 60)
    b = gpu_run(W, shot, 60)
    assert_same(a, b, "run twice")
    # 25 steps, snapshot, new context from the snapshot, 35 more steps
    first = gpu_run(W, shot, 25)
    rest = synth.config_small_layered(72, 66, 60, 8, 60, seed=51)
    rest.wavelet = np.ascontiguousarray(rest.wavelet[:, 25:])
    c = gpu_run(W, rest, 35, state=first)
    for key in ("u", "u_prev", "phi"):
        assert np.array_equal(c[key], a[key]), key
    assert np.array_equal(np.concatenate([first["traces"], c["traces"]]), a["traces"])


def test_error_paths(W):
    shot = synth.config_small_layered(32, 32, 32, 4, 10, seed=61)
    sh = W.shot_from_synth(shot, max_steps=10)
    assert W.wave_inject(sh.ctx, 32, 0, 0, np.zeros(3, np.float32)) == W.WAVE_EINVAL
    assert W.wave_inject(sh.ctx, 0, 0, 0, np.zeros(11, np.float32)) == W.WAVE_EINVAL
    assert W.wave_step(sh.ctx, 11) == W.WAVE_EINVAL        # trace buffer of 10 steps
    assert W.wave_step(sh.ctx, -1) == W.WAVE_EINVAL
    assert W.wave_write_field(sh.ctx, W.WAVE_FIELD_VP, np.zeros((32, 32, 32), np.float32)) \
        == W.WAVE_EINVAL
    assert W.wave_set_kernel(sh.ctx, W.WAVE_KERNEL_STREAM, 3, 3, 0) == W.WAVE_EINVAL
    assert W.wave_step(sh.ctx, 10) == W.WAVE_OK
    assert sh.step_count == 10
    sh.close()


def test_stream_copy_copies(W):
    import torch
    src = torch.arange(1 << 20, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    s = torch.cuda.current_stream()
    assert W.wave_stream_copy(dst.data_ptr(), src.data_ptr(), src.numel() * 4, s.cuda_stream) == 0
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
