"""The streaming sweep with the z terms summed by the semi-stencil
(WAVE_KERNEL_SEMI, Sec. IV "Semi-stencil", along the streaming axis).

It evaluates the same Laplacian as every other kernel, summed in another
order (c_zm u(z+m) and c_zm u(z-m) enter separately, in the order the planes
stream past, instead of c_zm (u(z+m) + u(z-m))), so it cannot equal the
float32 oracle bit for bit.  Checked here:

* one step from random states, every point: the difference from the float32
  oracle stays within a per-point bound derived from the two summation
  orders (below), phi' is equal bit for bit (its gradient keeps its order),
  and the kernel did take another order (some points differ);
* against the float64 oracle after N steps: within 1e-5 relative L2 on the
  field and the traces (C1, and a layered grid over 500 steps);
* the refusal of an eta array.

Per-point bound for one step.  Both sums run over the same 26 products
c_i u_i (a pair sum (u(+m) + u(-m)) rounds once more), so each is within
gamma_n S of the exact Laplacian, S = sum |c_i| |u_i|, n <= 16, and the two
differ by at most 2 gamma_16 S (Higham, Accuracy and Stability, Sec. 3.1).
The update then rounds the same operations on both sides: lap + phi, the fma
with vp, the division by 1 + 2 eta, the final add; each contributes at most
one rounding unit (2^-24 relative) of its result on each side, i.e. 2^-23 of
its magnitude to the difference.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
U = 2.0 ** -24
GAMMA16 = 16 * U / (1 - 16 * U)


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


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu(W, shot, steps, nw=16, zchunk=0, state=None, damping=True, storage="f32"):
    sh = W.shot_from_synth(shot, storage=storage, damping=damping, max_steps=max(steps, 1))
    assert W.wave_set_kernel(sh.ctx, W.WAVE_KERNEL_SEMI, 1, nw, zchunk) == W.WAVE_OK
    layer = damping and shot.w > 0   # a phi field exists
    if state is not None:
        sh.write(W.WAVE_FIELD_U, state["u"])
        sh.write(W.WAVE_FIELD_UPREV, state["u_prev"])
        if layer:
            sh.write(W.WAVE_FIELD_PHI, state["phi"])
    sh.step(steps)
    out = dict(u=sh.read(W.WAVE_FIELD_U), traces=sh.traces(),
               phi=sh.read(W.WAVE_FIELD_PHI) if layer else None)
    sh.close()
    return out


def layer_mask(shot):
    w = shot.w
    k = np.arange(shot.nz)[:, None, None]
    j = np.arange(shot.ny)[None, :, None]
    i = np.arange(shot.nx)[None, None, :]
    return ((i < w) | (i >= shot.nx - w) | (j < w) | (j >= shot.ny - w) |
            (k < w) | (k >= shot.nz - w))


def random_state(shot, seed, damping=True):
    rng = np.random.default_rng(seed)
    shape = (shot.nz, shot.ny, shot.nx)
    st = {"u": rng.standard_normal(shape, dtype=np.float32) * np.float32(1e-2),
          "u_prev": rng.standard_normal(shape, dtype=np.float32) * np.float32(1e-2)}
    lay = layer_mask(shot) if damping else np.zeros(shape, bool)
    st["phi"] = np.where(lay, rng.standard_normal(shape, dtype=np.float32) * np.float32(1e-3),
                         np.float32(0)).astype(np.float32)
    return st


def one_step_bound(shot, st, damping=True):
    """Per-point bound on |u'_semi - u'_oracle32| after one step from `st`
    (float64 magnitudes of the quantities each side rounds)."""
    c64 = oracle.coefficients(shot.dx, shot.dy, shot.dz)
    c = c64.astype(np.float32).astype(np.float64)
    u = st["u"].astype(np.float64)
    up = np.pad(u, 4)
    nz, ny, nx = u.shape
    S = np.abs(c[0]) * np.abs(u)
    lap = c[0] * u
    for m in range(1, 5):
        for ax, cm in ((2, c[m]), (1, c[4 + m]), (0, c[8 + m])):
            sl_p = [slice(4, 4 + nz), slice(4, 4 + ny), slice(4, 4 + nx)]
            sl_m = list(sl_p)
            sl_p[ax] = slice(4 + m, 4 + m + u.shape[ax])
            sl_m[ax] = slice(4 - m, 4 - m + u.shape[ax])
            a, b = up[tuple(sl_p)], up[tuple(sl_m)]
            S += np.abs(cm) * (np.abs(a) + np.abs(b))
            lap += cm * (a + b)
    ce = abs(float(np.float32(-(np.float32(c[0]) + 2 * np.float32(c[1:].sum())))))
    S += ce * np.abs(u)
    _, vp32 = oracle.vp(shot.vel, shot.dt)
    vp = vp32.astype(np.float64)
    if damping:
        _, e32 = oracle.eta_default(shot.nx, shot.ny, shot.nz, shot.w, shot.dx, shot.dy, shot.dz,
                                    shot.dt, float(shot.vel.max()))
        eta = e32.astype(np.float64)
        phi = st["phi"].astype(np.float64)
    else:
        eta = np.zeros_like(u)
        phi = np.zeros_like(u)
    t = np.abs(u - st["u_prev"]) + eta * eta * np.abs(u)
    num = np.abs(vp * (lap + phi)) + t
    q = num / (1.0 + 2.0 * eta)
    out = np.abs(u) + q
    b = (vp * (2 * GAMMA16 * S + 2 * U * (np.abs(lap) + np.abs(phi)))
         + 2 * U * num + 2 * U * q + 4 * U * out)   # the last term also covers a source add
    return 1.01 * b


GRIDS = [  # nx, ny, nz, w, damping, nw, zchunk
    (70, 45, 37, 5, True, 16, 0),
    (130, 33, 21, 7, True, 8, 5),       # chunks shorter than the 4-plane delay
    (65, 17, 40, 3, True, 16, 3),
    (96, 40, 30, 0, True, 16, 0),        # no layer
    (100, 36, 26, 6, False, 8, 0),       # damping off
    (40, 40, 40, 20, True, 16, 7),       # all layer
    (9, 9, 9, 3, True, 16, 0),           # smaller than a tile
]


@pytest.mark.parametrize("g", GRIDS, ids=lambda g: f"{g[0]}x{g[1]}x{g[2]}_w{g[3]}_nw{g[5]}_z{g[6]}")
def test_semi_one_step_within_rounding_bound(W, g):
    nx, ny, nz, w, damping, nw, zc = g
    shot = synth.config_small_layered(nx, ny, nz, w, 1, seed=nx + 7 * nz, nsrc=2)
    st = random_state(shot, nx * ny + nz, damping)
    say(f"case semi one step {g}")
    o = oracle.run_shot(shot, steps=1, precision="f32", state=st, damping=damping)
    r = gpu(W, shot, 1, nw, zc, st, damping)
    bound = one_step_bound(shot, st, damping)
    d = np.abs(r["u"].astype(np.float64) - o["u"])
    worst = np.unravel_index(np.argmax(d / bound), d.shape)
    say(f"  max |diff|/bound {float((d / bound)[worst]):.3f}, points differing "
        f"{np.count_nonzero(d)} of {d.size}")
    assert np.all(d <= bound), (worst, d[worst], bound[worst])
    if r["phi"] is not None:
        assert np.array_equal(r["phi"], o["phi"])
    if nx * ny * nz > 2000:
        assert np.count_nonzero(d) > 0   # another summation order really ran
    # traces sample u': same bound at the receivers
    rec = shot.rec
    tb = bound[rec[:, 2], rec[:, 1], rec[:, 0]]
    assert np.all(np.abs(r["traces"][0] - o["traces"][0]) <= tb)


def test_semi_c1_vs_fp64(W):
    shot = synth.config_c1(steps=100)
    say("case semi c1 100 steps")
    r = gpu(W, shot, 100)
    o64 = oracle.run_shot(shot, precision="f64")
    o32 = oracle.run_shot(shot, precision="f32")
    eu, et = rel_l2(r["u"], o64["u"]), rel_l2(r["traces"], o64["traces"])
    say(f"  rel L2 vs fp64: field {eu:.3e} traces {et:.3e}; vs fp32 oracle "
        f"{rel_l2(r['u'], o32['u']):.3e}")
    assert eu <= 1e-5 and et <= 1e-5


def test_semi_long_run_vs_fp64(W):
    """128x112x96 layered grid with a 20-cell layer, 500 steps: within 1e-5 of
    float64 on the field and the traces."""
    shot = synth.config_small_layered(128, 112, 96, 20, 500, seed=41)
    shot.src = [(64, 56, 25)]
    shot.wavelet = synth.ricker(500, shot.dt)[None, :]
    shot.rec = synth.receiver_line(128, 56, 25)
    say("case semi long run 128x112x96 500 steps")
    r = gpu(W, shot, 500)
    o64 = oracle.run_shot(shot, precision="f64")
    eu, et = rel_l2(r["u"], o64["u"]), rel_l2(r["traces"], o64["traces"])
    say(f"  rel L2 vs fp64: field {eu:.3e} traces {et:.3e}")
    assert eu <= 1e-5 and et <= 1e-5


def test_semi_full_size_one_step_within_bound(W):
    """512^3, 20-cell layer, layered model, from a random state: one step of
    the semi-stencil kernel at the benchmark's size within the per-point
    bound of the float32 oracle."""
    shot = synth.config_c2(steps=1)
    st = random_state(shot, 31)
    say("case semi 512^3 one step: oracle")
    o = oracle.run_shot(shot, steps=1, precision="f32", state=st)
    say("case semi 512^3 one step: GPU")
    r = gpu(W, shot, 1, 16, 64, st)
    say("case semi 512^3 one step: bound")
    bound = one_step_bound(shot, st)
    d = np.abs(r["u"].astype(np.float64) - o["u"])
    assert np.all(d <= bound)
    assert np.array_equal(r["phi"], o["phi"])


def test_semi_refuses_eta_array_and_bad_tiles(W):
    nx, ny, nz, w = 40, 30, 20, 4
    shot = synth.config_small_layered(nx, ny, nz, w, 4, seed=5)
    _, e32 = oracle.eta_default(nx, ny, nz, w, shot.dx, shot.dy, shot.dz, shot.dt,
                                float(shot.vel.max()))
    sh = W.shot_from_synth(shot, eta=e32)
    assert W.wave_set_kernel(sh.ctx, W.WAVE_KERNEL_SEMI, 1, 16, 0) == W.WAVE_EINVAL
    sh.close()
    sh = W.shot_from_synth(shot)
    for bad in [(7, 2, 16, 0), (7, 1, 4, 0), (7, 1, 16, -1)]:
        assert W.wave_set_kernel(sh.ctx, *bad) == W.WAVE_EINVAL, bad
    sh.close()
