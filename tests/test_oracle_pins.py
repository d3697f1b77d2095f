"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test targets a part of the oracle such that a plausible mistake there
(a dropped term, a wrong sign or index, a transposed operand) fails it:

P1  polynomial exactness of Eq. 3 (weights, centre term, h scaling)
P2  plane-wave dispersion relation of Eq. 2 + Eq. 3 (update, anisotropic h)
P3  stability threshold of the scheme
P4  discrete energy conservation with damping off (symmetry, variable vp)
P5  axis-permutation symmetry with the layer on (layer formula indexing)
P6  dense Kronecker brute force of the whole recurrence incl. layer/sources
P7  eta = 0 reduces the layer update to Eq. 2 exactly
P8  linearity in the source amplitude
P9  source/receiver reciprocity (damping off)
P10 causality cone of the radius-4 star stencil
P11 the paper's Table III block counts from the Sec. III-B decomposition
P12 free-space amplitude of a point source
P13 table-mode eta gradient: closed-form derivative of the quadratic profile
P14 the layer absorbs: after a pulse has left the inner region, the energy
    left there is a small fraction of what a rigid box of the same size keeps
plus closed forms of the damping profile, (V dt)^2 and 16-bit rounding.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from tests import kron_ref

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- P1 ------
def test_p1_coefficient_moments_match_taylor_conditions():
    c = oracle.coefficients(1.0, 1.0, 1.0)
    C = [c[0] / 3.0] + list(c[1:5])
    expect = {0: 0.0, 2: 2.0, 4: 0.0, 6: 0.0, 8: 0.0}
    for p, v in expect.items():
        mom = C[0] * (1.0 if p == 0 else 0.0) + sum(2.0 * C[m] * m ** p for m in range(1, 5))
        assert abs(mom - v) < 1e-12, (p, mom)
    # degree 10 is not exact: the moment is -1152 (exact rational arithmetic)
    Cr = kron_ref.second_difference_weights(4)
    assert sum(2 * Cr[m] * Fraction(m) ** 10 for m in range(1, 5)) == -1152
    mom10 = sum(2.0 * C[m] * m ** 10 for m in range(1, 5))
    assert abs(mom10 + 1152.0) < 1e-9
    # the oracle's weights equal the rationals derived from Taylor conditions
    for m in range(5):
        assert abs(C[m] - float(Cr[m])) < 1e-15


def _lap_via_run(u, dx, dy, dz, precision="f64"):
    """One oracle step from u^0 = u^{-1} = u with vp = 1 gives u^1 = u + lap u."""
    nz, ny, nx = u.shape
    vel = np.ones(u.shape, np.float32)
    out = oracle.run(nx, ny, nz, 0, dx, dy, dz, 1.0, vel, 1, damping=False,
                     precision=precision, state=dict(u=u, u_prev=u))
    return out["u"] - u


@pytest.mark.parametrize("h", [1.0, 10.0])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_p1_polynomial_exactness_through_the_run_loop(h, axis):
    n = 21
    idx = np.arange(n, dtype=np.float64) - 10.0
    coords = [idx * h] * 3
    Z, Y, X = np.meshgrid(coords[2], coords[1], coords[0], indexing="ij")
    var = [X, Y, Z][axis]
    interior = (slice(4, n - 4),) * 3
    for p in range(0, 10):
        u = var ** p
        lap = _lap_via_run(u, h, h, h)
        exact = p * (p - 1) * var ** (p - 2) if p >= 2 else np.zeros_like(var)
        scale = max(1.0, np.abs(u[interior]).max() / (h * h))
        err = np.abs(lap[interior] - exact[interior]).max() / scale
        assert err < 1e-12, (p, err)
    # degree 10: error is exactly -1152 h^8 (from the moment above)
    u = var ** 10
    lap = _lap_via_run(u, h, h, h)
    exact = 90.0 * var ** 8
    d = (lap - exact)[interior]
    assert np.allclose(d, -1152.0 * h ** 8, rtol=1e-6, atol=0)


def test_p1_mixed_polynomial_anisotropic_spacing():
    dx, dy, dz = 7.0, 11.0, 13.0
    n = 17
    i = np.arange(n) - 8.0
    Z, Y, X = np.meshgrid(i * dz, i * dy, i * dx, indexing="ij")
    u = X ** 3 * Y ** 2 + Z ** 9 - 3.0 * X * Y * Z + Y ** 7
    exact = 6 * X * Y ** 2 + 2 * X ** 3 + 72 * Z ** 7 + 42 * Y ** 5
    lap = _lap_via_run(u, dx, dy, dz)
    s = (slice(4, n - 4),) * 3
    assert np.abs(lap[s] - exact[s]).max() / np.abs(exact[s]).max() < 1e-12


# ---------------------------------------------------------------- P2 ------
def test_p2_plane_wave_dispersion_relation():
    nx, ny, nz = 40, 44, 48
    dx, dy, dz = 10.0, 12.0, 9.0
    v, dt = 2000.0, 1.5e-3
    kvec = np.array([2 * np.pi / (11.3 * dx), 2 * np.pi / (17.9 * dy), -2 * np.pi / (8.7 * dz)])
    C = oracle.coefficients(1.0, 1.0, 1.0)
    C0 = C[0] / 3.0
    K = 0.0
    for a, h in enumerate((dx, dy, dz)):
        K -= (C0 + 2.0 * sum(C[m] * np.cos(m * kvec[a] * h) for m in range(1, 5))) / (h * h)
    omega = 2.0 * np.arcsin(v * dt * np.sqrt(K) / 2.0) / dt
    k_, j_, i_ = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    phase = kvec[0] * i_ * dx + kvec[1] * j_ * dy + kvec[2] * k_ * dz
    u0 = np.cos(phase)
    um1 = np.cos(phase + omega * dt)
    steps = 4
    vel = np.full((nz, ny, nx), v, np.float32)
    out = oracle.run(nx, ny, nz, 0, dx, dy, dz, dt, vel, steps, damping=False,
                     state=dict(u=u0, u_prev=um1))
    # points unaffected by the zero values beyond the faces: > 4*steps cells in
    vp = (float(np.float32(v)) * dt) ** 2
    assert vp > 0
    m = 4 * steps + 1
    s = (slice(m, nz - m), slice(m, ny - m), slice(m, nx - m))
    expect = np.cos(phase - omega * steps * dt)
    err = np.abs(out["u"][s] - expect[s]).max()
    assert err < 1e-11, err
    # and a 1 % wrong phase speed is clearly detected
    wrong = np.cos(phase - 1.01 * omega * steps * dt)
    assert np.abs(out["u"][s] - wrong[s]).max() > 1e-4


# ---------------------------------------------------------------- P3 ------
def test_p3_stability_number_closed_form():
    S = kron_ref.second_difference_weights(4)
    sym = S[0] + 2 * sum(S[m] * (-1) ** m for m in range(1, 5))
    assert abs(float(sym) + 6.501587301587302) < 1e-12
    limit = 2.0 / math.sqrt(3.0 * abs(float(sym)))
    assert abs(limit - 0.45286) < 1e-5
    assert abs(oracle.stability(1.0, 1.0, 1.0, limit, 1.0) - 1.0) < 1e-12
    assert oracle.stability(10.0, 10.0, 10.0, 0.4 * 10.0 / 2000.0, 2000.0) < 1.0


@pytest.mark.parametrize("courant,grows", [(0.45, False), (0.47, True)])
def test_p3_nyquist_mode_growth(courant, grows):
    n = 24
    k_, j_, i_ = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    u0 = (-1.0) ** (i_ + j_ + k_)
    vel = np.ones((n, n, n), np.float32)
    out = oracle.run(n, n, n, 0, 1.0, 1.0, 1.0, courant, vel, 400, damping=False,
                     state=dict(u=u0, u_prev=u0))
    amp = np.abs(out["u"]).max()
    if grows:
        assert amp > 1e3
    else:
        assert amp < 10.0


def test_p3_layer_update_growth_factor_bound():
    """Without the Laplacian the damped update of one point has the growth
    factors lam of (1 + 2 eta) lam^2 - (2 + 2 eta - eta^2) lam + 1 = 0; a
    root leaves the unit circle through -1 at eta = 2 + 2 sqrt(2)."""
    bound = 2.0 + 2.0 * math.sqrt(2.0)
    for eta, unstable in [(bound - 1e-6, False), (bound + 1e-6, True), (1.0, False), (8.0, True)]:
        lam = np.roots([1.0 + 2.0 * eta, -(2.0 + 2.0 * eta - eta * eta), 1.0])
        assert (np.abs(lam).max() > 1.0) == unstable, (eta, lam)
    # at the bound -1 is a root exactly
    assert abs((1 + 2 * bound) + (2 + 2 * bound - bound * bound) + 1) < 1e-12


@pytest.mark.parametrize("w", [1, 2, 3, 4])
def test_p3_thin_layers_amplify_where_eta_exceeds_the_bound(w):
    """The oracle's layer update against that bound: the default profile's
    largest eta (a corner cell, three axis terms) lies above 2 + 2 sqrt(2)
    for 1- and 2-cell layers, and a random state then grows; from 3 cells
    it lies below and the state stays bounded."""
    n = 24
    shot = synth.config_small_layered(n, n, n, w, 12, seed=5, nsrc=1)
    e64, _ = oracle.eta_default(n, n, n, w, shot.dx, shot.dy, shot.dz, shot.dt,
                                float(shot.vel.max()))
    above = float(e64.max()) > 2.0 + 2.0 * math.sqrt(2.0)
    assert above == (w <= 2)
    rng = np.random.default_rng(9)
    st = {"u": rng.standard_normal((n, n, n)) * 1e-2,
          "u_prev": rng.standard_normal((n, n, n)) * 1e-2}
    out = oracle.run_shot(shot, steps=12, precision="f64", state=st)
    amp = float(np.abs(out["u"]).max())
    if above:
        assert amp > 10.0, amp
    else:
        assert amp < 1.0, amp


# ---------------------------------------------------------------- P4 ------
def test_p4_energy_conserved_with_damping_off():
    nx, ny, nz = 30, 26, 34
    shot = synth.config_small_layered(nx, ny, nz, 4, 10, seed=11)
    vp64, _ = oracle.vp(shot.vel, shot.dt)
    k_, j_, i_ = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    bump = np.exp(-(((i_ - 14) / 3.0) ** 2 + ((j_ - 12) / 2.5) ** 2 + ((k_ - 17) / 3.5) ** 2))
    state = dict(u=bump, u_prev=bump)
    e = []
    for _ in range(6):
        prev_u = state["u"].copy()
        out = oracle.run(nx, ny, nz, 0, shot.dx, shot.dy, shot.dz, shot.dt, shot.vel, 40,
                         damping=False, state=state)
        state = dict(u=out["u"], u_prev=out["u_prev"], phi=out["phi"])
        e.append(oracle.energy(vp64, out["u"], out["u_prev"], shot.dx, shot.dy, shot.dz))
        assert not np.array_equal(prev_u, out["u"])
    e = np.array(e)
    assert e[0] > 0
    assert np.abs(e - e[0]).max() / e[0] < 1e-12, (e - e[0]) / e[0]


def test_p4_energy_decays_with_damping_on():
    nx = ny = nz = 32
    w = 8
    vel = np.full((nz, ny, nx), 2000.0, np.float32)
    dt = 0.4 * 10.0 / 2000.0
    vp64, _ = oracle.vp(vel, dt)
    k_, j_, i_ = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    bump = np.exp(-(((i_ - 16) ** 2 + (j_ - 16) ** 2 + (k_ - 16) ** 2) / 4.0))
    out0 = oracle.run(nx, ny, nz, w, 10.0, 10.0, 10.0, dt, vel, 1, state=dict(u=bump, u_prev=bump))
    e0 = oracle.energy(vp64, out0["u"], out0["u_prev"], 10.0, 10.0, 10.0)
    out = oracle.run(nx, ny, nz, w, 10.0, 10.0, 10.0, dt, vel, 300, state=dict(u=bump, u_prev=bump))
    e1 = oracle.energy(vp64, out["u"], out["u_prev"], 10.0, 10.0, 10.0)
    assert e1 < 0.1 * e0


# ---------------------------------------------------------------- P5 ------
def test_p5_axis_permutation_symmetry_with_layer():
    n, w = 28, 6
    vel = np.full((n, n, n), 2000.0, np.float32)
    dt = 0.4 * 10.0 / 2000.0
    c = n // 2
    wav = synth.ricker(60, dt)[None, :]
    out = oracle.run(n, n, n, w, 10.0, 10.0, 10.0, dt, vel, 60, src=[(c, c, c)], wavelet=wav)
    u = out["u"]
    ph = out["phi"]
    scale = np.abs(u).max()
    assert scale > 0 and np.abs(ph).max() > 0
    for perm in [(0, 2, 1), (1, 0, 2), (2, 1, 0), (1, 2, 0), (2, 0, 1)]:
        assert np.abs(u - u.transpose(perm)).max() / scale < 1e-13, perm
        assert np.abs(ph - ph.transpose(perm)).max() / np.abs(ph).max() < 1e-12, perm


def test_p5_transposed_inputs_give_transposed_outputs():
    nx, ny, nz, w = 20, 24, 18, 4
    dx, dy, dz = 10.0, 12.0, 8.0
    rng = np.random.default_rng(3)
    vel = (2000 + 300 * rng.random((nz, ny, nx))).astype(np.float32)
    dt = 0.3 * 8.0 / float(vel.max())
    wav = synth.ricker(30, dt)[None, :]
    a = oracle.run(nx, ny, nz, w, dx, dy, dz, dt, vel, 30, src=[(7, 11, 9)], wavelet=wav)
    # swap x and z: array axes (z, y, x) -> (x, y, z)
    velT = np.ascontiguousarray(vel.transpose(2, 1, 0))
    b = oracle.run(nz, ny, nx, w, dz, dy, dx, dt, velT, 30, src=[(9, 11, 7)], wavelet=wav)
    ua, ub = a["u"], b["u"].transpose(2, 1, 0)
    assert np.abs(ua - ub).max() / np.abs(ua).max() < 1e-13


# ---------------------------------------------------------------- P6 ------
@pytest.mark.parametrize("w", [2, 3])
def test_p6_matches_dense_kronecker_form(w):
    nx, ny, nz = 7, 8, 9
    dx, dy, dz = 9.0, 10.0, 11.0
    rng = np.random.default_rng(42 + w)
    vel = rng.uniform(1500, 3000, (nz, ny, nx)).astype(np.float32)
    dt = 0.35 * 9.0 / float(vel.max())
    eta = np.zeros((nz, ny, nx))
    inner = np.zeros((nz, ny, nx), bool)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                inner[k, j, i] = oracle.is_inner(nx, ny, nz, w, i, j, k)
    eta[~inner] = rng.uniform(0.02, 0.3, (~inner).sum())
    src = [(3, 4, 4), (1, 6, 7)]
    steps = 10
    wav = rng.standard_normal((2, steps)).astype(np.float32)
    out = oracle.run(nx, ny, nz, w, dx, dy, dz, dt, vel, steps, src=src, wavelet=wav, eta=eta)
    vp64, _ = oracle.vp(vel, dt)
    u, up, ph = kron_ref.run(nx, ny, nz, w, dx, dy, dz, vp64.ravel(), eta.ravel(), src,
                             wav.astype(np.float64), steps, inner.ravel())
    for got, ref in ((out["u"], u), (out["u_prev"], up), (out["phi"], ph)):
        ref = ref.reshape(nz, ny, nx)
        assert np.abs(ref).max() > 0
        assert np.abs(got - ref).max() / np.abs(ref).max() < 1e-13
    # the layer really took part: phi is non-zero only in the layer
    assert np.abs(out["phi"][~inner]).max() > 0
    assert np.abs(out["phi"][inner]).max() == 0


# ---------------------------------------------------------------- P7 ------
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_p7_eta_zero_reduces_to_eq2_exactly(precision):
    shot = synth.config_small_layered(24, 20, 22, 5, 40, seed=5, nsrc=2)
    a = oracle.run_shot(shot, precision=precision, eta=np.zeros((22, 20, 24)))
    b = oracle.run_shot(shot, precision=precision, damping=False)
    assert np.abs(a["u"]).max() > 0
    assert np.array_equal(a["u"], b["u"])
    assert np.array_equal(a["traces"], b["traces"])


# ---------------------------------------------------------------- P8 ------
@pytest.mark.parametrize("precision,storage", [("f64", "f32"), ("f32", "f32"), ("f32", "bf16")])
def test_p8_linearity_in_source_amplitude(precision, storage):
    shot = synth.config_small_layered(24, 24, 24, 6, 30, seed=8)
    a = oracle.run_shot(shot, precision=precision, storage=storage)
    shot.wavelet = shot.wavelet * np.float32(2.0)
    b = oracle.run_shot(shot, precision=precision, storage=storage)
    big = np.abs(a["u"]) > 1e-20     # away from underflow at the front
    assert big.sum() > 1000
    assert np.array_equal(2.0 * a["u"][big], b["u"][big])


# ---------------------------------------------------------------- P9 ------
def test_p9_source_receiver_reciprocity():
    nx, ny, nz = 26, 24, 28
    shot = synth.config_small_layered(nx, ny, nz, 4, 80, seed=9)
    s, r = (6, 7, 9), (18, 15, 20)
    wav = shot.wavelet[:1]
    a = oracle.run(nx, ny, nz, 0, shot.dx, shot.dy, shot.dz, shot.dt, shot.vel, 80,
                   src=[s], wavelet=wav, rec=np.array([r]), damping=False)
    b = oracle.run(nx, ny, nz, 0, shot.dx, shot.dy, shot.dz, shot.dt, shot.vel, 80,
                   src=[r], wavelet=wav, rec=np.array([s]), damping=False)
    # injecting vp(s) w into u is a right-hand side w e_s of the symmetric
    # system diag(1/vp) (u' - 2u + u_prev) = lap u, so the response at r to
    # a source at s equals the response at s to a source at r
    ta = a["traces"][:, 0]
    tb = b["traces"][:, 0]
    assert np.abs(ta).max() > 0
    assert np.abs(ta - tb).max() / np.abs(ta).max() < 1e-12


# ---------------------------------------------------------------- P10 -----
def test_p10_causality_cone():
    n, w = 41, 8
    vel = np.full((n, n, n), 2000.0, np.float32)
    dt = 0.4 * 10.0 / 2000.0
    src = (20, 19, 21)
    steps = 4
    wav = np.ones((1, steps), np.float32)
    out = oracle.run(n, n, n, w, 10.0, 10.0, 10.0, dt, vel, steps, src=[src], wavelet=wav)
    k_, j_, i_ = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    d1 = np.abs(i_ - src[0]) + np.abs(j_ - src[1]) + np.abs(k_ - src[2])
    u = out["u"]
    # the source enters u^1; u^steps is supported within L1 distance 4(steps-1)
    reach = 4 * (steps - 1)
    assert np.all(u[d1 > reach] == 0.0)
    on_axis = u[src[2], src[1], src[0] + reach]
    assert on_axis != 0.0


# ---------------------------------------------------------------- P11 -----
def _table3():
    rows = []
    with open(os.path.join(GOLD, "table3_grid_sizes.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            t = line.split()
            rows.append((t[0], *map(int, t[1:])))
    return rows


def test_p11_table3_block_counts_from_decomposition():
    N, W = 1000, 27
    rows = _table3()
    assert len(rows) == 25
    r3 = oracle.regions(N, N, N, W, 0)
    r25 = oracle.regions(N, N, N, W, 1)
    cdiv = lambda a, b: -(-a // b)
    for name, Dx, Dy, Dz, inner, tb, fb, lr in rows:
        if Dz > 0:
            boxes = r3
            cnt = [cdiv(b[3], Dx) * cdiv(b[4], Dy) * cdiv(b[5], Dz) for b in boxes]
            # 3-D cut: [inner, top, bottom, front, back, left, right]
            got = (cnt[0], cnt[1], cnt[3], cnt[5])
            assert cnt[1] == cnt[2] and cnt[3] == cnt[4] and cnt[5] == cnt[6]
        else:
            boxes = r25
            cnt = [cdiv(b[3], Dx) * cdiv(b[4], Dy) for b in boxes]
            # streamed cut: x walls, y walls, z caps pair up with the table's
            # top/bottom, front/back, left/right columns respectively
            got = (cnt[0], cnt[1], cnt[3], cnt[5])
            assert cnt[1] == cnt[2] and cnt[3] == cnt[4] and cnt[5] == cnt[6]
        assert got == (inner, tb, fb, lr), name


@pytest.mark.parametrize("order", [0, 1])
def test_p11_regions_partition_the_grid(order):
    nx, ny, nz, w = 19, 23, 17, 4
    cover = np.zeros((nz, ny, nx), np.int32)
    boxes = oracle.regions(nx, ny, nz, w, order)
    for b in boxes:
        x0, y0, z0, ex, ey, ez = b
        cover[z0:z0 + ez, y0:y0 + ey, x0:x0 + ex] += 1
    assert np.all(cover == 1)
    x0, y0, z0, ex, ey, ez = boxes[0]
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                inside = x0 <= i < x0 + ex and y0 <= j < y0 + ey and z0 <= k < z0 + ez
                assert inside == oracle.is_inner(nx, ny, nz, w, i, j, k)


# ---------------------------------------------------------------- P12 -----
def test_p12_free_space_point_source_amplitude():
    n, w = 72, 4
    h, v = 10.0, 2000.0
    vel = np.full((n, n, n), v, np.float32)
    dt = 0.4 * h / v
    steps = 150
    wav = synth.ricker(steps, dt)[None, :]
    c = 36
    r_cells = 16
    rec = np.array([[c + r_cells, c, c], [c, c + r_cells, c], [c, c, c - r_cells]], np.int32)
    out = oracle.run(n, n, n, 0, h, h, h, dt, vel, steps, src=[(c, c, c)], wavelet=wav,
                     rec=rec, damping=False)
    r = r_cells * h
    t = (np.arange(steps) + 1) * dt
    tau = t - r / v
    pred = h ** 3 * ((1 - 2 * (np.pi * 15 * (tau - 1.5 / 15)) ** 2)
                     * np.exp(-(np.pi * 15 * (tau - 1.5 / 15)) ** 2)) / (4 * np.pi * r)
    # only before anything reflected from the faces comes back
    tr = out["traces"]
    for q in range(3):
        g = tr[:, q]
        assert abs(np.abs(g).max() / np.abs(pred).max() - 1.0) < 0.05
        assert abs(int(np.argmax(g)) - int(np.argmax(pred))) <= 2


def test_p14_layer_absorbs_what_a_rigid_box_reflects():
    """The layer (Sec. III-A, PML region) exists to absorb outgoing waves.
    A 15 Hz Ricker pulse at the centre of an 80^3 grid (16-cell layer, h =
    10 m, 2000 m/s) has left the 48^3 inner region by step 200 (0.4 s; its
    farthest corner is 416 m away); a rigid box of the same size (damping
    off: Eq. 2 on every cell, zero ghosts) sends it back in.  The paper
    prints no reflection figure, so the bounds are this test's: the inner L2
    norm with the layer at most 3 % of the rigid box's at steps 280 and 320
    (about 1.4 % and 0.85 % measured) and at most 1 % of its own peak by
    step 320 (about 0.4 %).  A layer with the wrong sign amplifies, one
    applied to the wrong cells reflects; both fail.  Before the wavefront
    reaches the layer the two runs agree."""
    n, w, h, v = 80, 16, 10.0, 2000.0
    dt = 0.4 * h / v
    vel = np.full((n, n, n), v, np.float32)
    c = n // 2
    wav = synth.ricker(400, dt)[None, :]
    inner = (slice(w, n - w),) * 3
    marks = (60, 100, 280, 320)

    def inner_norms(damping):
        out, state, done = {}, None, 0
        for t in marks:
            r = oracle.run(n, n, n, w, h, h, h, dt, vel, t - done, src=[(c, c, c)],
                           wavelet=wav, damping=damping, state=state, n0=done)
            state = dict(u=r["u"], u_prev=r["u_prev"], phi=r["phi"])
            done = t
            out[t] = float(np.linalg.norm(r["u"][inner]))
        return out

    lay, box = inner_norms(True), inner_norms(False)
    peak = max(lay[60], lay[100])
    assert abs(lay[60] / box[60] - 1.0) < 1e-3
    assert lay[280] <= 0.03 * box[280] and lay[320] <= 0.03 * box[320]
    assert lay[320] <= 0.01 * peak
    assert box[320] >= 0.3 * peak  # the rigid box keeps the energy in


# --------------------------------------------------- closed forms ---------
def test_eta_profile_closed_form():
    nx, ny, nz, w = 40, 36, 44, 8
    h, dt, vmax, refl = 10.0, 2e-3, 3000.0, 1e-3
    e64, e32 = oracle.eta_default(nx, ny, nz, w, h, h, h, dt, vmax, refl)
    d0 = 3.0 * vmax * math.log(1.0 / refl) / (2.0 * w * h)
    assert np.all(e64[w:nz - w, w:ny - w, w:nx - w] == 0.0)
    # outermost face-centre cell on x: one axis at full depth
    assert e64[nz // 2, ny // 2, 0] == pytest.approx(dt * d0, rel=1e-14)
    # first layer cell: depth 1 cell
    assert e64[nz // 2, ny // 2, w - 1] == pytest.approx(dt * d0 / w ** 2, rel=1e-14)
    # corner: three axes add
    assert e64[0, 0, 0] == pytest.approx(3 * dt * d0, rel=1e-14)
    # mirror symmetry about every mid-plane
    assert np.array_equal(e64, e64[:, :, ::-1])
    assert np.array_equal(e64, e64[:, ::-1, :])
    assert np.array_equal(e64, e64[::-1, :, :])
    assert np.array_equal(e32, e64.astype(np.float32))
    assert np.all(e64[~np.pad(np.ones((nz - 2 * w, ny - 2 * w, nx - 2 * w), bool), w)] > 0)


def test_eta_axis_tables_closed_form_and_sum():
    nx, ny, nz, w = 30, 26, 34, 6
    dx, dy, dz, dt, vmax, refl = 10.0, 12.5, 8.0, 1.5e-3, 3200.0, 1e-3
    tx, ty, tz = oracle.eta_axis_tables(nx, ny, nz, w, dx, dy, dz, vmax, refl)
    e64, _ = oracle.eta_default(nx, ny, nz, w, dx, dy, dz, dt, vmax, refl)
    for t, n, h in ((tx, nx, dx), (ty, ny, dy), (tz, nz, dz)):
        d0 = 3.0 * vmax * math.log(1.0 / refl) / (2.0 * w * h)
        assert t.shape == (n + 2,)
        for i in range(-1, n + 1):
            depth = w - i if i < w else (i - (n - 1 - w) if i > n - 1 - w else 0)
            assert t[i + 1] == pytest.approx(d0 * (depth / w) ** 2, rel=1e-14, abs=0.0), (n, i)
    # eta of the array is dt ((t_x + t_y) + t_z), bit for bit
    s = (tx[1:-1][None, None, :] + ty[1:-1][None, :, None]) + tz[1:-1][:, None, None]
    assert np.array_equal(dt * s, e64)


# ---------------------------------------------------------------- P13 -----
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_p13_table_gradient_is_the_profile_derivative(axis):
    """One float64 step from u = a ramp along one axis, u_prev = u, phi = 0:
    phi' = -(de_a / (4 h_a^2)) (u(+a) - u(-a)) / (1 + eta) on layer points.
    For the quadratic profile the central difference is exact:
    de_a(i) = -4 dt d0 (w - i) / w^2 in the low layer, +4 dt d0 (i - (n-1-w)) / w^2
    in the high one, 0 between -- including the outermost cells, where the
    profile continues past the face."""
    n3 = [22, 19, 24]
    w = 5
    h3 = [10.0, 12.0, 9.0]
    nz, ny, nx = n3[2], n3[1], n3[0]
    dt, vmax = 1e-3, 2500.0
    vel = np.full((nz, ny, nx), vmax, np.float32)
    idx = np.indices((nz, ny, nx))[2 - axis].astype(np.float64)
    u = 1.0 + idx                    # ramp along `axis`
    st = dict(u=u, u_prev=u.copy(), phi=np.zeros_like(u))
    r = oracle.run(nx, ny, nz, w, h3[0], h3[1], h3[2], dt, vel, 1, precision="f64",
                   state=st, eta="default")
    e64 = r["eta"]
    n = n3[axis]
    d0 = 3.0 * vmax * math.log(1.0 / 1e-3) / (2.0 * w * h3[axis])
    up = np.pad(u, 1)                # zero beyond the faces
    sl_p = [slice(1, -1)] * 3
    sl_m = [slice(1, -1)] * 3
    sl_p[2 - axis] = slice(2, None)
    sl_m[2 - axis] = slice(0, -2)
    du = up[tuple(sl_p)] - up[tuple(sl_m)]
    lay = ~np.pad(np.ones((nz - 2 * w, ny - 2 * w, nx - 2 * w), bool), w)
    de = np.where(lay, -r["phi"] * (1.0 + e64) * 4.0 * h3[axis] ** 2 / du, 0.0)
    i = idx.astype(int)
    # (the first inner cell next to the layer sees one layer neighbour of
    # depth 1: -+ dt d0 / w^2)
    want = np.where(i < w, -4.0 * dt * d0 * (w - i) / w ** 2,
                    np.where(i > n - 1 - w, 4.0 * dt * d0 * (i - (n - 1 - w)) / w ** 2, 0.0))
    want = np.where(i == w, -dt * d0 / w ** 2, np.where(i == n - 1 - w, dt * d0 / w ** 2, want))
    # points off the other axes' outer faces (there the zero beyond the face
    # gives the ramp a difference along those axes too)
    other = np.ones((nz, ny, nx), bool)
    for b in range(3):
        if b != axis:
            j = np.indices((nz, ny, nx))[2 - b]
            other &= (j >= 1) & (j <= n3[b] - 2)
    m = lay & other
    assert m.sum() > 100 and np.any(m & (i == 0)) and np.any(m & (i == n - 1))
    np.testing.assert_allclose(de[m], want[m], rtol=1e-9, atol=1e-15)
    # the float32 mode rounds the same differences once
    r32 = oracle.run(nx, ny, nz, w, h3[0], h3[1], h3[2], dt, vel, 1, precision="f32",
                     state=st, eta="default")
    np.testing.assert_allclose(r32["phi"][lay], r["phi"][lay], rtol=2e-6, atol=0)


def test_table_and_array_gradients_agree_off_the_faces():
    """The axis-term gradient equals the array difference wherever both
    neighbours are inside the grid (the other axes' terms cancel); they
    differ on the outermost cells, where the array is zero beyond the face."""
    nx, ny, nz, w = 20, 18, 16, 4
    dt, h = 1e-3, 10.0
    vel = np.full((nz, ny, nx), 2000.0, np.float32)
    rng = np.random.default_rng(5)
    st = dict(u=rng.standard_normal((nz, ny, nx)), u_prev=rng.standard_normal((nz, ny, nx)),
              phi=rng.standard_normal((nz, ny, nx)))
    a = oracle.run(nx, ny, nz, w, h, h, h, dt, vel, 1, precision="f64", state=st, eta="default")
    b = oracle.run(nx, ny, nz, w, h, h, h, dt, vel, 1, precision="f64", state=st,
                   eta="default-array")
    assert np.array_equal(a["u"], b["u"])             # the gradient only enters phi
    interior = np.zeros((nz, ny, nx), bool)
    interior[1:-1, 1:-1, 1:-1] = True
    np.testing.assert_allclose(a["phi"][interior], b["phi"][interior], rtol=1e-12, atol=1e-15)
    assert not np.allclose(a["phi"][~interior], b["phi"][~interior], rtol=1e-6)


def test_vp_is_v_dt_squared():
    vel = np.array([1500.0, 2000.0, 4321.5], np.float32)
    v64, v32 = oracle.vp(vel, 1.7e-3)
    assert np.array_equal(v64, (vel.astype(np.float64) * 1.7e-3) ** 2)
    assert np.array_equal(v32, v64.astype(np.float32))


def test_16bit_rounding_matches_ieee_library_conversions():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    xs = np.concatenate([
        rng.standard_normal(4000).astype(np.float32) * 10.0 ** rng.integers(-8, 5, 4000),
        np.array([0.0, -0.0, 65504.0, 65519.99, 65520.0, 1e-7, 6.1e-5, 5.96e-8, 2.9e-8,
                  3.0e-8, 1e-45, 3.4e38, -3.39e38, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8],
                 np.float32)])
    with np.errstate(over="ignore"):
        f16 = xs.astype(np.float16).astype(np.float32)
    b16 = torch.from_numpy(xs).to(torch.bfloat16).to(torch.float32).numpy()
    for x, a, b in zip(xs, f16, b16):
        ra, rb = oracle.round_f16(float(x)), oracle.round_bf16(float(x))
        assert (ra == a) or (math.isinf(ra) and math.isinf(a)), (x, ra, a)
        assert (rb == b) or (math.isinf(rb) and math.isinf(b)), (x, rb, b)


def test_fp32_mode_tracks_fp64_within_tolerance():
    shot = synth.config_c1(steps=100)
    a = oracle.run_shot(shot, precision="f64")
    b = oracle.run_shot(shot, precision="f32")
    rel = np.linalg.norm(b["u"] - a["u"]) / np.linalg.norm(a["u"])
    assert rel < 1e-5, rel
    rt = np.linalg.norm(b["traces"] - a["traces"]) / np.linalg.norm(a["traces"])
    assert rt < 1e-5, rt


def test_fp32_mode_long_damped_run_within_tolerance():
    """400 steps with the layer absorbing most of the wave: the float32 mode
    (Eq. 3 in its printed order with the float weights' residual removed,
    updates around the increment u - u_prev) stays within 1e-5 relative L2
    of float64."""
    shot = synth.config_small_layered(64, 56, 48, 10, 400, seed=41)
    shot.src = [(32, 28, 15)]
    shot.wavelet = synth.ricker(400, shot.dt)[None, :]
    shot.rec = synth.receiver_line(64, 28, 15)
    a = oracle.run_shot(shot, precision="f64")
    b = oracle.run_shot(shot, precision="f32")
    assert np.linalg.norm(b["u"] - a["u"]) / np.linalg.norm(a["u"]) < 1e-5
    assert np.linalg.norm(b["traces"] - a["traces"]) / np.linalg.norm(a["traces"]) < 1e-5
