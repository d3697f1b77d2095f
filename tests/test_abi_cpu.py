"""The C-ABI library loads, exports every declared symbol, and its host-only
helpers agree with the oracle (no device work: runs without a GPU)."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wave.h")
LIB = os.path.join(ROOT, "paper_2009_04619_amd", "libwave.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libwave.so not built")


@pytest.fixture(scope="module")
def W():
    from paper_2009_04619_amd import wave
    return wave


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(wave_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(W):
    names = declared_functions()
    assert len(names) >= 20
    lib = C.CDLL(LIB)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(W.EXPORTED) == names


def _desc(W, **kw):
    base = dict(nx=40, ny=36, nz=44, w=8, dx=10.0, dy=12.0, dz=9.0, dt=1e-3)
    base.update(kw)
    return W.make_desc(**base)


def test_coefficients_match_oracle_bitwise(W):
    for dx, dy, dz in [(10.0, 10.0, 10.0), (10.0, 12.0, 9.0), (1.0, 3.5, 0.25)]:
        d = _desc(W, dx=dx, dy=dy, dz=dz)
        rc, c = W.wave_coefficients(d)
        assert rc == 0
        assert np.array_equal(c, oracle.coefficients(dx, dy, dz).astype(np.float32))


def test_default_eta_matches_oracle_bitwise(W):
    d = _desc(W, dt=1.7e-3)
    rc, e = W.wave_eta_default(d, 3210.5)
    assert rc == 0
    _, e32 = oracle.eta_default(40, 36, 44, 8, 10.0, 12.0, 9.0, 1.7e-3, 3210.5, 1e-3)
    assert np.array_equal(e, e32)


def test_stability_matches_oracle(W):
    d = _desc(W, dt=1.3e-3)
    assert W.wave_stability(d, 2500.0) == pytest.approx(
        oracle.stability(10.0, 12.0, 9.0, 1.3e-3, 2500.0), rel=1e-14)


def test_bytes_required_and_validation(W):
    d = _desc(W)
    n = W.wave_bytes_required(d)
    # u^n, u^{n-1}, vp, phi padded float arrays (default profile: no eta array)
    pitch = ((40 + 8 + 63) // 64) * 64
    arr = (44 + 8) * (36 + 8) * pitch * 4
    assert n >= 4 * arr
    assert n % 256 == 0
    ne = W.wave_bytes_required(_desc(W, eta_array=True))
    assert ne >= 5 * arr and ne > n   # the eta array replaces the small profile tables
    assert W.wave_bytes_required(_desc(W, storage="bf16")) < n
    assert W.wave_bytes_required(_desc(W, damping=False)) < n
    for bad in (dict(nx=0), dict(w=-1), dict(w=19), dict(dx=0.0), dict(dt=-1.0),
                dict(dt=float("nan")), dict(storage=7), dict(refl=1.5), dict(max_rec=-1)):
        assert W.wave_bytes_required(_desc(W, **bad)) == 0, bad
    d = _desc(W)
    d.reserved = 1
    assert W.wave_bytes_required(d) == 0


def test_stochastic_rounding_flag_only_with_bf16_and_single_steps(W):
    """WAVE_STOCH_ROUND is a bf16-storage option: accepted there (same arena
    as plain bf16), refused with float32 or binary16 storage and together
    with WAVE_TWO_STEP."""
    plain = W.wave_bytes_required(_desc(W, storage="bf16"))
    assert W.wave_bytes_required(_desc(W, storage="bf16", stochastic_round=True)) == plain > 0
    assert W.wave_bytes_required(_desc(W, storage="f32", stochastic_round=True)) == 0
    assert W.wave_bytes_required(_desc(W, storage="f16", stochastic_round=True)) == 0
    assert W.wave_bytes_required(_desc(W, storage="bf16", stochastic_round=True, two_step=True)) == 0
    assert W.WAVE_STOCH_ROUND == 8


def test_alloc_rejects_bad_arguments_before_touching_a_device(W):
    d = _desc(W, dt=1e-3)
    vel = np.full((44, 36, 40), 2000.0, np.float32)
    need = W.wave_bytes_required(d)
    rc, _ = W.wave_alloc(d, vel, None, 0, need, 0)
    assert rc == W.WAVE_EINVAL                          # NULL arena
    rc, _ = W.wave_alloc(d, vel, None, 256 * 1000 + 8, need, 0)
    assert rc == W.WAVE_EINVAL                          # misaligned arena
    rc, _ = W.wave_alloc(d, vel, None, 256 * 1000, need - 256, 0)
    assert rc == W.WAVE_ENOMEM
    bad = vel.copy()
    bad[3, 4, 5] = np.nan
    rc, _ = W.wave_alloc(d, bad, None, 256 * 1000, need, 0)
    assert rc == W.WAVE_EINVAL
    fast = _desc(W, dt=0.1)
    rc, _ = W.wave_alloc(fast, vel, None, 256 * 1000, W.wave_bytes_required(fast), 0)
    assert rc == W.WAVE_EUNSTABLE
    assert "stability" in W.wave_last_error()
    neg = np.full((44, 36, 40), -1.0, np.float32)
    de = _desc(W, dt=1e-3, eta_array=True)
    rc, _ = W.wave_alloc(de, vel, neg, 256 * 1000, W.wave_bytes_required(de), 0)
    assert rc == W.WAVE_EINVAL                          # negative eta
    ok_eta = np.zeros((44, 36, 40), np.float32)
    rc, _ = W.wave_alloc(d, vel, ok_eta, 256 * 1000, need, 0)
    assert rc == W.WAVE_EINVAL                          # eta without the flag
    rc, _ = W.wave_alloc(de, vel, None, 256 * 1000, W.wave_bytes_required(de), 0)
    assert rc == W.WAVE_EINVAL                          # flag without eta


def test_null_context_is_rejected(W):
    assert W.wave_step(None, 1) == W.WAVE_EINVAL
    assert W.wave_free(None) == 0
    assert W.wave_strerror(W.WAVE_EUNSTABLE).startswith("time step")


def test_stream_copy_rejects_misaligned(W):
    assert W.wave_stream_copy(16, 32, 17, 0) == W.WAVE_EINVAL
    assert W.wave_stream_copy(8, 32, 16, 0) == W.WAVE_EINVAL


def _eta_limit(stab):
    return 2.0 + math.sqrt(8.0 - 4.0 * stab * stab)


@pytest.mark.parametrize("w,ok", [(1, False), (2, False), (3, True), (4, True), (20, True)])
def test_alloc_rejects_layers_whose_damped_update_amplifies(W, w, ok):
    """Courant number 0.4 with the default profile (refl 1e-3): the largest
    eta, 3 * 4.145 / w at a grid corner, reaches the damped update's bound
    2 + sqrt(8 - 4 s^2) (s the stability number) for 1- and 2-cell layers
    only; the check runs on the host before any device work."""
    n = 48
    vmax = 3000.0
    dt = 0.4 * 10.0 / vmax
    d = _desc(W, nx=n, ny=n, nz=n, w=w, dx=10.0, dy=10.0, dz=10.0, dt=dt)
    vel = np.full((n, n, n), vmax, np.float32)
    e64, _ = oracle.eta_default(n, n, n, w, 10.0, 10.0, 10.0, dt, vmax)
    lim = _eta_limit(oracle.stability(10.0, 10.0, 10.0, dt, vmax))
    assert (float(e64.max()) < lim) == ok
    # inputs are validated before the arena: a stable descriptor passes every
    # check and stops at the NULL arena (EINVAL) without touching a device
    rc, _ = W.wave_alloc(d, vel, None, 0, W.wave_bytes_required(d), 0)
    if ok:
        assert rc == W.WAVE_EINVAL and "arena" in W.wave_last_error()
    else:
        assert rc == W.WAVE_EUNSTABLE
        assert "eta" in W.wave_last_error()


def test_alloc_rejects_eta_arrays_at_the_bound(W):
    n = 24
    vmax = 2500.0
    dt = 0.3 * 10.0 / vmax
    de = _desc(W, nx=n, ny=n, nz=n, w=6, dx=10.0, dy=10.0, dz=10.0, dt=dt, eta_array=True)
    vel = np.full((n, n, n), vmax, np.float32)
    lim = _eta_limit(oracle.stability(10.0, 10.0, 10.0, dt, vmax))
    need = W.wave_bytes_required(de)
    for val, code in [(lim * 1.001, W.WAVE_EUNSTABLE), (lim * 0.999, W.WAVE_EINVAL)]:
        eta = np.zeros((n, n, n), np.float32)
        eta[0, 5, 7] = val
        # a stable input gets past every host check and stops at the NULL
        # arena (EINVAL) without touching a device
        rc, _ = W.wave_alloc(de, vel, eta, 0, need, 0)
        assert rc == code, (val, lim)
        if code == W.WAVE_EINVAL:
            assert "arena" in W.wave_last_error()


def test_admission_under_a_budget(W):
    d = _desc(W)
    need = W.wave_bytes_required(d)
    assert W.wave_admit(d, need, 0) == (W.WAVE_OK, need, True)
    assert W.wave_admit(d, 3 * need, 2 * need) == (W.WAVE_OK, need, True)
    assert W.wave_admit(d, 3 * need, 2 * need + 1) == (W.WAVE_OK, need, False)   # defer
    assert W.wave_admit(d, 3 * need, 5 * need) == (W.WAVE_OK, need, False)
    rc, n, fits = W.wave_admit(d, need - 1, 0)
    assert (rc, n, fits) == (W.WAVE_EBUDGET, need, False)                        # never fits
    assert "budget" in W.wave_last_error()
    assert W.wave_admit(_desc(W, nx=0), 10 ** 12, 0)[0] == W.WAVE_EINVAL
