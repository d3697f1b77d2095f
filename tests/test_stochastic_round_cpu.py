"""Stochastic rounding of bf16 storage in the oracle, pinned to its
definition and to the properties of its hash (CPU only).

The rounding takes a float to one of its two bfloat16 neighbours, the one
farther from zero with probability equal to the dropped fraction of an ulp;
so over all 2^16 values of the random bits it returns the float itself on
average, exactly.  The random bits come from the 32-bit "pcg" hash of
Jarzynski and Olano (JCGT 2020), a bijection of 32-bit words."""
import numpy as np
import pytest

import oracle


def test_pcg_hash_is_a_bijection_with_balanced_bits():
    """A PCG step and the RXS-M-XS permutation are both bijections of 32-bit
    words: distinct inputs give distinct outputs; and each output bit is set
    for about half of a run of consecutive inputs."""
    xs = list(range(1 << 16)) + [0xFFFFFFFF - i for i in range(1 << 12)] + [1 << b for b in range(32)]
    hs = [oracle.pcg_hash(x) for x in xs]
    assert len(set(hs)) == len(set(xs))
    bits = np.array([[(h >> b) & 1 for b in range(32)] for h in hs[:1 << 16]], dtype=np.float64)
    assert np.all(np.abs(bits.mean(axis=0) - 0.5) < 0.01)
    # flipping one input bit flips about half of the output bits
    flips = [bin(oracle.pcg_hash(x) ^ oracle.pcg_hash(x ^ (1 << b))).count("1")
             for x in range(0, 1 << 16, 97) for b in range(32)]
    assert abs(np.mean(flips) - 16.0) < 1.0


def _bf16_neighbours(x):
    b = np.float32(x).view(np.uint32)
    lo = np.uint32(b & np.uint32(0xFFFF0000)).view(np.float32)
    hi = np.uint32((b & np.uint32(0xFFFF0000)) + np.uint32(0x10000)).view(np.float32)
    return float(lo), float(hi)


SAMPLES = [1.0 + 2 ** -9, -3.14159265, 1e-38, 7.5e-41, 2.0 - 2 ** -20, -0.1, 1234.5678,
           float(np.nextafter(np.float32(1.0), np.float32(2.0))), 3.3895e38]


@pytest.mark.parametrize("x", SAMPLES)
def test_rounding_is_unbiased_over_all_random_bits(x):
    """Summed over every 16-bit random value the results equal 2^16 x: the
    expectation of the rounding is x itself (in float64 the sum is exact)."""
    x = float(np.float32(x))
    lo, hi = _bf16_neighbours(x)
    vals = np.array([oracle.round_bf16_sr(x, r) for r in range(1 << 16)], dtype=np.float64)
    assert set(np.unique(vals)) <= {lo, hi}
    assert vals.sum() == 65536.0 * x
    # more random bits never round a value back toward zero
    assert np.all(np.diff(np.abs(vals)) >= 0)
    assert vals[0] == lo    # r = 0: the truncation toward zero


def test_representable_values_are_kept_and_signs_mirror():
    rng = np.random.default_rng(3)
    for _ in range(200):
        x = float(np.float32(rng.standard_normal() * 10.0 ** rng.integers(-30, 30)))
        xb = float(np.uint32(np.float32(x).view(np.uint32) & np.uint32(0xFFFF0000)).view(np.float32))
        r = int(rng.integers(0, 1 << 16))
        assert oracle.round_bf16_sr(xb, r) == xb
        assert oracle.round_bf16_sr(-x, r) == -oracle.round_bf16_sr(x, r)
    assert np.isnan(oracle.round_bf16_sr(float("nan"), 123))
    assert oracle.round_bf16_sr(float("inf"), 65535) == float("inf")


def test_random_bits_take_the_documented_half_of_one_hash_word():
    """Point (i, j, k) at step n takes half i mod 2 of pcg(q xor pcg(n)),
    q = (k ny + j) ceil(nx / 2) + i / 2; the two x points of a pair share one
    word, and steps and points draw different bits."""
    nx, ny, nz = 13, 5, 7
    for (n, i, j, k) in [(0, 0, 0, 0), (3, 12, 4, 6), (17, 5, 2, 3), (1000, 9, 0, 1)]:
        q = (k * ny + j) * ((nx + 1) // 2) + i // 2
        want = (oracle.pcg_hash(q ^ oracle.pcg_hash(n)) >> (16 * (i % 2))) & 0xFFFF
        assert oracle.sr_bits(n, nx, ny, nz, i, j, k) == want
    seen = {oracle.sr_bits(n, nx, ny, nz, i, j, k)
            for n in range(2) for k in range(nz) for j in range(ny) for i in range(nx)}
    assert len(seen) > 0.98 * 2 * nx * ny * nz


def test_stochastically_rounded_run_stores_bf16_values_and_differs_from_nearest():
    """An oracle run with stochastic rounding keeps every u value in bf16, and
    its result is near, but not equal to, the round-to-nearest run."""
    import synth
    shot = synth.config_small_layered(24, 20, 18, 4, 30, seed=11)
    sr = oracle.run_shot(shot, precision="f32", storage="bf16sr")["u"]
    rn = oracle.run_shot(shot, precision="f32", storage="bf16")["u"]
    f64 = oracle.run_shot(shot, precision="f64")["u"]
    assert np.array_equal(sr.view(np.uint32) & np.uint32(0xFFFF), np.zeros_like(sr, dtype=np.uint32))
    assert not np.array_equal(sr, rn)
    rel = lambda a: np.linalg.norm(a - f64) / np.linalg.norm(f64)
    assert rel(sr) < 0.05 and rel(rn) < 0.05
    # the same run again gives the same bits
    assert np.array_equal(sr, oracle.run_shot(shot, precision="f32", storage="bf16sr")["u"])
