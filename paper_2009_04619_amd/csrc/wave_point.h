// wave_point.h -- per-point arithmetic and addressing helpers shared by the
// sweep kernels (one time step per launch in wave_kernels.hip, two in
// wave_kernels2.hip).
//
// Per-point arithmetic (identical in every sweep variant, so results do not
// depend on tiling): float32, explicit fused multiply-adds only where written
// (the library is built with -ffp-contract=off), correctly rounded division:
//   lap = c_xyz * u
//   lap = fma(c_am, u(+m) + u(-m), lap)   axis x, y, z; m = 1..4
//   lap = fma(c_e, u, lap)
// (Eq. 3 in its printed order.  In exact arithmetic c_xyz = -2 sum c_am, so
// a constant field has zero Laplacian; the float weights miss that identity
// by a residual, which would act as a spurious term proportional to u -- a
// frequency shift whose phase error grows with time.  c_e = fl32(-(c_xyz +
// 2 sum c_am)) over the float weights removes it.)
//   inner: u' = u + fma(vp, lap, u - u_prev)
//   layer: t  = fma(-(eta * eta), u, u - u_prev)
//          u' = u + fma(vp, lap + phi, t) / fma(2, eta, 1)
// (Eq. 2 and the layer update rearranged around the increment u - u_prev,
// which a smooth field gives exactly; every small term is then rounded
// relative to its own size and only the final add rounds at the size of u)
//          g  = (de_x * q_x) * (u(+x) - u(-x))
//          g  = fma(de_y * q_y, u(+y) - u(-y), g)
//          g  = fma(de_z * q_z, u(+z) - u(-z), g)
//          phi' = (phi - g) / (1 + eta)
// de_a is eta(+a) - eta(-a) of a per-point eta array (zero beyond the
// faces), or, for the default profile held as per-axis tables,
// fl32(dt (t_a(i+1) - t_a(i-1))): the central difference of a sum of
// one-axis functions along a involves only that axis' term (the tables
// continue the profile one cell past each face).
// The layer form with eta = phi = 0 gives the inner form bit for bit, which
// is the reduction of the damped update to Eq. 2.

#pragma once

#include <type_traits>

#include "wave_internal.h"

namespace wave {
namespace {

// Cache-policy bits of the buffer accesses (gfx950: bit 0 sc0, bit 1 nt,
// bit 4 sc1).  Loads of data read once per sweep (u^{n-1}, vp, phi) and the
// stores of u^{n+1} and phi carry the non-temporal hint, so they do not
// displace the u^n planes that neighbouring tiles and the next z chunk
// re-read from L2 (measured: 2.8 % faster at 512^3, 5.4 % at 1000^3; the
// hint on the loads alone is slower, on the stores alone neutral).
constexpr int kLdOnce = 2;
constexpr int kSt = 2;

// ---- wavefield storage types ------------------------------------------------
struct StF32 {
  using T = float;
  static constexpr bool kSR = false;  // stochastic rounding of u^{n+1} (bf16 only)
  static __device__ __forceinline__ float ld(const T* p, int64_t i) { return p[i]; }
  static __device__ __forceinline__ void st(T* p, int64_t i, float v) { p[i] = v; }
  static __device__ __forceinline__ float cvt(T v) { return v; }
  static __device__ __forceinline__ T enc(float v) { return v; }
  static __device__ __forceinline__ float bld(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, 0));
  }
  static __device__ __forceinline__ float bld1(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, kLdOnce));
  }
  static __device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so,
                                             float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)vo, (int)so, kSt);
  }
};

// float -> bfloat16, round to nearest even: gfx950 converts in one
// instruction (v_cvt_pk_bf16_f32), subnormals included (the library runs
// with float32 denormals enabled).
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  return __builtin_bit_cast(uint16_t, (__bf16)f);
}

// Stochastic rounding of bf16 storage (WAVE_STOCH_ROUND).  The random bits
// come from the "pcg" hash of Jarzynski and Olano ("Hash functions for GPU
// rendering", JCGT 2020): one step of the PCG linear congruential generator
// followed by its RXS-M-XS output permutation (O'Neill 2014), a bijection of
// 32-bit words.  The word of the point pair q = (k ny + j) ceil(nx / 2) +
// floor(i / 2) at step n is pcg(q xor pcg(n)) (q taken modulo 2^32); point i
// takes its 16-bit half i mod 2.  So the bits of a point depend on (n, k, j,
// i) only, never on the tile that computes it.
__host__ __device__ __forceinline__ uint32_t pcg_hash(uint32_t v) {
  const uint32_t state = v * 747796405u + 2891336453u;
  const uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
  return (word >> 22u) ^ word;
}
// word of the pair holding x in row (y, z); key = pcg_hash(step)
__device__ __forceinline__ uint32_t sr_word(uint32_t key, int nx, int ny, int x, int y, int z) {
  const uint32_t q = ((uint32_t)z * (uint32_t)ny + (uint32_t)y) * (uint32_t)((nx + 1) >> 1) +
                     (uint32_t)(x >> 1);
  return pcg_hash(q ^ key);
}

// float -> bfloat16 truncated toward zero and raised by one ulp in magnitude
// when the dropped 16 bits plus the random 16 bits carry; infinities and NaN
// take the round-to-nearest path.
__device__ __forceinline__ uint16_t f32_to_bf16_sr(float f, uint32_t r16) {
  const uint32_t b = __float_as_uint(f);
  if ((b & 0x7F800000u) == 0x7F800000u) return __builtin_bit_cast(uint16_t, (__bf16)f);
  return (uint16_t)((b + (r16 & 0xFFFFu)) >> 16);
}

struct StBF16 {
  using T = uint16_t;
  static constexpr bool kSR = false;
  static __device__ __forceinline__ float ld(const T* p, int64_t i) {
    return __uint_as_float((uint32_t)p[i] << 16);
  }
  static __device__ __forceinline__ void st(T* p, int64_t i, float v) { p[i] = f32_to_bf16_rne(v); }
  static __device__ __forceinline__ float cvt(T v) { return __uint_as_float((uint32_t)v << 16); }
  static __device__ __forceinline__ T enc(float v) { return f32_to_bf16_rne(v); }
  static __device__ __forceinline__ float bld(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    return cvt((uint16_t)__builtin_amdgcn_raw_buffer_load_b16(r, (int)vo, (int)so, 0));
  }
  static __device__ __forceinline__ float bld1(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    return cvt((uint16_t)__builtin_amdgcn_raw_buffer_load_b16(r, (int)vo, (int)so, kLdOnce));
  }
  static __device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so,
                                             float v) {
    __builtin_amdgcn_raw_buffer_store_b16(enc(v), r, (int)vo, (int)so, kSt);
  }
};

// bf16 storage whose sweeps round u^{n+1} stochastically (WAVE_STOCH_ROUND);
// every other access, the source add included, is the bf16 one.
struct StBF16SR : StBF16 {
  static constexpr bool kSR = true;
};

struct StF16 {
  using T = _Float16;
  static constexpr bool kSR = false;
  static __device__ __forceinline__ float ld(const T* p, int64_t i) { return (float)p[i]; }
  static __device__ __forceinline__ void st(T* p, int64_t i, float v) { p[i] = (_Float16)v; }
  static __device__ __forceinline__ float cvt(T v) { return (float)v; }
  static __device__ __forceinline__ T enc(float v) { return (_Float16)v; }
  static __device__ __forceinline__ float bld(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    return cvt(__builtin_bit_cast(
        _Float16, (uint16_t)__builtin_amdgcn_raw_buffer_load_b16(r, (int)vo, (int)so, 0)));
  }
  static __device__ __forceinline__ float bld1(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    return cvt(__builtin_bit_cast(
        _Float16, (uint16_t)__builtin_amdgcn_raw_buffer_load_b16(r, (int)vo, (int)so, kLdOnce)));
  }
  static __device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so,
                                             float v) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, enc(v)), r, (int)vo,
                                          (int)so, kSt);
  }
};

// ---- per-point update ---------------------------------------------------------
__device__ __forceinline__ float upd_inner(float c, float pu, float vp, float lap) {
  return c + __builtin_fmaf(vp, lap, c - pu);
}

__device__ __forceinline__ float upd_layer(float c, float pu, float vp, float lap, float e,
                                           float ph) {
  const float t = __builtin_fmaf(-(e * e), c, c - pu);
  const float num = __builtin_fmaf(vp, lap + ph, t);
  return c + num / __builtin_fmaf(2.0f, e, 1.0f);
}

// phi' from the products dq_a = fl32(de_a * q_a) of the eta differences and
// 1 / (4 h_a^2), and the u differences du_a.
__device__ __forceinline__ float upd_phi(float ph, float e, float dqx, float dux, float dqy,
                                         float duy, float dqz, float duz) {
  float g = dqx * dux;
  g = __builtin_fmaf(dqy, duy, g);
  g = __builtin_fmaf(dqz, duz, g);
  return (ph - g) / (1.0f + e);
}

// Buffer resource over memory starting at p (gfx9 family: stride 0, dword 3 =
// 0x00020000).  Built from a wave-uniform pointer it lives in scalar
// registers; accesses then take an unsigned 32-bit byte offset per lane plus
// a wave-uniform one.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_at(const void* p, uint32_t nbytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)nbytes,
                                           0x00020000);
}
__device__ __forceinline__ float bld_f32(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, 0));
}
__device__ __forceinline__ float bld1_f32(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, kLdOnce));
}
__device__ __forceinline__ void bst_f32(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so,
                                        float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)vo, (int)so, kSt);
}

// Lane offset that is out of range for every eta/phi resource (their range
// is one chunk window, below kWindowMax); nearby offsets (-4, -pitch) stay
// out of range, and adding a window offset cannot wrap 32 bits.
constexpr uint32_t kOOB = 0x80000000u;

// Bytes a chunk window of a float array may span (keeps every in-range offset
// plus kOOB below 2^32 and kOOB out of range).
constexpr int64_t kWindowMax = 0x7FF00000;

__host__ __device__ inline int cdiv(int a, int b) { return (a + b - 1) / b; }

struct ChunkInfo {
  int zb, ze;
  bool cap;  // every point of the chunk is in a z cap of the layer
};

// z chunks: pieces of at most zc planes.  With a layer, the z caps [0, w)
// and [nz-w, nz) and the interior [w, nz-w) are cut separately (a grid with
// 2w >= nz is all cap).
__host__ __device__ inline int chunk_count(int nz, int w, int zc, bool damp) {
  if (!damp || w == 0 || 2 * w >= nz) return cdiv(nz, zc);
  return 2 * cdiv(w, zc) + cdiv(nz - 2 * w, zc);
}
__device__ inline ChunkInfo chunk_of(int ch, int nz, int w, int zc, bool damp) {
  ChunkInfo c;
  if (!damp || w == 0 || 2 * w >= nz) {
    c.zb = ch * zc;
    c.ze = min(c.zb + zc, nz);
    c.cap = damp && w > 0;
    return c;
  }
  const int nc = cdiv(w, zc), ni = cdiv(nz - 2 * w, zc);
  if (ch < nc) {
    c.zb = ch * zc;
    c.ze = min(c.zb + zc, w);
    c.cap = true;
  } else if (ch < nc + ni) {
    c.zb = w + (ch - nc) * zc;
    c.ze = min(c.zb + zc, nz - w);
    c.cap = false;
  } else {
    c.zb = nz - w + (ch - nc - ni) * zc;
    c.ze = min(c.zb + zc, nz);
    c.cap = true;
  }
  return c;
}

// XCD-aware tile order of the streaming sweeps.  Dispatch sends block b to
// XCD b % 8.  The tile rows are padded to 8 slabs of sh = ceil(tiles_y / 8)
// rows (blocks of padding rows exit at once), so every XCD gets the same
// number of blocks.  Each XCD owns a slab of tile rows for every z chunk and
// walks it chunk by chunk: the tiles it runs at once are x and y
// neighbours, so halos come from its L2.  The slab an XCD owns moves on by 3
// (coprime to 8) from one chunk to the next, so the slabs holding the y
// walls of the damping layer, which cost more, are spread over all XCDs
// instead of loading the first and the last.  With hold = h the slab moves
// on only every 2^h chunks, so the warm-up planes a chunk reads below its
// first plane were written to this XCD's L2 by the chunk before (the
// persistent sweep, which walks the chunks of a slab in order, takes h = 1).
// Block b (counted from a multiple of 8) -> tile column tx, tile row ty
// (>= tiles_y: padding), z chunk ch.
struct TileAt {
  int tx, ty, ch;
};
__device__ inline TileAt tile_at(int64_t b, int tiles_x, int tiles_y, int hold = 0) {
  const int xcd = (int)(b & 7);
  const int64_t slot = b >> 3;
  const int sh = (tiles_y + 7) >> 3;
  const int64_t t2 = slot / tiles_x;
  TileAt t;
  t.tx = (int)(slot % tiles_x);
  t.ch = (int)(t2 / sh);
  t.ty = ((xcd + 3 * (t.ch >> hold)) & 7) * sh + (int)(t2 % sh);
  return t;
}

// Member of a batch launch that block b belongs to: the last member whose
// first block is <= b (members' ranges are back to back, in order).
template <class Shot>
__device__ inline int batch_member(const Shot* shots, int nshots, int64_t b) {
  int lo = 0, hi = nshots - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (shots[mid].block_begin <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

}  // namespace
}  // namespace wave
