// wave_kernels.hip -- gfx950 kernels of one time step of the 3-D acoustic
// wave equation (paper Sec. III-A, Eq. 2-3; damping layer after Sec. III-B).
//
// Per-point arithmetic (identical in every sweep variant, so results do not
// depend on tiling): float32, explicit fused multiply-adds only where written
// (the library is built with -ffp-contract=off), correctly rounded division:
//   lap = 0
//   lap = fma(c_am, (u(+m) - u) + (u(-m) - u), lap)   axis x, y, z; m = 1..4
// (Eq. 3 with the centre weight folded into the pairs: c_xyz equals
// -2 sum c_am exactly, and in this form separately rounded float weights
// cannot add a spurious term proportional to u, which would shift the
// frequency and make the phase error grow with time)
//   inner: u' = u + fma(vp, lap, u - u_prev)
//   layer: t  = fma(-(eta * eta), u, u - u_prev)
//          u' = u + fma(vp, lap + phi, t) / fma(2, eta, 1)
// (Eq. 2 and the layer update rearranged around the increment u - u_prev,
// which a smooth field gives exactly; every small term is then rounded
// relative to its own size and only the final add rounds at the size of u)
//          g  = ((eta(+x) - eta(-x)) * q_x) * (u(+x) - u(-x))
//          g  = fma((eta(+y) - eta(-y)) * q_y, u(+y) - u(-y), g)
//          g  = fma((eta(+z) - eta(-z)) * q_z, u(+z) - u(-z), g)
//          phi' = (phi - g) / (1 + eta)
// The layer form with eta = phi = 0 gives the inner form bit for bit, which
// is the reduction of the damped update to Eq. 2.
#include <type_traits>

#include "wave_internal.h"

namespace wave {
namespace {

// ---- wavefield storage types ------------------------------------------------
struct StF32 {
  using T = float;
  static __device__ __forceinline__ float ld(const T* p, int64_t i) { return p[i]; }
  static __device__ __forceinline__ void st(T* p, int64_t i, float v) { p[i] = v; }
  static __device__ __forceinline__ float cvt(T v) { return v; }
  static __device__ __forceinline__ T enc(float v) { return v; }
  static __device__ __forceinline__ float bld(__amdgpu_buffer_rsrc_t r, uint32_t boff) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)boff, 0, 0));
  }
  static __device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, uint32_t boff, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)boff, 0, 0);
  }
};

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

struct StBF16 {
  using T = uint16_t;
  static __device__ __forceinline__ float ld(const T* p, int64_t i) {
    return __uint_as_float((uint32_t)p[i] << 16);
  }
  static __device__ __forceinline__ void st(T* p, int64_t i, float v) { p[i] = f32_to_bf16_rne(v); }
  static __device__ __forceinline__ float cvt(T v) { return __uint_as_float((uint32_t)v << 16); }
  static __device__ __forceinline__ T enc(float v) { return f32_to_bf16_rne(v); }
  static __device__ __forceinline__ float bld(__amdgpu_buffer_rsrc_t r, uint32_t boff) {
    return cvt((uint16_t)__builtin_amdgcn_raw_buffer_load_b16(r, (int)boff, 0, 0));
  }
  static __device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, uint32_t boff, float v) {
    __builtin_amdgcn_raw_buffer_store_b16(enc(v), r, (int)boff, 0, 0);
  }
};

struct StF16 {
  using T = _Float16;
  static __device__ __forceinline__ float ld(const T* p, int64_t i) { return (float)p[i]; }
  static __device__ __forceinline__ void st(T* p, int64_t i, float v) { p[i] = (_Float16)v; }
  static __device__ __forceinline__ float cvt(T v) { return (float)v; }
  static __device__ __forceinline__ T enc(float v) { return (_Float16)v; }
  static __device__ __forceinline__ float bld(__amdgpu_buffer_rsrc_t r, uint32_t boff) {
    return cvt(__builtin_bit_cast(_Float16,
                                  (uint16_t)__builtin_amdgcn_raw_buffer_load_b16(r, (int)boff, 0, 0)));
  }
  static __device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, uint32_t boff, float v) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, enc(v)), r, (int)boff, 0, 0);
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

__device__ __forceinline__ float upd_phi(float ph, float e, float dex, float dux, float dey,
                                         float duy, float dez, float duz, float qx, float qy,
                                         float qz) {
  float g = (dex * qx) * dux;
  g = __builtin_fmaf(dey * qy, duy, g);
  g = __builtin_fmaf(dez * qz, duz, g);
  return (ph - g) / (1.0f + e);
}

// Default damping profile in table mode: eta(x, y, z) = fl32(dt * ((tx[x] +
// ty[y]) + tz[z])) inside the grid, 0 outside (the profile is a sum of three
// per-axis terms; the double operations match the host's).
__device__ __forceinline__ float eta_tab(const SweepArgs& a, int x, int y, int z) {
  if (x < 0 || x >= a.nx || y < 0 || y >= a.ny || z < 0 || z >= a.nz) return 0.0f;
  const double* tx = a.etab + 1;
  const double* ty = tx + a.nx + 2;
  const double* tz = ty + a.ny + 2;
  return (float)(a.dt * ((tx[x] + ty[y]) + tz[z]));
}

__device__ __forceinline__ bool in_layer(const SweepArgs& a, int x, int y, int z) {
  return x < a.w || x >= a.nx - a.w || y < a.w || y >= a.ny - a.w || z < a.w ||
         z >= a.nz - a.w;
}

// ---- variant 0: one thread per point, every operand read from memory -------
template <class S>
__global__ __launch_bounds__(256) void k_sweep_direct(SweepArgs a) {
  using T = typename S::T;
  const int x = blockIdx.x * kTX + threadIdx.x;
  const int y = blockIdx.y * 4 + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= a.nx || y >= a.ny) return;
  const T* u = static_cast<const T*>(a.cur);
  T* un = static_cast<T*>(a.nxt);
  const int64_t P = a.pitch, Q = a.plane;
  const int64_t p = (int64_t)z * Q + (int64_t)y * P + x;
  const float c = S::ld(u, p);
  float lap = 0.0f;
#pragma unroll
  for (int m = 1; m <= kR; ++m)
    lap = __builtin_fmaf(a.c[m], (S::ld(u, p + m) - c) + (S::ld(u, p - m) - c), lap);
#pragma unroll
  for (int m = 1; m <= kR; ++m)
    lap = __builtin_fmaf(a.c[4 + m], (S::ld(u, p + m * P) - c) + (S::ld(u, p - m * P) - c), lap);
#pragma unroll
  for (int m = 1; m <= kR; ++m)
    lap = __builtin_fmaf(a.c[8 + m], (S::ld(u, p + m * Q) - c) + (S::ld(u, p - m * Q) - c), lap);
  const float pu = S::ld(un, p);
  const float vp = a.vp[p];
  float r;
  if (a.damping && in_layer(a, x, y, z)) {
    float e, exm, exp_, eym, eyp, ezm, ezp;
    if (a.etab) {
      e = eta_tab(a, x, y, z);
      exm = eta_tab(a, x - 1, y, z);
      exp_ = eta_tab(a, x + 1, y, z);
      eym = eta_tab(a, x, y - 1, z);
      eyp = eta_tab(a, x, y + 1, z);
      ezm = eta_tab(a, x, y, z - 1);
      ezp = eta_tab(a, x, y, z + 1);
    } else {
      e = a.eta[p];
      exm = a.eta[p - 1];
      exp_ = a.eta[p + 1];
      eym = a.eta[p - P];
      eyp = a.eta[p + P];
      ezm = a.eta[p - Q];
      ezp = a.eta[p + Q];
    }
    const float ph = a.phi[p];
    r = upd_layer(c, pu, vp, lap, e, ph);
    a.phi[p] = upd_phi(ph, e, exp_ - exm, S::ld(u, p + 1) - S::ld(u, p - 1), eyp - eym,
                       S::ld(u, p + P) - S::ld(u, p - P), ezp - ezm,
                       S::ld(u, p + Q) - S::ld(u, p - Q), a.q[0], a.q[1], a.q[2]);
  } else {
    r = upd_inner(c, pu, vp, lap);
  }
  S::st(un, p, r);
}

// ---- variant 1: 2.5-D streaming ------------------------------------------------
// A workgroup of NW wavefronts owns a 64 x TY xy tile (TY = RY * NW; each
// wavefront owns RY rows, one x column per lane) and streams it through the
// planes [zb, ze) of one z chunk.  Per plane:
//  * the 9 z-values u(z-4..z+4) of every owned column sit in registers (a
//    10-slot queue, the 10th slot receives the prefetch of u(z+5));
//  * the centre plane of the tile plus its 4-wide x and y halos is staged in
//    LDS (double-buffered: one barrier per plane), from which the x and y
//    neighbours are read;
//  * every operand of plane z+1 is prefetched while plane z is computed.
// The loop is unrolled by 10 so every queue/buffer index is a compile-time
// constant (no modulo).  Blocks are remapped so that consecutive tiles
// (which share halos) run on the same XCD and its L2.
//
// Damping layer: z chunks are cut at the layer faces (z caps are chunks of
// their own), so whether a lane is a layer point is fixed for a workgroup.
// Workgroups that touch no layer point run a loop without eta/phi.  The
// others issue the eta/phi loads and the phi store unconditionally; a lane
// outside the layer gets an offset beyond the buffer's range, which reads 0
// and writes nothing, so it fetches no bytes, and eta = phi = 0 turns the
// layer update into the inner one bit for bit.  Memory operations are thus
// identical on every path, which keeps the prefetch overlapping the compute.

// Buffer resource over memory starting at p (gfx9 family: stride 0, dword 3 =
// 0x00020000).  Built from a wave-uniform pointer it lives in scalar
// registers; accesses then take an unsigned 32-bit byte offset per lane.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_at(const void* p, uint32_t nbytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)nbytes,
                                           0x00020000);
}
__device__ __forceinline__ float bld_f32(__amdgpu_buffer_rsrc_t r, uint32_t boff) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)boff, 0, 0));
}
__device__ __forceinline__ void bst_f32(__amdgpu_buffer_rsrc_t r, uint32_t boff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)boff, 0, 0);
}

// Offset that is out of range for every eta/phi resource (their range is one
// plane, < 2 GiB); nearby offsets (+-4, +-pitch) stay out of range too.
constexpr uint32_t kOOB = 0xC0000000u;

struct ChunkInfo {
  int zb, ze;
  bool cap;  // every point of the chunk is in a z cap of the layer
};

// z chunks: without a layer, [c*zc, (c+1)*zc); with one, [0, w), then the
// interior [w, nz-w) in pieces of zc, then [nz-w, nz).
__host__ __device__ inline int chunk_count(int nz, int w, int zc, bool damp) {
  if (!damp || w == 0) return (nz + zc - 1) / zc;
  if (2 * w >= nz) return 1;
  return 2 + (nz - 2 * w + zc - 1) / zc;
}
__device__ inline ChunkInfo chunk_of(int ch, int nz, int w, int zc, bool damp) {
  ChunkInfo c;
  if (!damp || w == 0) {
    c.zb = ch * zc;
    c.ze = min(c.zb + zc, nz);
    c.cap = false;
  } else if (2 * w >= nz) {
    c.zb = 0;
    c.ze = nz;
    c.cap = true;
  } else {
    const int nin = (nz - 2 * w + zc - 1) / zc;
    if (ch == 0) {
      c.zb = 0; c.ze = w; c.cap = true;
    } else if (ch == nin + 1) {
      c.zb = nz - w; c.ze = nz; c.cap = true;
    } else {
      c.zb = w + (ch - 1) * zc;
      c.ze = min(c.zb + zc, nz - w);
      c.cap = false;
    }
  }
  return c;
}

// Per-thread slot of a tile: which point it owns and where that point lives.
template <int RY>
struct Slots {
  int x[RY], y[RY];  // grid coordinates of the point
  uint32_t ro[RY];   // in-plane element offset ((y + 4) * pitch + x)
  int ls[RY];        // LDS index of the point in the staged plane
  bool valid[RY];    // inside the grid (else the clamped ghost row/column)
  bool lay[RY];      // a damping-layer point
};

// The streaming loop over planes [zb, ze) for one wavefront's slots.
// EM = 0: no layer point.  EM = 1, 2: the wavefront owns at least one layer
// point and evaluates the layer update for all its points (eta and phi read
// as 0 and phi' dropped for the others, which gives the inner update
// exactly); eta comes from the per-point array (EM = 1) or from the default
// profile's tables (EM = 2, no eta traffic).
template <class S, int RY, int NW, int EM>
__device__ __forceinline__ void stream_loop(const SweepArgs& a,
                                            float (*sm)[(RY * NW + 2 * kR) * (kTX + 2 * kR) + 64],
                                            const Slots<RY>& sl, const int* hl, const uint32_t* ho,
                                            int zb, int ze) {
  using T = typename S::T;
  constexpr int TY = RY * NW;
  constexpr int LW = kTX + 2 * kR;
  constexpr int NT = 64 * NW;
  constexpr int NHALO = 2 * kR * kTX + 2 * kR * TY;
  constexpr int HPT = (NHALO + NT - 1) / NT;
  constexpr uint32_t ES = sizeof(T);
  const int64_t Q = a.plane;
  const int P = a.pitch;
  const uint32_t planeb = (uint32_t)(Q * 4);
  const uint32_t p4 = (uint32_t)P * 4u;
  const int64_t b4 = 4 * (int64_t)P;
  const T* u = static_cast<const T*>(a.cur) - b4;
  T* un = static_cast<T*>(a.nxt) - b4;
  const float* vpa = a.vp - b4;

  constexpr bool LAYER = EM != 0;
  constexpr bool EARR = EM == 1;
  uint32_t eo[RY];   // eta/phi byte offset; out of range for non-layer points
  if (LAYER) {
#pragma unroll
    for (int r = 0; r < RY; ++r) eo[r] = sl.lay[r] ? sl.ro[r] * 4u : kOOB;
  }
  // EM = 2: partial sums of the profile tables that do not depend on z
  // (centre, x-1, x+1, y-1, y+1), and whether x+-1, y+-1 are inside the grid
  double tsc[RY], tsxm[RY], tsxp[RY], tsym[RY], tsyp[RY];
  bool okxm[RY], okxp[RY], okym[RY], okyp[RY];
  const double* tzt = nullptr;
  if (EM == 2) {
    const double* tx = a.etab + 1;
    const double* ty = tx + a.nx + 2;
    tzt = ty + a.ny + 2;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const int x = sl.x[r], y = sl.y[r];
      const double t0 = tx[x], ty0 = ty[y];
      tsc[r] = t0 + ty0;
      tsxm[r] = tx[x - 1] + ty0;
      tsxp[r] = tx[x + 1] + ty0;
      tsym[r] = t0 + ty[y - 1];
      tsyp[r] = t0 + ty[y + 1];
      okxm[r] = x >= 1;
      okxp[r] = x + 1 < a.nx;
      okym[r] = y >= 1;
      okyp[r] = y + 1 < a.ny;
    }
  }

  float q[10][RY];
  float pv[2][RY], vv[2][RY];
  float hh[2][HPT];
  // LAYER: eta of the own column in a 10-slot ring like the u queue (at slot
  // Sl, er[(Sl + j) % 10] holds eta(z - 1 + j), j = 0..2, and slot
  // (Sl + 3) % 10 receives the prefetch of eta(z + 2)); eta x/y neighbours and
  // phi double-buffered by plane parity
  float er[10][RY];
  float ex0[2][RY], ex1[2][RY], ey0[2][RY], ey1[2][RY], ph[2][RY];

  // prologue: planes zb-4 .. zb+4 into queue slots 0..8; plane zb operands
#pragma unroll
  for (int j = 0; j < 2 * kR + 1; ++j) {
    const auto ru = rsrc_at(u + (int64_t)(zb - kR + j) * Q, 0xffffffffu);
#pragma unroll
    for (int r = 0; r < RY; ++r) q[j][r] = S::bld(ru, sl.ro[r] * ES);
  }
  {
    const auto ru = rsrc_at(u + (int64_t)zb * Q, 0xffffffffu);
    const auto rp = rsrc_at(un + (int64_t)zb * Q, 0xffffffffu);
    const auto rv = rsrc_at(vpa + (int64_t)zb * Q, 0xffffffffu);
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      pv[0][r] = S::bld(rp, sl.ro[r] * ES);
      vv[0][r] = bld_f32(rv, sl.ro[r] * 4u);
    }
#pragma unroll
    for (int k = 0; k < HPT; ++k) hh[0][k] = S::bld(ru, ho[k] * ES);
    if (LAYER) {
      const auto rph = rsrc_at(a.phi - b4 + (int64_t)zb * Q, planeb);
#pragma unroll
      for (int r = 0; r < RY; ++r) ph[0][r] = bld_f32(rph, eo[r]);
    }
    if (EARR) {
      const float* e = a.eta - b4 + (int64_t)zb * Q;
      const auto rem = rsrc_at(e - Q, planeb), re0 = rsrc_at(e, planeb), rep = rsrc_at(e + Q, planeb);
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        er[0][r] = bld_f32(rem, eo[r]);
        er[1][r] = bld_f32(re0, eo[r]);
        er[2][r] = bld_f32(rep, eo[r]);
        ex0[0][r] = bld_f32(re0, eo[r] - 4u);
        ex1[0][r] = bld_f32(re0, eo[r] + 4u);
        ey0[0][r] = bld_f32(re0, eo[r] - p4);
        ey1[0][r] = bld_f32(re0, eo[r] + p4);
      }
    }
  }

  auto body = [&](auto SC, const int z) {
    constexpr int Sl = decltype(SC)::value;
    constexpr int B = Sl & 1;        // buffers of this plane
    constexpr int NB = B ^ 1;        // buffers of the next plane
    // prefetch plane z+1 operands and u(z+5), unconditionally so that the
    // number of loads in flight is the same on every path (the last plane
    // clamps to ghost planes, which stay inside the allocation)
    {
      const int z1 = z + 1;                   // <= nz: a ghost plane at most
      const int z5 = min(z + 1 + kR, a.nz + kR - 1);
      const auto ru1 = rsrc_at(u + (int64_t)z1 * Q, 0xffffffffu);
      const auto ru5 = rsrc_at(u + (int64_t)z5 * Q, 0xffffffffu);
      const auto rp1 = rsrc_at(un + (int64_t)z1 * Q, 0xffffffffu);
      const auto rv1 = rsrc_at(vpa + (int64_t)z1 * Q, 0xffffffffu);
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        q[(Sl + 9) % 10][r] = S::bld(ru5, sl.ro[r] * ES);
        pv[NB][r] = S::bld(rp1, sl.ro[r] * ES);
        vv[NB][r] = bld_f32(rv1, sl.ro[r] * 4u);
      }
#pragma unroll
      for (int k = 0; k < HPT; ++k) hh[NB][k] = S::bld(ru1, ho[k] * ES);
      if (LAYER) {
        const auto rph1 = rsrc_at(a.phi - b4 + (int64_t)z1 * Q, planeb);
#pragma unroll
        for (int r = 0; r < RY; ++r) ph[NB][r] = bld_f32(rph1, eo[r]);
      }
      if (EARR) {
        // eta planes z+1 and z+2 (z+2 <= nz: a ghost plane at most)
        const float* e1 = a.eta - b4 + (int64_t)z1 * Q;
        const auto re1 = rsrc_at(e1, planeb), re2 = rsrc_at(e1 + Q, planeb);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
          er[(Sl + 3) % 10][r] = bld_f32(re2, eo[r]);
          ex0[NB][r] = bld_f32(re1, eo[r] - 4u);
          ex1[NB][r] = bld_f32(re1, eo[r] + 4u);
          ey0[NB][r] = bld_f32(re1, eo[r] - p4);
          ey1[NB][r] = bld_f32(re1, eo[r] + p4);
        }
      }
    }
    // stage the centre plane and its halo
    float* s = sm[B];
#pragma unroll
    for (int r = 0; r < RY; ++r) s[sl.ls[r]] = q[(Sl + kR) % 10][r];
#pragma unroll
    for (int k = 0; k < HPT; ++k) s[hl[k]] = hh[B][k];
    __syncthreads();

    const auto rn = rsrc_at(un + (int64_t)z * Q, 0xffffffffu);
    const auto rph = rsrc_at(a.phi - b4 + (int64_t)z * Q, planeb);
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const float* row = s + sl.ls[r];
      const float c = q[(Sl + kR) % 10][r];
      float lap = 0.0f;
#pragma unroll
      for (int m = 1; m <= kR; ++m)
        lap = __builtin_fmaf(a.c[m], (row[m] - c) + (row[-m] - c), lap);
#pragma unroll
      for (int m = 1; m <= kR; ++m)
        lap = __builtin_fmaf(a.c[4 + m], (row[m * LW] - c) + (row[-m * LW] - c), lap);
#pragma unroll
      for (int m = 1; m <= kR; ++m)
        lap = __builtin_fmaf(a.c[8 + m],
                             (q[(Sl + kR + m) % 10][r] - c) + (q[(Sl + kR - m) % 10][r] - c), lap);
      const float pu = pv[B][r];
      const float vp = vv[B][r];
      float res;
      if (LAYER) {
        float e, dex, dey, dez;
        if (EARR) {
          e = er[(Sl + 1) % 10][r];
          dex = ex1[B][r] - ex0[B][r];
          dey = ey1[B][r] - ey0[B][r];
          dez = er[(Sl + 2) % 10][r] - er[Sl % 10][r];
        } else {
          // table mode: eta of the point and of its six neighbours (0 outside
          // the grid); non-layer points read eta = 0 like the array mode's
          // out-of-range loads
          const bool okzm = z >= 1, okzp = z + 1 < a.nz;
          const double tz0 = tzt[z], tzm = tzt[z - 1], tzp = tzt[z + 1];
          const bool ly = sl.lay[r];
          e = ly ? (float)(a.dt * (tsc[r] + tz0)) : 0.0f;
          const float exm = (ly && okxm[r]) ? (float)(a.dt * (tsxm[r] + tz0)) : 0.0f;
          const float exp_ = (ly && okxp[r]) ? (float)(a.dt * (tsxp[r] + tz0)) : 0.0f;
          const float eym = (ly && okym[r]) ? (float)(a.dt * (tsym[r] + tz0)) : 0.0f;
          const float eyp = (ly && okyp[r]) ? (float)(a.dt * (tsyp[r] + tz0)) : 0.0f;
          const float ezm = (ly && okzm) ? (float)(a.dt * (tsc[r] + tzm)) : 0.0f;
          const float ezp = (ly && okzp) ? (float)(a.dt * (tsc[r] + tzp)) : 0.0f;
          dex = exp_ - exm;
          dey = eyp - eym;
          dez = ezp - ezm;
        }
        res = upd_layer(c, pu, vp, lap, e, ph[B][r]);
        const float nph = upd_phi(ph[B][r], e, dex, row[1] - row[-1], dey, row[LW] - row[-LW],
                                  dez, q[(Sl + kR + 1) % 10][r] - q[(Sl + kR - 1) % 10][r],
                                  a.q[0], a.q[1], a.q[2]);
        // stored for every point; points outside the layer have an out-of-
        // range offset, so their store is dropped
        bst_f32(rph, eo[r], nph);
      } else {
        res = upd_inner(c, pu, vp, lap);
      }
      // points past the grid (clamped to ghost cells) write zero there: no
      // branch around the store
      S::bst(rn, sl.ro[r] * ES, sl.valid[r] ? res : 0.0f);
    }
  };

  using std::integral_constant;
  for (int z = zb; z < ze; z += 10) {
    body(integral_constant<int, 0>{}, z);
    if (z + 1 >= ze) break;
    body(integral_constant<int, 1>{}, z + 1);
    if (z + 2 >= ze) break;
    body(integral_constant<int, 2>{}, z + 2);
    if (z + 3 >= ze) break;
    body(integral_constant<int, 3>{}, z + 3);
    if (z + 4 >= ze) break;
    body(integral_constant<int, 4>{}, z + 4);
    if (z + 5 >= ze) break;
    body(integral_constant<int, 5>{}, z + 5);
    if (z + 6 >= ze) break;
    body(integral_constant<int, 6>{}, z + 6);
    if (z + 7 >= ze) break;
    body(integral_constant<int, 7>{}, z + 7);
    if (z + 8 >= ze) break;
    body(integral_constant<int, 8>{}, z + 8);
    if (z + 9 >= ze) break;
    body(integral_constant<int, 9>{}, z + 9);
  }
}

template <class S, int RY, int NW>
__device__ __forceinline__ void stream_tile(const SweepArgs& a,
                                            float (*sm)[(RY * NW + 2 * kR) * (kTX + 2 * kR) + 64],
                                            int x0, int y0, int zb, int ze, bool cap) {
  constexpr int TY = RY * NW;
  constexpr int LW = kTX + 2 * kR;   // LDS row length
  constexpr int LR = TY + 2 * kR;    // LDS rows
  constexpr int NT = 64 * NW;
  constexpr int NYH = 2 * kR * kTX;  // y-halo elements per plane
  constexpr int NHALO = NYH + 2 * kR * TY;
  constexpr int HPT = (NHALO + NT - 1) / NT;

  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int P = a.pitch;
  const int ylast = a.ny + kR - 1;
  const bool damp = a.damping != 0;

  Slots<RY> sl;
  bool any_lay = false;
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int col = lane, row = wv * RY + r;
    const int x = x0 + col, y = y0 + row;
    sl.x[r] = min(x, a.nx - 1);
    sl.y[r] = min(y, a.ny - 1);
    sl.valid[r] = x < a.nx && y < a.ny;
    sl.ro[r] = (uint32_t)((min(y, ylast) + kR) * P + x);
    sl.ls[r] = (kR + row) * LW + kR + col;
    sl.lay[r] = damp && sl.valid[r] &&
                (cap || y < a.w || y >= a.ny - a.w || x < a.w || x >= a.nx - a.w);
    any_lay = any_lay || sl.lay[r];
  }

  // halo bookkeeping: LDS index and in-plane element offset
  int hl[HPT];
  uint32_t ho[HPT];
#pragma unroll
  for (int k = 0; k < HPT; ++k) {
    const int h = threadIdx.x + k * NT;
    int rl, cl, gy, gx;
    if (h < NYH) {
      const int hr = h / kTX, hc = h % kTX;
      rl = (hr < kR) ? hr : TY + hr;
      gy = (hr < kR) ? y0 - kR + hr : y0 + TY + (hr - kR);
      cl = kR + hc;
      gx = x0 + hc;
    } else if (h < NHALO) {
      const int kk = h - NYH;
      const int row = kk / (2 * kR), cc = kk % (2 * kR);
      rl = kR + row;
      gy = y0 + row;
      cl = (cc < kR) ? cc : kTX + cc;
      gx = (cc < kR) ? x0 - kR + cc : x0 + kTX + (cc - kR);
    } else {
      rl = LR;  // dump row
      cl = lane;
      gy = ylast;
      gx = x0 + lane;
    }
    gy = min(gy, ylast);
    hl[k] = rl * LW + cl;
    ho[k] = (uint32_t)((gy + kR) * P + gx);
  }

  // wavefront-uniform choice of the loop
  if (!__any(any_lay))
    stream_loop<S, RY, NW, 0>(a, sm, sl, hl, ho, zb, ze);
  else if (a.etab)
    stream_loop<S, RY, NW, 2>(a, sm, sl, hl, ho, zb, ze);
  else
    stream_loop<S, RY, NW, 1>(a, sm, sl, hl, ho, zb, ze);
}

// Occupancy target in wavefronts per SIMD for one-row tiles.
#ifndef WAVE_STREAM_WAVES_PER_SIMD
#define WAVE_STREAM_WAVES_PER_SIMD 5
#endif
template <class S, int RY, int NW>
__global__ __launch_bounds__(64 * NW, RY == 1 ? WAVE_STREAM_WAVES_PER_SIMD : 2) void k_sweep_stream(
    SweepArgs a, int tiles_x, int tiles_y, int zchunk) {
  constexpr int TY = RY * NW;
  constexpr int LSZ = (TY + 2 * kR) * (kTX + 2 * kR) + 64;  // + a dump row
  __shared__ float sm[2][LSZ];

  // XCD-aware tile order: dispatch sends block b to XCD b % 8; give each XCD
  // a contiguous range of logical tiles.
  const int nb = gridDim.x, bid = blockIdx.x;
  const int per = nb >> 3, rem = nb & 7, xcd = bid & 7, slot = bid >> 3;
  const int logical = (xcd < rem) ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
  const int tx = logical % tiles_x;
  const int t2 = logical / tiles_x;
  const int ty = t2 % tiles_y;
  const int ch = t2 / tiles_y;
  const int x0 = tx * kTX, y0 = ty * TY;
  const bool damp = a.damping != 0;
  const ChunkInfo c = chunk_of(ch, a.nz, a.w, zchunk, damp);
  if (c.zb >= c.ze) return;
  stream_tile<S, RY, NW>(a, sm, x0, y0, c.zb, c.ze, damp && c.cap);
}

// ---- many shots per launch ---------------------------------------------------
// One workgroup grid covers every member of a batch: the workgroup index (after
// the same XCD-aware remap) is located in the members' block ranges, the
// member's parity picks u^n and u^{n-1}, and the tile is swept exactly as in
// a single-shot launch.  Members that have taken their steps for this run exit
// at once, so a captured sequence of launches stays valid as members finish.
template <class S, int RY, int NW>
__global__ __launch_bounds__(64 * NW, RY == 1 ? WAVE_STREAM_WAVES_PER_SIMD : 2) void k_sweep_batch(
    const BatchShot* __restrict__ shots, const BatchState* __restrict__ state, int nshots) {
  constexpr int TY = RY * NW;
  constexpr int LSZ = (TY + 2 * kR) * (kTX + 2 * kR) + 64;
  __shared__ float sm[2][LSZ];
  const int nb = gridDim.x, bid = blockIdx.x;
  const int per = nb >> 3, rem = nb & 7, xcd = bid & 7, slot = bid >> 3;
  const int64_t logical = (xcd < rem) ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
  // member of this workgroup: last member whose first block is <= logical
  int lo = 0, hi = nshots - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (shots[mid].block_begin <= logical) lo = mid; else hi = mid - 1;
  }
  const BatchShot& b = shots[lo];
  const BatchState st = state[lo];
  if (st.done >= b.target) return;
  SweepArgs a = b.sa;
  a.cur = b.u[st.cur];
  a.nxt = b.u[st.cur ^ 1];
  const int64_t local = logical - b.block_begin;
  const int tx = (int)(local % b.tiles_x);
  const int64_t t2 = local / b.tiles_x;
  const int ty = (int)(t2 % b.tiles_y);
  const int ch = (int)(t2 / b.tiles_y);
  const int x0 = tx * kTX, y0 = ty * TY;
  const bool damp = a.damping != 0;
  const ChunkInfo c = chunk_of(ch, a.nz, a.w, b.zchunk, damp);
  if (c.zb >= c.ze) return;
  stream_tile<S, RY, NW>(a, sm, x0, y0, c.zb, c.ze, damp && c.cap);
}

// One workgroup per member: source add, receiver sample, then the member's
// time level advances (rotation = parity flip).
template <class S>
__global__ __launch_bounds__(256) void k_inject_batch(const BatchShot* __restrict__ shots,
                                                      BatchState* __restrict__ state) {
  using T = typename S::T;
  const BatchShot& b = shots[blockIdx.x];
  const BatchState st = state[blockIdx.x];
  if (st.done >= b.target) return;
  const InjectArgs& a = b.inj;
  T* u = static_cast<T*>(b.u[st.cur ^ 1]);
  if (threadIdx.x == 0) {
    for (int s = 0; s < a.nsrc; ++s) {
      const int64_t p = a.src_off[s];
      const float wv = (st.step < a.max_steps) ? a.wavelet[(int64_t)s * a.max_steps + st.step] : 0.0f;
      S::st(u, p, __builtin_fmaf(a.vp[p], wv, S::ld(u, p)));
    }
  }
  __syncthreads();
  if (a.nrec > 0) {
    double* row = a.traces + (int64_t)st.trace_row * a.nrec;
    for (int r = threadIdx.x; r < a.nrec; r += blockDim.x) row[r] = (double)S::ld(u, a.rec_off[r]);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    BatchState ns = st;
    ns.cur ^= 1;
    ns.step += 1;
    ns.done += 1;
    if (a.nrec > 0) ns.trace_row += 1;
    state[blockIdx.x] = ns;
  }
}

// ---- source add and receiver sample (after the sweep, Alg. 1) --------------
template <class S>
__global__ __launch_bounds__(256) void k_inject_record(InjectArgs a) {
  using T = typename S::T;
  T* u = static_cast<T*>(a.u);
  if (threadIdx.x == 0) {
    // sequential so that several sources on one cell add in list order
    for (int s = 0; s < a.nsrc; ++s) {
      const int64_t p = a.src_off[s];
      const float wv = (a.step < a.max_steps) ? a.wavelet[(int64_t)s * a.max_steps + a.step] : 0.0f;
      S::st(u, p, __builtin_fmaf(a.vp[p], wv, S::ld(u, p)));
    }
  }
  __syncthreads();
  if (a.traces) {
    double* row = a.traces + (int64_t)a.trace_row * a.nrec;
    for (int r = threadIdx.x; r < a.nrec; r += blockDim.x) row[r] = (double)S::ld(u, a.rec_off[r]);
  }
}

// ---- float64 energy (check quantity) -----------------------------------------
template <class S>
__global__ __launch_bounds__(256) void k_energy_rows(EnergyArgs a) {
  using T = typename S::T;
  const int y = blockIdx.x, z = blockIdx.y;
  const T* un = static_cast<const T*>(a.cur);
  const T* u = static_cast<const T*>(a.prev);
  const int64_t P = a.pitch, Q = a.plane;
  double kin = 0.0, pot = 0.0;
  for (int x = threadIdx.x; x < a.nx; x += blockDim.x) {
    const int64_t p = (int64_t)z * Q + (int64_t)y * P + x;
    const double vn = S::ld(un, p), v0 = S::ld(u, p);
    const double d = vn - v0;
    kin += d * d / (double)a.vp[p];
    double L = a.c[0] * v0;
    for (int m = 1; m <= kR; ++m) {
      L += a.c[m] * ((double)S::ld(u, p + m) + (double)S::ld(u, p - m));
      L += a.c[4 + m] * ((double)S::ld(u, p + m * P) + (double)S::ld(u, p - m * P));
      L += a.c[8 + m] * ((double)S::ld(u, p + m * Q) + (double)S::ld(u, p - m * Q));
    }
    pot += vn * L;
  }
  __shared__ double sk[256], sp[256];
  sk[threadIdx.x] = kin;
  sp[threadIdx.x] = pot;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      sk[threadIdx.x] += sk[threadIdx.x + h];
      sp[threadIdx.x] += sp[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int64_t row = (int64_t)z * a.ny + y;
    a.partial[2 * row] = sk[0];
    a.partial[2 * row + 1] = sp[0];
  }
}

__global__ __launch_bounds__(1024) void k_energy_final(double* partial, int64_t nrows,
                                                       double* result) {
  __shared__ double sk[1024], sp[1024];
  double kin = 0.0, pot = 0.0;
  for (int64_t r = threadIdx.x; r < nrows; r += blockDim.x) {
    kin += partial[2 * r];
    pot += partial[2 * r + 1];
  }
  sk[threadIdx.x] = kin;
  sp[threadIdx.x] = pot;
  __syncthreads();
  for (int h = 512; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      sk[threadIdx.x] += sk[threadIdx.x + h];
      sp[threadIdx.x] += sp[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    result[0] = sk[0];
    result[1] = sp[0];
  }
}

// ---- plain copy (bandwidth reference) -------------------------------------------
// Each thread moves four 16-byte words, all four loads issued before the
// stores, so every wavefront keeps 4 KB in flight.
__global__ __launch_bounds__(256) void k_stream_copy(const float4* __restrict__ s,
                                                     float4* __restrict__ d, int64_t n) {
  const int64_t base = (int64_t)blockIdx.x * (256 * 4) + threadIdx.x;
  float4 v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t i = base + k * 256;
    if (i < n) v[k] = s[i];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t i = base + k * 256;
    if (i < n) d[i] = v[k];
  }
}

template <class S>
hipError_t sweep_direct_t(const SweepArgs& a, hipStream_t st) {
  dim3 block(kTX, 4, 1);
  dim3 grid((a.nx + kTX - 1) / kTX, (a.ny + 3) / 4, a.nz);
  hipLaunchKernelGGL(k_sweep_direct<S>, grid, block, 0, st, a);
  return hipGetLastError();
}

template <class S, int RY, int NW>
hipError_t sweep_stream_t(const SweepArgs& a, int zchunk, hipStream_t st) {
  constexpr int TY = RY * NW;
  const int tiles_x = (a.nx + kTX - 1) / kTX;
  const int tiles_y = (a.ny + TY - 1) / TY;
  const int chunks = chunk_count(a.nz, a.w, zchunk, a.damping != 0);
  const int64_t blocks = (int64_t)tiles_x * tiles_y * chunks;
  if (blocks <= 0 || blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_sweep_stream<S, RY, NW>), dim3((unsigned)blocks), dim3(64 * NW), 0, st, a,
                     tiles_x, tiles_y, zchunk);
  return hipGetLastError();
}

template <class S>
hipError_t sweep_stream_s(const SweepArgs& a, int ry, int nw, int zchunk, hipStream_t st) {
  if (ry == 1 && nw == 16) return sweep_stream_t<S, 1, 16>(a, zchunk, st);
  if (ry == 1 && nw == 8) return sweep_stream_t<S, 1, 8>(a, zchunk, st);
  if (ry == 2 && nw == 8) return sweep_stream_t<S, 2, 8>(a, zchunk, st);
  if (ry == 2 && nw == 4) return sweep_stream_t<S, 2, 4>(a, zchunk, st);
  return hipErrorInvalidValue;
}

}  // namespace

bool stream_config_supported(int ry, int nw) {
  return (ry == 1 && nw == 16) || (ry == 1 && nw == 8) || (ry == 2 && nw == 8) ||
         (ry == 2 && nw == 4);
}

int auto_zchunk(int nx, int ny, int nz, int ry, int nw) {
  // enough workgroups to give every CU several (256 CUs), but chunks long
  // enough that the 8-plane queue warm-up stays a small overhead
  const int64_t tiles = (int64_t)((nx + kTX - 1) / kTX) * ((ny + ry * nw - 1) / (ry * nw));
  int64_t chunks = (2048 + tiles - 1) / tiles;
  if (chunks < 1) chunks = 1;
  int zc = (int)((nz + chunks - 1) / chunks);
  const int minz = nz < 32 ? nz : 32;
  if (zc < minz) zc = minz;
  return zc;
}

hipError_t launch_sweep_direct(const SweepArgs& a, int storage, hipStream_t s) {
  switch (storage) {
    case 0: return sweep_direct_t<StF32>(a, s);
    case 1: return sweep_direct_t<StBF16>(a, s);
    case 2: return sweep_direct_t<StF16>(a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sweep_stream(const SweepArgs& a, int storage, int ry, int nw, int zchunk,
                               hipStream_t s) {
  if (zchunk <= 0) return hipErrorInvalidValue;
  switch (storage) {
    case 0: return sweep_stream_s<StF32>(a, ry, nw, zchunk, s);
    case 1: return sweep_stream_s<StBF16>(a, ry, nw, zchunk, s);
    case 2: return sweep_stream_s<StF16>(a, ry, nw, zchunk, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_inject_record(const InjectArgs& a, int storage, hipStream_t s) {
  switch (storage) {
    case 0: hipLaunchKernelGGL(k_inject_record<StF32>, dim3(1), dim3(256), 0, s, a); break;
    case 1: hipLaunchKernelGGL(k_inject_record<StBF16>, dim3(1), dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_inject_record<StF16>, dim3(1), dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_energy(const EnergyArgs& a, int storage, hipStream_t s) {
  dim3 grid(a.ny, a.nz);
  switch (storage) {
    case 0: hipLaunchKernelGGL(k_energy_rows<StF32>, grid, dim3(256), 0, s, a); break;
    case 1: hipLaunchKernelGGL(k_energy_rows<StBF16>, grid, dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_energy_rows<StF16>, grid, dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(1024), 0, s, a.partial,
                     (int64_t)a.ny * a.nz, a.result);
  return hipGetLastError();
}

hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const int64_t n = (int64_t)(bytes / 16);
  if (n == 0) return hipSuccess;
  const int64_t blocks = (n + 1023) / 1024;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, s,
                     static_cast<const float4*>(src), static_cast<float4*>(dst), n);
  return hipGetLastError();
}

int stream_chunk_count(int nz, int w, int zchunk, bool damping) {
  return chunk_count(nz, w, zchunk, damping);
}

int stream_tiles_y(int ny, int ry, int nw) { return (ny + ry * nw - 1) / (ry * nw); }

template <class S>
hipError_t sweep_batch_s(const BatchShot* shots, BatchState* state, int nshots, int64_t blocks,
                         int ry, int nw, hipStream_t st) {
  if (blocks <= 0 || blocks > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 g((unsigned)blocks);
#define WAVE_BATCH_CASE(RY_, NW_)                                                             \
  if (ry == RY_ && nw == NW_) {                                                               \
    hipLaunchKernelGGL((k_sweep_batch<S, RY_, NW_>), g, dim3(64 * NW_), 0, st, shots, state, \
                       nshots);                                                               \
    return hipGetLastError();                                                                 \
  }
  WAVE_BATCH_CASE(1, 16)
  WAVE_BATCH_CASE(1, 8)
  WAVE_BATCH_CASE(2, 8)
  WAVE_BATCH_CASE(2, 4)
#undef WAVE_BATCH_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_sweep_batch(const BatchShot* shots, BatchState* state, int nshots,
                              int64_t total_blocks, int storage, int ry, int nw, hipStream_t s) {
  switch (storage) {
    case 0: return sweep_batch_s<StF32>(shots, state, nshots, total_blocks, ry, nw, s);
    case 1: return sweep_batch_s<StBF16>(shots, state, nshots, total_blocks, ry, nw, s);
    case 2: return sweep_batch_s<StF16>(shots, state, nshots, total_blocks, ry, nw, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_inject_batch(const BatchShot* shots, BatchState* state, int nshots, int storage,
                               hipStream_t s) {
  if (nshots <= 0) return hipSuccess;
  switch (storage) {
    case 0: hipLaunchKernelGGL(k_inject_batch<StF32>, dim3(nshots), dim3(256), 0, s, shots, state); break;
    case 1: hipLaunchKernelGGL(k_inject_batch<StBF16>, dim3(nshots), dim3(256), 0, s, shots, state); break;
    case 2: hipLaunchKernelGGL(k_inject_batch<StF16>, dim3(nshots), dim3(256), 0, s, shots, state); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace wave

