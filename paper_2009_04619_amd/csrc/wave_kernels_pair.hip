// wave_kernels_pair.hip -- the 2.5-D streaming sweep with two x-adjacent
// points per lane (paper Eq. 2-3 and the damping layer of Sec. III-B; the
// per-point arithmetic is wave_point.h's, operand for operand).
//
// A wavefront covers 128 x points of one row: lane l owns x0 + 2l and
// x0 + 2l + 1.  Every global access of a lane moves the pair at once (a
// 32-bit word of two 16-bit values, or 64 bits of two floats), and the x and
// y neighbours of the pair come from LDS as 64-bit words, so a point costs
// about half the memory and LDS instructions of the one-point kernel.  This
// matters where the one-point loop runs short of instruction issue rather
// than of bandwidth (16-bit storage moves fewer bytes per instruction).
//
// Structure as in k_sweep_stream: a 128 x TY tile (one row per wavefront, or
// two half rows where the tile holds an x wall of the layer)
// streamed through a z chunk, u(z-4..z+4) of the own pair in a register ring
// with 3 more planes requested ahead, the centre plane and its 4-cell halo
// staged in double-buffered LDS (one barrier per plane), operands of plane
// z+3 requested while plane z computes, tile rows padded to 8 slabs that
// rotate over the XCDs per chunk.  The default profile's tables only (no
// eta array).
#include <algorithm>

#include "wave_internal.h"
#include "wave_point.h"

namespace wave {
namespace {

constexpr int kPX = 2 * kTX;               // x points per wavefront / tile
constexpr int kPW = kPX + 2 * kR;          // staged row length (floats)
constexpr int kPPD = 3;                    // planes requested ahead
constexpr int kPL = 2 * kR + 1 + kPPD;     // u ring length = unroll length
constexpr int kPNR = kPPD + 1;             // operand ring length
static_assert(kPL % kPNR == 0 && kPL % 2 == 0, "ring lengths must divide the unroll");
constexpr uint32_t kPairGhost = 0xffffffffu;

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef const double __attribute__((address_space(4))) PCDouble;
typedef const float __attribute__((address_space(4))) PCFloat;

// pair access per storage type: load two values (byte offset of the first),
// store two values
template <class S> struct PairIO;
template <> struct PairIO<StF32> {
  static __device__ __forceinline__ f32x2 ld(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, 0);
    return f32x2{__uint_as_float(v[0]), __uint_as_float(v[1])};
  }
  static __device__ __forceinline__ f32x2 ld1(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, kLdOnce);
    return f32x2{__uint_as_float(v[0]), __uint_as_float(v[1])};
  }
  static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so,
                                            float a, float b) {
    __builtin_amdgcn_raw_buffer_store_b64(u32x2{__float_as_uint(a), __float_as_uint(b)}, r,
                                          (int)vo, (int)so, kSt);
  }
};
template <> struct PairIO<StBF16> {
  static __device__ __forceinline__ f32x2 unpack(uint32_t v) {
    return f32x2{__uint_as_float(v << 16), __uint_as_float(v & 0xffff0000u)};
  }
  static __device__ __forceinline__ f32x2 ld(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    return unpack(__builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, 0));
  }
  static __device__ __forceinline__ f32x2 ld1(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    return unpack(__builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, kLdOnce));
  }
  static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so,
                                            float a, float b) {
    const uint32_t v = (uint32_t)StBF16::enc(a) | ((uint32_t)StBF16::enc(b) << 16);
    __builtin_amdgcn_raw_buffer_store_b32(v, r, (int)vo, (int)so, kSt);
  }
};
template <> struct PairIO<StBF16SR> : PairIO<StBF16> {};
template <> struct PairIO<StF16> {
  static __device__ __forceinline__ f32x2 unpack(uint32_t v) {
    return f32x2{(float)__builtin_bit_cast(_Float16, (uint16_t)(v & 0xffffu)),
                 (float)__builtin_bit_cast(_Float16, (uint16_t)(v >> 16))};
  }
  static __device__ __forceinline__ f32x2 ld(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    return unpack(__builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, 0));
  }
  static __device__ __forceinline__ f32x2 ld1(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    return unpack(__builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, kLdOnce));
  }
  static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so,
                                            float a, float b) {
    const uint32_t v = (uint32_t)__builtin_bit_cast(uint16_t, StF16::enc(a)) |
                       ((uint32_t)__builtin_bit_cast(uint16_t, StF16::enc(b)) << 16);
    __builtin_amdgcn_raw_buffer_store_b32(v, r, (int)vo, (int)so, kSt);
  }
};

__device__ __forceinline__ f32x2 ld_f32x2(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so,
                                          bool once) {
  const u32x2 v = once ? __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, kLdOnce)
                       : __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, 0);
  return f32x2{__uint_as_float(v[0]), __uint_as_float(v[1])};
}

// One wavefront's pair of points: coordinates and per-point flags.
struct PairSlot {
  int x, y;            // grid coordinates of the first point (clamped into the grid)
  uint32_t ro;         // in-plane element offset of the first point
  int ls;              // LDS index of the first point in the staged plane
  bool inrow;          // the pair lies inside the padded row (x + 1 < pitch)
  bool valid[2];       // inside the grid
  bool lay[2];         // damping-layer point
  bool phl[2];         // phi read and written back (layer, or on an x-wall line)
};

template <class S, int TY, int EM>
__device__ __forceinline__ void pair_loop(const SweepArgs& a, float (*sm)[(TY + 2 * kR) * kPW + 128],
                                          const PairSlot& sl, const int* hl, const uint32_t* ho,
                                          int zb, int ze) {
  using T = typename S::T;
  using IO = PairIO<S>;
  constexpr int NT = 64 * TY;
  constexpr int NHP = (2 * kR * kPX + 2 * kR * TY) / 2;   // halo pairs per plane
  constexpr int HPT = (NHP + NT - 1) / NT;
  constexpr uint32_t ES = sizeof(T);
  constexpr int PD = kPPD, L = kPL, NR = kPNR;
  constexpr bool LAYER = EM != 0;

  const int64_t Q = a.plane;
  const int P = a.pitch;
  const uint32_t pe = (uint32_t)Q * ES, p4 = (uint32_t)Q * 4u;
  const int64_t w0 = (int64_t)(zb - kR) * Q - (int64_t)kR * P;
  const uint32_t wlen = (uint32_t)(ze - zb + 2 * kR) * p4;
  const int zlast = ze - zb + kR - 1;
  // every resource spans the chunk's window, so an out-of-range offset
  // (kOOB) reads 0 and drops stores
  const uint32_t wlen_e = (uint32_t)(ze - zb + 2 * kR) * pe;
  const auto ru = rsrc_at(static_cast<const T*>(a.cur) + w0, wlen_e);
  const auto rn = rsrc_at(static_cast<T*>(a.nxt) + w0, wlen_e);
  const auto rv = rsrc_at(a.vp + w0, wlen);
  const auto rph = rsrc_at(LAYER ? (const void*)(a.phi + w0) : nullptr, LAYER ? wlen : 0u);

  // a pair past the grid (in the row padding, beyond the padded row, or on
  // a row clamped to the ghost row) touches nothing: its offsets are out of
  // range, so it reads zeros, the ghost values, and stores nothing (padding
  // and ghosts stay as the set-up zeroed them).  A pair whose second point
  // is the first ghost column still stores that point's 0.
  const bool live = sl.inrow && sl.valid[0];
  const uint32_t vo = live ? sl.ro * ES : kOOB, vo4 = live ? sl.ro * 4u : kOOB;
  uint32_t hoe[HPT];
#pragma unroll
  for (int k = 0; k < HPT; ++k) hoe[k] = ho[k] == kPairGhost ? kOOB : ho[k] * ES;
  const uint32_t fo = (LAYER && sl.inrow && (sl.phl[0] || sl.phl[1])) ? vo4 : kOOB;

  double tsc[2] = {0.0, 0.0};
  float dqx[2] = {0.0f, 0.0f}, dqy = 0.0f;
  const PCDouble* tzt = nullptr;
  const PCFloat* dqzt = nullptr;
  if (EM == 2) {
    const double* tx = a.etab + 1;
    const double* ty = tx + a.nx + 2;
    tzt = (const PCDouble*)(ty + a.ny + 2);
    dqzt = (const PCFloat*)(a.etq + a.nx + a.ny);
    const int x1 = min(sl.x + 1, a.nx - 1);
    tsc[0] = tx[sl.x] + ty[sl.y];
    tsc[1] = tx[x1] + ty[sl.y];
    dqx[0] = a.etq[sl.x];
    dqx[1] = a.etq[x1];
    dqy = a.etq[a.nx + sl.y];
  }

  f32x2 q[L];
  f32x2 pv[NR], vv[NR], ph[NR];
  f32x2 hh[NR][HPT];
  double tzr[NR];
  float dzr[NR];

#pragma unroll
  for (int j = 0; j < L - 1; ++j) q[j] = IO::ld(ru, vo, (uint32_t)min(j, zlast + kR) * pe);
#pragma unroll
  for (int j = 0; j < PD; ++j) {
    const uint32_t kp = (uint32_t)min(j + kR, zlast);
    const uint32_t se = kp * pe, s4 = kp * p4;
    pv[j] = IO::ld1(rn, vo, se);
    vv[j] = ld_f32x2(rv, vo4, s4, true);
#pragma unroll
    for (int k = 0; k < HPT; ++k) hh[j][k] = IO::ld(ru, hoe[k], se);
    if (LAYER) ph[j] = ld_f32x2(rph, fo, s4, true);
    if (EM == 2) {
      const int zt = zb - kR + (int)kp;
      tzr[j] = tzt[zt];
      dzr[j] = dqzt[zt];
    }
  }

  auto body = [&](auto SC, const int z) {
    constexpr int Sl = decltype(SC)::value;
    constexpr int B = Sl % NR, BP = (Sl + PD) % NR, LB = Sl & 1;
    const int kz = z - zb + kR;
    {
      const uint32_t kp = (uint32_t)min(kz + PD, zlast);
      const uint32_t se = kp * pe, s4 = kp * p4;
      q[(Sl + L - 1) % L] = IO::ld(ru, vo, se + 4u * pe);
      pv[BP] = IO::ld1(rn, vo, se);
      vv[BP] = ld_f32x2(rv, vo4, s4, true);
#pragma unroll
      for (int k = 0; k < HPT; ++k) hh[BP][k] = IO::ld(ru, hoe[k], se);
      if (LAYER) ph[BP] = ld_f32x2(rph, fo, s4, true);
      if (EM == 2) {
        const int zt = zb - kR + (int)kp;
        tzr[BP] = tzt[zt];
        dzr[BP] = dqzt[zt];
      }
    }
    float* s = sm[LB];
    *reinterpret_cast<f32x2*>(s + sl.ls) = q[(Sl + kR) % L];
#pragma unroll
    for (int k = 0; k < HPT; ++k) *reinterpret_cast<f32x2*>(s + hl[k]) = hh[B][k];
    __syncthreads();

    // neighbours of the pair from LDS as 64-bit words: x from columns
    // ls-4 .. ls+5, y from rows +-1..4 at the pair's columns
    const float* row = s + sl.ls;
    const f32x2 xm4 = *reinterpret_cast<const f32x2*>(row - 4);
    const f32x2 xm2 = *reinterpret_cast<const f32x2*>(row - 2);
    const f32x2 xp2 = *reinterpret_cast<const f32x2*>(row + 2);
    const f32x2 xp4 = *reinterpret_cast<const f32x2*>(row + 4);
    const float xv[10] = {xm4[0], xm4[1], xm2[0], xm2[1], 0.0f, 0.0f, xp2[0], xp2[1], xp4[0], xp4[1]};
    f32x2 ym[kR], yp[kR];
#pragma unroll
    for (int m = 1; m <= kR; ++m) {
      ym[m - 1] = *reinterpret_cast<const f32x2*>(row - m * kPW);
      yp[m - 1] = *reinterpret_cast<const f32x2*>(row + m * kPW);
    }
    const f32x2 cc = q[(Sl + kR) % L];
    const uint32_t sz = (uint32_t)kz * pe, sz4 = (uint32_t)kz * p4;
    float res[2], nph[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      // x neighbour at offset d of point i: xv[4 + i + d] (the centre pair
      // occupies slots 4, 5 and is not needed there)
      auto xn = [&](int d) { return (i + d == 0) ? cc[0] : (i + d == 1) ? cc[1] : xv[4 + i + d]; };
      const float c = cc[i];
      float lap = a.c[0] * c;
#pragma unroll
      for (int m = 1; m <= kR; ++m) lap = __builtin_fmaf(a.c[m], xn(m) + xn(-m), lap);
#pragma unroll
      for (int m = 1; m <= kR; ++m) lap = __builtin_fmaf(a.c[4 + m], yp[m - 1][i] + ym[m - 1][i], lap);
#pragma unroll
      for (int m = 1; m <= kR; ++m)
        lap = __builtin_fmaf(a.c[8 + m], q[(Sl + kR + m) % L][i] + q[(Sl + kR - m) % L][i], lap);
      lap = __builtin_fmaf(a.ce, c, lap);
      const float pu = pv[B][i], vp = vv[B][i];
      if (LAYER) {
        const float e = sl.lay[i] ? (float)(a.dt * (tsc[i] + tzr[B])) : 0.0f;
        const float phv = sl.lay[i] ? ph[B][i] : 0.0f;
        res[i] = upd_layer(c, pu, vp, lap, e, phv);
        const float g = upd_phi(phv, e, dqx[i], xn(1) - xn(-1), dqy, yp[0][i] - ym[0][i], dzr[B],
                                q[(Sl + kR + 1) % L][i] - q[(Sl + kR - 1) % L][i]);
        nph[i] = sl.lay[i] ? g : ph[B][i];
      } else {
        res[i] = upd_inner(c, pu, vp, lap);
      }
      res[i] = sl.valid[i] ? res[i] : 0.0f;
    }
    if (LAYER) {
      const u32x2 pw{__float_as_uint(nph[0]), __float_as_uint(nph[1])};
      __builtin_amdgcn_raw_buffer_store_b64(pw, rph, (int)fo, (int)sz4, kSt);
    }
    if constexpr (S::kSR) {  // stochastic rounding of bf16 storage (WAVE_STOCH_ROUND);
                             // x is even, so both points take their bits from one word
      const uint32_t wd = sr_word(pcg_hash((uint32_t)a.step), a.nx, a.ny, sl.x, sl.y, z);
      const uint32_t lo = f32_to_bf16_sr(res[0], wd);
      const uint32_t hi = f32_to_bf16_sr(res[1], wd >> 16);
      __builtin_amdgcn_raw_buffer_store_b32(lo | (hi << 16), rn, (int)vo, (int)sz, kSt);
    } else {
      IO::st(rn, vo, sz, res[0], res[1]);
    }
  };

  using std::integral_constant;
  static_assert(L == 12, "unrolled loop below covers ring length 12");
  for (int z = zb; z < ze; z += L) {
#define WAVE_PAIR_BODY(J)                              \
    if ((J) > 0 && z + (J) >= ze) break;               \
    body(integral_constant<int, (J)>{}, z + (J));
    WAVE_PAIR_BODY(0) WAVE_PAIR_BODY(1) WAVE_PAIR_BODY(2) WAVE_PAIR_BODY(3)
    WAVE_PAIR_BODY(4) WAVE_PAIR_BODY(5) WAVE_PAIR_BODY(6) WAVE_PAIR_BODY(7)
    WAVE_PAIR_BODY(8) WAVE_PAIR_BODY(9) WAVE_PAIR_BODY(10) WAVE_PAIR_BODY(11)
#undef WAVE_PAIR_BODY
  }
}

// Sweep of the 128 x TY tile at (x0, y0) through planes [zb, ze); `cap`: the
// chunk is a z cap of the damping layer.
template <class S, int TY>
__device__ __forceinline__ void pair_tile(const SweepArgs& a, float (*sm)[(TY + 2 * kR) * kPW + 128],
                                          int x0, int y0, int zb, int ze, bool cap) {
  constexpr int LR = TY + 2 * kR;
  constexpr int NT = 64 * TY;
  constexpr int NHP = (2 * kR * kPX + 2 * kR * TY) / 2;
  constexpr int HPT = (NHP + NT - 1) / NT;
  const bool damp = a.damping != 0;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int P = a.pitch;
  const int ylast = a.ny + kR - 1;

  // A tile that holds an x wall of the layer lays its lanes out as 64
  // columns (32 pairs) x 2 rows per wavefront, the first TY/2 wavefronts on
  // the left half of the tile and the others on the right half, so a wall of
  // up to 64 cells lands in half the wavefronts and the rest run the inner
  // loop; other tiles keep one 128-column row per wavefront.
  const bool split = (TY % 2 == 0) && damp && !cap && a.w > 0 &&
                     (x0 < a.w || x0 + kPX > a.nx - a.w);
  constexpr int HW = TY / 2;
  const int col = split ? (wv / HW) * (kPX / 2) + 2 * (lane & 31) : 2 * lane;
  const int row = split ? (wv % HW) * 2 + (lane >> 5) : wv;
  PairSlot sl;
  bool any_lay = false;
  {
    const int x = x0 + col, y = y0 + row;
    sl.x = min(x, a.nx - 1);
    sl.y = min(y, a.ny - 1);
    sl.inrow = x + 1 < P;
    sl.ro = (uint32_t)((min(y, ylast) + kR) * P + min(x, P - 2));
    sl.ls = (kR + row) * kPW + kR + col;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int xi = x + i;
      sl.valid[i] = xi < a.nx && y < a.ny;
      sl.lay[i] = damp && sl.valid[i] &&
                  (cap || y < a.w || y >= a.ny - a.w || xi < a.w || xi >= a.nx - a.w);
      sl.phl[i] = sl.lay[i] || (damp && sl.valid[i] && a.w > 0 &&
                                (xi < ((a.w + 31) & ~31) || xi >= ((a.nx - a.w) & ~31)));
      any_lay = any_lay || sl.lay[i];
    }
  }

  // halo pairs: the 4 rows above and below (64 pairs each), then the 4
  // columns left and right of every tile row (2 pairs each side)
  int hl[HPT];
  uint32_t ho[HPT];
#pragma unroll
  for (int k = 0; k < HPT; ++k) {
    const int h = threadIdx.x + k * NT;
    int rl, cl, gy, gx;
    if (h < 2 * kR * (kPX / 2)) {
      const int hr = h / (kPX / 2), hp = h % (kPX / 2);
      rl = (hr < kR) ? hr : TY + hr;
      gy = (hr < kR) ? y0 - kR + hr : y0 + TY + (hr - kR);
      cl = kR + 2 * hp;
      gx = x0 + 2 * hp;
    } else if (h < NHP) {
      const int kk = h - 2 * kR * (kPX / 2);
      const int rr = kk / 4, pp = kk % 4;
      rl = kR + rr;
      gy = y0 + rr;
      cl = (pp < 2) ? 2 * pp : kPX + kR + 2 * (pp - 2);
      gx = (pp < 2) ? x0 - kR + 2 * pp : x0 + kPX + 2 * (pp - 2);
    } else {
      rl = LR;  // dump area
      cl = 2 * lane;
      gy = ylast;
      gx = x0;
    }
    const bool ghost = h >= NHP || gx >= a.nx || gx + 1 < 0 || gy < 0 || gy >= a.ny;
    gy = min(gy, ylast);
    hl[k] = rl * kPW + cl;
    ho[k] = ghost ? kPairGhost : (uint32_t)((gy + kR) * P + gx);
  }

  if (!__any(any_lay))
    pair_loop<S, TY, 0>(a, sm, sl, hl, ho, zb, ze);
  else
    pair_loop<S, TY, 2>(a, sm, sl, hl, ho, zb, ze);
}


template <class S, int TY>
__global__ __launch_bounds__(64 * TY) void k_sweep_pair(SweepArgs a, int tiles_x, int tiles_y,
                                                      int zchunk) {
  constexpr int LR = TY + 2 * kR;
  // staged plane plus a dump area of 128 floats for the threads without a
  // halo pair
  __shared__ __attribute__((aligned(16))) float sm[2][LR * kPW + 128];

  // tile order as in k_sweep_stream (tile_at)
  const TileAt t = tile_at(blockIdx.x, tiles_x, tiles_y);
  if (t.ty >= tiles_y) return;
  const bool damp = a.damping != 0;
  const ChunkInfo c = chunk_of(t.ch, a.nz, a.w, zchunk, damp);
  if (c.zb >= c.ze) return;
  pair_tile<S, TY>(a, sm, t.tx * kPX, t.ty * TY, c.zb, c.ze, damp && c.cap);
}

// Batch: one grid over the members' block ranges (each a multiple of 8
// blocks, padded slabs of 128 x TY tiles), as k_sweep_batch.
template <class S, int TY>
__global__ __launch_bounds__(64 * TY) void k_sweep_batch_pair(const BatchShot* __restrict__ shots,
                                                            const BatchState* __restrict__ state,
                                                            int nshots) {
  constexpr int LR = TY + 2 * kR;
  __shared__ __attribute__((aligned(16))) float sm[2][LR * kPW + 128];
  const int64_t bid = blockIdx.x;
  const int m = batch_member(shots, nshots, bid);
  const BatchShot& b = shots[m];
  const BatchState st = state[m];
  if (st.done >= b.target) return;
  SweepArgs a = b.sa;
  a.cur = b.u[st.cur];
  a.nxt = b.u[st.cur ^ 1];
  a.step = st.step;
  const TileAt t = tile_at(bid - b.block_begin, b.tiles_x, b.tiles_y);
  if (t.ty >= b.tiles_y) return;
  const bool damp = a.damping != 0;
  const ChunkInfo c = chunk_of(t.ch, a.nz, a.w, b.zchunk, damp);
  if (c.zb >= c.ze) return;
  pair_tile<S, TY>(a, sm, t.tx * kPX, t.ty * TY, c.zb, c.ze, damp && c.cap);
}

template <class S, int TY>
hipError_t pair_t(const SweepArgs& a, int zchunk, hipStream_t st) {
  const int tiles_x = (a.nx + kPX - 1) / kPX;
  const int tiles_y = (a.ny + TY - 1) / TY;
  if (zchunk <= 0 || zchunk > stream_zchunk_limit(a.plane)) return hipErrorInvalidValue;
  const int chunks = chunk_count(a.nz, a.w, zchunk, a.damping != 0);
  const int64_t blocks = (int64_t)tiles_x * 8 * ((tiles_y + 7) / 8) * chunks;
  if (blocks <= 0 || blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_sweep_pair<S, TY>), dim3((unsigned)blocks), dim3(64 * TY), 0, st, a,
                     tiles_x, tiles_y, zchunk);
  return hipGetLastError();
}

template <class S>
hipError_t pair_s(const SweepArgs& a, int ty, int zchunk, hipStream_t st) {
  if (ty == 8) return pair_t<S, 8>(a, zchunk, st);
  if (ty == 16) return pair_t<S, 16>(a, zchunk, st);
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_sweep_batch_pair(const BatchShot* shots, BatchState* state, int nshots,
                                   int64_t total_blocks, int storage, int ty, hipStream_t s) {
  if (total_blocks <= 0 || total_blocks > 0x7fffffff || (ty != 8 && ty != 16))
    return hipErrorInvalidValue;
  const dim3 g((unsigned)total_blocks);
#define WAVE_BATCH_PAIR(S_, T_)                                                                \
  hipLaunchKernelGGL((k_sweep_batch_pair<S_, T_>), g, dim3(64 * T_), 0, s, shots, state, nshots); \
  return hipGetLastError();
  switch (storage) {
    case 0: if (ty == 8) { WAVE_BATCH_PAIR(StF32, 8) } else { WAVE_BATCH_PAIR(StF32, 16) }
    case 1: if (ty == 8) { WAVE_BATCH_PAIR(StBF16, 8) } else { WAVE_BATCH_PAIR(StBF16, 16) }
    case 2: if (ty == 8) { WAVE_BATCH_PAIR(StF16, 8) } else { WAVE_BATCH_PAIR(StF16, 16) }
    case 3: if (ty == 8) { WAVE_BATCH_PAIR(StBF16SR, 8) } else { WAVE_BATCH_PAIR(StBF16SR, 16) }
  }
#undef WAVE_BATCH_PAIR
  return hipErrorInvalidValue;
}

hipError_t launch_sweep_pair(const SweepArgs& a, int storage, int ty, int zchunk, hipStream_t s) {
  if (a.damping && !a.etab) return hipErrorInvalidValue;   // eta arrays: not in this kernel
  switch (storage) {
    case 0: return pair_s<StF32>(a, ty, zchunk, s);
    case 1: return pair_s<StBF16>(a, ty, zchunk, s);
    case 2: return pair_s<StF16>(a, ty, zchunk, s);
    case 3: return pair_s<StBF16SR>(a, ty, zchunk, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace wave
