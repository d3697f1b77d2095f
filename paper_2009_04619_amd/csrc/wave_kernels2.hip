// wave_kernels2.hip -- two time steps per launch on gfx950 (temporal
// blocking of Alg. 1's loop: the 2.5-D stream of wave_kernels.hip with a
// second step that trails the first by 4 planes along z, "3.5-D" blocking).
//
// Each workgroup owns a 56 x 16 output tile and a 64 x 24 first-step region
// around it (the output tile plus the 4-cell halo the second step's stencil
// needs).  Per iteration it
//  * stages plane za of u^n (with a further 4-cell halo) in LDS and computes
//    u^{n+1} (and phi^{n+1}) at plane za over the whole first-step region,
//    adds the sources of step n, rounds to the storage type, and keeps the
//    result in an LDS ring of 5 planes (phi^{n+1} of the output rows too);
//    the output points of u^{n+1} also go to memory;
//  * computes u^{n+2} (and phi^{n+2}) at plane za - 4 of the output tile from
//    the ring (x and y neighbours) and a per-column register queue of
//    u^{n+1} (z neighbours), with u^n of that plane as "u_prev".
// So u^n, u^{n-1}, vp and phi^n cross HBM once for two steps.  The per-point
// arithmetic is that of wave_point.h, operand for operand, so every value
// equals the one two single steps produce (the first-step region's halo is
// recomputed by neighbouring tiles with identical results).
//
// Buffers: u^{n-1}, u^n and phi^n are read; u^{n+1}, u^{n+2} and phi^{n+2}
// go to three other arrays (a neighbouring tile still reads u^{n-1}, u^n and
// phi^n at points this tile has finished, so nothing is written in place).
// Supported: damping off, or the default profile held as tables.
#include <algorithm>
#include <unordered_map>

#include "wave_internal.h"
#include "wave_point.h"

namespace wave {
namespace {

constexpr int kW2 = 16;                   // wavefronts per workgroup
constexpr int kTY2 = 24;                  // output rows per tile
constexpr int kOX2 = kTX - 2 * kR;        // output columns per tile (lanes 4..59)
constexpr int kAR = kTY2 + 2 * kR;        // first-step rows (32)
constexpr int kRA = kAR / kW2;            // first-step rows per wavefront (2)
constexpr int kSR = kAR + 2 * kR;         // staged rows (40)
constexpr int kSW = kTX + 2 * kR;         // staged columns (72)
constexpr int kSPL = kSR * kSW;           // staged plane (floats)
constexpr int kNT2 = 64 * kW2;            // threads
constexpr int kNH2 = kSPL - kAR * kTX;    // staged halo elements (832)
constexpr int kRPL = kAR * kTX;           // u^{n+1} ring plane (floats)
constexpr int kRing = 5;                  // u^{n+1} planes za-4 .. za in LDS
constexpr int kL2 = 10;                   // register ring length = unroll length
constexpr int kMaxZc2 = 512;              // longest z chunk (the z tables sit in LDS)
constexpr int kZT = kMaxZc2 + 4 * kR;     // window planes of the longest chunk
static_assert(kRA == 2 && kAR == 2 * kW2 && kNH2 <= kNT2, "row split assumed below");
static_assert(kL2 % kRing == 0 && kL2 % 2 == 0, "ring lengths must divide the unroll");

// Rows of the first-step region (index a, y = y0 - 4 + a) owned by wavefront
// wv: a = 4 + wv (an output row), and a = 12 + wv for wv >= 8 (an output
// row), else one of the halo rows 0-3, 28-31.  Each wavefront's second-step
// rows are thus among its own first-step rows, so their u^{n+1} and phi^{n+1}
// along z stay in its registers.
__device__ __forceinline__ int region_row(int wv, int k) {
  return k == 0 ? kR + wv : (wv >= 8 ? 12 + wv : (wv < 4 ? wv : kTY2 + wv));
}

// A source that falls in a tile's first-step region and chunk window: lane
// (x - x0), y, z and its wavelet sample w[n].
struct TileSrc {
  int lane, y, z;
  float wq;
};
constexpr int kMaxTileSrc = 32;

struct Smem2 {
  float sa[2][kSPL];                 // staged u^n plane (double-buffered)
  float rb[kRing][kRPL];             // u^{n+1}, first-step region
  float f1[kRing][kTY2 * kTX];       // phi^{n+1}, output rows (each wavefront its own)
  double ts[kAR][kTX];               // default profile: tx + ty of the region's points
  double tz[kZT];                    // default profile: tz and dq_z of the window's planes
  float dqz[kZT];
  float dump[kNT2 - kNH2 + 64];
  TileSrc src[kMaxTileSrc];          // the tile's sources, in list order
  int nsrc;
};

// z chunks of the two-step sweep: as the single-step ones, with caps 4
// planes deeper so that the first step of an interior chunk (planes zb-4 ..
// ze+3) stays out of the z caps.
__device__ inline ChunkInfo chunk2_of(int ch, int nz, int w, int zc, bool damp) {
  return chunk_of(ch, nz, (damp && w > 0) ? w + kR : 0, zc, damp && w > 0);
}

template <class S, int EM>
__device__ __forceinline__ void s2_loop(const Sweep2Args& g, Smem2& sm, int x0, int y0, int zb,
                                        int ze) {
  using T = typename S::T;
  const SweepArgs& a = g.s;
  constexpr uint32_t ES = sizeof(T);
  constexpr bool LAYER = EM != 0;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const bool out1 = wv >= 8;           // the second row is an output row too
  const int P = a.pitch;
  const int64_t Q = a.plane;
  const uint32_t pe = (uint32_t)Q * ES, p4 = (uint32_t)Q * 4u;
  const int nx = a.nx, ny = a.ny, nz = a.nz, w = a.w;

  // window: planes wz0 .. wz1 of every array, from row -4
  const int wz0 = max(zb - 2 * kR, -kR), wz1 = min(ze + 2 * kR - 1, nz + kR - 1);
  const int64_t w0 = (int64_t)wz0 * Q - (int64_t)kR * P;
  const uint32_t wl_e = (uint32_t)(wz1 - wz0 + 1) * pe, wl_4 = (uint32_t)(wz1 - wz0 + 1) * p4;
  const auto ru = rsrc_at(static_cast<const T*>(a.cur) + w0, 0xffffffffu);
  const auto rp = rsrc_at(static_cast<const T*>(g.prev) + w0, 0xffffffffu);
  const auto rv = rsrc_at(a.vp + w0, 0xffffffffu);
  const auto ro1 = rsrc_at(static_cast<T*>(g.out1) + w0, wl_e);
  const auto ro2 = rsrc_at(static_cast<T*>(g.out2) + w0, wl_e);
  const auto rph = rsrc_at(LAYER ? (const void*)(a.phi + w0) : nullptr, LAYER ? wl_4 : 0u);
  const auto rpo = rsrc_at(LAYER ? (const void*)(g.phi_out + w0) : nullptr, LAYER ? wl_4 : 0u);
  auto wk = [&](int z) { return (uint32_t)(min(max(z, wz0), wz1) - wz0); };  // window index

  // in-plane element offset of (x, y), clamped to cells that exist (values of
  // clamped cells are never used by a point inside the grid)
  auto poff = [&](int x, int y) {
    const int yy = min(max(y, -kR), ny + kR - 1);
    const int xx = min(max(x, -kR), P + kR - 1);
    return (uint32_t)max((yy + kR) * P + xx, 0);
  };

  const int x = x0 + lane;
  const bool vx = x >= 0 && x < nx;
  const bool ownx = lane >= kR && lane < kR + kOX2 && vx;
  const bool layx = x < w || x >= nx - w;

  uint32_t vo[kRA], vo4[kRA], eo[kRA], sta[kRA], rbo[kRA];
  bool va[kRA], lxa[kRA], own[kRA];
  int yr[kRA];
#pragma unroll
  for (int k = 0; k < kRA; ++k) {
    const int ar = region_row(wv, k);
    const int y = y0 - kR + ar;
    yr[k] = y;
    va[k] = vx && y >= 0 && y < ny;
    lxa[k] = va[k] && (layx || y < w || y >= ny - w);
    own[k] = ownx && (k == 0 || out1) && y < ny;
    const uint32_t o = poff(x, y);
    vo[k] = o * ES;
    vo4[k] = o * 4u;
    sta[k] = (uint32_t)((kR + ar) * kSW + kR + lane);
    rbo[k] = (uint32_t)(ar * kTX + lane);
  }
  // staged halo: element h of the staged plane's frame (rows 0-3, 36-39 of 72
  // columns, then columns 0-3, 68-71 of rows 4-35); threads beyond it write
  // to a dump area
  int hl;
  uint32_t ho;
  {
    const int h = threadIdx.x;
    int sr, sc;
    if (h < 2 * kR * kSW) {
      const int rr = h / kSW;
      sr = rr < kR ? rr : kAR + rr;
      sc = h % kSW;
    } else if (h < kNH2) {
      const int kk = h - 2 * kR * kSW;
      sr = kR + kk / (2 * kR);
      const int cc = kk % (2 * kR);
      sc = cc < kR ? cc : kTX + cc;
    } else {
      sr = -1;
      sc = h - kNH2;
    }
    hl = sr >= 0 ? sr * kSW + sc : -1 - sc;
    ho = poff(x0 - kR + sc, y0 - 2 * kR + max(sr, 0)) * ES;
  }

  // default profile tables (EM = 2); tx + ty of the own points go to LDS
  float dqx = 0.0f, dqy[kRA];
  uint32_t tso[kRA];
#pragma unroll
  for (int k = 0; k < kRA; ++k) tso[k] = (uint32_t)(region_row(wv, k) * kTX + lane);
  if (EM == 2) {
    const double* tx = a.etab + 1;
    const double* ty = tx + nx + 2;
    const int xc = min(max(x, 0), nx - 1);
    dqx = a.etq[xc];
#pragma unroll
    for (int k = 0; k < kRA; ++k) {
      const int yc = min(max(yr[k], 0), ny - 1);
      (&sm.ts[0][0])[tso[k]] = tx[xc] + ty[yc];
      dqy[k] = a.etq[nx + yc];
    }
  }

  float q[kL2][kRA];                    // u^n(za-4 .. za+5)
  float q1[kL2][kRA];                   // u^{n+1}(za-9 .. za) of the own rows
  float pva[2][kRA], vva[2][kRA], pha[2][kRA], vvb[kRA];
  float hh[2];
  uint32_t f1o[kRA];                    // own output row in the phi^{n+1} ring
#pragma unroll
  for (int k = 0; k < kRA; ++k) f1o[k] = (uint32_t)((region_row(wv, k) - kR) * kTX + lane);

  auto load_a = [&](int B, int z) {     // first-step operands of plane z
    const uint32_t k = wk(z);
#pragma unroll
    for (int r = 0; r < kRA; ++r) {
      pva[B][r] = S::bld(rp, vo[r], k * pe);
      vva[B][r] = bld_f32(rv, vo4[r], k * p4);
      if (LAYER) pha[B][r] = bld_f32(rph, eo[r], k * p4);
    }
    hh[B] = S::bld(ru, ho, k * pe);
  };
  auto load_b = [&](int z) {            // second-step operand of plane z (vp)
    const uint32_t k = wk(z);
#pragma unroll
    for (int r = 0; r < kRA; ++r) vvb[r] = bld_f32(rv, vo4[r], k * p4);
  };

  // phi^n offsets: layer points of the first-step region, out of range for
  // the others (z caps decided per plane in the loop)
  auto set_eo = [&](int z) {
    const bool capz = z < w || z >= nz - w;
#pragma unroll
    for (int r = 0; r < kRA; ++r) eo[r] = (va[r] && (lxa[r] || capz)) ? vo4[r] : kOOB;
  };

  // the tile's sources, gathered once in list order (wave 0, 64 at a time):
  // the plane loop then tests LDS entries instead of reading the source
  // list from memory, whose waits would also drain the operand prefetch
  if (wv == 0) {
    int n = 0;
    for (int base = 0; base < g.nsrc; base += 64) {
      const int q2 = base + lane;
      bool hit = false;
      TileSrc e{0, 0, 0, 0.0f};
      if (q2 < g.nsrc) {
        const int sx = g.src_ijk[3 * q2], sy = g.src_ijk[3 * q2 + 1], sz = g.src_ijk[3 * q2 + 2];
        hit = sx >= x0 && sx < x0 + kTX && sy >= y0 - kR && sy < y0 + kTY2 + kR &&
              sz >= zb - kR && sz < ze + kR;
        if (hit)
          e = TileSrc{sx - x0, sy, sz,
                      g.step < g.max_steps ? g.wavelet[(int64_t)q2 * g.max_steps + g.step] : 0.0f};
      }
      const uint64_t m = __ballot(hit);
      if (hit) {
        const int pos = n + __popcll(m & ((1ull << lane) - 1ull));
        if (pos < kMaxTileSrc) sm.src[pos] = e;
      }
      n += __popcll(m);
    }
    if (lane == 0) sm.nsrc = n;
  }
  // z terms of the default profile for the window's planes (read per plane
  // from LDS with a uniform address)
  if (a.damping && a.etab) {
    const double* tzt = a.etab + 1 + (nx + 2) + (ny + 2);
    const float* dqzt = a.etq + nx + ny;
    for (int i = threadIdx.x; i <= wz1 - wz0; i += kNT2) {
      const int zc = min(max(wz0 + i, 0), nz - 1);
      sm.tz[i] = tzt[zc];
      sm.dqz[i] = dqzt[zc];
    }
  }
  __syncthreads();
  // (the host runs single steps instead when a tile would hold more; the
  // bound only keeps the reads inside the list)
  const int nts = min(__builtin_amdgcn_readfirstlane(sm.nsrc), kMaxTileSrc);

  const int za0 = zb - kR;
  if (LAYER) set_eo(za0);
#pragma unroll
  for (int j = 0; j < 2 * kR + 1; ++j) {
    const uint32_t k = wk(za0 - kR + j);
#pragma unroll
    for (int r = 0; r < kRA; ++r) q[j][r] = S::bld(ru, vo[r], k * pe);
  }
  load_a(0, za0);

  // Iteration za: stage u^n(za), one barrier, first step at za (into the
  // LDS ring and the own registers), second step at za - 4 (x/y neighbours
  // from the ring plane written 4 iterations ago, z neighbours from the own
  // registers).  A ring slot is rewritten 5 iterations after it was written,
  // after the barrier that follows its last read; a staged buffer 2
  // iterations after, likewise.
  auto body = [&](auto SC, const int za) {
    constexpr int Sl = decltype(SC)::value;
    constexpr int B = Sl & 1, NB = B ^ 1;
    constexpr int RS = Sl % kRing;            // ring slot of plane za
    constexpr int RQ = (Sl + 1) % kRing;      // ring slot of plane za - 4
    const int zq = za - kR;
    // requests: u^n(za+5) and the first-step operands of za+1 for the next
    // iteration, vp of za-4 for this iteration's second step (all clamped
    // to the window)
    {
      const uint32_t k5 = wk(za + kR + 1);
#pragma unroll
      for (int r = 0; r < kRA; ++r) q[(Sl + 2 * kR + 1) % kL2][r] = S::bld(ru, vo[r], k5 * pe);
      if (LAYER) set_eo(za + 1);
      load_a(NB, za + 1);
      load_b(zq);
    }
    // stage u^n(za) with its halo
    float* s = sm.sa[B];
#pragma unroll
    for (int r = 0; r < kRA; ++r) s[sta[r]] = q[(Sl + kR) % kL2][r];
    if (hl >= 0) s[hl] = hh[B];
    else sm.dump[-1 - hl] = hh[B];
    __syncthreads();

    // ---- first step: u^{n+1}, phi^{n+1} at plane za ----
    const bool inz = za >= 0 && za < nz;
    const bool ownz = za >= zb && za < ze;
    const bool capza = za < w || za >= nz - w;
    float res[kRA], nph[kRA];
    bool lay[kRA];
#pragma unroll
    for (int r = 0; r < kRA; ++r) {
      const float* row = s + sta[r];
      const float c = q[(Sl + kR) % kL2][r];
      float lap = a.c[0] * c;
#pragma unroll
      for (int m = 1; m <= kR; ++m) lap = __builtin_fmaf(a.c[m], row[m] + row[-m], lap);
#pragma unroll
      for (int m = 1; m <= kR; ++m)
        lap = __builtin_fmaf(a.c[4 + m], row[m * kSW] + row[-m * kSW], lap);
#pragma unroll
      for (int m = 1; m <= kR; ++m)
        lap = __builtin_fmaf(a.c[8 + m], q[(Sl + kR + m) % kL2][r] + q[(Sl + kR - m) % kL2][r], lap);
      lap = __builtin_fmaf(a.ce, c, lap);
      nph[r] = 0.0f;
      lay[r] = false;
      if (LAYER) {
        lay[r] = va[r] && (lxa[r] || capza);
        const uint32_t kz = wk(za);
        const float e = lay[r] ? (float)(a.dt * ((&sm.ts[0][0])[tso[r]] + sm.tz[kz])) : 0.0f;
        res[r] = upd_layer(c, pva[B][r], vva[B][r], lap, e, pha[B][r]);
        nph[r] = upd_phi(pha[B][r], e, dqx, row[1] - row[-1], dqy[r], row[kSW] - row[-kSW],
                         sm.dqz[kz], q[(Sl + kR + 1) % kL2][r] - q[(Sl + kR - 1) % kL2][r]);
      } else {
        res[r] = upd_inner(c, pva[B][r], vva[B][r], lap);
      }
      // the stored value (storage rounding)
      res[r] = S::cvt(S::enc(res[r]));
    }
    // then the sources of step n in list order, each stored in turn (Alg. 1:
    // the source add follows the sweep); entries of other planes are skipped
    // with a scalar test, and the add is a select, not a branch
    for (int q2 = 0; q2 < nts; ++q2) {
      const TileSrc e = sm.src[q2];
      if (__builtin_amdgcn_readfirstlane(e.z) != za) continue;
#pragma unroll
      for (int r = 0; r < kRA; ++r) {
        const float v = S::cvt(S::enc(__builtin_fmaf(vva[B][r], e.wq, res[r])));
        res[r] = (lane == e.lane && y0 - kR + region_row(wv, r) == e.y) ? v : res[r];
      }
    }
#pragma unroll
    for (int r = 0; r < kRA; ++r) {
      const bool live = inz && va[r];
      const float u1 = live ? res[r] : 0.0f;
      sm.rb[RS][rbo[r]] = u1;
      S::bst(ro1, (ownz && own[r]) ? vo[r] : kOOB, wk(za) * pe, u1);
      q1[Sl][r] = u1;
      if (LAYER && (r == 0 || out1)) sm.f1[RS][f1o[r]] = (live && lay[r]) ? nph[r] : 0.0f;
    }

    // ---- second step: u^{n+2}, phi^{n+2} at plane zq = za - 4 ----
    if (zq >= zb && zq < ze) {
      const bool capzq = zq < w || zq >= nz - w;
      const uint32_t kq = wk(zq);
      const float* rbq = sm.rb[RQ];
#pragma unroll
      for (int r = 0; r < kRA; ++r) {
        if (r == 1 && !out1) break;
        const float* row = rbq + rbo[r];
        const float c = q1[(Sl + kL2 - kR) % kL2][r];
        float lap = a.c[0] * c;
#pragma unroll
        for (int m = 1; m <= kR; ++m) lap = __builtin_fmaf(a.c[m], row[m] + row[-m], lap);
#pragma unroll
        for (int m = 1; m <= kR; ++m)
          lap = __builtin_fmaf(a.c[4 + m], row[m * kTX] + row[-m * kTX], lap);
#pragma unroll
        for (int m = 1; m <= kR; ++m)
          lap = __builtin_fmaf(a.c[8 + m],
                               q1[(Sl + kL2 - kR + m) % kL2][r] + q1[(Sl + kL2 - kR - m) % kL2][r], lap);
        lap = __builtin_fmaf(a.ce, c, lap);
        const float un = q[Sl % kL2][r];       // u^n(zq), the second step's "previous" level
        float res2;
        if (LAYER) {
          const bool lay2 = own[r] && (lxa[r] || capzq);
          const float e = lay2 ? (float)(a.dt * ((&sm.ts[0][0])[tso[r]] + sm.tz[kq])) : 0.0f;
          const float ph = sm.f1[RQ][f1o[r]];
          res2 = upd_layer(c, un, vvb[r], lap, e, ph);
          const float nph2 =
              upd_phi(ph, e, dqx, row[1] - row[-1], dqy[r], row[kTX] - row[-kTX], sm.dqz[kq],
                      q1[(Sl + kL2 - kR + 1) % kL2][r] - q1[(Sl + kL2 - kR - 1) % kL2][r]);
          bst_f32(rpo, lay2 ? vo4[r] : kOOB, kq * p4, nph2);
        } else {
          res2 = upd_inner(c, un, vvb[r], lap);
        }
        S::bst(ro2, own[r] ? vo[r] : kOOB, kq * pe, res2);
      }
    }
  };

  using std::integral_constant;
  for (int za = za0; za < ze + kR; za += kL2) {
#define WAVE_BODY2(J)                                   \
    if ((J) > 0 && za + (J) >= ze + kR) break;          \
    body(integral_constant<int, (J)>{}, za + (J));
    WAVE_BODY2(0) WAVE_BODY2(1) WAVE_BODY2(2) WAVE_BODY2(3) WAVE_BODY2(4)
    WAVE_BODY2(5) WAVE_BODY2(6) WAVE_BODY2(7) WAVE_BODY2(8) WAVE_BODY2(9)
#undef WAVE_BODY2
  }
}

template <class S>
__global__ __launch_bounds__(kNT2) void k_sweep2(Sweep2Args g, int tiles_x, int tiles_y,
                                                 int zchunk) {
  __shared__ Smem2 sm;
  const SweepArgs& a = g.s;
  const int nb = gridDim.x, bid = blockIdx.x;
  const int per = nb >> 3, rem = nb & 7, xcd = bid & 7, slot = bid >> 3;
  const int logical = (xcd < rem) ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
  const int tx = logical % tiles_x;
  const int t2 = logical / tiles_x;
  const int ty = t2 % tiles_y;
  const int ch = t2 / tiles_y;
  const int x0 = tx * kOX2 - kR, y0 = ty * kTY2;
  const bool damp = a.damping != 0;
  const ChunkInfo c = chunk2_of(ch, a.nz, a.w, zchunk, damp);
  if (c.zb >= c.ze) return;
  // wavefront-uniform choice of the loop: any layer point among the
  // wavefront's rows, in any plane of the chunk
  bool lay = false;
  if (damp) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int x = x0 + lane;
    const bool lx = x < a.w || x >= a.nx - a.w;
    for (int k = 0; k < kRA; ++k) {
      const int y = y0 - kR + region_row(wv, k);
      lay = lay || (x >= 0 && x < a.nx && y >= 0 && y < a.ny && (lx || y < a.w || y >= a.ny - a.w));
    }
    lay = lay || c.cap;
  }
  if (!__any(lay))
    s2_loop<S, 0>(g, sm, x0, y0, c.zb, c.ze);
  else
    s2_loop<S, 2>(g, sm, x0, y0, c.zb, c.ze);
}

template <class S>
hipError_t sweep2_t(const Sweep2Args& g, int zchunk, hipStream_t st) {
  const SweepArgs& a = g.s;
  const int tiles_x = (a.nx + kOX2 - 1) / kOX2;
  const int tiles_y = (a.ny + kTY2 - 1) / kTY2;
  const bool damp = a.damping != 0 && a.w > 0;
  const int chunks = chunk_count(a.nz, damp ? a.w + kR : 0, zchunk, damp);
  const int64_t blocks = (int64_t)tiles_x * tiles_y * chunks;
  if (blocks <= 0 || blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sweep2<S>, dim3((unsigned)blocks), dim3(kNT2), 0, st, g, tiles_x, tiles_y,
                     zchunk);
  return hipGetLastError();
}

}  // namespace

int stream2_zchunk_limit(int64_t plane) {
  const int64_t z = kWindowMax / (plane * 4) - 4 * kR;
  return (int)std::min<int64_t>(z, kMaxZc2);
}

bool sweep2_sources_fit(const int32_t* ijk, int n) {
  // first-step region of tile (tx, ty): x in [56 tx - 4, 56 tx + 60),
  // y in [24 ty - 4, 24 ty + 28); each point lies in at most 2 x 2 tiles
  std::unordered_map<int64_t, int> count;
  for (int s = 0; s < n; ++s) {
    const int i = ijk[3 * s], j = ijk[3 * s + 1];
    const int tx1 = (i + kR) / kOX2, ty1 = (j + kR) / kTY2;
    for (int tx = std::max(tx1 - 1, 0); tx <= tx1; ++tx) {
      if (i < tx * kOX2 - kR || i >= tx * kOX2 - kR + kTX) continue;
      for (int ty = std::max(ty1 - 1, 0); ty <= ty1; ++ty) {
        if (j < ty * kTY2 - kR || j >= ty * kTY2 + kTY2 + kR) continue;
        if (++count[((int64_t)tx << 32) | (uint32_t)ty] > kMaxTileSrc) return false;
      }
    }
  }
  return true;
}

int auto_zchunk2(int nx, int ny, int nz) {
  // long chunks: each one recomputes 8 planes of the first step and reads 16
  // extra planes of u^n; about nz/8 planes, at least 64
  const int64_t tiles = (int64_t)((nx + kOX2 - 1) / kOX2) * ((ny + kTY2 - 1) / kTY2);
  const int64_t chunks = (4096 + tiles - 1) / tiles;
  int zc = (int)std::min<int64_t>(nz / 8, (nz + chunks - 1) / chunks);
  zc = std::max(zc, 64);
  return std::min(std::min(zc, nz), kMaxZc2);
}

hipError_t launch_sweep2(const Sweep2Args& g, int storage, int zchunk, hipStream_t s) {
  if (zchunk <= 0 || zchunk > stream2_zchunk_limit(g.s.plane)) return hipErrorInvalidValue;
  if (g.s.damping && !g.s.etab) return hipErrorInvalidValue;   // eta arrays: single steps only
  switch (storage) {
    case 0: return sweep2_t<StF32>(g, zchunk, s);
    case 1: return sweep2_t<StBF16>(g, zchunk, s);
    case 2: return sweep2_t<StF16>(g, zchunk, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace wave
