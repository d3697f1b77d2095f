// wave_kernels.hip -- gfx950 kernels of one time step of the 3-D acoustic
// wave equation (paper Sec. III-A, Eq. 2-3; damping layer after Sec. III-B):
// the per-point sweeps (direct and 2.5-D streaming, single shot and batched),
// source add and receiver sample, the float64 energy, set-up and copy.  The
// per-point arithmetic they share is in wave_point.h.
#include <algorithm>

#include "wave_direct.h"
#include "wave_internal.h"
#include "wave_point.h"

namespace wave {
namespace {

// ---- variant 0: one thread per point, every operand read from memory -------
template <class S>
__global__ __launch_bounds__(256) void k_sweep_direct(SweepArgs a) {
  const int x = blockIdx.x * kTX + threadIdx.x;
  const int y = blockIdx.y * 4 + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= a.nx || y >= a.ny) return;
  direct_point<S>(a, x, y, z);
}

// ---- variant 1: 2.5-D streaming ------------------------------------------------
// A workgroup of NW wavefronts owns a 64 x TY xy tile (TY = RY * NW; each
// wavefront owns RY rows, one x column per lane, or, in a tile that holds an
// x wall of the layer, 2 RY half rows of 32 columns) and streams it through the
// planes [zb, ze) of one z chunk.  Per plane z:
//  * the values u(z-4..z+4) of every owned column sit in registers, in a ring
//    that also holds the kPD planes of u already requested beyond z+4;
//  * the centre plane of the tile plus its 4-wide x and y halos is staged in
//    LDS (double-buffered: one barrier per plane), from which the x and y
//    neighbours are read;
//  * the operands of plane z + kPD (u^{n-1}, vp, halo, phi, eta) are
//    requested while plane z is computed, so about kPD planes of loads are in
//    flight per wavefront.
// The loop is unrolled by the ring length so every ring index is a
// compile-time constant.  Blocks are remapped so that consecutive tiles
// (which share halos) run on the same XCD and its L2.
//
// Addressing: each array is reached through one buffer resource per tile
// whose base is plane zb-4, row -4 of the chunk's window (planes zb-4 ..
// ze+3); a lane's offset inside a plane is fixed for the whole loop and the
// plane enters as a wave-uniform offset, so the loop does no 64-bit address
// arithmetic.  The window of every float array is below 2 GiB (checked by the
// launcher), so 32-bit offsets cover it.
//
// Damping layer: z chunks are cut at the layer faces (chunks in the z caps
// hold only cap planes), so whether a lane is a layer point is fixed for a
// workgroup.  Wavefronts that own no layer point run a loop without eta/phi.
// The others issue the eta/phi loads and the phi store unconditionally; a
// lane outside the layer gets an offset beyond the resource's range, which
// reads 0 and writes nothing, so it fetches no bytes, and eta = phi = 0
// turns the layer update into the inner one bit for bit.  Memory operations
// are thus identical on every path, which keeps the prefetch overlapping the
// compute.

// Prefetch distance in planes (the u ring then has 9 + kPD slots and the
// per-plane operand rings kPD + 1; both divide the unroll length).
#ifndef WAVE_STREAM_PD
#define WAVE_STREAM_PD 3
#endif
constexpr int kPD = WAVE_STREAM_PD;
static_assert(kPD == 1 || kPD == 3 || kPD == 7, "prefetch distance must make kPD + 1 divide 9 + kPD");

// Per-thread slot of a tile: which point it owns and where that point lives.
template <int RY>
struct Slots {
  int x[RY], y[RY];  // grid coordinates of the point
  uint32_t ro[RY];   // in-plane element offset ((y + 4) * pitch + x)
  int ls[RY];        // LDS index of the point in the staged plane
  bool valid[RY];    // inside the grid (else the clamped ghost row/column)
  bool lay[RY];      // a damping-layer point
  bool phl[RY];      // phi is read and written back here: a layer point, or an
                     // inner point sharing a 128-byte line with an x-wall one
  // x neighbours by wavefront shuffles (XS): the lane's position in its row
  // segment of xw lanes (64, or 32 in a tile holding an x wall), and the
  // in-plane offset of the x-halo cell this lane loads for its row segment
  // (lanes 0..3: the 4 cells right of the segment, lanes xw-4..xw-1: the 4
  // cells left of it; kHaloGhost for the others and for ghost cells)
  int xli, xw;
  uint32_t xho[RY];
};

// Halo offset marking a ghost cell (never a real in-plane offset).
constexpr uint32_t kHaloGhost = 0xffffffffu;

// Read-only tables in the constant address space (scalar loads when the
// index is wave-uniform).
typedef const double __attribute__((address_space(4))) CDouble;
typedef const float __attribute__((address_space(4))) CFloat;

// The streaming loop over planes [zb, ze) for one wavefront's slots.
// EM = 0: no layer point.  EM = 1, 2: the wavefront owns at least one layer
// point and evaluates the layer update for all its points (eta and phi read
// as 0 and phi' dropped for the others, which gives the inner update
// exactly); eta comes from the per-point array (EM = 1) or from the default
// profile's tables (EM = 2, no eta traffic).
//
// ZS: the z terms of the Laplacian by the semi-stencil (Sec. IV,
// "Semi-stencil"): each u plane enters the sums of its 8 z neighbours the
// plane it becomes the staged one, in two phases.  Forward: u(p) is the -m
// neighbour of the outputs p+m, whose partial sums F collect
// c_z4 u(p+m-4) + .. + c_z1 u(p+m-1) before their own plane is staged.
// Backward: u(p) is the +m neighbour of the outputs p-m, whose sums A
// (centre, x and y terms, plus F, formed when their plane was staged) it
// completes in the order m = 1..4; the output p-4 is then final and is
// written.  So an output trails the staged plane by 4 planes, its operands
// (u^{n-1}, vp, phi, the profile's z term) are requested for that plane, and
// each z term is c_zm u rather than c_zm (u(+m) + u(-m)): the same
// Laplacian summed in another order, so results differ from the other
// kernels by rounding only.  The phi update is unchanged (its gradient
// keeps the x, y, z order: the z difference u(p+1) - u(p-1) is added the
// plane after p was staged).  Default-profile tables only (no eta array).
// XS: the x neighbours come from wavefront shuffles (ds_bpermute) of the
// lanes' own values instead of the staged plane; a lane at the end of its row
// segment takes the x-halo value another lane of the segment loaded.  The
// values, and so the results, are the same as from LDS.
template <class S, int RY, int NW, int EM, bool ZS = false, bool XS = false>
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
  constexpr int PD = kPD;
  constexpr int L = 2 * kR + 1 + PD;                    // u ring
  constexpr int NR = PD + 1;                            // per-plane operand rings
  constexpr int NE = (L % (PD + 3) == 0) ? PD + 3 : L;  // eta column ring
  static_assert(L % NR == 0 && L % NE == 0 && L % 2 == 0, "ring lengths must divide the unroll");
  constexpr bool LAYER = EM != 0;
  constexpr bool EARR = EM == 1;
  static_assert(!ZS || EM != 1, "the z semi-stencil takes the default profile's tables only");
  static_assert(!(ZS && XS), "one variant at a time");
  constexpr int ZD = ZS ? kR : 0;  // planes an output trails the staged plane

  const int64_t Q = a.plane;
  const int P = a.pitch;
  const uint32_t pe = (uint32_t)Q * ES;  // bytes per plane, wavefield arrays
  const uint32_t p4 = (uint32_t)Q * 4u;  // bytes per plane, float arrays
  const uint32_t rb4 = (uint32_t)P * 4u;
  // window of the chunk: planes zb-4 .. ze+3, from row -4
  const int64_t w0 = (int64_t)(zb - kR) * Q - (int64_t)kR * P;
  const uint32_t wlen = (uint32_t)(ze - zb + 2 * kR) * p4;
  const int zlast = ze - zb + kR - 1;  // window index of plane ze-1
  // every resource is limited to the window, so a load at kOOB (a ghost
  // halo cell, a lane past the grid) fetches nothing and reads 0, the
  // ghost's value, and a store there is dropped
  const auto ru = rsrc_at(static_cast<const T*>(a.cur) + w0, (uint32_t)(ze - zb + 2 * kR) * pe);
  const auto rn = rsrc_at(static_cast<T*>(a.nxt) + w0, (uint32_t)(ze - zb + 2 * kR) * pe);
  const auto rv = rsrc_at(a.vp + w0, wlen);
  const auto rph = rsrc_at(LAYER ? (const void*)(a.phi + w0) : nullptr, LAYER ? wlen : 0u);
  const auto ret = rsrc_at(EARR ? (const void*)(a.eta + w0) : nullptr, EARR ? wlen : 0u);

  // lane byte offsets in a plane; a lane past the grid (its column in the
  // row padding, or its row clamped to the ghost row) reads zeros and
  // stores nothing: padding and ghosts are zero from the set-up on
  uint32_t vo[RY], vo4[RY];
  uint32_t hoe[HPT];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    vo[r] = sl.valid[r] ? sl.ro[r] * ES : kOOB;
    vo4[r] = sl.valid[r] ? sl.ro[r] * 4u : kOOB;
  }
#pragma unroll
  for (int k = 0; k < HPT; ++k) hoe[k] = ho[k] == kHaloGhost ? kOOB : ho[k] * ES;
  uint32_t eo[RY];  // eta lane offset; out of range for non-layer points
  uint32_t fo[RY];  // phi lane offset; out of range where phi is not touched
  if (LAYER) {
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      eo[r] = sl.lay[r] ? vo4[r] : kOOB;
      fo[r] = sl.phl[r] ? vo4[r] : kOOB;
    }
  }
  // EM = 2: the z-independent part of the profile sum, tx + ty, and the x and
  // y difference products of the point; per plane tz(z) and dq_z(z), which
  // are the same for every lane, travel in operand rings (read through the
  // constant address space, so they are scalar loads that do not queue
  // behind the vector loads)
  double tsc[RY];
  float dqx[RY], dqy[RY];
  const CDouble* tzt = nullptr;
  const CFloat* dqzt = nullptr;
  if (EM == 2) {
    const double* tx = a.etab + 1;
    const double* ty = tx + a.nx + 2;
    tzt = (const CDouble*)(ty + a.ny + 2);
    dqzt = (const CFloat*)(a.etq + a.nx + a.ny);
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const int x = sl.x[r], y = sl.y[r];
      tsc[r] = tx[x] + ty[y];
      dqx[r] = a.etq[x];
      dqy[r] = a.etq[a.nx + y];
    }
  }

  float q[L][RY];
  float pv[NR][RY], vv[NR][RY];
  float hh[NR][HPT];
  // LAYER: eta of the own column in a ring (at slot Sl, er[(Sl + j) % NE]
  // holds eta(z - 1 + j)); phi and the eta x/y neighbours in operand rings
  float er[NE][RY];
  float ex0[NR][RY], ex1[NR][RY], ey0[NR][RY], ey1[NR][RY], ph[NR][RY];
  double tzr[NR];
  float dzr[NR];
  // ZS: sums of the outputs in flight (A: planes z-3..z, F: z+1..z+4, G: the
  // phi gradient of z-3..z), and dq_z of the staged planes
  float A[ZS ? 4 : 1][RY], F[ZS ? 4 : 1][RY], G[ZS && LAYER ? 4 : 1][RY];
  float dzs[ZS ? NR : 1] = {};
  // XS: the x-halo values of the row segments, per operand slot, and the
  // shuffle sources: for +m the lane reads lane (li + m) mod xw of its segment
  // from a register that holds, in lanes li < m, the x-halo value (the right
  // halo sits in lanes 0..3); for -m lane (li - m) mod xw of a register that
  // holds the left halo in lanes li >= xw - m
  float hx[XS ? NR : 1][RY];
  uint32_t xhe[XS ? RY : 1];
  int xap[XS ? kR : 1], xam[XS ? kR : 1];
  bool xcp[XS ? kR : 1], xcm[XS ? kR : 1];
  if constexpr (XS) {
    const int lane = threadIdx.x & 63;
    const int base = lane & ~(sl.xw - 1);
#pragma unroll
    for (int m = 1; m <= kR; ++m) {
      xap[m - 1] = 4 * (base | ((sl.xli + m) & (sl.xw - 1)));
      xam[m - 1] = 4 * (base | ((sl.xli - m) & (sl.xw - 1)));
      xcp[m - 1] = sl.xli < m;
      xcm[m - 1] = sl.xli >= sl.xw - m;
    }
#pragma unroll
    for (int r = 0; r < RY; ++r) xhe[r] = sl.xho[r] == kHaloGhost ? kOOB : sl.xho[r] * ES;
  }
  // x neighbours (m = 1..4, +m and -m) of u value c with row-segment halo h
  auto xshuffle = [&](float c, float h, float (&xp)[kR], float (&xm)[kR]) {
#pragma unroll
    for (int m = 0; m < kR; ++m) {
      xp[m] = __int_as_float(__builtin_amdgcn_ds_bpermute(xap[m], __float_as_int(xcp[m] ? h : c)));
      xm[m] = __int_as_float(__builtin_amdgcn_ds_bpermute(xam[m], __float_as_int(xcm[m] ? h : c)));
    }
  };

  // store u^{n+1} of lane row r at output plane zo (window byte offset so):
  // bf16 storage rounded stochastically when the context asks for it
  const uint32_t srkey = S::kSR ? pcg_hash((uint32_t)a.step) : 0u;
  auto store_u = [&](int r, uint32_t so, float v, int zo) {
    if constexpr (S::kSR) {
      const int x = sl.x[r];
      const uint32_t r16 = sr_word(srkey, a.nx, a.ny, x, sl.y[r], zo) >> (16 * (x & 1));
      __builtin_amdgcn_raw_buffer_store_b16(f32_to_bf16_sr(v, r16), rn, (int)vo[r], (int)so, kSt);
    } else {
      S::bst(rn, vo[r], so, v);
    }
  };

  // prologue: u(zb-4 .. zb+3+PD) into ring slots 0 .. L-2, operands of planes
  // zb .. zb+PD-1 into operand slots 0 .. PD-1, eta(zb-1 .. zb+PD) into eta
  // slots 0 .. PD+1 (window indices clamped to the window)
#pragma unroll
  for (int j = 0; j < L - 1; ++j) {
    const uint32_t so = (uint32_t)min(j, zlast + kR) * pe;
#pragma unroll
    for (int r = 0; r < RY; ++r) q[j][r] = S::bld(ru, vo[r], so);
  }
#pragma unroll
  for (int j = 0; j < PD; ++j) {
    // operands of the output plane zb - ZD + j, halo of the staged plane zb + j
    // (ZS: output planes before the chunk are never written; their operand
    // loads take an out-of-range offset and fetch nothing)
    const uint32_t kp = (uint32_t)min(j + kR - ZD, zlast);
    const uint32_t se = kp * pe, s4 = kp * p4;
    const uint32_t sh = (uint32_t)min(j + kR, zlast) * pe;
    const bool none = ZS && j < ZD;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      pv[j][r] = S::bld1(rn, none ? kOOB : vo[r], se);
      vv[j][r] = bld1_f32(rv, none ? kOOB : vo4[r], s4);
    }
#pragma unroll
    for (int k = 0; k < HPT; ++k) hh[j][k] = S::bld(ru, hoe[k], sh);
    if constexpr (XS) {
#pragma unroll
      for (int r = 0; r < RY; ++r) hx[j][r] = S::bld(ru, xhe[r], sh);
    }
    if (ZS && LAYER) dzs[j] = dqzt[min(zb + j, a.nz - 1)];
    if (LAYER) {
#pragma unroll
      for (int r = 0; r < RY; ++r) ph[j][r] = bld1_f32(rph, none ? kOOB : fo[r], s4);
    }
    if (EM == 2) {
      const int zt = zb - kR + (int)kp;
      tzr[j] = tzt[zt];
      dzr[j] = dqzt[zt];
    }
    if (EARR) {
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        ex0[j][r] = bld_f32(ret, eo[r] - 4u, s4);
        ex1[j][r] = bld_f32(ret, eo[r] + 4u, s4);
        ey0[j][r] = bld_f32(ret, eo[r] - rb4, s4);
        ey1[j][r] = bld_f32(ret, eo[r] + rb4, s4);
      }
    }
  }
  if (EARR) {
#pragma unroll
    for (int j = 0; j < PD + 2; ++j) {
      const uint32_t s4 = (uint32_t)min(j - 1 + kR, zlast + 1) * p4;
#pragma unroll
      for (int r = 0; r < RY; ++r) er[j][r] = bld_f32(ret, eo[r], s4);
    }
  }
  if constexpr (ZS) {
    // forward phase of the planes zb-4 .. zb-1 (ring slots 0..3): F(zb+i)
    // starts with c_z4 u(zb+i-4) and gathers the nearer planes in turn
#pragma unroll
    for (int r = 0; r < RY; ++r) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        A[i][r] = 0.0f;
        if (LAYER) G[i][r] = 0.0f;
        float f = a.c[12] * q[i][r];
#pragma unroll
        for (int m = 3; m >= 1; --m)
          if (i + 4 - m < 4) f = __builtin_fmaf(a.c[8 + m], q[i + 4 - m][r], f);
        F[i][r] = f;
      }
    }
  }

  auto body = [&](auto SC, const int z) {
    constexpr int Sl = decltype(SC)::value;
    constexpr int B = Sl % NR;          // operand slot of plane z - ZD
    constexpr int BP = (Sl + PD) % NR;  // operand slot of plane z - ZD + PD
    constexpr int LB = Sl & 1;          // LDS buffer
    const int kz = z - zb + kR;         // window index of plane z
    // ZS: dq_z of plane z - 1 (its slot is refilled below)
    const float dz1 = ZS && LAYER ? dzs[(Sl + NR - 1) % NR] : 0.0f;
    // request the halo of plane zh = min(z + PD, ze - 1), u(zh + 4) and the
    // operands of output plane zh - ZD, unconditionally so that the number
    // of loads in flight is the same on every path (past the chunk's end the
    // loads repeat its last planes, which are in cache, and are never used)
    {
      const uint32_t kh = (uint32_t)min(kz + PD, zlast);
      const uint32_t kp = (uint32_t)min(kz - ZD + PD, zlast);
      const uint32_t se = kp * pe, s4 = kp * p4, sh = kh * pe;
      const bool none = ZS && kz - ZD + PD < kR;  // an output plane before the chunk
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        q[(Sl + L - 1) % L][r] = S::bld(ru, vo[r], sh + 4u * pe);
        pv[BP][r] = S::bld1(rn, none ? kOOB : vo[r], se);
        vv[BP][r] = bld1_f32(rv, none ? kOOB : vo4[r], s4);
      }
#pragma unroll
      for (int k = 0; k < HPT; ++k) hh[BP][k] = S::bld(ru, hoe[k], sh);
      if constexpr (XS) {
#pragma unroll
        for (int r = 0; r < RY; ++r) hx[BP][r] = S::bld(ru, xhe[r], sh);
      }
      if (ZS && LAYER) dzs[BP] = dqzt[min(zb - kR + (int)kh, a.nz - 1)];
      if (LAYER) {
#pragma unroll
        for (int r = 0; r < RY; ++r) ph[BP][r] = bld1_f32(rph, none ? kOOB : fo[r], s4);
      }
      if (EM == 2) {
        const int zt = zb - kR + (int)kp;
        tzr[BP] = tzt[zt];
        dzr[BP] = dqzt[zt];
      }
      if (EARR) {
#pragma unroll
        for (int r = 0; r < RY; ++r) {
          er[(Sl + PD + 2) % NE][r] = bld_f32(ret, eo[r], s4 + p4);
          ex0[BP][r] = bld_f32(ret, eo[r] - 4u, s4);
          ex1[BP][r] = bld_f32(ret, eo[r] + 4u, s4);
          ey0[BP][r] = bld_f32(ret, eo[r] - rb4, s4);
          ey1[BP][r] = bld_f32(ret, eo[r] + rb4, s4);
        }
      }
    }
    if constexpr (ZS) {
      const bool stage = z < ze;        // plane z is an output plane of the chunk
      const bool emit = z - ZD >= zb;   // output plane z - 4 is complete
      float* s = sm[LB];
      if (stage) {
#pragma unroll
        for (int r = 0; r < RY; ++r) s[sl.ls[r]] = q[(Sl + kR) % L][r];
#pragma unroll
        for (int k = 0; k < HPT; ++k) s[hl[k]] = hh[Sl % NR][k];
        __syncthreads();
      }
      const uint32_t so = (uint32_t)(kz - ZD) * pe, so4 = (uint32_t)(kz - ZD) * p4;
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        const float c = q[(Sl + kR) % L][r];  // u(z)
        float xy = 0.0f, gxy = 0.0f;
        if (stage) {
          const float* row = s + sl.ls[r];
          xy = a.c[0] * c;
#pragma unroll
          for (int m = 1; m <= kR; ++m) xy = __builtin_fmaf(a.c[m], row[m] + row[-m], xy);
#pragma unroll
          for (int m = 1; m <= kR; ++m)
            xy = __builtin_fmaf(a.c[4 + m], row[m * LW] + row[-m * LW], xy);
          if (LAYER) {
            gxy = dqx[r] * (row[1] - row[-1]);
            gxy = __builtin_fmaf(dqy[r], row[LW] - row[-LW], gxy);
          }
        }
        // backward phase: u(z) is the +m neighbour of the outputs z - m
        A[(Sl + 3) % 4][r] = __builtin_fmaf(a.c[9], c, A[(Sl + 3) % 4][r]);
        A[(Sl + 2) % 4][r] = __builtin_fmaf(a.c[10], c, A[(Sl + 2) % 4][r]);
        A[(Sl + 1) % 4][r] = __builtin_fmaf(a.c[11], c, A[(Sl + 1) % 4][r]);
        A[Sl % 4][r] = __builtin_fmaf(a.c[12], c, A[Sl % 4][r]);
        if (LAYER)  // z part of the phi gradient of plane z - 1
          G[(Sl + 3) % 4][r] =
              __builtin_fmaf(dz1, c - q[(Sl + kR - 2) % L][r], G[(Sl + 3) % 4][r]);
        if (emit) {
          const float cz = q[Sl % L][r];  // u(z - 4)
          const float lap = __builtin_fmaf(a.ce, cz, A[Sl % 4][r]);
          const float pu = pv[B][r];
          const float vp = vv[B][r];
          float res;
          if (LAYER) {
            const float e = sl.lay[r] ? (float)(a.dt * (tsc[r] + tzr[B])) : 0.0f;
            const float phv = sl.lay[r] ? ph[B][r] : 0.0f;
            res = upd_layer(cz, pu, vp, lap, e, phv);
            const float nph = (phv - G[Sl % 4][r]) / (1.0f + e);
            bst_f32(rph, fo[r], so4, sl.lay[r] ? nph : ph[B][r]);
          } else {
            res = upd_inner(cz, pu, vp, lap);
          }
          store_u(r, so, res, z - ZD);
        }
        if (stage) {
          A[Sl % 4][r] = xy + F[Sl % 4][r];
          if (LAYER) G[Sl % 4][r] = gxy;
        }
        // forward phase: u(z) is the -m neighbour of the outputs z + m
        F[Sl % 4][r] = a.c[12] * c;
        F[(Sl + 3) % 4][r] = __builtin_fmaf(a.c[11], c, F[(Sl + 3) % 4][r]);
        F[(Sl + 2) % 4][r] = __builtin_fmaf(a.c[10], c, F[(Sl + 2) % 4][r]);
        F[(Sl + 1) % 4][r] = __builtin_fmaf(a.c[9], c, F[(Sl + 1) % 4][r]);
      }
    } else {
      // stage the centre plane and its halo
      float* s = sm[LB];
  #pragma unroll
      for (int r = 0; r < RY; ++r) s[sl.ls[r]] = q[(Sl + kR) % L][r];
  #pragma unroll
      for (int k = 0; k < HPT; ++k) s[hl[k]] = hh[B][k];
      __syncthreads();

      const uint32_t sz = (uint32_t)kz * pe, sz4 = (uint32_t)kz * p4;
  #pragma unroll
      for (int r = 0; r < RY; ++r) {
        const float* row = s + sl.ls[r];
        const float c = q[(Sl + kR) % L][r];
        float xp[kR], xm[kR];
        if constexpr (XS) {
          xshuffle(c, hx[B][r], xp, xm);
        } else {
  #pragma unroll
          for (int m = 0; m < kR; ++m) {
            xp[m] = row[m + 1];
            xm[m] = row[-(m + 1)];
          }
        }
        float lap = a.c[0] * c;
  #pragma unroll
        for (int m = 1; m <= kR; ++m) lap = __builtin_fmaf(a.c[m], xp[m - 1] + xm[m - 1], lap);
  #pragma unroll
        for (int m = 1; m <= kR; ++m)
          lap = __builtin_fmaf(a.c[4 + m], row[m * LW] + row[-m * LW], lap);
  #pragma unroll
        for (int m = 1; m <= kR; ++m)
          lap = __builtin_fmaf(a.c[8 + m], q[(Sl + kR + m) % L][r] + q[(Sl + kR - m) % L][r], lap);
        lap = __builtin_fmaf(a.ce, c, lap);
        const float pu = pv[B][r];
        const float vp = vv[B][r];
        float res;
        if (LAYER) {
          float e, gx, gy, gz;
          if (EARR) {
            e = er[(Sl + 1) % NE][r];
            gx = (ex1[B][r] - ex0[B][r]) * a.q[0];
            gy = (ey1[B][r] - ey0[B][r]) * a.q[1];
            gz = (er[(Sl + 2) % NE][r] - er[Sl % NE][r]) * a.q[2];
          } else {
            // table mode: non-layer points take eta = 0 like the array mode's
            // out-of-range loads (their phi' is dropped, so gx..gz do not
            // matter there)
            e = sl.lay[r] ? (float)(a.dt * (tsc[r] + tzr[B])) : 0.0f;
            gx = dqx[r];
            gy = dqy[r];
            gz = dzr[B];
          }
          // phi of a point outside the layer counts as 0 (the loaded value is
          // only written back)
          const float phv = sl.lay[r] ? ph[B][r] : 0.0f;
          res = upd_layer(c, pu, vp, lap, e, phv);
          const float nph = upd_phi(phv, e, gx, xp[0] - xm[0], gy, row[LW] - row[-LW], gz,
                                    q[(Sl + kR + 1) % L][r] - q[(Sl + kR - 1) % L][r]);
          // stored for every point; points where phi is not touched have an
          // out-of-range offset, so their store is dropped
          bst_f32(rph, fo[r], sz4, sl.lay[r] ? nph : ph[B][r]);
        } else {
          res = upd_inner(c, pu, vp, lap);
        }
        // points past the grid have an out-of-range offset: no branch around
        // the store
        store_u(r, sz, res, z);
      }
    }
  };

  using std::integral_constant;
  static_assert(L == 10 || L == 12 || L == 16, "unrolled loop below covers ring lengths 10, 12, 16");
  for (int z = zb; z < ze + ZD; z += L) {
#define WAVE_BODY(J)                                   \
  if constexpr ((J) < L) {                             \
    if ((J) > 0 && z + (J) >= ze + ZD) break;          \
    body(integral_constant<int, (J) % L>{}, z + (J));  \
  }
    WAVE_BODY(0) WAVE_BODY(1) WAVE_BODY(2) WAVE_BODY(3) WAVE_BODY(4) WAVE_BODY(5)
    WAVE_BODY(6) WAVE_BODY(7) WAVE_BODY(8) WAVE_BODY(9) WAVE_BODY(10) WAVE_BODY(11)
    WAVE_BODY(12) WAVE_BODY(13) WAVE_BODY(14) WAVE_BODY(15)
#undef WAVE_BODY
  }
}

// EA: the kernel instance also serves contexts with a per-point eta array
// (its loop holds more registers; contexts with the default profile's tables
// run instances without it).
template <class S, int RY, int NW, bool ZS = false, bool EA = false, bool XS = false>
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

  // Lanes of a tile that holds an x wall of the layer are laid out as 32
  // columns x 2 rows per wavefront: the first half of the wavefronts takes
  // the tile's left 32 columns, the second half its right 32, so a wall of
  // up to 32 cells lands in half the wavefronts and the other half run the
  // inner loop (with 64 x 1 every wavefront of such a tile would take the
  // layer loop).  The halves are the first and the last NW/2 wavefronts, so
  // SIMDs that take a workgroup's wavefronts in turn get as many of either.
  // Other tiles keep one row per wavefront.
  const bool split = (NW % 2 == 0) && damp && !cap && a.w > 0 &&
                     (x0 < a.w || x0 + kTX > a.nx - a.w);
  const int hw = NW / 2;
  Slots<RY> sl;
  bool any_lay = false;
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int col = split ? (wv / hw) * 32 + (lane & 31) : lane;
    const int row = split ? (wv % hw) * 2 * RY + 2 * r + (lane >> 5) : wv * RY + r;
    const int x = x0 + col, y = y0 + row;
    sl.x[r] = min(x, a.nx - 1);
    sl.y[r] = min(y, a.ny - 1);
    sl.valid[r] = x < a.nx && y < a.ny;
    sl.ro[r] = (uint32_t)((min(y, ylast) + kR) * P + x);
    sl.ls[r] = (kR + row) * LW + kR + col;
    sl.lay[r] = damp && sl.valid[r] &&
                (cap || y < a.w || y >= a.ny - a.w || x < a.w || x >= a.nx - a.w);
    // the x walls' phi rows are widened to whole 128-byte lines (32 floats
    // from x = 0, which is line-aligned): full-line writes instead of
    // partial ones, which the memory would have to merge
    sl.phl[r] = sl.lay[r] || (damp && sl.valid[r] && a.w > 0 &&
                              (x < ((a.w + 31) & ~31) || x >= ((a.nx - a.w) & ~31)));
    any_lay = any_lay || sl.lay[r];
    if (XS) {
      // the x-halo cell this lane loads for its row segment
      sl.xw = split ? 32 : 64;
      sl.xli = col & (sl.xw - 1);
      const int xs0 = x - sl.xli;  // first column of the segment
      const int xh = sl.xli < kR ? xs0 + sl.xw + sl.xli
                     : sl.xli >= sl.xw - kR ? xs0 - kR + (sl.xli - (sl.xw - kR))
                                            : -1;
      sl.xho[r] = (xh < 0 || xh >= a.nx || y >= a.ny) ? kHaloGhost
                                                       : (uint32_t)((y + kR) * P + xh);
    }
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
    // ghost cells (outside the grid) and the dump row are zero or unused:
    // no load (a line of row padding would be fetched for 16 bytes); with
    // XS the x halo is not staged (the row segments load it themselves)
    const bool ghost = h >= NHALO || gx < 0 || gx >= a.nx || gy < 0 || gy >= a.ny ||
                       (XS && h >= NYH);
    gy = min(gy, ylast);
    hl[k] = rl * LW + cl;
    ho[k] = ghost ? kHaloGhost : (uint32_t)((gy + kR) * P + gx);
  }

  // wavefront-uniform choice of the loop
  if (!__any(any_lay))
    stream_loop<S, RY, NW, 0, ZS, XS>(a, sm, sl, hl, ho, zb, ze);
  else if (!EA || a.etab)
    stream_loop<S, RY, NW, 2, ZS, XS>(a, sm, sl, hl, ho, zb, ze);
  else
    stream_loop<S, RY, NW, EA && !ZS ? 1 : 2, ZS, XS>(a, sm, sl, hl, ho, zb, ze);
}

// Occupancy: one-row tiles and 16-wavefront workgroups run 4 wavefronts per
// SIMD (at most 128 VGPRs), the other two-row tiles 2.
#define WAVE_STREAM_WPS(RY, NW) ((RY) == 1 || (NW) == 16 ? WAVE_STREAM_WAVES_PER_SIMD : 2)

// Occupancy target in wavefronts per SIMD for one-row tiles.
#ifndef WAVE_STREAM_WAVES_PER_SIMD
#define WAVE_STREAM_WAVES_PER_SIMD 4
#endif
template <class S, int RY, int NW, bool ZS = false, bool EA = false, bool XS = false>
__global__ __launch_bounds__(64 * NW, WAVE_STREAM_WPS(RY, NW)) void k_sweep_stream(
    SweepArgs a, int tiles_x, int tiles_y, int zchunk) {
  constexpr int TY = RY * NW;
  constexpr int LSZ = (TY + 2 * kR) * (kTX + 2 * kR) + 64;  // + a dump row
  __shared__ float sm[2][LSZ];

  // XCD-aware tile order (tile_at)
  const TileAt t = tile_at(blockIdx.x, tiles_x, tiles_y);
  if (t.ty >= tiles_y) return;
  const bool damp = a.damping != 0;
  const ChunkInfo c = chunk_of(t.ch, a.nz, a.w, zchunk, damp);
  if (c.zb >= c.ze) return;
  stream_tile<S, RY, NW, ZS, EA, XS>(a, sm, t.tx * kTX, t.ty * TY, c.zb, c.ze, damp && c.cap);
}

// The same sweep as one persistent launch: 8 G workgroups (G per XCD, one
// per CU), each sweeping a fixed list of work items -- the (tile, z chunk)
// pairs that k_sweep_stream runs as workgroups -- one after the other.
// Items keep k_sweep_stream's order and XCD, except that an XCD's slab of
// tile rows moves on every second z chunk instead of every chunk (tile_at
// with hold 1: a chunk's warm-up planes are then still in the XCD's L2 from
// the chunk before; measured 1 % faster at 512^3).  The items of workgroup
// b's XCD (b mod 8) are the blocks 8 s + b mod 8, s = 0, 1, ..  They are dealt out
// in rounds of G: in round k, workgroup g = b / 8 takes s = k G +
// (g + 5 k) mod G, so that over the rounds every workgroup meets every tile
// position of a row (5 is coprime to the 8 of a tile row of a 512-wide
// grid): wall tiles, which take longer, do not all land on the same
// workgroups.  Each tile is swept by the same code as in k_sweep_stream, so
// results are the same bit for bit.  No workgroup waits for the end of
// another to start its next tile, and no atomics are needed.
template <class S, int RY, int NW, bool EA = false>
__global__ __launch_bounds__(64 * NW, WAVE_STREAM_WPS(RY, NW)) void k_sweep_persist(
    SweepArgs a, int tiles_x, int tiles_y, int zchunk) {
  constexpr int TY = RY * NW;
  constexpr int LSZ = (TY + 2 * kR) * (kTX + 2 * kR) + 64;
  __shared__ float sm[2][LSZ];
  const int xcd = blockIdx.x & 7;
  const int g = blockIdx.x >> 3;
  const int G = gridDim.x >> 3;
  const int sh = (tiles_y + 7) >> 3;  // tile rows per slab (tile_at)
  const bool damp = a.damping != 0;
  const int items = tiles_x * sh * chunk_count(a.nz, a.w, zchunk, damp);
  for (int k = 0; k * G < items; ++k) {
    const int slot = k * G + (g + 5 * k) % G;
    if (slot >= items) continue;
    const TileAt t = tile_at(8 * (int64_t)slot + xcd, tiles_x, tiles_y, 1);
    const ChunkInfo c = chunk_of(t.ch, a.nz, a.w, zchunk, damp);
    if (t.ty >= tiles_y || c.zb >= c.ze) continue;
    stream_tile<S, RY, NW, false, EA>(a, sm, t.tx * kTX, t.ty * TY, c.zb, c.ze, damp && c.cap);
    __syncthreads();  // the next tile's staging reuses the LDS planes
  }
}

// ---- many shots per launch ---------------------------------------------------
// One workgroup grid covers every member of a batch: the workgroup index is
// located in the members' block ranges, the member's parity picks u^n and
// u^{n-1}, and the tile is swept exactly as in a single-shot launch.  Members that have taken their steps for this run exit
// at once, so a captured sequence of launches stays valid as members finish.
template <class S, int RY, int NW, bool EA = false>
__global__ __launch_bounds__(64 * NW, WAVE_STREAM_WPS(RY, NW)) void k_sweep_batch(
    const BatchShot* __restrict__ shots, const BatchState* __restrict__ state, int nshots) {
  constexpr int TY = RY * NW;
  constexpr int LSZ = (TY + 2 * kR) * (kTX + 2 * kR) + 64;
  __shared__ float sm[2][LSZ];
  const int64_t bid = blockIdx.x;
  const int m = batch_member(shots, nshots, bid);
  const BatchShot& b = shots[m];
  const BatchState st = state[m];
  if (st.done >= b.target) return;
  SweepArgs a = b.sa;
  a.cur = b.u[st.cur];
  a.nxt = b.u[st.cur ^ 1];
  a.step = st.step;
  // each member's range starts at a multiple of 8 blocks, so the member-local
  // index keeps the XCD in its low 3 bits; tiles follow the single-shot order
  const TileAt t = tile_at(bid - b.block_begin, b.tiles_x, b.tiles_y);
  if (t.ty >= b.tiles_y) return;
  const bool damp = a.damping != 0;
  const ChunkInfo c = chunk_of(t.ch, a.nz, a.w, b.zchunk, damp);
  if (c.zb >= c.ze) return;
  stream_tile<S, RY, NW, false, EA>(a, sm, t.tx * kTX, t.ty * TY, c.zb, c.ze, damp && c.cap);
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

// ---- set-up: compact host-order field -> padded layout --------------------------
// dst points at element (0, 0, 0) of a padded array.  With dt > 0 the value
// stored is vp = fl32((v dt)^2) formed in double (Eq. 2's dt^2 V^2),
// otherwise the value itself.
__global__ __launch_bounds__(256) void k_setup_field(float* __restrict__ dst,
                                                     const float* __restrict__ src, int nx,
                                                     int ny, int64_t n, int pitch, int64_t plane,
                                                     double dt) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += stride) {
    const int64_t i = p % nx, r = p / nx;
    const int64_t j = r % ny, k = r / ny;
    const float v = src[p];
    float o = v;
    if (dt > 0.0) {
      const double s = (double)v * dt;
      o = (float)(s * s);
    }
    dst[k * plane + j * pitch + i] = o;
  }
}

// ---- plain copy (bandwidth reference) -------------------------------------------
// One 16-byte word per thread (measured as fast as any of the shapes tried:
// several words per thread, non-temporal hints, 4-byte words; about 6.1 TB/s
// for 2 GiB).
__global__ __launch_bounds__(256) void k_stream_copy(const float4* __restrict__ s,
                                                     float4* __restrict__ d, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) d[i] = s[i];
}

// Plain streams with other access mixes (the measured ceilings an access
// pattern can reach): read only (a sum that is stored only if it hits an
// impossible value, which keeps the loads), and three reads with one write,
// the mix of an inner point of the sweep (u^n, u^{n-1}, vp in; u^{n+1} out).
__global__ __launch_bounds__(256) void k_stream_read(const float4* __restrict__ s,
                                                     float* __restrict__ sink, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const float4 v = i < n ? s[i] : float4{0.0f, 0.0f, 0.0f, 0.0f};
  const float t = (v.x + v.y) + (v.z + v.w);
  if (t == -1.5e38f) sink[0] = t;
}
__global__ __launch_bounds__(256) void k_stream_mix31(const float4* __restrict__ a,
                                                      const float4* __restrict__ b,
                                                      const float4* __restrict__ c,
                                                      float4* __restrict__ d, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    const float4 x = a[i], y = b[i], z = c[i];
    d[i] = float4{__builtin_fmaf(y.x, z.x, x.x), __builtin_fmaf(y.y, z.y, x.y),
                  __builtin_fmaf(y.z, z.z, x.z), __builtin_fmaf(y.w, z.w, x.w)};
  }
}

template <class S>
hipError_t sweep_direct_t(const SweepArgs& a, hipStream_t st) {
  dim3 block(kTX, 4, 1);
  dim3 grid((a.nx + kTX - 1) / kTX, (a.ny + 3) / 4, a.nz);
  hipLaunchKernelGGL(k_sweep_direct<S>, grid, block, 0, st, a);
  return hipGetLastError();
}

template <class S, int RY, int NW, bool ZS = false, bool EA = false, bool XS = false>
hipError_t sweep_stream_t(const SweepArgs& a, int zchunk, hipStream_t st) {
  constexpr int TY = RY * NW;
  const int tiles_x = (a.nx + kTX - 1) / kTX;
  const int tiles_y = (a.ny + TY - 1) / TY;
  if (zchunk > stream_zchunk_limit(a.plane)) return hipErrorInvalidValue;
  const int chunks = chunk_count(a.nz, a.w, zchunk, a.damping != 0);
  // tile rows padded to a multiple of 8 (see k_sweep_stream)
  const int64_t blocks = (int64_t)tiles_x * 8 * ((tiles_y + 7) / 8) * chunks;
  if (blocks <= 0 || blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_sweep_stream<S, RY, NW, ZS, EA, XS>), dim3((unsigned)blocks), dim3(64 * NW),
                     0, st, a, tiles_x, tiles_y, zchunk);
  return hipGetLastError();
}

template <class S, int RY, int NW, bool EA = false>
hipError_t sweep_persist_t(const SweepArgs& a, int zchunk, int groups, hipStream_t st) {
  constexpr int TY = RY * NW;
  const int tiles_x = (a.nx + kTX - 1) / kTX;
  const int tiles_y = (a.ny + TY - 1) / TY;
  if (zchunk > stream_zchunk_limit(a.plane) || groups < 8 || groups % 8 != 0)
    return hipErrorInvalidValue;
  const int chunks = chunk_count(a.nz, a.w, zchunk, a.damping != 0);
  const int64_t blocks = (int64_t)tiles_x * 8 * ((tiles_y + 7) / 8) * chunks;
  if (blocks <= 0 || blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_sweep_persist<S, RY, NW, EA>), dim3((unsigned)groups), dim3(64 * NW), 0, st,
                     a, tiles_x, tiles_y, zchunk);
  return hipGetLastError();
}

template <class S>
hipError_t sweep_stream_s(const SweepArgs& a, int ry, int nw, int zchunk, hipStream_t st) {
  if (a.eta) {  // a per-point eta array
    if (ry == 1 && nw == 16) return sweep_stream_t<S, 1, 16, false, true>(a, zchunk, st);
    if (ry == 1 && nw == 8) return sweep_stream_t<S, 1, 8, false, true>(a, zchunk, st);
    if (ry == 2 && nw == 8) return sweep_stream_t<S, 2, 8, false, true>(a, zchunk, st);
    if (ry == 2 && nw == 4) return sweep_stream_t<S, 2, 4, false, true>(a, zchunk, st);
    return hipErrorInvalidValue;
  }
  if (ry == 1 && nw == 16) return sweep_stream_t<S, 1, 16>(a, zchunk, st);
  if (ry == 1 && nw == 8) return sweep_stream_t<S, 1, 8>(a, zchunk, st);
  if (ry == 2 && nw == 8) return sweep_stream_t<S, 2, 8>(a, zchunk, st);
  if (ry == 2 && nw == 4) return sweep_stream_t<S, 2, 4>(a, zchunk, st);
  if (ry == 2 && nw == 16) return sweep_stream_t<S, 2, 16>(a, zchunk, st);
  return hipErrorInvalidValue;
}

}  // namespace

bool stream_config_supported(int ry, int nw, bool eta_array) {
  return (ry == 1 && nw == 16) || (ry == 1 && nw == 8) || (ry == 2 && nw == 8) ||
         (ry == 2 && nw == 4) || (ry == 2 && nw == 16 && !eta_array);
}

int stream_zchunk_limit(int64_t plane) {
  const int64_t z = kWindowMax / (plane * 4) - 2 * kR;
  return (int)std::min<int64_t>(z, 1 << 30);
}

int auto_zchunk(int nx, int ny, int nz, int ry, int nw) {
  // 64 planes (the measured optimum at 512^3 and 1024^3 with the slab tile
  // order), shortened when the grid would have fewer than ~2048 workgroups,
  // but at least 32 planes so a chunk's 8-plane warm-up stays a modest cost.
  const int64_t tiles = (int64_t)((nx + kTX - 1) / kTX) * ((ny + ry * nw - 1) / (ry * nw));
  const int64_t chunks = (2048 + tiles - 1) / tiles;
  int zc = (int)std::min<int64_t>(64, (nz + chunks - 1) / chunks);
  zc = std::max(zc, 32);
  return std::min(zc, nz);
}

hipError_t launch_sweep_direct(const SweepArgs& a, int storage, hipStream_t s) {
  switch (storage) {
    case 0: return sweep_direct_t<StF32>(a, s);
    case 1: return sweep_direct_t<StBF16>(a, s);
    case 2: return sweep_direct_t<StF16>(a, s);
    case 3: return sweep_direct_t<StBF16SR>(a, s);
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
    case 3: return sweep_stream_s<StBF16SR>(a, ry, nw, zchunk, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sweep_persist(const SweepArgs& a, int storage, int ry, int nw, int zchunk,
                                int groups, hipStream_t s) {
  if (zchunk <= 0) return hipErrorInvalidValue;
#define WAVE_PERSIST_CASE(S_)                                                              \
  if (a.eta) {                                                                               \
    if (ry == 1 && nw == 16) return sweep_persist_t<S_, 1, 16, true>(a, zchunk, groups, s);  \
    if (ry == 1 && nw == 8) return sweep_persist_t<S_, 1, 8, true>(a, zchunk, groups, s);    \
    return hipErrorInvalidValue;                                                             \
  }                                                                                          \
  if (ry == 1 && nw == 16) return sweep_persist_t<S_, 1, 16>(a, zchunk, groups, s);          \
  if (ry == 1 && nw == 8) return sweep_persist_t<S_, 1, 8>(a, zchunk, groups, s);            \
  return hipErrorInvalidValue;
  switch (storage) {
    case 0: { WAVE_PERSIST_CASE(StF32) }
    case 1: { WAVE_PERSIST_CASE(StBF16) }
    case 2: { WAVE_PERSIST_CASE(StF16) }
    case 3: { WAVE_PERSIST_CASE(StBF16SR) }
  }
#undef WAVE_PERSIST_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_sweep_shuffle(const SweepArgs& a, int storage, int nw, int zchunk, hipStream_t s) {
  if (zchunk <= 0 || (nw != 8 && nw != 16)) return hipErrorInvalidValue;
#define WAVE_XS_CASE(S_)                                                                  \
  if (a.eta)                                                                              \
    return nw == 16 ? sweep_stream_t<S_, 1, 16, false, true, true>(a, zchunk, s)          \
                    : sweep_stream_t<S_, 1, 8, false, true, true>(a, zchunk, s);          \
  return nw == 16 ? sweep_stream_t<S_, 1, 16, false, false, true>(a, zchunk, s)           \
                  : sweep_stream_t<S_, 1, 8, false, false, true>(a, zchunk, s);
  switch (storage) {
    case 0: { WAVE_XS_CASE(StF32) }
    case 1: { WAVE_XS_CASE(StBF16) }
    case 2: { WAVE_XS_CASE(StF16) }
    case 3: { WAVE_XS_CASE(StBF16SR) }
  }
#undef WAVE_XS_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_sweep_semi(const SweepArgs& a, int storage, int nw, int zchunk, hipStream_t s) {
  if (zchunk <= 0 || (nw != 8 && nw != 16)) return hipErrorInvalidValue;
  if (a.damping && !a.etab) return hipErrorInvalidValue;  // eta arrays: not in this kernel
#define WAVE_SEMI_CASE(S_)                                                      \
  return nw == 16 ? sweep_stream_t<S_, 1, 16, true>(a, zchunk, s)               \
                  : sweep_stream_t<S_, 1, 8, true>(a, zchunk, s);
  switch (storage) {
    case 0: WAVE_SEMI_CASE(StF32)
    case 1: WAVE_SEMI_CASE(StBF16)
    case 2: WAVE_SEMI_CASE(StF16)
    case 3: WAVE_SEMI_CASE(StBF16SR)
  }
#undef WAVE_SEMI_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_inject_record(const InjectArgs& a, int storage, hipStream_t s) {
  switch (storage) {
    case 0: hipLaunchKernelGGL(k_inject_record<StF32>, dim3(1), dim3(256), 0, s, a); break;
    case 1: hipLaunchKernelGGL(k_inject_record<StBF16>, dim3(1), dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_inject_record<StF16>, dim3(1), dim3(256), 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_inject_record<StBF16SR>, dim3(1), dim3(256), 0, s, a); break;
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
    case 3: hipLaunchKernelGGL(k_energy_rows<StBF16SR>, grid, dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(1024), 0, s, a.partial,
                     (int64_t)a.ny * a.nz, a.result);
  return hipGetLastError();
}

hipError_t launch_setup_field(float* dst, const float* src, int nx, int ny, int nz, int pitch,
                              int64_t plane, double dt, hipStream_t s) {
  const int64_t n = (int64_t)nx * ny * nz;
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_setup_field, dim3((unsigned)blocks), dim3(256), 0, s, dst, src, nx, ny, n,
                     pitch, plane, dt);
  return hipGetLastError();
}

hipError_t launch_stream_mix(int kind, void* d, const void* a, const void* b, const void* c,
                             size_t bytes, hipStream_t s) {
  const int64_t n = (int64_t)(bytes / 16);
  if (n == 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (kind == 0)
    hipLaunchKernelGGL(k_stream_read, dim3((unsigned)blocks), dim3(256), 0, s,
                       static_cast<const float4*>(a), static_cast<float*>(d), n);
  else
    hipLaunchKernelGGL(k_stream_mix31, dim3((unsigned)blocks), dim3(256), 0, s,
                       static_cast<const float4*>(a), static_cast<const float4*>(b),
                       static_cast<const float4*>(c), static_cast<float4*>(d), n);
  return hipGetLastError();
}

hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const int64_t n = (int64_t)(bytes / 16);
  if (n == 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
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
                         int ry, int nw, bool eta_array, hipStream_t st) {
  if (blocks <= 0 || blocks > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 g((unsigned)blocks);
#define WAVE_BATCH_CASE(RY_, NW_, EA_)                                                           \
  if (ry == RY_ && nw == NW_ && eta_array == EA_) {                                              \
    hipLaunchKernelGGL((k_sweep_batch<S, RY_, NW_, EA_>), g, dim3(64 * NW_), 0, st, shots, state, \
                       nshots);                                                                  \
    return hipGetLastError();                                                                    \
  }
  WAVE_BATCH_CASE(1, 16, false)
  WAVE_BATCH_CASE(1, 8, false)
  WAVE_BATCH_CASE(2, 8, false)
  WAVE_BATCH_CASE(2, 4, false)
  WAVE_BATCH_CASE(2, 16, false)
  WAVE_BATCH_CASE(1, 16, true)
  WAVE_BATCH_CASE(1, 8, true)
  WAVE_BATCH_CASE(2, 8, true)
  WAVE_BATCH_CASE(2, 4, true)
#undef WAVE_BATCH_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_sweep_batch(const BatchShot* shots, BatchState* state, int nshots,
                              int64_t total_blocks, int storage, int ry, int nw, bool eta_array,
                              hipStream_t s) {
  switch (storage) {
    case 0: return sweep_batch_s<StF32>(shots, state, nshots, total_blocks, ry, nw, eta_array, s);
    case 1: return sweep_batch_s<StBF16>(shots, state, nshots, total_blocks, ry, nw, eta_array, s);
    case 2: return sweep_batch_s<StF16>(shots, state, nshots, total_blocks, ry, nw, eta_array, s);
    case 3: return sweep_batch_s<StBF16SR>(shots, state, nshots, total_blocks, ry, nw, eta_array, s);
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
    case 3: hipLaunchKernelGGL(k_inject_batch<StBF16SR>, dim3(nshots), dim3(256), 0, s, shots, state); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace wave

