// wave_shapes.hip -- the paper's other code shapes for one sweep (Sec. IV:
// 3-D tiles whose threads read every stencil operand from global memory, the
// 2.5-D ring of 2R+1 shared planes, and the 2.5-D shared plane with a shifted
// register queue along z), written for gfx950 so that they can be timed
// beside the streaming kernel of wave_kernels.hip (Table II's comparison).
// Every point is evaluated with the operations of wave_direct.h in the same
// order, so all shapes give identical fields.
#include <algorithm>

#include "wave_direct.h"
#include "wave_internal.h"
#include "wave_point.h"

namespace wave {
namespace {

// ---- 3-D tiles: one thread per point, every operand from memory ---------------
template <class S, int BX, int BY, int BZ>
__global__ __launch_bounds__(BX * BY * BZ) void k_sweep_gmem(SweepArgs a) {
  const int x = blockIdx.x * BX + threadIdx.x;
  const int y = blockIdx.y * BY + threadIdx.y;
  const int z = blockIdx.z * BZ + threadIdx.z;
  if (x >= a.nx || y >= a.ny || z >= a.nz) return;
  direct_point<S>(a, x, y, z);
}

template <class S, int BX, int BY, int BZ>
hipError_t gmem_t(const SweepArgs& a, hipStream_t st) {
  const dim3 grid((a.nx + BX - 1) / BX, (a.ny + BY - 1) / BY, (a.nz + BZ - 1) / BZ);
  if (grid.y > 65535 || grid.z > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_sweep_gmem<S, BX, BY, BZ>), grid, dim3(BX, BY, BZ), 0, st, a);
  return hipGetLastError();
}

// ---- 2.5-D shapes: a 64 x TY tile streamed through a chunk of z planes ----------
// Staged planes cover the tile plus a 4-cell halo: (TY + 8) rows of 72
// columns.  Element e of a staged plane is (x0 - 4 + e % 72, y0 - 4 + e / 72);
// rows below the grid's last ghost row are clamped to it (their values only
// feed points outside the grid, whose results are discarded), columns stay in
// the padded row or the next row's leading ghosts.
constexpr int kSW3 = kTX + 2 * kR;

template <int TY>
struct Tile25 {
  int x0, y0, zb, ze;
};

template <int TY>
__device__ __forceinline__ Tile25<TY> tile25(const SweepArgs& a, int tiles_x, int tiles_y,
                                             int zchunk) {
  const int b = blockIdx.x;
  const int tx = b % tiles_x, t2 = b / tiles_x;
  const int ty = t2 % tiles_y, ch = t2 / tiles_y;
  Tile25<TY> t;
  t.x0 = tx * kTX;
  t.y0 = ty * TY;
  t.zb = ch * zchunk;
  t.ze = min(a.nz, t.zb + zchunk);
  return t;
}

__device__ __forceinline__ int64_t staged_elem(const SweepArgs& a, int x0, int y0, int z, int e) {
  const int r = e / kSW3, c = e % kSW3;
  const int y = min(y0 - kR + r, a.ny + kR - 1);
  return (int64_t)z * a.plane + (int64_t)y * a.pitch + (x0 - kR + c);
}

// st_smem: a ring of 2R+1 staged planes in LDS; every neighbour (x, y and z)
// is read from the ring.  Per plane: stage plane z+4 into the slot of plane
// z-5, barrier, compute plane z, barrier (the next plane overwrites the slot
// of plane z-4).
template <class S, int TY>
__global__ __launch_bounds__(64 * TY) void k_sweep_ring(SweepArgs a, int tiles_x, int tiles_y,
                                                      int zchunk) {
  using T = typename S::T;
  constexpr int PL = (TY + 2 * kR) * kSW3;
  constexpr int NR = 2 * kR + 1;
  constexpr int NT = 64 * TY;
  __shared__ float ring[NR][PL];
  const Tile25<TY> t = tile25<TY>(a, tiles_x, tiles_y, zchunk);
  if (t.zb >= t.ze) return;
  const T* u = static_cast<const T*>(a.cur);
  const int tid = threadIdx.y * 64 + threadIdx.x;
  auto slot = [](int z) { return (z + NR) % NR; };  // z >= -4
  auto stage = [&](int z) {
    float* dst = ring[slot(z)];
    for (int e = tid; e < PL; e += NT) dst[e] = S::ld(u, staged_elem(a, t.x0, t.y0, z, e));
  };
  for (int z = t.zb - kR; z < t.zb + kR; ++z) stage(z);
  const int x = t.x0 + threadIdx.x, y = t.y0 + threadIdx.y;
  const bool valid = x < a.nx && y < a.ny;
  const int ci = (threadIdx.y + kR) * kSW3 + threadIdx.x + kR;
  for (int z = t.zb; z < t.ze; ++z) {
    stage(z + kR);
    __syncthreads();
    if (valid) {
      const float* s0 = ring[slot(z)];
      const float c = s0[ci];
      float lap = a.c[0] * c;
#pragma unroll
      for (int m = 1; m <= kR; ++m) lap = __builtin_fmaf(a.c[m], s0[ci + m] + s0[ci - m], lap);
#pragma unroll
      for (int m = 1; m <= kR; ++m)
        lap = __builtin_fmaf(a.c[4 + m], s0[ci + m * kSW3] + s0[ci - m * kSW3], lap);
#pragma unroll
      for (int m = 1; m <= kR; ++m)
        lap = __builtin_fmaf(a.c[8 + m], ring[slot(z + m)][ci] + ring[slot(z - m)][ci], lap);
      lap = __builtin_fmaf(a.ce, c, lap);
      const int64_t p = (int64_t)z * a.plane + (int64_t)y * a.pitch + x;
      point_tail<S>(a, x, y, z, p, c, lap, s0[ci + 1] - s0[ci - 1], s0[ci + kSW3] - s0[ci - kSW3],
                    ring[slot(z + 1)][ci] - ring[slot(z - 1)][ci]);
    }
    __syncthreads();
  }
}

// st_reg_shft: one staged plane in LDS for the x and y neighbours; the 2R+1
// values of the own column along z sit in registers and shift by one each
// plane.  The plane's interior comes from the registers, the halo frame from
// memory.
template <class S, int TY>
__global__ __launch_bounds__(64 * TY) void k_sweep_shift(SweepArgs a, int tiles_x, int tiles_y,
                                                       int zchunk) {
  using T = typename S::T;
  constexpr int H = TY + 2 * kR;
  constexpr int NT = 64 * TY;
  constexpr int NF = 2 * kR * kSW3 + TY * 2 * kR;  // halo frame elements
  __shared__ float pl[H * kSW3];
  const Tile25<TY> t = tile25<TY>(a, tiles_x, tiles_y, zchunk);
  if (t.zb >= t.ze) return;
  const T* u = static_cast<const T*>(a.cur);
  const int tid = threadIdx.y * 64 + threadIdx.x;
  const int x = t.x0 + threadIdx.x, y = t.y0 + threadIdx.y;
  const bool valid = x < a.nx && y < a.ny;
  const int ci = (threadIdx.y + kR) * kSW3 + threadIdx.x + kR;
  const int64_t col = (int64_t)min(y, a.ny + kR - 1) * a.pitch + x;  // own column
  float qz[2 * kR + 1];
#pragma unroll
  for (int j = 0; j < 2 * kR; ++j) qz[j] = S::ld(u, (int64_t)(t.zb - kR + j) * a.plane + col);
  for (int z = t.zb; z < t.ze; ++z) {
    qz[2 * kR] = S::ld(u, (int64_t)(z + kR) * a.plane + col);
    pl[ci] = qz[kR];
    for (int f = tid; f < NF; f += NT) {
      int e;
      if (f < 2 * kR * kSW3) {
        const int r = f / kSW3;
        e = (r < kR ? r : TY + r) * kSW3 + f % kSW3;
      } else {
        const int g = f - 2 * kR * kSW3, cc = g % (2 * kR);
        e = (kR + g / (2 * kR)) * kSW3 + (cc < kR ? cc : kTX + cc);
      }
      pl[e] = S::ld(u, staged_elem(a, t.x0, t.y0, z, e));
    }
    __syncthreads();
    if (valid) {
      const float c = qz[kR];
      float lap = a.c[0] * c;
#pragma unroll
      for (int m = 1; m <= kR; ++m) lap = __builtin_fmaf(a.c[m], pl[ci + m] + pl[ci - m], lap);
#pragma unroll
      for (int m = 1; m <= kR; ++m)
        lap = __builtin_fmaf(a.c[4 + m], pl[ci + m * kSW3] + pl[ci - m * kSW3], lap);
#pragma unroll
      for (int m = 1; m <= kR; ++m) lap = __builtin_fmaf(a.c[8 + m], qz[kR + m] + qz[kR - m], lap);
      lap = __builtin_fmaf(a.ce, c, lap);
      const int64_t p = (int64_t)z * a.plane + (int64_t)y * a.pitch + x;
      point_tail<S>(a, x, y, z, p, c, lap, pl[ci + 1] - pl[ci - 1], pl[ci + kSW3] - pl[ci - kSW3],
                    qz[kR + 1] - qz[kR - 1]);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 2 * kR; ++j) qz[j] = qz[j + 1];
  }
}

template <class S, int TY>
hipError_t sweep25_t(const SweepArgs& a, int shape, int zchunk, hipStream_t st) {
  const int tiles_x = (a.nx + kTX - 1) / kTX;
  const int tiles_y = (a.ny + TY - 1) / TY;
  const int chunks = (a.nz + zchunk - 1) / zchunk;
  const int64_t blocks = (int64_t)tiles_x * tiles_y * chunks;
  if (blocks <= 0 || blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (shape == 0)
    hipLaunchKernelGGL((k_sweep_ring<S, TY>), dim3((unsigned)blocks), dim3(64, TY), 0, st, a, tiles_x,
                       tiles_y, zchunk);
  else
    hipLaunchKernelGGL((k_sweep_shift<S, TY>), dim3((unsigned)blocks), dim3(64, TY), 0, st, a,
                       tiles_x, tiles_y, zchunk);
  return hipGetLastError();
}

template <class S>
hipError_t gmem_s(const SweepArgs& a, int bx, int by, int bz, hipStream_t st) {
#define WAVE_GMEM_CASE(X, Y, Z) \
  if (bx == X && by == Y && bz == Z) return gmem_t<S, X, Y, Z>(a, st);
  WAVE_GMEM_CASE(8, 8, 8)
  WAVE_GMEM_CASE(4, 4, 4)
  WAVE_GMEM_CASE(16, 16, 4)
  WAVE_GMEM_CASE(32, 32, 1)
  WAVE_GMEM_CASE(64, 4, 1)
  WAVE_GMEM_CASE(64, 4, 4)
#undef WAVE_GMEM_CASE
  return hipErrorInvalidValue;
}

template <class S>
hipError_t sweep25_s(const SweepArgs& a, int shape, int ty, int zchunk, hipStream_t st) {
  if (ty == 8) return sweep25_t<S, 8>(a, shape, zchunk, st);
  if (ty == 16) return sweep25_t<S, 16>(a, shape, zchunk, st);
  return hipErrorInvalidValue;
}

}  // namespace

bool gmem_config_supported(int bx, int by, int bz) {
  const int ok[][3] = {{8, 8, 8}, {4, 4, 4}, {16, 16, 4}, {32, 32, 1}, {64, 4, 1}, {64, 4, 4}};
  for (const auto& s : ok)
    if (s[0] == bx && s[1] == by && s[2] == bz) return true;
  return false;
}

hipError_t launch_sweep_gmem(const SweepArgs& a, int storage, int bx, int by, int bz,
                             hipStream_t s) {
  switch (storage) {
    case 0: return gmem_s<StF32>(a, bx, by, bz, s);
    case 1: return gmem_s<StBF16>(a, bx, by, bz, s);
    case 2: return gmem_s<StF16>(a, bx, by, bz, s);
    case 3: return gmem_s<StBF16SR>(a, bx, by, bz, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sweep_25d(const SweepArgs& a, int storage, int shape, int ty, int zchunk,
                            hipStream_t s) {
  if (zchunk <= 0) return hipErrorInvalidValue;
  switch (storage) {
    case 0: return sweep25_s<StF32>(a, shape, ty, zchunk, s);
    case 1: return sweep25_s<StBF16>(a, shape, ty, zchunk, s);
    case 2: return sweep25_s<StF16>(a, shape, ty, zchunk, s);
    case 3: return sweep25_s<StBF16SR>(a, shape, ty, zchunk, s);
  }
  return hipErrorInvalidValue;
}

int auto_zchunk25(int nx, int ny, int nz, int ty) {
  // about 2048 workgroups, chunks of 16 to 64 planes
  const int64_t tiles = (int64_t)((nx + kTX - 1) / kTX) * ((ny + ty - 1) / ty);
  const int64_t chunks = (2048 + tiles - 1) / tiles;
  int zc = (int)std::min<int64_t>(64, (nz + chunks - 1) / chunks);
  zc = std::max(zc, 16);
  return std::min(zc, nz);
}

}  // namespace wave
