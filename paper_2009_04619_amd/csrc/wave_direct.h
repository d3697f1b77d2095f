// wave_direct.h -- one point of the sweep with every operand addressed
// directly in the padded arrays (paper Eq. 2-3, damping layer of Sec. III-B):
// the shared tail of the kernels that do not stream a register queue (the
// direct kernel, the 3-D tiles and the 2.5-D shapes of wave_shapes.hip).
#pragma once

#include "wave_internal.h"
#include "wave_point.h"

namespace wave {
namespace {

// Default damping profile in table mode: eta(x, y, z) = fl32(dt * ((tx[x] +
// ty[y]) + tz[z])) (the profile is a sum of three per-axis terms; the double
// operations match the host's).  Its differences come from the dq tables.
__device__ __forceinline__ float eta_tab(const SweepArgs& a, int x, int y, int z) {
  const double* tx = a.etab + 1;
  const double* ty = tx + a.nx + 2;
  const double* tz = ty + a.ny + 2;
  return (float)(a.dt * ((tx[x] + ty[y]) + tz[z]));
}

__device__ __forceinline__ bool in_layer(const SweepArgs& a, int x, int y, int z) {
  return x < a.w || x >= a.nx - a.w || y < a.w || y >= a.ny - a.w || z < a.w ||
         z >= a.nz - a.w;
}

// Update of point (x, y, z) at element p from its centre value c, its
// Laplacian lap (Eq. 3, in the canonical order) and its central u differences
// du_a = u(+1) - u(-1) along each axis: reads u^{n-1} and vp (and phi, eta in
// the layer), writes u^{n+1} over u^{n-1} (and phi^{n+1}).
template <class S>
__device__ __forceinline__ void point_tail(const SweepArgs& a, int x, int y, int z, int64_t p,
                                           float c, float lap, float dux, float duy, float duz) {
  using T = typename S::T;
  T* un = static_cast<T*>(a.nxt);
  const int64_t P = a.pitch, Q = a.plane;
  const float pu = S::ld(un, p);
  const float vp = a.vp[p];
  float r;
  if (a.damping && in_layer(a, x, y, z)) {
    float e, dqx, dqy, dqz;
    if (a.etab) {
      e = eta_tab(a, x, y, z);
      dqx = a.etq[x];
      dqy = a.etq[a.nx + y];
      dqz = a.etq[a.nx + a.ny + z];
    } else {
      e = a.eta[p];
      dqx = (a.eta[p + 1] - a.eta[p - 1]) * a.q[0];
      dqy = (a.eta[p + P] - a.eta[p - P]) * a.q[1];
      dqz = (a.eta[p + Q] - a.eta[p - Q]) * a.q[2];
    }
    const float ph = a.phi[p];
    r = upd_layer(c, pu, vp, lap, e, ph);
    a.phi[p] = upd_phi(ph, e, dqx, dux, dqy, duy, dqz, duz);
  } else {
    r = upd_inner(c, pu, vp, lap);
  }
  if constexpr (S::kSR) {  // stochastic rounding of bf16 storage (WAVE_STOCH_ROUND)
    const uint32_t r16 = sr_word(pcg_hash((uint32_t)a.step), a.nx, a.ny, x, y, z) >> (16 * (x & 1));
    un[p] = f32_to_bf16_sr(r, r16);
  } else {
    S::st(un, p, r);
  }
}

// Point (x, y, z) with every stencil operand read from memory.
template <class S>
__device__ __forceinline__ void direct_point(const SweepArgs& a, int x, int y, int z) {
  using T = typename S::T;
  const T* u = static_cast<const T*>(a.cur);
  const int64_t P = a.pitch, Q = a.plane;
  const int64_t p = (int64_t)z * Q + (int64_t)y * P + x;
  const float c = S::ld(u, p);
  float lap = a.c[0] * c;
#pragma unroll
  for (int m = 1; m <= kR; ++m) lap = __builtin_fmaf(a.c[m], S::ld(u, p + m) + S::ld(u, p - m), lap);
#pragma unroll
  for (int m = 1; m <= kR; ++m)
    lap = __builtin_fmaf(a.c[4 + m], S::ld(u, p + m * P) + S::ld(u, p - m * P), lap);
#pragma unroll
  for (int m = 1; m <= kR; ++m)
    lap = __builtin_fmaf(a.c[8 + m], S::ld(u, p + m * Q) + S::ld(u, p - m * Q), lap);
  lap = __builtin_fmaf(a.ce, c, lap);
  point_tail<S>(a, x, y, z, p, c, lap, S::ld(u, p + 1) - S::ld(u, p - 1),
                S::ld(u, p + P) - S::ld(u, p - P), S::ld(u, p + Q) - S::ld(u, p - Q));
}

}  // namespace
}  // namespace wave
