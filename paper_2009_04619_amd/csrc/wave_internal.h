// wave_internal.h -- shared declarations between the host runtime and the
// kernels of the wave library (not part of the public C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace wave {

// Radius of the Eq. 3 stencil along each axis.
constexpr int kR = 4;
// Width of one wavefront along x: the x extent of every tile.
constexpr int kTX = 64;

// Padded device layout of every field (same for all arrays of a context):
//   element (x, y, z) lives at  base + ((z + 4) * rows + (y + 4)) * pitch + x
//   pitch = round_up(nx + 8, 64) elements, rows = ny + 8, planes = nz + 8.
// x in [nx, pitch) of each row is zero: those cells are the +x ghosts of the
// row and the -x ghosts of the next row (x = -4..-1 wrap into the previous
// row's tail).  Rows y = -4..-1, ny..ny+3 and planes z = -4..-1, nz..nz+3 are
// zero.  Ghost cells are never written, so the stencil needs no bounds tests.
// `base` leaves kGuard zero elements before the first plane and after the
// last so that the x-halo wrap of the first/last row stays inside.
constexpr int64_t kGuard = 64;

struct Layout {
  int32_t nx, ny, nz;
  int32_t pitch;        // elements per row
  int64_t plane;        // elements per plane = (ny + 8) * pitch
  int64_t origin;       // element index of (0, 0, 0) from the array start
  int64_t elems;        // total elements of one array incl. guards
};

inline Layout make_layout(int32_t nx, int32_t ny, int32_t nz) {
  Layout L;
  L.nx = nx; L.ny = ny; L.nz = nz;
  L.pitch = ((nx + 8 + 63) / 64) * 64;
  L.plane = (int64_t)(ny + 8) * L.pitch;
  L.origin = kGuard + 4 * L.plane + 4 * (int64_t)L.pitch;
  L.elems = 2 * kGuard + (int64_t)(nz + 8) * L.plane;
  return L;
}

// Everything one sweep kernel needs.  Pointers are element pointers already
// offset to (0, 0, 0).
struct SweepArgs {
  const void* cur;      // u^n     (storage type)
  void* nxt;            // u^{n-1} on entry, u^{n+1} on exit (storage type)
  const float* vp;      // (V dt)^2
  const float* eta;     // damping eta per point (array mode), else null
  const double* etab;   // default profile tables (table mode), else null:
                        // tx[-1..nx], ty[-1..ny], tz[-1..nz] back to back
  const float* etq;     // table mode: dqx[nx], dqy[ny], dqz[nz] back to back,
                        // dq_a = fl32(fl32(dt (t_a(i+1) - t_a(i-1))) * q_a)
  double dt;            // eta = fl32(dt * ((tx + ty) + tz)) in table mode
  float* phi;           // phi^n on entry, phi^{n+1} on exit
  int32_t nx, ny, nz, w;
  int32_t pitch;
  int64_t plane;
  float c[13];          // Eq. 3 weights (float32)
  float ce;             // -(c[0] + 2 sum c[1..12]): removes the weights' residual
  float q[3];           // 1 / (4 h_a^2)
  int32_t damping;      // 0: Eq. 2 everywhere
  int32_t step;         // time level n of u^n (counter of the random bits of
                        // stochastically rounded bf16 storage)
};

// Two steps per launch (wave_kernels2.hip): u^{n-1}, u^n, phi^n in;
// u^{n+1}, u^{n+2}, phi^{n+2} out, all distinct arrays; the sources of step n
// enter u^{n+1} inside the kernel.
struct Sweep2Args {
  SweepArgs s;               // s.cur = u^n, s.phi = phi^n (s.nxt unused)
  const void* prev;          // u^{n-1}
  void* out1;                // u^{n+1}
  void* out2;                // u^{n+2}
  float* phi_out;            // phi^{n+2}
  int32_t nsrc;
  const int32_t* src_ijk;    // [nsrc][3] grid indices (i, j, k)
  const float* wavelet;      // [nsrc][max_steps]
  int32_t max_steps;
  int32_t step;              // n
};

struct InjectArgs {
  void* u;              // u^{n+1} (storage type), offset to (0,0,0)
  const float* vp;
  int32_t nsrc;
  const int64_t* src_off;     // element offsets of the sources
  const float* wavelet;       // [max_src][max_steps]
  int32_t max_steps;
  int32_t step;               // time step index n (w[n] is added)
  int32_t nrec;
  const int64_t* rec_off;
  double* traces;             // [max_steps][nrec] row `trace_row`
  int32_t trace_row;
};

// One member of a batch (device table entry).  The sweep arguments' cur/nxt
// pointers are chosen per step from u[] and the member's parity.
struct BatchShot {
  SweepArgs sa;
  void* u[2];            // origins of the two u buffers
  int32_t tiles_x, tiles_y, zchunk, pad0;
  int64_t block_begin;   // first workgroup of this member in a batch launch
  int32_t target;        // steps to take in the current run
  int32_t pad1;
  InjectArgs inj;        // sources/receivers (u, step, trace_row set per step)
};

// Per-member step state in device memory, advanced by the batch
// source/receiver kernel after each sweep.
struct BatchState {
  int32_t cur;           // index of u^n in BatchShot::u
  int32_t step;          // time level n
  int32_t done;          // steps taken in the current run
  int32_t trace_row;     // next trace row
};

struct EnergyArgs {
  const void* cur;      // u^n
  const void* prev;     // u^{n-1}
  const float* vp;
  int32_t nx, ny, nz;
  int32_t pitch;
  int64_t plane;
  double c[13];         // Eq. 3 weights in float64
  double* partial;      // [nz*ny][2] (kinetic, potential) per row
  double* result;       // [2]
};

// Kernel launchers (defined in wave_kernels.hip).  storage: 0 f32, 1 bf16,
// 2 f16.  Return the hipError_t of the launch.
hipError_t launch_sweep_direct(const SweepArgs& a, int storage, hipStream_t s);
hipError_t launch_sweep_stream(const SweepArgs& a, int storage, int ry, int nw,
                               int zchunk, hipStream_t s);
// Compiled tiles (rows_per_wave, waves_per_group); 2 x 16 (64 x 32 tiles)
// only for contexts without a per-point eta array.
bool stream_config_supported(int ry, int nw, bool eta_array);
// The streaming kernel as one persistent launch of `groups` workgroups (a
// multiple of 8; one per CU), each sweeping its share of the tiles in turn.
// Tiles 64 x nw, ry = 1, nw in {8, 16}.
hipError_t launch_sweep_persist(const SweepArgs& a, int storage, int ry, int nw, int zchunk,
                                int groups, hipStream_t s);
// The streaming kernel with the x neighbours exchanged by wavefront shuffles
// (ds_bpermute) instead of read from the staged plane (64 x nw tiles, nw in
// {8, 16}; the same results bit for bit).
hipError_t launch_sweep_shuffle(const SweepArgs& a, int storage, int nw, int zchunk, hipStream_t s);
// The streaming kernel with the z terms summed by the semi-stencil (64 x nw
// tiles, nw in {8, 16}; default-profile tables or damping off only).
hipError_t launch_sweep_semi(const SweepArgs& a, int storage, int nw, int zchunk, hipStream_t s);
int auto_zchunk(int nx, int ny, int nz, int ry, int nw);
// Largest z chunk the streaming kernels accept for planes of `plane`
// elements (their float arrays are addressed with 32-bit offsets inside a
// window of zchunk + 8 planes); below 1 when one plane is too large.
int stream_zchunk_limit(int64_t plane);
hipError_t launch_inject_record(const InjectArgs& a, int storage, hipStream_t s);
// Two-step sweep (wave_kernels2.hip): damping off or the default profile's
// tables; zchunk <= stream2_zchunk_limit(plane) (window of zchunk + 16 planes).
hipError_t launch_sweep2(const Sweep2Args& g, int storage, int zchunk, hipStream_t s);
int stream2_zchunk_limit(int64_t plane);
// Whether every two-step tile holds at most the number of sources the kernel
// gathers per tile (ijk: [n][3] grid indices, host memory).
bool sweep2_sources_fit(const int32_t* ijk, int n);
int auto_zchunk2(int nx, int ny, int nz);
// The paper's other code shapes (wave_shapes.hip): 3-D tiles of bx x by x bz
// threads reading every operand from memory, and 2.5-D tiles of 64 x ty
// streamed through z chunks, shape 0 = ring of 9 staged planes, 1 = staged
// plane plus a shifted register queue along z.
bool gmem_config_supported(int bx, int by, int bz);
hipError_t launch_sweep_gmem(const SweepArgs& a, int storage, int bx, int by, int bz,
                             hipStream_t s);
hipError_t launch_sweep_25d(const SweepArgs& a, int storage, int shape, int ty, int zchunk,
                            hipStream_t s);
int auto_zchunk25(int nx, int ny, int nz, int ty);
// Streaming sweep with two x-adjacent points per lane (wave_kernels_pair.hip):
// 128 x ty tiles, ty in {8, 16}; the default profile's tables only (no eta
// array); zchunk <= stream_zchunk_limit(plane).
hipError_t launch_sweep_pair(const SweepArgs& a, int storage, int ty, int zchunk, hipStream_t s);
// Batched form: the members' block ranges laid out for 128 x ty tiles.
hipError_t launch_sweep_batch_pair(const BatchShot* shots, BatchState* state, int nshots,
                                   int64_t total_blocks, int storage, int ty, hipStream_t s);
hipError_t launch_energy(const EnergyArgs& a, int storage, hipStream_t s);
hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
// kind 0: read a (bytes), d a 4-byte sink; kind 1: d = a + b c over bytes each.
hipError_t launch_stream_mix(int kind, void* d, const void* a, const void* b, const void* c,
                             size_t bytes, hipStream_t s);
// Scatter a compact [nz][ny][nx] float field into a padded array whose
// element (0, 0, 0) is at dst; with dt > 0 store fl32((v dt)^2) instead of v.
hipError_t launch_setup_field(float* dst, const float* src, int nx, int ny, int nz, int pitch,
                              int64_t plane, double dt, hipStream_t s);
int stream_chunk_count(int nz, int w, int zchunk, bool damping);
int stream_tiles_y(int ny, int ry, int nw);
// eta_array: some member holds a per-point eta array.
hipError_t launch_sweep_batch(const BatchShot* shots, BatchState* state, int nshots,
                              int64_t total_blocks, int storage, int ry, int nw, bool eta_array,
                              hipStream_t s);
hipError_t launch_inject_batch(const BatchShot* shots, BatchState* state, int nshots,
                               int storage, hipStream_t s);

}  // namespace wave
