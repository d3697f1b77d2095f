// wave_runtime.hip -- host side of the C ABI declared in include/wave.h:
// argument checking, arena layout, set-up of vp and eta, step enqueueing,
// state transfers and timing.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "wave.h"
#include "wave_internal.h"

using wave::Layout;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

// Eq. 3 weights: standard 8th-order central second-difference weights.
constexpr double kW0 = -205.0 / 72.0;
constexpr double kWm[4] = {8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int storage_bytes(int32_t storage) { return storage == WAVE_F32 ? 4 : 2; }

// Workgroups of a persistent sweep on the current device: one per CU, a
// multiple of 8 (the XCD count of the tile order); 0 if the count is unknown.
int persistent_groups() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return n >= 8 ? n / 8 * 8 : 0;
}

bool desc_ok(const wave_desc* d, std::string* why) {
  auto bad = [&](const char* m) {
    if (why) *why = m;
    return false;
  };
  if (!d) return bad("descriptor is NULL");
  if (d->nx < 1 || d->ny < 1 || d->nz < 1) return bad("extents must be >= 1");
  if (d->nx > 32768 || d->ny > 32768 || d->nz > 32768) return bad("extent above 32768");
  {
    // in-plane byte offsets are unsigned 32-bit in the kernels
    const Layout L = wave::make_layout(d->nx, d->ny, d->nz);
    if ((int64_t)L.plane * 4 > 0x7fffffffLL) return bad("one z plane exceeds 2 GiB");
  }
  if (d->w < 0 || 2 * (int64_t)d->w > std::min({d->nx, d->ny, d->nz}))
    return bad("layer width must satisfy 0 <= 2w <= min extent");
  if (!(d->dx > 0 && d->dy > 0 && d->dz > 0) || !isfinite(d->dx) || !isfinite(d->dy) ||
      !isfinite(d->dz))
    return bad("grid spacing must be finite and > 0");
  if (!(d->dt > 0) || !isfinite(d->dt)) return bad("dt must be finite and > 0");
  if (d->storage != WAVE_F32 && d->storage != WAVE_BF16 && d->storage != WAVE_F16)
    return bad("unknown storage type");
  if (d->flags & ~(WAVE_DAMPING_OFF | WAVE_ETA_ARRAY | WAVE_TWO_STEP | WAVE_STOCH_ROUND))
    return bad("unknown flags");
  if ((d->flags & WAVE_STOCH_ROUND) && d->storage != WAVE_BF16)
    return bad("WAVE_STOCH_ROUND applies to bf16 storage only");
  if ((d->flags & WAVE_STOCH_ROUND) && (d->flags & WAVE_TWO_STEP))
    return bad("WAVE_STOCH_ROUND is not available with WAVE_TWO_STEP");
  if ((d->flags & WAVE_TWO_STEP) && (d->flags & WAVE_ETA_ARRAY) && !(d->flags & WAVE_DAMPING_OFF))
    return bad("WAVE_TWO_STEP supports the default damping profile only, not an eta array");
  if (!(d->flags & WAVE_DAMPING_OFF) && d->w > 0 && !(d->refl > 0 && d->refl < 1))
    return bad("refl must be in (0, 1)");
  if (d->max_src < 0 || d->max_rec < 0 || d->max_steps < 0) return bad("negative capacity");
  if (d->reserved != 0) return bad("reserved must be 0");
  return true;
}

bool damping_on(const wave_desc* d) { return !(d->flags & WAVE_DAMPING_OFF) && d->w > 0; }
bool eta_array(const wave_desc* d) { return damping_on(d) && (d->flags & WAVE_ETA_ARRAY); }
bool two_step(const wave_desc* d) { return (d->flags & WAVE_TWO_STEP) != 0; }
bool stoch_round(const wave_desc* d) { return (d->flags & WAVE_STOCH_ROUND) != 0; }
// Storage code of the kernel instances a context runs: the wave_storage
// value, or 3 for bf16 storage rounded stochastically.
int kernel_storage(const wave_desc* d) {
  return d->storage == WAVE_BF16 && stoch_round(d) ? 3 : d->storage;
}

size_t eta_tables_bytes(const wave_desc* d);

struct ArenaPlan {
  size_t u[4], vp, eta, etab, phi[2], src_off, src_ijk, wavelet, rec_off, traces, partial, eres, total;
};

ArenaPlan plan_arena(const wave_desc* d) {
  const Layout L = wave::make_layout(d->nx, d->ny, d->nz);
  ArenaPlan a;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = align_up(off, 256);
    size_t o = off;
    off += bytes;
    return o;
  };
  const size_t es = storage_bytes(d->storage);
  a.u[0] = take((size_t)L.elems * es);
  a.u[1] = take((size_t)L.elems * es);
  // two steps per launch write u^{n+1}, u^{n+2} and phi^{n+2} to arrays of
  // their own
  a.u[2] = two_step(d) ? take((size_t)L.elems * es) : (size_t)-1;
  a.u[3] = two_step(d) ? take((size_t)L.elems * es) : (size_t)-1;
  a.vp = take((size_t)L.elems * 4);
  const bool damp = damping_on(d);
  a.eta = eta_array(d) ? take((size_t)L.elems * 4) : (size_t)-1;
  a.etab = (damp && !eta_array(d)) ? take(eta_tables_bytes(d)) : (size_t)-1;
  a.phi[0] = damp ? take((size_t)L.elems * 4) : (size_t)-1;
  a.phi[1] = (damp && two_step(d)) ? take((size_t)L.elems * 4) : (size_t)-1;
  a.src_off = take((size_t)std::max(d->max_src, 1) * 8);
  a.src_ijk = take((size_t)std::max(d->max_src, 1) * 12);
  a.wavelet = take((size_t)std::max(d->max_src, 1) * std::max(d->max_steps, 1) * 4);
  a.rec_off = take((size_t)std::max(d->max_rec, 1) * 8);
  a.traces = take((size_t)std::max(d->max_rec, 1) * std::max(d->max_steps, 1) * 8);
  a.partial = take((size_t)d->ny * d->nz * 2 * 8);
  a.eres = take(2 * 8);
  a.total = align_up(off, 256);
  return a;
}

void coefficients64(const wave_desc* d, double c[13]) {
  const double ix = 1.0 / (d->dx * d->dx), iy = 1.0 / (d->dy * d->dy), iz = 1.0 / (d->dz * d->dz);
  c[0] = kW0 * (ix + iy + iz);
  for (int m = 0; m < 4; ++m) {
    c[1 + m] = kWm[m] / (d->dx * d->dx);
    c[5 + m] = kWm[m] / (d->dy * d->dy);
    c[9 + m] = kWm[m] / (d->dz * d->dz);
  }
}

// Depth into the layer (cells) of index i on an axis of extent n.
double depth_cells(int i, int n, int w) {
  if (i < w) return (double)(w - i);
  if (i > n - 1 - w) return (double)(i - (n - 1 - w));
  return 0.0;
}

// One z plane of the default eta profile (float [ny][nx]).
void eta_plane(const wave_desc* d, double vmax, int k, float* out) {
  const double h[3] = {d->dx, d->dy, d->dz};
  double d0[3];
  for (int a = 0; a < 3; ++a) d0[a] = 3.0 * vmax * log(1.0 / d->refl) / (2.0 * ((double)d->w * h[a]));
  const double cz = depth_cells(k, d->nz, d->w);
  for (int j = 0; j < d->ny; ++j) {
    const double cy = depth_cells(j, d->ny, d->w);
    for (int i = 0; i < d->nx; ++i) {
      const double cx = depth_cells(i, d->nx, d->w);
      const double cells[3] = {cx, cy, cz};
      double s = 0.0;
      for (int a = 0; a < 3; ++a) {
        if (cells[a] > 0.0) {
          const double r = cells[a] / (double)d->w;
          s += d0[a] * r * r;
        }
      }
      out[(size_t)j * d->nx + i] = (float)(d->dt * s);
    }
  }
}

// Tables of the default profile in table mode, back to back:
//  * double t_a[i + 1] = d0_a (depth/w)^2 for i = -1..n_a, axes x, y, z (the
//    depth continues one cell beyond each face: w + 1 there), so that
//    eta = fl32(dt * ((tx + ty) + tz)), the sum eta_plane forms;
//  * float dq_a[i] = fl32(fl32(dt * (t_a[i + 1] - t_a[i - 1])) * q_a) for
//    i = 0..n_a-1: the profile's central difference along axis a (the other
//    axes' terms cancel in a sum of one-axis functions) times q_a.
size_t eta_tables_bytes(const wave_desc* d) {
  const size_t n = (size_t)d->nx + d->ny + d->nz;
  return (n + 6) * 8 + align_up(n * 4, 8);
}

void eta_tables(const wave_desc* d, double vmax, const float q[3], std::vector<unsigned char>& out) {
  const double h[3] = {d->dx, d->dy, d->dz};
  const int n[3] = {d->nx, d->ny, d->nz};
  std::vector<double> t((size_t)d->nx + d->ny + d->nz + 6, 0.0);
  std::vector<float> dq((size_t)d->nx + d->ny + d->nz, 0.0f);
  size_t base = 0, qbase = 0;
  for (int a = 0; a < 3; ++a) {
    const double d0 = 3.0 * vmax * log(1.0 / d->refl) / (2.0 * ((double)d->w * h[a]));
    for (int i = -1; i <= n[a]; ++i) {
      const double cells = depth_cells(i, n[a], d->w);
      if (cells > 0.0) {
        const double r = cells / (double)d->w;
        t[base + 1 + i] = d0 * r * r;
      }
    }
    for (int i = 0; i < n[a]; ++i) {
      const float de = (float)(d->dt * (t[base + 2 + i] - t[base + i]));
      dq[qbase + i] = de * q[a];
    }
    base += (size_t)n[a] + 2;
    qbase += (size_t)n[a];
  }
  out.assign(eta_tables_bytes(d), 0);
  memcpy(out.data(), t.data(), t.size() * 8);
  memcpy(out.data() + t.size() * 8, dq.data(), dq.size() * 4);
}

// Largest eta of the default profile: at a corner of the grid, where the
// depth into the layer is w on every axis, eta = fl32(dt * sum_a d0_a).
double max_default_eta(const wave_desc* d, double vmax) {
  const double h[3] = {d->dx, d->dy, d->dz};
  double s = 0.0;
  for (int a = 0; a < 3; ++a) s += 3.0 * vmax * log(1.0 / d->refl) / (2.0 * ((double)d->w * h[a]));
  return (double)(float)(d->dt * s);
}

// Largest eta the damped update tolerates at stability number stab <= 1:
// 2 + sqrt(8 - 4 stab^2) (2 + 2 sqrt 2 without the Laplacian, 4 at stab 1).
double eta_limit(double stab) { return 2.0 + sqrt(8.0 - 4.0 * stab * stab); }

uint16_t host_bf16(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

float host_from_bf16(uint16_t b) {
  uint32_t u = (uint32_t)b << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

}  // namespace

struct wave_ctx {
  wave_batch* batch;      // non-null while a batch member
  wave_desc d;
  Layout L;
  ArenaPlan plan;
  hipStream_t stream;
  char* arena;
  int es;                 // bytes per u element
  int icur, iprev;         // which of plan.u hold u^n and u^{n-1}
  int iphi;               // which of plan.phi holds phi^n
  int zchunk2;            // z chunk of the two-step sweep (0 = automatic)
  int64_t step;           // time level n
  bool broken;
  bool damp;
  float c[13];
  float q[3];
  double c64[13];
  double vmax;
  int nsrc, nrec, trace_count;
  std::vector<int32_t> src_host;   // (i, j, k) of the sources
  bool src_fit2;                   // the sources fit the two-step kernel's tiles
  int variant, ry, nw, zchunk;
  int shp[3];             // WAVE_KERNEL_GMEM: block (bx, by, bz); RING/SHIFT: (1, ty, zchunk)
  int groups;             // workgroups of a persistent launch (one per CU)
  bool timing;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  size_t events_used;
  hipEvent_t ev_join;         // orders a batch after this context's stream
  hipEvent_t ev_left;         // batch work up to this context's removal
  bool left_pending;          // the stream has not yet waited on ev_left
  double timing_ms;
  int64_t timing_launches;

  char* at(size_t off) const { return arena + off; }
  char* u_base(int idx) const { return at(plan.u[idx]); }
  void* u_origin(int idx) const { return u_base(idx) + (size_t)L.origin * es; }
  float* f_origin(size_t off) const {
    return off == (size_t)-1 ? nullptr : reinterpret_cast<float*>(at(off)) + L.origin;
  }
};

namespace {

int dev_fail(wave_ctx* c, hipError_t e, const char* what) {
  if (c) c->broken = true;
  return fail(WAVE_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define CHECK_CTX(c)                                                       \
  do {                                                                     \
    if (!(c)) return fail(WAVE_EINVAL, "context is NULL");                 \
    if ((c)->broken) return fail(WAVE_ESTATE, "context broken by an earlier device error"); \
  } while (0)

#define HIPCHK(c, expr, what)                     \
  do {                                            \
    hipError_t _e = (expr);                       \
    if (_e != hipSuccess) return dev_fail((c), _e, (what)); \
  } while (0)

// Whole-field transfers between a compact host array [nz][ny][nx] and a
// padded device array.  They go through a pinned host buffer laid out as a
// run of padded planes (rows y = -4 .. ny+3 of `pitch` elements, zero outside
// the grid), so each run moves as one contiguous copy.  The ghost rows and
// the row padding it writes are zero, as the device layout holds them.  (A
// pitched copy straight from pageable memory moves row by row: at 512^3 a
// field took about a second that way.)  fill(k, y, row) writes the nx
// elements of row y of plane k into a row of the buffer; take(k, y, row)
// reads them back.
constexpr size_t kStageBytes = size_t(64) << 20;

template <class Fill>
int upload_field(wave_ctx* c, char* dev_base, int esz, Fill fill) {
  const Layout& L = c->L;
  const size_t plane_b = (size_t)L.plane * esz;
  const int run = (int)std::max<size_t>(1, std::min<size_t>(L.nz, kStageBytes / plane_b));
  void* stage = nullptr;
  if (hipHostMalloc(&stage, (size_t)run * plane_b, hipHostMallocDefault) != hipSuccess)
    return fail(WAVE_EDEVICE, "hipHostMalloc of the transfer buffer failed");
  memset(stage, 0, (size_t)run * plane_b);
  hipError_t e = hipSuccess;
  for (int k0 = 0; k0 < L.nz && e == hipSuccess; k0 += run) {
    const int nk = std::min(run, L.nz - k0);
    for (int k = 0; k < nk; ++k)
      for (int y = 0; y < L.ny; ++y)
        fill(k0 + k, y, static_cast<char*>(stage) +
                            ((size_t)k * L.plane + (size_t)(y + wave::kR) * L.pitch) * esz);
    char* dst = dev_base + ((size_t)L.origin + (size_t)k0 * L.plane - (size_t)wave::kR * L.pitch) * esz;
    e = hipMemcpyAsync(dst, stage, (size_t)nk * plane_b, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);  // the buffer is refilled next
  }
  (void)hipHostFree(stage);
  return e == hipSuccess ? WAVE_OK : dev_fail(c, e, "field upload");
}

template <class Take>
int download_field(wave_ctx* c, const char* dev_base, int esz, Take take) {
  const Layout& L = c->L;
  const size_t plane_b = (size_t)L.plane * esz;
  const int run = (int)std::max<size_t>(1, std::min<size_t>(L.nz, kStageBytes / plane_b));
  void* stage = nullptr;
  if (hipHostMalloc(&stage, (size_t)run * plane_b, hipHostMallocDefault) != hipSuccess)
    return fail(WAVE_EDEVICE, "hipHostMalloc of the transfer buffer failed");
  hipError_t e = hipSuccess;
  for (int k0 = 0; k0 < L.nz && e == hipSuccess; k0 += run) {
    const int nk = std::min(run, L.nz - k0);
    const char* src =
        dev_base + ((size_t)L.origin + (size_t)k0 * L.plane - (size_t)wave::kR * L.pitch) * esz;
    e = hipMemcpyAsync(stage, src, (size_t)nk * plane_b, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) break;
    for (int k = 0; k < nk; ++k)
      for (int y = 0; y < L.ny; ++y)
        take(k0 + k, y, static_cast<const char*>(stage) +
                            ((size_t)k * L.plane + (size_t)(y + wave::kR) * L.pitch) * esz);
  }
  (void)hipHostFree(stage);
  return e == hipSuccess ? WAVE_OK : dev_fail(c, e, "field download");
}

// A float field [nz][ny][nx] to or from a padded float array.
int upload_f32(wave_ctx* c, char* dev_base, const float* host) {
  const size_t nx = c->L.nx, ny = c->L.ny;
  return upload_field(c, dev_base, 4, [&](int k, int y, char* row) {
    memcpy(row, host + ((size_t)k * ny + y) * nx, nx * 4);
  });
}

int download_f32(wave_ctx* c, const char* dev_base, float* host) {
  const size_t nx = c->L.nx, ny = c->L.ny;
  return download_field(c, dev_base, 4, [&](int k, int y, const char* row) {
    memcpy(host + ((size_t)k * ny + y) * nx, row, nx * 4);
  });
}

// Upload a float field into a u buffer, rounding to the storage format.
int upload_u(wave_ctx* c, int idx, const float* host) {
  const size_t nx = c->L.nx, ny = c->L.ny;
  const int storage = c->d.storage;
  if (c->es == 4) return upload_f32(c, c->u_base(idx), host);
  return upload_field(c, c->u_base(idx), 2, [&](int k, int y, char* row) {
    const float* src = host + ((size_t)k * ny + y) * nx;
    uint16_t* dst = reinterpret_cast<uint16_t*>(row);
    if (storage == WAVE_BF16) {
      for (size_t i = 0; i < nx; ++i) dst[i] = host_bf16(src[i]);
    } else {
      for (size_t i = 0; i < nx; ++i) {
        const _Float16 h = (_Float16)src[i];
        memcpy(&dst[i], &h, 2);
      }
    }
  });
}

int download_u(wave_ctx* c, int idx, float* host) {
  const size_t nx = c->L.nx, ny = c->L.ny;
  const int storage = c->d.storage;
  if (c->es == 4) return download_f32(c, c->u_base(idx), host);
  return download_field(c, c->u_base(idx), 2, [&](int k, int y, const char* row) {
    float* dst = host + ((size_t)k * ny + y) * nx;
    const uint16_t* src = reinterpret_cast<const uint16_t*>(row);
    if (storage == WAVE_BF16) {
      for (size_t i = 0; i < nx; ++i) dst[i] = host_from_bf16(src[i]);
    } else {
      for (size_t i = 0; i < nx; ++i) {
        _Float16 h;
        memcpy(&h, &src[i], 2);
        dst[i] = (float)h;
      }
    }
  });
}

// Sweep arguments of a context (cur/nxt are set per step).
wave::SweepArgs sweep_args(const wave_ctx* c) {
  const Layout& L = c->L;
  wave::SweepArgs sa;
  sa.cur = nullptr;
  sa.nxt = nullptr;
  sa.vp = c->f_origin(c->plan.vp);
  sa.eta = c->f_origin(c->plan.eta);
  sa.etab = c->plan.etab == (size_t)-1 ? nullptr : reinterpret_cast<const double*>(c->at(c->plan.etab));
  sa.etq = sa.etab ? reinterpret_cast<const float*>(sa.etab + (L.nx + L.ny + L.nz + 6)) : nullptr;
  sa.dt = c->d.dt;
  sa.phi = c->f_origin(c->plan.phi[c->iphi]);
  sa.nx = L.nx;
  sa.ny = L.ny;
  sa.nz = L.nz;
  sa.w = c->d.w;
  sa.pitch = L.pitch;
  sa.plane = L.plane;
  memcpy(sa.c, c->c, sizeof(sa.c));
  // residual of the float weights: c_xyz + 2 sum c_am is zero in exact
  // arithmetic; summed in double it is exact for float weights
  double e = (double)sa.c[0];
  for (int m = 1; m < 13; ++m) e += 2.0 * (double)sa.c[m];
  sa.ce = (float)(-e);
  memcpy(sa.q, c->q, sizeof(sa.q));
  sa.damping = c->damp ? 1 : 0;
  sa.step = (int32_t)c->step;
  return sa;
}

// Source/receiver arguments of a context (u, step, trace_row set per step).
wave::InjectArgs inject_args(const wave_ctx* c) {
  wave::InjectArgs ia;
  ia.u = nullptr;
  ia.vp = c->f_origin(c->plan.vp);
  ia.nsrc = c->nsrc;
  ia.src_off = reinterpret_cast<const int64_t*>(c->at(c->plan.src_off));
  ia.wavelet = reinterpret_cast<const float*>(c->at(c->plan.wavelet));
  ia.max_steps = std::max(c->d.max_steps, 1);
  ia.step = 0;
  ia.nrec = c->nrec;
  ia.rec_off = reinterpret_cast<const int64_t*>(c->at(c->plan.rec_off));
  ia.traces = c->nrec > 0 ? reinterpret_cast<double*>(c->at(c->plan.traces)) : nullptr;
  ia.trace_row = 0;
  return ia;
}

int64_t offset_of(const wave_ctx* c, int i, int j, int k) {
  return (int64_t)k * c->L.plane + (int64_t)j * c->L.pitch + i;
}

bool in_grid(const wave_ctx* c, int i, int j, int k) {
  return i >= 0 && i < c->d.nx && j >= 0 && j < c->d.ny && k >= 0 && k < c->d.nz;
}

}  // namespace

struct wave_batch {
  int32_t storage;
  int32_t kstore;             // kernel storage code of the members (3: bf16 rounded stochastically)
  int32_t max_shots;
  hipStream_t user_stream;   // the members' stream
  hipStream_t stream;        // the batch's own stream (graphs can be captured on it)
  hipEvent_t ev_in, ev_out;
  hipEvent_t ev_copy[2];      // table upload from pinned slot k done
  char* pinned[2];            // pinned host copies of the tables, alternating
  int64_t runs;               // runs issued (selects the pinned slot)
  char* arena;
  size_t arena_bytes;
  wave::BatchShot* d_shots;
  wave::BatchState* d_state;
  std::vector<wave_ctx*> members;
  std::vector<int32_t> remaining;
  std::vector<wave::BatchShot> h_shots;
  std::vector<wave::BatchState> h_state;
  int ry, nw;
  bool eta_any;               // some member holds a per-point eta array
  int64_t total_blocks;
  bool layout_dirty;          // membership or tile shape changed
  int graph_steps;            // steps per captured graph (0 = plain launches)
  // captured step blocks, one per number of active members K (the active
  // members are the first K: runs order members by steps left)
  std::vector<std::pair<int, hipGraphExec_t>> graphs;
  std::vector<int64_t> prefix_blocks;  // workgroups of the first k members
  bool broken;
};

namespace {
// Orders the context stream after the batch work that touched the context:
// the latest run while it is a member (unless its stream is the batch's
// caller stream, which waits on every run already), or the runs up to its
// removal.  Every context entry point that enqueues work calls it first.
int join_batch_work(wave_ctx* c) {
  if (c->batch && c->stream != c->batch->user_stream)
    HIPCHK(c, hipStreamWaitEvent(c->stream, c->batch->ev_out, 0), "hipStreamWaitEvent");
  if (c->left_pending) {
    HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_left, 0), "hipStreamWaitEvent");
    c->left_pending = false;
  }
  return WAVE_OK;
}
}  // namespace

#define JOIN_CTX(c)                          \
  do {                                       \
    const int _rc = join_batch_work(c);      \
    if (_rc != WAVE_OK) return _rc;          \
  } while (0)

namespace {

size_t batch_table_bytes(int32_t max_shots, size_t* state_off) {
  const size_t a = align_up((size_t)std::max(max_shots, 1) * sizeof(wave::BatchShot), 256);
  if (state_off) *state_off = a;
  return a + align_up((size_t)std::max(max_shots, 1) * sizeof(wave::BatchState), 256);
}

int batch_fail(wave_batch* b, hipError_t e, const char* what) {
  if (b) b->broken = true;
  return fail(WAVE_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define BCHK(b, expr, what)                                        \
  do {                                                             \
    hipError_t _e = (expr);                                        \
    if (_e != hipSuccess) return batch_fail((b), _e, (what));      \
  } while (0)

#define CHECK_BATCH(b)                                                                      \
  do {                                                                                      \
    if (!(b)) return fail(WAVE_EINVAL, "batch is NULL");                                    \
    if ((b)->broken) return fail(WAVE_ESTATE, "batch broken by an earlier device error");  \
  } while (0)

// z-chunk length a streaming sweep of this context uses with tile (ry, nw):
// the requested one (or the automatic one), cut to what the kernels' 32-bit
// chunk window allows.  0 when even one plane is too large to stream.
int stream_zchunk(const wave_ctx* c, int ry, int nw, int zchunk) {
  const int lim = wave::stream_zchunk_limit(c->L.plane);
  if (lim < 1) return 0;
  const int zc = zchunk > 0 ? zchunk : wave::auto_zchunk(c->L.nx, c->L.ny, c->L.nz, ry, nw);
  return std::min(zc, lim);
}

// Automatic z chunk of the persistent launch: half the streaming kernel's
// (its workgroups do not wait for dispatch between items, so shorter items
// cost little and balance the last round better; measured at 512^3 and
// 1024^3), at least 16 planes.
int persist_zchunk(const wave_ctx* c, int ry, int nw, int zchunk) {
  if (zchunk > 0) return stream_zchunk(c, ry, nw, zchunk);
  const int za = wave::auto_zchunk(c->L.nx, c->L.ny, c->L.nz, ry, nw);
  return stream_zchunk(c, ry, nw, std::min(za, std::max(16, za / 2)));
}

// z-chunk length of the pair kernel (128 x ty tiles): as stream_zchunk, the
// automatic length chosen for the tile count of 128-wide tiles; 0 when the
// context holds an eta array (the kernel reads the default profile's tables
// only) or one plane is too large to stream.
// z chunk of the kernels that take the default profile's tables only: the
// two-points-per-lane tiles (128 x ty; semi_nw = 0) and the semi-stencil
// tiles (64 x semi_nw); 0 with an eta array or planes too large to stream.
int pair_zchunk(const wave_ctx* c, int ty, int zchunk, int semi_nw = 0) {
  if (eta_array(&c->d)) return 0;
  const int lim = wave::stream_zchunk_limit(c->L.plane);
  if (lim < 1) return 0;
  const int zc = zchunk > 0  ? zchunk
                 : semi_nw  ? wave::auto_zchunk(c->L.nx, c->L.ny, c->L.nz, 1, semi_nw)
                            : wave::auto_zchunk((c->L.nx + 1) / 2, c->L.ny, c->L.nz, 1, ty);
  return std::min(zc, lim);
}

void batch_drop_graphs(wave_batch* b) {
  for (auto& g : b->graphs) (void)hipGraphExecDestroy(g.second);
  b->graphs.clear();
}

// Rebuild the member tables (static part); targets are filled per run.
void batch_layout(wave_batch* b) {
  b->h_shots.resize(b->members.size());
  b->prefix_blocks.assign(1, 0);
  int64_t begin = 0;
  // rows_per_wave 0: two points per lane, 128 x nw tiles
  const bool pair = b->ry == 0;
  const int ty = pair ? b->nw : b->ry * b->nw;
  for (size_t i = 0; i < b->members.size(); ++i) {
    wave_ctx* c = b->members[i];
    wave::BatchShot& e = b->h_shots[i];
    memset(&e, 0, sizeof(e));
    e.sa = sweep_args(c);
    e.u[0] = c->u_origin(std::min(c->icur, c->iprev));
    e.u[1] = c->u_origin(std::max(c->icur, c->iprev));
    e.tiles_x = (c->L.nx + (pair ? 2 : 1) * wave::kTX - 1) / ((pair ? 2 : 1) * wave::kTX);
    e.tiles_y = (c->L.ny + ty - 1) / ty;
    e.zchunk = pair ? pair_zchunk(c, b->nw, c->zchunk) : stream_zchunk(c, b->ry, b->nw, c->zchunk);
    const int chunks = wave::stream_chunk_count(c->L.nz, c->d.w, e.zchunk, c->damp);
    e.block_begin = begin;
    // tile rows padded to 8 slabs: a multiple of 8 blocks per member
    begin += (int64_t)e.tiles_x * 8 * ((e.tiles_y + 7) / 8) * chunks;
    b->prefix_blocks.push_back(begin);
    e.target = 0;
    e.inj = inject_args(c);
  }
  b->total_blocks = begin;
  b->eta_any = false;
  for (wave_ctx* c : b->members) b->eta_any = b->eta_any || eta_array(&c->d);
  b->layout_dirty = false;
  batch_drop_graphs(b);
}

// One step of the first k members (those still taking steps in this run).
hipError_t batch_launch_step(wave_batch* b, int k) {
  hipError_t e = b->ry == 0
                     ? wave::launch_sweep_batch_pair(b->d_shots, b->d_state, k, b->prefix_blocks[k],
                                                     b->kstore, b->nw, b->stream)
                     : wave::launch_sweep_batch(b->d_shots, b->d_state, k, b->prefix_blocks[k],
                                                b->kstore, b->ry, b->nw, b->eta_any, b->stream);
  if (e != hipSuccess) return e;
  return wave::launch_inject_batch(b->d_shots, b->d_state, k, b->kstore, b->stream);
}

// The captured block of graph_steps steps for the first k members.
hipError_t batch_graph(wave_batch* b, int k, hipGraphExec_t* out) {
  for (auto& g : b->graphs)
    if (g.first == k) {
      *out = g.second;
      return hipSuccess;
    }
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return e;
  for (int t = 0; t < b->graph_steps && e == hipSuccess; ++t) e = batch_launch_step(b, k);
  hipError_t e2 = hipStreamEndCapture(b->stream, &g);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e == hipSuccess) b->graphs.emplace_back(k, *out);
  return e;
}

}  // namespace

extern "C" {

size_t wave_bytes_required(const wave_desc* d) {
  std::string why;
  if (!desc_ok(d, &why)) {
    g_last_error = why;
    return 0;
  }
  return plan_arena(d).total;
}

int wave_admit(const wave_desc* d, size_t budget_bytes, size_t in_use_bytes, size_t* need_out,
               int32_t* fits_now) {
  std::string why;
  if (need_out) *need_out = 0;
  if (fits_now) *fits_now = 0;
  if (!desc_ok(d, &why)) return fail(WAVE_EINVAL, why);
  const size_t need = plan_arena(d).total;
  if (need_out) *need_out = need;
  if (need > budget_bytes)
    return fail(WAVE_EBUDGET, "request needs " + std::to_string(need) +
                                  " bytes of arena, more than the whole budget of " +
                                  std::to_string(budget_bytes));
  if (fits_now) *fits_now = in_use_bytes <= budget_bytes && need <= budget_bytes - in_use_bytes;
  return WAVE_OK;
}

int wave_coefficients(const wave_desc* d, float out[13]) {
  std::string why;
  if (!desc_ok(d, &why)) return fail(WAVE_EINVAL, why);
  if (!out) return fail(WAVE_EINVAL, "out is NULL");
  double c[13];
  coefficients64(d, c);
  for (int m = 0; m < 13; ++m) out[m] = (float)c[m];
  return WAVE_OK;
}

double wave_stability(const wave_desc* d, double vmax) {
  std::string why;
  if (!desc_ok(d, &why) || !(vmax > 0) || !isfinite(vmax)) {
    g_last_error = why.empty() ? "vmax must be finite and > 0" : why;
    return -1.0;
  }
  // symbol of Eq. 3 at the Nyquist wavenumber, per unit h^-2
  double s = kW0;
  for (int m = 0; m < 4; ++m) s += 2.0 * kWm[m] * (((m + 1) & 1) ? -1.0 : 1.0);
  s = fabs(s);
  const double k = s / (d->dx * d->dx) + s / (d->dy * d->dy) + s / (d->dz * d->dz);
  return vmax * d->dt * sqrt(k) / 2.0;
}

int wave_eta_default(const wave_desc* d, double vmax, float* out) {
  std::string why;
  if (!desc_ok(d, &why)) return fail(WAVE_EINVAL, why);
  if (!out || !(vmax > 0) || !isfinite(vmax)) return fail(WAVE_EINVAL, "bad vmax or out");
  const size_t pn = (size_t)d->nx * d->ny;
  if (d->w == 0) {
    memset(out, 0, pn * d->nz * sizeof(float));
    return WAVE_OK;
  }
  for (int k = 0; k < d->nz; ++k) eta_plane(d, vmax, k, out + (size_t)k * pn);
  return WAVE_OK;
}

int wave_alloc(const wave_desc* d, const float* vel, const float* eta, void* dev_arena,
               size_t arena_bytes, void* hip_stream, wave_ctx** out) {
  std::string why;
  if (!out) return fail(WAVE_EINVAL, "out is NULL");
  *out = nullptr;
  if (!desc_ok(d, &why)) return fail(WAVE_EINVAL, why);
  if (!vel) return fail(WAVE_EINVAL, "velocity is NULL");
  const size_t n = (size_t)d->nx * d->ny * d->nz;
  double vmax = 0.0;
  for (size_t p = 0; p < n; ++p) {
    const float v = vel[p];
    if (!(v > 0.0f) || !isfinite(v)) return fail(WAVE_EINVAL, "velocity must be finite and > 0");
    vmax = std::max(vmax, (double)v);
  }
  const bool damp = damping_on(d);
  if (eta_array(d) && !eta) return fail(WAVE_EINVAL, "WAVE_ETA_ARRAY set but eta is NULL");
  if (eta && !eta_array(d))
    return fail(WAVE_EINVAL, "eta given without WAVE_ETA_ARRAY (or with damping off)");
  if (damp && eta) {
    for (size_t p = 0; p < n; ++p)
      if (!(eta[p] >= 0.0f) || !isfinite(eta[p])) return fail(WAVE_EINVAL, "eta must be finite and >= 0");
  }
  const double stab = wave_stability(d, vmax);
  if (stab > 1.0)
    return fail(WAVE_EUNSTABLE, "stability number " + std::to_string(stab) + " > 1 (reduce dt)");
  if (damp) {
    // the damped layer update amplifies where eta is too large: frozen at
    // one point, with s = vp K its share of the Laplacian's symbol, its
    // growth factor solves (1 + 2 eta) l^2 - (2 + 2 eta - eta^2 - s) l + 1 = 0,
    // whose root leaves [-1, 1] through -1 once eta^2 - 4 eta - (4 - s) >= 0,
    // i.e. eta >= 2 + sqrt(8 - s); s is at most 4 stab^2 (the leapfrog
    // bound), so the bound is taken there
    double emax = 0.0;
    if (eta) {
      for (size_t p = 0; p < n; ++p) emax = std::max(emax, (double)eta[p]);
    } else {
      emax = max_default_eta(d, vmax);
    }
    const double lim = eta_limit(stab);
    if (emax >= lim)
      return fail(WAVE_EUNSTABLE, "largest damping eta " + std::to_string(emax) +
                                      " reaches the layer update's bound " + std::to_string(lim) +
                                      " (widen the layer or reduce dt)");
  }
  // the inputs are checked first, so a host without a device can validate a
  // descriptor and its arrays by passing a NULL arena
  if (!dev_arena || ((uintptr_t)dev_arena & 255)) return fail(WAVE_EINVAL, "arena NULL or not 256-byte aligned");
  const ArenaPlan plan = plan_arena(d);
  if (arena_bytes < plan.total)
    return fail(WAVE_ENOMEM, "arena of " + std::to_string(arena_bytes) + " bytes < required " +
                                 std::to_string(plan.total));

  wave_ctx* c = new wave_ctx();
  c->batch = nullptr;
  c->d = *d;
  c->L = wave::make_layout(d->nx, d->ny, d->nz);
  c->plan = plan;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->arena = static_cast<char*>(dev_arena);
  c->es = storage_bytes(d->storage);
  c->icur = 0;
  c->iprev = 1;
  c->iphi = 0;
  c->zchunk2 = 0;
  c->step = 0;
  c->broken = false;
  c->damp = damp;
  c->vmax = vmax;
  coefficients64(d, c->c64);
  for (int m = 0; m < 13; ++m) c->c[m] = (float)c->c64[m];
  c->q[0] = (float)(1.0 / (4.0 * d->dx * d->dx));
  c->q[1] = (float)(1.0 / (4.0 * d->dy * d->dy));
  c->q[2] = (float)(1.0 / (4.0 * d->dz * d->dz));
  c->nsrc = c->nrec = c->trace_count = 0;
  c->src_host.clear();
  c->src_fit2 = true;
  c->shp[0] = c->shp[1] = c->shp[2] = 0;
  c->groups = persistent_groups();
  // default launch (measured one shot at a time, 20-cell layer): the
  // streaming tiles as one persistent launch of 64 x 16 tiles where the grid
  // takes whole 64-plane chunks (512^3: 0.444 ms against 0.447 for one
  // workgroup per tile); on smaller grids the persistent launch's short
  // chunks and few items per workgroup cost more than its balance gains,
  // and one workgroup per 64 x 8 tile is the fastest (160^3: 29.5 us
  // against 44.9; 384^3: 181 against 209)
  const bool large = wave::auto_zchunk(c->L.nx, c->L.ny, c->L.nz, 1, 16) >= 64;
  c->variant = c->groups >= 8 && large ? WAVE_KERNEL_PERSIST : WAVE_KERNEL_STREAM;
  c->ry = 1;
  c->nw = large ? 16 : 8;
  c->zchunk = 0;
  c->timing = false;
  c->events_used = 0;
  c->ev_join = nullptr;
  c->ev_left = nullptr;
  c->left_pending = false;
  c->timing_ms = 0.0;
  c->timing_launches = 0;

  auto bail = [&](int rc) {
    delete c;
    return rc;
  };
  // Set-up runs on the context stream without waiting between steps: zero
  // the arena, bring the compact velocity (and eta) over in one copy each to
  // a staging area (the two u arrays, zeroed again afterwards), and let
  // kernels form vp = (V dt)^2 and scatter into the padded layout.
  const size_t stage_bytes = plan.u[1] + (size_t)c->L.elems * c->es - plan.u[0];
  if (n * 4 > stage_bytes) return bail(fail(WAVE_EINVAL, "internal: staging area too small"));
  char* stage = c->at(plan.u[0]);
  hipError_t e = hipMemsetAsync(c->arena, 0, plan.total, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(stage, vel, n * 4, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = wave::launch_setup_field(reinterpret_cast<float*>(c->at(plan.vp)) + c->L.origin,
                                 reinterpret_cast<const float*>(stage), d->nx, d->ny, d->nz,
                                 c->L.pitch, c->L.plane, d->dt, c->stream);
  if (e == hipSuccess && eta_array(d)) {
    e = hipMemcpyAsync(stage, eta, n * 4, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
      e = wave::launch_setup_field(reinterpret_cast<float*>(c->at(plan.eta)) + c->L.origin,
                                   reinterpret_cast<const float*>(stage), d->nx, d->ny, d->nz,
                                   c->L.pitch, c->L.plane, 0.0, c->stream);
  }
  if (e == hipSuccess) e = hipMemsetAsync(stage, 0, stage_bytes, c->stream);
  if (e != hipSuccess) return bail(dev_fail(nullptr, e, "set-up"));
  std::vector<unsigned char> t;
  if (damp && !eta_array(d)) {
    eta_tables(d, vmax, c->q, t);
    e = hipMemcpyAsync(c->at(plan.etab), t.data(), t.size(), hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return bail(dev_fail(nullptr, e, "eta tables upload"));
  }
  // the host buffers above are pageable and local: wait once, here
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return bail(dev_fail(nullptr, e, "set-up"));
  *out = c;
  return WAVE_OK;
}

int wave_free(wave_ctx* c) {
  if (!c) return WAVE_OK;
  if (c->batch) (void)wave_batch_remove(c->batch, c);
  if (!c->broken) {
    (void)join_batch_work(c);
    (void)hipStreamSynchronize(c->stream);
  }
  for (auto& ev : c->events) {
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  if (c->ev_left) (void)hipEventDestroy(c->ev_left);
  delete c;
  return WAVE_OK;
}

int wave_inject(wave_ctx* c, int32_t i, int32_t j, int32_t k, const float* samples,
                int32_t nsamples) {
  CHECK_CTX(c);
  // a batch copies its members' source and receiver tables when they join
  if (c->batch) return fail(WAVE_EINVAL, "context is a batch member (remove it to add sources)");
  JOIN_CTX(c);
  if (!in_grid(c, i, j, k)) return fail(WAVE_EINVAL, "source index outside the grid");
  if (nsamples < 0 || nsamples > c->d.max_steps) return fail(WAVE_EINVAL, "nsamples outside [0, max_steps]");
  if (nsamples > 0 && !samples) return fail(WAVE_EINVAL, "samples is NULL");
  if (c->nsrc >= c->d.max_src) return fail(WAVE_EINVAL, "source table full (max_src)");
  for (int s = 0; s < nsamples; ++s)
    if (!isfinite(samples[s])) return fail(WAVE_EINVAL, "non-finite wavelet sample");
  std::vector<float> row((size_t)std::max(c->d.max_steps, 1), 0.0f);
  if (nsamples) memcpy(row.data(), samples, (size_t)nsamples * 4);
  const int64_t off = offset_of(c, i, j, k);
  float* wl = reinterpret_cast<float*>(c->at(c->plan.wavelet)) + (size_t)c->nsrc * std::max(c->d.max_steps, 1);
  int64_t* so = reinterpret_cast<int64_t*>(c->at(c->plan.src_off)) + c->nsrc;
  int32_t* sijk = reinterpret_cast<int32_t*>(c->at(c->plan.src_ijk)) + 3 * c->nsrc;
  const int32_t ijk3[3] = {i, j, k};
  HIPCHK(c, hipMemcpyAsync(wl, row.data(), row.size() * 4, hipMemcpyHostToDevice, c->stream), "hipMemcpyAsync");
  HIPCHK(c, hipMemcpyAsync(so, &off, 8, hipMemcpyHostToDevice, c->stream), "hipMemcpyAsync");
  HIPCHK(c, hipMemcpyAsync(sijk, ijk3, 12, hipMemcpyHostToDevice, c->stream), "hipMemcpyAsync");
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  c->nsrc += 1;
  c->src_host.insert(c->src_host.end(), ijk3, ijk3 + 3);
  c->src_fit2 = wave::sweep2_sources_fit(c->src_host.data(), c->nsrc);
  return WAVE_OK;
}

int wave_record(wave_ctx* c, const int32_t* ijk, int32_t nrec) {
  CHECK_CTX(c);
  if (c->batch) return fail(WAVE_EINVAL, "context is a batch member (remove it to set receivers)");
  JOIN_CTX(c);
  if (nrec < 0 || nrec > c->d.max_rec) return fail(WAVE_EINVAL, "nrec outside [0, max_rec]");
  if (nrec > 0 && !ijk) return fail(WAVE_EINVAL, "receiver list is NULL");
  std::vector<int64_t> off((size_t)std::max(nrec, 1));
  for (int r = 0; r < nrec; ++r) {
    if (!in_grid(c, ijk[3 * r], ijk[3 * r + 1], ijk[3 * r + 2]))
      return fail(WAVE_EINVAL, "receiver index outside the grid");
    off[r] = offset_of(c, ijk[3 * r], ijk[3 * r + 1], ijk[3 * r + 2]);
  }
  if (nrec > 0) {
    HIPCHK(c, hipMemcpyAsync(c->at(c->plan.rec_off), off.data(), (size_t)nrec * 8, hipMemcpyHostToDevice, c->stream),
           "hipMemcpyAsync");
    HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  }
  c->nrec = nrec;
  c->trace_count = 0;
  return WAVE_OK;
}

namespace {
// Events around one sweep launch when timing is on (reused across calls).
int timing_begin(wave_ctx* c, hipEvent_t* e1) {
  *e1 = nullptr;
  if (!c->timing) return WAVE_OK;
  if (c->events_used == c->events.size()) {
    hipEvent_t a, b;
    HIPCHK(c, hipEventCreate(&a), "hipEventCreate");
    HIPCHK(c, hipEventCreate(&b), "hipEventCreate");
    c->events.emplace_back(a, b);
  }
  hipEvent_t e0 = c->events[c->events_used].first;
  *e1 = c->events[c->events_used].second;
  c->events_used += 1;
  HIPCHK(c, hipEventRecord(e0, c->stream), "hipEventRecord");
  return WAVE_OK;
}

// z chunk of the two-step sweep (0: it cannot run for this context).
int stream2_zchunk(const wave_ctx* c, int zchunk) {
  if (!two_step(&c->d) || eta_array(&c->d)) return 0;
  const int lim = wave::stream2_zchunk_limit(c->L.plane);
  if (lim < 1) return 0;
  const int zc = zchunk > 0 ? zchunk : wave::auto_zchunk2(c->L.nx, c->L.ny, c->L.nz);
  return std::min(zc, lim);
}

// Steps n+1 and n+2 in one launch, then receivers of step n and sources and
// receivers of step n+1 (Alg. 1 order; the sources of step n are added
// inside the sweep).
int step_pair(wave_ctx* c, int zc) {
  int other[2], k = 0;
  for (int i = 0; i < 4 && k < 2; ++i)
    if (i != c->icur && i != c->iprev) other[k++] = i;
  wave::Sweep2Args g;
  g.s = sweep_args(c);
  g.s.cur = c->u_origin(c->icur);
  g.s.nxt = nullptr;
  g.prev = c->u_origin(c->iprev);
  g.out1 = c->u_origin(other[0]);
  g.out2 = c->u_origin(other[1]);
  g.phi_out = c->damp ? c->f_origin(c->plan.phi[1 - c->iphi]) : nullptr;
  g.nsrc = c->nsrc;
  g.src_ijk = reinterpret_cast<const int32_t*>(c->at(c->plan.src_ijk));
  g.wavelet = reinterpret_cast<const float*>(c->at(c->plan.wavelet));
  g.max_steps = std::max(c->d.max_steps, 1);
  g.step = (int32_t)c->step;
  hipEvent_t e1;
  int rc = timing_begin(c, &e1);
  if (rc) return rc;
  hipError_t e = wave::launch_sweep2(g, c->d.storage, zc, c->stream);
  if (e != hipSuccess) return dev_fail(c, e, "two-step sweep launch");
  if (e1) HIPCHK(c, hipEventRecord(e1, c->stream), "hipEventRecord");
  wave::InjectArgs ia = inject_args(c);
  double* traces = c->nrec > 0 ? reinterpret_cast<double*>(c->at(c->plan.traces)) : nullptr;
  if (c->nrec > 0) {   // receivers of step n: u^{n+1}, its sources already in
    ia.u = g.out1;
    ia.nsrc = 0;
    ia.step = (int32_t)c->step;
    ia.traces = traces;
    ia.trace_row = c->trace_count;
    e = wave::launch_inject_record(ia, kernel_storage(&c->d), c->stream);
    if (e != hipSuccess) return dev_fail(c, e, "record launch");
  }
  if (c->nsrc > 0 || c->nrec > 0) {   // sources and receivers of step n+1
    ia.u = g.out2;
    ia.nsrc = c->nsrc;
    ia.step = (int32_t)c->step + 1;
    ia.traces = traces;
    ia.trace_row = c->trace_count + (c->nrec > 0 ? 1 : 0);
    e = wave::launch_inject_record(ia, kernel_storage(&c->d), c->stream);
    if (e != hipSuccess) return dev_fail(c, e, "inject/record launch");
  }
  c->iprev = other[0];
  c->icur = other[1];
  if (c->damp) c->iphi = 1 - c->iphi;
  c->step += 2;
  if (c->nrec > 0) c->trace_count += 2;
  return WAVE_OK;
}
}  // namespace

int wave_step(wave_ctx* c, int32_t n) {
  CHECK_CTX(c);
  JOIN_CTX(c);
  if (c->batch) return fail(WAVE_EINVAL, "context is a batch member (step it with wave_batch_run)");
  if (n < 0) return fail(WAVE_EINVAL, "n < 0");
  if (c->nrec > 0 && (int64_t)c->trace_count + n > c->d.max_steps)
    return fail(WAVE_EINVAL, "trace buffer would overflow max_steps");
  if (c->step + n > 0x7fffffff) return fail(WAVE_EINVAL, "step counter overflow");
  // two steps per launch while at least two remain (and the sources fit its
  // tiles' lists)
  if (c->variant == WAVE_KERNEL_STREAM2 && c->src_fit2) {
    const int zc2 = stream2_zchunk(c, c->zchunk2);
    if (zc2 >= 1) {
      for (; n >= 2; n -= 2) {
        const int rc = step_pair(c, zc2);
        if (rc) return rc;
      }
    }
  }
  if (n == 0) return WAVE_OK;
  wave::SweepArgs sa = sweep_args(c);
  const int zc = c->variant == WAVE_KERNEL_PERSIST ? persist_zchunk(c, c->ry, c->nw, c->zchunk)
                                                    : stream_zchunk(c, c->ry, c->nw, c->zchunk);
  const bool direct = c->variant == WAVE_KERNEL_DIRECT || zc < 1;
  const bool shape25 = c->variant == WAVE_KERNEL_RING || c->variant == WAVE_KERNEL_SHIFT;
  const int zcp = c->variant == WAVE_KERNEL_PAIR   ? pair_zchunk(c, c->shp[1], c->shp[2])
                  : c->variant == WAVE_KERNEL_SEMI ? pair_zchunk(c, 0, c->shp[2], c->shp[1])
                                                   : 0;
  const int zc25 = !shape25 ? 0
                   : c->shp[2] > 0 ? std::min(c->shp[2], c->L.nz)
                                   : wave::auto_zchunk25(c->L.nx, c->L.ny, c->L.nz, c->shp[1]);
  auto launch_one = [&](const wave::SweepArgs& s) -> hipError_t {
    if (c->variant == WAVE_KERNEL_GMEM)
      return wave::launch_sweep_gmem(s, kernel_storage(&c->d), c->shp[0], c->shp[1], c->shp[2], c->stream);
    if (shape25)
      return wave::launch_sweep_25d(s, kernel_storage(&c->d), c->variant == WAVE_KERNEL_RING ? 0 : 1,
                                    c->shp[1], zc25, c->stream);
    if (c->variant == WAVE_KERNEL_PAIR)
      return wave::launch_sweep_pair(s, kernel_storage(&c->d), c->shp[1], zcp, c->stream);
    if (c->variant == WAVE_KERNEL_SEMI)
      return wave::launch_sweep_semi(s, kernel_storage(&c->d), c->shp[1], zcp, c->stream);
    if (c->variant == WAVE_KERNEL_SHUFFLE)
      return wave::launch_sweep_shuffle(s, kernel_storage(&c->d), c->shp[1],
                                        stream_zchunk(c, 1, c->shp[1], c->shp[2]), c->stream);
    if (c->variant == WAVE_KERNEL_PERSIST && !direct)
      return wave::launch_sweep_persist(s, kernel_storage(&c->d), c->ry, c->nw, zc, c->groups, c->stream);
    return direct ? wave::launch_sweep_direct(s, kernel_storage(&c->d), c->stream)
                  : wave::launch_sweep_stream(s, kernel_storage(&c->d), c->ry, c->nw, zc, c->stream);
  };

  wave::InjectArgs ia = inject_args(c);

  for (int t = 0; t < n; ++t) {
    sa.cur = c->u_origin(c->icur);
    sa.nxt = c->u_origin(c->iprev);
    sa.step = (int32_t)c->step;
    hipEvent_t e1;
    int rc = timing_begin(c, &e1);
    if (rc) return rc;
    hipError_t e = launch_one(sa);
    if (e != hipSuccess) return dev_fail(c, e, "sweep launch");
    if (e1) HIPCHK(c, hipEventRecord(e1, c->stream), "hipEventRecord");
    if (c->nsrc > 0 || c->nrec > 0) {
      ia.u = sa.nxt;
      ia.step = (int32_t)c->step;
      ia.traces = c->nrec > 0 ? reinterpret_cast<double*>(c->at(c->plan.traces)) : nullptr;
      ia.trace_row = c->trace_count;
      e = wave::launch_inject_record(ia, kernel_storage(&c->d), c->stream);
      if (e != hipSuccess) return dev_fail(c, e, "inject/record launch");
    }
    std::swap(c->icur, c->iprev);
    c->step += 1;
    if (c->nrec > 0) c->trace_count += 1;
  }
  return WAVE_OK;
}

int wave_sync(wave_ctx* c) {
  CHECK_CTX(c);
  JOIN_CTX(c);
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  return WAVE_OK;
}

int64_t wave_step_count(const wave_ctx* c) { return c ? c->step : -1; }

int wave_read_field(wave_ctx* c, int32_t which, float* out) {
  CHECK_CTX(c);
  JOIN_CTX(c);
  if (!out) return fail(WAVE_EINVAL, "out is NULL");
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  const size_t pn = (size_t)c->L.nx * c->L.ny;
  switch (which) {
    case WAVE_FIELD_U: return download_u(c, c->icur, out);
    case WAVE_FIELD_UPREV: return download_u(c, c->iprev, out);
    case WAVE_FIELD_ETA:
      if (c->plan.etab != (size_t)-1) {   // default profile held as tables
        for (int k = 0; k < c->L.nz; ++k) eta_plane(&c->d, c->vmax, k, out + (size_t)k * pn);
        return WAVE_OK;
      }
      [[fallthrough]];
    case WAVE_FIELD_PHI:
    case WAVE_FIELD_VP: {
      const size_t off = which == WAVE_FIELD_PHI ? c->plan.phi[c->iphi] : which == WAVE_FIELD_VP ? c->plan.vp : c->plan.eta;
      if (off == (size_t)-1) {
        memset(out, 0, pn * c->L.nz * sizeof(float));
        return WAVE_OK;
      }
      return download_f32(c, c->at(off), out);
    }
  }
  return fail(WAVE_EINVAL, "unknown field id");
}

int wave_write_field(wave_ctx* c, int32_t which, const float* in) {
  CHECK_CTX(c);
  JOIN_CTX(c);
  if (!in) return fail(WAVE_EINVAL, "input is NULL");
  const size_t n = (size_t)c->L.nx * c->L.ny * c->L.nz;
  for (size_t p = 0; p < n; ++p)
    if (!isfinite(in[p])) return fail(WAVE_EINVAL, "non-finite value");
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  switch (which) {
    case WAVE_FIELD_U: return upload_u(c, c->icur, in);
    case WAVE_FIELD_UPREV: return upload_u(c, c->iprev, in);
    case WAVE_FIELD_PHI: {
      if (c->plan.phi[c->iphi] == (size_t)-1) return fail(WAVE_EINVAL, "no phi field with damping off");
      return upload_f32(c, c->at(c->plan.phi[c->iphi]), in);
    }
  }
  return fail(WAVE_EINVAL, "field is read-only or unknown");
}

int wave_read_traces(wave_ctx* c, double* out, int32_t* steps_out) {
  CHECK_CTX(c);
  JOIN_CTX(c);
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  if (steps_out) *steps_out = c->trace_count;
  if (out && c->nrec > 0 && c->trace_count > 0) {
    HIPCHK(c,
           hipMemcpyAsync(out, c->at(c->plan.traces), (size_t)c->trace_count * c->nrec * 8,
                          hipMemcpyDeviceToHost, c->stream),
           "hipMemcpyAsync");
    HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  }
  return WAVE_OK;
}

int wave_energy(wave_ctx* c, double* out) {
  CHECK_CTX(c);
  JOIN_CTX(c);
  if (!out) return fail(WAVE_EINVAL, "out is NULL");
  wave::EnergyArgs ea;
  ea.cur = c->u_origin(c->icur);
  ea.prev = c->u_origin(c->iprev);
  ea.vp = c->f_origin(c->plan.vp);
  ea.nx = c->L.nx;
  ea.ny = c->L.ny;
  ea.nz = c->L.nz;
  ea.pitch = c->L.pitch;
  ea.plane = c->L.plane;
  memcpy(ea.c, c->c64, sizeof(ea.c));
  ea.partial = reinterpret_cast<double*>(c->at(c->plan.partial));
  ea.result = reinterpret_cast<double*>(c->at(c->plan.eres));
  hipError_t e = wave::launch_energy(ea, kernel_storage(&c->d), c->stream);
  if (e != hipSuccess) return dev_fail(c, e, "energy launch");
  double r[2];
  HIPCHK(c, hipMemcpyAsync(r, ea.result, 16, hipMemcpyDeviceToHost, c->stream), "hipMemcpyAsync");
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  *out = r[0] - r[1];
  return WAVE_OK;
}

// ---- energy without allocation ---------------------------------------------
// Workspace of wave_energy_noalloc: the per-row partial sums of the energy
// (kinetic, potential) for up to kScratchRows rows (ny * nz), then the two
// totals.  One copy per GPU, kept until the process ends (16 MiB).  In host
// code `scratch` only names the symbol; its device address, per GPU, comes
// from hipGetSymbolAddress with that GPU current.
namespace {
constexpr int64_t kScratchRows = int64_t(1) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[2 * kScratchRows + 2];
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the GPU that holds the context's arena,
// looked up once per GPU.
int scratch_for(wave_ctx* c, double** out) {
  hipPointerAttribute_t at;
  HIPCHK(c, hipPointerGetAttributes(&at, c->arena), "hipPointerGetAttributes");
  const int dev = at.device;
  if (dev < 0 || dev >= kMaxDevices) return fail(WAVE_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = 0;
    HIPCHK(c, hipGetDevice(&cur), "hipGetDevice");
    if (cur != dev) HIPCHK(c, hipSetDevice(dev), "hipSetDevice");
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) HIPCHK(c, hipSetDevice(cur), "hipSetDevice");
    if (e != hipSuccess) return dev_fail(c, e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return WAVE_OK;
}
}  // namespace

int wave_energy_noalloc(wave_ctx* c, double* dev_out) {
  CHECK_CTX(c);
  JOIN_CTX(c);
  if (!dev_out) return fail(WAVE_EINVAL, "dev_out is NULL");
  const int64_t rows = (int64_t)c->L.ny * c->L.nz;
  if (rows > kScratchRows)
    return fail(WAVE_EINVAL, "ny * nz = " + std::to_string(rows) + " exceeds the " +
                                 std::to_string(kScratchRows) + " rows of the static workspace");
  double* ws = nullptr;
  const int rc = scratch_for(c, &ws);
  if (rc != WAVE_OK) return rc;
  wave::EnergyArgs ea;
  ea.cur = c->u_origin(c->icur);
  ea.prev = c->u_origin(c->iprev);
  ea.vp = c->f_origin(c->plan.vp);
  ea.nx = c->L.nx;
  ea.ny = c->L.ny;
  ea.nz = c->L.nz;
  ea.pitch = c->L.pitch;
  ea.plane = c->L.plane;
  memcpy(ea.c, c->c64, sizeof(ea.c));
  ea.partial = ws;
  ea.result = dev_out;
  const hipError_t e = wave::launch_energy(ea, kernel_storage(&c->d), c->stream);
  if (e != hipSuccess) return dev_fail(c, e, "energy launch");
  return WAVE_OK;
}

int wave_set_kernel(wave_ctx* c, int32_t variant, int32_t ry, int32_t nw, int32_t zchunk) {
  CHECK_CTX(c);
  if (variant == WAVE_KERNEL_DIRECT) {
    c->variant = variant;
    return WAVE_OK;
  }
  if (variant == WAVE_KERNEL_STREAM2) {
    if (stream2_zchunk(c, 0) < 1)
      return fail(WAVE_EINVAL, "two steps per launch need WAVE_TWO_STEP, no eta array, and planes small enough");
    if (zchunk < 0) return fail(WAVE_EINVAL, "zchunk < 0");
    c->variant = variant;
    c->zchunk2 = zchunk;
    return WAVE_OK;
  }
  if (variant == WAVE_KERNEL_GMEM) {
    if (!wave::gmem_config_supported(ry, nw, zchunk))
      return fail(WAVE_EINVAL, "3-D tile (bx, by, bz) not compiled");
    c->variant = variant;
    c->shp[0] = ry;
    c->shp[1] = nw;
    c->shp[2] = zchunk;
    return WAVE_OK;
  }
  if (variant == WAVE_KERNEL_PAIR) {
    if (ry != 1 || (nw != 8 && nw != 16)) return fail(WAVE_EINVAL, "pair kernel needs rows_per_wave 1, 8 or 16 rows");
    if (zchunk < 0) return fail(WAVE_EINVAL, "zchunk < 0");
    if (pair_zchunk(c, nw, zchunk) < 1)
      return fail(WAVE_EINVAL, "pair kernel: no eta array, and planes small enough to stream");
    c->variant = variant;
    c->shp[0] = 1;
    c->shp[1] = nw;
    c->shp[2] = zchunk;
    return WAVE_OK;
  }
  if (variant == WAVE_KERNEL_SEMI) {
    if (ry != 1 || (nw != 8 && nw != 16)) return fail(WAVE_EINVAL, "semi-stencil kernel needs rows_per_wave 1, 8 or 16 rows");
    if (zchunk < 0) return fail(WAVE_EINVAL, "zchunk < 0");
    if (pair_zchunk(c, 0, zchunk, nw) < 1)
      return fail(WAVE_EINVAL, "semi-stencil kernel: no eta array, and planes small enough to stream");
    c->variant = variant;
    c->shp[0] = 1;
    c->shp[1] = nw;
    c->shp[2] = zchunk;
    return WAVE_OK;
  }
  if (variant == WAVE_KERNEL_SHUFFLE) {
    if (ry != 1 || (nw != 8 && nw != 16)) return fail(WAVE_EINVAL, "shuffle kernel needs rows_per_wave 1, 8 or 16 rows");
    if (zchunk < 0) return fail(WAVE_EINVAL, "zchunk < 0");
    if (stream_zchunk(c, 1, nw, zchunk) < 1) return fail(WAVE_EINVAL, "planes too large to stream");
    c->variant = variant;
    c->shp[0] = 1;
    c->shp[1] = nw;
    c->shp[2] = zchunk;
    return WAVE_OK;
  }
  if (variant == WAVE_KERNEL_RING || variant == WAVE_KERNEL_SHIFT) {
    if (ry != 1 || (nw != 8 && nw != 16)) return fail(WAVE_EINVAL, "2.5-D shape needs rows_per_wave 1, 8 or 16 rows");
    if (zchunk < 0) return fail(WAVE_EINVAL, "zchunk < 0");
    c->variant = variant;
    c->shp[0] = 1;
    c->shp[1] = nw;
    c->shp[2] = zchunk;
    return WAVE_OK;
  }
  if (variant == WAVE_KERNEL_PERSIST && (ry != 1 || (nw != 8 && nw != 16)))
    return fail(WAVE_EINVAL, "persistent sweep tiles: (1, 8), (1, 16)");
  if (variant != WAVE_KERNEL_STREAM && variant != WAVE_KERNEL_PERSIST)
    return fail(WAVE_EINVAL, "unknown kernel variant");
  if (!wave::stream_config_supported(ry, nw, eta_array(&c->d)))
    return fail(WAVE_EINVAL, "tile (rows_per_wave, waves) not compiled for this context");
  if (zchunk < 0) return fail(WAVE_EINVAL, "zchunk < 0");
  c->variant = variant;
  c->ry = ry;
  c->nw = nw;
  c->zchunk = zchunk;
  return WAVE_OK;
}

namespace {
// Tile shapes compiled into the library, in tuning order.
constexpr int kShapes[][2] = {{1, 16}, {2, 16}, {1, 8}, {2, 8}, {2, 4}};
}  // namespace

int wave_tune(wave_ctx* c, int32_t trial_steps, int32_t chosen[4]) {
  CHECK_CTX(c);
  if (c->batch) return fail(WAVE_EINVAL, "context is a batch member (use wave_batch_tune)");
  if (trial_steps < 1) return fail(WAVE_EINVAL, "trial_steps < 1");
  const int nshape = (int)(sizeof(kShapes) / sizeof(kShapes[0]));
  const int nz = c->L.nz;
  // candidates {variant, rows_per_wave, waves_per_group, zchunk}
  std::vector<std::array<int, 4>> cand;
  auto add = [&](const std::array<int, 4>& e) {
    if (std::find(cand.begin(), cand.end(), e) == cand.end()) cand.push_back(e);
  };
  const bool ea = eta_array(&c->d);
  // the persistent launch first (the default), at its automatic chunk and
  // twice that
  for (const auto& t : {std::array<int, 2>{1, 16}, std::array<int, 2>{1, 8}}) {
    if (c->groups < 8) continue;
    const int za = persist_zchunk(c, t[0], t[1], 0);
    for (int z : {za, std::min(nz, 2 * za)}) {
      const int zc = stream_zchunk(c, t[0], t[1], z);
      if (zc >= 1) add({WAVE_KERNEL_PERSIST, t[0], t[1], zc});
    }
  }
  for (int k = 0; k < nshape; ++k) {
    const int ry = kShapes[k][0], nw = kShapes[k][1];
    if (!wave::stream_config_supported(ry, nw, ea)) continue;
    const int za = wave::auto_zchunk(c->L.nx, c->L.ny, nz, ry, nw);
    for (int z : {za, std::max(8, za / 2), std::min(nz, 2 * za)}) {
      const int zc = stream_zchunk(c, ry, nw, z);
      if (zc >= 1) add({WAVE_KERNEL_STREAM, ry, nw, zc});
    }
  }
  if (stream2_zchunk(c, 0) >= 1) {
    const int za = wave::auto_zchunk2(c->L.nx, c->L.ny, nz);
    for (int z : {za, std::max(32, za / 2), std::min(nz, 2 * za)}) {
      const int zc = stream2_zchunk(c, z);
      if (zc >= 1) add({WAVE_KERNEL_STREAM2, c->ry, c->nw, zc});
    }
  }
  // two points per lane, at the automatic and the doubled chunk length
  for (int ty : {16, 8}) {
    const int za = pair_zchunk(c, ty, 0);
    if (za < 1) continue;
    add({WAVE_KERNEL_PAIR, 1, ty, za});
    const int z2 = pair_zchunk(c, ty, std::min(nz, 2 * za));
    if (z2 != za) add({WAVE_KERNEL_PAIR, 1, ty, z2});
  }
  // x neighbours by wavefront shuffles, at the automatic chunk
  for (int nw : {16, 8}) {
    const int zc = stream_zchunk(c, 1, nw, 0);
    if (zc >= 1) add({WAVE_KERNEL_SHUFFLE, 1, nw, zc});
  }
  // the paper's other code shapes, last (they must beat the streaming kernel
  // by the margin below to be picked)
  if (!cand.empty()) {
    add({WAVE_KERNEL_GMEM, 8, 8, 8});
    add({WAVE_KERNEL_GMEM, 64, 4, 4});
    add({WAVE_KERNEL_RING, 1, 16, 0});
    add({WAVE_KERNEL_SHIFT, 1, 16, 0});
  }
  if (cand.empty()) {  // planes too large to stream: the direct kernel is the only choice
    c->variant = WAVE_KERNEL_DIRECT;
    if (chosen) chosen[0] = chosen[1] = chosen[2] = chosen[3] = 0;
    return WAVE_OK;
  }
  // a two-step candidate runs an even number of steps
  const int32_t trial2 = trial_steps + (trial_steps & 1);
  int64_t total = 0;
  // each candidate first takes one untimed step (the first launch after a
  // kernel switch runs cold), then its timed trial
  for (const auto& e : cand) total += 1 + (e[0] == WAVE_KERNEL_STREAM2 ? trial2 : trial_steps);
  if (c->nrec > 0 && (int64_t)c->trace_count + total > c->d.max_steps)
    return fail(WAVE_EINVAL, "tuning steps would overflow the trace buffer");
  if (c->step + total > 0x7fffffff) return fail(WAVE_EINVAL, "step counter overflow");
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0), "hipEventCreate");
  HIPCHK(c, hipEventCreate(&e1), "hipEventCreate");
  const int variant = c->variant, ry0 = c->ry, nw0 = c->nw, zc0 = c->zchunk, zc20 = c->zchunk2;
  const int shp0[3] = {c->shp[0], c->shp[1], c->shp[2]};
  auto is_shape = [](int v) {
    return v == WAVE_KERNEL_GMEM || v == WAVE_KERNEL_RING || v == WAVE_KERNEL_SHIFT ||
           v == WAVE_KERNEL_PAIR || v == WAVE_KERNEL_SEMI || v == WAVE_KERNEL_SHUFFLE;
  };
  float best = 0.0f;
  std::array<int, 4> pick = {variant, ry0, nw0, zc0};
  int rc = WAVE_OK;
  for (const auto& e : cand) {
    c->variant = e[0];
    if (is_shape(e[0])) {
      for (int k = 0; k < 3; ++k) c->shp[k] = e[k + 1];
    } else {
      c->ry = e[1];
      c->nw = e[2];
      if (e[0] == WAVE_KERNEL_STREAM2) c->zchunk2 = e[3]; else c->zchunk = e[3];
    }
    const int32_t steps = e[0] == WAVE_KERNEL_STREAM2 ? trial2 : trial_steps;
    rc = wave_step(c, 1);
    if (rc != WAVE_OK) break;
    hipError_t he = hipEventRecord(e0, c->stream);
    if (he == hipSuccess) rc = wave_step(c, steps);
    if (he == hipSuccess && rc == WAVE_OK) he = hipEventRecord(e1, c->stream);
    if (he == hipSuccess && rc == WAVE_OK) he = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (he == hipSuccess && rc == WAVE_OK) he = hipEventElapsedTime(&ms, e0, e1);
    if (he != hipSuccess) rc = dev_fail(c, he, "tuning");
    if (rc != WAVE_OK) break;
    // a later candidate must win by 1.5 %: shapes within timing noise of
    // each other keep the earlier (default-first) order, so runs pick stably
    const float per = ms / (float)steps;
    if (best == 0.0f || per < best * 0.985f) {
      best = per;
      pick = e;
    }
    // the single-step settings stay those of the best single-step candidate
    if (e[0] == WAVE_KERNEL_STREAM2) c->zchunk2 = zc20;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != WAVE_OK) {
    c->variant = variant;
    c->ry = ry0;
    c->nw = nw0;
    c->zchunk = zc0;
    c->zchunk2 = zc20;
    for (int k = 0; k < 3; ++k) c->shp[k] = shp0[k];
    return rc;
  }
  c->variant = pick[0];
  if (is_shape(pick[0])) {
    for (int k = 0; k < 3; ++k) c->shp[k] = pick[k + 1];
  } else {
    c->ry = pick[1];
    c->nw = pick[2];
    if (pick[0] == WAVE_KERNEL_STREAM2) {
      c->zchunk2 = pick[3];
    } else {
      c->zchunk = pick[3];
    }
  }
  if (chosen)
    for (int k = 0; k < 4; ++k) chosen[k] = pick[k];
  return WAVE_OK;
}

int wave_set_timing(wave_ctx* c, int32_t on) {
  CHECK_CTX(c);
  JOIN_CTX(c);
  c->timing = on != 0;
  c->events_used = 0;
  c->timing_ms = 0.0;
  c->timing_launches = 0;
  return WAVE_OK;
}

int wave_read_timing(wave_ctx* c, double* ms_total, int64_t* launches) {
  CHECK_CTX(c);
  JOIN_CTX(c);
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  for (size_t k = 0; k < c->events_used; ++k) {
    float ms = 0.0f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->events[k].first, c->events[k].second), "hipEventElapsedTime");
    c->timing_ms += ms;
    c->timing_launches += 1;
  }
  c->events_used = 0;
  if (ms_total) *ms_total = c->timing_ms;
  if (launches) *launches = c->timing_launches;
  return WAVE_OK;
}

double wave_sweep_bytes(const wave_ctx* c) {
  if (!c) return -1.0;
  const double total = (double)c->d.nx * c->d.ny * c->d.nz;
  double inner = total;
  if (c->damp) {
    const double w2 = 2.0 * c->d.w;
    inner = (c->d.nx - w2) * (c->d.ny - w2) * (c->d.nz - w2);
  }
  const double layer = total - inner;
  const double es = c->es;
  const double eta_b = c->plan.eta == (size_t)-1 ? 0.0 : 4.0;
  if (c->variant == WAVE_KERNEL_STREAM2 && c->src_fit2 && stream2_zchunk(c, c->zchunk2) >= 1)
    // one launch = two steps: u^n, u^{n-1}, vp read, u^{n+1}, u^{n+2}
    // written; a layer point adds phi^n read and phi^{n+2} written
    return inner * (4.0 * es + 4.0) + layer * (4.0 * es + 12.0);
  return inner * (3.0 * es + 4.0) + layer * (3.0 * es + 12.0 + eta_b);
}

int wave_stream_copy(void* dst, const void* src, size_t bytes, void* hip_stream) {
  if (!dst || !src || (bytes % 16) || ((uintptr_t)dst & 15) || ((uintptr_t)src & 15))
    return fail(WAVE_EINVAL, "copy needs 16-byte aligned pointers and a multiple of 16 bytes");
  hipError_t e = wave::launch_stream_copy(dst, src, bytes, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return dev_fail(nullptr, e, "copy launch");
  return WAVE_OK;
}

int wave_stream_mix(int32_t kind, void* dst, const void* a, const void* b, const void* c,
                    size_t bytes, void* hip_stream) {
  auto al = [](const void* p) { return p && ((uintptr_t)p & 15) == 0; };
  if ((kind != 0 && kind != 1) || !al(dst) || !al(a) || (bytes % 16) ||
      (kind == 1 && (!al(b) || !al(c))))
    return fail(WAVE_EINVAL, "kind 0 or 1, 16-byte aligned pointers, a multiple of 16 bytes");
  hipError_t e = wave::launch_stream_mix(kind, dst, a, b, c, bytes, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return dev_fail(nullptr, e, "stream launch");
  return WAVE_OK;
}

size_t wave_batch_bytes_required(int32_t max_shots) {
  if (max_shots < 1 || max_shots > 65536) {
    g_last_error = "max_shots outside [1, 65536]";
    return 0;
  }
  return batch_table_bytes(max_shots, nullptr);
}

namespace {
// Releases what wave_batch_create acquired (any subset of it).
void batch_release(wave_batch* b) {
  batch_drop_graphs(b);
  for (int k = 0; k < 2; ++k) {
    if (b->ev_copy[k]) (void)hipEventDestroy(b->ev_copy[k]);
    if (b->pinned[k]) (void)hipHostFree(b->pinned[k]);
  }
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}
}  // namespace

int wave_batch_create(int32_t storage, int32_t max_shots, void* dev_arena, size_t arena_bytes,
                      void* hip_stream, wave_batch** out) {
  if (!out) return fail(WAVE_EINVAL, "out is NULL");
  *out = nullptr;
  if (storage != WAVE_F32 && storage != WAVE_BF16 && storage != WAVE_F16)
    return fail(WAVE_EINVAL, "unknown storage type");
  if (max_shots < 1 || max_shots > 65536) return fail(WAVE_EINVAL, "max_shots outside [1, 65536]");
  if (!dev_arena || ((uintptr_t)dev_arena & 255)) return fail(WAVE_EINVAL, "arena NULL or not 256-byte aligned");
  size_t soff = 0;
  const size_t need = batch_table_bytes(max_shots, &soff);
  if (arena_bytes < need) return fail(WAVE_ENOMEM, "batch arena too small");
  wave_batch* b = new wave_batch();
  b->storage = storage;
  b->kstore = storage;
  b->max_shots = max_shots;
  b->user_stream = static_cast<hipStream_t>(hip_stream);
  b->arena = static_cast<char*>(dev_arena);
  b->arena_bytes = arena_bytes;
  b->d_shots = reinterpret_cast<wave::BatchShot*>(b->arena);
  b->d_state = reinterpret_cast<wave::BatchState*>(b->arena + soff);
  b->ry = 1;
  b->nw = 16;
  b->eta_any = false;
  b->total_blocks = 0;
  b->layout_dirty = true;
  b->graph_steps = 0;
  b->broken = false;
  b->runs = 0;
  b->stream = nullptr;
  b->ev_in = b->ev_out = b->ev_copy[0] = b->ev_copy[1] = nullptr;
  b->pinned[0] = b->pinned[1] = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
  for (int k = 0; k < 2 && e == hipSuccess; ++k) {
    e = hipEventCreateWithFlags(&b->ev_copy[k], hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&b->pinned[k]), need, hipHostMallocDefault);
  }
  if (e != hipSuccess) {
    batch_release(b);
    return fail(WAVE_EDEVICE, std::string("batch stream/events/pinned tables: ") + hipGetErrorString(e));
  }
  *out = b;
  return WAVE_OK;
}

int wave_batch_add(wave_batch* b, wave_ctx* c, int32_t nsteps) {
  CHECK_BATCH(b);
  CHECK_CTX(c);
  if (c->batch) return fail(WAVE_EINVAL, "context already in a batch");
  if (c->d.storage != b->storage) return fail(WAVE_EINVAL, "storage type differs from the batch's");
  if (!b->members.empty() && kernel_storage(&c->d) != b->kstore)
    return fail(WAVE_EINVAL, "rounding (WAVE_STOCH_ROUND) differs from the batch members'");
  if ((int)b->members.size() >= b->max_shots) return fail(WAVE_EINVAL, "batch full");
  if (nsteps < 0) return fail(WAVE_EINVAL, "nsteps < 0");
  if (c->nrec > 0 && (int64_t)c->trace_count + nsteps > c->d.max_steps)
    return fail(WAVE_EINVAL, "trace buffer would overflow max_steps");
  if (c->step + nsteps > 0x7fffffff) return fail(WAVE_EINVAL, "step counter overflow");
  if (wave::stream_zchunk_limit(c->L.plane) < 1)
    return fail(WAVE_EINVAL, "z planes too large for the batched streaming kernel");
  if (b->ry == 0 && eta_array(&c->d))
    return fail(WAVE_EINVAL, "the batch runs the two-points-per-lane kernel, which takes no eta array");
  if (b->ry > 0 && !wave::stream_config_supported(b->ry, b->nw, eta_array(&c->d)))
    return fail(WAVE_EINVAL, "the batch's tile is not compiled for a member with an eta array");
  // the batch's launches come after everything queued so far on the member's stream
  JOIN_CTX(c);
  if (c->stream != b->user_stream) {
    if (!c->ev_join) HIPCHK(c, hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming), "hipEventCreate");
    HIPCHK(c, hipEventRecord(c->ev_join, c->stream), "hipEventRecord");
    BCHK(b, hipStreamWaitEvent(b->stream, c->ev_join, 0), "hipStreamWaitEvent");
  }
  if (b->members.empty()) b->kstore = kernel_storage(&c->d);
  b->members.push_back(c);
  b->remaining.push_back(nsteps);
  c->batch = b;
  b->layout_dirty = true;
  return WAVE_OK;
}

int wave_batch_remove(wave_batch* b, wave_ctx* c) {
  CHECK_BATCH(b);
  if (!c || c->batch != b) return fail(WAVE_EINVAL, "context is not a member");
  for (size_t i = 0; i < b->members.size(); ++i) {
    if (b->members[i] == c) {
      b->members.erase(b->members.begin() + i);
      b->remaining.erase(b->remaining.begin() + i);
      break;
    }
  }
  c->batch = nullptr;
  b->layout_dirty = true;
  if (c->stream != b->user_stream && !b->broken) {
    // the context's next work waits for the runs it took part in
    if (!c->ev_left) HIPCHK(c, hipEventCreateWithFlags(&c->ev_left, hipEventDisableTiming), "hipEventCreate");
    HIPCHK(c, hipEventRecord(c->ev_left, b->stream), "hipEventRecord");
    c->left_pending = true;
  }
  return WAVE_OK;
}

int wave_batch_remaining(const wave_batch* b, const wave_ctx* c, int32_t* remaining) {
  if (!b || !c || !remaining) return fail(WAVE_EINVAL, "NULL argument");
  for (size_t i = 0; i < b->members.size(); ++i)
    if (b->members[i] == c) {
      *remaining = b->remaining[i];
      return WAVE_OK;
    }
  return fail(WAVE_EINVAL, "context is not a member");
}

int wave_batch_set_kernel(wave_batch* b, int32_t ry, int32_t nw) {
  CHECK_BATCH(b);
  if (ry == 0) {   // two points per lane
    if (nw != 8 && nw != 16) return fail(WAVE_EINVAL, "two points per lane: 8 or 16 rows");
    for (wave_ctx* c : b->members)
      if (eta_array(&c->d)) return fail(WAVE_EINVAL, "a member holds an eta array (two points per lane takes none)");
  } else {
    bool ea = false;
    for (wave_ctx* c : b->members) ea = ea || eta_array(&c->d);
    if (!wave::stream_config_supported(ry, nw, ea))
      return fail(WAVE_EINVAL, "tile (rows_per_wave, waves) not compiled for these members");
  }
  b->ry = ry;
  b->nw = nw;
  b->layout_dirty = true;
  return WAVE_OK;
}

int wave_batch_set_graph(wave_batch* b, int32_t steps_per_graph) {
  CHECK_BATCH(b);
  if (steps_per_graph < 0 || steps_per_graph > 4096) return fail(WAVE_EINVAL, "steps_per_graph outside [0, 4096]");
  b->graph_steps = steps_per_graph;
  batch_drop_graphs(b);
  return WAVE_OK;
}

int wave_batch_run(wave_batch* b, int32_t n) {
  CHECK_BATCH(b);
  if (n < 0) return fail(WAVE_EINVAL, "n < 0");
  for (wave_ctx* c : b->members)
    if (c->broken) return fail(WAVE_ESTATE, "a member context is broken");
  const size_t nm = b->members.size();
  if (nm == 0 || n == 0) return WAVE_OK;
  // members ordered by the steps they take in this run, most first: at every
  // step the members still running are a prefix, and only their workgroups
  // are launched
  {
    std::vector<size_t> order(nm);
    for (size_t i = 0; i < nm; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) {
      return std::min(b->remaining[x], n) > std::min(b->remaining[y], n);
    });
    bool moved = false;
    for (size_t i = 0; i < nm; ++i) moved = moved || order[i] != i;
    if (moved) {
      std::vector<wave_ctx*> m(nm);
      std::vector<int32_t> r(nm);
      for (size_t i = 0; i < nm; ++i) {
        m[i] = b->members[order[i]];
        r[i] = b->remaining[order[i]];
      }
      b->members.swap(m);
      b->remaining.swap(r);
      b->layout_dirty = true;
    }
  }
  if (b->layout_dirty) batch_layout(b);
  // per-run targets and start state
  int32_t steps = 0;
  b->h_state.resize(nm);
  for (size_t i = 0; i < nm; ++i) {
    wave_ctx* c = b->members[i];
    const int32_t t = std::min(b->remaining[i], n);
    b->h_shots[i].target = t;
    b->h_state[i].cur = c->icur < c->iprev ? 0 : 1;
    b->h_state[i].step = (int32_t)c->step;
    b->h_state[i].done = 0;
    b->h_state[i].trace_row = c->trace_count;
    steps = std::max(steps, t);
  }
  if (steps == 0) return WAVE_OK;
  // order after the caller's stream, upload tables, launch
  BCHK(b, hipEventRecord(b->ev_in, b->user_stream), "hipEventRecord");
  BCHK(b, hipStreamWaitEvent(b->stream, b->ev_in, 0), "hipStreamWaitEvent");
  // tables go up from a pinned slot (asynchronous); a slot is rewritten only
  // after the copy that last used it has completed, so runs queue up without
  // waiting for each other
  {
    const int k = (int)(b->runs & 1);
    BCHK(b, hipEventSynchronize(b->ev_copy[k]), "hipEventSynchronize");
    size_t soff = 0;
    (void)batch_table_bytes(b->max_shots, &soff);
    memcpy(b->pinned[k], b->h_shots.data(), nm * sizeof(wave::BatchShot));
    memcpy(b->pinned[k] + soff, b->h_state.data(), nm * sizeof(wave::BatchState));
    BCHK(b, hipMemcpyAsync(b->d_shots, b->pinned[k], nm * sizeof(wave::BatchShot), hipMemcpyHostToDevice, b->stream),
         "hipMemcpyAsync");
    BCHK(b, hipMemcpyAsync(b->d_state, b->pinned[k] + soff, nm * sizeof(wave::BatchState), hipMemcpyHostToDevice,
                           b->stream),
         "hipMemcpyAsync");
    BCHK(b, hipEventRecord(b->ev_copy[k], b->stream), "hipEventRecord");
    b->runs += 1;
  }
  // segments of constant active count k: steps [j, t_{k-1}) run the first k
  // members; whole captured blocks where a segment is long enough
  int32_t j = 0;
  size_t k = nm;
  while (j < steps) {
    while (k > 0 && b->h_shots[k - 1].target <= j) --k;
    const int32_t seg_end = b->h_shots[k - 1].target;
    int32_t left = seg_end - j;
    if (b->graph_steps > 0 && left >= b->graph_steps) {
      hipGraphExec_t g = nullptr;
      hipError_t e = batch_graph(b, (int)k, &g);
      if (e != hipSuccess) return batch_fail(b, e, "batch graph capture");
      for (; left >= b->graph_steps; left -= b->graph_steps)
        BCHK(b, hipGraphLaunch(g, b->stream), "hipGraphLaunch");
    }
    for (; left > 0; --left) {
      hipError_t e = batch_launch_step(b, (int)k);
      if (e != hipSuccess) return batch_fail(b, e, "batch launch");
    }
    j = seg_end;
  }
  BCHK(b, hipEventRecord(b->ev_out, b->stream), "hipEventRecord");
  BCHK(b, hipStreamWaitEvent(b->user_stream, b->ev_out, 0), "hipStreamWaitEvent");
  // host mirrors of each member's state after its `target` steps
  for (size_t i = 0; i < nm; ++i) {
    wave_ctx* c = b->members[i];
    const int32_t t = b->h_shots[i].target;
    if (t & 1) std::swap(c->icur, c->iprev);
    c->step += t;
    if (c->nrec > 0) c->trace_count += t;
    b->remaining[i] -= t;
  }
  return WAVE_OK;
}

int wave_batch_tune(wave_batch* b, int32_t trial_steps, int32_t chosen[2]) {
  CHECK_BATCH(b);
  if (trial_steps < 1) return fail(WAVE_EINVAL, "trial_steps < 1");
  const int nshape = (int)(sizeof(kShapes) / sizeof(kShapes[0]));
  const int ry0 = b->ry, nw0 = b->nw;
  float best = 0.0f;
  int pr = ry0, pn = nw0;
  // the compiled one-point tiles, then two points per lane (128 x 16, 128 x 8)
  // when no member holds an eta array
  std::vector<std::array<int, 2>> shapes;
  bool pair_ok = true;
  for (wave_ctx* c : b->members) pair_ok = pair_ok && !eta_array(&c->d);
  for (int k = 0; k < nshape; ++k)
    if (wave::stream_config_supported(kShapes[k][0], kShapes[k][1], !pair_ok))
      shapes.push_back({kShapes[k][0], kShapes[k][1]});
  if (pair_ok) {
    shapes.push_back({0, 16});
    shapes.push_back({0, 8});
  }
  for (const auto& sh : shapes) {
    b->ry = sh[0];
    b->nw = sh[1];
    b->layout_dirty = true;
    hipEvent_t e0, e1;
    BCHK(b, hipEventCreate(&e0), "hipEventCreate");
    BCHK(b, hipEventCreate(&e1), "hipEventCreate");
    BCHK(b, hipEventRecord(e0, b->user_stream), "hipEventRecord");
    int rc = wave_batch_run(b, trial_steps);
    if (rc != WAVE_OK) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return rc;
    }
    BCHK(b, hipEventRecord(e1, b->user_stream), "hipEventRecord");
    BCHK(b, hipEventSynchronize(e1), "hipEventSynchronize");
    float ms = 0.0f;
    BCHK(b, hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best == 0.0f || ms < best * 0.985f) {   // as in wave_tune
      best = ms;
      pr = sh[0];
      pn = sh[1];
    }
  }
  b->ry = pr;
  b->nw = pn;
  b->layout_dirty = true;
  if (chosen) {
    chosen[0] = pr;
    chosen[1] = pn;
  }
  return WAVE_OK;
}

int wave_batch_free(wave_batch* b) {
  if (!b) return WAVE_OK;
  if (!b->broken) (void)hipStreamSynchronize(b->stream);
  for (wave_ctx* c : b->members) c->batch = nullptr;
  batch_release(b);
  return WAVE_OK;
}

const char* wave_strerror(int s) {
  switch (s) {
    case WAVE_OK: return "ok";
    case WAVE_EINVAL: return "invalid argument";
    case WAVE_ENOMEM: return "arena too small";
    case WAVE_EUNSTABLE: return "time step violates the stability bound";
    case WAVE_EDEVICE: return "device error";
    case WAVE_ESTATE: return "context broken by an earlier device error";
    case WAVE_EBUDGET: return "request can never fit the memory budget";
  }
  return "unknown status";
}

const char* wave_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
