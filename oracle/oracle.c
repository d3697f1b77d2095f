/*
 * oracle.c -- plain, slow, obviously correct CPU implementation of time
 * stepping for the 3-D constant-density acoustic wave equation with the
 * 25-point radius-4 Laplacian, leapfrog in time, a damping (PML) layer,
 * point sources and receivers.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header, table or constant with
 * the HIP library: every number below is derived here from the paper's
 * definitions.
 *
 * What is computed (paper: Sec. III-A, Eq. 1-3 and Alg. 1):
 *   (1/V^2) u_tt - lap(u) = f                                   Eq. 1
 *   u^{n+1} - Q u^n + u^{n-1} = dt^2 V^2 f^n,  Q = 2 + dt^2 V^2 lap  Eq. 2
 *   lap u(i,j,k) = c_xyz u + sum_{m=1..4} c_xm [u(i+m)+u(i-m)]
 *                           + c_ym [...] + c_zm [...]           Eq. 3
 *   Alg. 1: u^0 = 0; each step sweeps every point, then adds the source.
 * The inner region applies Eq. 2; the surrounding layer applies a PML
 * update that reads u with the 25-point stencil and eta with a 7-point
 * star (Sec. III-A, last paragraphs; Sec. IV "3D Blocking Using Shared
 * Memory for Boundary Regions").  The paper does not print the layer
 * equations or the stencil weights; the readings taken here are:
 *   - weights: standard 8th-order central second-difference weights
 *     C = [-205/72, 8/5, -1/5, 8/315, -1/560], c_am = C_m / h_a^2,
 *     c_xyz = C_0 (1/dx^2 + 1/dy^2 + 1/dz^2);
 *   - layer: leapfrog form of u_tt + 2 d u_t + d^2 u = V^2 (lap u + phi),
 *     phi_t + d phi = -grad d . grad u, with eta = dt d (dimensionless):
 *       u^{n+1} = [(2 + 2 eta - eta^2) u^n - u^{n-1} + vp (lap + phi^n)]
 *                 / (1 + 2 eta)
 *       phi^{n+1} = [phi^n - sum_a (eta(p+e_a) - eta(p-e_a))
 *                             (u(p+e_a) - u(p-e_a)) / (4 h_a^2)] / (1 + eta)
 *     which reduces to Eq. 2 exactly when eta = phi = 0;
 *   - vp = (V dt)^2 (Eq. 2), sources add vp(s) w[n] into u^{n+1} after the
 *     sweep (Alg. 1 order, Eq. 2 scaling); receivers read u^{n+1} after the
 *     source add;
 *   - u^{-1} = u^0 = phi^0 = 0; values beyond every face are zero
 *     (4 ghost cells for u, 1 for eta), never updated;
 *   - the grid size includes the layer; the inner box is [w, n-w) per axis.
 *
 * Two precisions: ora_run_f64 is the truth (plain double expressions);
 * ora_run_f32 evaluates the same recurrence in float with a fixed
 * per-point operation order (explicit fmaf where a fused multiply-add is
 * meant, nothing else fused; compile with -ffp-contract=off):
 *   lap = c_xyz * u
 *   for axis x, y, z; for m = 1..4:
 *       lap = fmaf(c_am, u(+m) + u(-m), lap)
 *   lap = fmaf(c_e, u, lap)
 *   (Eq. 3 in its printed order, then a correction for the float weights:
 *   c_e = fl32(-(c_xyz + 2 sum c_am)) over the float weights, see lap32)
 *   inner: u' = u + fmaf(vp, lap, u - u_prev)
 *   layer: t  = fmaf(-(eta * eta), u, u - u_prev)
 *          u' = u + fmaf(vp, lap + phi, t) / fmaf(2, eta, 1)
 *   (the same updates as above, rearranged around the increment u - u_prev:
 *   [(2 + 2 eta - eta^2) u - u_prev + X] / (1 + 2 eta)
 *   = u + [(u - u_prev) - eta^2 u + X] / (1 + 2 eta).  The increment of a
 *   smooth field is computed exactly and every small term is rounded
 *   relative to its own size, so only the final add rounds at the size of u;
 *   with eta = 0 the layer form is the inner form bit for bit)
 *          g  = (de_x * q_x) * (u(+x) - u(-x))
 *          g  = fmaf(de_y * q_y, u(+y) - u(-y), g)
 *          g  = fmaf(de_z * q_z, u(+z) - u(-z), g)
 *          phi' = (phi - g) / (1 + eta),   q_a = fl32(1 / (4 h_a^2))
 *   with de_a = eta(+a) - eta(-a) from an eta array, or, for the default
 *   profile given as axis terms (ora_eta_axis_tables),
 *   de_a = fl32(dt (t_a(i+1) - t_a(i-1))) in double before the rounding
 *   source: u'(s) = fmaf(vp(s), w_s[n], u'(s)), sources in list order
 * With 16-bit storage the float value is rounded to the storage format
 * (round to nearest, ties to even) wherever u is written.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define R 4

/* Eq. 3 weights (standard 8th-order central second difference). */
static const double C8[R + 1] = {
    -205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};

/* c[0] = c_xyz, c[1..4] = c_xm, c[5..8] = c_ym, c[9..12] = c_zm */
void ora_coefficients(double dx, double dy, double dz, double *c)
{
    c[0] = C8[0] * (1.0 / (dx * dx) + 1.0 / (dy * dy) + 1.0 / (dz * dz));
    for (int m = 1; m <= R; ++m) {
        c[m] = C8[m] / (dx * dx);
        c[4 + m] = C8[m] / (dy * dy);
        c[8 + m] = C8[m] / (dz * dz);
    }
}

/* Stability number of the leapfrog scheme for velocity vmax: the scheme is
 * stable when  vmax dt sqrt(sum_a |S| / h_a^2) / 2 <= 1, with S the Eq. 3
 * stencil symbol at the Nyquist wavenumber, S = C_0 + 2 sum_m C_m (-1)^m. */
double ora_stability(double dx, double dy, double dz, double dt, double vmax)
{
    double s = C8[0];
    for (int m = 1; m <= R; ++m)
        s += 2.0 * C8[m] * ((m & 1) ? -1.0 : 1.0);
    s = fabs(s);
    double k = s / (dx * dx) + s / (dy * dy) + s / (dz * dz);
    return vmax * dt * sqrt(k) / 2.0;
}

static inline size_t IDX(int nx, int ny, int i, int j, int k)
{
    return ((size_t)k * (size_t)ny + (size_t)j) * (size_t)nx + (size_t)i;
}

int ora_is_inner(int nx, int ny, int nz, int w, int i, int j, int k)
{
    return i >= w && i < nx - w && j >= w && j < ny - w && k >= w && k < nz - w;
}

/* vp = (V dt)^2 in double; the float copy is the double rounded once. */
void ora_vp(const float *vel, size_t n, double dt, double *vp64, float *vp32)
{
    for (size_t p = 0; p < n; ++p) {
        double v = (double)vel[p] * dt;
        double q = v * v;
        if (vp64) vp64[p] = q;
        if (vp32) vp32[p] = (float)q;
    }
}

/* Default damping profile (the paper defers the PML to another report;
 * this is the quadratic profile d(delta) = d0 (delta/L)^2, L = w h_a,
 * d0 = 3 vmax ln(1/refl) / (2 L)).  delta_a is the distance into the layer
 * along axis a (cells beyond the inner box, times h_a); eta = dt sum_a d_a.
 * Zero in the inner box. */
static double layer_depth(int i, int n, int w)
{
    if (i < w) return (double)(w - i);
    if (i >= n - w) return (double)(i - (n - w - 1));
    return 0.0;
}

void ora_eta_default(int nx, int ny, int nz, int w, double dx, double dy, double dz,
                     double dt, double vmax, double refl, double *eta64, float *eta32)
{
    double h[3] = {dx, dy, dz};
    double d0[3];
    for (int a = 0; a < 3; ++a) {
        double L = (double)w * h[a];
        d0[a] = (w > 0) ? 3.0 * vmax * log(1.0 / refl) / (2.0 * L) : 0.0;
    }
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double s = 0.0;
                double cells[3] = {layer_depth(i, nx, w), layer_depth(j, ny, w),
                                   layer_depth(k, nz, w)};
                for (int a = 0; a < 3; ++a) {
                    if (cells[a] > 0.0) {
                        double r = cells[a] / (double)w;    /* delta / L */
                        s += d0[a] * r * r;
                    }
                }
                double e = dt * s;
                size_t p = IDX(nx, ny, i, j, k);
                if (eta64) eta64[p] = e;
                if (eta32) eta32[p] = (float)e;
            }
}

/* Per-axis terms of the same profile, t_a(i) = d0_a (depth_a(i) / w)^2, for
 * i = -1..n_a, stored at index i + 1, so that eta = dt ((t_x + t_y) + t_z)
 * (the sum above, in the same order).  The depth formula continues one cell
 * beyond each face of the grid (depth w + 1 there): the profile extended by
 * its own formula.  In table mode the layer's eta gradient is taken from
 * these terms: the profile is a sum of one-axis functions, so its central
 * difference along axis a is dt (t_a(i+1) - t_a(i-1)), free of the other
 * axes' terms. */
void ora_eta_axis_tables(int nx, int ny, int nz, int w, double dx, double dy, double dz,
                         double vmax, double refl, double *tx, double *ty, double *tz)
{
    const int n[3] = {nx, ny, nz};
    const double h[3] = {dx, dy, dz};
    double *t[3] = {tx, ty, tz};
    for (int a = 0; a < 3; ++a) {
        double d0 = (w > 0) ? 3.0 * vmax * log(1.0 / refl) / (2.0 * ((double)w * h[a])) : 0.0;
        for (int i = -1; i <= n[a]; ++i) {
            double cells = layer_depth(i, n[a], w);
            double v = 0.0;
            if (cells > 0.0) {
                double r = cells / (double)w;
                v = d0 * r * r;
            }
            t[a][i + 1] = v;
        }
    }
}

/* ---- rounding to 16-bit storage formats, from the IEEE definition ------
 * round-to-nearest-even at the format's precision, done in double where
 * every step below is exact: a float is exact in double, scaling by a power
 * of two is exact, and nearbyint rounds ties to even in the default mode.
 * mant = significand bits incl. the hidden one, emin = min normal exponent,
 * maxv = largest finite value. */
static double round_fmt(double x, int mant, int emin, double maxv)
{
    if (x == 0.0 || isnan(x) || isinf(x)) return x;
    int e;
    frexp(fabs(x), &e);           /* |x| = f 2^e, f in [0.5, 1) -> exponent e-1 */
    int ex = e - 1;
    if (ex < emin) ex = emin;     /* subnormal range: fixed quantum */
    double quantum = ldexp(1.0, ex - (mant - 1));
    double r = nearbyint(x / quantum) * quantum;
    /* overflow: values at or beyond maxv + half an ulp round to infinity */
    double ulp_top = ldexp(1.0, (int)floor(log2(maxv)) - (mant - 1));
    if (fabs(r) > maxv || fabs(x) >= maxv + 0.5 * ulp_top) return copysign(INFINITY, x);
    return r;
}

float ora_round_bf16(float x)
{   /* bfloat16: 8 significand bits, emin -126, max (2 - 2^-7) 2^127 */
    return (float)round_fmt((double)x, 8, -126, ldexp(2.0 - ldexp(1.0, -7), 127));
}

float ora_round_f16(float x)
{   /* binary16: 11 significand bits, emin -14, max 65504 */
    return (float)round_fmt((double)x, 11, -14, 65504.0);
}

/* ---- stochastic rounding to bfloat16 (the library's WAVE_STOCH_ROUND) ---
 * The "pcg" hash of Jarzynski and Olano ("Hash functions for GPU
 * rendering", JCGT 2020): one step of the PCG linear congruential generator
 * (multiplier 747796405, increment 2891336453) followed by PCG's RXS-M-XS
 * output permutation (O'Neill 2014: a random shift of 4..19 chosen by the top
 * four bits, multiply by 277803737, xor-shift by 22). */
uint32_t ora_pcg_hash(uint32_t v)
{
    uint32_t state = v * 747796405u + 2891336453u;
    uint32_t shift = (state >> 28) + 4u;
    uint32_t word = ((state >> shift) ^ state) * 277803737u;
    return (word >> 22) ^ word;
}

/* The 16 random bits of point (i, j, k) at step n: the pair index
 * q = (k ny + j) ceil(nx / 2) + floor(i / 2), taken modulo 2^32, gives the
 * word pcg(q xor pcg(n)); point i takes its 16-bit half number i mod 2. */
unsigned ora_sr_bits(int n, int nx, int ny, int nz, int i, int j, int k)
{
    (void)nz;
    uint32_t half_row = (uint32_t)(nx + 1) / 2;
    uint32_t q = ((uint32_t)k * (uint32_t)ny + (uint32_t)j) * half_row + (uint32_t)(i / 2);
    uint32_t word = ora_pcg_hash(q ^ ora_pcg_hash((uint32_t)n));
    return (word >> (16 * (i % 2))) & 0xFFFFu;
}

/* Stochastic rounding of a float to bfloat16 with 16 uniform random bits r:
 * the two bfloat16 neighbours of a finite x are its truncation toward zero
 * (its top 16 bits) and the next value away from zero; the farther one is
 * taken with probability equal to the dropped fraction f / 2^16 of an ulp,
 * i.e. exactly when f + r >= 2^16.  Infinities and NaN round to nearest. */
float ora_round_bf16_sr(float x, unsigned r)
{
    if (!isfinite(x)) return ora_round_bf16(x);
    uint32_t bits;
    memcpy(&bits, &x, 4);
    uint32_t f = bits & 0xFFFFu;
    uint32_t t = bits - f;                               /* truncation toward zero */
    uint32_t out = (f + (r & 0xFFFFu) >= 0x10000u) ? t + 0x10000u : t;
    float y;
    memcpy(&y, &out, 4);
    return y;
}

/* storage: 0 float, 1 bfloat16, 2 binary16 (round to nearest even); 3
 * bfloat16 written by the sweep with stochastic rounding, whose source add
 * rounds to nearest like 1. */
static inline float store16(float x, int storage)
{
    if (storage == 1 || storage == 3) return ora_round_bf16(x);
    if (storage == 2) return ora_round_f16(x);
    return x;
}

/* store16 over an array in place (storage 1 bf16, 2 binary16): the rounding
 * of an initial state to the storage type, one element at a time. */
void ora_round_array(float *a, long long n, int storage)
{
    #pragma omp parallel for schedule(static)
    for (long long i = 0; i < n; ++i) a[i] = store16(a[i], storage);
}

/* ---- the recurrence ----------------------------------------------------- */

typedef struct {
    int nx, ny, nz, w;
} grid_t;

static inline double U64(const double *u, grid_t g, int i, int j, int k)
{
    if (i < 0 || i >= g.nx || j < 0 || j >= g.ny || k < 0 || k >= g.nz) return 0.0;
    return u[IDX(g.nx, g.ny, i, j, k)];
}

static inline float U32(const float *u, grid_t g, int i, int j, int k)
{
    if (i < 0 || i >= g.nx || j < 0 || j >= g.ny || k < 0 || k >= g.nz) return 0.0f;
    return u[IDX(g.nx, g.ny, i, j, k)];
}

/* Eq. 3 in double. */
static double lap64(const double *u, grid_t g, const double *c, int i, int j, int k)
{
    double s = c[0] * U64(u, g, i, j, k);
    for (int m = 1; m <= R; ++m)
        s += c[m] * (U64(u, g, i + m, j, k) + U64(u, g, i - m, j, k));
    for (int m = 1; m <= R; ++m)
        s += c[4 + m] * (U64(u, g, i, j + m, k) + U64(u, g, i, j - m, k));
    for (int m = 1; m <= R; ++m)
        s += c[8 + m] * (U64(u, g, i, j, k + m) + U64(u, g, i, j, k - m));
    return s;
}

/* Eq. 3 in float, in the printed order (centre term, then the x, y and z
 * pairs for m = 1..4), plus one correction term.  In exact arithmetic
 * c_xyz = -2 sum_a sum_m c_am, so a constant field has a zero Laplacian;
 * the 13 weights rounded to float separately miss that identity by a
 * residual e = c_xyz + 2 sum c_am (of the float weights), which would act as
 * a spurious term e u, a frequency shift whose phase error grows with time.
 * The last operation removes it with c_e = fl32(-e) (e is exact in double:
 * 13 floats of nearby magnitude). */
static float lap32(const float *u, grid_t g, const float *c, float ce, int i, int j, int k)
{
    const float uc = U32(u, g, i, j, k);
    float s = c[0] * uc;
    for (int m = 1; m <= R; ++m)
        s = fmaf(c[m], U32(u, g, i + m, j, k) + U32(u, g, i - m, j, k), s);
    for (int m = 1; m <= R; ++m)
        s = fmaf(c[4 + m], U32(u, g, i, j + m, k) + U32(u, g, i, j - m, k), s);
    for (int m = 1; m <= R; ++m)
        s = fmaf(c[8 + m], U32(u, g, i, j, k + m) + U32(u, g, i, j, k - m), s);
    return fmaf(ce, uc, s);
}

/* The correction weight c_e of lap32 for the float weights c[0..12]. */
static float weight_residual32(const float *c)
{
    double e = (double)c[0];
    for (int m = 1; m < 13; ++m) e += 2.0 * (double)c[m];
    return (float)(-e);
}

/*
 * ora_run_f64: advance `steps` time steps from the state (u_cur = u^n,
 * u_prev = u^{n-1}, phi = phi^n) starting at step index n0; on return the
 * three arrays hold the state after the last step.  Arrays are [nz][ny][nx]
 * with x fastest.  Sources: src_ijk[nsrc][3], wavelets[nsrc][nsamp] (w[n],
 * zero beyond nsamp).  Receivers: rec_ijk[nrec][3]; traces[steps][nrec]
 * (may be NULL).  eta NULL means no damping: Eq. 2 everywhere.  Returns 0,
 * or -1 on bad arguments / allocation failure.
 */
int ora_run_f64(int nx, int ny, int nz, int w, double dx, double dy, double dz,
                const double *vp, const double *eta, const double *etab, double eta_dt,
                int nsrc, const int32_t *src_ijk, const float *wavelets, int nsamp,
                int nrec, const int32_t *rec_ijk, double *traces,
                int n0, int steps, double *u_cur, double *u_prev, double *phi)
{
    if (nx <= 0 || ny <= 0 || nz <= 0 || w < 0 || steps < 0) return -1;
    grid_t g = {nx, ny, nz, w};
    size_t n = (size_t)nx * ny * nz;
    double c[13];
    ora_coefficients(dx, dy, dz, c);
    double h2[3] = {dx * dx, dy * dy, dz * dz};
    double *u_next = (double *)calloc(n, sizeof(double));
    double *phi_next = (double *)calloc(n, sizeof(double));
    if (!u_next || !phi_next) { free(u_next); free(phi_next); return -1; }

    for (int t = 0; t < steps; ++t) {
        const int step = n0 + t;
        /* Alg. 1: sweep every point of the wavefield */
#pragma omp parallel for schedule(static)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    size_t p = IDX(nx, ny, i, j, k);
                    double L = lap64(u_cur, g, c, i, j, k);
                    if (eta == NULL || ora_is_inner(nx, ny, nz, w, i, j, k)) {
                        /* inner region: Eq. 2 solved for u^{n+1} */
                        u_next[p] = 2.0 * u_cur[p] - u_prev[p] + vp[p] * L;
                        phi_next[p] = phi[p];
                    } else {
                        /* damping layer: two-statement update */
                        double e = eta[p];
                        u_next[p] = ((2.0 + 2.0 * e - e * e) * u_cur[p] - u_prev[p]
                                     + vp[p] * (L + phi[p])) / (1.0 + 2.0 * e);
                        /* central differences of eta: of the array (zero
                         * beyond the faces), or of the profile's axis terms */
                        double dex, dey, dez;
                        if (etab) {
                            const double *tx = etab, *ty = tx + nx + 2, *tz = ty + ny + 2;
                            dex = eta_dt * (tx[i + 2] - tx[i]);
                            dey = eta_dt * (ty[j + 2] - ty[j]);
                            dez = eta_dt * (tz[k + 2] - tz[k]);
                        } else {
                            dex = U64(eta, g, i + 1, j, k) - U64(eta, g, i - 1, j, k);
                            dey = U64(eta, g, i, j + 1, k) - U64(eta, g, i, j - 1, k);
                            dez = U64(eta, g, i, j, k + 1) - U64(eta, g, i, j, k - 1);
                        }
                        double gsum = 0.0;
                        gsum += dex * (U64(u_cur, g, i + 1, j, k) - U64(u_cur, g, i - 1, j, k))
                              / (4.0 * h2[0]);
                        gsum += dey * (U64(u_cur, g, i, j + 1, k) - U64(u_cur, g, i, j - 1, k))
                              / (4.0 * h2[1]);
                        gsum += dez * (U64(u_cur, g, i, j, k + 1) - U64(u_cur, g, i, j, k - 1))
                              / (4.0 * h2[2]);
                        phi_next[p] = (phi[p] - gsum) / (1.0 + e);
                    }
                }
        /* Alg. 1: add the source after the sweep, scaled per Eq. 2 */
        for (int s = 0; s < nsrc; ++s) {
            double wv = (step < nsamp) ? (double)wavelets[(size_t)s * nsamp + step] : 0.0;
            size_t p = IDX(nx, ny, src_ijk[3 * s], src_ijk[3 * s + 1], src_ijk[3 * s + 2]);
            u_next[p] += vp[p] * wv;
        }
        if (traces)
            for (int r = 0; r < nrec; ++r)
                traces[(size_t)t * nrec + r] =
                    u_next[IDX(nx, ny, rec_ijk[3 * r], rec_ijk[3 * r + 1], rec_ijk[3 * r + 2])];
        /* rotate time levels: (u^{n-1}, u^n, phi^n) <- (u^n, u^{n+1}, phi^{n+1}) */
        memcpy(u_prev, u_cur, n * sizeof(double));
        memcpy(u_cur, u_next, n * sizeof(double));
        memcpy(phi, phi_next, n * sizeof(double));
    }
    free(u_next);
    free(phi_next);
    return 0;
}

/* Same recurrence in float with the fixed operation order given at the top
 * of this file.  vp and eta are the float copies (rounded once from double).
 * storage: 0 = float, 1 = bfloat16, 2 = binary16 for u (values are kept in
 * float arrays but every written u is rounded to the storage format); 3 =
 * bfloat16 with the sweep's u^{n+1} rounded stochastically (see above). */
int ora_run_f32(int nx, int ny, int nz, int w, double dx, double dy, double dz,
                const float *vp, const float *eta, const double *etab, double eta_dt,
                int storage,
                int nsrc, const int32_t *src_ijk, const float *wavelets, int nsamp,
                int nrec, const int32_t *rec_ijk, double *traces,
                int n0, int steps, float *u_cur, float *u_prev, float *phi)
{
    if (nx <= 0 || ny <= 0 || nz <= 0 || w < 0 || steps < 0) return -1;
    if (storage < 0 || storage > 3) return -1;
    grid_t g = {nx, ny, nz, w};
    size_t n = (size_t)nx * ny * nz;
    double c64[13];
    ora_coefficients(dx, dy, dz, c64);
    float c[13];
    for (int m = 0; m < 13; ++m) c[m] = (float)c64[m];
    const float ce = weight_residual32(c);
    float q[3] = {(float)(1.0 / (4.0 * dx * dx)), (float)(1.0 / (4.0 * dy * dy)),
                  (float)(1.0 / (4.0 * dz * dz))};
    float *u_next = (float *)calloc(n, sizeof(float));
    float *phi_next = (float *)calloc(n, sizeof(float));
    if (!u_next || !phi_next) { free(u_next); free(phi_next); return -1; }

    for (int t = 0; t < steps; ++t) {
        const int step = n0 + t;
#pragma omp parallel for schedule(static)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    size_t p = IDX(nx, ny, i, j, k);
                    float L = lap32(u_cur, g, c, ce, i, j, k);
                    float un;
                    if (eta == NULL || ora_is_inner(nx, ny, nz, w, i, j, k)) {
                        un = u_cur[p] + fmaf(vp[p], L, u_cur[p] - u_prev[p]);
                        phi_next[p] = phi[p];
                    } else {
                        float e = eta[p];
                        float t = fmaf(-(e * e), u_cur[p], u_cur[p] - u_prev[p]);
                        float num = fmaf(vp[p], L + phi[p], t);
                        un = u_cur[p] + num / fmaf(2.0f, e, 1.0f);
                        float dex, dey, dez;
                        if (etab) {
                            const double *tx = etab, *ty = tx + nx + 2, *tz = ty + ny + 2;
                            dex = (float)(eta_dt * (tx[i + 2] - tx[i]));
                            dey = (float)(eta_dt * (ty[j + 2] - ty[j]));
                            dez = (float)(eta_dt * (tz[k + 2] - tz[k]));
                        } else {
                            dex = U32(eta, g, i + 1, j, k) - U32(eta, g, i - 1, j, k);
                            dey = U32(eta, g, i, j + 1, k) - U32(eta, g, i, j - 1, k);
                            dez = U32(eta, g, i, j, k + 1) - U32(eta, g, i, j, k - 1);
                        }
                        float gs = (dex * q[0])
                                 * (U32(u_cur, g, i + 1, j, k) - U32(u_cur, g, i - 1, j, k));
                        gs = fmaf(dey * q[1],
                                  U32(u_cur, g, i, j + 1, k) - U32(u_cur, g, i, j - 1, k), gs);
                        gs = fmaf(dez * q[2],
                                  U32(u_cur, g, i, j, k + 1) - U32(u_cur, g, i, j, k - 1), gs);
                        phi_next[p] = (phi[p] - gs) / (1.0f + e);
                    }
                    u_next[p] = storage == 3
                                    ? ora_round_bf16_sr(un, ora_sr_bits(step, nx, ny, nz, i, j, k))
                                    : store16(un, storage);
                }
        for (int s = 0; s < nsrc; ++s) {
            float wv = (step < nsamp) ? wavelets[(size_t)s * nsamp + step] : 0.0f;
            size_t p = IDX(nx, ny, src_ijk[3 * s], src_ijk[3 * s + 1], src_ijk[3 * s + 2]);
            u_next[p] = store16(fmaf(vp[p], wv, u_next[p]), storage);
        }
        if (traces)
            for (int r = 0; r < nrec; ++r)
                traces[(size_t)t * nrec + r] = (double)
                    u_next[IDX(nx, ny, rec_ijk[3 * r], rec_ijk[3 * r + 1], rec_ijk[3 * r + 2])];
        memcpy(u_prev, u_cur, n * sizeof(float));
        memcpy(u_cur, u_next, n * sizeof(float));
        memcpy(phi, phi_next, n * sizeof(float));
    }
    free(u_next);
    free(phi_next);
    return 0;
}

/* Discrete energy of the leapfrog scheme with damping off:
 *   E^{n+1/2} = sum_p (u^{n+1}_p - u^n_p)^2 / vp_p - sum_p u^{n+1}_p (lap u^n)_p
 * (lap is Eq. 3 with zero values beyond the faces, a symmetric operator,
 * so E is exactly conserved by Eq. 2 in exact arithmetic). */
double ora_energy(int nx, int ny, int nz, double dx, double dy, double dz,
                  const double *vp, const double *u_next, const double *u_now)
{
    grid_t g = {nx, ny, nz, 0};
    double c[13];
    ora_coefficients(dx, dy, dz, c);
    double kin = 0.0, pot = 0.0;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t p = IDX(nx, ny, i, j, k);
                double d = u_next[p] - u_now[p];
                kin += d * d / vp[p];
                pot += u_next[p] * lap64(u_now, g, c, i, j, k);
            }
    return kin - pot;
}

/* The paper's third decomposition (Sec. III-B): the inner region plus six
 * layer sub-regions.  Writes 7 boxes as (x0, y0, z0, ex, ey, ez) into out[42]
 * in the order inner, T, B, F, Bk, L, R.  order 0 is the 3-D cut (z caps of
 * full xy extent first, then y walls over the inner z range, then x walls over
 * the inner y and z ranges); order 1 is the cut used with streaming along z
 * (x walls over full y and z first, then y walls over the inner x range and
 * full z, then z caps over the inner x and y ranges). */
void ora_regions(int nx, int ny, int nz, int w, int order, int *out)
{
    int ix = nx - 2 * w, iy = ny - 2 * w, iz = nz - 2 * w;
    int b[7][6];
    int r = 0;
#define BOX(a, bb, cc, d, e, f) do { b[r][0]=a; b[r][1]=bb; b[r][2]=cc; b[r][3]=d; b[r][4]=e; b[r][5]=f; ++r; } while (0)
    BOX(w, w, w, ix, iy, iz);
    if (order == 0) {
        BOX(0, 0, 0, nx, ny, w);          BOX(0, 0, nz - w, nx, ny, w);
        BOX(0, 0, w, nx, w, iz);          BOX(0, ny - w, w, nx, w, iz);
        BOX(0, w, w, w, iy, iz);          BOX(nx - w, w, w, w, iy, iz);
    } else {
        BOX(0, 0, 0, w, ny, nz);          BOX(nx - w, 0, 0, w, ny, nz);
        BOX(w, 0, 0, ix, w, nz);          BOX(w, ny - w, 0, ix, w, nz);
        BOX(w, w, 0, ix, iy, w);          BOX(w, w, nz - w, ix, iy, w);
    }
#undef BOX
    memcpy(out, b, sizeof(b));
}
