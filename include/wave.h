/*
 * wave.h -- C ABI of the MI355X (gfx950) acoustic wave-propagation library.
 *
 * The library time-steps the 3-D constant-density acoustic wave equation
 * (paper Sec. III-A, Eq. 1) discretised with the 25-point radius-4
 * 8th-order Laplacian (Eq. 3) and second-order leapfrog in time (Eq. 2),
 * with a damping (PML) layer around the inner region (Sec. III-A, last
 * paragraphs; Sec. III-B), point sources added after each sweep (Alg. 1)
 * and receivers sampled after the source add.
 *
 * Conventions for every entry point
 *  - Return value: 0 (WAVE_OK) or a negative wave_status.  No exception or
 *    C++ type crosses this interface.  wave_last_error() gives a message for
 *    the last failure on the calling thread.
 *  - A HIP runtime failure inside a call returns WAVE_EDEVICE and marks the
 *    context broken; every later call on it returns WAVE_ESTATE, except
 *    wave_free.
 *  - Arrays passed as host pointers are read or written during the call and
 *    not retained.  Host arrays are [nz][ny][nx] with x fastest (Sec. IV,
 *    one flat array with x innermost) unless stated otherwise.
 *  - Grid indices (i, j, k) are (x, y, z), 0-based, and count the damping
 *    layer: the total extent includes it, and the inner region is
 *    [w, n - w) on every axis (Table III is reproduced by a 1000^3 total grid
 *    with a 27-cell layer).
 *  - Device memory is a caller-owned arena (one device allocation of at
 *    least wave_bytes_required() bytes, e.g. a torch uint8 tensor).  The
 *    library carves every device array from it, never frees it, and the
 *    arena must outlive the context.  The context object itself is a small
 *    host allocation owned by the library until wave_free.
 *  - Work is enqueued on the HIP stream given to wave_alloc; calls that
 *    return data to the host synchronise that stream first.
 *  - One context must not be used from two threads at once.
 */
#ifndef WAVE_H
#define WAVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum wave_status {
    WAVE_OK = 0,
    WAVE_EINVAL = -1,    /* bad argument: sizes, indices, pointers, counts */
    WAVE_ENOMEM = -2,    /* arena smaller than wave_bytes_required() */
    WAVE_EUNSTABLE = -3, /* time step violates the stability bound */
    WAVE_EDEVICE = -4,   /* a HIP call failed (context is now broken) */
    WAVE_ESTATE = -5,    /* context broken by an earlier device failure */
    WAVE_EBUDGET = -6    /* request can never fit the memory budget */
} wave_status;

/* Storage type of the wavefield u (arithmetic is always float32). */
typedef enum wave_storage { WAVE_F32 = 0, WAVE_BF16 = 1, WAVE_F16 = 2 } wave_storage;

/* wave_desc.flags */
#define WAVE_DAMPING_OFF 1 /* eta := 0: Eq. 2 on every point */
#define WAVE_ETA_ARRAY 2   /* eta is supplied per point at wave_alloc (else the
                              default profile, kept as three 1-D tables) */
#define WAVE_TWO_STEP 4    /* reserve two more u arrays (and a second phi) so
                              that wave_step can take two time steps per
                              launch (WAVE_KERNEL_STREAM2); not with an eta
                              array */
#define WAVE_STOCH_ROUND 8 /* bf16 storage only: every u^{n+1} the sweep writes
                              is rounded stochastically instead of to nearest
                              even: its float32 value is truncated to bf16 and
                              rounded up in magnitude with probability equal
                              to the dropped fraction of the bf16 ulp.  The
                              16 random bits of point (i, j, k) at step n are
                              half number i mod 2 of pcg(q xor pcg(n)), pcg
                              being the 32-bit hash of Jarzynski and Olano
                              (JCGT 2020: a PCG step and its RXS-M-XS output
                              permutation) and q = (k ny + j) ceil(nx / 2) +
                              floor(i / 2) modulo 2^32.  So results are
                              reproducible and do not depend on the launch
                              shape.  The source add stays
                              round-to-nearest.  Not with WAVE_TWO_STEP; the
                              3-D code shapes (GMEM, RING, SHIFT) refuse such
                              contexts */

typedef struct wave_desc {
    int32_t nx, ny, nz;  /* total extents incl. the layer, 1..32768, and
                            one padded xy plane below 2 GiB               */
    int32_t w;           /* layer width per face, 0 <= 2w <= min(nx,ny,nz) */
    double dx, dy, dz;   /* grid spacing (m), > 0                          */
    double dt;           /* time step (s), > 0                             */
    int32_t storage;     /* wave_storage of u                              */
    int32_t flags;       /* WAVE_DAMPING_OFF | WAVE_ETA_ARRAY | WAVE_TWO_STEP |
                            WAVE_STOCH_ROUND */
    double refl;         /* target reflection of the default eta profile,
                            0 < refl < 1 (1e-3 is typical)                 */
    int32_t max_src;     /* source table capacity, >= 0                    */
    int32_t max_rec;     /* receiver table capacity, >= 0                  */
    int32_t max_steps;   /* wavelet length and trace capacity (steps) >= 0 */
    int32_t reserved;    /* must be 0                                      */
} wave_desc;

typedef struct wave_ctx wave_ctx;

/* ---- host-only calls (no device work; usable without a GPU) ------------ */

/* Bytes of device arena that wave_alloc needs for `d` (fields u^n, u^{n-1},
 * vp, eta, phi in the padded device layout, plus source, receiver, trace
 * and reduction tables).  Returns 0 if `d` is invalid. */
size_t wave_bytes_required(const wave_desc *d);

/* Admission of a request under a device-memory budget (serving; not in
 * the paper).  *need_out = wave_bytes_required(d); *fits_now = 1 when that
 * many bytes fit beside in_use_bytes (need + in_use <= budget_bytes), else
 * 0.  Returns OK when the request fits the budget now or once enough of
 * in_use_bytes is released, EBUDGET when it needs more than the whole
 * budget (it can never be admitted), EINVAL for an invalid descriptor.
 * Either pointer may be NULL. */
int wave_admit(const wave_desc *d, size_t budget_bytes, size_t in_use_bytes, size_t *need_out,
               int32_t *fits_now);

/* The 13 float32 stencil weights of Eq. 3 used by the kernels:
 * out[0] = c_xyz, out[1..4] = c_x1..4, out[5..8] = c_y1..4,
 * out[9..12] = c_z1..4.  Weights are the standard 8th-order central
 * second-difference weights C_m / h^2 (the paper calls them discretisation
 * parameters without values); c_xyz = C_0 (1/dx^2 + 1/dy^2 + 1/dz^2). */
int wave_coefficients(const wave_desc *d, float out[13]);

/* Stability number of the scheme for peak velocity vmax (m/s): the
 * leapfrog scheme with Eq. 3 is stable when this is <= 1.  Returns a
 * negative value for an invalid descriptor. */
double wave_stability(const wave_desc *d, double vmax);

/* The default damping profile used when wave_alloc gets no eta: quadratic
 * in the depth into the layer on each axis, summed over axes, scaled by dt
 * (eta = dt * d, dimensionless), zero in the inner region.  out is a host
 * float array [nz][ny][nx]. */
int wave_eta_default(const wave_desc *d, double vmax, float *out);

/* ---- context lifetime -------------------------------------------------- */

/* Create a simulation context (Alg. 1 initial state u^0 = u^{-1} = 0,
 * phi = 0, step counter n = 0).
 *   vel_host   velocity V (m/s), float [nz][ny][nx], finite and > 0.
 *              vp = (V dt)^2 (the dt^2 V^2 factor of Eq. 2) is computed
 *              from it in double and rounded once to float.
 *   eta_host   with WAVE_ETA_ARRAY: damping eta >= 0 per point, float
 *              [nz][ny][nx] (stored as a device array).  Without the flag:
 *              NULL, and the default profile (wave_eta_default with vmax =
 *              max V) is used; being a sum of three per-axis profiles it is
 *              kept as 1-D tables and evaluated in the kernels with the same
 *              float64 operations as on the host (same float result), so no
 *              eta array is stored or read.  Its differences in the layer
 *              update are those of the per-axis terms, which continue the
 *              profile one cell past each face (an eta array instead has
 *              zeros beyond the faces).  Ignored (must be NULL) with
 *              WAVE_DAMPING_OFF.
 *   dev_arena  device pointer, 256-byte aligned, arena_bytes long.
 *   hip_stream hipStream_t (NULL = the null stream).  Set-up is enqueued
 *              there (one host-to-device copy per input array, kernels form
 *              vp and the padded layout) and waited for once before return.
 * Errors: EINVAL (descriptor, pointers, alignment, non-finite input, eta
 * given without WAVE_ETA_ARRAY or missing with it), ENOMEM (arena too
 * small), EUNSTABLE (wave_stability > 1, or, with damping on, a largest
 * eta at or above 2 + sqrt(8 - 4 s^2), s = wave_stability: there the damped
 * layer update of one point, (1 + 2 eta) u' = (2 + 2 eta - eta^2 - vp K) u
 * - u_prev for a mode with Laplacian symbol -K, has a growth factor below -1;
 * the default profile reaches it with 1- or 2-cell layers at Courant
 * number 0.4), EDEVICE.  The inputs are checked before the arena, so a
 * NULL arena validates a descriptor and its arrays without device work
 * (EINVAL naming the arena when they are valid). */
int wave_alloc(const wave_desc *d, const float *vel_host, const float *eta_host,
               void *dev_arena, size_t arena_bytes, void *hip_stream, wave_ctx **out);

/* Release the context (host memory only; the arena stays the caller's).
 * Synchronises the stream first.  NULL is accepted. */
int wave_free(wave_ctx *ctx);

/* ---- sources and receivers ---------------------------------------------- */

/* Add a point source at (i, j, k) with wavelet samples w[n], n = 0 ..
 * nsamples-1 (zero afterwards).  After the sweep of step n the library adds
 * vp(s) * w[n] into u^{n+1}(s) (Alg. 1 source add, scaled per Eq. 2).
 * Several sources at one cell are added in the order they were given.
 * Errors: EINVAL (index outside the grid, nsamples > max_steps, table
 * full, the context is a batch member: a batch copies its members' source
 * tables when they join). */
int wave_inject(wave_ctx *ctx, int32_t i, int32_t j, int32_t k,
                const float *samples_host, int32_t nsamples);

/* Set the receiver list (replacing any earlier one) and clear the traces.
 * After each step n the library records u^{n+1}(rec_r) (after the source
 * add) as float64 into traces[t][r], t counting steps since this call.
 * ijk_host is int32 [nrec][3] = (i, j, k).  Errors: EINVAL (index outside
 * the grid, nrec > max_rec, the context is a batch member). */
int wave_record(wave_ctx *ctx, const int32_t *ijk_host, int32_t nrec);

/* ---- time stepping ------------------------------------------------------ */

/* Enqueue n time steps (Alg. 1 loop body n times) on the context stream and
 * return without waiting.  Each step: one sweep over every grid point
 * (Eq. 2 in the inner region, the layer update elsewhere), then the source
 * add, then the receiver sample, then the time levels rotate.
 * Errors: EINVAL (n < 0, or receivers set and the trace buffer would
 * overflow max_steps). */
int wave_step(wave_ctx *ctx, int32_t n);

/* Wait for all enqueued work of the context. */
int wave_sync(wave_ctx *ctx);

/* Number of steps taken so far (the time level n of u^n). */
int64_t wave_step_count(const wave_ctx *ctx);

/* ---- state access --------------------------------------------------------- */

/* Field ids for wave_read_field / wave_write_field */
#define WAVE_FIELD_U 0      /* u^n (current)                     */
#define WAVE_FIELD_UPREV 1  /* u^{n-1}                           */
#define WAVE_FIELD_PHI 2    /* phi^n (layer auxiliary field)     */
#define WAVE_FIELD_VP 3     /* vp = (V dt)^2 (read only)         */
#define WAVE_FIELD_ETA 4    /* eta (read only)                   */

/* Copy a field to a host float array [nz][ny][nx] (16-bit storage is
 * widened exactly).  Synchronises.  The copy goes through a pinned host
 * buffer of at most 64 MB (or one padded plane, if larger), allocated and
 * freed by the call.  Errors: EINVAL; EDEVICE when a copy fails (sticky,
 * as for every device error) or no pinned memory is left for the buffer
 * (not sticky). */
int wave_read_field(wave_ctx *ctx, int32_t which, float *host_out);

/* Overwrite u^n, u^{n-1} or phi^n from a host float array [nz][ny][nx]
 * (rounded to nearest-even into 16-bit storage).  For restarts and tests.
 * Synchronises; the copy goes through a pinned buffer as in
 * wave_read_field.  Errors: EINVAL (read-only field, non-finite values),
 * EDEVICE as for wave_read_field. */
int wave_write_field(wave_ctx *ctx, int32_t which, const float *host_in);

/* Copy the traces recorded since wave_record: float64 [steps][nrec].
 * *steps_out receives the number of recorded steps (host_out may be NULL to
 * query it).  Synchronises. */
int wave_read_traces(wave_ctx *ctx, double *host_out, int32_t *steps_out);

/* Discrete energy of the current state in float64 on the device:
 *   E = sum_p (u^n_p - u^{n-1}_p)^2 / vp_p - sum_p u^n_p (lap u^{n-1})_p
 * with lap = Eq. 3 evaluated in float64.  With damping off and no source
 * it is conserved by Eq. 2 up to the rounding of the stored fields; it is a
 * check quantity, not part of the time step.  Deterministic (fixed
 * reduction order).  Synchronises. */
int wave_energy(wave_ctx *ctx, double *out);

/* wave_energy for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * kernels and reduction order, but the per-row partial sums go to a static
 * workspace of the library (one per GPU, 16 MiB, held until the process
 * ends) instead of the context's arena, nothing is allocated, and nothing
 * waits: the kernels are enqueued on the context stream and write
 * {kinetic, potential} to dev_out (device memory, 2 doubles), so that
 * E = dev_out[0] - dev_out[1] equals wave_energy's value once the stream
 * reaches that point.  Limit: ny * nz <= 1048576 rows (EINVAL beyond).
 * Every call on one GPU shares that GPU's workspace: calls that can overlap
 * on one GPU (contexts on different streams) race and must be ordered by
 * the caller.  Errors: EINVAL (NULL dev_out, too many rows). */
int wave_energy_noalloc(wave_ctx *ctx, double *dev_out);

/* ---- kernel selection and timing ----------------------------------------- */

/* Kernel variants for the sweep. */
#define WAVE_KERNEL_DIRECT 0 /* one thread per point, all reads from memory */
#define WAVE_KERNEL_STREAM 1 /* xy tile in LDS, z neighbours in registers,
                                streamed along z (default)               */
#define WAVE_KERNEL_STREAM2 2 /* two time steps per launch: the second
                                trails the first by 4 planes along z, the
                                first step's results stay on chip (needs
                                WAVE_TWO_STEP); an odd remaining step runs
                                the single-step kernel, and so do all
                                steps while some 56 x 24 output tile's
                                region (plus 4 cells) holds more than 32
                                sources                                 */

/* The paper's other code shapes (Sec. IV), for comparison and tuning; each
 * evaluates every point with the same operations as the others. */
#define WAVE_KERNEL_GMEM 3   /* 3-D tile, one thread per point, every stencil
                                operand read from memory; the block extents
                                (bx, by, bz) are passed as (rows_per_wave,
                                waves_per_group, zchunk): (8,8,8), (4,4,4),
                                (16,16,4), (32,32,1), (64,4,1), (64,4,4)  */
#define WAVE_KERNEL_RING 4   /* 2.5-D: 64 x ty tile streamed along z through
                                a ring of 9 staged planes in LDS (all
                                neighbours from LDS); rows_per_wave = 1,
                                waves_per_group = ty in {8, 16}, zchunk as
                                for the streaming kernel (0 = automatic)  */
#define WAVE_KERNEL_SHIFT 5  /* 2.5-D: one staged plane in LDS for the x/y
                                neighbours, the z neighbours in 9 registers
                                shifted each plane; parameters as RING     */
#define WAVE_KERNEL_PAIR 6   /* the streaming kernel with two x-adjacent
                                points per lane (128 x ty tiles, paired
                                loads and stores); rows_per_wave = 1,
                                waves_per_group = ty in {8, 16}, zchunk as
                                for WAVE_KERNEL_STREAM; not with an eta
                                array (EINVAL)                            */
#define WAVE_KERNEL_SEMI 7   /* the streaming kernel with the z terms of
                                Eq. 3 summed by the semi-stencil (Sec. IV,
                                "Semi-stencil"), along the streaming axis:
                                each staged plane adds c_zm u to the sums of
                                its z neighbours in a forward phase (outputs
                                ahead) and a backward phase (outputs behind,
                                the fourth of which it completes), so an
                                output is written 4 planes after it was
                                staged.  The same Laplacian summed in
                                another order: results differ from the
                                other variants by float32 rounding only (a
                                per-point bound is tested), which is why the
                                autotuner never picks it.  rows_per_wave = 1,
                                waves_per_group in {8, 16}, zchunk as for
                                WAVE_KERNEL_STREAM; not with an eta array
                                (EINVAL)                                 */
#define WAVE_KERNEL_PERSIST 8 /* the streaming kernel (the same tile code,
                                so the same results bit for bit) as one
                                persistent launch: one workgroup per CU,
                                each sweeping a fixed, rotated share of the
                                (tile, z chunk) items one after the other,
                                so no CU waits for a new workgroup to be
                                dispatched; rows_per_wave = 1,
                                waves_per_group in {8, 16}, zchunk as for
                                WAVE_KERNEL_STREAM                        */
#define WAVE_KERNEL_SHUFFLE 9 /* the streaming kernel with the x neighbours
                                exchanged by wavefront shuffles
                                (ds_bpermute across the lanes of a row
                                segment, the x halo loaded by the segment's
                                end lanes) instead of read from the staged
                                plane; the same values, so the same results
                                bit for bit; rows_per_wave = 1,
                                waves_per_group in {8, 16}, zchunk as for
                                WAVE_KERNEL_STREAM                        */

/* Select the sweep kernel and its tile: rows_per_wave (RY) and
 * waves_per_group (NW) give a 64 x (RY*NW) xy tile; zchunk is the number of
 * z planes one workgroup streams (0 = automatic).  Only compiled
 * combinations are accepted (EINVAL otherwise): (RY, NW) in
 * {(1,16), (1,8), (2,8), (2,4)}, and (2,16) (64 x 32 tiles) without an eta
 * array.  The default is WAVE_KERNEL_PERSIST with (1,16) tiles and its
 * automatic chunk (half the streaming kernel's) on grids large enough for
 * 64-plane chunks of 64 x 16 tiles with about 2048 workgroups (512^3 and
 * up for cubes), else WAVE_KERNEL_STREAM with (1,8) tiles (also where the
 * CU count cannot be queried).  The streaming
 * kernel addresses a chunk's planes with 32-bit offsets, so zchunk is cut
 * to what keeps zchunk + 8 float planes below 2 GiB; a grid whose single
 * plane is too large for that runs the direct kernel.  With
 * WAVE_KERNEL_STREAM2 (needs WAVE_TWO_STEP) rows_per_wave and
 * waves_per_group are ignored and zchunk is the two-step chunk (0 =
 * automatic; a window of zchunk + 16 planes).  Results do not depend on the
 * choice: every variant but WAVE_KERNEL_SEMI evaluates each point with the
 * same operations in the same order. */
int wave_set_kernel(wave_ctx *ctx, int32_t variant, int32_t rows_per_wave,
                    int32_t waves_per_group, int32_t zchunk);

/* Autotuner: advance the simulation by one untimed and `trial_steps` timed
 * real steps under the persistent launch (16 and 8 rows, two z-chunk
 * lengths), each compiled streaming tile shape at a few z-chunk lengths,
 * with WAVE_TWO_STEP the two-step kernel with a few z-chunk lengths
 * (trial_steps rounded up to even there), the two-points-per-lane kernel
 * (both tile heights, two z-chunk lengths; not with an eta array), the
 * shuffle kernel (both tile heights), then four of the paper's other code
 * shapes (WAVE_KERNEL_GMEM 8x8x8 and 64x4x4, RING and SHIFT with 16 rows);
 * never WAVE_KERNEL_SEMI, which rounds differently.  Every candidate computes
 * identical results, so the trials are ordinary steps of the run.  Each is
 * timed with HIP events; the fastest per step is kept (a candidate later in
 * the list must be at least 1.5 % faster to replace an earlier one, so
 * near-ties pick stably).  *chosen (may be NULL) receives the
 * wave_set_kernel arguments {variant, rows_per_wave, waves_per_group,
 * zchunk} of the pick; {0, 0, 0, 0} when the planes are too large to stream
 * and the direct kernel is kept.  Synchronises.  EINVAL if the steps would
 * overflow the trace buffer. */
int wave_tune(wave_ctx *ctx, int32_t trial_steps, int32_t chosen[4]);

/* When on, wave_step brackets every sweep-kernel launch with HIP events on
 * the context stream; wave_read_timing returns the summed kernel time (ms)
 * and the launch count since timing was switched on, and synchronises. */
int wave_set_timing(wave_ctx *ctx, int32_t on);
int wave_read_timing(wave_ctx *ctx, double *ms_total, int64_t *launches);

/* Algorithmic HBM bytes one sweep of this context moves: every array read
 * or written once per point.  Float32 storage: 16 bytes per inner point
 * (u^n, u^{n-1}, vp read, u^{n+1} written); a layer point adds phi read and
 * written (8) and, with WAVE_ETA_ARRAY, eta read (4).  u is 2 bytes per
 * access with 16-bit storage.  When the two-step kernel is in use, one
 * launch covers two steps: u^n, u^{n-1}, vp read and u^{n+1}, u^{n+2}
 * written per point (20 bytes in float32), phi read and written once more
 * in the layer. */
double wave_sweep_bytes(const wave_ctx *ctx);

/* Device-to-device copy of `bytes` (multiple of 16, both pointers 16-byte
 * aligned) with a plain streaming kernel on `hip_stream`: the reference
 * point for measured memory bandwidth.  Does not wait. */
int wave_stream_copy(void *dst, const void *src, size_t bytes, void *hip_stream);

/* Plain streams with other access mixes, the measured ceilings beside the
 * copy (an empirical roofline in the sense of Sec. V-C's ERT figures):
 * kind 0 reads `bytes` at a (dst: a 4-byte device sink, written only in a
 * case that does not occur, so the loads stay); kind 1 writes
 * dst = a + b c over `bytes` each (float4 words), the three-reads-one-write
 * mix of an inner point of the sweep.  16-byte aligned pointers, bytes a
 * multiple of 16 (EINVAL otherwise).  Does not wait. */
int wave_stream_mix(int32_t kind, void *dst, const void *a, const void *b, const void *c,
                    size_t bytes, void *hip_stream);

/* ---- many shots per launch (batching) ------------------------------------------ */

/* A batch advances several contexts together: every time step is one sweep
 * launch covering all members (their tiles side by side in one grid) plus
 * one launch for all members' sources and receivers.  Each member takes the
 * same steps, with the same arithmetic, as under wave_step, so its results
 * are identical to a run on its own.  Members must share the batch's storage
 * type; their streams may differ from the batch's: the batch's launches
 * wait (by event) for the work queued on a member's stream when it is
 * added, and a member's own later calls wait for the runs it took part in,
 * so set-up and read-out on other streams overlap with running blocks.
 * While a context is a member, wave_step on it returns
 * WAVE_EINVAL; state access (read/write field, traces, energy) stays valid
 * between runs. */
typedef struct wave_batch wave_batch;

/* Device bytes of the batch tables for up to max_shots members. */
size_t wave_batch_bytes_required(int32_t max_shots);

/* Create a batch.  storage is the members' wave_storage; the arena (256-byte
 * aligned, >= wave_batch_bytes_required) holds the member tables and stays
 * the caller's; hip_stream is the caller's stream.  The batch keeps a
 * stream of its own for its launches (ordered after and before the caller's
 * stream with events) so that step blocks can be captured as graphs, and
 * two pinned host buffers for its tables, so runs are enqueued without
 * waiting for earlier runs. */
int wave_batch_create(int32_t storage, int32_t max_shots, void *dev_arena, size_t arena_bytes,
                      void *hip_stream, wave_batch **out);

/* Add ctx with `nsteps` steps still to take (EINVAL: wrong storage, a
 * WAVE_STOCH_ROUND flag that differs from the current members' (a batch
 * runs one kernel instance), already a member, batch full, trace buffer
 * too small, z planes too large for the streaming kernel). */
int wave_batch_add(wave_batch *b, wave_ctx *ctx, int32_t nsteps);

/* Remove ctx (it keeps its state and may step on its own again). */
int wave_batch_remove(wave_batch *b, wave_ctx *ctx);

/* Enqueue up to n steps for every member (a member stops when its own
 * remaining count reaches 0) and return without waiting. */
int wave_batch_run(wave_batch *b, int32_t n);

/* Steps ctx still has to take in this batch. */
int wave_batch_remaining(const wave_batch *b, const wave_ctx *ctx, int32_t *remaining);

/* Tile shape of the batch sweep (same combinations as wave_set_kernel, or
 * rows_per_wave = 0 for the two-points-per-lane kernel with 128 x
 * waves_per_group tiles, waves_per_group in {8, 16}; EINVAL while a member
 * holds an eta array, and such a member cannot join then) and the number of
 * steps captured into one graph (0 = plain launches). */
int wave_batch_set_kernel(wave_batch *b, int32_t rows_per_wave, int32_t waves_per_group);
int wave_batch_set_graph(wave_batch *b, int32_t steps_per_graph);

/* Autotuner for a batch: runs trial_steps steps under each compiled tile
 * shape (and the two-points-per-lane tiles when no member holds an eta
 * array) and keeps the fastest; *chosen = {rows_per_wave, waves_per_group}
 * as wave_batch_set_kernel takes them. */
int wave_batch_tune(wave_batch *b, int32_t trial_steps, int32_t chosen[2]);

/* Wait for the batch's work, release it (members stay valid contexts). */
int wave_batch_free(wave_batch *b);

/* ---- diagnostics ----------------------------------------------------------- */

const char *wave_strerror(int status);
const char *wave_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* WAVE_H */
