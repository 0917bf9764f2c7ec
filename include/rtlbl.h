/*
 * rtlbl.h -- C ABI of the MI355X (gfx950) line-by-line Monte-Carlo radiative
 * ray tracer.
 *
 * The calls follow the problem as the paper states it (Collange, Daumas,
 * Defour, "Graphic processors to speed-up simulations for the design of high
 * performance solar receptors", Section 3): a finite-volume code holds per
 * volume the temperature, pressure and density of absorbing gas; line-by-line
 * spectra give each volume its absorption coefficient (Eqs. (1)-(2));
 * Monte-Carlo rays are marched volume after volume with Beer-Lambert
 * attenuation and Planck emission (Eqs. (3)-(4)); the power exchanged,
 * a sum of I_in - I_out, is returned to the host.
 *
 * Conventions shared by every call
 *   - Units: wavenumbers and half widths in cm^-1, line strengths in
 *     cm/molecule, temperatures in K, pressures in atm, cell edge in m,
 *     kappa in cm^-1, radiance in W m^-2 sr^-1 (cm^-1)^-1, power in W.
 *   - Cells are indexed c = ix + nx*(iy + ny*iz).
 *   - Host arrays passed in are copied before the call returns; the caller
 *     may free them afterwards.
 *   - Device buffers passed in (kappa, Planck table) stay owned by the
 *     caller and must stay alive until every call that reads them has
 *     completed on the stream.
 *   - All device work is ordered on the stream given at creation; only
 *     rt_tally, rt_debug_segments, rt_get_stats and rt_destroy synchronise.
 *   - A handle is not thread-safe: use one handle per host thread.
 *   - Every call returns RT_OK or a negative rt_status; it never aborts.
 *     rt_last_error gives the message of the last failure on the handle.
 */
#ifndef RTLBL_H
#define RTLBL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rt_ctx_s* rt_ctx;

typedef enum {
  RT_OK = 0,
  RT_EINVAL = -1,       /* an argument is out of range, NULL or not finite */
  RT_ENOMEM = -2,       /* a device or host allocation failed              */
  RT_EDEVICE = -3,      /* a HIP call failed                               */
  RT_ESTATE = -4,       /* calls made out of order                         */
  RT_EUNSUPPORTED = -5  /* mode not available in this build                */
} rt_status;

typedef enum {
  RT_KAPPA_PLAIN = 0,        /* FP32 line sum                               */
  RT_KAPPA_COMPENSATED = 1,  /* the precision form's line sum: FP32 only --
                                compensated summation, and the Eq. (1)
                                factors from FP32 exponentials (Cody-Waite
                                range reduction on FP32-pair arguments) of
                                per-cell and per-line inputs the host forms in
                                FP64 (1/T_ref - 1/T, c2/T, c2 E, nu, u, p)   */
  RT_KAPPA_SURROGATE = 2,    /* learned form (rt_surrogate_train/load), with
                                line-sum fallback and a sampled check       */
  RT_KAPPA_TABLE16 = 3,      /* the paper's own formulation (Section 3 and its
                                listing): each line contributes at the 16 grid
                                points m-7 .. m+8 around its centre through a
                                profile tabulated once at the reference state
                                (Lorentz, gamma_ref, 1 atm), scaled per cell by
                                the density and the Eq. (1) strength ratio;
                                multiply-adds only, no per-cell half width.  An
                                approximation of the plain sum, every gas. */
  RT_KAPPA_ADAPTIVE = 4,     /* the paper's announced next version (its
                                conclusion): the points evaluated per line
                                follow the local temperature and the line's
                                intensity.  The FP32 line sum of the plain
                                mode over adaptive windows: see
                                rt_set_line_tolerance.  Gas 0 only. */
  RT_KAPPA_ADAPTIVE_WINGS = 5 /* an extension of RT_KAPPA_ADAPTIVE, not in
                                the paper: the same windows and line sum,
                                plus per cell the Lorentz mass of the points
                                the windows drop, returned as one constant
                                over the band.  Each dropped range a..b of
                                line i (in its plain window, on the grid)
                                counts its midpoint-rule integral, u S_i s_ci
                                (atan((b + 1/2 - r_i) dnu / g) - atan((a -
                                1/2 - r_i) dnu / g)) / (pi dnu), and cell c
                                adds the sum over its lines, divided by n_nu,
                                at every point: the band integral of the plain
                                sum is kept to within the midpoint rule's
                                error on the wings (Eq. (2) with the cutoff).
                                Gas 0 only; needs rt_set_line_tolerance. */
} rt_kappa_mode;

/* Cells sharing one line window in RT_KAPPA_ADAPTIVE: cell c belongs to the
 * run c / RT_ADAPTIVE_GROUP of consecutive cells (x fastest). */
#define RT_ADAPTIVE_GROUP 8

/* Form of the march (Eq. (3)).  In both, the per-segment sums over a
 * wavefront are formed in a fixed order and added to per-cell accumulators
 * that are exact fixed-point integers (digits of 2^-112 W up to 2^80 W), so
 * the tallies do not depend on the order in which the GPU delivers them: the
 * same rays give the same tallies bit for bit, however they are split over
 * calls.  Each added value is rounded to 29 significant bits first.
 *   RT_TALLY_F32: plain form.  Planck values evaluated in registers (FP32),
 *     1 - exp(-tau) from the hardware exponential with a degree-3 series
 *     below tau = 1/32, per-wavefront partial sums in FP32.
 *   RT_TALLY_F64: precision form.  Planck values read from the table of
 *     rt_compute_kappa (required), degree-5 series below tau = 1/4, all in
 *     FP32; FP64 only in the tally (per-lane partial sums and the weighted
 *     values added to the accumulators). */
typedef enum {
  RT_TALLY_F32 = 0,
  RT_TALLY_F64 = 1
} rt_tally_prec;

typedef struct {
  double line_evals;        /* in-window (cell, line, nu) triples evaluated by
                               rt_compute_kappa since the last reset          */
  double kappa_ms;          /* device time of the line-sum kernels since then */
  double updates;           /* ray-cell-nu updates since the last reset       */
  double segments;          /* ray-cell segments since the last reset         */
  double trace_ms;          /* device time of rt_trace_rays since the reset   */
  double march_ms;          /* of which in the march kernel                    */
  double rays;              /* rays traced since the last reset               */
  double march_launches;    /* march kernel launches since the last reset     */
  double batch_line_evals;  /* line evaluations of the last batched launch    */
  double batch_updates;     /* ray-cell-nu updates of the last batched launch */
  double batch_ms;          /* device time of the last batched launch         */
} rt_stats;

/* Create a handle bound to HIP device `hip_device` and the borrowed stream
 * `hip_stream` (a hipStream_t; NULL = the null stream).  The stream is not
 * owned: it must outlive the handle.
 * hip_device = RT_NO_DEVICE (stream NULL) creates a host-only handle, for
 * checking inputs where there is no GPU: it makes no HIP call, checks every
 * call's arguments and the call order exactly as a device handle does
 * (RT_EINVAL, RT_ESTATE), accepts rt_setup_grid and rt_setup_lines (keeping
 * only their sizes and spectral grid), and returns RT_EUNSUPPORTED from every
 * call that would run on a device. */
#define RT_NO_DEVICE (-1)
rt_status rt_create(rt_ctx* out, int hip_device, void* hip_stream);

/* Synchronise the stream and free everything the handle owns. */
rt_status rt_destroy(rt_ctx ctx);

/* Message of the last failed call on `ctx` (or of rt_create when ctx is
 * NULL); valid until the next call on the handle. */
const char* rt_last_error(rt_ctx ctx);

/* The finite-volume grid (Section 3: isothermal homogeneous volumes).
 * nx, ny, nz >= 1, nx*ny*nz < 2^31, each <= 2^20; cubic cells of edge
 * cell_m > 0 metres; T_K > 0, 0 <= x_h2o <= 1, p_atm > 0 per cell (host
 * arrays of nx*ny*nz doubles, copied); T_wall_K >= 0 is the temperature of
 * the black walls (0: cold walls, nothing enters).  Resets the tallies and
 * invalidates a previous rt_compute_kappa. */
rt_status rt_setup_grid(rt_ctx ctx, int nx, int ny, int nz, double cell_m,
                        const double* T_K, const double* x_h2o,
                        const double* p_atm, double T_wall_K);

/* The line list (Eqs. (1)-(2)) and the spectral grid nu_j = nu0_cm + j*dnu_cm,
 * 0 <= j < n_nu.  Per line: centre nu_cm, strength S_ref at T_ref_K [cm per
 * molecule] (>= 0), Lorentz half width gamma_ref_cm at T_ref and 1 atm (> 0),
 * half-width temperature exponent n_T, lower-state energy E_lower_cm (>= 0;
 * NULL: the strength is taken as temperature independent, Eq. (1) ratio 1).
 * Each line is evaluated on the points with |nu_j - nu_line| <= cutoff_cm;
 * cutoff_cm/dnu_cm must be an integer (to 1e-9 relative).  n_lines >= 0,
 * n_nu >= 1, dnu_cm > 0.  Host arrays are copied.  Invalidates a previous
 * rt_compute_kappa.  nu0_cm > 0. */
rt_status rt_setup_lines(rt_ctx ctx, int n_lines, const double* nu_cm,
                         const double* S_ref, const double* gamma_ref_cm,
                         const double* n_T, const double* E_lower_cm,
                         double T_ref_K, double cutoff_cm, double nu0_cm,
                         double dnu_cm, int n_nu);

/* A further absorbing gas: Eq. (2) sums over gases, each with its own line
 * list and density.  gas in 1..3 (gas 0 is the one of rt_setup_grid's x_h2o
 * and rt_setup_lines).  x is the gas's mole fraction per cell (host, nx*ny*nz
 * doubles in [0, 1], copied); the lines are given as for rt_setup_lines
 * (E_lower_cm may be NULL for this gas alone) and placed on gas 0's spectral
 * grid with its cutoff and T_ref.  n_lines == 0 removes the gas (x may then
 * be NULL).  rt_compute_kappa in the plain and compensated modes then writes
 * the sum over gases (each gas's line sum is added to the table in turn);
 * the surrogate mode and the batched form take gas 0 only and return
 * RT_EUNSUPPORTED while a further gas is set.  Needs rt_setup_grid and
 * rt_setup_lines first (RT_ESTATE); calling either of them again removes
 * gases 1..3.  Invalidates a previous rt_compute_kappa. */
rt_status rt_setup_gas(rt_ctx ctx, int gas, const double* x, int n_lines, const double* nu_cm,
                       const double* S_ref, const double* gamma_ref_cm, const double* n_T,
                       const double* E_lower_cm);

/* Smallest admissible row pitch (in floats) of the kappa and Planck tables
 * for the current spectral grid: n_nu rounded up to the march chunk (1536);
 * -1 before rt_setup_lines. */
int64_t rt_required_pitch(rt_ctx ctx);

/* The march's spectral chunk in points (64 lanes x points per lane): table
 * pitches and the batched form's chunk_points are multiples of it. */
int rt_march_chunk(void);

/* Eq. (2) with Eq. (1) per cell: kappa_dev[c*ld + j] = kappa_c(nu_j) in
 * cm^-1, and, when planck_dev is not NULL, Eq. (4): planck_dev[c*ld + j] =
 * B(nu_j, T_c), evaluated in FP32 (c1 nu^3 over an FP32 expm1 of the pair
 * product c2 nu / T; within 1e-6 relative).  The walls' row is evaluated the
 * same way.  Both are caller
 * allocated, 16-byte aligned device buffers of nx*ny*nz rows of `ld` floats,
 * ld a multiple of 1536 and >= rt_required_pitch (columns n_nu .. ld-1 are
 * written with zeros).  The handle keeps both pointers for rt_trace_rays;
 * the Planck table is needed by the precision form of the march only.
 * mode: rt_kappa_mode. */
rt_status rt_compute_kappa(rt_ctx ctx, int mode, float* kappa_dev,
                           float* planck_dev, int64_t ld);

/* Tolerance eps of RT_KAPPA_ADAPTIVE, 0 < eps < 1 (finite), kept by the
 * handle until changed.  The windows (decided in binary64, from the
 * conclusion's announced adaptive evaluation of the lines):
 *   - reference level of cell c: the band mean of its untruncated line sum,
 *     u_c sbar_c with sbar_c = sum_i S_i s_ci / (n_nu dnu) over the lines
 *     whose hard-cutoff window meets the grid (s_ci the Eq. (1) ratio);
 *   - line i keeps point j in cell c while its Lorentz value there is at
 *     least eps u_c sbar_c, i.e. within w_ci = sqrt(S_i s_ci g / (pi eps
 *     sbar_c) - g^2) / dnu grid points of its centre (g = gamma_ci; no point
 *     when the root is imaginary);
 *   - the window is shared by the RT_ADAPTIVE_GROUP cells of a run: the
 *     widest w_ci among them, capped by the hard cutoff, so each cell keeps
 *     at least what its own rule asks for;
 *   - point j is kept when it lies in the plain mode's window and
 *     |j - r_i| <= that half width, r_i = (nu_i - nu0)/dnu.
 * With sbar_c = 0 (no line strength at all) the plain window is kept.
 * Every dropped term of cell c is below eps u_c sbar_c.  rt_get_stats
 * counts the kept (cell, line, point) evaluations as line_evals.  The
 * windows are recomputed by every rt_compute_kappa in this mode, in a
 * table the handle owns: 4 bytes per (run of cells, kept line).
 * Needs cutoff/dnu <= 32767.  Returns RT_EINVAL for eps outside (0, 1). */
rt_status rt_set_line_tolerance(rt_ctx ctx, double eps);

/* Monte-Carlo rays (Section 3: the host directs the rays and averages their
 * effect).  Traces rays ray_begin .. ray_begin+ray_count-1 of a set of
 * n_rays_total rays drawn with `seed`: a uniform point on the boundary and
 * a cosine-weighted inward direction from a Philox4x64-10 stream, exact
 * integer traversal, then Eq. (3) cell after cell for every nu_j with ray
 * weight pi * A_boundary * dnu / n_rays_total.  Adds to the per-cell
 * absorbed/emitted power and to the energy balance; ranges may be traced in
 * any order and any split (tallies add).  tally_prec: rt_tally_prec.
 * The rays of a call are traced in batches of up to about 1 GiB of segment
 * scratch (owned by the handle); a batch of 2^15 rays or more is marched in
 * a coherent order (rays sorted by direction and position), which changes
 * only the order of the floating-point additions.
 * Requires rt_compute_kappa. */
rt_status rt_trace_rays(rt_ctx ctx, uint64_t seed, uint64_t n_rays_total,
                        uint64_t ray_begin, uint64_t ray_count,
                        int tally_prec);

/* rt_trace_rays for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same rays, kernels and tallies as rt_trace_rays -- bit for bit the same
 * tallies -- but the call allocates nothing.  Its ray segments, order keys,
 * permutation and histogram live in a static 64 MiB device array that the
 * library holds on every GPU it runs on until the process ends; the tallies
 * are the handle's own (allocated by rt_setup_grid).  Rays are traced in
 * batches of as many as fit: 12 + 8 (nx+ny+nz) bytes per ray, at most 2^21
 * rays per batch.  RT_EINVAL when not even 256 rays of the grid fit
 * (nx+ny+nz above about 32,000).  Records no timing for rt_get_stats.
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind: calls that overlap on one GPU (other handles, other streams, other
 * host threads) race and must be serialised by the caller.  Other arguments,
 * errors and requirements as rt_trace_rays. */
rt_status rt_trace_rays_noalloc(rt_ctx ctx, uint64_t seed, uint64_t n_rays_total,
                                uint64_t ray_begin, uint64_t ray_count, int tally_prec);

/* Rays given explicitly in the fixed-point frame (one cell edge = 2^21
 * units): origin O[3*r..] on the boundary, inward integer direction
 * D[3*r..] (|D_k| <= 2^21), host arrays, n_rays >= 1, with the given
 * weight (0 <= weight <= 2^40).  For closed-form checks (slabs, axis-normal
 * rays).  If exit_I is not NULL it is a host array of n_rays*n_nu doubles
 * receiving the radiance at exit.  Synchronises when exit_I is given. */
rt_status rt_trace_explicit(rt_ctx ctx, int n_rays, const int64_t* O,
                            const int64_t* D, double weight, int tally_prec,
                            double* exit_I);

/* The power exchanged with each volume, summed over rays and wavenumbers
 * (Section 3: the host receives the sum of I_in - I_out over the volumes, as
 * absorbed minus emitted; both are returned).  Copies the tallies to the host
 * (synchronises): absorbed_W[c] and emitted_W[c] (host arrays of nx*ny*nz
 * doubles, each may be NULL) and balance[4] = {entering, emitted, absorbed,
 * escaped} in W (may be NULL); emitted and absorbed in the balance are exact
 * sums of the per-cell accumulators, converted once.  RT_EDEVICE if a traced
 * power fell outside the accumulators' range (negative, not finite or not
 * below 2^80 W). */
rt_status rt_tally(rt_ctx ctx, double* absorbed_W, double* emitted_W,
                   double* balance);

/* Zeroes the tallies, the work counters and the timers (may synchronise). */
rt_status rt_reset_tally(rt_ctx ctx);

/* Traversal of rays ray_begin .. ray_begin+count-1 (as rt_trace_rays draws
 * them) for bit-exact checks: counts[r] segments, cells[r*max_segs + k] and
 * len_cm[r*max_segs + k]; host arrays; max_segs >= nx+ny+nz.  Also returns
 * the integer origin O[3r..] and direction D[3r..] when those are not NULL.
 * Synchronises. */
rt_status rt_debug_segments(rt_ctx ctx, uint64_t seed, uint64_t ray_begin,
                            uint64_t count, int max_segs, int32_t* counts,
                            int32_t* cells, float* len_cm, int64_t* O,
                            int64_t* D);

/* Work counters and device times (synchronises). */
rt_status rt_get_stats(rt_ctx ctx, rt_stats* out);


/* ------------------------------------------------------------------------
 * Batched form: many independent receiver cases (each its own grid, wall
 * temperature, ray count and seed) sharing the line list and spectral grid
 * of rt_setup_lines, run as one HIP graph launch.  The line sum and the
 * march are fused per spectral chunk: a chunk's kappa is built into a slab
 * and marched at once, so no full kappa table is ever stored.  Two launch
 * shapes give the same tallies bit for bit:
 *   RT_BATCH_CHUNKED    per chunk, one line-sum launch over the cells of
 *                       every case into a slab of all cells, then one march
 *                       launch over the rays of every case; with slots > 1
 *                       the line sums run on a second stream, up to
 *                       slots - 1 chunks ahead of the marches
 *                       (kappa_groups, march_rays, blocks_per_cu unused);
 *   RT_BATCH_PERSISTENT one persistent work-queue kernel over (case, chunk)
 *                       pairs, each pair's kappa in one of `slots` slabs of
 *                       the largest case (less memory).
 * Plain-form march (rt_tally_prec RT_TALLY_F32); kappa_mode as
 * rt_compute_kappa.
 * ---------------------------------------------------------------------- */
typedef struct {
  int nx, ny, nz;        /* as rt_setup_grid                                */
  double cell_m;
  const double* T_K;     /* host, nx*ny*nz each; read by rt_batch_prepare   */
  const double* x_h2o;
  const double* p_atm;
  double T_wall_K;
  uint64_t seed;         /* Philox seed of the case's rays                  */
  uint64_t n_rays;       /* >= 1                                            */
} rt_case;

enum { RT_BATCH_CHUNKED = 0, RT_BATCH_PERSISTENT = 1 };

typedef struct {
  int chunk_points;   /* nu points per spectral chunk, multiple of
                         rt_march_chunk() (1536)                            */
  int kappa_groups;   /* persistent: groups of 8 cells per line-sum item    */
  int march_rays;     /* persistent: rays per march item, multiple of 4     */
  int blocks_per_cu;  /* persistent: blocks per compute unit, 1..8          */
  int slots;          /* kappa slabs in flight: persistent 2..8, chunked
                         1..8                                               */
  int mode;           /* RT_BATCH_CHUNKED or RT_BATCH_PERSISTENT            */
} rt_batch_tuning;

/* A tuning that is valid for any batch: chunked, 3072 points per chunk,
 * one slab (persistent fields 16, 64, 2; the queue needs slots >= 2). */
rt_status rt_batch_default_tuning(rt_batch_tuning* out);

/* Device workspace the batch needs with this tuning (tuning NULL: default):
 * segments of every ray, `slots` kappa slabs (chunked: chunk_points for
 * every cell of every case; persistent: for the largest case),
 * per-case tables, accumulators and the work plan. */
rt_status rt_batch_workspace_size(rt_ctx ctx, int n_cases, const rt_case* cases,
                                  const rt_batch_tuning* tuning, int64_t* bytes);

/* Validates the cases, copies their fields into the caller-owned device
 * workspace (at least rt_batch_workspace_size bytes, 256-byte aligned),
 * derives per-cell parameters and builds the work plan and its HIP graph.
 * The workspace must stay alive until the last rt_batch_results. */
rt_status rt_batch_prepare(rt_ctx ctx, int n_cases, const rt_case* cases,
                           int kappa_mode, const rt_batch_tuning* tuning,
                           void* workspace_dev, int64_t workspace_bytes);

/* One launch of the prepared graph on the handle's stream (asynchronous):
 * clears the accumulators, traces all cases and reduces the per-case
 * balances.  May be repeated. */
rt_status rt_batch_launch(rt_ctx ctx);

/* Synchronises and copies the results of the last launch: absorbed_W and
 * emitted_W concatenate the cases' cells in case order (host arrays of the
 * total cell count, each may be NULL); balance holds 4 doubles per case
 * {entering, emitted, absorbed, escaped} (may be NULL).  RT_EDEVICE if the
 * persistent kernel reported a stalled dependency wait. */
rt_status rt_batch_results(rt_ctx ctx, double* absorbed_W, double* emitted_W,
                           double* balance);

/* The whole batched form in one call, for callers that do not keep a
 * prepared batch: the workspace is allocated here (rt_batch_workspace_size
 * bytes of device memory, freed before returning), then rt_batch_prepare,
 * one rt_batch_launch and rt_batch_results as above.  tuning NULL: the
 * default.  Synchronises; leaves no batch prepared.  RT_ENOMEM when the
 * workspace cannot be allocated. */
rt_status rt_batch_run(rt_ctx ctx, int n_cases, const rt_case* cases, int kappa_mode,
                       const rt_batch_tuning* tuning, double* absorbed_W, double* emitted_W,
                       double* balance);

/* Picks the mode, chunk_points, kappa_groups, march_rays, blocks_per_cu and slots by timing
 * launches restricted to the first spectral chunks of every case (a sweep
 * one parameter at a time from the default), and remembers the winner in a
 * JSON file keyed by device architecture and a bucket of the batch shape
 * (cache_path NULL: no file).  A cached entry is returned without timing.
 * Leaves no batch prepared. */
rt_status rt_batch_autotune(rt_ctx ctx, int n_cases, const rt_case* cases,
                            int kappa_mode, void* workspace_dev,
                            int64_t workspace_bytes, const char* cache_path,
                            rt_batch_tuning* best);


/* ------------------------------------------------------------------------
 * Learned form: an MLP 4 -> 512 -> 512 -> 512 -> 256 (SiLU, BF16 weights,
 * FP32 accumulation on MFMA) maps (T, x_H2O, p, spectral-chunk index) to
 * the 256 values of ln(kappa/u) of a 256-point chunk, each output
 * normalised over the training spectra.  It is trained on spectra of the
 * exact line sum (Eqs. (1)-(2)) for the current line list and spectral
 * grid.  rt_compute_kappa in RT_KAPPA_SURROGATE mode fills the kappa table
 * from it (a last chunk that the spectrum ends inside is summed exactly
 * instead when fewer than 256 lines meet a 512-point tile), recomputes with the line sum every cell outside the training
 * box, checks every chunk against the line sum on `check_cells` sampled
 * cells and recomputes the whole chunk for all cells when the relative error
 * of the chunk's absorptance along one cell edge h,
 * |sum (a_mlp - a)| / sum a with a = 1 - exp(-kappa h), exceeds `tolerance`.
 * ---------------------------------------------------------------------- */
typedef struct {
  int n_samples;              /* training gas states (>= 64)               */
  const double* T_K;          /* host arrays of n_samples states           */
  const double* x_h2o;
  const double* p_atm;
  double T_min, T_max;        /* validity box of the surrogate             */
  double x_min, x_max;
  double p_min, p_max;
  int epochs;                 /* passes over the (sample, chunk) rows      */
  int batch;                  /* rows per Adam step, multiple of 64        */
  float lr;                   /* initial Adam step (cosine decay)          */
  uint64_t seed;              /* weight initialisation and shuffling       */
  int check_cells;            /* cells sampled per inference check, 0..256 */
  double tolerance;           /* checked absorptance error for fallback    */
} rt_surrogate_cfg;

typedef struct {
  double check_error;         /* largest checked chunk error, last inference */
  int fallback_chunks;        /* chunks recomputed with the line sum         */
  int fallback_cells;         /* out-of-range cells recomputed               */
  int n_chunks;
  double infer_ms, check_ms, fallback_ms;  /* device times of the last
                                 inference when it ran with phase timing on
                                 (rt_surrogate_time_phases), else 0: the
                                 network's launch (with the check's exact
                                 rows, unless a long line list puts them on a
                                 second stream, the exact last chunk and the
                                 walls' row); from its end to the end of the
                                 check; the fallback                         */
  double train_loss;          /* mean squared normalised error, last epoch   */
  double param_count;
  int exact_chunks;           /* last inference: 1 when the spectrum ends
                                 inside the last chunk and the line list is
                                 light, the chunk's points then summed exactly
                                 beside the network (never counted as a
                                 fallback), else 0                           */
} rt_surrogate_stats;

/* Trains a new surrogate for the current line list and spectral grid
 * (replaces any previous one).  final_loss may be NULL. */
rt_status rt_surrogate_train(rt_ctx ctx, const rt_surrogate_cfg* cfg, double* final_loss);

/* Versioned binary blob with an FNV-1a checksum; load validates it. */
rt_status rt_surrogate_save(rt_ctx ctx, const char* path);
rt_status rt_surrogate_load(rt_ctx ctx, const char* path);

/* Raw network outputs (normalised ln(kappa/u)) for n_rows host input rows of
 * 4 normalised features each; outputs: host n_rows * 256 floats.  Synchronous. */
rt_status rt_surrogate_forward(rt_ctx ctx, int n_rows, const float* inputs, float* outputs);

/* FP32 master parameters W1 [4][512], b1, W2 [512][512], b2, W3, b3,
 * W4 [512][256], b4 (row-major [in][out]) into a host array of n floats. */
rt_status rt_surrogate_weights(rt_ctx ctx, float* out, int64_t n);

rt_status rt_surrogate_get_stats(rt_ctx ctx, rt_surrogate_stats* out);

/* Phase timing of the learned form's inference.  With on != 0, each later
 * rt_compute_kappa call in RT_KAPPA_SURROGATE mode records timing events
 * between its kernels (before and after the network, after the check and
 * after the fallback), which rt_surrogate_get_stats
 * reports; off (the default), it records none and reports the phase times
 * as 0.  The events cost the call several microseconds.  Needs no device
 * and no trained surrogate; RT_EINVAL for a NULL handle. */
rt_status rt_surrogate_time_phases(rt_ctx ctx, int on);

/* ------------------------------------------------------------------------
 * FP32 arithmetic characterisation of the device (the paper's Section 2
 * test vectors, Table 2): rounding near ties, fused or unfused multiply-add,
 * product symmetry and error, overflow inside a composite, subnormals and
 * NaNs.  rt_arith_eval applies one operation element-wise with the
 * instruction named below and stores each FP32 result bit for bit; the
 * expected values and errors are for the caller to work out from exact
 * arithmetic.  Composites (RT_AR_FMA_ERR, RT_AR_ADD_SUB, RT_AR_SUB_SUB) keep
 * their intermediate in a register, so extended precision or exponent range
 * inside the unit would show.
 * ------------------------------------------------------------------------ */
typedef enum {
  RT_AR_COPY = 0,     /* x: load and store only (subnormals, NaN payloads)    */
  RT_AR_ADD = 1,      /* x + y            v_add_f32                            */
  RT_AR_SUB = 2,      /* x - y            v_sub_f32                            */
  RT_AR_MUL = 3,      /* x * y            v_mul_f32                            */
  RT_AR_FMA = 4,      /* x * y + z, one rounding          v_fma_f32            */
  RT_AR_MUL_ADD = 5,  /* x * y + z, product rounded first v_mul_f32, v_add_f32 */
  RT_AR_FMA_ERR = 6,  /* fma(x, y, -(x * y)): the product's rounding error     */
  RT_AR_ADD_SUB = 7,  /* (x + y) - z, intermediate in a register              */
  RT_AR_SUB_SUB = 8,  /* (x - y) - z, intermediate in a register              */
  RT_AR_DIV = 9,      /* x / y as the compiler expands it (IEEE division)      */
  RT_AR_EXP2 = 10,    /* 2^x              v_exp_f32                            */
  RT_AR_LOG2 = 11,    /* log2 x           v_log_f32                            */
  RT_AR_RCP = 12,     /* 1 / x            v_rcp_f32                            */
  RT_AR_RSQ = 13,     /* 1 / sqrt(x)      v_rsq_f32                            */
  RT_AR_SQRT = 14     /* sqrt(x)          v_sqrt_f32                           */
} rt_arith_op;

/* out[k] = op(a[k], b[k], c[k]) for k < n, on the handle's device and
 * stream (asynchronous).  a, b, c and out are device pointers to FP32
 * arrays of n elements owned by the caller; b must be non-NULL for
 * two-operand ops and b and c for three-operand ops (a NULL operand an op
 * does not use is fine).  Returns RT_EINVAL for an unknown op, a missing
 * operand, n < 0 or NULL out; n == 0 does nothing.  Needs no setup call. */
rt_status rt_arith_eval(rt_ctx ctx, int op, const float* a, const float* b, const float* c,
                        float* out, int64_t n);

#ifdef __cplusplus
}
#endif

#endif /* RTLBL_H */
