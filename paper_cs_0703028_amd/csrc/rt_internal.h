// rt_internal.h -- state and device helpers shared by the translation units
// of librtlbl (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/rtlbl.h"

namespace rt {

// Fixed-point traversal frame: one cell edge is 2^21 integer units.
constexpr int64_t kCellUnits = int64_t(1) << 21;
#ifndef RT_MARCH_POINTS_PER_LANE
#define RT_MARCH_POINTS_PER_LANE 24
#endif
// march: nu points per wavefront (64 lanes x contiguous points per lane); a
// multiple of the 512-point line-sum tile
constexpr int kChunk = 64 * RT_MARCH_POINTS_PER_LANE;
constexpr int kMaxAxis = 1 << 20; // largest admissible cells per axis

// Physical constants (SI 2019 exact values).
constexpr double kPlanckH = 6.62607015e-34;
constexpr double kLightC = 299792458.0;
constexpr double kBoltzmann = 1.380649e-23;
constexpr double kAtm = 101325.0;
inline double second_radiation_cm_K() { return kPlanckH * kLightC / kBoltzmann * 100.0; }
inline double first_radiation_wavenumber() { return 2.0 * kPlanckH * kLightC * kLightC * 1e8; }

// Per-line data after sorting by centre (device, structure of arrays).
struct LineSet {
  int n = 0;              // lines kept (window meets the grid)
  int32_t* m = nullptr;   // floor((nu - nu0)/dnu)
  float* phi = nullptr;   // (nu - nu0)/dnu - m, rounded to float
  int32_t* wlo = nullptr; // first grid point of the window: m - K + [phi > 0]
  int32_t* whi = nullptr; // last grid point of the window:  m + K
  float* S = nullptr;     // S_ref, divided by (1 - exp(-c2 nu/T_ref)) with energies
  double* E2 = nullptr;   // c2 * E_lower  (0 without energies)
  double* nu = nullptr;   // centre, cm^-1
  float* gamma = nullptr; // half width at T_ref, 1 atm
  float* nexp = nullptr;  // half-width temperature exponent
  // the paper's tabulated profile: per line, the Lorentz shape at the
  // reference state, gamma_ref / (pi ((j - r)^2 dnu^2 + gamma_ref^2)), at the
  // 16 grid points j = m - 7 .. m + 8 (FP64, stored FP32), [n][16]
  float* prof16 = nullptr;
  // lines whose 16 points meet 256-point tile t of the grid: [lo, hi) of the
  // sorted list, int2 per tile (t = 0 .. n_tiles16 - 1)
  int2* tile16 = nullptr;
  int n_tiles16 = 0;
  // per 64-point span b of the grid (points 64 b .. 64 b + 63), indices into
  // the sorted list: x the first line whose window reaches point 64 b or
  // beyond (whi >= 64 b), y the first starting beyond point 64 b + 63
  // (wlo > 64 b + 63), z the first with whi >= 64 b + 63, w the first with
  // wlo > 64 b.  The line sum's blocks and wavefronts start and end on
  // spans, so their line ranges are table reads instead of binary searches.
  // Spans from n_spans on lie past every window: (n, n, n, n).
  int4* span4 = nullptr;
  int n_spans = 0;
  // binary64 line data for the adaptive windows: r = (nu - nu0)/dnu,
  // S_ref, gamma_ref, n_T, a = -c2 E and 1/expm1(-c2 nu / T_ref)
  double* r64 = nullptr;
  double* S64 = nullptr;
  double* g64 = nullptr;
  double* n64 = nullptr;
  double* aE = nullptr;
  double* rN = nullptr;
  // inputs of the precision form's FP32 line parameters: c2 E and the centre
  // nu, each split on the host into an FP32 pair hi + lo
  float2* E2p = nullptr;
  float2* nup = nullptr;
};

// Per-cell derived parameters (device), from FP64 on the device.
struct CellSet {
  float* G = nullptr;       // u q / (pi dnu): density x partition ratio, grid scale
  double* beta = nullptr;   // 1/T_ref - 1/T
  double* theta = nullptr;  // c2 / T
  float* lam2 = nullptr;    // log2(T_ref / T)
  float* P = nullptr;       // p / dnu
  // The precision form's per-cell inputs, FP32 on the device: the host forms
  // u/(pi dnu), log2(T_ref/T) and p/dnu and the exponent factors 1/T_ref - 1/T
  // and c2/T (as FP32 pairs hi + lo) from the FP64 gas state; every
  // exponential, Gq = u q / (pi dnu) with q = 2^(1.5 log2(T_ref/T)) among
  // them, is evaluated on the device in FP32.
  float* uf = nullptr;
  float* lamf = nullptr;
  float* Pf = nullptr;
  float2* beta2 = nullptr;
  float2* theta2 = nullptr;
  float* Gq = nullptr;
};

// A further absorbing gas: lines, mole fraction per cell (FP64, device) and
// the per-cell factor u q / (pi dnu) it gives (FP32, device).
constexpr int kMaxGases = 4;
struct ExtraGas {
  bool active = false;
  bool have_E = false;
  LineSet lines;
  double* x = nullptr;
  float* G = nullptr;
  double line_evals_per_cell = 0;
  std::vector<double> hx;     // host copy of x (for the precision form's uf)
  float* uf = nullptr;        // u/(pi dnu) from the host, FP32
  float* Gq = nullptr;        // u q/(pi dnu), FP32 on the device
};

struct Stats {
  double line_evals = 0;
  double kappa_ms = 0;
  double trace_ms = 0;
  double march_ms = 0;
  double rays = 0;
  double march_launches = 0;
  double batch_line_evals = 0;
  double batch_updates = 0;
  double batch_ms = 0;
};

// Device memory one batch of rays is traced in: per ray a fixed stride of
// max_segs (cell, length) segments and their count, the coherent-order key
// and permutation, and the order's histogram (kOrderBuckets words).
struct RayScratch {
  int2* segs = nullptr;
  int32_t* counts = nullptr;
  uint32_t* keys = nullptr;
  uint32_t* perm = nullptr;
  uint32_t* hist = nullptr;
  int max_segs = 0;
  int64_t cap = 0;  // rays per batch
};

struct BatchPlan;
struct Surrogate;
}  // namespace rt

struct rt_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;

  // grid
  bool have_grid = false;
  double T_min = 0, T_max = 0;  // cell temperature range of the grid
  int64_t T_argmin = 0, T_argmax = 0;
  uint64_t grid_epoch = 0;      // bumped by every rt_setup_grid
  int nx = 0, ny = 0, nz = 0;
  int64_t n_cells = 0;
  double cell_m = 0, T_wall = 0;
  double* d_T = nullptr;
  double* d_x = nullptr;
  double* d_p = nullptr;
  std::vector<double> hT, hx, hp;  // host copies (the precision form's inputs)

  // lines + spectral grid
  bool have_lines = false;
  bool have_E = false;
  int n_nu = 0;
  int K = 0;
  double nu0 = 0, dnu = 0, T_ref = 0;
  rt::LineSet lines;
  double line_evals_per_cell = 0;

  // further absorbing gases (the outer sum over gases of Eq. (2)): gas g in
  // 1..kMaxGases-1 has its own line list on gas 0's spectral grid, cutoff
  // and T_ref, and its own mole fraction per cell
  rt::ExtraGas gas[rt::kMaxGases - 1];

  // adaptive line windows (RT_KAPPA_ADAPTIVE): tolerance (0 = not set),
  // per-cell sbar and partition ratio (FP64, [2][cells]) followed by the
  // screening's FP32 cell records (8 floats per cell),
  // window table
  // [run of cells][line] (owned) and the device count of kept evaluations
  // since the last reset
  double line_tol = 0;
  double* d_sbar = nullptr;
  int64_t sbar_cap = 0;
  uint32_t* d_win = nullptr;
  int64_t win_cap = 0;
  // windows the FP32 screening leaves to binary64: [0] count, then indices
  unsigned long long* d_und = nullptr;
  int64_t und_cap = 0;
  unsigned long long* d_adapt_evals = nullptr;

  // derived per-cell parameters and tables
  rt::CellSet cells;
  bool cells_valid = false;
  bool cells32_valid = false;  // the precision form's FP32 fields of `cells`
  bool have_kappa = false;
  float* kappa = nullptr;   // caller owned
  float* planck = nullptr;  // caller owned
  int64_t ld = 0;
  float* d_bwall = nullptr; // B(nu_j, T_wall), ld floats (owned)
  int64_t bwall_len = 0;

  // tallies (owned): fixed-point accumulator rows [n_cells + kBalRows][2][kAccDigits]
  // (rows from n_cells: entering, escaped) followed by the overflow flag; the
  // per-cell powers and the balance converted from them by rt_tally
  unsigned long long* d_acc = nullptr;
  unsigned* d_ovf = nullptr;
  double* d_abs = nullptr;
  double* d_emi = nullptr;
  double* d_balance = nullptr;
  unsigned long long* d_segcount = nullptr;

  // ray batch scratch (owned)
  int64_t batch_rays = 0;
  int max_segs = 0;
  int2* d_segs = nullptr;
  int32_t* d_counts = nullptr;
  int64_t* d_rays_explicit = nullptr;  // [n][6]: O(3), D(3)
  uint32_t* d_keys = nullptr;   // coherent-order key per batch ray
  uint32_t* d_perm = nullptr;   // batch slot -> ray offset in the batch
  uint32_t* d_hist = nullptr;   // [kOrderBuckets] counts, then offsets
  int64_t explicit_cap = 0;
  float* d_exit = nullptr;
  int64_t exit_cap = 0;

  void* noalloc_scratch = nullptr;  // this device's static scratch (rt_trace_rays_noalloc)

  rt::BatchPlan* batch = nullptr;  // prepared batched launch (owned)
  rt::Surrogate* surrogate = nullptr;  // learned form (owned)

  rt::Stats stats;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> trace_events, march_events, kappa_events,
      batch_events;
};

namespace rt {
// Fixed-point tally accumulators: kAccDigits digits of kAccBits bits, digit k
// worth 2^(kAccBits k + kAccLsb) W, each in a 64-bit word with room for the
// carries of 2^36 additions; a row holds the digits of the absorbed (or
// entering) and emitted (or escaped) power.
constexpr int kAccBits = 28;
constexpr int kAccDigits = 7;
constexpr int kAccLsb = -112;
constexpr int kAccRow = 2 * kAccDigits;
// terms one launch may add to one accumulator word (rays x spectral chunks)
constexpr int64_t kAccMaxTerms = int64_t(1) << 35;
// Balance rows (entering, escaped) per grid: rays spread over them so that
// their additions do not all meet in one accumulator.
constexpr int kBalRows = 1024;
// Coherent ray order: 6 dominant directions x 3 x 3 transverse direction
// bins x 64 x 64 positions on the mid-plane; used for batches of at least
// kOrderMinRays rays.
constexpr int kOrderBuckets = 6 * 9 * 4096;
constexpr int64_t kOrderMinRays = int64_t(1) << 15;

// kernel launchers (defined in the .hip files)
hipError_t launch_cell_params(rt_ctx c);
// per-cell factor G of extra gas g (after launch_cell_params' other tables)
hipError_t launch_gas_factor(rt_ctx c, int g);
hipError_t launch_kappa(rt_ctx c, bool compensated);
// the precision form's Gq per cell (gas 0 and every further gas), FP32
hipError_t launch_cell_params32(rt_ctx c);
// The paper's kappa formulation (16 tabulated points per line, multiply-adds
// only), every gas, into c->kappa.
hipError_t launch_kappa_table16(rt_ctx c);
// Adaptive line windows for gas 0 into c->kappa: per-cell band means, the
// window table (c->d_win, sized by the caller) and the windowed line sum;
// adds the kept evaluations to *c->d_adapt_evals.
hipError_t launch_kappa_adaptive(rt_ctx c);
// the Planck table (when c->planck is set) and the wall row, both evaluated in
// FP32 from the precision form's inputs
hipError_t launch_planck(rt_ctx c);
// the handle's own ray scratch (rt_trace_rays, rt_trace_explicit, rt_debug_segments)
RayScratch owned_rays(rt_ctx c);
hipError_t launch_raygen(rt_ctx c, const RayScratch& s, uint64_t seed, uint64_t begin,
                         int64_t count, bool explicit_rays, int64_t* rays_out, bool count_work,
                         const uint32_t* perm);
hipError_t launch_order(rt_ctx c, const RayScratch& s, uint64_t seed, uint64_t begin,
                        int64_t count);
// whether the plain march needs the second-order term of its Planck expansion
bool planck_needs_quadratic(double T_min, double T_max, double nu0, double dnu, int n_nu);
// FP32 arithmetic characterisation (arith.hip): operands each op reads (0 for
// an unknown op) and the element-wise launch.
int arith_operands(int op);
hipError_t launch_arith(rt_ctx c, int op, const float* a, const float* b, const float* z,
                        float* out, int64_t n);
hipError_t launch_march(rt_ctx c, const RayScratch& s, int64_t count, double weight, bool prec,
                        float* exit_dev);
hipError_t launch_tally(rt_ctx c);
hipError_t launch_zero(rt_ctx c);
void destroy_batch(rt_ctx c);
void free_surrogate(rt_ctx c);
rt_status surrogate_kappa(rt_ctx c);
bool surrogate_ready(rt_ctx c);
}  // namespace rt
