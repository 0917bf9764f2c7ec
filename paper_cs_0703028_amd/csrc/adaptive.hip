// adaptive.hip -- adaptive line windows on gfx950: the paper's announced
// next version (its conclusion), in which the number of points evaluated per
// line follows the local temperature and the line's intensity.
//
//   adaptive_sbar_kernel   : per cell, sbar = sum_i S_i s_i / (n_nu dnu)
//                            (band mean of the untruncated line sum over the
//                            density) and the partition ratio q, in binary64
//   adaptive_window_kernel : per (run of 8 cells, line), the shared window
//                            [lo, hi] around m_i, packed as two 16-bit
//                            offsets, wherever FP32 bounds on the half width
//                            already fix it; counts the kept evaluations
//   adaptive_window_list_kernel, adaptive_window_scan_kernel : the rest, in
//                            binary64 (the screening lists them; the scan
//                            takes any the list had no room for)
//   kappa_adaptive_kernel  : the plain FP32 line sum of Eq. (2) over those
//                            windows.  A block stages only the lines whose
//                            kept window meets its 512 points; a wavefront
//                            sums its 128 points in passes (two of 64, or
//                            from eps = 3e-4 four of 32 with 4 cells per
//                            lane), each over the staged lines whose window
//                            meets it: first those covering all of its
//                            points (no membership test), then the rest
//   adaptive_wing_kernel   : (wing-return form, an extension) per cell, the
//                            Lorentz mass of the points its run's windows
//                            drop, priced by the midpoint rule and spread
//                            over the band as one constant that the line sum
//                            adds to every point
//
// A line keeps point j of cell c while its Lorentz value there is at least
// eps u_c sbar_c: |j - r_i| <= w_ci = sqrt(S s g / (pi eps sbar) - g^2)/dnu
// (no point when the root is imaginary).  The run's window is the widest of
// its cells', capped by the hard cutoff, and intersected with the plain
// window [m - K + [phi > 0], m + K].  The decision is taken in binary64, as
// in the definition: only the last bits of the exponentials and of the
// order of the strength ratio's operations can differ, and a window moves
// only if its half width lies within that of a grid point's distance.
#include <algorithm>

#include "adaptive.h"
#include "device_common.h"

namespace rt {
namespace {

using namespace dev;

static_assert(kKappaCells == RT_ADAPTIVE_GROUP, "a line-sum block holds one run of cells");
static_assert(kLineTile <= 256, "staged line indices are kept in bytes");

constexpr int kAdThreads = 256;
constexpr int kCellF = 8;  // floats per cell in the screening's cell record
constexpr int kAdRec = kLineRec;  // floats per staged line
// passes per wavefront of the windowed sum: two of 64 points (32^3 workload:
// 20.3 against 22.5 ms at eps = 1e-3, 71.0 against 70.1 ms at 1e-6)
constexpr int kAdPasses = 2;
// From this tolerance on, the windowed sum takes four passes of 32 points
// with 4 cells per lane: windows of a few tens of points (32^3 workload:
// 16.1 against 17.3 ms at eps = 1e-3, 11.7 against 12.7 at 1e-2 with the
// wing return; equal at 1e-4; 51.8 against 49.2 at 1e-5).
constexpr double kAdNarrowTol = 3e-4;

// Eq. (1) strength ratio in binary64: q exp(-c2 E/T) / exp(-c2 E/T_ref)
// * expm1(-c2 nu/T) / expm1(-c2 nu/T_ref), taken as
// q exp(c2 E (1/T_ref - 1/T)) expm1(-nu c2/T) / expm1(-c2 nu/T_ref) with the
// per-cell beta = 1/T_ref - 1/T, theta = c2/T and q = (T_ref/T)^1.5 and the
// per-line reciprocal of expm1(-c2 nu/T_ref): the same value in the same
// precision, one exponential and one expm1 per (cell, line).
__device__ inline double sratio64(const LineSet& L, int i, const CellSet& C, int64_t c, double q,
                                  int have_E) {
#pragma clang fp contract(off)
  if (!have_E) return 1.0;
  return q * exp(-L.aE[i] * C.beta[c]) * (expm1(-L.nu[i] * C.theta[c]) * L.rN[i]);
}

// Per cell: sbar = sum_i S_i s_ci / (n_nu dnu) (binary64, the lines in their
// sorted order), q = (T_ref/T)^1.5, and the screening's FP32 record of the
// cell (kCellF floats: 1/(pi eps sbar dnu), the factor that turns S s g / dnu
// into the screening's ratio in grid units, then q, 1/T_ref - 1/T, c2/T,
// log2(T_ref/T), p/dnu and sbar == 0).  Block 0 also clears the count of
// undecided windows.
__global__ __launch_bounds__(kAdThreads) void adaptive_sbar_kernel(LineSet L, CellSet C,
                                                                   const double* __restrict__ T,
                                                                   double T_ref, int have_E, double band,
                                                                   double pi_eps_dnu, int64_t n_cells,
                                                                   double* __restrict__ cellv,
                                                                   float* __restrict__ cellf,
                                                                   unsigned long long* __restrict__ und) {
#pragma clang fp contract(off)
  __shared__ double red[kAdThreads];
  const int64_t c = blockIdx.x;
  if (c == 0 && threadIdx.x == 0) *und = 0;
  const double q = have_E ? pow(T_ref / T[c], 1.5) : 1.0;
  double acc = 0.0;
  for (int i = threadIdx.x; i < L.n; i += kAdThreads) acc += L.S64[i] * sratio64(L, i, C, c, q, have_E);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = kAdThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double sb = red[0] / band;
    const double inv_den = 1.0 / (pi_eps_dnu * sb);
    cellv[c] = sb;
    cellv[n_cells + c] = q;
    float* f = cellf + kCellF * c;
    f[0] = (float)inv_den;
    f[1] = (float)q;
    f[2] = (float)C.beta[c];
    f[3] = (float)C.theta[c];
    f[4] = C.lam2[c];
    f[5] = C.P[c];
    f[6] = sb == 0.0 ? 1.f : 0.f;
    f[7] = 0.f;
  }
}

struct WindowArgs {
  LineSet L;
  CellSet C;
  const double* T;
  const double* p;
  const double* sbar;
  const double* q;
  const float* cellf;     // the screening's FP32 cell records
  int64_t n_cells;
  int64_t n_runs;
  int have_E;
  double T_ref, dnu, eps;
  int K, n_nu;
  uint32_t* win;
  unsigned long long* kept;
  unsigned long long* und;  // [0]: undecided count, [1 .. und_cap]: their indices
  int64_t und_cap;
};

// A window entry not decided by the screening pass (lo offset 32767 with hi
// offset -32768: no real window, whose offsets lie in [-K, K] with K <= 32767).
constexpr uint32_t kUndecided = 0x80007fffu;

// Half width in grid points of line i in cell c, -1 for none, in binary64.
__device__ inline double window_points(const WindowArgs& a, int i, int64_t c) {
#pragma clang fp contract(off)
  const double sb = a.sbar[c];
  if (sb == 0.0) return (double)a.K;
  const double Tc = a.T[c];
  const double s = sratio64(a.L, i, a.C, c, a.q[c], a.have_E);
  const double g = a.L.g64[i] * a.p[c] * pow(a.T_ref / Tc, a.L.n64[i]);
  const double num = a.L.S64[i] * s * g;
  const double den = M_PI * a.eps * sb;
  const double W2 = num / den - g * g;
  if (W2 < 0.0) return -1.0;
  return sqrt(W2) / a.dnu;
}

// Bounds [lo, hi] on window_points(a, i, c), in grid units, from FP32
// arithmetic: ratio = S s gp / (pi eps sbar dnu) and gp = g / dnu, so that
// w = sqrt(ratio - gp^2).  Every FP32 input is one rounding (6e-8) from its
// binary64 value and so is every product; v_exp_f32 is within 1 ulp (1.2e-7).
// Relative errors (y_b = c2 E (1/T_ref - 1/T), y_s = c2 nu / T,
// y_g = n log2(T_ref/T), each off by 1.8e-7 of itself):
//   exp(y_b): 4.3e-7 |y_b| + 1.2e-7 (the log2(e) scaling adds 6e-8 |y_b|);
//   1 - exp(-y_s): 5.5e-7 by its series below 1/4, else at most 3.5 times
//     the error of exp(-y_s) there, 6.3e-7, plus the subtraction: 7e-7;
//   2^y_g: 1.25e-7 |y_g| + 1.2e-7;
//   t = S / (1 - exp(-c2 nu/T_ref)) / (pi eps sbar dnu), q, gamma, p/dnu and
//   the six products: 6e-8 each.
// So ratio is within 1.5e-6 + 4.3e-7 |y_b| + 1.25e-7 |y_g| and gp^2 within
// 8e-7 + 2.5e-7 |y_g| of their exact values, W2 = ratio - gp^2 (one more
// rounding) within the larger sum times (ratio + gp^2); twice that is the
// bound used.  The square root (1 ulp) and the scalings are covered by the
// factors 1 -+ 1e-6.  -1 stands for "no point".  Returns false outside the
// ranges where this holds (then binary64 decides).
struct CellF {
  float inv_den, q, beta, theta, lam2, P;
  bool zero;
};

// One line's data for the screening, loaded once per thread and kept in
// registers over the runs it screens.
struct LineF {
  float S, E2, nu, nexp, gamma;
  double r;
  int wlo, whi, m;
};

__device__ inline LineF load_line(const WindowArgs& a, int i) {
  LineF ln;
  ln.S = a.L.S[i];
  ln.E2 = a.have_E ? (float)a.L.E2[i] : 0.f;
  ln.nu = a.have_E ? (float)a.L.nu[i] : 0.f;
  ln.nexp = a.L.nexp[i];
  ln.gamma = a.L.gamma[i];
  ln.r = a.L.r64[i];
  ln.wlo = a.L.wlo[i];
  ln.whi = a.L.whi[i];
  ln.m = a.L.m[i];
  return ln;
}

__device__ inline bool window_bounds(const WindowArgs& a, const LineF& ln, const CellF& cf, float& lo,
                                     float& hi) {
  if (cf.zero) {
    lo = hi = (float)a.K;
    return true;
  }
  const float S = ln.S;
  if (!(S == 0.f || S >= 1.2e-38f)) return false;       // normal or zero
  const float t = S * cf.inv_den;
  if (!(t < 1e30f)) return false;
  float s = 1.f, eb = 0.f;
  if (a.have_E) {
    const float yb = ln.E2 * cf.beta;                   // c2 E (1/T_ref - 1/T)
    const float ys = ln.nu * cf.theta;                  // c2 nu / T
    if (!(fabsf(yb) < 80.f) || !(ys < 80.f)) return false;
    const float boltz = fast_exp2(yb * 1.44269504f);
    float stim;
    if (ys < 0.25f) {
      float p = fmaf(ys, -1.0f / 720.0f, 1.0f / 120.0f);
      p = fmaf(ys, p, -1.0f / 24.0f);
      p = fmaf(ys, p, 1.0f / 6.0f);
      p = fmaf(ys, p, -0.5f);
      p = fmaf(ys, p, 1.0f);
      stim = ys * p;
    } else {
      stim = 1.0f - fast_exp2(-ys * 1.44269504f);
    }
    s = cf.q * boltz * stim;
    eb = fabsf(yb);
  }
  const float yg = ln.nexp * cf.lam2;                    // n log2(T_ref / T)
  if (!(fabsf(yg) < 16.f)) return false;
  const float gp = ln.gamma * cf.P * fast_exp2(yg);
  const float ratio = t * s * gp;
  const float g2 = gp * gp;
  const float W2 = ratio - g2;
  const float coef = 2.f * (1.5e-6f + 4.3e-7f * eb + 2.5e-7f * fabsf(yg));
  const float err = coef * (ratio + g2);
  if (!(ratio < 1e30f)) return false;
  // v_sqrt_f32 (within 1 ulp; a flushed denormal stays >= 0, which is all
  // the kept-point test uses of so small a half width)
  hi = W2 + err < 0.f ? -1.f : __builtin_amdgcn_sqrtf(W2 + err) * (1.f + 1e-6f);
  lo = W2 - err < 0.f ? -1.f : __builtin_amdgcn_sqrtf(W2 - err) * (1.f - 1e-6f);
  return true;
}

// The kept points of a line with half width hw: {j : |j - r| <= hw} (an
// interval, |j - r| growing away from r) within the plain window
// [wlo, whi].  The ends from the rounded r +- hw are off by at most one and
// are settled by the test itself.  False when empty.
__device__ inline bool kept_interval(double r, double hw, int wlo, int whi, int& lo, int& hi) {
  if (hw < 0.0) return false;
  auto in = [&](int j) { return fabs((double)j - r) <= hw; };
  int h = (int)floor(r + hw);
  if (in(h + 1)) ++h;
  else if (!in(h)) --h;
  int l = (int)ceil(r - hw);
  if (in(l - 1)) --l;
  else if (!in(l)) ++l;
  if (!(l <= h && in(l) && in(h))) return false;
  lo = l > wlo ? l : wlo;
  hi = h < whi ? h : whi;
  return lo <= hi;
}

// Packs the window and returns the kept in-grid evaluations of the run.
__device__ inline unsigned long long store_window(const WindowArgs& a, int64_t idx, int m,
                                                  bool any, int lo, int hi, int members) {
  int lo_off = 1, hi_off = 0;  // empty
  unsigned long long kept = 0;
  if (any) {
    lo_off = (int)(lo - m);
    hi_off = (int)(hi - m);
    const int g0 = lo > 0 ? lo : 0;
    const int g1 = hi < a.n_nu - 1 ? hi : a.n_nu - 1;
    if (g1 >= g0) kept = (unsigned long long)(g1 - g0 + 1) * (unsigned long long)members;
  }
  a.win[idx] = (uint32_t)(uint16_t)(int16_t)lo_off | ((uint32_t)(uint16_t)(int16_t)hi_off << 16);
  return kept;
}

__device__ inline void add_block_count(unsigned long long v, unsigned long long* total) {
  __shared__ unsigned long long red[kAdThreads];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int h = kAdThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0] != 0) atomicAdd(total, red[0]);
}

__device__ __forceinline__ int lanes_below(uint64_t mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Screening pass over (run, line): the run's half width lies between the
// largest lower and the largest upper bound of its cells; when the kept
// points are the same at both ends they are those of the binary64 value
// (the kept set grows with hw), else the entry is marked undecided and
// listed for the binary64 pass.  Block (x, y) takes lines 256 x .. 256 x +
// 255 of the runs y, y + gridDim.y, ...: the run, and so every cell
// quantity, is the same across a block.  Counts stay in registers and
// undecided indices are gathered in LDS, leaving a few global atomics per
// block (same-address atomics serialise in L2).
constexpr int kUndBuf = 1024;
__global__ __launch_bounds__(kAdThreads) void adaptive_window_kernel(WindowArgs a) {
  __shared__ unsigned long long ubuf[kUndBuf];
  __shared__ unsigned ucount;
  __shared__ unsigned long long ubase;
  const int nl = a.L.n;
  const int i = (int)blockIdx.x * kAdThreads + (int)threadIdx.x;
  if (threadIdx.x == 0) ucount = 0;
  __syncthreads();
  unsigned long long kept = 0;
  LineF ln{};
  if (i < nl) ln = load_line(a, i);
  auto flush = [&]() {
    __syncthreads();
    const unsigned n = ucount;
    if (n > 0) {
      if (threadIdx.x == 0) ubase = atomicAdd(a.und, (unsigned long long)n);
      __syncthreads();
      for (unsigned k = threadIdx.x; k < n; k += kAdThreads)
        if (ubase + k < (unsigned long long)a.und_cap) a.und[1 + ubase + k] = ubuf[k];
      __syncthreads();
      if (threadIdx.x == 0) ucount = 0;
    }
    __syncthreads();
  };
  for (int64_t run = blockIdx.y; run < a.n_runs; run += gridDim.y) {
    const int64_t c0 = run * RT_ADAPTIVE_GROUP;
    const int members = (int)min<int64_t>(RT_ADAPTIVE_GROUP, a.n_cells - c0);
    CellF cf[RT_ADAPTIVE_GROUP];
#pragma unroll
    for (int k = 0; k < RT_ADAPTIVE_GROUP; ++k) {
      const int64_t c = c0 + (k < members ? k : 0);
      const float4* f = reinterpret_cast<const float4*>(a.cellf + kCellF * c);
      const float4 f0 = f[0], f1 = f[1];
      cf[k].inv_den = f0.x;
      cf[k].q = f0.y;
      cf[k].beta = f0.z;
      cf[k].theta = f0.w;
      cf[k].lam2 = f1.x;
      cf[k].P = f1.y;
      cf[k].zero = f1.z != 0.f;
    }
    if (i < nl) {
      const int64_t idx = run * nl + i;
      float wl = -1.f, wu = -1.f;
      bool ok = true;
#pragma unroll
      for (int k = 0; k < RT_ADAPTIVE_GROUP; ++k) {
        if (k < members) {
          float l = -1.f, h = -1.f;
          ok = window_bounds(a, ln, cf[k], l, h) && ok;
          wl = fmaxf(wl, l);
          wu = fmaxf(wu, h);
        }
      }
      const double K = (double)a.K;
      int l0 = 0, h0 = 0, l1 = 0, h1 = 0;
      const bool e0 = ok && kept_interval(ln.r, fmin((double)wl, K), ln.wlo, ln.whi, l0, h0);
      const bool e1 = ok && kept_interval(ln.r, fmin((double)wu, K), ln.wlo, ln.whi, l1, h1);
      if (ok && e0 == e1 && (!e0 || (l0 == l1 && h0 == h1))) {
        kept += store_window(a, idx, ln.m, e0, l0, h0, members);
      } else {
        a.win[idx] = kUndecided;
        ubuf[atomicAdd(&ucount, 1u)] = (unsigned long long)idx;  // < kUndBuf: flushed below
      }
    }
    __syncthreads();
    if (ucount > (unsigned)(kUndBuf - kAdThreads)) flush();
  }
  flush();
  add_block_count(kept, a.kept);
}

// The binary64 decision of one undecided entry.
__device__ inline unsigned long long decide_exact(const WindowArgs& a, int64_t idx) {
#pragma clang fp contract(off)
  const int nl = a.L.n;
  const int64_t run = idx / nl;
  const int i = (int)(idx - run * nl);
  const int64_t c0 = run * RT_ADAPTIVE_GROUP;
  const int members = (int)min<int64_t>(RT_ADAPTIVE_GROUP, a.n_cells - c0);
  double w = -1.0;
  for (int k = 0; k < members; ++k) {
    const double wc = window_points(a, i, c0 + k);
    if (wc > w) w = wc;
  }
  const double hw = w < (double)a.K ? w : (double)a.K;
  int lo = 0, hi = 0;
  const bool any = kept_interval(a.L.r64[i], hw, a.L.wlo[i], a.L.whi[i], lo, hi);
  return store_window(a, idx, a.L.m[i], any, lo, hi, members);
}

// Binary64 pass over the listed undecided entries (grid-stride).
__global__ __launch_bounds__(kAdThreads) void adaptive_window_list_kernel(WindowArgs a) {
  const unsigned long long n = min(*a.und, (unsigned long long)a.und_cap);
  unsigned long long kept = 0;
  for (unsigned long long k = (unsigned long long)blockIdx.x * kAdThreads + threadIdx.x; k < n;
       k += (unsigned long long)gridDim.x * kAdThreads)
    kept += decide_exact(a, (int64_t)a.und[1 + k]);
  add_block_count(kept, a.kept);
}

// Entries beyond the list's capacity (none unless more than und_cap were
// undecided): a scan of the whole table, each block leaving at once when
// the list held them all.
__global__ __launch_bounds__(kAdThreads) void adaptive_window_scan_kernel(WindowArgs a) {
  if (*a.und <= (unsigned long long)a.und_cap) return;
  const int64_t idx = (int64_t)blockIdx.x * kAdThreads + threadIdx.x;
  unsigned long long kept = 0;
  if (idx < a.n_runs * a.L.n && a.win[idx] == kUndecided) kept = decide_exact(a, idx);
  add_block_count(kept, a.kept);
}

// Adds one staged line to P points x CPL cells of a lane: the cells
// cg CPL .. cg CPL + CPL - 1 of the run (their amplitudes and squared half
// widths sit at rec + 4 + 2 CPL cg).  As dev::add_line_terms otherwise.
template <bool FULL, int P, int CPL>
__device__ __forceinline__ void add_line_terms_cells(const float* rec, const float (&jf)[P], int cg,
                                                     float (&part)[P][CPL]) {
  const float4 h = *reinterpret_cast<const float4*>(rec);
  float dv[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const float t = jf[p] - h.x;
    const float d = t - h.y;
    if (FULL) {
      dv[p] = d;
    } else {
      const bool in = (t >= h.z) & (t <= h.w);
      dv[p] = in ? d : __builtin_inff();
    }
  }
  const float* ag = rec + 4 + 2 * CPL * cg;
#pragma unroll
  for (int c = 0; c < CPL; c += 2) {
    const float4 v = *reinterpret_cast<const float4*>(ag + 2 * c);
#pragma unroll
    for (int p = 0; p < P; ++p) {
      part[p][c] = fmaf(v.x, fast_rcp(fmaf(dv[p], dv[p], v.y)), part[p][c]);
      part[p][c + 1] = fmaf(v.z, fast_rcp(fmaf(dv[p], dv[p], v.w)), part[p][c + 1]);
    }
  }
}

// One block: points [j0, j0 + 512) of the run of 8 cells `run`, as the plain
// line-sum tile (dev::kappa_tile) with a window per (run, line): the staged
// line records (dev::kLineRec) carry the run's window offsets lo, hi.  Each
// wavefront owns 128 points and sums them in NQ passes: a pass lists only
// the staged lines whose window meets its points, so a narrow window costs
// the points of the passes it meets rather than all 128.  CPL = 8: a lane
// takes one point of a 64-point row for all 8 cells; CPL = 4: a half
// wavefront takes 32 points for 4 cells, which halves a pass's span for
// windows of a few tens of points.
template <int NQ, int CPL>
__global__ __launch_bounds__(kKappaThreads) __attribute__((amdgpu_waves_per_eu(6, 8))) void kappa_adaptive_kernel(KappaTile a,
                                                                       const uint32_t* __restrict__ win,
                                                                       int n_tiles,
                                                                       const double* __restrict__ wing) {
  constexpr int C = kKappaCells;
  constexpr int ROW = 64 * CPL / C;                 // points of a row of lanes
  constexpr int P = 64 * kKappaPoints / (ROW * NQ); // points per lane per pass
  static_assert(C % CPL == 0 && P * ROW * NQ == 64 * kKappaPoints, "passes split the wave's points evenly");
  __shared__ float4 lds4[kLineTile * kAdRec / 4];
  __shared__ uint8_t lists[kKappaThreads / 64][kLineTile];
  __shared__ int sel[kLineTile];
  __shared__ int wkeep[kKappaThreads / 64];
  static_assert(kLineTile == kKappaThreads, "one candidate line per thread");
  float* lds = reinterpret_cast<float*>(lds4);
  const int tile = blockIdx.x % n_tiles;
  const int64_t run = blockIdx.x / n_tiles;
  const int j0 = tile * kKappaTilePoints;
  const int64_t cell0 = run * C;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int pt = lane % ROW, cg = lane / ROW;       // point in the row, cell group
  const int span = ROW * P;                         // points of one pass
  const int wj0 = j0 + wave * 64 * kKappaPoints;
  const int nl = a.L.n;
  // the block's line range from the per-span table (tiles start and end on
  // 64-point spans)
  const int b0 = j0 / 64, b1 = (j0 + kKappaTilePoints - 1) / 64;
  const int* sp = reinterpret_cast<const int*>(a.L.span4);
  const int blk_first = b0 < a.L.n_spans ? sp[4 * b0] : nl;
  const int blk_end = b1 < a.L.n_spans ? sp[4 * b1 + 1] : nl;
  const uint32_t* wrow = win + run * (int64_t)nl;

  float jf[NQ][P];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int p = 0; p < P; ++p) jf[q][p] = (float)(wj0 + q * span + ROW * p + pt);
  float acc[NQ][P][CPL];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
      for (int c = 0; c < CPL; ++c) acc[q][p][c] = 0.f;

  for (int base = blk_first; base < blk_end; base += kLineTile) {
    // the candidates base .. base + 255 (hard window meets the block) whose
    // kept window meets the block's points, compacted in order: only they
    // are staged, so a narrow window costs no amplitude evaluations in the
    // blocks it misses
    const int nc = min(kLineTile, blk_end - base);
    bool keep = false;
    if (tid < nc) {
      const uint32_t w = wrow[base + tid];
      const int lo = (int16_t)(uint16_t)(w & 0xffffu), hi = (int16_t)(uint16_t)(w >> 16);
      const int m = a.L.m[base + tid];
      keep = lo <= hi && m + lo <= j0 + kKappaTilePoints - 1 && m + hi >= j0;
    }
    const uint64_t bk = __ballot(keep);
    __syncthreads();  // the previous tile's records, lists and selection read
    if (lane == 0) wkeep[wave] = __popcll(bk);
    __syncthreads();
    int off = 0, nt = 0;
#pragma unroll
    for (int v = 0; v < kKappaThreads / 64; ++v) {
      off += v < wave ? wkeep[v] : 0;
      nt += wkeep[v];
    }
    if (keep) sel[off + lanes_below(bk)] = base + tid;
    __syncthreads();
    if (nt == 0) continue;
    for (int q = tid; q < nt * C; q += kKappaThreads) {
      const int li = q / C, cc = q % C;
      const int i = sel[li];
      int64_t cell = cell0 + cc;
      if (cell >= a.n_cells) cell = a.n_cells - 1;
      float* rec = lds + li * kAdRec;
      if (cc == 0) {
        const uint32_t w = wrow[i];
        rec[0] = (float)a.L.m[i];
        rec[1] = a.L.phi[i];
        rec[2] = (float)(int16_t)(uint16_t)(w & 0xffffu);
        rec[3] = (float)(int16_t)(uint16_t)(w >> 16);
      }
      line_cell_params(a.L, a.C, i, cell, a.have_E, rec[4 + 2 * cc], rec[5 + 2 * cc]);
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int s0 = wj0 + q * span;
      __syncthreads();  // records staged; the previous pass's list read
      // this pass's lines: those whose window meets [s0, s0 + span); indices
      // of lines covering all of it from the front of the list, the others
      // from the back
      int nf = 0, np = 0;
      for (int l0 = 0; l0 < nt; l0 += 64) {
        const int l = l0 + lane;
        bool meet = false, full = false;
        if (l < nt) {
          const float4 h = *reinterpret_cast<const float4*>(lds + l * kAdRec);
          const int m = (int)h.x, w0 = m + (int)h.z, w1 = m + (int)h.w;
          meet = w0 <= w1 && w0 <= s0 + span - 1 && w1 >= s0;
          full = meet && w0 <= s0 && w1 >= s0 + span - 1;
        }
        const uint64_t bf = __ballot(full), bp = __ballot(meet && !full);
        if (full) lists[wave][nf + lanes_below(bf)] = (uint8_t)l;
        if (meet && !full) lists[wave][kLineTile - 1 - (np + lanes_below(bp))] = (uint8_t)l;
        nf += __popcll(bf);
        np += __popcll(bp);
      }
      __syncthreads();
      if constexpr (CPL == C) {
        for (int e = 0; e < nf; ++e) add_line_terms<true, P>(lds + lists[wave][e] * kAdRec, jf[q], acc[q]);
        for (int e = 0; e < np; ++e)
          add_line_terms<false, P>(lds + lists[wave][kLineTile - 1 - e] * kAdRec, jf[q], acc[q]);
      } else {
        for (int e = 0; e < nf; ++e)
          add_line_terms_cells<true, P, CPL>(lds + lists[wave][e] * kAdRec, jf[q], cg, acc[q]);
        for (int e = 0; e < np; ++e)
          add_line_terms_cells<false, P, CPL>(lds + lists[wave][kLineTile - 1 - e] * kAdRec, jf[q], cg,
                                              acc[q]);
      }
    }
  }

#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    const int64_t cell = cell0 + cg * CPL + c;
    if (cell >= a.n_cells) break;
    const float add = wing ? (float)wing[cell] : 0.f;
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int p = 0; p < P; ++p) {
        const int64_t j = wj0 + q * span + ROW * p + pt;
        if (j < a.ld_out) a.out[cell * a.ld_out + j] = (j < a.n_nu) ? acc[q][p][c] + add : 0.f;
      }
  }
}

// atan(x1 + d) - atan(x1), d > 0: when both ends have one sign, as
// atan(d / (1 + x1 (x1 + d))), which keeps the relative accuracy of a narrow
// span far out in a wing (two arctangents near +-pi/2 would cancel); across
// the centre the two arctangents have opposite signs and simply add.  The
// quotient takes the hardware reciprocal (within 1 ulp).
__device__ inline float atan_span(float x1, float d) {
  const float x2 = x1 + d;
  if (x1 >= 0.f || x2 <= 0.f) return atanf(d * __builtin_amdgcn_rcpf(fmaf(x1, x2, 1.f)));
  return atanf(x2) - atanf(x1);
}

// Wing return, one block per run of cells.  The points line i drops in the
// run are those of its plain window on the grid, [max(wlo, 0), min(whi,
// n_nu - 1)], outside the run's kept interval: at most two ranges, the same
// for the run's cells.  Range [a, b] of cell c carries, by the midpoint rule
// in grid units, amp_ci / g_ci (atan((b + 1/2 - r)/g) - atan((a - 1/2 -
// r)/g)), with amp_ci and g_ci (half width in grid points) those of the line
// sum.  Terms in FP32, sums in binary64; wing[c] = sum / n_nu.
__global__ __launch_bounds__(kAdThreads) void adaptive_wing_kernel(LineSet L, CellSet C,
                                                                  const uint32_t* __restrict__ win,
                                                                  int64_t n_cells, int n_nu,
                                                                  int have_E,
                                                                  double* __restrict__ wing) {
  constexpr int G = RT_ADAPTIVE_GROUP;
  __shared__ double red[G][kAdThreads];
  const int64_t run = blockIdx.x;
  const int64_t cell0 = run * G;
  const uint32_t* wrow = win + run * (int64_t)L.n;
  double acc[G];
#pragma unroll
  for (int c = 0; c < G; ++c) acc[c] = 0.0;
  for (int i = threadIdx.x; i < L.n; i += kAdThreads) {
    const int m = L.m[i];
    const uint32_t w = wrow[i];
    const int lo_off = (int16_t)(uint16_t)(w & 0xffffu), hi_off = (int16_t)(uint16_t)(w >> 16);
    const int h0 = max(L.wlo[i], 0), h1 = min(L.whi[i], n_nu - 1);
    const int k0 = max(m + lo_off, 0), k1 = min(m + hi_off, n_nu - 1);
    // dropped ranges (empty when a > b): the whole in-grid window when the
    // run keeps none of it, else what lies below and above the kept points
    int a0 = h0, b0 = h1, a1 = 1, b1 = 0;
    if (lo_off <= hi_off && k0 <= k1) {
      b0 = k0 - 1;
      a1 = k1 + 1;
      b1 = h1;
    }
    const bool r0 = a0 <= b0, r1 = a1 <= b1;
    if (!r0 && !r1) continue;
    const float phi = L.phi[i];
    // range ends' offsets from the centre r = m + phi, and the widths
    const float e0 = (float)(a0 - m) - 0.5f - phi, n0 = (float)(b0 - a0 + 1);
    const float e1 = (float)(a1 - m) - 0.5f - phi, n1 = (float)(b1 - a1 + 1);
#pragma unroll
    for (int c = 0; c < G; ++c) {
      const int64_t cell = cell0 + c < n_cells ? cell0 + c : n_cells - 1;
      float amp, g2;
      line_cell_params(L, C, i, cell, have_E, amp, g2);
      const float ig = __builtin_amdgcn_rsqf(g2);  // 1 / g, within 1 ulp
      float span = 0.f;
      if (r0) span += atan_span(e0 * ig, n0 * ig);
      if (r1) span += atan_span(e1 * ig, n1 * ig);
      acc[c] += (double)(amp * ig * span);
    }
  }
#pragma unroll
  for (int c = 0; c < G; ++c) red[c][threadIdx.x] = acc[c];
  __syncthreads();
  for (int h = kAdThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
#pragma unroll
      for (int c = 0; c < G; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + h];
    __syncthreads();
  }
  if ((int)threadIdx.x < G && cell0 + threadIdx.x < n_cells)
    wing[cell0 + threadIdx.x] = red[threadIdx.x][0] / (double)n_nu;
}

}  // namespace

static hipError_t launch_adaptive(rt_ctx c, bool wings) {
  const LineSet& L = c->lines;
  const int64_t runs = (c->n_cells + RT_ADAPTIVE_GROUP - 1) / RT_ADAPTIVE_GROUP;
  const int n_tiles = (int)((c->ld + kKappaTilePoints - 1) / kKappaTilePoints);
  const int64_t blocks = runs * n_tiles;
  const int64_t pairs = runs * (int64_t)L.n;
  const int64_t wblocks = (pairs + kAdThreads - 1) / kAdThreads;
  const int line_blocks = (L.n + kAdThreads - 1) / kAdThreads;
  const int64_t sblocks = runs * line_blocks;
  if (blocks > 0x7fffffffLL || wblocks > 0x7fffffffLL || sblocks > 0x7fffffffLL ||
      c->n_cells > 0x7fffffffLL)
    return hipErrorInvalidValue;
  double* cellv = c->d_sbar;  // [2][cells]: sbar, q; then the FP32 records
  float* cellf = reinterpret_cast<float*>(c->d_sbar + 2 * c->n_cells);
  hipLaunchKernelGGL(adaptive_sbar_kernel, dim3((unsigned)c->n_cells), dim3(kAdThreads), 0, c->stream,
                     L, c->cells, c->d_T, c->T_ref, c->have_E ? 1 : 0, (double)c->n_nu * c->dnu,
                     M_PI * c->line_tol * c->dnu, c->n_cells, cellv, cellf, c->d_und);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (pairs > 0) {
    WindowArgs w;
    w.L = L;
    w.C = c->cells;
    w.T = c->d_T;
    w.p = c->d_p;
    w.sbar = cellv;
    w.q = cellv + c->n_cells;
    w.cellf = cellf;
    w.n_cells = c->n_cells;
    w.n_runs = runs;
    w.have_E = c->have_E ? 1 : 0;
    w.T_ref = c->T_ref;
    w.dnu = c->dnu;
    w.eps = c->line_tol;
    w.K = c->K;
    w.n_nu = c->n_nu;
    w.win = c->d_win;
    w.kept = c->d_adapt_evals;
    w.und = c->d_und;
    w.und_cap = c->und_cap;
    const int64_t gy = std::min<int64_t>(runs, std::max<int64_t>(1, 4096 / line_blocks));
    hipLaunchKernelGGL(adaptive_window_kernel, dim3((unsigned)line_blocks, (unsigned)gy), dim3(kAdThreads),
                       0, c->stream, w);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t lblocks = std::min<int64_t>((c->und_cap + kAdThreads - 1) / kAdThreads, 4096);
    hipLaunchKernelGGL(adaptive_window_list_kernel, dim3((unsigned)lblocks), dim3(kAdThreads), 0,
                       c->stream, w);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(adaptive_window_scan_kernel, dim3((unsigned)wblocks), dim3(kAdThreads), 0,
                       c->stream, w);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  double* wing = nullptr;
  if (wings) {
    wing = adaptive_wing_constants(c);
    hipLaunchKernelGGL(adaptive_wing_kernel, dim3((unsigned)runs), dim3(kAdThreads), 0, c->stream, L,
                       c->cells, c->d_win, c->n_cells, c->n_nu, c->have_E ? 1 : 0, wing);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  KappaTile t;
  t.L = L;
  t.C = c->cells;
  t.n_cells = c->n_cells;
  t.n_nu = c->n_nu;
  t.K = c->K;
  t.have_E = c->have_E ? 1 : 0;
  t.out = c->kappa;
  t.ld_out = c->ld;
  t.col0 = 0;
  t.col_end = c->ld;
  if (c->line_tol >= kAdNarrowTol)
    hipLaunchKernelGGL((kappa_adaptive_kernel<4, 4>), dim3((unsigned)blocks), dim3(kKappaThreads), 0,
                       c->stream, t, c->d_win, n_tiles, wing);
  else
    hipLaunchKernelGGL((kappa_adaptive_kernel<kAdPasses, kKappaCells>), dim3((unsigned)blocks),
                       dim3(kKappaThreads), 0, c->stream, t, c->d_win, n_tiles, wing);
  return hipGetLastError();
}

hipError_t launch_kappa_adaptive(rt_ctx c) { return launch_adaptive(c, false); }

hipError_t launch_kappa_adaptive_wings(rt_ctx c) { return launch_adaptive(c, true); }

}  // namespace rt
