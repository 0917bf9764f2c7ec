// device_common.h -- device code shared by the single-case kernels and the
// persistent batched kernel (gfx950): the line-sum tile, Philox ray
// sampling, exact integer traversal, wavefront reductions and the march of
// one wavefront over one spectral chunk of one ray.
#pragma once

#include <type_traits>

#include "rt_internal.h"

namespace rt {
namespace dev {

constexpr int kKappaThreads = 256;
constexpr int kLineTile = 256;
constexpr int kKappaCells = 8;   // cells per lane in the line sum
constexpr int kKappaPoints = 2;  // nu points per lane in the line sum
constexpr int kKappaTilePoints = kKappaThreads * kKappaPoints;
constexpr int kQ = kChunk / 64;  // contiguous nu points per lane in the march

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// e^y for a double argument: range reduction y*log2(e) = n + f in FP64,
// |f| <= 1/2, then 2^f with the hardware base-2 exponential and an exact
// power-of-two scaling.  Error ~1.5e-7 relative over the whole range (the
// FP32 rounding of f contributes < 2.1e-8).
__device__ __forceinline__ float exp_split(double y) {
  double z = y * 1.4426950408889634074;
  double n = rint(z);
  float f = (float)(z - n);
  return ldexpf(fast_exp2(f), (int)n);
}

// 1 - e^{-x} for x >= 0 without cancellation: Taylor series of
// (1 - e^{-x})/x to degree 5 for x < 1/4 (truncation < 5e-8 relative),
// otherwise 1 - e^{-x} (the subtraction loses at most a factor 3.5).
__device__ __forceinline__ float one_minus_exp_neg_d(double x) {
  float xf = (float)x;
  if (xf < 0.25f) {
    float p = fmaf(xf, -1.0f / 720.0f, 1.0f / 120.0f);
    p = fmaf(xf, p, -1.0f / 24.0f);
    p = fmaf(xf, p, 1.0f / 6.0f);
    p = fmaf(xf, p, -0.5f);
    p = fmaf(xf, p, 1.0f);
    return xf * p;
  }
  return 1.0f - exp_split(-x);
}

// ------------------------------------------------- FP32 exponentials (pairs)
// The precision form evaluates every exponential in FP32.  An argument comes
// as an FP32 pair x = h + l (products of pairs keep about 46 bits, so the
// argument's own rounding does not limit the result), e^x is taken by Cody
// and Waite's range reduction with log2(e) split as L_h + L_l:
//   n = rint(h L_h),  f = fma(h, L_h, -n) + (h L_l + l L_h),  e^x = 2^n 2^f,
// |f| <= 1/2 + 2^-20, with the hardware base-2 exponential for 2^f (below
// one ulp) and an exact scaling by 2^n.  Relative error about 1e-7 for
// |x| < 80.
struct Pair {
  float h, l;
};

__device__ __forceinline__ Pair pair_of(float2 v) { return Pair{v.x, v.y}; }

// (a.h + a.l)(b.h + b.l) to about 2^-46 relative: the exact rounding error
// of a.h b.h (one FMA) plus the cross terms; a.l b.l is dropped.
__device__ __forceinline__ Pair pair_mul(Pair a, Pair b) {
  const float p = a.h * b.h;
  const float e = fmaf(a.h, b.l, fmaf(a.l, b.h, fmaf(a.h, b.h, -p)));
  return Pair{p, e};
}

__device__ __forceinline__ float exp_pair(Pair x) {
  constexpr float L_h = 1.44269502162933349609375f;  // log2(e) rounded to FP32
  constexpr float L_l = 1.925962989e-08f;             // log2(e) - L_h
  const float n = rintf(x.h * L_h);
  const float f = fmaf(x.h, L_h, -n) + fmaf(x.h, L_l, x.l * L_h);
  return ldexpf(__builtin_amdgcn_exp2f(f), (int)n);
}

// e^x - 1 for x >= 0: below 1/2 the Taylor series to degree 10 (truncation
// below 3e-10 relative) in Horner form, otherwise exp_pair(x) - 1 (the
// subtraction loses at most a factor e^(1/2)/(e^(1/2) - 1) = 2.5).
__device__ __forceinline__ float expm1_pair(Pair x) {
  if (x.h < 0.5f) {
    const float t = x.h + x.l;
    float p = 1.0f + t * (1.0f / 10.0f);
#pragma unroll
    for (int k = 9; k >= 2; --k) p = fmaf(t * (1.0f / (float)k), p, 1.0f);
    return t * p;
  }
  return exp_pair(x) - 1.0f;
}

// 1 - e^{-x} for x >= 0: the alternating series to degree 10 below 1/2,
// otherwise 1 - exp_pair(-x) (loses at most a factor 1/(1 - e^(-1/2)) = 2.5).
__device__ __forceinline__ float one_minus_exp_neg_pair(Pair x) {
  if (x.h < 0.5f) {
    const float t = x.h + x.l;
    float p = 1.0f - t * (1.0f / 10.0f);
#pragma unroll
    for (int k = 9; k >= 2; --k) p = fmaf(-t * (1.0f / (float)k), p, 1.0f);
    return t * p;
  }
  return 1.0f - exp_pair(Pair{-x.h, -x.l});
}

// nu_j = nu0 + j dnu as an FP32 pair, from the pairs of nu0 and dnu: the
// product j dnu.h with its exact rounding error (one FMA), then Knuth's
// TwoSum with nu0.h.
__device__ __forceinline__ Pair nu_at(int64_t j, Pair nu0, Pair dnu) {
  const float jf = (float)j;  // exact below 2^24
  const float ph = jf * dnu.h;
  const float pl = fmaf(jf, dnu.h, -ph) + jf * dnu.l;
  const float s = nu0.h + ph;
  const float bp = s - nu0.h;
  const float err = (nu0.h - (s - bp)) + (ph - bp);
  return Pair{s, err + pl + nu0.l};
}

// Eq. (4) in FP32: B = c1 nu^3 / expm1(theta nu), theta = c2 / T, with the
// argument theta nu formed as a pair product and expm1_pair.
__device__ __forceinline__ float planck_f32(Pair nu, Pair theta, float c1) {
  const float em1 = expm1_pair(pair_mul(nu, theta));
  const float v = nu.h + nu.l;
  return c1 * v * v * v / em1;
}

// Knuth's TwoSum: s + x = s' + err exactly.
__device__ __forceinline__ void two_sum_acc(float& s, float& comp, float x) {
  float t = s + x;
  float bp = t - s;
  float err = (s - (t - bp)) + (x - bp);
  s = t;
  comp += err;
}

// ------------------------------------------------------------ line records
// A staged line: (m, phi, lo, hi) -- the integer centre, the fraction, and
// the first and last offsets from m of the points the line contributes to
// -- then, per cell, (A, g2): the Lorentz amplitude u S s gamma / (pi dnu^2)
// and the squared half width (gamma/dnu)^2 in grid units, so that the line
// adds A / ((j - m - phi)^2 + g2) at point j.
constexpr int kLineRec = 4 + 2 * kKappaCells;  // floats per staged line

// The per-cell part of a record for line i and cell `cell` (Eqs. (1)-(2)).
__device__ __forceinline__ void line_cell_params(const LineSet& L, const CellSet& C, int i,
                                                 int64_t cell, int have_E, float& amp, float& g2) {
  const float gp = L.gamma[i] * C.P[cell] * fast_exp2(L.nexp[i] * C.lam2[cell]);
  float a = C.G[cell] * L.S[i] * gp;
  if (have_E) {
    a *= exp_split(L.E2[i] * C.beta[cell]);
    a *= one_minus_exp_neg_d(L.nu[i] * C.theta[cell]);
  }
  amp = a;
  g2 = gp * gp;
}

// The same record in FP32 only (the precision form): the Eq. (1) factors from
// the host-formed FP32 inputs with exp_pair, the half width's temperature
// power and the partition ratio (in Gq) with the hardware base-2 exponential.
__device__ __forceinline__ void line_cell_params_f32(const LineSet& L, const CellSet& C, int i,
                                                     int64_t cell, int have_E, float& amp,
                                                     float& g2) {
  const float gp = L.gamma[i] * C.Pf[cell] * fast_exp2(L.nexp[i] * C.lamf[cell]);
  float a = C.Gq[cell] * L.S[i] * gp;
  if (have_E) {
    a *= exp_pair(pair_mul(pair_of(L.E2p[i]), pair_of(C.beta2[cell])));
    a *= one_minus_exp_neg_pair(pair_mul(pair_of(L.nup[i]), pair_of(C.theta2[cell])));
  }
  amp = a;
  g2 = gp * gp;
}

// Adds one staged line to P points x kKappaCells cells of a lane: jf are the
// lane's points as floats.  FULL: every point is inside [m + lo, m + hi];
// otherwise a point outside gets an infinite offset, whose term is 0.
template <bool FULL, int P>
__device__ __forceinline__ void add_line_terms(const float* rec, const float (&jf)[P],
                                               float (&part)[P][kKappaCells]) {
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
#pragma unroll
  for (int c = 0; c < kKappaCells; c += 2) {
    const float4 ag = *reinterpret_cast<const float4*>(rec + 4 + 2 * c);
#pragma unroll
    for (int p = 0; p < P; ++p) {
      part[p][c] = fmaf(ag.x, fast_rcp(fmaf(dv[p], dv[p], ag.y)), part[p][c]);
      part[p][c + 1] = fmaf(ag.z, fast_rcp(fmaf(dv[p], dv[p], ag.w)), part[p][c + 1]);
    }
  }
}

// ------------------------------------------------------------ line sum tile
// Eq. (2) with the Eq. (1) strength ratio for one block: nu points
// [j0, j0 + 512) x kKappaCells cells starting at cell0.  Wave w owns the
// points j0 + 128 w + 64 p + lane (p < 2).  Lines whose window meets the
// block's points are staged kLineTile at a time as line records (m, phi,
// the window's offsets -K + [phi > 0] and K, and per cell the Lorentz
// amplitude A = u S s gamma / (pi dnu^2) and the squared half width
// g2 = (gamma/dnu)^2), so that a line adds
//   A / ((j - r_i)^2 + g2)
// to kappa at point j.  Grid units: line i sits at r_i = (nu_i - nu0)/dnu =
// m_i + phi_i with integer m_i; the offset j - r_i is the exact float
// difference (j - m_i) minus phi_i, so no absolute-wavenumber cancellation
// occurs in FP32.  Window membership is the integer range
// [m_i - K + [phi_i > 0], m_i + K], the exact form of |j - r_i| <= K.
// Output: out[(cell - 0) * ld_out + (j - col0)] for col0 <= j < col_end;
// points at or beyond n_nu are written as 0.  Must be called by all 256
// threads of the block; `lds` holds kLineTile * kLineRec floats.
struct KappaTile {
  LineSet L;
  CellSet C;          // per-cell factors of this grid (row 0 = its first cell)
  int64_t n_cells;
  int n_nu;
  int K;
  int have_E;
  float* out;
  int64_t ld_out;
  int64_t col0;
  int64_t col_end;
  const int32_t* cell_list = nullptr;  // logical cell i -> cell_list[i] when set
  int compact_rows = 0;                // with a list: write row i instead of cell_list[i]
  int accumulate = 0;                  // add to the row instead of storing (a further gas)
  // the block sums part line_part of line_parts equal shares of the lines
  // its points need (its output is then a partial sum of the row)
  int line_parts = 1;
  int line_part = 0;
};

// Optional device-side gating of a launch of line-sum tiles, decided per
// block before any barrier: a block runs if its group of cells is marked
// with the current epoch in group_flag, or if one of the width-chunk_w
// spectral chunks its tile touches has chunk_err above tol.
struct TileGate {
  const unsigned* group_flag = nullptr;
  unsigned epoch = 0;
  const float* chunk_err = nullptr;
  float tol = 0;
  int chunk_w = 0;
  int n_chunks = 0;
};

// F32: line records from line_cell_params_f32 (the precision form).
// active (uniform over the wavefront): false leaves this wavefront's points
// untouched; it still stages line records with the others.  P: points per
// lane (the tile is 256 P points); every point's sum runs over the same
// lines in the same order whatever P is, so the values do not depend on it.
template <bool COMP, bool F32 = false, int P = kKappaPoints>
__device__ void kappa_tile(const KappaTile& a, int j0, int64_t cell0, float* lds,
                           bool active = true) {
  constexpr int C = kKappaCells;
  constexpr int REC = kLineRec;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int span = 64 * P;
  const int wj0 = j0 + wave * span;

  const int nl = a.L.n;
  // line ranges of the block's points and of the wavefront's (both start
  // and end on 64-point spans)
  auto bound = [&](int b, int k) {  // field k of span b (all n past the table)
    return b < a.L.n_spans ? reinterpret_cast<const int*>(a.L.span4)[4 * b + k] : nl;
  };
  int blk_first = bound(j0 / 64, 0);
  int blk_end = bound((j0 + kKappaThreads * P - 1) / 64, 1);
  if (a.line_parts > 1) {
    const int share = (blk_end - blk_first + a.line_parts - 1) / a.line_parts;
    blk_first = min(blk_end, blk_first + a.line_part * share);
    blk_end = min(blk_end, blk_first + share);
  }
  const int wb0 = wj0 / 64, wb1 = (wj0 + span - 1) / 64;
  const int w_first = bound(wb0, 0);
  const int w_end = bound(wb1, 1);

  float jf[P];
#pragma unroll
  for (int p = 0; p < P; ++p) jf[p] = (float)(wj0 + 64 * p + lane);

  // windows are non-decreasing along the sorted list, so the lines whose
  // window covers [wj0, wj0 + span) are the contiguous range [f_first, f_end)
  const int f_first = bound(wb1, 2);
  const int f_end = bound(wb0, 3);

  float acc[P][C];
  float cmp[P][C];
#pragma unroll
  for (int p = 0; p < P; ++p)
#pragma unroll
    for (int c = 0; c < C; ++c) { acc[p][c] = 0.f; cmp[p][c] = 0.f; }

  // Adds lines [l0, l1) of the staged tile starting at line `base`.  FULL:
  // every point is inside the window.  Otherwise a point outside it gets an
  // infinite offset, whose reciprocal term is 0.  COMP: blocks of 16 lines
  // are summed plainly and folded into (acc, cmp) with TwoSum.
  auto sum_lines = [&](auto full_tag, int base, int l0, int l1) {
    constexpr bool FULL = decltype(full_tag)::value;
    for (int s0 = l0; s0 < l1;) {
      const int s1 = COMP ? min(s0 + 16, l1) : l1;
      float part[P][C];
#pragma unroll
      for (int p = 0; p < P; ++p)
#pragma unroll
        for (int c = 0; c < C; ++c) part[p][c] = COMP ? 0.f : acc[p][c];
      for (int l = s0; l < s1; ++l) add_line_terms<FULL, P>(lds + (l - base) * REC, jf, part);
#pragma unroll
      for (int p = 0; p < P; ++p)
#pragma unroll
        for (int c = 0; c < C; ++c) {
          if (COMP) two_sum_acc(acc[p][c], cmp[p][c], part[p][c]);
          else acc[p][c] = part[p][c];
        }
      s0 = s1;
    }
  };

  for (int base = blk_first; base < blk_end; base += kLineTile) {
    const int nt = min(kLineTile, blk_end - base);
    __syncthreads();
    for (int q = tid; q < nt * C; q += kKappaThreads) {
      const int li = q / C, cc = q % C;
      const int i = base + li;
      int64_t cell = cell0 + cc;
      if (cell >= a.n_cells) cell = a.n_cells - 1;
      if (a.cell_list) cell = a.cell_list[cell];
      float* rec = lds + li * REC;
      if (cc == 0) {
        rec[0] = (float)a.L.m[i];
        rec[1] = a.L.phi[i];
        rec[2] = (float)(a.L.wlo[i] - a.L.m[i]);  // -K + [phi > 0]
        rec[3] = (float)a.K;
      }
      if (F32)
        line_cell_params_f32(a.L, a.C, i, cell, a.have_E, rec[4 + 2 * cc], rec[5 + 2 * cc]);
      else
        line_cell_params(a.L, a.C, i, cell, a.have_E, rec[4 + 2 * cc], rec[5 + 2 * cc]);
    }
    __syncthreads();

    if (!active) continue;
    const int lb = max(base, w_first), le = min(base + nt, w_end);
    // lines [f_first, f_end) cover all of the wave's points: no membership test
    const int fb = min(le, max(lb, f_first)), fe = max(fb, min(le, f_end));
    sum_lines(std::false_type(), base, lb, fb);
    sum_lines(std::true_type(), base, fb, fe);
    sum_lines(std::false_type(), base, fe, le);
  }
  if (!active) return;

#pragma unroll
  for (int c = 0; c < C; ++c) {
    int64_t cell = cell0 + c;
    if (cell >= a.n_cells) break;
    if (a.cell_list && !a.compact_rows) cell = a.cell_list[cell];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int64_t j = wj0 + 64 * p + lane;
      if (j >= a.col0 && j < a.col_end) {
        const float v = COMP ? acc[p][c] + cmp[p][c] : acc[p][c];
        float* o = a.out + cell * a.ld_out + (j - a.col0);
        *o = (j < a.n_nu) ? (a.accumulate ? *o + v : v) : 0.f;
      }
    }
  }
}

// ------------------------------------------------------------ Philox4x64-10
// Salmon et al., SC'11: ten rounds of two 64x64->128 products by the round
// multipliers, high halves xored with the other words and the key, with a
// Weyl key bump between rounds.
__device__ __forceinline__ void philox4x64_10(uint64_t x[4], uint64_t k0, uint64_t k1) {
  const uint64_t m0 = 0xD2E7470EE14C6C93ULL, m1 = 0xCA5A826395121157ULL;
  const uint64_t w0 = 0x9E3779B97F4A7C15ULL, w1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t lo0 = m0 * x[0], hi0 = __umul64hi(m0, x[0]);
    const uint64_t lo1 = m1 * x[2], hi1 = __umul64hi(m1, x[2]);
    const uint64_t y0 = hi1 ^ x[1] ^ k0;
    const uint64_t y2 = hi0 ^ x[3] ^ k1;
    x[0] = y0; x[1] = lo1; x[2] = y2; x[3] = lo0;
    k0 += w0; k1 += w1;
  }
}

__device__ __forceinline__ int64_t isqrt64(int64_t v) {  // floor(sqrt(v)), v < 2^50
  int64_t s = (int64_t)sqrt((double)v);
  while (s * s > v) --s;
  while ((s + 1) * (s + 1) <= v) ++s;
  return s;
}

// Ray r of the set drawn with `seed`: key (seed, 1), counter (r, block, 0, 0).
// Block 0: word 0 picks the face with probability proportional to its area,
// words 1-2 the odd in-face fixed-point coordinates, word 3 the first disk
// candidate; blocks 1..15 give further candidates, four per block.  A
// candidate word gives two 21-bit signed integers (A, B), accepted when
// A^2 + B^2 < 2^40; the inward component is isqrt(2^40 - A^2 - B^2).
__device__ inline void sample_ray(uint64_t seed, uint64_t r, int nx, int ny, int nz,
                                  int64_t O[3], int64_t D[3]) {
  const int64_t n[3] = {nx, ny, nz};
  uint64_t w[4] = {r, 0, 0, 0};
  philox4x64_10(w, seed, 1);
  const uint64_t ax = (uint64_t)(ny) * nz, ay = (uint64_t)(nz) * nx, az = (uint64_t)(nx) * ny;
  const uint64_t total = 2 * (ax + ay + az);
  const uint64_t u = __umul64hi(w[0], total);
  int face;
  if (u < ax) face = 0;
  else if (u < 2 * ax) face = 1;
  else if (u < 2 * ax + ay) face = 2;
  else if (u < 2 * ax + 2 * ay) face = 3;
  else if (u < 2 * ax + 2 * ay + az) face = 4;
  else face = 5;
  const int axis = face >> 1, side = face & 1;
  const int t1 = (axis + 1) % 3, t2 = (axis + 2) % 3;
  O[axis] = side ? n[axis] * kCellUnits : 0;
  O[t1] = 2 * (int64_t)__umul64hi(w[1], (uint64_t)n[t1] << 20) + 1;
  O[t2] = 2 * (int64_t)__umul64hi(w[2], (uint64_t)n[t2] << 20) + 1;

  const int64_t R = int64_t(1) << 20, R2 = R * R, M21 = (int64_t(1) << 21) - 1;
  int64_t A = 0, B = 0;
  uint64_t cand = w[3];
  for (int k = 0; k < 61; ++k) {
    if (k > 0) {
      const int pos = (k - 1) & 3;
      if (pos == 0) {
        w[0] = r; w[1] = (uint64_t)(1 + ((k - 1) >> 2)); w[2] = 0; w[3] = 0;
        philox4x64_10(w, seed, 1);
      }
      cand = w[pos];
    }
    const int64_t a = (int64_t)(cand & (uint64_t)M21) - R;
    const int64_t b = (int64_t)((cand >> 21) & (uint64_t)M21) - R;
    if (a * a + b * b < R2) { A = a; B = b; break; }
  }
  const int64_t Cn = isqrt64(R2 - A * A - B * B);
  D[axis] = side ? -Cn : Cn;
  D[t1] = A;
  D[t2] = B;
}

// Incremental traversal with exact integer comparisons.  The parameter of
// the next plane along axis k is tnum_k / tden_k (tden_k = |D_k|); the
// smallest one is found by cross-multiplication, every axis reaching it
// steps at once (edges and corners are crossed in one step), and the
// segment length is the exact integer numerator of t_next - t_prev over
// its denominator, times |D| h / 2^21, rounded once to FP32.
__device__ inline int traverse(int nx, int ny, int nz, double unit_cm, const int64_t O[3],
                               const int64_t D[3], int max_segs, int2* out) {
  const int64_t n[3] = {nx, ny, nz};
  int64_t idx[3], tnum[3], tden[3];
  bool live[3];
  for (int k = 0; k < 3; ++k) {
    const int64_t q = O[k] / kCellUnits;  // O >= 0
    const bool on_plane = (O[k] % kCellUnits) == 0;
    idx[k] = (on_plane && D[k] < 0) ? q - 1 : q;
    live[k] = D[k] != 0;
    tden[k] = D[k] < 0 ? -D[k] : D[k];
    if (D[k] > 0) tnum[k] = (idx[k] + 1) * kCellUnits - O[k];
    else if (D[k] < 0) tnum[k] = O[k] - idx[k] * kCellUnits;
    else tnum[k] = 0;
  }
  const double dlen = sqrt((double)D[0] * (double)D[0] + (double)D[1] * (double)D[1] +
                           (double)D[2] * (double)D[2]);
  int64_t pnum = 0, pden = 1;
  int count = 0;
  while (idx[0] >= 0 && idx[0] < n[0] && idx[1] >= 0 && idx[1] < n[1] && idx[2] >= 0 &&
         idx[2] < n[2] && count < max_segs) {
    int m = -1;
    for (int k = 0; k < 3; ++k) {
      if (!live[k]) continue;
      if (m < 0 || tnum[k] * tden[m] < tnum[m] * tden[k]) m = k;
    }
    const int64_t mnum = tnum[m], mden = tden[m];
    const int64_t dnum = mnum * pden - pnum * mden;
    const int64_t dden = mden * pden;
    const double len = ((double)dnum / (double)dden) * dlen * unit_cm;
    const int cell = (int)(idx[0] + n[0] * (idx[1] + n[1] * idx[2]));
    out[count] = make_int2(cell, __float_as_int((float)len));
    ++count;
    for (int k = 0; k < 3; ++k) {
      if (live[k] && tnum[k] * mden == mnum * tden[k]) {
        idx[k] += D[k] > 0 ? 1 : -1;
        tnum[k] += kCellUnits;
      }
    }
    pnum = mnum;
    pden = mden;
  }
  return count;
}

// ------------------------------------------------------------ ray order
// Rays that run nearly parallel through nearby cells read the same kappa
// rows.  Marching them together (and on one XCD, see march_kernel) lets those
// rows be served from L2 instead of beyond it.  The key is the dominant axis
// and sign of D, a 3 x 3 bin of the two transverse direction ratios, and the
// Morton index (6 bits per axis) of the point where the ray's line crosses
// the grid's mid-plane normal to the dominant axis, over [-N, 2N] cells.
// The order changes only the order of the FP64 tally additions.
__device__ __forceinline__ uint32_t spread6(uint32_t v) {  // bits 0..5 -> even bits
  v = (v | (v << 4)) & 0x30fu;
  v = (v | (v << 2)) & 0x333u;
  v = (v | (v << 1)) & 0x555u;
  return v;
}

__device__ inline uint32_t order_key(const int64_t O[3], const int64_t D[3], int nx, int ny, int nz) {
  const int64_t n[3] = {nx, ny, nz};
  int ax = 0;
  for (int k = 1; k < 3; ++k)
    if (llabs(D[k]) > llabs(D[ax])) ax = k;
  const int a1 = ax == 2 ? 0 : ax + 1, a2 = ax == 0 ? 2 : ax - 1;
  const double dax = (double)D[ax];
  const double inv = 1.0 / fabs(dax);
  const int b1 = min(2, (int)(((double)D[a1] * inv + 1.0) * 1.5));
  const int b2 = min(2, (int)(((double)D[a2] * inv + 1.0) * 1.5));
  const double t = (0.5 * (double)(n[ax] * kCellUnits) - (double)O[ax]) / dax;
  const double N = (double)max(nx, max(ny, nz));
  const double scale = 64.0 / (3.0 * N * (double)kCellUnits);
  const double p1 = ((double)O[a1] + t * (double)D[a1] + N * kCellUnits) * scale;
  const double p2 = ((double)O[a2] + t * (double)D[a2] + N * kCellUnits) * scale;
  const uint32_t q1 = (uint32_t)fmin(63.0, fmax(0.0, p1));
  const uint32_t q2 = (uint32_t)fmin(63.0, fmax(0.0, p2));
  const uint32_t dir = (uint32_t)((ax * 2 + (D[ax] > 0)) * 9 + b1 * 3 + b2);
  return dir * 4096u + (spread6(q1) | (spread6(q2) << 1));
}

// ---------------------------------------------------- wavefront reductions
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, false));
}
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_f64(double v) {
  const int2 h = *reinterpret_cast<int2*>(&v);
  int2 r;
  r.x = __builtin_amdgcn_update_dpp(0, h.x, CTRL, ROW_MASK, 0xf, false);
  r.y = __builtin_amdgcn_update_dpp(0, h.y, CTRL, ROW_MASK, 0xf, false);
  return *reinterpret_cast<double*>(&r);
}

// a = 1 - e^{-tau} for tau >= 0, two accuracy levels.
//   precision form: degree-5 Taylor polynomial of (1 - e^{-tau})/tau below
//     tau = 1/4 (truncation < 5e-8), 1 - 2^{-tau log2 e} above (<= 5e-7);
//   plain form (in march_wave): the same series to tau^3 below tau = 1/32
//     (truncation < 1.3e-6), written in the exponent argument, and
//     1 - 2^{-tau log2 e} above (<= 1.5e-6 just above the switch, falling
//     as 1/tau); the series is skipped by the whole wavefront when no lane
//     needs it.
// The exponent is folded into base 2 per segment, as the paper's listing
// folds 1/ln 2 into the per-volume scalar.
__device__ __forceinline__ float poly5(float tau) {
  float p = fmaf(tau, -1.0f / 720.0f, 1.0f / 120.0f);
  p = fmaf(tau, p, -1.0f / 24.0f);
  p = fmaf(tau, p, 1.0f / 6.0f);
  p = fmaf(tau, p, -0.5f);
  p = fmaf(tau, p, 1.0f);
  return tau * p;
}

template <bool F64>
struct Partial { using T = float; };
template <>
struct Partial<true> { using T = double; };

template <int CTRL>
__device__ __forceinline__ float dpp_pt(float v) { return dpp_f32<CTRL>(v); }
template <int CTRL>
__device__ __forceinline__ double dpp_pt(double v) { return dpp_f64<CTRL>(v); }

// ------------------------------------------------------ fixed-point tallies
// The absorbed and emitted power of every cell, and the entering and escaped
// power of the balance, are kept as exact integers: kAccDigits digits of
// kAccBits bits, digit k worth 2^(kAccBits k + kAccLsb) W, each held in a
// 64-bit word whose upper bits take the carries of up to 2^35 additions
// until the words are normalised (after every launch).  A value is rounded to
// kAccSig significant bits (relative error below 2^-kAccSig), which then
// span at most two digits, and added with integer atomics; integer additions
// commute, so every tally comes out the same bit for bit whatever order the
// wavefronts deliver their sums in.  Values below 2^kAccLsb W are dropped
// (truncation, the same in every order); a value that is NaN, negative or
// not below 2^80 W sets the overflow flag instead.
constexpr int kAccSig = kAccBits + 1;
static_assert(kAccSig + kAccBits - 1 <= 2 * kAccBits, "a rounded value spans two digits");
static_assert((80 - kAccSig - kAccLsb) / kAccBits + 1 <= kAccDigits - 1, "values below 2^80 W fit");
constexpr unsigned long long kAccMask = (1ull << kAccBits) - 1;

__device__ __forceinline__ void acc_add(unsigned long long* d, double v, unsigned* ovf) {
  if (!(v >= 0.0 && v < 0x1p80)) {
    atomicOr(ovf, 1u);
    return;
  }
  if (v == 0.0) return;
  int e;
  const double mant = frexp(v, &e);  // v = mant 2^e, 1/2 <= mant < 1, e <= 80
  unsigned long long m = (unsigned long long)rint(ldexp(mant, kAccSig));
  if (m >> kAccSig) {                // rounded up to 2^kAccSig
    m >>= 1;
    ++e;
  }
  int p = e - kAccSig - kAccLsb;     // accumulator bit of m's lowest bit
  if (p < 0) {
    if (p <= -kAccSig) return;       // wholly below the lowest digit
    m >>= -p;
    p = 0;
  }
  const int k = p / kAccBits, s = p % kAccBits;
  const unsigned long long w = m << s;  // below 2^(2 kAccBits): digits k, k + 1
  atomicAdd(d + k, w & kAccMask);
  const unsigned long long hi = w >> kAccBits;
  if (hi) atomicAdd(d + k + 1, hi);
}

// Carries every digit's upper bits into the next digit.
__device__ __forceinline__ void acc_normalize(unsigned long long* d) {
  unsigned long long carry = 0;
#pragma unroll
  for (int k = 0; k < kAccDigits - 1; ++k) {
    const unsigned long long s = d[k] + carry;
    d[k] = s & kAccMask;
    carry = s >> kAccBits;
  }
  d[kAccDigits - 1] += carry;
}

// The value of normalised digits, summed from the top digit down.
__device__ __forceinline__ double acc_value(const unsigned long long* d) {
  double v = 0.0;
#pragma unroll
  for (int k = kAccDigits - 1; k >= 0; --k) v += ldexp((double)d[k], kAccBits * k + kAccLsb);
  return v;
}

// --------------------------------------------------------------- the march
// One wavefront, one ray, one chunk of kChunk points: Eq. (3) cell after cell
// for every point, I <- I - (I - B) a with a = 1 - e^{-tau}.  Each lane owns
// kQ contiguous points starting at the absolute index j.  Per segment every
// lane's partial sums of the chunk's absorbed (sum I a) and emitted (sum B a)
// radiance are staged in LDS; TallyStage<PREC>::kSegs segments at a time they
// are summed across the wavefront in a fixed order, weighted and added to the
// cells' fixed-point accumulators (tally_flush).  The ray's entering and
// escaped radiance over the chunk go the same way to the balance row.  PREC
// selects the precision form: Planck values from the table, the degree-5
// branch and FP64 partial sums.  Otherwise the Planck values of a lane's
// points come from one exact value at its first point nu_a and the
// second-order expansion of ln B:
//   B(nu_a + d) = B_a (1 + g1 d + (g1^2 + g2) d^2 / 2),
//   g1 = 3/nu - theta (1 + r),  g2 = -3/nu^2 + theta^2 r (1 + r),
//   theta = c2 / T,  r = 1 / (exp(theta nu) - 1);
// for d <= (kQ - 1) dnu the neglected terms are below 1e-9 relative.
struct MarchWave {
  const float* kappa;   // row c at kappa + c * ld, column j - col0
  const float* planck;  // same layout (precision form)
  int64_t ld;
  int64_t col0;
  const double* theta;  // c2 / T per cell (plain form)
  const float* bwall;   // B(nu_j, T_wall), indexed by absolute j
  double nu0, dnu, c1, weight;
  unsigned long long* acc;  // accumulator rows, kAccRow words each
  int64_t row0;             // row of cell 0
  int64_t bal_row0;         // first of the balance rows (entering, escaped)
  int bal_mask;             // balance rows - 1 (a power of two): a ray adds to
                            // row bal_row0 + (its slot & bal_mask)
  unsigned* ovf;            // set by acc_add for a value out of range
};

// Per-wavefront LDS staging of the per-segment partial sums: [kSegs][2][64].
template <bool PREC>
struct TallyStage {
  static constexpr int kSegs = PREC ? 4 : 8;
  static constexpr int kEntries = kSegs * 2 * 64;
};

// Adds np staged entries to the accumulators.  Entry s is segment k0 + s of
// the ray, or the ray's balance row bal_row once k0 + s reaches ns.  Value v = 2 s + q
// (q = 0 absorbed or entering, 1 emitted or escaped) is summed by
// 64 / (2 kSegs) lanes, each over a fixed run of the 64 partials, then across
// those lanes with DPP: the same order every time.
template <bool PREC>
__device__ __forceinline__ void tally_flush(const MarchWave& a,
                                            const typename Partial<PREC>::T* stage,
                                            const int2* sg, int ns, int k0, int np, int lane,
                                            int64_t bal_row) {
  using PT = typename Partial<PREC>::T;
  constexpr int V = 2 * TallyStage<PREC>::kSegs;
  constexpr int LPV = 64 / V;  // lanes per value
  constexpr int E = 64 / LPV;  // partials per lane
  static_assert(LPV == 4 || LPV == 8, "flush layout");
  __builtin_amdgcn_wave_barrier();
  // a flush runs once per kSegs segments: its lane-derived addresses are
  // formed here rather than hoisted and kept live across the march loop
  int ln = lane;
  asm volatile("" : "+v"(ln));
  const int v = ln / LPV, part = ln % LPV;
  const PT* src = stage + v * 64 + part * E;
  PT s = src[0];
#pragma unroll
  for (int i = 1; i < E; ++i) s += src[i];
  s += dpp_pt<0xB1>(s);  // quad_perm [1,0,3,2]
  s += dpp_pt<0x4E>(s);  // quad_perm [2,3,0,1]
  if (LPV == 8) s += dpp_pt<0x141>(s);  // row_half_mirror: the two quads of 8 lanes
  __builtin_amdgcn_wave_barrier();
  const int seg = v >> 1;
  if (part == 0 && seg < np) {
    const int k = k0 + seg;
    const int64_t row = k < ns ? a.row0 + sg[k].x : bal_row;
    acc_add(a.acc + row * kAccRow + (v & 1) * kAccDigits, (double)s * a.weight, a.ovf);
  }
}

// QUAD: keep the second-order term of the per-lane Planck expansion (plain
// form); the host drops it when its relative size over a lane's span is
// below FP32 unit roundoff for every cell temperature and wavenumber.
// stage: this wavefront's TallyStage<PREC>::kEntries LDS entries; slot: the
// ray's index in its launch, which picks its balance row.
template <bool PREC, bool EXIT, bool QUAD = true>
__device__ __forceinline__ void march_wave(const MarchWave& a, const int2* sg, int ns, int64_t j,
                                           int lane, float* exit_row,
                                           typename Partial<PREC>::T* stage, int64_t slot) {
  using PT = typename Partial<PREC>::T;
  constexpr int kSegs = TallyStage<PREC>::kSegs;
  const int64_t col = j - a.col0;
  float I[kQ];
#pragma unroll
  for (int h = 0; h < kQ / 4; ++h) {
    const float4 v = *reinterpret_cast<const float4*>(a.bwall + j + 4 * h);
    I[4 * h] = v.x; I[4 * h + 1] = v.y; I[4 * h + 2] = v.z; I[4 * h + 3] = v.w;
  }
  double nu_a = 0.0;
  float c1nu3 = 0.f, three_nu = 0.f, three_nu2 = 0.f;
  const float dnu_f = (float)a.dnu;
  if (!PREC) {
    nu_a = a.nu0 + (double)j * a.dnu;
    c1nu3 = (float)(a.c1 * nu_a * nu_a * nu_a);
    three_nu = (float)(3.0 / nu_a);
    three_nu2 = (float)(3.0 / (nu_a * nu_a));
  }
  PT enter = 0;
#pragma unroll
  for (int q = 0; q < kQ; ++q) enter += (PT)I[q];
  const float nlog2e = -1.4426950408889634f;
  int np = 0, k0 = 0;  // staged entries, and the segment of the first
  for (int k = 0; k < ns; ++k) {
    const int2 s = sg[k];
    const int64_t c = s.x;
    const float l = __int_as_float(s.y);
    const float xs = l * nlog2e;
    float kv[kQ], bv[kQ];
#pragma unroll
    for (int h = 0; h < kQ / 4; ++h) {
      const float4 v = *reinterpret_cast<const float4*>(a.kappa + c * a.ld + col + 4 * h);
      kv[4 * h] = v.x; kv[4 * h + 1] = v.y; kv[4 * h + 2] = v.z; kv[4 * h + 3] = v.w;
    }
    if (PREC) {
#pragma unroll
      for (int h = 0; h < kQ / 4; ++h) {
        const float4 v = *reinterpret_cast<const float4*>(a.planck + c * a.ld + col + 4 * h);
        bv[4 * h] = v.x; bv[4 * h + 1] = v.y; bv[4 * h + 2] = v.z; bv[4 * h + 3] = v.w;
      }
    } else {
      const double th = a.theta[c];  // c2 / T
      // exp(theta nu_a) with FP64 range reduction: 2^n 2^f, |f| <= 1/2
      const double z = th * 1.4426950408889634074 * nu_a;
      const double n = rint(z);
      const float f = (float)(z - n);
      const float e = ldexpf(__builtin_amdgcn_exp2f(f), (int)n);
      float em1 = e - 1.0f;
      if (__ballot(z < 0.36)) {  // theta nu < 1/4: expm1 by its series
        const float x = (float)(th * nu_a);
        float p = fmaf(x, 1.0f / 720.0f, 1.0f / 120.0f);
        p = fmaf(x, p, 1.0f / 24.0f);
        p = fmaf(x, p, 1.0f / 6.0f);
        p = fmaf(x, p, 0.5f);
        p = fmaf(x, p, 1.0f);
        if (z < 0.36) em1 = x * p;
      }
      const float r = __builtin_amdgcn_rcpf(em1);
      const float B0 = c1nu3 * r;
      const float thf = (float)th;
      const float t1 = 1.0f + r;
      const float g1 = fmaf(-thf, t1, three_nu);
      const float g2 = fmaf(thf * thf, r * t1, -three_nu2);
      const float K1 = B0 * g1 * dnu_f;
      if (QUAD) {
        const float K2 = 0.5f * B0 * fmaf(g1, g1, g2) * (dnu_f * dnu_f);
#pragma unroll
        for (int q = 0; q < kQ; ++q) bv[q] = fmaf(fmaf(K2, (float)q, K1), (float)q, B0);
      } else {
#pragma unroll
        for (int q = 0; q < kQ; ++q) bv[q] = fmaf(K1, (float)q, B0);
      }
    }
    // a = 1 - e^{-tau} per point
    float av[kQ];
    if (PREC) {
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const float tau = kv[q] * l;
        const float big = 1.0f - __builtin_amdgcn_exp2f(kv[q] * xs);
        av[q] = tau < 0.25f ? poly5(tau) : big;
      }
    } else {
      float kmin = kv[0];
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        av[q] = 1.0f - __builtin_amdgcn_exp2f(kv[q] * xs);
        kmin = fminf(kmin, kv[q]);
      }
      if (__ballot(kmin * l < 0.03125f)) {
        // some lane has tau < 1/32: there a = tau - tau^2/2 + tau^3/6 written
        // in x = -tau log2(e), i.e. a = -sum_k (x ln 2)^k / k!, k = 1..3
        // (truncation below tau^3/24 = 1.3e-6 relative); at tau >= 1/32 the
        // error of 1 - 2^x, about one unit in the last place of 2^x, is
        // below 1.5e-6 relative to a
        constexpr float L1 = -0.69314718055994531f, L2 = -0.24022650695910071f,
                        L3 = -0.055504108664821576f;
        constexpr float xlim = -0.03125f * 1.4426950408889634f;
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
          const float x = kv[q] * xs;
          const float ser = x * fmaf(x, fmaf(x, L3, L2), L1);
          av[q] = x > xlim ? ser : av[q];
        }
      }
    }
    PT ab = 0, em = 0;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      ab += (PT)(I[q] * av[q]);
      em += (PT)(bv[q] * av[q]);
      I[q] = fmaf(-(I[q] - bv[q]), av[q], I[q]);
    }
    // the update of I is complete here, so a[] dies before the staging and
    // the flush below (the scheduler would otherwise sink the updates past
    // them and keep a[] and B[] live across the flush)
#pragma unroll
    for (int q = 0; q < kQ; ++q) asm volatile("" ::"v"(I[q]));
    PT* st = stage + np * 128;
    st[lane] = ab;
    st[64 + lane] = em;
    if (++np == kSegs) {
      tally_flush<PREC>(a, stage, sg, ns, k0, np, lane, 0);
      k0 += np;
      np = 0;
    }
  }
  PT esc = 0;
#pragma unroll
  for (int q = 0; q < kQ; ++q) esc += (PT)I[q];
  if (EXIT) {
#pragma unroll
    for (int h = 0; h < kQ / 4; ++h)
      *reinterpret_cast<float4*>(exit_row + col + 4 * h) =
          make_float4(I[4 * h], I[4 * h + 1], I[4 * h + 2], I[4 * h + 3]);
  }
  // np < kSegs here: one more entry, the balance row's (entering, escaped)
  PT* st = stage + np * 128;
  st[lane] = enter;
  st[64 + lane] = esc;
  tally_flush<PREC>(a, stage, sg, ns, k0, np + 1, lane, a.bal_row0 + (slot & a.bal_mask));
}

}  // namespace dev

// Line-sum tiles [tile_begin, tile_begin + n_tiles) for n_cell_groups groups
// of kKappaCells cells (kappa.hip).
hipError_t launch_kappa_tiles(rt_ctx c, const dev::KappaTile& t, int64_t n_cell_groups,
                              int tile_begin, int n_tiles, bool comp, hipStream_t s,
                              const dev::TileGate& gate = dev::TileGate(), int parts = 1,
                              int64_t part_stride = 0);

}  // namespace rt
