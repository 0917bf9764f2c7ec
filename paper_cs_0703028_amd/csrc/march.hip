// march.hip -- Monte-Carlo rays through the cell grid on gfx950.
//
//   raygen_dda : Philox4x64-10 ray sampling (uniform boundary point,
//                cosine-weighted inward direction) and exact integer
//                traversal -> per-ray list of (cell, length) segments
//   march      : Eq. (3) applied cell after cell for every nu point; each
//                wavefront owns one ray and a 512-point spectral chunk
//                (8 contiguous points per lane); per segment the absorbed
//                and emitted power of the chunk is combined across the
//                wavefront with DPP reductions and added to the cell's FP64
//                accumulator
//   tally      : deterministic FP64 reductions for the energy balance
#include "rt_internal.h"

namespace rt {
namespace {

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
__device__ void sample_ray(uint64_t seed, uint64_t r, int nx, int ny, int nz,
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
__device__ int traverse(int nx, int ny, int nz, double unit_cm, const int64_t O[3],
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

__global__ void raygen_dda_kernel(uint64_t seed, uint64_t begin, int64_t count, int nx, int ny,
                                  int nz, double unit_cm, int max_segs,
                                  const int64_t* __restrict__ explicit_rays, int64_t* rays_out,
                                  int2* segs, int32_t* counts, unsigned long long* seg_total) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int ns = 0;
  if (i < count) {
    int64_t O[3], D[3];
    if (explicit_rays) {
      for (int k = 0; k < 3; ++k) {
        O[k] = explicit_rays[6 * i + k];
        D[k] = explicit_rays[6 * i + 3 + k];
      }
    } else {
      sample_ray(seed, begin + (uint64_t)i, nx, ny, nz, O, D);
    }
    if (rays_out)
      for (int k = 0; k < 3; ++k) {
        rays_out[6 * i + k] = O[k];
        rays_out[6 * i + 3 + k] = D[k];
      }
    ns = traverse(nx, ny, nz, unit_cm, O, D, max_segs, segs + i * max_segs);
    counts[i] = ns;
  }
  // one atomic per wavefront for the work counter
  unsigned long long v = (unsigned long long)ns;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if (seg_total && (threadIdx.x & 63) == 0 && v) atomicAdd(seg_total, v);
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

// Sum over the 64 lanes: butterflies inside each row of 16 (quad
// permutations, half-row and row mirrors), then the row totals are combined
// with the row broadcasts; lane 63 ends with the total, which is returned
// to every lane.  Disabled rows receive 0, so the adds are no-ops there.
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_f32<0xB1>(v);        // quad_perm [1,0,3,2]
  v += dpp_f32<0x4E>(v);        // quad_perm [2,3,0,1]
  v += dpp_f32<0x141>(v);       // row_half_mirror
  v += dpp_f32<0x140>(v);       // row_mirror
  v += dpp_f32<0x142, 0xA>(v);  // row_bcast:15 -> rows 1, 3
  v += dpp_f32<0x143, 0xC>(v);  // row_bcast:31 -> rows 2, 3
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xB1>(v);
  v += dpp_f64<0x4E>(v);
  v += dpp_f64<0x141>(v);
  v += dpp_f64<0x140>(v);
  v += dpp_f64<0x142, 0xA>(v);
  v += dpp_f64<0x143, 0xC>(v);
  int2 h = *reinterpret_cast<int2*>(&v);
  int2 r;
  r.x = __builtin_amdgcn_readlane(h.x, 63);
  r.y = __builtin_amdgcn_readlane(h.y, 63);
  return *reinterpret_cast<double*>(&r);
}

// a = 1 - e^{-tau} for tau >= 0, two accuracy levels.
//   precision form: degree-5 Taylor polynomial of (1 - e^{-tau})/tau below
//     tau = 1/4 (truncation < 5e-8), 1 - 2^{-tau log2 e} above (<= 5e-7);
//   plain form: degree-3 polynomial below tau = 1/16 (truncation < 1.3e-7),
//     1 - 2^{-tau log2 e} above (<= 2e-6 just above the switch, falling as
//     1/tau), and the polynomial is skipped by the whole wavefront when no
//     lane needs it.
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
__device__ __forceinline__ float poly3(float tau) {
  float p = fmaf(tau, -1.0f / 24.0f, 1.0f / 6.0f);
  p = fmaf(tau, p, -0.5f);
  p = fmaf(tau, p, 1.0f);
  return tau * p;
}

struct MarchArgs {
  const float* kappa;
  const float* planck;   // precision form only
  const double* theta;   // plain form: c2 / T per cell
  const float* bwall;
  int64_t ld;
  int n_chunks;
  int64_t ray_blocks;
  const int2* segs;
  const int32_t* counts;
  int max_segs;
  int64_t n_rays;
  double weight;
  double nu0, dnu, c1;
  double* acc_abs;
  double* acc_emi;
  double* slots;
  float* exit_I;
};

template <bool F64>
struct Partial { using T = float; };
template <>
struct Partial<true> { using T = double; };

constexpr int kQ = kChunk / 64;  // contiguous nu points per lane

// Block = 4 wavefronts = 4 consecutive rays on one spectral chunk; blocks run
// chunk-major so that the waves in flight share kappa[:, chunk].  Each lane
// owns kQ contiguous points.  PREC selects the precision form: Planck values
// from the FP64-derived table, the degree-5 branch and FP64 partial sums;
// otherwise the Planck values are formed in registers (one exponential and
// one reciprocal per lane and segment), which halves the table traffic.
template <bool PREC, bool EXIT>
__global__ __launch_bounds__(256) void march_kernel(MarchArgs a) {
  using PT = typename Partial<PREC>::T;
  const int64_t b = blockIdx.x;
  const int chunk = (int)(b / a.ray_blocks);
  const int64_t rb = b % a.ray_blocks;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t ray = rb * 4 + wave;
  if (ray >= a.n_rays) return;
  const int64_t j = (int64_t)chunk * kChunk + lane * kQ;

  float I[kQ];
#pragma unroll
  for (int h = 0; h < kQ / 4; ++h) {
    const float4 v = *reinterpret_cast<const float4*>(a.bwall + j + 4 * h);
    I[4 * h] = v.x; I[4 * h + 1] = v.y; I[4 * h + 2] = v.z; I[4 * h + 3] = v.w;
  }
  // plain form: Planck values of the lane's kQ points from one exact value
  // at its first point nu_a and the second-order expansion of ln B:
  //   B(nu_a + d) = B_a (1 + g1 d + (g1^2 + g2) d^2 / 2),
  //   g1 = 3/nu - theta (1 + r),  g2 = -3/nu^2 + theta^2 r (1 + r),
  //   theta = c2 / T,  r = 1 / (exp(theta nu) - 1);
  // for d <= (kQ - 1) dnu the neglected terms are below 1e-9 relative.
  double nu_a = 0.0;
  float c1nu3 = 0.f, three_nu = 0.f, three_nu2 = 0.f;
  const float dnu_f = (float)a.dnu;
  if (!PREC) {
    nu_a = a.nu0 + (double)j * a.dnu;
    c1nu3 = (float)(a.c1 * nu_a * nu_a * nu_a);
    three_nu = (float)(3.0 / nu_a);
    three_nu2 = (float)(3.0 / (nu_a * nu_a));
  }
  float enter = 0.f;
#pragma unroll
  for (int q = 0; q < kQ; ++q) enter += I[q];
  const int ns = a.counts[ray];
  const int2* sg = a.segs + ray * a.max_segs;
  const float nlog2e = -1.4426950408889634f;
  for (int k = 0; k < ns; ++k) {
    const int2 s = sg[k];
    const int64_t c = s.x;
    const float l = __int_as_float(s.y);
    const float xs = l * nlog2e;
    float kv[kQ], bv[kQ];
#pragma unroll
    for (int h = 0; h < kQ / 4; ++h) {
      const float4 v = *reinterpret_cast<const float4*>(a.kappa + c * a.ld + j + 4 * h);
      kv[4 * h] = v.x; kv[4 * h + 1] = v.y; kv[4 * h + 2] = v.z; kv[4 * h + 3] = v.w;
    }
    if (PREC) {
#pragma unroll
      for (int h = 0; h < kQ / 4; ++h) {
        const float4 v = *reinterpret_cast<const float4*>(a.planck + c * a.ld + j + 4 * h);
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
      const float K2 = 0.5f * B0 * fmaf(g1, g1, g2) * (dnu_f * dnu_f);
#pragma unroll
      for (int q = 0; q < kQ; ++q) bv[q] = fmaf(fmaf(K2, (float)q, K1), (float)q, B0);
    }
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
      if (__ballot(kmin * l < 0.0625f)) {
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
          const float tau = kv[q] * l;
          av[q] = tau < 0.0625f ? poly3(tau) : av[q];
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
    const PT tab = wave_sum(ab);
    const PT tem = wave_sum(em);
    if (lane == 0) {
      unsafeAtomicAdd(a.acc_abs + c, a.weight * (double)tab);
      unsafeAtomicAdd(a.acc_emi + c, a.weight * (double)tem);
    }
  }
  float esc = 0.f;
#pragma unroll
  for (int q = 0; q < kQ; ++q) esc += I[q];
  if (EXIT) {
#pragma unroll
    for (int h = 0; h < kQ / 4; ++h)
      *reinterpret_cast<float4*>(a.exit_I + ray * a.ld + j + 4 * h) =
          make_float4(I[4 * h], I[4 * h + 1], I[4 * h + 2], I[4 * h + 3]);
  }
  const PT te = wave_sum((PT)enter);
  const PT tx = wave_sum((PT)esc);
  if (lane == 0) {
    const int slot = (int)(b % kSlots);
    unsafeAtomicAdd(a.slots + slot, a.weight * (double)te);
    unsafeAtomicAdd(a.slots + kSlots + slot, a.weight * (double)tx);
  }
}

// Deterministic FP64 sums: balance = {entering, sum emitted, sum absorbed,
// escaped}; fixed strided partial sums then a fixed tree.
__global__ __launch_bounds__(1024) void tally_kernel(const double* __restrict__ abs_,
                                                     const double* __restrict__ emi,
                                                     int64_t n_cells,
                                                     const double* __restrict__ slots,
                                                     double* balance) {
  __shared__ double red[4][1024];
  const int t = threadIdx.x;
  double s_abs = 0, s_emi = 0;
  for (int64_t c = t; c < n_cells; c += 1024) { s_abs += abs_[c]; s_emi += emi[c]; }
  red[0][t] = slots[t];
  red[1][t] = s_emi;
  red[2][t] = s_abs;
  red[3][t] = slots[kSlots + t];
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (t < off)
      for (int q = 0; q < 4; ++q) red[q][t] += red[q][t + off];
    __syncthreads();
  }
  if (t < 4) balance[t] = red[t][0];
}

__global__ void zero_f64_kernel(double* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

}  // namespace

static_assert(kSlots == 1024, "tally kernel assumes 1024 slots");

hipError_t launch_raygen(rt_ctx c, uint64_t seed, uint64_t begin, int64_t count,
                         bool explicit_rays, int64_t* rays_out, bool count_work) {
  const int threads = 256;
  const int64_t blocks = (count + threads - 1) / threads;
  const double unit_cm = c->cell_m * 100.0 / (double)kCellUnits;
  hipLaunchKernelGGL(raygen_dda_kernel, dim3((unsigned)blocks), dim3(threads), 0, c->stream,
                     seed, begin, count, c->nx, c->ny, c->nz, unit_cm, c->max_segs,
                     explicit_rays ? c->d_rays_explicit : nullptr, rays_out, c->d_segs,
                     c->d_counts, count_work ? c->d_segcount : nullptr);
  return hipGetLastError();
}

hipError_t launch_march(rt_ctx c, int64_t count, double weight, bool prec, float* exit_dev) {
  MarchArgs a;
  a.kappa = c->kappa;
  a.planck = c->planck;
  a.theta = c->cells.theta;
  a.bwall = c->d_bwall;
  a.ld = c->ld;
  a.n_chunks = (int)(c->ld / kChunk);
  a.ray_blocks = (count + 3) / 4;
  a.segs = c->d_segs;
  a.counts = c->d_counts;
  a.max_segs = c->max_segs;
  a.n_rays = count;
  a.weight = weight;
  a.nu0 = c->nu0;
  a.dnu = c->dnu;
  a.c1 = first_radiation_wavenumber();
  a.acc_abs = c->d_abs;
  a.acc_emi = c->d_emi;
  a.slots = c->d_slots;
  a.exit_I = exit_dev;
  const int64_t blocks = a.ray_blocks * a.n_chunks;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 g((unsigned)blocks), t(256);
  if (prec) {
    if (exit_dev) hipLaunchKernelGGL((march_kernel<true, true>), g, t, 0, c->stream, a);
    else hipLaunchKernelGGL((march_kernel<true, false>), g, t, 0, c->stream, a);
  } else {
    if (exit_dev) hipLaunchKernelGGL((march_kernel<false, true>), g, t, 0, c->stream, a);
    else hipLaunchKernelGGL((march_kernel<false, false>), g, t, 0, c->stream, a);
  }
  return hipGetLastError();
}

hipError_t launch_tally(rt_ctx c) {
  hipLaunchKernelGGL(tally_kernel, dim3(1), dim3(1024), 0, c->stream, c->d_abs, c->d_emi,
                     c->n_cells, c->d_slots, c->d_balance);
  return hipGetLastError();
}

hipError_t launch_zero(rt_ctx c) {
  auto z = [&](double* p, int64_t n) {
    hipLaunchKernelGGL(zero_f64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       c->stream, p, n);
  };
  z(c->d_abs, c->n_cells);
  z(c->d_emi, c->n_cells);
  z(c->d_slots, 2 * kSlots);
  z(c->d_balance, 4);
  z(reinterpret_cast<double*>(c->d_segcount), 1);
  return hipGetLastError();
}

}  // namespace rt
