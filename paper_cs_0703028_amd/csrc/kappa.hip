// kappa.hip -- per-cell spectral properties on gfx950.
//
//   cell_params   : per-cell gas state -> FP32/FP64 factors (FP64 arithmetic)
//   kappa_linesum : Eq. (2) with the Eq. (1) strength ratio, Lorentz lines on
//                   the uniform nu grid with an inclusive hard cutoff; line
//                   tiles are staged in LDS, every lane owns P nu points of
//                   C cells and writes kappa coalesced along nu
//   planck_table  : Eq. (4), wavenumber form, per (cell, nu) and for the walls
//
// Grid units: a line i sits at r_i = (nu_i - nu0)/dnu = m_i + phi_i with
// integer m_i; for grid point j the offset j - r_i is formed as the exact
// float difference (j - m_i) minus phi_i, so no absolute-wavenumber
// cancellation occurs in FP32.  Window membership is the integer range
// [m_i - K + [phi_i > 0], m_i + K], the exact form of |j - r_i| <= K.
#include "rt_internal.h"

namespace rt {
namespace {

constexpr int kKappaThreads = 256;
constexpr int kLineTile = 256;

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

// ---------------------------------------------------------------- cells
// u = x p / (k_B T) [cm^-3]; q = (T_ref/T)^1.5 (partition-function ratio of
// Eq. (1)); G = u q / (pi dnu) with energies, u / (pi dnu) without.
__global__ void cell_params_kernel(int64_t n, const double* __restrict__ T,
                                   const double* __restrict__ x,
                                   const double* __restrict__ p, double T_ref,
                                   double dnu, double c2, int have_E,
                                   float* G, double* beta, double* theta,
                                   float* lam2, float* P, float* theta2) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  double Tc = T[c];
  double u = x[c] * p[c] * kAtm / (kBoltzmann * Tc) * 1e-6;
  double q = have_E ? pow(T_ref / Tc, 1.5) : 1.0;
  G[c] = (float)(u * q / (M_PI * dnu));
  beta[c] = 1.0 / T_ref - 1.0 / Tc;
  theta[c] = c2 / Tc;
  lam2[c] = (float)log2(T_ref / Tc);
  P[c] = (float)(p[c] / dnu);
  theta2[c] = (float)(c2 / Tc * 1.4426950408889634074);
}

__device__ __forceinline__ int first_ge(const int32_t* a, int n, int v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] >= v) hi = mid; else lo = mid + 1;
  }
  return lo;
}
__device__ __forceinline__ int first_gt(const int32_t* a, int n, int v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] > v) hi = mid; else lo = mid + 1;
  }
  return lo;
}

// Knuth's TwoSum: s + x = s' + err exactly.
__device__ __forceinline__ void two_sum_acc(float& s, float& comp, float x) {
  float t = s + x;
  float bp = t - s;
  float err = (s - (t - bp)) + (x - bp);
  s = t;
  comp += err;
}

struct KappaArgs {
  LineSet L;
  CellSet C;
  int64_t n_cells;
  int n_nu;
  int64_t ld;
  int K;
  int have_E;
  int n_tiles;
  float* out;
};

// One block: nu tile of 256*P points x C cells.  Wave w owns the points
// j0 + 64*P*w + 64*p + lane (p < P).  Lines whose window meets the block's
// tile are staged kLineTile at a time: per line (m, phi, window start) and,
// per cell, the Lorentz amplitude A = u S s gamma / (pi dnu^2) and the
// squared half width g2 = (gamma/dnu)^2, so that a line adds
//   A / ((j - r_i)^2 + g2)
// to kappa at point j.
template <int C, int P, bool COMP>
__global__ __launch_bounds__(kKappaThreads) void kappa_linesum_kernel(KappaArgs a) {
  constexpr int REC = 4 + 2 * C;  // floats per staged line
  __shared__ float4 lds4[kLineTile * REC / 4];
  float* lds = reinterpret_cast<float*>(lds4);

  const int tile = blockIdx.x % a.n_tiles;
  const int64_t cg = blockIdx.x / a.n_tiles;
  const int64_t cell0 = cg * C;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int span = 64 * P;
  const int j0 = tile * kKappaThreads * P;
  const int wj0 = j0 + wave * span;

  const int nl = a.L.n;
  const int blk_first = first_ge(a.L.whi, nl, j0);
  const int blk_end = first_gt(a.L.wlo, nl, j0 + kKappaThreads * P - 1);
  const int w_first = first_ge(a.L.whi, nl, wj0);
  const int w_end = first_gt(a.L.wlo, nl, wj0 + span - 1);

  float jf[P];
#pragma unroll
  for (int p = 0; p < P; ++p) jf[p] = (float)(wj0 + 64 * p + lane);
  const float Kf = (float)a.K;

  float acc[P][C];
  float cmp[P][C];
#pragma unroll
  for (int p = 0; p < P; ++p)
#pragma unroll
    for (int c = 0; c < C; ++c) { acc[p][c] = 0.f; cmp[p][c] = 0.f; }

  // per-cell factors for the staging threads
  for (int base = blk_first; base < blk_end; base += kLineTile) {
    const int nt = min(kLineTile, blk_end - base);
    __syncthreads();
    for (int q = tid; q < nt * C; q += kKappaThreads) {
      const int li = q / C, cc = q % C;
      const int i = base + li;
      int64_t cell = cell0 + cc;
      if (cell >= a.n_cells) cell = a.n_cells - 1;
      float* rec = lds + li * REC;
      if (cc == 0) {
        rec[0] = (float)a.L.m[i];
        rec[1] = a.L.phi[i];
        rec[2] = (float)(a.L.wlo[i] - a.L.m[i]);  // -K + [phi > 0]
        rec[3] = 0.f;
      }
      const float gp = a.L.gamma[i] * a.C.P[cell] * fast_exp2(a.L.nexp[i] * a.C.lam2[cell]);
      float amp = a.C.G[cell] * a.L.S[i] * gp;
      if (a.have_E) {
        amp *= exp_split(a.L.E2[i] * a.C.beta[cell]);
        amp *= one_minus_exp_neg_d(a.L.nu[i] * a.C.theta[cell]);
      }
      rec[4 + 2 * cc] = amp;
      rec[5 + 2 * cc] = gp * gp;
    }
    __syncthreads();

    const int lb = max(base, w_first), le = min(base + nt, w_end);
    if (COMP) {
      // blocks of 16 lines summed plainly, then folded in with TwoSum
      for (int l0 = lb; l0 < le; l0 += 16) {
        const int l1 = min(l0 + 16, le);
        float part[P][C];
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
          for (int c = 0; c < C; ++c) part[p][c] = 0.f;
        for (int l = l0; l < l1; ++l) {
          const float* rec = lds + (l - base) * REC;
          const float4 h = *reinterpret_cast<const float4*>(rec);
          float dd[P];
#pragma unroll
          for (int p = 0; p < P; ++p) {
            const float t = jf[p] - h.x;
            const float d = t - h.y;
            const bool in = (t >= h.z) & (t <= Kf);
            dd[p] = in ? d * d : __builtin_inff();
          }
#pragma unroll
          for (int c = 0; c < C; c += 2) {
            const float4 ag = *reinterpret_cast<const float4*>(rec + 4 + 2 * c);
#pragma unroll
            for (int p = 0; p < P; ++p) {
              part[p][c] = fmaf(ag.x, fast_rcp(dd[p] + ag.y), part[p][c]);
              part[p][c + 1] = fmaf(ag.z, fast_rcp(dd[p] + ag.w), part[p][c + 1]);
            }
          }
        }
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
          for (int c = 0; c < C; ++c) two_sum_acc(acc[p][c], cmp[p][c], part[p][c]);
      }
    } else {
      for (int l = lb; l < le; ++l) {
        const float* rec = lds + (l - base) * REC;
        const float4 h = *reinterpret_cast<const float4*>(rec);
        float dd[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
          const float t = jf[p] - h.x;
          const float d = t - h.y;
          const bool in = (t >= h.z) & (t <= Kf);
          dd[p] = in ? d * d : __builtin_inff();
        }
#pragma unroll
        for (int c = 0; c < C; c += 2) {
          const float4 ag = *reinterpret_cast<const float4*>(rec + 4 + 2 * c);
#pragma unroll
          for (int p = 0; p < P; ++p) {
            acc[p][c] = fmaf(ag.x, fast_rcp(dd[p] + ag.y), acc[p][c]);
            acc[p][c + 1] = fmaf(ag.z, fast_rcp(dd[p] + ag.w), acc[p][c + 1]);
          }
        }
      }
    }
  }

#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int64_t cell = cell0 + c;
    if (cell >= a.n_cells) break;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int j = wj0 + 64 * p + lane;
      if (j < a.ld) {
        float v = COMP ? acc[p][c] + cmp[p][c] : acc[p][c];
        a.out[cell * a.ld + j] = (j < a.n_nu) ? v : 0.f;
      }
    }
  }
}

// Eq. (4): B = c1 nu^3 / (exp(c2 nu / T) - 1), evaluated in FP64 and stored
// in FP32; one block per (cell, 256-point segment of the row).
__global__ void planck_table_kernel(const double* __restrict__ T, int64_t n_cells,
                                    int n_nu, int64_t ld, int tiles_per_row,
                                    double nu0, double dnu, double c1, double c2,
                                    float* __restrict__ B) {
  const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
  const int64_t cell = b / tiles_per_row;
  if (cell >= n_cells) return;
  const int64_t j = (b % tiles_per_row) * 256 + threadIdx.x;
  if (j >= ld) return;
  float v = 0.f;
  if (j < n_nu) {
    double nu = nu0 + (double)j * dnu;
    v = (float)(c1 * nu * nu * nu / expm1(c2 * nu / T[cell]));
  }
  B[cell * ld + j] = v;
}

__global__ void wall_table_kernel(double T_wall, int n_nu, int64_t ld, double nu0,
                                  double dnu, double c1, double c2, float* bw) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ld) return;
  float v = 0.f;
  if (j < n_nu && T_wall > 0.0) {
    double nu = nu0 + (double)j * dnu;
    v = (float)(c1 * nu * nu * nu / expm1(c2 * nu / T_wall));
  }
  bw[j] = v;
}

}  // namespace

hipError_t launch_cell_params(rt_ctx c) {
  const int64_t n = c->n_cells;
  const int threads = 256;
  const int64_t blocks = (n + threads - 1) / threads;
  hipLaunchKernelGGL(cell_params_kernel, dim3((unsigned)blocks), dim3(threads), 0, c->stream,
                     n, c->d_T, c->d_x, c->d_p, c->T_ref, c->dnu, second_radiation_cm_K(),
                     c->have_E ? 1 : 0, c->cells.G, c->cells.beta, c->cells.theta,
                     c->cells.lam2, c->cells.P, c->cells.theta2);
  return hipGetLastError();
}

hipError_t launch_kappa(rt_ctx c, bool compensated) {
  constexpr int C = 4, P = 2;
  KappaArgs a;
  a.L = c->lines;
  a.C = c->cells;
  a.n_cells = c->n_cells;
  a.n_nu = c->n_nu;
  a.ld = c->ld;
  a.K = c->K;
  a.have_E = c->have_E ? 1 : 0;
  a.n_tiles = (int)((c->ld + kKappaThreads * P - 1) / (kKappaThreads * P));
  a.out = c->kappa;
  const int64_t groups = (c->n_cells + C - 1) / C;
  const int64_t blocks = groups * a.n_tiles;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  if (compensated)
    hipLaunchKernelGGL((kappa_linesum_kernel<C, P, true>), dim3((unsigned)blocks),
                       dim3(kKappaThreads), 0, c->stream, a);
  else
    hipLaunchKernelGGL((kappa_linesum_kernel<C, P, false>), dim3((unsigned)blocks),
                       dim3(kKappaThreads), 0, c->stream, a);
  return hipGetLastError();
}

hipError_t launch_planck(rt_ctx c) {
  const double c1 = first_radiation_wavenumber(), c2 = second_radiation_cm_K();
  const int tiles = (int)((c->ld + 255) / 256);
  if (c->planck) {
    const int64_t blocks = c->n_cells * tiles;
    const unsigned gx = (unsigned)std::min<int64_t>(blocks, 65536);
    const unsigned gy = (unsigned)((blocks + gx - 1) / gx);
    hipLaunchKernelGGL(planck_table_kernel, dim3(gx, gy), dim3(256), 0, c->stream, c->d_T,
                       c->n_cells, c->n_nu, c->ld, tiles, c->nu0, c->dnu, c1, c2, c->planck);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(wall_table_kernel, dim3((unsigned)((c->ld + 255) / 256)), dim3(256), 0,
                     c->stream, c->T_wall, c->n_nu, c->ld, c->nu0, c->dnu, c1, c2, c->d_bwall);
  return hipGetLastError();
}

}  // namespace rt
