// march.hip -- Monte-Carlo rays through the cell grid on gfx950.
//
//   order      : a coherent processing order for the rays of a batch
//                (counting sort on a direction/position key)
//   raygen_dda : Philox4x64-10 ray sampling (uniform boundary point,
//                cosine-weighted inward direction) and exact integer
//                traversal -> per-ray list of (cell, length) segments
//   march      : Eq. (3) applied cell after cell for every nu point; each
//                wavefront owns one ray and a kChunk-point spectral chunk
//                (dev::march_wave); the absorbed and emitted power of the
//                chunk per segment is summed across the wavefront in a fixed
//                order and added to the cell's fixed-point accumulator
//   tally      : the accumulators as FP64 powers per cell, and the energy
//                balance from exact sums of the accumulators
#include "device_common.h"

namespace rt {
namespace {

using namespace dev;

__global__ void order_key_kernel(uint64_t seed, uint64_t begin, int64_t count, int nx, int ny,
                                 int nz, uint32_t* keys, uint32_t* hist) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  int64_t O[3], D[3];
  sample_ray(seed, begin + (uint64_t)i, nx, ny, nz, O, D);
  const uint32_t k = order_key(O, D, nx, ny, nz);
  keys[i] = k;
  atomicAdd(hist + k, 1u);
}

// Exclusive prefix sum of hist[0..n) in place; one block of 1024 threads,
// each owning a contiguous run.
__global__ __launch_bounds__(1024) void order_scan_kernel(uint32_t* hist, int n) {
  __shared__ uint32_t part[1024];
  const int t = threadIdx.x;
  const int run = (n + 1023) / 1024;
  const int lo = min(n, t * run), hi = min(n, lo + run);
  uint32_t s = 0;
  for (int i = lo; i < hi; ++i) s += hist[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const uint32_t v = t >= off ? part[t - off] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint32_t acc = part[t] - s;  // exclusive
  for (int i = lo; i < hi; ++i) {
    const uint32_t v = hist[i];
    hist[i] = acc;
    acc += v;
  }
}

__global__ void order_scatter_kernel(const uint32_t* __restrict__ keys, int64_t count,
                                     uint32_t* offsets, uint32_t* perm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  perm[atomicAdd(offsets + keys[i], 1u)] = (uint32_t)i;
}

__global__ void zero_u32_kernel(uint32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// Slot i of the batch holds ray begin + perm[i] (begin + i without perm).
__global__ void raygen_dda_kernel(uint64_t seed, uint64_t begin, int64_t count, int nx, int ny,
                                  int nz, double unit_cm, int max_segs,
                                  const int64_t* __restrict__ explicit_rays, int64_t* rays_out,
                                  int2* segs, int32_t* counts, unsigned long long* seg_total,
                                  const uint32_t* __restrict__ perm) {
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
      sample_ray(seed, begin + (perm ? (uint64_t)perm[i] : (uint64_t)i), nx, ny, nz, O, D);
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

struct MarchArgs {
  MarchWave w;
  int n_chunks;
  int64_t ray_blocks_x;  // ray blocks per XCD
  const int2* segs;
  const int32_t* counts;
  int max_segs;
  int64_t n_rays;
  float* exit_I;
};

// Block = 4 wavefronts = 4 consecutive rays (batch slots) on one spectral
// chunk.  Workgroups are dispatched to the 8 XCDs round-robin, so block b
// runs on XCD b % 8; that XCD is given a contiguous range of ray blocks,
// chunk-major, so the waves in flight on it march neighbouring rays of the
// coherent order through one chunk and share kappa rows in its L2.
template <bool PREC, bool EXIT, bool QUAD>
__device__ __forceinline__ void march_block(const MarchArgs& a,
                                            typename Partial<PREC>::T (*stage)[TallyStage<PREC>::kEntries]) {
  const int64_t b = blockIdx.x;
  const int64_t xcd = b & 7, local = b >> 3;
  const int chunk = (int)(local / a.ray_blocks_x);
  const int64_t rb = xcd * a.ray_blocks_x + local % a.ray_blocks_x;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t ray = rb * 4 + wave;
  if (ray >= a.n_rays) return;
  const int64_t j = (int64_t)chunk * kChunk + lane * kQ;
  march_wave<PREC, EXIT, QUAD>(a.w, a.segs + ray * a.max_segs, a.counts[ray], j, lane,
                               EXIT ? a.exit_I + ray * a.w.ld : nullptr, stage[wave], ray);
}

// Plain form.  Five wavefronts per SIMD (at most 96 VGPRs): the kappa rows
// of the next segments are in flight while other wavefronts compute.
template <bool EXIT, bool QUAD>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8))) void march_kernel(
    MarchArgs a) {
  __shared__ float stage[4][TallyStage<false>::kEntries];
  march_block<false, EXIT, QUAD>(a, stage);
}

// Precision form (Planck table, FP64 partial sums).
template <bool EXIT>
__global__ __launch_bounds__(256) void march_prec_kernel(MarchArgs a) {
  __shared__ double stage[4][TallyStage<true>::kEntries];
  march_block<true, EXIT, true>(a, stage);
}

// Carries of every accumulator row (rows x 2 digit groups).
__global__ void acc_normalize_kernel(unsigned long long* acc, int64_t groups) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < groups) acc_normalize(acc + i * kAccDigits);
}

// Per-cell powers from the normalised accumulators.
__global__ void acc_cells_kernel(const unsigned long long* __restrict__ acc, int64_t n_cells,
                                 double* abs_, double* emi) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_cells) return;
  abs_[c] = acc_value(acc + c * kAccRow);
  emi[c] = acc_value(acc + c * kAccRow + kAccDigits);
}

// The exact sum of accumulator rows [first, first + n): each digit is summed
// over the rows as an integer (normalised digits are below 2^28 and there are
// fewer than 2^31 rows), in a fixed-order tree over the block's 256 threads;
// thread 0 gets the normalised digits in d.
__device__ void acc_rows_sum(const unsigned long long* __restrict__ acc, int64_t first, int64_t n,
                             unsigned long long (*red)[256], unsigned long long* d) {
  const int t = threadIdx.x;
  unsigned long long s[kAccRow];
#pragma unroll
  for (int k = 0; k < kAccRow; ++k) s[k] = 0;
  for (int64_t r = first + t; r < first + n; r += 256)
#pragma unroll
    for (int k = 0; k < kAccRow; ++k) s[k] += acc[r * kAccRow + k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kAccRow; ++k) red[k][t] = s[k];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off)
#pragma unroll
      for (int k = 0; k < kAccRow; ++k) red[k][t] += red[k][t + off];
    __syncthreads();
  }
  if (t == 0) {
#pragma unroll
    for (int k = 0; k < kAccRow; ++k) d[k] = red[k][0];
    acc_normalize(d);
    acc_normalize(d + kAccDigits);
  }
}

// balance = {entering, sum emitted, sum absorbed, escaped}, each from the
// exact sum of its accumulators (cells, or the balance rows), converted once.
__global__ __launch_bounds__(256) void tally_kernel(const unsigned long long* __restrict__ acc,
                                                    int64_t n_cells, double* balance) {
  __shared__ unsigned long long red[kAccRow][256];
  unsigned long long cells[kAccRow], bal[kAccRow];
  acc_rows_sum(acc, 0, n_cells, red, cells);
  acc_rows_sum(acc, n_cells, kBalRows, red, bal);
  if (threadIdx.x == 0) {
    balance[0] = acc_value(bal);
    balance[1] = acc_value(cells + kAccDigits);
    balance[2] = acc_value(cells);
    balance[3] = acc_value(bal + kAccDigits);
  }
}

__global__ void zero_f64_kernel(double* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

}  // namespace

RayScratch owned_rays(rt_ctx c) {
  RayScratch s;
  s.segs = c->d_segs;
  s.counts = c->d_counts;
  s.keys = c->d_keys;
  s.perm = c->d_perm;
  s.hist = c->d_hist;
  s.max_segs = c->max_segs;
  s.cap = c->batch_rays;
  return s;
}

hipError_t launch_order(rt_ctx c, const RayScratch& s, uint64_t seed, uint64_t begin,
                        int64_t count) {
  const int threads = 256;
  const unsigned blocks = (unsigned)((count + threads - 1) / threads);
  hipLaunchKernelGGL(zero_u32_kernel, dim3((kOrderBuckets + threads - 1) / threads), dim3(threads),
                     0, c->stream, s.hist, (int64_t)kOrderBuckets);
  hipLaunchKernelGGL(order_key_kernel, dim3(blocks), dim3(threads), 0, c->stream, seed, begin,
                     count, c->nx, c->ny, c->nz, s.keys, s.hist);
  hipLaunchKernelGGL(order_scan_kernel, dim3(1), dim3(1024), 0, c->stream, s.hist,
                     kOrderBuckets);
  hipLaunchKernelGGL(order_scatter_kernel, dim3(blocks), dim3(threads), 0, c->stream, s.keys,
                     count, s.hist, s.perm);
  return hipGetLastError();
}

hipError_t launch_raygen(rt_ctx c, const RayScratch& s, uint64_t seed, uint64_t begin,
                         int64_t count, bool explicit_rays, int64_t* rays_out, bool count_work,
                         const uint32_t* perm) {
  const int threads = 256;
  const int64_t blocks = (count + threads - 1) / threads;
  const double unit_cm = c->cell_m * 100.0 / (double)kCellUnits;
  hipLaunchKernelGGL(raygen_dda_kernel, dim3((unsigned)blocks), dim3(threads), 0, c->stream,
                     seed, begin, count, c->nx, c->ny, c->nz, unit_cm, s.max_segs,
                     explicit_rays ? c->d_rays_explicit : nullptr, rays_out, s.segs,
                     s.counts, count_work ? c->d_segcount : nullptr, perm);
  return hipGetLastError();
}

// The plain march expands B(nu_a + s) = B0 (1 + g1 s + (g1^2 + g2) s^2 / 2
// + ...) about a lane's first point nu_a, s <= (kQ - 1) dnu, with
// g1 = d ln B / d nu = 3/nu - theta (1 + r), g2 = d g1 / d nu
// = -3/nu^2 + theta^2 r (1 + r), theta = c2/T, r = 1/(exp(theta nu) - 1).
// The second-order term is needed unless its relative size stays below FP32
// unit roundoff (2^-24) over the grid's temperatures and wavenumbers
// (checked at the extremes and midpoints of both ranges).
bool planck_needs_quadratic(double T_min, double T_max, double nu0, double dnu, int n_nu) {
  const double c2 = second_radiation_cm_K();
  const double span = (kQ - 1) * dnu;
  const double nu_lo = nu0, nu_hi = nu0 + (n_nu - 1) * dnu;
  const double Ts[3] = {T_min, T_max, std::sqrt(T_min * T_max)};
  const double nus[3] = {nu_lo, nu_hi, 0.5 * (nu_lo + nu_hi)};
  double worst = 0;
  for (double T : Ts)
    for (double nu : nus) {
      const double th = c2 / T, r = 1.0 / std::expm1(th * nu);
      const double g1 = 3.0 / nu - th * (1.0 + r);
      const double g2 = -3.0 / (nu * nu) + th * th * r * (1.0 + r);
      worst = std::max(worst, 0.5 * std::fabs(g1 * g1 + g2) * span * span);
    }
  return !(worst < std::ldexp(1.0, -24));
}

hipError_t launch_march(rt_ctx c, const RayScratch& s, int64_t count, double weight, bool prec,
                        float* exit_dev) {
  MarchArgs a;
  a.w.kappa = c->kappa;
  a.w.planck = c->planck;
  a.w.ld = c->ld;
  a.w.col0 = 0;
  a.w.theta = c->cells.theta;
  a.w.bwall = c->d_bwall;
  a.w.nu0 = c->nu0;
  a.w.dnu = c->dnu;
  a.w.c1 = first_radiation_wavenumber();
  a.w.weight = weight;
  a.w.acc = c->d_acc;
  a.w.row0 = 0;
  a.w.bal_row0 = c->n_cells;
  a.w.bal_mask = kBalRows - 1;
  a.w.ovf = c->d_ovf;
  a.n_chunks = (int)(c->ld / kChunk);
  a.ray_blocks_x = ((count + 3) / 4 + 7) / 8;
  a.segs = s.segs;
  a.counts = s.counts;
  a.max_segs = s.max_segs;
  a.n_rays = count;
  a.exit_I = exit_dev;
  const int64_t blocks = 8 * a.ray_blocks_x * a.n_chunks;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 g((unsigned)blocks), t(256);
  if (prec) {
    if (exit_dev) hipLaunchKernelGGL((march_prec_kernel<true>), g, t, 0, c->stream, a);
    else hipLaunchKernelGGL((march_prec_kernel<false>), g, t, 0, c->stream, a);
  } else if (planck_needs_quadratic(c->T_min, c->T_max, c->nu0, c->dnu, c->n_nu)) {
    if (exit_dev) hipLaunchKernelGGL((march_kernel<true, true>), g, t, 0, c->stream, a);
    else hipLaunchKernelGGL((march_kernel<false, true>), g, t, 0, c->stream, a);
  } else {
    if (exit_dev) hipLaunchKernelGGL((march_kernel<true, false>), g, t, 0, c->stream, a);
    else hipLaunchKernelGGL((march_kernel<false, false>), g, t, 0, c->stream, a);
  }
  const int64_t groups = 2 * (c->n_cells + kBalRows);
  hipLaunchKernelGGL(acc_normalize_kernel, dim3((unsigned)((groups + 255) / 256)), dim3(256), 0,
                     c->stream, c->d_acc, groups);
  return hipGetLastError();
}

hipError_t launch_tally(rt_ctx c) {
  hipLaunchKernelGGL(acc_cells_kernel, dim3((unsigned)((c->n_cells + 255) / 256)), dim3(256), 0,
                     c->stream, c->d_acc, c->n_cells, c->d_abs, c->d_emi);
  hipLaunchKernelGGL(tally_kernel, dim3(1), dim3(256), 0, c->stream, c->d_acc, c->n_cells,
                     c->d_balance);
  return hipGetLastError();
}

hipError_t launch_zero(rt_ctx c) {
  auto z = [&](double* p, int64_t n) {
    hipLaunchKernelGGL(zero_f64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       c->stream, p, n);
  };
  z(c->d_abs, c->n_cells);
  z(c->d_emi, c->n_cells);
  z(reinterpret_cast<double*>(c->d_acc), (c->n_cells + kBalRows) * kAccRow + 1);  // + overflow flag
  z(c->d_balance, 4);
  z(reinterpret_cast<double*>(c->d_segcount), 1);
  return hipGetLastError();
}

}  // namespace rt
