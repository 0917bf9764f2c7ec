// batch.hip -- many independent receiver cases in one graph launch, in one
// of two shapes that give the same tallies bit for bit.
//
// Chunked: the rays of every case are generated and traversed in one
// launch; then, chunk after chunk of the spectrum, one line-sum launch
// fills a slab with the chunk's kappa for the cells of every case, and one
// march launch takes the rays of every case through it.  Each launch fills
// the GPU however small the cases, and the kernels are the single-case ones
// with a case lookup per block.  With several slabs the line sums run on a
// second stream, overlapping the march of the previous chunk.
//
// Persistent: work is a queue of items in a fixed order; every block pops
// the next item with one atomic and runs it:
//   RAYGEN (case, 256 rays)            rays and exact traversal -> segments
//   KAPPA  (case, chunk, tile, groups) line sum of a spectral chunk for a
//                                      range of cells into a kappa slab
//   MARCH  (case, chunk, ray range)    Eq. (3) over the chunk for the rays,
//                                      reading the slab
// The stage order is RAYGEN for every case, then K(0) K(1) M(0) K(2) M(1)
// ... over (case, chunk) pairs, so the line sum of the next pair overlaps
// the march of the current one.  Pair p writes slab p % slots.  An item
// only ever waits for items that precede it in the queue, and those are
// held by running blocks, so every wait ends; each wait is also bounded by
// a spin limit after which the item is skipped and an error flag is set,
// so the grid always drains.
//
// Memory ordering: items that produce data read by other blocks (segments,
// slabs) end with an agent-scope release by every thread before their
// completion counter is bumped; a block acquires once per pair before its
// first march item of that pair.  A march item only reads its slab, so its
// completion (which frees the slot for reuse) is counted with a relaxed
// atomic after its loads have returned.
#include "device_common.h"
#include "batch_plan.h"

namespace rt {
namespace {

using namespace dev;

struct BatchArgs {
  const BatchStage* stages;
  int n_stages;
  int64_t total_items;
  const BatchCase* cases;
  LineSet L;
  CellSet C;        // packed over all cases
  int n_nu, K, have_E, comp;
  float* slabs;     // [slots][max_cells][chunk_points]
  int64_t slab_stride;
  int chunk_points;
  int tiles_per_chunk;
  int kappa_groups;
  int march_rays;
  int slots;
  int2* segs;
  int32_t* counts;
  const uint32_t* perm;  // per case: slot -> ray index (coherent order)
  const float* bwall;  // [case][bwall_ld]
  int64_t bwall_ld;
  unsigned long long* acc;  // accumulator rows (see BatchPlan::d_acc)
  unsigned* ovf;
  double nu0, dnu, c1;
  unsigned long long* queue;
  unsigned* rg_done;
  unsigned* k_done;
  unsigned* m_done;
  unsigned* error;
  unsigned spin_limit;
};

__device__ __forceinline__ int find_stage(const BatchStage* st, int n, int64_t item) {
  int lo = 0, hi = n - 1;  // last stage with first <= item
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (st[mid].first <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Spin (thread 0 only) until *p >= target, relaxed loads; false on timeout.
__device__ __forceinline__ bool wait_count(const unsigned* p, unsigned target, unsigned limit) {
  unsigned it = 0;
  while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    if (++it > limit) return false;
    __builtin_amdgcn_s_sleep(4);
  }
  return true;
}

template <bool QUAD>
// Five wavefronts per SIMD (at most 102 VGPRs): the march items wait on memory
// and need the wavefronts to hide it.  Left alone the combined code paths take
// 142 VGPRs and three wavefronts; at five, 33 VGPRs go to scratch, a few
// accesses per march segment, which costs less than the two wavefronts gain
// (measured: 4.57 s at three, 4.33 s at four, 4.26 s at five for the 64-case
// launch; six spills 62 and is not used).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8))) void batch_kernel(BatchArgs a) {
  // line-sum tiles stage line records here; march items stage their
  // per-segment partial sums (4 wavefronts) in the same memory
  constexpr int kLdsFloats = kLineTile * (4 + 2 * kKappaCells);
  static_assert(kLdsFloats >= 4 * TallyStage<false>::kEntries, "march staging fits");
  __shared__ float4 lds4[kLdsFloats / 4];
  __shared__ long long s_item;
  __shared__ int s_ok;
  float* lds = reinterpret_cast<float*>(lds4);
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  int ready_pair = -1;  // pair whose segments and slab this block has acquired

  for (;;) {
    __syncthreads();
    if (tid == 0) {
      s_item = (long long)atomicAdd(a.queue, 1ull);
      s_ok = __hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
    }
    __syncthreads();
    const int64_t item = s_item;
    if (item >= a.total_items) break;
    const BatchStage st = a.stages[find_stage(a.stages, a.n_stages, item)];
    const BatchCase cs = a.cases[st.cas];
    const int64_t local = item - st.first;
    if (!s_ok) continue;  // a wait timed out somewhere: drain the queue

    if (st.kind == kStageRaygen) {
      // slot r of the case holds ray perm[r] of the coherent order
      const int64_t r = local * 256 + tid;
      if (r < cs.n_rays) {
        int64_t O[3], D[3];
        sample_ray(cs.seed, (uint64_t)a.perm[cs.ray_off + r], cs.nx, cs.ny, cs.nz, O, D);
        const int ns = traverse(cs.nx, cs.ny, cs.nz, cs.unit_cm, O, D, cs.max_segs,
                                a.segs + cs.seg_off + r * cs.max_segs);
        a.counts[cs.ray_off + r] = ns;
      }
      __atomic_thread_fence(__ATOMIC_RELEASE);  // agent scope: segments visible
      __syncthreads();
      if (tid == 0) __hip_atomic_fetch_add(a.rg_done + st.cas, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      continue;
    }

    float* slab = a.slabs + (int64_t)st.slot * a.slab_stride;
    if (st.kind == kStageKappa) {
      if (st.wait_pair >= 0) {  // the slab's previous pair must be marched
        if (tid == 0) {
          const BatchStage& ms = a.stages[st.wait_stage];
          if (!wait_count(a.m_done + st.wait_pair, (unsigned)ms.count, a.spin_limit)) {
            atomicOr(a.error, 1u);
            s_ok = 0;
          }
        }
        __syncthreads();
        if (!s_ok) continue;
      }
      KappaTile t;
      t.L = a.L;
      t.C.G = a.C.G + cs.cell_off;
      t.C.beta = a.C.beta + cs.cell_off;
      t.C.theta = a.C.theta + cs.cell_off;
      t.C.lam2 = a.C.lam2 + cs.cell_off;
      t.C.P = a.C.P + cs.cell_off;
      t.n_cells = cs.n_cells;
      t.n_nu = a.n_nu;
      t.K = a.K;
      t.have_E = a.have_E;
      t.out = slab;
      t.ld_out = a.chunk_points;
      t.col0 = (int64_t)st.chunk * a.chunk_points;
      t.col_end = t.col0 + a.chunk_points;
      const int tile = (int)(local % a.tiles_per_chunk);
      const int64_t gb = local / a.tiles_per_chunk;
      const int64_t n_groups = (cs.n_cells + kKappaCells - 1) / kKappaCells;
      const int j0 = (int)(t.col0 + (int64_t)tile * kKappaTilePoints);
      const int64_t g_end = min((gb + 1) * a.kappa_groups, n_groups);
      for (int64_t g = gb * a.kappa_groups; g < g_end; ++g) {
        if (a.comp) kappa_tile<true>(t, j0, g * kKappaCells, lds);
        else kappa_tile<false>(t, j0, g * kKappaCells, lds);
      }
      __atomic_thread_fence(__ATOMIC_RELEASE);  // agent scope: slab visible
      __syncthreads();
      if (tid == 0) __hip_atomic_fetch_add(a.k_done + st.pair, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      continue;
    }

    // MARCH
    if (ready_pair != st.pair) {
      if (tid == 0) {
        const BatchStage& ks = a.stages[st.wait_stage];
        const BatchStage& rs = a.stages[st.raygen_stage];
        bool ok = wait_count(a.rg_done + st.cas, (unsigned)rs.count, a.spin_limit) &&
                  wait_count(a.k_done + st.pair, (unsigned)ks.count, a.spin_limit);
        if (!ok) {
          atomicOr(a.error, 1u);
          s_ok = 0;
        }
        __atomic_thread_fence(__ATOMIC_ACQUIRE);  // agent scope
      }
      __syncthreads();
      if (!s_ok) continue;
      ready_pair = st.pair;
    }
    MarchWave w;
    w.kappa = slab;
    w.planck = nullptr;
    w.ld = a.chunk_points;
    w.col0 = (int64_t)st.chunk * a.chunk_points;
    w.theta = a.C.theta + cs.cell_off;
    w.bwall = a.bwall + (int64_t)st.cas * a.bwall_ld;
    w.nu0 = a.nu0;
    w.dnu = a.dnu;
    w.c1 = a.c1;
    w.weight = cs.weight;
    w.acc = a.acc;
    w.row0 = cs.cell_off + (int64_t)st.cas * kCaseBalRows;
    w.bal_row0 = w.row0 + cs.n_cells;
    w.bal_mask = kCaseBalRows - 1;
    w.ovf = a.ovf;
    float* stage = lds + wave * TallyStage<false>::kEntries;
    const int64_t r0 = local * a.march_rays;
    const int64_t r1 = min(r0 + a.march_rays, cs.n_rays);
    for (int64_t r = r0 + wave; r < r1; r += 4) {
      const int2* sg = a.segs + cs.seg_off + r * cs.max_segs;
      const int ns = a.counts[cs.ray_off + r];
      for (int sub = 0; sub < a.chunk_points / kChunk; ++sub) {
        const int64_t j = w.col0 + (int64_t)sub * kChunk + lane * kQ;
        march_wave<false, false, QUAD>(w, sg, ns, j, lane, nullptr, stage, r);
      }
    }
    __syncthreads();
    if (tid == 0) __hip_atomic_fetch_add(a.m_done + st.pair, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Carries of every accumulator row (rows x 2 digit groups).
__global__ void batch_acc_normalize_kernel(unsigned long long* acc, int64_t groups) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < groups) acc_normalize(acc + i * kAccDigits);
}

// The exact sum of accumulator rows [first, first + n): each digit is summed
// over the rows as an integer (normalised digits are below 2^28 and there are
// fewer than 2^31 rows), in a fixed-order tree over the block's 256 threads;
// thread 0 gets the normalised digits in d.
__device__ void case_rows_sum(const unsigned long long* __restrict__ acc, int64_t first,
                              int64_t n, unsigned long long (*red)[256], unsigned long long* d) {
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

// Per-cell powers of every case from its accumulator rows; one block per
// case then forms its balance = {entering, sum emitted, sum absorbed,
// escaped} from exact integer sums of its rows.
__global__ __launch_bounds__(256) void case_tally_kernel(const BatchCase* cases,
                                                         const unsigned long long* __restrict__ acc,
                                                         double* abs_, double* emi,
                                                         double* balance) {
  __shared__ unsigned long long red[kAccRow][256];
  const BatchCase cs = cases[blockIdx.x];
  const int64_t row0 = cs.cell_off + (int64_t)blockIdx.x * kCaseBalRows;
  for (int64_t c = threadIdx.x; c < cs.n_cells; c += 256) {
    const unsigned long long* r = acc + (row0 + c) * kAccRow;
    abs_[cs.cell_off + c] = acc_value(r);
    emi[cs.cell_off + c] = acc_value(r + kAccDigits);
  }
  unsigned long long cells[kAccRow], bal[kAccRow];
  case_rows_sum(acc, row0, cs.n_cells, red, cells);
  case_rows_sum(acc, row0 + cs.n_cells, kCaseBalRows, red, bal);
  if (threadIdx.x == 0) {
    double* b = balance + 4 * blockIdx.x;
    b[0] = acc_value(bal);
    b[1] = acc_value(cells + kAccDigits);
    b[2] = acc_value(cells);
    b[3] = acc_value(bal + kAccDigits);
  }
}

// Coherent ray order per case (see order_key): counting sort of every
// case's rays by key, run before the persistent kernel in the same graph.
__device__ __forceinline__ int case_of_ray(const BatchCase* cases, int n_cases, int64_t r) {
  int lo = 0, hi = n_cases - 1;  // last case with ray_off <= r
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cases[mid].ray_off <= r) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void batch_order_key_kernel(const BatchCase* __restrict__ cases, int n_cases,
                                       int64_t total_rays, uint32_t* keys, uint32_t* hist) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total_rays) return;
  const int k = case_of_ray(cases, n_cases, i);
  const BatchCase cs = cases[k];
  int64_t O[3], D[3];
  sample_ray(cs.seed, (uint64_t)(i - cs.ray_off), cs.nx, cs.ny, cs.nz, O, D);
  const uint32_t key = order_key(O, D, cs.nx, cs.ny, cs.nz);
  keys[i] = key;
  atomicAdd(hist + (int64_t)k * kOrderBuckets + key, 1u);
}

// one block of 1024 threads per case: exclusive prefix sum of its histogram
__global__ __launch_bounds__(1024) void batch_order_scan_kernel(uint32_t* hist) {
  __shared__ uint32_t part[1024];
  uint32_t* h = hist + (int64_t)blockIdx.x * kOrderBuckets;
  const int t = threadIdx.x;
  constexpr int run = (kOrderBuckets + 1023) / 1024;
  const int lo = min(kOrderBuckets, t * run), hi = min(kOrderBuckets, lo + run);
  uint32_t s = 0;
  for (int i = lo; i < hi; ++i) s += h[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const uint32_t v = t >= off ? part[t - off] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint32_t acc = part[t] - s;
  for (int i = lo; i < hi; ++i) {
    const uint32_t v = h[i];
    h[i] = acc;
    acc += v;
  }
}

__global__ void batch_order_scatter_kernel(const BatchCase* __restrict__ cases, int n_cases,
                                           int64_t total_rays, const uint32_t* __restrict__ keys,
                                           uint32_t* hist, uint32_t* perm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total_rays) return;
  const int k = case_of_ray(cases, n_cases, i);
  const int64_t off = cases[k].ray_off;
  const uint32_t pos = atomicAdd(hist + (int64_t)k * kOrderBuckets + keys[i], 1u);
  perm[off + pos] = (uint32_t)(i - off);
}

// Chunked mode, rays: slot r of case k holds ray perm[ray_off + r] of the
// case (its coherent order), traversed into the case's segment lists.
__global__ void batch_raygen_kernel(const BatchCase* __restrict__ cases, int n_cases,
                                    int64_t total_rays, const uint32_t* __restrict__ perm,
                                    int2* segs, int32_t* counts) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total_rays) return;
  const BatchCase cs = cases[case_of_ray(cases, n_cases, i)];
  const int64_t r = i - cs.ray_off;
  int64_t O[3], D[3];
  sample_ray(cs.seed, (uint64_t)perm[i], cs.nx, cs.ny, cs.nz, O, D);
  counts[i] = traverse(cs.nx, cs.ny, cs.nz, cs.unit_cm, O, D, cs.max_segs,
                       segs + cs.seg_off + r * cs.max_segs);
}

struct ChunkMarchArgs {
  const BatchCase* cases;
  int n_cases;
  const float* slab;     // the chunk's slab: [total cells][chunk_points]
  int chunk_points;
  int64_t col0;          // first point of the chunk
  const double* theta;   // packed over the cases
  const float* bwall;    // [case][bwall_ld]
  int64_t bwall_ld;
  double nu0, dnu, c1;
  const int2* segs;
  const int32_t* counts;
  unsigned long long* acc;
  unsigned* ovf;
};

// last case whose first block row is <= local
__device__ __forceinline__ int case_of_block(const BatchCase* cases, int n_cases, int64_t local) {
  int lo = 0, hi = n_cases - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cases[mid].blk_off <= local) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Chunked mode, march: block = 4 wavefronts = 4 consecutive slots of one
// case on one kChunk-point part of the chunk.  Workgroups go to the 8 XCDs
// round-robin (block b runs on XCD b % 8); the rows of 8 blocks (b / 8) run
// case after case, and within a case each XCD takes a contiguous eighth of
// its ray blocks, part-major: the single-case kernel's order, so that all
// XCDs work on one case's slab rows at a time and its working set stays in
// the last-level cache.  Each wavefront adds to the same accumulator rows as
// the persistent kernel's march items.
template <bool QUAD>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8))) void chunk_march_kernel(
    ChunkMarchArgs a) {
  __shared__ float stage[4][TallyStage<false>::kEntries];
  const int64_t b = blockIdx.x;
  const int64_t xcd = b & 7, local = b >> 3;
  const int k = case_of_block(a.cases, a.n_cases, local);
  const BatchCase& cs = a.cases[k];
  const int64_t nb = (cs.n_rays + 3) / 4, rbx = (nb + 7) / 8;
  const int64_t idx = local - cs.blk_off;
  const int part = (int)(idx / rbx);
  const int64_t rb = xcd * rbx + idx % rbx;
  if (rb >= nb) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t r = rb * 4 + wave;
  if (r >= cs.n_rays) return;
  MarchWave w;
  w.kappa = a.slab + cs.cell_off * a.chunk_points;
  w.planck = nullptr;
  w.ld = a.chunk_points;
  w.col0 = a.col0;
  w.theta = a.theta + cs.cell_off;
  w.bwall = a.bwall + (int64_t)k * a.bwall_ld;
  w.nu0 = a.nu0;
  w.dnu = a.dnu;
  w.c1 = a.c1;
  w.weight = cs.weight;
  w.acc = a.acc;
  w.row0 = cs.cell_off + (int64_t)k * kCaseBalRows;
  w.bal_row0 = w.row0 + cs.n_cells;
  w.bal_mask = kCaseBalRows - 1;
  w.ovf = a.ovf;
  const int64_t j = a.col0 + (int64_t)part * kChunk + lane * kQ;
  march_wave<false, false, QUAD>(w, a.segs + cs.seg_off + r * cs.max_segs,
                                 a.counts[cs.ray_off + r], j, lane, nullptr, stage[wave], r);
}

__global__ void fill_u32_kernel(unsigned* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}
__global__ void fill_f64_kernel(double* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// B(nu_j, T_wall) rows per case, evaluated in FP32 as the single-case walls'
// row (planck_f32).
__global__ void case_wall_kernel(const BatchCase* __restrict__ cases, int n_cases, int n_nu,
                                 int64_t ld, float2 nu0, float2 dnu, float c1, float* bw) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n_cases * ld) return;
  const int cs = (int)(i / ld);
  const int64_t j = i % ld;
  const float2 th = cases[cs].theta_wall;
  float v = 0.f;
  if (j < n_nu && th.x > 0.f) v = planck_f32(nu_at(j, pair_of(nu0), pair_of(dnu)), pair_of(th), c1);
  bw[i] = v;
}

}  // namespace

static float2 host_pair(double v) {
  const float h = (float)v;
  return make_float2(h, (float)(v - (double)h));
}

hipError_t launch_batch_prep(rt_ctx c, const BatchPlan& pl, hipStream_t s) {
  const float c1 = (float)first_radiation_wavenumber();
  const int64_t nw = (int64_t)pl.n_cases * pl.bwall_ld;
  hipLaunchKernelGGL(case_wall_kernel, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s,
                     pl.d_cases, pl.n_cases, c->n_nu, pl.bwall_ld, host_pair(c->nu0),
                     host_pair(c->dnu), c1, pl.d_bwall);
  return hipGetLastError();
}

hipError_t launch_batch(rt_ctx c, const BatchPlan& pl, hipStream_t s) {
  auto fill_u = [&](unsigned* p, int64_t n) {
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  };
  auto fill_d = [&](double* p, int64_t n) {
    hipLaunchKernelGGL(fill_f64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  };
  fill_u(pl.d_counters, pl.n_counters);
  fill_u(pl.d_hist, (int64_t)pl.n_cases * kOrderBuckets);
  const unsigned ray_blocks = (unsigned)((pl.total_rays + 255) / 256);
  hipLaunchKernelGGL(batch_order_key_kernel, dim3(ray_blocks), dim3(256), 0, s, pl.d_cases,
                     pl.n_cases, pl.total_rays, pl.d_keys, pl.d_hist);
  hipLaunchKernelGGL(batch_order_scan_kernel, dim3((unsigned)pl.n_cases), dim3(1024), 0, s,
                     pl.d_hist);
  hipLaunchKernelGGL(batch_order_scatter_kernel, dim3(ray_blocks), dim3(256), 0, s, pl.d_cases,
                     pl.n_cases, pl.total_rays, pl.d_keys, pl.d_hist, pl.d_perm);
  const int64_t acc_words = (pl.total_cells + (int64_t)pl.n_cases * kCaseBalRows) * kAccRow;
  fill_d(reinterpret_cast<double*>(pl.d_acc), acc_words + 1);  // + overflow flag
  unsigned* ovf = reinterpret_cast<unsigned*>(pl.d_acc + acc_words);
  const int64_t groups = acc_words / kAccDigits;
  auto finish = [&]() {
    hipLaunchKernelGGL(batch_acc_normalize_kernel, dim3((unsigned)((groups + 255) / 256)),
                       dim3(256), 0, s, pl.d_acc, groups);
    hipLaunchKernelGGL(case_tally_kernel, dim3((unsigned)pl.n_cases), dim3(256), 0, s,
                       pl.d_cases, pl.d_acc, pl.d_abs, pl.d_emi, pl.d_balance);
    return hipGetLastError();
  };
  if (pl.chunked) {
    hipLaunchKernelGGL(batch_raygen_kernel, dim3(ray_blocks), dim3(256), 0, s, pl.d_cases,
                       pl.n_cases, pl.total_rays, pl.d_perm, pl.d_segs, pl.d_counts);
    const int cp = pl.tuning.chunk_points;
    const int tiles = cp / dev::kKappaTilePoints;
    KappaTile t;
    t.L = c->lines;
    t.C = pl.cells;
    t.n_cells = pl.total_cells;
    t.n_nu = c->n_nu;
    t.K = c->K;
    t.have_E = c->have_E ? 1 : 0;
    t.out = pl.d_slabs;
    t.ld_out = cp;
    ChunkMarchArgs m;
    m.cases = pl.d_cases;
    m.n_cases = pl.n_cases;
    m.slab = pl.d_slabs;
    m.chunk_points = cp;
    m.theta = pl.cells.theta;
    m.bwall = pl.d_bwall;
    m.bwall_ld = pl.bwall_ld;
    m.nu0 = c->nu0;
    m.dnu = c->dnu;
    m.c1 = first_radiation_wavenumber();
    m.segs = pl.d_segs;
    m.counts = pl.d_counts;
    m.acc = pl.d_acc;
    m.ovf = ovf;
    const int64_t march_blocks = 8 * pl.ray_blocks;
    if (march_blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const int64_t n_groups = (pl.total_cells + kKappaCells - 1) / kKappaCells;
    // chunk ch uses slab ch % slots.  With one slab everything runs in
    // order on s.  With more, the line sums run on the side stream, ahead
    // of the marches by up to slots - 1 chunks (the line sum of a chunk
    // overlaps the march of the previous one): march ch waits for line sum
    // ch, and line sum ch waits for the march that last read its slab.
    const int slots = pl.tuning.slots;
    const bool two = slots > 1;
    hipStream_t ks = two ? pl.side_stream : s;
    hipEvent_t* ev = two ? const_cast<hipEvent_t*>(pl.events.data()) : nullptr;
    hipError_t e = hipSuccess;
    if (two) {
      e = hipEventRecord(ev[0], s);
      if (e == hipSuccess) e = hipStreamWaitEvent(ks, ev[0], 0);
    }
    for (int ch = 0; ch < pl.n_chunks && e == hipSuccess; ++ch) {
      float* slab = pl.d_slabs + (int64_t)(ch % slots) * pl.slab_stride;
      t.out = slab;
      t.col0 = (int64_t)ch * cp;
      t.col_end = t.col0 + cp;
      if (two && ch >= slots) e = hipStreamWaitEvent(ks, ev[1 + pl.n_chunks + ch - slots], 0);
      if (e == hipSuccess) e = launch_kappa_tiles(c, t, n_groups, ch * tiles, tiles, pl.comp, ks);
      if (two && e == hipSuccess) e = hipEventRecord(ev[1 + ch], ks);
      if (two && e == hipSuccess) e = hipStreamWaitEvent(s, ev[1 + ch], 0);
      if (e != hipSuccess) break;
      m.slab = slab;
      m.col0 = t.col0;
      if (pl.planck_quad)
        hipLaunchKernelGGL(chunk_march_kernel<true>, dim3((unsigned)march_blocks), dim3(256), 0, s, m);
      else
        hipLaunchKernelGGL(chunk_march_kernel<false>, dim3((unsigned)march_blocks), dim3(256), 0, s, m);
      if (two) e = hipEventRecord(ev[1 + pl.n_chunks + ch], s);
    }
    if (e != hipSuccess) return e;
    return finish();
  }
  BatchArgs a;
  a.stages = pl.d_stages;
  a.n_stages = pl.n_stages;
  a.total_items = pl.total_items;
  a.cases = pl.d_cases;
  a.L = c->lines;
  a.C = pl.cells;
  a.n_nu = c->n_nu;
  a.K = c->K;
  a.have_E = c->have_E ? 1 : 0;
  a.comp = pl.comp ? 1 : 0;
  a.slabs = pl.d_slabs;
  a.slab_stride = pl.slab_stride;
  a.chunk_points = pl.tuning.chunk_points;
  a.tiles_per_chunk = pl.tuning.chunk_points / dev::kKappaTilePoints;
  a.kappa_groups = pl.tuning.kappa_groups;
  a.march_rays = pl.tuning.march_rays;
  a.slots = pl.tuning.slots;
  a.segs = pl.d_segs;
  a.counts = pl.d_counts;
  a.perm = pl.d_perm;
  a.bwall = pl.d_bwall;
  a.bwall_ld = pl.bwall_ld;
  a.acc = pl.d_acc;
  a.ovf = ovf;
  a.nu0 = c->nu0;
  a.dnu = c->dnu;
  a.c1 = first_radiation_wavenumber();
  a.queue = reinterpret_cast<unsigned long long*>(pl.d_counters);
  a.error = pl.d_counters + 2;
  a.rg_done = pl.d_counters + 4;
  a.k_done = a.rg_done + pl.n_cases;
  a.m_done = a.k_done + pl.n_pairs;
  a.spin_limit = 1u << 24;
  if (pl.planck_quad)
    hipLaunchKernelGGL(batch_kernel<true>, dim3((unsigned)pl.grid_blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(batch_kernel<false>, dim3((unsigned)pl.grid_blocks), dim3(256), 0, s, a);
  return finish();
}

}  // namespace rt
