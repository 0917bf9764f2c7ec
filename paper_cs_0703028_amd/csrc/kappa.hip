// kappa.hip -- per-cell spectral properties on gfx950.
//
//   cell_params   : per-cell gas state -> FP32/FP64 factors (FP64 arithmetic)
//   kappa_linesum : Eq. (2) with the Eq. (1) strength ratio (line tiles staged
//                   in LDS, each lane owns 2 nu points of 8 cells, kappa
//                   written coalesced along nu; see dev::kappa_tile)
//   planck_table  : Eq. (4), wavenumber form, per (cell, nu) and for the walls,
//                   evaluated in FP32 (pair arguments, exp_pair/expm1_pair)
#include "batch_plan.h"
#include "device_common.h"

namespace rt {
namespace {

using namespace dev;

// ---------------------------------------------------------------- cells
// u = x p / (k_B T) [cm^-3]; q = (T_ref/T)^1.5 (partition-function ratio of
// Eq. (1)); G = u q / (pi dnu) with energies, u / (pi dnu) without.
__device__ inline float cell_G(double T, double x, double p, double T_ref, double dnu,
                               int have_E) {
  const double u = x * p * kAtm / (kBoltzmann * T) * 1e-6;
  const double q = have_E ? pow(T_ref / T, 1.5) : 1.0;
  return (float)(u * q / (M_PI * dnu));
}

__global__ void cell_params_kernel(int64_t n, const double* __restrict__ T,
                                   const double* __restrict__ x,
                                   const double* __restrict__ p, double T_ref,
                                   double dnu, double c2, int have_E,
                                   float* G, double* beta, double* theta,
                                   float* lam2, float* P) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  double Tc = T[c];
  G[c] = cell_G(Tc, x[c], p[c], T_ref, dnu, have_E);
  beta[c] = 1.0 / T_ref - 1.0 / Tc;
  theta[c] = c2 / Tc;
  lam2[c] = (float)log2(T_ref / Tc);
  P[c] = (float)(p[c] / dnu);
}

// The precision form's Gq = u q / (pi dnu) per cell, in FP32: u/(pi dnu) and
// log2(T_ref/T) come from the host, q = 2^(1.5 log2(T_ref/T)) with energies
// (the partition ratio of Eq. (1)), 1 without.
__global__ void cell_params32_kernel(int64_t n, const float* __restrict__ uf,
                                     const float* __restrict__ lamf, int have_E, float* Gq) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  Gq[c] = have_E ? uf[c] * fast_exp2(1.5f * lamf[c]) : uf[c];
}

// G of a further gas: its own mole fraction and partition-ratio choice.
__global__ void gas_factor_kernel(int64_t n, const double* __restrict__ T,
                                  const double* __restrict__ x, const double* __restrict__ p,
                                  double T_ref, double dnu, int have_E, float* G) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  G[c] = cell_G(T[c], x[c], p[c], T_ref, dnu, have_E);
}

struct KappaArgs {
  KappaTile t;
  int n_tiles;
  int tile_begin;
  TileGate gate;
  int parts = 1;             // line shares per tile, each into its own output
  int64_t part_stride = 0;   // floats between the shares' outputs
};

// The plain sum is held to 64 registers (eight wavefronts per SIMD), the
// compensated one needs more.
template <bool COMP, bool F32 = false, int P = kKappaPoints>
__global__ __launch_bounds__(kKappaThreads)
__attribute__((amdgpu_waves_per_eu(COMP ? 1 : 8))) void kappa_linesum_kernel(KappaArgs a) {
  __shared__ float4 lds4[kLineTile * (4 + 2 * kKappaCells) / 4];
  const int part = (int)(blockIdx.x % (unsigned)a.parts);
  const int64_t tb = blockIdx.x / (unsigned)a.parts;
  const int tile = (int)(tb % a.n_tiles);
  const int64_t cg = tb / a.n_tiles;
  constexpr int kTilePoints = kKappaThreads * P;
  const int j0 = (a.tile_begin + tile) * kTilePoints;
  bool wave_on = true;
  if (a.gate.group_flag || a.gate.chunk_err) {
    const bool marked = a.gate.group_flag && a.gate.group_flag[cg] == a.gate.epoch;
    bool need = marked;
    if (a.gate.chunk_err) {
      const int c0 = j0 / a.gate.chunk_w;
      const int c1 = min(a.gate.n_chunks - 1, (j0 + kTilePoints - 1) / a.gate.chunk_w);
      for (int k = c0; k <= c1; ++k) need = need || a.gate.chunk_err[k] > a.gate.tol;
      // a wavefront's 64 P points lie in one chunk when chunks are a
      // multiple of that span: then only the wavefronts of chunks over
      // tolerance (or of marked cells) evaluate and write; the others only
      // help stage the line records
      constexpr int kSpan = 64 * P;
      if (!marked && a.gate.chunk_w % kSpan == 0) {
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const int k = (j0 + wave * kSpan) / a.gate.chunk_w;
        wave_on = k < a.gate.n_chunks && a.gate.chunk_err[k] > a.gate.tol;
      }
    }
    if (!need) return;
  }
  if (a.parts > 1) {
    KappaTile t = a.t;
    t.line_parts = a.parts;
    t.line_part = part;
    t.out += part * a.part_stride;
    kappa_tile<COMP, F32, P>(t, j0, cg * kKappaCells, reinterpret_cast<float*>(lds4), wave_on);
    return;
  }
  kappa_tile<COMP, F32, P>(a.t, j0, cg * kKappaCells, reinterpret_cast<float*>(lds4), wave_on);
}

// Planck table: one block per (cell, 256-point segment of the row).
__global__ void planck_table_kernel(const float2* __restrict__ theta2, int64_t n_cells,
                                    int n_nu, int64_t ld, int tiles_per_row, float2 nu0,
                                    float2 dnu, float c1, float* __restrict__ B) {
  const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
  const int64_t cell = b / tiles_per_row;
  if (cell >= n_cells) return;
  const int64_t j = (b % tiles_per_row) * 256 + threadIdx.x;
  if (j >= ld) return;
  float v = 0.f;
  if (j < n_nu) v = planck_f32(nu_at(j, pair_of(nu0), pair_of(dnu)), pair_of(theta2[cell]), c1);
  B[cell * ld + j] = v;
}

// The walls' row B(nu_j, T_wall); theta_wall = c2 / T_wall (zero: cold walls).
__global__ void wall_table_kernel(float2 theta_wall, int n_nu, int64_t ld, float2 nu0,
                                  float2 dnu, float c1, float* bw) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ld) return;
  float v = 0.f;
  if (j < n_nu && theta_wall.x > 0.f)
    v = planck_f32(nu_at(j, pair_of(nu0), pair_of(dnu)), pair_of(theta_wall), c1);
  bw[j] = v;
}

// The paper's own formulation of Eq. (2) (Section 3 and its listing): line i
// contributes u S_i s_i(T) f_i(j) at the 16 grid points j = m_i - 7 .. m_i + 8,
// f_i the reference-state Lorentz shape tabulated once per line (prof16);
// u S s is the plain line sum's amplitude without the half width (G pi dnu S
// and the Eq. (1) factors).  One block per (8 cells, 256 points); the lines
// whose 16 points meet the block's points (tile16, found once per line list)
// are staged in LDS 128 at a time: m, the 16 values and the amplitude for
// each of the 8 cells.  Each thread owns one point of the 8 cells and sums
// over the staged lines that meet its wavefront's 64 points, one
// multiply-add per cell where its point is among a line's 16.  ACC adds to
// the rows (a further gas).
constexpr int kT16Points = 256;
constexpr int kT16Cells = 8;
constexpr int kT16Stage = 128;
template <bool ACC>
__global__ __launch_bounds__(kT16Points) void kappa_table16_kernel(
    LineSet L, CellSet C, int have_E, int64_t n_cells, int n_nu, int64_t ld, int n_tiles,
    double pi_dnu, float* __restrict__ out) {
  __shared__ int s_m[kT16Stage];
  __shared__ float s_tab[kT16Stage * 16];
  __shared__ float s_amp[kT16Stage * kT16Cells];
  const int tile = blockIdx.x % n_tiles;
  const int64_t cell0 = (int64_t)(blockIdx.x / n_tiles) * kT16Cells;
  const int tid = threadIdx.x;
  const int j = tile * kT16Points + tid;
  const int2 range = tile < L.n_tiles16 ? L.tile16[tile] : make_int2(0, 0);
  const int wj = __builtin_amdgcn_readfirstlane(tile * kT16Points + (tid & ~63));
  float acc[kT16Cells];
#pragma unroll
  for (int c = 0; c < kT16Cells; ++c) acc[c] = 0.f;
  for (int base = range.x; base < range.y; base += kT16Stage) {
    const int nt = min(kT16Stage, range.y - base);
    __syncthreads();
    for (int q = tid; q < nt * kT16Cells; q += kT16Points) {
      const int li = q / kT16Cells, cc = q % kT16Cells;
      const int i = base + li;
      const int64_t cell = min(cell0 + cc, n_cells - 1);
      float amp = (float)((double)C.G[cell] * pi_dnu) * L.S[i];
      if (have_E) {
        amp *= exp_split(L.E2[i] * C.beta[cell]);
        amp *= one_minus_exp_neg_d(L.nu[i] * C.theta[cell]);
      }
      s_amp[li * kT16Cells + cc] = amp;
      if (cc == 0) s_m[li] = L.m[i];
    }
    for (int q = tid; q < nt * 16; q += kT16Points) s_tab[q] = L.prof16[(int64_t)base * 16 + q];
    __syncthreads();
    // staged lines meeting this wavefront's points: m in [wj - 8, wj + 70]
    int l0 = 0, l1 = nt;
    {
      int a = 0, b = nt;
      while (a < b) { const int mid = (a + b) >> 1; if (s_m[mid] < wj - 8) a = mid + 1; else b = mid; }
      l0 = a;
      b = nt;
      while (a < b) { const int mid = (a + b) >> 1; if (s_m[mid] <= wj + 70) a = mid + 1; else b = mid; }
      l1 = a;
    }
    for (int li = l0; li < l1; ++li) {
      const int t = j - s_m[li] + 7;
      if (t >= 0 && t < 16) {
        const float f = s_tab[li * 16 + t];
#pragma unroll
        for (int c = 0; c < kT16Cells; ++c) acc[c] = fmaf(s_amp[li * kT16Cells + c], f, acc[c]);
      }
    }
  }
  if (j < ld) {
#pragma unroll
    for (int c = 0; c < kT16Cells; ++c) {
      const int64_t cell = cell0 + c;
      if (cell >= n_cells) break;
      float* o = out + cell * ld + j;
      const float v = j < n_nu ? acc[c] : 0.f;
      *o = ACC ? *o + v : v;
    }
  }
}

}  // namespace

hipError_t launch_kappa_table16(rt_ctx c) {
  const int n_tiles = (int)((c->ld + kT16Points - 1) / kT16Points);
  const int64_t blocks = (c->n_cells + kT16Cells - 1) / kT16Cells * n_tiles;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  const double pi_dnu = M_PI * c->dnu;
  hipLaunchKernelGGL((kappa_table16_kernel<false>), dim3((unsigned)blocks), dim3(kT16Points), 0,
                     c->stream, c->lines, c->cells, c->have_E ? 1 : 0, c->n_cells, c->n_nu,
                     c->ld, n_tiles, pi_dnu, c->kappa);
  hipError_t e = hipGetLastError();
  for (int g = 1; g < kMaxGases && e == hipSuccess; ++g) {
    const ExtraGas& gs = c->gas[g - 1];
    if (!gs.active) continue;
    CellSet cg = c->cells;
    cg.G = gs.G;
    hipLaunchKernelGGL((kappa_table16_kernel<true>), dim3((unsigned)blocks), dim3(kT16Points), 0,
                       c->stream, gs.lines, cg, gs.have_E ? 1 : 0, c->n_cells, c->n_nu, c->ld,
                       n_tiles, pi_dnu, c->kappa);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_cell_params(rt_ctx c) {
  const int64_t n = c->n_cells;
  const int threads = 256;
  const int64_t blocks = (n + threads - 1) / threads;
  hipLaunchKernelGGL(cell_params_kernel, dim3((unsigned)blocks), dim3(threads), 0, c->stream,
                     n, c->d_T, c->d_x, c->d_p, c->T_ref, c->dnu, second_radiation_cm_K(),
                     c->have_E ? 1 : 0, c->cells.G, c->cells.beta, c->cells.theta,
                     c->cells.lam2, c->cells.P);
  return hipGetLastError();
}

hipError_t launch_cell_params_on(rt_ctx c, int64_t n, const double* T, const double* x,
                                 const double* p, const CellSet& cells, hipStream_t s) {
  const int threads = 256;
  const int64_t blocks = (n + threads - 1) / threads;
  hipLaunchKernelGGL(cell_params_kernel, dim3((unsigned)blocks), dim3(threads), 0, s, n, T, x, p,
                     c->T_ref, c->dnu, second_radiation_cm_K(), c->have_E ? 1 : 0, cells.G,
                     cells.beta, cells.theta, cells.lam2, cells.P);
  return hipGetLastError();
}

hipError_t launch_cell_params32(rt_ctx c) {
  const int64_t n = c->n_cells;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(cell_params32_kernel, dim3(blocks), dim3(256), 0, c->stream, n, c->cells.uf,
                     c->cells.lamf, c->have_E ? 1 : 0, c->cells.Gq);
  for (int g = 1; g < kMaxGases; ++g) {
    const ExtraGas& gs = c->gas[g - 1];
    if (!gs.active) continue;
    hipLaunchKernelGGL(cell_params32_kernel, dim3(blocks), dim3(256), 0, c->stream, n, gs.uf,
                       c->cells.lamf, gs.have_E ? 1 : 0, gs.Gq);
  }
  return hipGetLastError();
}

hipError_t launch_gas_factor(rt_ctx c, int g) {
  const ExtraGas& gs = c->gas[g - 1];
  const int64_t n = c->n_cells;
  hipLaunchKernelGGL(gas_factor_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream,
                     n, c->d_T, gs.x, c->d_p, c->T_ref, c->dnu, gs.have_E ? 1 : 0, gs.G);
  return hipGetLastError();
}

hipError_t launch_kappa(rt_ctx c, bool compensated) {
  KappaArgs a;
  a.t.L = c->lines;
  a.t.C = c->cells;
  a.t.n_cells = c->n_cells;
  a.t.n_nu = c->n_nu;
  a.t.K = c->K;
  a.t.have_E = c->have_E ? 1 : 0;
  a.t.out = c->kappa;
  a.t.ld_out = c->ld;
  a.t.col0 = 0;
  a.t.col_end = c->ld;
  a.n_tiles = (int)((c->ld + kKappaTilePoints - 1) / kKappaTilePoints);
  a.tile_begin = 0;
  const int64_t groups = (c->n_cells + kKappaCells - 1) / kKappaCells;
  const int64_t blocks = groups * a.n_tiles;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  auto launch = [&]() {
    if (compensated)  // the precision form: FP32 line parameters
      hipLaunchKernelGGL((kappa_linesum_kernel<true, true>), dim3((unsigned)blocks),
                         dim3(kKappaThreads), 0, c->stream, a);
    else
      hipLaunchKernelGGL((kappa_linesum_kernel<false>), dim3((unsigned)blocks),
                         dim3(kKappaThreads), 0, c->stream, a);
    return hipGetLastError();
  };
  hipError_t e = launch();
  // further gases add their line sums, each with its own lines and G
  for (int g = 1; g < kMaxGases && e == hipSuccess; ++g) {
    const ExtraGas& gs = c->gas[g - 1];
    if (!gs.active) continue;
    a.t.L = gs.lines;
    a.t.C.G = gs.G;
    a.t.C.Gq = gs.Gq;
    a.t.have_E = gs.have_E ? 1 : 0;
    a.t.accumulate = 1;
    e = launch();
  }
  return e;
}

hipError_t launch_kappa_tiles(rt_ctx c, const KappaTile& t, int64_t n_cell_groups,
                              int tile_begin, int n_tiles, bool comp, hipStream_t s,
                              const TileGate& gate, int parts, int64_t part_stride) {
  KappaArgs a;
  a.t = t;
  a.gate = gate;
  a.n_tiles = n_tiles;
  a.tile_begin = tile_begin;
  a.parts = parts < 1 ? 1 : parts;
  a.part_stride = part_stride;
  const int64_t blocks = n_cell_groups * n_tiles * a.parts;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  if (blocks == 0) return hipSuccess;
  if (comp)
    hipLaunchKernelGGL((kappa_linesum_kernel<true>), dim3((unsigned)blocks), dim3(kKappaThreads),
                       0, s, a);
  else
    hipLaunchKernelGGL((kappa_linesum_kernel<false>), dim3((unsigned)blocks), dim3(kKappaThreads),
                       0, s, a);
  return hipGetLastError();
}

// The plain line sum in 256-point tiles of one point per lane: twice the
// blocks of launch_kappa_tiles, each with half its work, for launches that
// cover only part of the table (the learned form's fallback), where the
// latency of one block rather than the total work sets the time.  The
// values are the same bit for bit.
hipError_t launch_kappa_tiles_fine(rt_ctx c, const KappaTile& t, int64_t n_cell_groups,
                                   int n_tiles, hipStream_t s, const TileGate& gate) {
  KappaArgs a;
  a.t = t;
  a.gate = gate;
  a.n_tiles = n_tiles;
  a.tile_begin = 0;
  const int64_t blocks = n_cell_groups * n_tiles;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL((kappa_linesum_kernel<false, false, 1>), dim3((unsigned)blocks),
                     dim3(kKappaThreads), 0, s, a);
  return hipGetLastError();
}

// v as an FP32 pair hi + lo (host).
static float2 host_pair(double v) {
  const float h = (float)v;
  return make_float2(h, (float)(v - (double)h));
}

hipError_t launch_planck(rt_ctx c) {
  const float c1 = (float)first_radiation_wavenumber();
  const double c2 = second_radiation_cm_K();
  const float2 nu0 = host_pair(c->nu0), dnu = host_pair(c->dnu);
  const int tiles = (int)((c->ld + 255) / 256);
  if (c->planck) {
    const int64_t blocks = c->n_cells * tiles;
    const unsigned gx = (unsigned)std::min<int64_t>(blocks, 65536);
    const unsigned gy = (unsigned)((blocks + gx - 1) / gx);
    hipLaunchKernelGGL(planck_table_kernel, dim3(gx, gy), dim3(256), 0, c->stream,
                       c->cells.theta2, c->n_cells, c->n_nu, c->ld, tiles, nu0, dnu, c1,
                       c->planck);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const float2 theta_wall = c->T_wall > 0.0 ? host_pair(c2 / c->T_wall) : make_float2(0.f, 0.f);
  hipLaunchKernelGGL(wall_table_kernel, dim3((unsigned)((c->ld + 255) / 256)), dim3(256), 0,
                     c->stream, theta_wall, c->n_nu, c->ld, nu0, dnu, c1, c->d_bwall);
  return hipGetLastError();
}

}  // namespace rt
