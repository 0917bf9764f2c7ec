// surrogate.hip -- learned form of the line sum (gfx950).
//
// An MLP 4 -> 512 -> 512 -> 512 -> 256 (SiLU) maps the gas state and a
// spectral-chunk index, (T, x_H2O, p, k), encoded as (1/T, x, ln p, k), to
// the 256 values of
// ln(kappa / u) on chunk k, each output normalised by its mean and standard
// deviation over the training spectra; kappa = u exp(mean + std * y).
// Weights are BF16, products accumulate in FP32 on MFMA
// (v_mfma_f32_32x32x16_bf16); in training the first layer (K = 4) runs on
// the VALU, in inference on MFMA with exact BF16 splits of its inputs.
// Training data are spectra of the exact line sum (the same kernel as
// rt_compute_kappa) for caller-supplied gas states; training is plain Adam
// on the mean squared error of the normalised outputs, one training step
// captured in a HIP graph and replayed.
//
// Inference fills the kappa table; cells outside the training box are
// recomputed with the line sum; every chunk is checked against the line
// sum on a few sampled cells and recomputed for all cells when the relative
// error of its summed absorptance exceeds the tolerance.
#include <algorithm>
#include <type_traits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <string>
#include <vector>

#include "device_common.h"
#include "surrogate.h"

namespace rt {

hipError_t launch_cell_params_on(rt_ctx c, int64_t n, const double* T, const double* x,
                                 const double* p, const CellSet& cells, hipStream_t s);
// the plain line sum in 256-point tiles (kappa.hip)
hipError_t launch_kappa_tiles_fine(rt_ctx c, const dev::KappaTile& t, int64_t n_cell_groups,
                                   int n_tiles, hipStream_t s, const dev::TileGate& gate);

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// ------------------------------------------------------------------ GEMM
// C[m][n] = sum_r A[m][r] B[n][r] (both operands contiguous along r), FP32
// out.  Block = 4 wavefronts = 64 x 64 outputs, each wavefront a 32 x 32
// MFMA tile; operands are read straight from global memory (the layers are
// small and stay in L2).  M, N multiples of 64, R of 16.
__global__ __launch_bounds__(256) void gemm_nt_kernel(const bf16* __restrict__ A, int lda,
                                                      const bf16* __restrict__ B, int ldb,
                                                      float* __restrict__ C, int ldc, int R) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m0 = blockIdx.y * 64 + (wave >> 1) * 32;
  const int n0 = blockIdx.x * 64 + (wave & 1) * 32;
  const bf16* a = A + (size_t)(m0 + (lane & 31)) * lda + (lane >> 5) * 8;
  const bf16* b = B + (size_t)(n0 + (lane & 31)) * ldb + (lane >> 5) * 8;
  f32x16 acc;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.f;
  for (int r = 0; r < R; r += 16) {
    const bf16x8 av = *reinterpret_cast<const bf16x8*>(a + r);
    const bf16x8 bv = *reinterpret_cast<const bf16x8*>(b + r);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int row = m0 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
    C[(size_t)row * ldc + n0 + (lane & 31)] = acc[i];
  }
}

// logistic function from the hardware base-2 exponential and reciprocal
// (about 1 ulp each); training and inference use the same one
__device__ __forceinline__ float sigmoid(float z) {
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * z));
}

// Z = X0 W1 + b1 (K = 4, FP32 with BF16-rounded weights); H = SiLU(Z).
__global__ void layer1_kernel(const float* __restrict__ X0, const bf16* __restrict__ W1k,
                              const float* __restrict__ b1, int M, float* Z, bf16* H, bf16* HT) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int N = kMlpDims[1];
  if (i >= (int64_t)M * N) return;
  const int m = (int)(i / N), n = (int)(i % N);
  float z = b1[n];
#pragma unroll
  for (int k = 0; k < 4; ++k) z = fmaf(X0[4 * m + k], (float)W1k[k * N + n], z);
  const float h = z * sigmoid(z);
  if (Z) Z[i] = z;
  H[i] = (bf16)h;
  if (HT) HT[(int64_t)n * M + m] = (bf16)h;
}

// Z = C + b; H = SiLU(Z) (BF16, optionally transposed too); Z kept in C.
__global__ void bias_act_kernel(float* __restrict__ C, const float* __restrict__ b, int M, int N,
                                bf16* H, bf16* HT) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)M * N) return;
  const int m = (int)(i / N), n = (int)(i % N);
  const float z = C[i] + b[n];
  C[i] = z;
  const float h = z * sigmoid(z);
  H[i] = (bf16)h;
  if (HT) HT[(int64_t)n * M + m] = (bf16)h;
}

__global__ void bias_kernel(float* __restrict__ C, const float* __restrict__ b, int M, int N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)M * N) return;
  C[i] += b[i % N];
}

// dP = 2 (P - Y) / (M 256) on valid outputs (0 beyond n_nu); the squared
// error of each block, summed in FP64 in a fixed tree, is added into a
// fixed-point accumulator (sse: kAccDigits words, then an overflow word), so
// the reported loss does not depend on the order the blocks finish in.
__global__ void loss_grad_kernel(const float* __restrict__ P, const float* __restrict__ Y,
                                 const int32_t* __restrict__ row_chunk, int M, int n_nu,
                                 bf16* dP, bf16* dPT, unsigned long long* sse) {
  __shared__ double red[256];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double e2 = 0;
  if (i < (int64_t)M * kMlpWidth) {
    const int m = (int)(i / kMlpWidth), n = (int)(i % kMlpWidth);
    const bool valid = (int64_t)row_chunk[m] * kMlpWidth + n < n_nu;
    const float d = valid ? P[i] - Y[i] : 0.f;
    e2 = (double)d * d;
    const float g = 2.0f * d / ((float)M * kMlpWidth);
    dP[i] = (bf16)g;
    dPT[(int64_t)n * M + m] = (bf16)g;
  }
  red[threadIdx.x] = e2;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    dev::acc_add(sse, red[0], reinterpret_cast<unsigned*>(sse + kAccDigits));
}

// The loss accumulator as one FP64 value (carries propagated first).
__global__ void sse_value_kernel(unsigned long long* sse, double* out) {
  dev::acc_normalize(sse);
  *out = dev::acc_value(sse);
}

// dZ = dH * SiLU'(Z); BF16 (and transposed) or FP32 output.
__global__ void act_bwd_kernel(const float* __restrict__ dH, const float* __restrict__ Z, int M,
                               int N, bf16* dZ, bf16* dZT, float* dZf) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)M * N) return;
  const int m = (int)(i / N), n = (int)(i % N);
  const float z = Z[i];
  const float s = sigmoid(z);
  const float g = dH[i] * s * (1.0f + z * (1.0f - s));
  if (dZf) dZf[i] = g;
  if (dZ) dZ[i] = (bf16)g;
  if (dZT) dZT[(int64_t)n * M + m] = (bf16)g;
}

// Column sums in two passes with a fixed order (training repeats bit for
// bit): pass 1, one block per (64 columns, 64 rows), 4 row groups (rows g,
// g + 4, ...) reduced in LDS into part[row block][column]; pass 2 adds the
// row blocks' partials in order.
// db[n] = sum_m G[m][n] (FP32 or BF16 source), pass 1.
template <class T>
__global__ __launch_bounds__(256) void colsum_kernel(const T* __restrict__ G, int M, int N,
                                                     float* part) {
  __shared__ float red[4][64];
  const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + c;
  const int m0 = blockIdx.y * 64;
  float s = 0.f;
  if (n < N)
    for (int m = m0 + g; m < min(m0 + 64, M); m += 4) s += (float)G[(int64_t)m * N + n];
  red[g][c] = s;
  __syncthreads();
  if (g == 0 && n < N)
    part[(int64_t)blockIdx.y * N + n] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
}

// out[i] = sum_b part[b][i] over nb row blocks, in order (pass 2).
__global__ void sum_blocks_kernel(const float* __restrict__ part, int nb, int n, float* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int b = 0; b < nb; ++b) s += part[(int64_t)b * n + i];
  out[i] = s;
}

// dW1[k][n] = sum_m X0[m][k] dZ1[m][n] and db1[n] = sum_m dZ1[m][n], pass 1
// (part[row block][q][n], q = k or 4 for the bias), same decomposition.
__global__ __launch_bounds__(256) void layer1_wgrad_kernel(const float* __restrict__ X0,
                                                           const float* __restrict__ dZ1, int M,
                                                           float* part) {
  __shared__ float red[5][4][64];
  const int N = kMlpDims[1];
  const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + c;
  const int m0 = blockIdx.y * 64;
  float s[5] = {0, 0, 0, 0, 0};
  for (int m = m0 + g; m < min(m0 + 64, M); m += 4) {
    const float d = dZ1[(int64_t)m * N + n];
    for (int k = 0; k < 4; ++k) s[k] = fmaf(X0[4 * m + k], d, s[k]);
    s[4] += d;
  }
  for (int q = 0; q < 5; ++q) red[q][g][c] = s[q];
  __syncthreads();
  if (g == 0)
    for (int q = 0; q < 5; ++q)
      part[((int64_t)blockIdx.y * 5 + q) * N + n] =
          (red[q][0][c] + red[q][1][c]) + (red[q][2][c] + red[q][3][c]);
}

// dW1 [4][N] and db1 [N] from the pass-1 partials of layer1_wgrad_kernel.
__global__ void layer1_sum_kernel(const float* __restrict__ part, int nb, float* dW1, float* db1) {
  const int N = kMlpDims[1];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // q * N + n
  if (i >= 5 * N) return;
  float s = 0.f;
  for (int b = 0; b < nb; ++b) s += part[(int64_t)b * 5 * N + i];
  if (i < 4 * N) dW1[i] = s;
  else db1[i - 4 * N] = s;
}

__global__ void zero_f32_kernel(float* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

// Adam on W [K][N] (gradient given either as [K][N] or transposed [N][K])
// and its bias; refreshes the BF16 copies [N][K] and [K][N].  Cosine decay
// of the learning rate over total_steps.
__global__ void adam_kernel(float* W, float* mW, float* vW, const float* __restrict__ g,
                            int g_transposed, float* b, float* mb, float* vb,
                            const float* __restrict__ gb, int K, int N, const int* step,
                            int total_steps, float lr0, bf16* Wt, bf16* Wk) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const int t = *step + 1;
  const float lr = lr0 * 0.5f * (1.0f + cospif(fminf((float)(t - 1) / (float)total_steps, 1.0f)));
  const float c1 = 1.0f / (1.0f - powf(b1, (float)t)), c2 = 1.0f / (1.0f - powf(b2, (float)t));
  if (i < (int64_t)K * N) {
    const int k = (int)(i / N), n = (int)(i % N);
    const float gi = g_transposed ? g[(int64_t)n * K + k] : g[i];
    const float m = b1 * mW[i] + (1 - b1) * gi;
    const float v = b2 * vW[i] + (1 - b2) * gi * gi;
    mW[i] = m;
    vW[i] = v;
    const float w = W[i] - lr * (m * c1) / (sqrtf(v * c2) + eps);
    W[i] = w;
    Wt[(int64_t)n * K + k] = (bf16)w;
    Wk[i] = (bf16)w;
  }
  if (i < N) {
    const float m = b1 * mb[i] + (1 - b1) * gb[i];
    const float v = b2 * vb[i] + (1 - b2) * gb[i] * gb[i];
    mb[i] = m;
    vb[i] = v;
    b[i] -= lr * (m * c1) / (sqrtf(v * c2) + eps);
  }
}

__global__ void step_kernel(int* step) { *step += 1; }

__global__ void to_bf16_kernel(const float* __restrict__ W, int K, int N, bf16* Wt, bf16* Wk) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)K * N) return;
  const int k = (int)(i / N), n = (int)(i % N);
  Wt[(int64_t)n * K + k] = (bf16)W[i];
  Wk[i] = (bf16)W[i];
}

// W^T [N][512] (BF16) -> fragment order, see Surrogate::wf
__global__ void pack_fragments_kernel(const bf16* __restrict__ wt, int N, bf16* wf) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)N * 512) return;
  const int e = (int)(i & 7), l = (int)((i >> 3) & 63);
  const int64_t st = i >> 9;  // ct * 32 + s
  const int s = (int)(st & 31), ct = (int)(st >> 5);
  wf[i] = wt[(int64_t)(ct * 32 + (l & 31)) * 512 + s * 16 + (l >> 5) * 8 + e];
}

// Input encoding: 1/T, x and ln p, each mapped linearly onto [-1, 1] over
// the training box, and the chunk index onto [-1, 1].  ln(kappa/u) is close
// to linear in 1/T (Boltzmann factor of Eq. (1)) and in ln p (half widths).
struct Box { float T0, Ts, x0, xs, p0, ps; int n_chunks; };

__device__ __forceinline__ float chunk_feature(const Box& bx, int k) {
  return bx.n_chunks > 1 ? 2.0f * k / (float)(bx.n_chunks - 1) - 1.0f : 0.0f;
}

__device__ __forceinline__ void features(const Box& bx, double T, double x, double p, int k,
                                         float* f) {
  f[0] = ((float)(1.0 / T) - bx.T0) * bx.Ts;
  f[1] = ((float)x - bx.x0) * bx.xs;
  f[2] = ((float)log(p) - bx.p0) * bx.ps;
  f[3] = chunk_feature(bx, k);
}

// Training batch: rows perm[step*M .. +M) of the (sample, chunk) table.
__global__ void gather_kernel(const int32_t* __restrict__ perm, const int* step, int64_t n_rows,
                              int M, const double* __restrict__ T, const double* __restrict__ x,
                              const double* __restrict__ p, Box bx,
                              const float* __restrict__ Yall, int64_t ld_s, float* X0,
                              float* Y, int32_t* row_chunk) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)M * kMlpWidth) return;
  const int m = (int)(i / kMlpWidth), n = (int)(i % kMlpWidth);
  const int64_t row = perm[((int64_t)*step * M + m) % n_rows];
  const int64_t s = row / bx.n_chunks;
  const int k = (int)(row % bx.n_chunks);
  Y[i] = Yall[s * ld_s + (int64_t)k * kMlpWidth + n];
  if (n == 0) {
    float f[4];
    features(bx, T[s], x[s], p[s], k, f);
    for (int q = 0; q < 4; ++q) X0[4 * m + q] = f[q];
    row_chunk[m] = k;
  }
}

__device__ __forceinline__ double gas_density(double T, double x, double p) {
  return x * p * kAtm / (kBoltzmann * T) * 1e-6;
}

// ------------------------------------------------------------ fused inference
// One block of 8 wavefronts takes 32 RT rows (RT = 2 or 3) through all four
// layers.  The hidden activations stay in LDS as BF16 (each row padded by 8
// elements so that the fragment reads of 32 consecutive rows spread over the
// banks).  Each wavefront computes a 64-column slice of a layer (32 of the
// output layer) as RT x 2 (RT x 1) tiles of 32 x 32 MFMA with FP32
// accumulators, layer 1 included (its K = 4 padded to one K = 16 step with
// exact BF16 splits of the inputs and bias); its weight fragments are read
// from L2, where the 1.3 MB of BF16 weights stay.  The layers are computed
// transposed (see mfma_layer), so that each lane's results are runs of
// contiguous features of one row: the epilogues write 8-byte runs to LDS,
// and the output layer writes kappa straight from its accumulators.
// Layers 2-4 are the layer-by-layer kernels' arithmetic (the same products
// summed in the same k order, the same bias and SiLU); layer 1 sums its
// exact products in the MFMA instead of an FMA chain, which moves z by an
// FP32 rounding at most.
// Inputs are either given features (FROM_STATE false) or gas states and the
// chunk index of each row, chunk-major (row = k * n_cells + cell, so that the
// rows of a wavefront mostly share their chunk's output normalisation, read
// once per wavefront instead of gathered row by row); the output is either
// the raw last layer or kappa = u exp(mean + std * y), written straight into
// the table with zeros beyond n_nu.
constexpr int kFuseThreads = 512;  // 8 wavefronts
constexpr int kHidden = 512;
constexpr int kLdsRow = kHidden + 8;

struct FusedArgs {
  const bf16* W1k;  // [4][512]
  const float* b1;
  const bf16* wt2;  // fragment order (Surrogate::wf)
  const float* b2;
  const bf16* wt3;
  const float* b3;
  const bf16* wt4;
  const float* b4;
  int64_t rows;
  int64_t n_cells;  // FROM_STATE: rows = (chunks given to the network) x n_cells
  const float* X0;  // [rows][4] features
  // FROM_STATE: the cells' gas states, the training box, and the marks of
  // the cells outside it (and of their line-sum groups) with this call's
  // epoch, set by the rows of chunk 0
  const double* T;
  const double* x;
  const double* p;
  double T_lo, T_hi, x_lo, x_hi, p_lo, p_hi;
  unsigned epoch;
  unsigned* cell_flag;
  unsigned* group_flag;
  Box bx;
  float* P;         // [rows][256]
  const float* mean;
  const float* stdv;
  float* kappa;
  int64_t ld;
  int n_nu;
  // TO_KAPPA: the blocks past the network's, in this order, on the CUs the
  // network's blocks leave free:
  //   x_blocks = x_groups x x_tiles: the exact rows of the sampled cells (xt);
  //   tail_blocks: the exact line sum of every cell over the last chunk when
  //     the spectrum ends inside it (tt, 256-point tiles at tail_j0);
  //   wall_blocks: the walls' row B(nu_j, T_wall) of Eq. (4), 512 points each
  //     (theta = c2 / T_wall as an FP32 pair, zero for cold walls).
  int64_t net_blocks;
  dev::KappaTile xt;
  int x_tiles;
  int64_t x_blocks;
  dev::KappaTile tt;
  int tail_j0;
  int64_t tail_blocks;
  int64_t wall_blocks;
  float2 w_theta, w_nu0, w_dnu;
  float w_c1;
  float* wall;
};

// Points per lane of the exact rows computed beside the network (tiles of
// 256 kExactPoints points): few, long blocks, one per free CU.
constexpr int kExactPoints = 4;
static_assert(sizeof(bf16) * 64 * kLdsRow >= sizeof(float) * dev::kLineTile * dev::kLineRec,
              "the line-sum blocks stage their line records in the activations' LDS");

// The transposed product of one layer, Z^T += W^T H^T over K = 512, for RT
// row tiles x NT column tiles: the weights are the MFMA's A operand, the
// activations (rows of H) its B operand, so lane l of a 32 x 32 result tile
// holds row l % 32 and the 16 features 8 g + 4 (l / 32) + m (g, m < 4):
// four runs of four contiguous features of one row, which the epilogues
// store as whole runs.  Weights come in fragment order from L2, loaded
// kPrefetch k-steps ahead through a ring of registers (the k loop is
// unrolled so that every ring index is static), which covers the L2
// latency behind the MFMAs; activation fragments come from LDS one step
// ahead.
template <int RT>
constexpr int prefetch_steps() { return 8; }

template <int RT, int NT>
__device__ __forceinline__ void mfma_layer(const bf16* __restrict__ H, const bf16* __restrict__ wf,
                                           int n_base, int lane, f32x16 (&acc)[RT][NT]) {
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ct = 0; ct < NT; ++ct)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[rt][ct][i] = 0.f;
  const int r = lane & 31, kh = (lane >> 5) * 8;
  const bf16* hrow[RT];
  const bf16* wrow[NT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) hrow[rt] = H + (rt * 32 + r) * kLdsRow + kh;
#pragma unroll
  for (int ct = 0; ct < NT; ++ct) wrow[ct] = wf + ((size_t)(n_base / 32 + ct) * 32 * 64 + lane) * 8;
  constexpr int kSteps = kHidden / 16;
  constexpr int kPrefetch = prefetch_steps<RT>();
  bf16x8 bq[kPrefetch][NT];
  bf16x8 aq[2][RT];
#pragma unroll
  for (int d = 0; d < kPrefetch; ++d)
#pragma unroll
    for (int ct = 0; ct < NT; ++ct) bq[d][ct] = *reinterpret_cast<const bf16x8*>(wrow[ct] + d * 512);
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) aq[0][rt] = *reinterpret_cast<const bf16x8*>(hrow[rt]);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int st = 0; st < kSteps; ++st) {
    if (st + 1 < kSteps)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
        aq[(st + 1) & 1][rt] = *reinterpret_cast<const bf16x8*>(hrow[rt] + (st + 1) * 16);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < NT; ++ct)
        acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bq[st % kPrefetch][ct], aq[st & 1][rt],
                                                               acc[rt][ct], 0, 0, 0);
    if (st + kPrefetch < kSteps)
#pragma unroll
      for (int ct = 0; ct < NT; ++ct)
        bq[st % kPrefetch][ct] = *reinterpret_cast<const bf16x8*>(wrow[ct] + (st + kPrefetch) * 512);
    // keep each step's loads in its step: left free, the scheduler sinks
    // the weight loads to just before their MFMAs (to save registers), and
    // every k-step then waits a full L2 round trip
    __builtin_amdgcn_sched_barrier(0);
  }
}

__device__ __forceinline__ float f4_at(const float4& v, int m) {
  return m == 0 ? v.x : m == 1 ? v.y : m == 2 ? v.z : v.w;
}

// z (+ bias) -> SiLU(z) = z sigmoid(z) of a wavefront's transposed tiles
// into H as BF16: per row tile, column tile and g, one 8-byte run of four
// features.  Eight values at a time, so that the exponentials and
// reciprocals of independent values interleave.
template <int RT, int NT, bool BIAS>
__device__ __forceinline__ void silu_to_lds(const f32x16 (&acc)[RT][NT], const float* __restrict__ b,
                                            bf16* H, int n_base, int lane) {
  const int h = lane >> 5;
  float4 bb[NT][4];
#pragma unroll
  for (int ct = 0; ct < NT; ++ct)
#pragma unroll
    for (int g = 0; g < 4; ++g)
      bb[ct][g] = BIAS ? *reinterpret_cast<const float4*>(b + n_base + 32 * ct + 8 * g + 4 * h)
                       : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    bf16* hrow = H + (rt * 32 + (lane & 31)) * kLdsRow + n_base + 4 * h;
#pragma unroll
    for (int ct = 0; ct < NT; ++ct)
#pragma unroll
      for (int g2 = 0; g2 < 4; g2 += 2) {
        float z[8], e[8];
#pragma unroll
        for (int q = 0; q < 8; ++q)
          z[q] = acc[rt][ct][4 * g2 + q] + (BIAS ? f4_at(bb[ct][g2 + q / 4], q % 4) : 0.f);
#pragma unroll
        for (int q = 0; q < 8; ++q) e[q] = __builtin_amdgcn_exp2f(-1.4426950408889634f * z[q]);
#pragma unroll
        for (int q = 0; q < 8; ++q) e[q] = __builtin_amdgcn_rcpf(1.0f + e[q]);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          bf16x4 v;
#pragma unroll
          for (int m = 0; m < 4; ++m) v[m] = (bf16)(z[4 * u + m] * e[4 * u + m]);
          *reinterpret_cast<bf16x4*>(hrow + 32 * ct + 8 * (g2 + u)) = v;
        }
      }
  }
}

// x = hi + mid + lo in BF16 parts: hi and mid exact roundings of x and of
// x - hi (both differences are exact in FP32), lo the rounding of the rest
// (below 2^-26 |x|)
__device__ __forceinline__ void split3(float x, bf16& hi, bf16& mid, bf16& lo) {
  hi = (bf16)x;
  const float r = x - (float)hi;
  mid = (bf16)r;
  lo = (bf16)(r - (float)mid);
}

template <int RT, bool FROM_STATE, bool TO_KAPPA>
__global__ __launch_bounds__(kFuseThreads) void mlp_fused_kernel(FusedArgs a) {
  constexpr int kFuseRows = 32 * RT;
  __shared__ __align__(16) bf16 H[kFuseRows * kLdsRow];
  __shared__ __align__(16) float F[kFuseRows][4];
  __shared__ float U[kFuseRows];
  __shared__ int64_t RowBase[kFuseRows];  // kappa offset of the row's chunk (-1: no row)
  __shared__ int RowJ[kFuseRows];         // first wavenumber index of the row's chunk
  __shared__ int RowK[kFuseRows];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t row0 = (int64_t)blockIdx.x * kFuseRows;
  const int n_chunks = a.bx.n_chunks;
  const int h = lane >> 5;
  if (TO_KAPPA && (int64_t)blockIdx.x >= a.net_blocks) {
    int64_t xb = (int64_t)blockIdx.x - a.net_blocks;
    if (xb >= a.x_blocks + a.tail_blocks) {  // the walls' row
      const int64_t wb = xb - a.x_blocks - a.tail_blocks;
      if (a.net_blocks == 0) {
        // no network block clears the pitch columns [n_chunks 256, ld): these
        // blocks do, an equal share of the cells each
        const int64_t pad0 = (int64_t)n_chunks * kMlpWidth;
        const int64_t share = (a.n_cells + a.wall_blocks - 1) / a.wall_blocks;
        const int64_t c0 = wb * share, c1 = min(a.n_cells, c0 + share);
        for (int64_t c = c0; c < c1; ++c)
          for (int64_t j = pad0 + tid; j < a.ld; j += kFuseThreads) a.kappa[c * a.ld + j] = 0.f;
      }
      const int64_t j = wb * kFuseThreads + tid;
      if (j < a.ld) {
        float v = 0.f;
        if (j < a.n_nu && a.w_theta.x > 0.f)
          v = dev::planck_f32(dev::nu_at(j, dev::pair_of(a.w_nu0), dev::pair_of(a.w_dnu)),
                              dev::pair_of(a.w_theta), a.w_c1);
        a.wall[j] = v;
      }
      return;
    }
    // a line-sum block (Eq. (2)) over one tile of 8 cells, by its first four
    // wavefronts (the line sum's block shape; the others end here, and a
    // barrier waits only for the wavefronts still running), with the line
    // records staged in H
    if (wave >= dev::kKappaThreads / 64) return;
    float* lds = reinterpret_cast<float*>(H);
    if (xb < a.x_blocks) {
      const int tile = (int)(xb % a.x_tiles);
      dev::kappa_tile<false, false, kExactPoints>(a.xt, tile * dev::kKappaThreads * kExactPoints,
                                                  (xb / a.x_tiles) * dev::kKappaCells, lds);
    } else {
      dev::kappa_tile<false, false, 1>(a.tt, a.tail_j0, (xb - a.x_blocks) * dev::kKappaCells,
                                       lds);
    }
    return;
  }
  if (TO_KAPPA) {
    // the pitch columns [n_chunks 256, ld) of every cell are zero: each block
    // clears those of an equal share of the cells (no block is left with
    // more than a few rows of them)
    const int64_t pad0 = (int64_t)n_chunks * kMlpWidth;
    const int64_t share = (a.n_cells + a.net_blocks - 1) / a.net_blocks;
    const int64_t c0 = (int64_t)blockIdx.x * share, c1 = min(a.n_cells, c0 + share);
    for (int64_t c = c0; c < c1; ++c)
      for (int64_t j = pad0 + tid; j < a.ld; j += kFuseThreads) a.kappa[c * a.ld + j] = 0.f;
  }
  if (tid < kFuseRows) {
    const int64_t row = row0 + tid;
    float f[4] = {0.f, 0.f, 0.f, 0.f};
    float u = 0.f;
    int64_t base = -1;
    int k = 0;
    if (row < a.rows) {
      if (FROM_STATE) {
        k = (int)(row / a.n_cells);
        const int64_t cell = row - (int64_t)k * a.n_cells;
        const double t = a.T[cell], xc = a.x[cell], pc = a.p[cell];
        features(a.bx, t, xc, pc, k, f);
        u = (float)gas_density(t, xc, pc);
        base = cell * a.ld + (int64_t)k * kMlpWidth;
        if (k == 0 && !(t >= a.T_lo && t <= a.T_hi && xc >= a.x_lo && xc <= a.x_hi &&
                        pc >= a.p_lo && pc <= a.p_hi)) {
          a.cell_flag[cell] = a.epoch;
          a.group_flag[cell / dev::kKappaCells] = a.epoch;
        }
      } else {
        for (int q = 0; q < 4; ++q) f[q] = a.X0[4 * row + q];
        base = row * kMlpWidth;
      }
    }
    for (int q = 0; q < 4; ++q) F[tid][q] = f[q];
    U[tid] = u;
    RowBase[tid] = base;
    RowK[tid] = k;
    RowJ[tid] = k * kMlpWidth;
  }
  __syncthreads();
  // layer 1 (K = 4) as one K = 16 MFMA per tile, exact to FP32 rounding:
  //   k       0-3      4-7       8-11     12-14                15
  //   input   x_hi     x_mid     x_lo     1, 1, 1              0
  //   weight  W1       W1        W1       b_hi, b_mid, b_lo    0
  // (W1 is BF16 already; the bias is split like the inputs).  Wavefront w
  // computes columns [64 w, 64 w + 64).
  {
    const int n_base = wave * 64;
    bf16x8 wq[2];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const int n = n_base + 32 * ct + (lane & 31);
      bf16 w[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) w[k] = a.W1k[k * kHidden + n];
      bf16 bh, bm, bl;
      split3(a.b1[n], bh, bm, bl);
      const bf16 zero = (bf16)0.f;
      wq[ct] = h == 0 ? bf16x8{w[0], w[1], w[2], w[3], w[0], w[1], w[2], w[3]}
                      : bf16x8{w[0], w[1], w[2], w[3], bh, bm, bl, zero};
    }
    f32x16 acc[RT][2];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const float4 f = *reinterpret_cast<const float4*>(F[rt * 32 + (lane & 31)]);
      bf16 p[3][4];
      split3(f.x, p[0][0], p[1][0], p[2][0]);
      split3(f.y, p[0][1], p[1][1], p[2][1]);
      split3(f.z, p[0][2], p[1][2], p[2][2]);
      split3(f.w, p[0][3], p[1][3], p[2][3]);
      const bf16 one = (bf16)1.f, zero = (bf16)0.f;
      const bf16x8 xq = h == 0 ? bf16x8{p[0][0], p[0][1], p[0][2], p[0][3],
                                        p[1][0], p[1][1], p[1][2], p[1][3]}
                               : bf16x8{p[2][0], p[2][1], p[2][2], p[2][3], one, one, one, zero};
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[rt][ct][i] = 0.f;
        acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wq[ct], xq, acc[rt][ct], 0, 0, 0);
      }
    }
    silu_to_lds<RT, 2, false>(acc, nullptr, H, n_base, lane);
  }
  __syncthreads();
  // layers 2 and 3: wavefront w computes columns [64 w, 64 w + 64)
  for (int l = 0; l < 2; ++l) {
    const bf16* wt = l == 0 ? a.wt2 : a.wt3;
    const float* b = l == 0 ? a.b2 : a.b3;
    const int n_base = wave * 64;
    f32x16 acc[RT][2];
    mfma_layer<RT, 2>(H, wt, n_base, lane, acc);
    __syncthreads();  // every wavefront has read the layer input
    silu_to_lds<RT, 2, true>(acc, b, H, n_base, lane);
    __syncthreads();
  }
  // output layer (wavefront w: columns [32 w, 32 w + 32)), written straight
  // from the accumulators: per row tile and g, one 16-byte run of a row
  // (nothing is written to LDS any more, so no barrier follows)
  {
    const int n_base = wave * 32;
    f32x16 acc[RT][1];
    mfma_layer<RT, 1>(H, a.wt4, n_base, lane, acc);
    const float* __restrict__ mean = a.mean;
    const float* __restrict__ stdv = a.stdv;
    float4 bb[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) bb[g] = *reinterpret_cast<const float4*>(a.b4 + n_base + 8 * g + 4 * h);
    if (!TO_KAPPA) {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const int64_t base = RowBase[rt * 32 + (lane & 31)];
        if (base < 0) continue;
#pragma unroll
        for (int g = 0; g < 4; ++g)
          *reinterpret_cast<float4*>(a.P + base + n_base + 8 * g + 4 * h) =
              make_float4(acc[rt][0][4 * g] + bb[g].x, acc[rt][0][4 * g + 1] + bb[g].y,
                          acc[rt][0][4 * g + 2] + bb[g].z, acc[rt][0][4 * g + 3] + bb[g].w);
      }
    } else {
      // kappa = u exp(mean + std y), to ~1e-6 relative, far inside the
      // network's own error; zeros past n_nu.  The normalisation of every
      // row tile is loaded before any of it is used (one L2 round trip;
      // a missing row reads chunk 0's and stores nothing).
      float4 m[RT][4], sd[RT][4];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const int t0 = RowK[rt * 32 + (lane & 31)] * kMlpWidth + n_base + 4 * h;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          m[rt][g] = *reinterpret_cast<const float4*>(mean + t0 + 8 * g);
          sd[rt][g] = *reinterpret_cast<const float4*>(stdv + t0 + 8 * g);
        }
      }
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const int row = rt * 32 + (lane & 31);
        const int64_t base = RowBase[row];
        const float u = U[row];
        const int j0 = RowJ[row] + n_base + 4 * h;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int j = j0 + 8 * g;
          float v[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float y = acc[rt][0][4 * g + e] + f4_at(bb[g], e);
            v[e] = j + e < a.n_nu
                       ? u * __builtin_amdgcn_exp2f(1.4426950408889634f *
                                                    fmaf(f4_at(sd[rt][g], e), y, f4_at(m[rt][g], e)))
                       : 0.f;
          }
          if (base >= 0 && j < a.ld)
            *reinterpret_cast<float4*>(a.kappa + base + n_base + 8 * g + 4 * h) =
                make_float4(v[0], v[1], v[2], v[3]);
        }
      }
    }
  }
}

// Targets: y = ln(kappa / u) in place over the sample table; tiny floor.
__global__ void log_target_kernel(float* K, int64_t n_samples, int64_t ld_s, int n_nu,
                                  const double* __restrict__ T, const double* __restrict__ x,
                                  const double* __restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_samples * ld_s) return;
  const int64_t s = i / ld_s, j = i % ld_s;
  if (j >= n_nu) { K[i] = 0.f; return; }
  const double u = gas_density(T[s], x[s], p[s]);
  K[i] = (float)log(fmax((double)K[i] / u, 1e-45));
}

// mean and std per column over samples (FP64 sums), then normalise in place.
__global__ void col_stats_kernel(const float* __restrict__ Y, int64_t n_samples, int64_t ld_s,
                                 int n_cols, float* mean, float* stdv) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_cols) return;
  double s = 0, s2 = 0;
  for (int64_t r = 0; r < n_samples; ++r) {
    const double v = Y[r * ld_s + j];
    s += v;
    s2 += v * v;
  }
  const double m = s / n_samples;
  const double var = fmax(s2 / n_samples - m * m, 0.0);
  mean[j] = (float)m;
  stdv[j] = (float)fmax(sqrt(var), 1e-3);
}

__global__ void normalize_kernel(float* Y, int64_t n_samples, int64_t ld_s, int n_cols,
                                 const float* __restrict__ mean, const float* __restrict__ stdv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_samples * ld_s) return;
  const int j = (int)(i % ld_s);
  if (j < n_cols) Y[i] = (Y[i] - mean[j]) / stdv[j];
}

// out-of-range cells -> list

// per chunk: the relative error of the chunk's absorptance over the sampled
// cells, |sum (a_mlp - a)| / sum a with a = 1 - exp(-kappa l) along one
// cell edge l -- the quantity the absorbed and emitted power are linear in
// for thin points and saturate in for thick ones.  Cells outside the
// training box (recomputed exactly anyway) are left out.
// The check's exact rows arrive as `parts` partial sums over shares of the
// lines (parts blocks per line-sum tile keep the GPU busy on a few sampled
// cells); they are added into the first share, in share order.
__global__ __launch_bounds__(256) void sum_parts_kernel(float* __restrict__ x, int64_t n, int parts,
                                                        int64_t stride) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  float v = x[i];
  for (int q = 1; q < parts; ++q) v += x[q * stride + i];
  x[i] = v;
}

// One block of 1024 threads per chunk: thread t owns point k * 256 + t % 256
// of the sampled cells t / 256, t / 256 + 4, ...; each wavefront sums its
// lanes with a fixed butterfly, and thread 0 adds the 16 wavefront sums in
// order (the same order on every call).
constexpr int kCheckThreads = 1024;
__global__ __launch_bounds__(kCheckThreads) void check_kernel(
    const float* __restrict__ kappa, int64_t ld, const float* __restrict__ exact, int64_t ld_e,
    const int32_t* __restrict__ cells, int n_check, int n_nu, float l_cm,
    const unsigned* __restrict__ cell_flag, unsigned epoch, float* err) {
  const int k = blockIdx.x;  // chunk
  const int t = threadIdx.x;
  constexpr int kGroups = kCheckThreads / kMlpWidth;
  constexpr int kWaves = kCheckThreads / 64;
  __shared__ int64_t row[kMaxCheckCells];  // kappa row offset, -1: left out
  __shared__ float rd[kWaves], rs[kWaves];
  for (int ci = t; ci < n_check; ci += kCheckThreads) {
    const int cell = cells[ci];
    row[ci] = cell_flag[cell] == epoch ? -1 : (int64_t)cell * ld;
  }
  __syncthreads();
  const int j = k * kMlpWidth + (t % kMlpWidth);
  float d = 0, s = 0;
  if (j < n_nu) {
    // kU cells at a time, their loads issued together
    constexpr int kU = 8;
    for (int c0 = t / kMlpWidth; c0 < n_check; c0 += kGroups * kU) {
      float ev[kU], gv[kU];
      bool on[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int ci = c0 + u * kGroups;
        on[u] = ci < n_check && row[ci] >= 0;
        ev[u] = on[u] ? exact[(int64_t)ci * ld_e + j] : 0.f;
        gv[u] = on[u] ? kappa[row[ci] + j] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        if (!on[u]) continue;
        const float e = -expm1f(-ev[u] * l_cm);
        const float g = -expm1f(-gv[u] * l_cm);
        d += g - e;
        s += e;
      }
    }
  }
  // every lane ends with the same sums (a + b == b + a)
  for (int off = 32; off > 0; off >>= 1) {
    d += __shfl_xor(d, off);
    s += __shfl_xor(s, off);
  }
  if ((t & 63) == 0) {
    rd[t >> 6] = d;
    rs[t >> 6] = s;
  }
  __syncthreads();
  if (t == 0) {
    float D = 0, S = 0;
    for (int w = 0; w < kWaves; ++w) {
      D += rd[w];
      S += rs[w];
    }
    err[k] = S > 0 ? fabsf(D) / S : (D != 0 ? 1e30f : 0.0f);
  }
}

int64_t grid1(int64_t n) { return (n + 255) / 256; }

// v as an FP32 pair hi + lo.
float2 host_pair(double v) {
  const float h = (float)v;
  return make_float2(h, (float)(v - (double)h));
}


// deterministic 64-bit generator for weight init and shuffles (splitmix64)
struct SplitMix {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
  }
  double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

rt_status sfail(rt_ctx c, rt_status s, const std::string& m) {
  c->err = m;
  return s;
}

#define RT_SHIP(ctx, call)                                                              \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return (void)hipGetLastError(), /* not left for the next launch check */          \
             sfail(ctx, (e_ == hipErrorOutOfMemory) ? RT_ENOMEM : RT_EDEVICE,           \
                   std::string(#call) + ": " + hipGetErrorString(e_));                  \
  } while (0)

template <class T>
hipError_t dalloc(T** p, int64_t n) {
  *p = nullptr;
  const hipError_t e = hipMalloc(reinterpret_cast<void**>(p), (size_t)std::max<int64_t>(n, 1) * sizeof(T));
  if (e != hipSuccess) (void)hipGetLastError();  // not left for the next launch check
  return e;
}
template <class T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

rt_status alloc_params(rt_ctx c, Surrogate& S) {
  S.param_count = 0;
  for (int l = 0; l < kMlpLayers; ++l) {
    const int K = kMlpDims[l], N = kMlpDims[l + 1];
    RT_SHIP(c, dalloc(&S.w[l], (int64_t)K * N));
    RT_SHIP(c, dalloc(&S.b[l], N));
    RT_SHIP(c, dalloc(&S.mw[l], (int64_t)K * N));
    RT_SHIP(c, dalloc(&S.vw[l], (int64_t)K * N));
    RT_SHIP(c, dalloc(&S.mb[l], N));
    RT_SHIP(c, dalloc(&S.vb[l], N));
    RT_SHIP(c, dalloc(&S.wt[l], (int64_t)K * N));
    RT_SHIP(c, dalloc(&S.wk[l], (int64_t)K * N));
    if (l > 0) RT_SHIP(c, dalloc(&S.wf[l], (int64_t)K * N));
    S.param_count += (int64_t)K * N + N;
  }
  RT_SHIP(c, dalloc(&S.mean, (int64_t)S.n_chunks * kMlpWidth));
  RT_SHIP(c, dalloc(&S.stdv, (int64_t)S.n_chunks * kMlpWidth));
  return RT_OK;
}

// Activation buffers for M rows.
struct Acts {
  int M = 0;
  float *X0 = nullptr, *Z[3] = {}, *P = nullptr, *Y = nullptr, *dH = nullptr, *dZ1 = nullptr;
  bf16 *H[3] = {}, *HT[3] = {}, *dP = nullptr, *dPT = nullptr, *dZ[3] = {}, *dZT[3] = {};
  float *gW[kMlpLayers] = {}, *gb[kMlpLayers] = {};
  float* part = nullptr;  // column-sum partials: [M / 64][5][512]
  int32_t* row_chunk = nullptr;
  unsigned long long* sse = nullptr;  // kAccDigits + 1 words (see loss_grad_kernel)
  double* sse_value = nullptr;
  int* step = nullptr;
  void release() {
    dfree(X0); dfree(P); dfree(Y); dfree(dH); dfree(dZ1); dfree(dP); dfree(dPT);
    for (int l = 0; l < 3; ++l) { dfree(Z[l]); dfree(H[l]); dfree(HT[l]); dfree(dZ[l]); dfree(dZT[l]); }
    for (int l = 0; l < kMlpLayers; ++l) { dfree(gW[l]); dfree(gb[l]); }
    dfree(part);
    dfree(row_chunk); dfree(sse); dfree(sse_value); dfree(step);
  }
};

rt_status alloc_acts(rt_ctx c, Acts& a, int M, bool train) {
  a.M = M;
  const int W = 512;
  RT_SHIP(c, dalloc(&a.X0, (int64_t)M * 4));
  RT_SHIP(c, dalloc(&a.P, (int64_t)M * kMlpWidth));
  for (int l = 0; l < 3; ++l) {
    RT_SHIP(c, dalloc(&a.Z[l], (int64_t)M * W));
    RT_SHIP(c, dalloc(&a.H[l], (int64_t)M * W));
  }
  if (!train) return RT_OK;
  RT_SHIP(c, dalloc(&a.Y, (int64_t)M * kMlpWidth));
  RT_SHIP(c, dalloc(&a.dH, (int64_t)M * W));
  RT_SHIP(c, dalloc(&a.dZ1, (int64_t)M * W));
  RT_SHIP(c, dalloc(&a.part, (int64_t)(M / 64) * 5 * W));
  RT_SHIP(c, dalloc(&a.dP, (int64_t)M * kMlpWidth));
  RT_SHIP(c, dalloc(&a.dPT, (int64_t)M * kMlpWidth));
  for (int l = 0; l < 3; ++l) {
    RT_SHIP(c, dalloc(&a.HT[l], (int64_t)M * W));
    RT_SHIP(c, dalloc(&a.dZ[l], (int64_t)M * W));
    RT_SHIP(c, dalloc(&a.dZT[l], (int64_t)M * W));
  }
  for (int l = 0; l < kMlpLayers; ++l) {
    RT_SHIP(c, dalloc(&a.gW[l], (int64_t)kMlpDims[l] * kMlpDims[l + 1]));
    RT_SHIP(c, dalloc(&a.gb[l], kMlpDims[l + 1]));
  }
  RT_SHIP(c, dalloc(&a.row_chunk, M));
  RT_SHIP(c, dalloc(&a.sse, kAccDigits + 1));
  RT_SHIP(c, dalloc(&a.sse_value, 1));
  RT_SHIP(c, dalloc(&a.step, 1));
  return RT_OK;
}

void gemm(const bf16* A, int lda, const bf16* B, int ldb, float* C, int ldc, int M, int N, int R,
          hipStream_t s) {
  hipLaunchKernelGGL(gemm_nt_kernel, dim3(N / 64, M / 64), dim3(256), 0, s, A, lda, B, ldb, C,
                     ldc, R);
}

// forward pass over a.M rows (X0 filled); train: keep transposes
void forward(const Surrogate& S, Acts& a, bool train, hipStream_t s) {
  const int M = a.M, W = 512;
  hipLaunchKernelGGL(layer1_kernel, dim3(grid1((int64_t)M * W)), dim3(256), 0, s, a.X0, S.wk[0],
                     S.b[0], M, a.Z[0], a.H[0], train ? a.HT[0] : nullptr);
  for (int l = 1; l <= 2; ++l) {
    gemm(a.H[l - 1], W, S.wt[l], W, a.Z[l], W, M, W, W, s);
    hipLaunchKernelGGL(bias_act_kernel, dim3(grid1((int64_t)M * W)), dim3(256), 0, s, a.Z[l],
                       S.b[l], M, W, a.H[l], train ? a.HT[l] : nullptr);
  }
  gemm(a.H[2], W, S.wt[3], W, a.P, kMlpWidth, M, kMlpWidth, W, s);
  hipLaunchKernelGGL(bias_kernel, dim3(grid1((int64_t)M * kMlpWidth)), dim3(256), 0, s, a.P,
                     S.b[3], M, kMlpWidth);
}

void colsum_bf16(const bf16* G, int M, int N, float* part, float* db, hipStream_t s) {
  hipLaunchKernelGGL(colsum_kernel<bf16>, dim3((N + 63) / 64, M / 64), dim3(256), 0, s, G, M, N,
                     part);
  hipLaunchKernelGGL(sum_blocks_kernel, dim3((N + 255) / 256), dim3(256), 0, s, part, M / 64, N,
                     db);
}

void backward(const Surrogate& S, Acts& a, hipStream_t s) {
  const int M = a.M, W = 512, O = kMlpWidth;
  // layer 4: dW4^T [256][512] = dP^T H3^T^T ; dH3 = dP W4
  gemm(a.dPT, M, a.HT[2], M, a.gW[3], W, O, W, M, s);
  colsum_bf16(a.dP, M, O, a.part, a.gb[3], s);
  gemm(a.dP, O, S.wk[3], O, a.dH, W, M, W, O, s);
  for (int l = 2; l >= 1; --l) {  // hidden layers 3 and 2
    hipLaunchKernelGGL(act_bwd_kernel, dim3(grid1((int64_t)M * W)), dim3(256), 0, s, a.dH,
                       a.Z[l], M, W, a.dZ[l], a.dZT[l], (float*)nullptr);
    gemm(a.dZT[l], M, a.HT[l - 1], M, a.gW[l], W, W, W, M, s);
    colsum_bf16(a.dZ[l], M, W, a.part, a.gb[l], s);
    gemm(a.dZ[l], W, S.wk[l], W, a.dH, W, M, W, W, s);
  }
  hipLaunchKernelGGL(act_bwd_kernel, dim3(grid1((int64_t)M * W)), dim3(256), 0, s, a.dH, a.Z[0],
                     M, W, (bf16*)nullptr, (bf16*)nullptr, a.dZ1);
  hipLaunchKernelGGL(layer1_wgrad_kernel, dim3(W / 64, M / 64), dim3(256), 0, s, a.X0, a.dZ1, M,
                     a.part);
  hipLaunchKernelGGL(layer1_sum_kernel, dim3((5 * W + 255) / 256), dim3(256), 0, s, a.part, M / 64,
                     a.gW[0], a.gb[0]);
}

void adam(Surrogate& S, Acts& a, int total_steps, float lr, hipStream_t s) {
  for (int l = 0; l < kMlpLayers; ++l) {
    const int K = kMlpDims[l], N = kMlpDims[l + 1];
    hipLaunchKernelGGL(adam_kernel, dim3(grid1((int64_t)K * N)), dim3(256), 0, s, S.w[l],
                       S.mw[l], S.vw[l], a.gW[l], l == 0 ? 0 : 1, S.b[l], S.mb[l], S.vb[l],
                       a.gb[l], K, N, a.step, total_steps, lr, S.wt[l], S.wk[l]);
  }
  hipLaunchKernelGGL(step_kernel, dim3(1), dim3(1), 0, s, a.step);
}

Box make_box(const Surrogate& S) {
  Box b;
  const double u0 = 1.0 / S.T_max, u1 = 1.0 / S.T_min;
  b.T0 = (float)(0.5 * (u0 + u1));
  b.Ts = (float)(2.0 / (u1 - u0));
  b.x0 = (float)(0.5 * (S.x_min + S.x_max));
  b.xs = (float)(S.x_max > S.x_min ? 2.0 / (S.x_max - S.x_min) : 0.0);
  const double l0 = std::log(S.p_min), l1 = std::log(S.p_max);
  b.p0 = (float)(0.5 * (l0 + l1));
  b.ps = (float)(2.0 / (l1 - l0));
  b.n_chunks = S.n_chunks;
  return b;
}

Surrogate& surrogate(rt_ctx c) {
  if (!c->surrogate) c->surrogate = new Surrogate();
  return *c->surrogate;
}

uint64_t fnv1a(const void* p, size_t n, uint64_t h = 14695981039346656037ULL) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) { h ^= b[i]; h *= 1099511628211ULL; }
  return h;
}

void pack_weights(const Surrogate& S, hipStream_t s) {
  for (int l = 1; l < kMlpLayers; ++l) {
    const int N = kMlpDims[l + 1];
    hipLaunchKernelGGL(pack_fragments_kernel, dim3(grid1((int64_t)N * 512)), dim3(256), 0, s,
                       S.wt[l], N, S.wf[l]);
  }
}

// The fused kernel over `rows` rows: features X0 or gas states in, raw
// outputs P or the kappa table out.
// What an inference launch does besides the network (see FusedArgs).
struct InferJob {
  int64_t n_cells;
  unsigned epoch;
  const dev::KappaTile* xt = nullptr;  // exact rows of the sampled cells
  int64_t x_groups = 0;
  const dev::KappaTile* tt = nullptr;  // the last chunk's exact line sum
  int tail_j0 = 0;
  int64_t tail_groups = 0;
};

// job null: the network alone on given features, raw outputs into P.
// Otherwise inference from the cells' states into the kappa table, with the
// job's line-sum blocks and the walls' row in the same launch.
void launch_fused(rt_ctx c, const Surrogate& S, int64_t rows, const float* X0, float* P,
                  hipStream_t s, const InferJob* job) {
  FusedArgs a;
  a.W1k = S.wk[0]; a.b1 = S.b[0];
  a.wt2 = S.wf[1]; a.b2 = S.b[1];
  a.wt3 = S.wf[2]; a.b3 = S.b[2];
  a.wt4 = S.wf[3]; a.b4 = S.b[3];
  a.rows = rows;
  a.n_cells = job ? job->n_cells : 0;
  a.X0 = X0;
  a.T = c->d_T; a.x = c->d_x; a.p = c->d_p;
  a.T_lo = S.T_min; a.T_hi = S.T_max;
  a.x_lo = S.x_min; a.x_hi = S.x_max;
  a.p_lo = S.p_min; a.p_hi = S.p_max;
  a.epoch = job ? job->epoch : 0;
  a.cell_flag = S.d_cell_flag;
  a.group_flag = S.d_group_flag;
  a.bx = make_box(S);
  a.P = P;
  a.mean = S.mean; a.stdv = S.stdv;
  a.kappa = c->kappa; a.ld = c->ld; a.n_nu = c->n_nu;
  // rows per block 32 RT; either size holds one block per CU (registers:
  // two wavefronts per SIMD); pick the size with the fewest row tiles on the
  // busiest CU (on a tie, the fewest weight reads)
  const int64_t cus = 256;
  int best = 2;
  double best_cost = 1e300;
  for (int rt : {2, 3}) {
    const int64_t blocks = (rows + 32 * rt - 1) / (32 * rt);
    const double cost = (double)((blocks + cus - 1) / cus) * rt - 1e-3 * rt;
    if (cost < best_cost) { best_cost = cost; best = rt; }
  }
  const dim3 t(kFuseThreads);
  a.x_tiles = 1;
  a.x_blocks = a.tail_blocks = a.wall_blocks = 0;
  if (job) {
    if (job->xt && job->x_groups > 0) {
      a.xt = *job->xt;
      a.x_tiles = (int)((c->ld + dev::kKappaThreads * kExactPoints - 1) /
                        (dev::kKappaThreads * kExactPoints));
      a.x_blocks = job->x_groups * a.x_tiles;
    }
    if (job->tt && job->tail_groups > 0) {
      a.tt = *job->tt;
      a.tail_j0 = job->tail_j0;
      a.tail_blocks = job->tail_groups;
    }
    a.wall_blocks = (c->ld + kFuseThreads - 1) / kFuseThreads;
    a.w_theta = c->T_wall > 0.0 ? host_pair(second_radiation_cm_K() / c->T_wall)
                                : make_float2(0.f, 0.f);
    a.w_nu0 = host_pair(c->nu0);
    a.w_dnu = host_pair(c->dnu);
    a.w_c1 = (float)first_radiation_wavenumber();
    a.wall = c->d_bwall;
  }
  auto go = [&](auto rt_tag) {
    constexpr int RT = decltype(rt_tag)::value;
    a.net_blocks = (rows + 32 * RT - 1) / (32 * RT);
    const dim3 g((unsigned)(a.net_blocks + a.x_blocks + a.tail_blocks + a.wall_blocks));
    if (job) hipLaunchKernelGGL((mlp_fused_kernel<RT, true, true>), g, t, 0, s, a);
    else hipLaunchKernelGGL((mlp_fused_kernel<RT, false, false>), g, t, 0, s, a);
  };
  if (best == 2) go(std::integral_constant<int, 2>());
  else go(std::integral_constant<int, 3>());
}

}  // namespace

void free_surrogate(rt_ctx c) {
  if (!c->surrogate) return;
  Surrogate& S = *c->surrogate;
  for (int l = 0; l < kMlpLayers; ++l) {
    dfree(S.w[l]); dfree(S.b[l]); dfree(S.mw[l]); dfree(S.vw[l]); dfree(S.mb[l]); dfree(S.vb[l]);
    dfree(S.wt[l]); dfree(S.wk[l]); dfree(S.wf[l]);
  }
  dfree(S.mean); dfree(S.stdv);
  dfree(S.d_cell_flag); dfree(S.d_group_flag); dfree(S.d_err); dfree(S.d_check);
  dfree(S.d_exact);
  for (auto& e : S.ev)
    if (e) (void)hipEventDestroy(e);
  if (S.fork) (void)hipEventDestroy(S.fork);
  if (S.join) (void)hipEventDestroy(S.join);
  if (S.side) (void)hipStreamDestroy(S.side);
  delete c->surrogate;
  c->surrogate = nullptr;
}

bool surrogate_ready(rt_ctx c) {
  return c->surrogate && c->surrogate->trained && c->surrogate->n_nu == c->n_nu;
}

// Learned kappa into c->kappa, stream-ordered launches with every decision
// taken on the device (no host round trip):
//   1. one launch: the fused network writes kappa and marks cells outside
//      the training box (and their line-sum groups) with this call's epoch;
//      beside it, on the CUs its blocks leave free, the exact rows of the
//      sampled cells (with long line lists: on a second stream instead,
//      forked before the launch and joined before 2), a last chunk that the
//      spectrum ends inside (light line lists) and the walls' row;
//   2. the checked error per chunk (marked cells left out);
//   3. the line sum over every tile that touches a chunk over tolerance or a
//      marked group of cells.
// Line shares per tile of the check's line sum: enough blocks (about 2,048)
// that a few sampled cells do not leave most of the GPU idle, but no share
// under about 128 lines (a tile's window meets n (512 + 2K) / n_nu lines on
// average), and at most 32.
// Lines whose window meets a line-sum tile of kKappaTilePoints points, on
// average over the spectrum.
double lines_per_tile(rt_ctx c) {
  return (double)c->lines.n * (dev::kKappaTilePoints + 2.0 * c->K) / std::max(1, c->n_nu);
}

int check_parts(rt_ctx c, int n_check) {
  const int64_t tiles = (c->ld + dev::kKappaTilePoints - 1) / dev::kKappaTilePoints;
  const int64_t blocks = (int64_t)((n_check + dev::kKappaCells - 1) / dev::kKappaCells) * tiles;
  if (blocks <= 0) return 1;
  const int64_t by_lines = (int64_t)(lines_per_tile(c) / 128.0);
  const int64_t by_blocks = (2048 + blocks - 1) / blocks;
  return (int)std::max<int64_t>(1, std::min<int64_t>(32, std::min(by_lines, by_blocks)));
}

// 1 when the spectrum ends inside the last 256-point chunk and the line
// list is light (fewer than 256 lines meet a tile, as when the check's exact
// rows run in the network's launch): that chunk is then summed exactly beside
// the network; else 0 (with many lines per point its blocks would outlast
// the network).
int exact_tail_chunks(rt_ctx c, const Surrogate& S) {
  return S.n_chunks > 0 && (int64_t)S.n_chunks * kMlpWidth > c->n_nu &&
                 lines_per_tile(c) < 256.0
             ? 1
             : 0;
}

// The counts and timings are read back lazily by rt_surrogate_get_stats.
// Called by rt_compute_kappa in surrogate mode.
rt_status surrogate_kappa(rt_ctx c) {
  Surrogate& S = *c->surrogate;
  const int64_t n_cells = c->n_cells;
  const int64_t rows = n_cells * S.n_chunks;
  if (rows > (int64_t)1 << 28) return sfail(c, RT_EINVAL, "surrogate: too many (cell, chunk) rows");
  const int n_check = (int)std::min<int64_t>(S.check_cells, n_cells);
  const int64_t groups_all = (n_cells + dev::kKappaCells - 1) / dev::kKappaCells;
  auto chk = [&](hipError_t e) { return e == hipSuccess; };
  hipStream_t s = c->stream;
  bool ok = true;
  if (S.inf_cells != n_cells || S.inf_ld != c->ld || S.inf_check != n_check ||
      S.inf_chunks != S.n_chunks || !S.d_cell_flag) {
    dfree(S.d_cell_flag); dfree(S.d_group_flag); dfree(S.d_err); dfree(S.d_check);
    dfree(S.d_exact);
    ok = chk(dalloc(&S.d_cell_flag, n_cells)) && chk(dalloc(&S.d_group_flag, groups_all)) &&
         chk(dalloc(&S.d_err, S.n_chunks)) && chk(dalloc(&S.d_check, std::max(1, n_check))) &&
         chk(dalloc(&S.d_exact, std::max<int64_t>(1, (int64_t)check_parts(c, n_check) * n_check * c->ld)));
    // marks start at 0, which no call uses as its epoch
    ok = ok && chk(hipMemsetAsync(S.d_cell_flag, 0, n_cells * 4, s)) &&
         chk(hipMemsetAsync(S.d_group_flag, 0, groups_all * 4, s));
    if (!ok) return sfail(c, RT_ENOMEM, "surrogate inference: device allocation failed");
    S.inf_cells = n_cells;
    S.inf_ld = c->ld;
    S.inf_check = n_check;
    S.inf_chunks = S.n_chunks;
    S.pick_epoch = ~0ull;
  }
  for (auto& e : S.ev)
    if (!e && hipEventCreate(&e) != hipSuccess) return sfail(c, RT_EDEVICE, "surrogate: event");
  if (!S.side) {
    if (hipStreamCreateWithFlags(&S.side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&S.fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&S.join, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      return sfail(c, RT_EDEVICE, "surrogate: side stream");
    }
  }

  if (S.pick_epoch != c->grid_epoch && n_check > 0) {
    // sampled cells: the coldest and the hottest (where the network is least
    // constrained), then uniformly drawn cells
    std::vector<int32_t> pick;
    for (int64_t e : {c->T_argmin, c->T_argmax})
      if ((int)pick.size() < n_check && std::find(pick.begin(), pick.end(), (int32_t)e) == pick.end())
        pick.push_back((int32_t)e);
    SplitMix g{S.check_seed ^ 0xC0FFEEULL};
    std::vector<int32_t> all(n_cells);
    for (int64_t i = 0; i < n_cells; ++i) all[i] = (int32_t)i;
    for (int i = 0; (int)pick.size() < n_check && i < n_cells; ++i) {
      const int64_t r = i + (int64_t)(g.uniform() * (double)(n_cells - i));
      std::swap(all[i], all[std::min<int64_t>(r, n_cells - 1)]);
      if (std::find(pick.begin(), pick.end(), all[i]) == pick.end()) pick.push_back(all[i]);
    }
    ok = chk(hipMemcpyAsync(S.d_check, pick.data(), pick.size() * 4, hipMemcpyHostToDevice, s)) &&
         chk(hipStreamSynchronize(s));  // the host vector goes out of scope
    if (!ok) return sfail(c, RT_EDEVICE, "surrogate inference: copy of the sampled cells failed");
    S.pick_epoch = c->grid_epoch;
  }
  S.epoch = S.epoch + 1 == 0 ? 1 : S.epoch + 1;
  dev::KappaTile t;
  t.L = c->lines;
  t.C = c->cells;
  t.n_cells = n_cells;
  t.n_nu = c->n_nu;
  t.K = c->K;
  t.have_E = c->have_E ? 1 : 0;
  t.out = c->kappa;
  t.ld_out = c->ld;
  t.col0 = 0;
  t.col_end = c->ld;
  const int tiles_all = (int)((c->ld + dev::kKappaTilePoints - 1) / dev::kKappaTilePoints);

  // The exact rows of the sampled cells do not depend on the network, so they
  // are summed while it runs.  When they are few and light (one line share
  // per tile), extra blocks of the network's own launch compute them on the
  // CUs its blocks leave free; otherwise (long line lists, many blocks) they
  // run on a second stream, forked before the network and joined before the
  // check.  The fork is recorded first, but the side stream's launches are
  // issued after the network's, so that the handle's stream starts at once.
  // When the spectrum ends inside the last chunk and the line list is light,
  // that chunk's few points are not given to the network (its check, over
  // those few points, is the noisiest): extra blocks of the same launch sum
  // them exactly for every cell.  The same launch also writes the walls' row
  // of Eq. (4).
  // Phase times, when asked for, come from events recorded between the
  // kernels (before and after the network, after the check and after the
  // fallback); each costs the call several microseconds, so by default none
  // are recorded.
  S.timed_last = S.time_phases;
  auto mark = [&](int i) {
    if (S.time_phases) (void)hipEventRecord(S.ev[i], s);
  };
  dev::KappaTile te = t;
  te.cell_list = S.d_check;
  te.n_cells = n_check;
  te.out = S.d_exact;
  te.compact_rows = 1;
  const int64_t check_groups = (n_check + dev::kKappaCells - 1) / dev::kKappaCells;
  const int parts = n_check > 0 ? check_parts(c, n_check) : 1;
  const bool side = n_check > 0 && parts > 1;
  if (ok && side) ok = chk(hipEventRecord(S.fork, s));
  const int net_chunks = S.n_chunks - exact_tail_chunks(c, S);
  S.exact_chunks = S.n_chunks - net_chunks;
  InferJob job;
  job.n_cells = n_cells;
  job.epoch = S.epoch;
  if (n_check > 0 && !side) {
    job.xt = &te;
    job.x_groups = check_groups;
  }
  if (net_chunks < S.n_chunks) {
    job.tt = &t;
    job.tail_j0 = net_chunks * kMlpWidth;
    job.tail_groups = groups_all;
  }
  mark(0);
  launch_fused(c, S, n_cells * net_chunks, nullptr, nullptr, s, &job);
  mark(1);
  ok = ok && chk(hipGetLastError());
  if (ok && side) {
    const int64_t part_stride = (int64_t)n_check * c->ld;
    ok = chk(hipStreamWaitEvent(S.side, S.fork, 0)) &&
         chk(launch_kappa_tiles(c, te, check_groups, 0, tiles_all, false, S.side,
                                dev::TileGate(), parts, part_stride));
    if (ok)
      hipLaunchKernelGGL(sum_parts_kernel, dim3((unsigned)grid1(part_stride)), dim3(256), 0,
                         S.side, S.d_exact, part_stride, parts, part_stride);
    ok = ok && chk(hipGetLastError()) && chk(hipEventRecord(S.join, S.side)) &&
         chk(hipStreamWaitEvent(s, S.join, 0));
  }
  if (ok && n_check > 0) {
    hipLaunchKernelGGL(check_kernel, dim3(S.n_chunks), dim3(kCheckThreads), 0, s, c->kappa, c->ld,
                       S.d_exact, c->ld, S.d_check, n_check, c->n_nu,
                       (float)(c->cell_m * 100.0), S.d_cell_flag, S.epoch, S.d_err);
  } else if (ok) {
    hipLaunchKernelGGL(zero_f32_kernel, dim3(grid1(S.n_chunks)), dim3(256), 0, s, S.d_err,
                       (int64_t)S.n_chunks);
  }
  mark(2);
  if (ok) {
    dev::TileGate gate;
    gate.group_flag = S.d_group_flag;
    gate.epoch = S.epoch;
    gate.chunk_err = S.d_err;
    gate.tol = (float)S.tolerance;
    gate.chunk_w = kMlpWidth;
    gate.n_chunks = S.n_chunks;
    const int tiles_fine = (int)((c->ld + dev::kKappaThreads - 1) / dev::kKappaThreads);
    ok = chk(launch_kappa_tiles_fine(c, t, groups_all, tiles_fine, s, gate));
  }
  mark(3);
  ok = ok && chk(hipGetLastError());
  S.stats_pending = true;
  if (!ok) return sfail(c, RT_EDEVICE, "surrogate inference: a HIP call failed");
  return RT_OK;
}

// Counts and timings of the last inference (synchronises the stream once).
rt_status surrogate_finish_stats(rt_ctx c) {
  Surrogate& S = *c->surrogate;
  if (!S.stats_pending) return RT_OK;
  std::vector<float> err(S.n_chunks, 0.f);
  std::vector<unsigned> flag(S.inf_cells, 0u);
  hipStream_t s = c->stream;
  hipError_t e = hipMemcpyAsync(err.data(), S.d_err, S.n_chunks * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(flag.data(), S.d_cell_flag, flag.size() * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return sfail(c, RT_EDEVICE, "surrogate statistics: read-back failed");
  S.check_error = 0;
  S.fallback_chunks = 0;
  for (float v : err) {
    S.check_error = std::max(S.check_error, (double)v);
    if (v > (float)S.tolerance) ++S.fallback_chunks;
  }
  S.fallback_cells = (int)std::count(flag.begin(), flag.end(), S.epoch);
  float f1 = 0, f2 = 0, f3 = 0;
  if (S.timed_last) {
    (void)hipEventElapsedTime(&f1, S.ev[0], S.ev[1]);
    (void)hipEventElapsedTime(&f2, S.ev[1], S.ev[2]);
    (void)hipEventElapsedTime(&f3, S.ev[2], S.ev[3]);
  }
  S.infer_ms = f1;
  S.check_ms = f2;
  S.fallback_ms = f3;
  S.stats_pending = false;
  return RT_OK;
}

}  // namespace rt

using namespace rt;

extern "C" {

rt_status rt_surrogate_train(rt_ctx c, const rt_surrogate_cfg* cfg, double* final_loss) {
  if (!c || !cfg) return RT_EINVAL;
  if (!c->have_lines) return sfail(c, RT_ESTATE, "rt_surrogate_train: call rt_setup_lines first");
  const int n = cfg->n_samples;
  if (n < 64 || !cfg->T_K || !cfg->x_h2o || !cfg->p_atm)
    return sfail(c, RT_EINVAL, "rt_surrogate_train: need >= 64 samples with T, x, p");
  if (cfg->epochs < 1 || cfg->batch < 64 || cfg->batch % 64 != 0 || !(cfg->lr > 0))
    return sfail(c, RT_EINVAL, "rt_surrogate_train: epochs >= 1, batch a multiple of 64, lr > 0");
  if (!(cfg->T_min > 0 && cfg->T_max > cfg->T_min && cfg->x_min >= 0 && cfg->x_max > cfg->x_min &&
        cfg->x_max <= 1 && cfg->p_min > 0 && cfg->p_max > cfg->p_min))
    return sfail(c, RT_EINVAL, "rt_surrogate_train: invalid training box");
  if (cfg->check_cells < 0 || cfg->check_cells > kMaxCheckCells || !(cfg->tolerance > 0))
    return sfail(c, RT_EINVAL, "rt_surrogate_train: 0 <= check_cells <= 256 and tolerance > 0");
  for (int i = 0; i < n; ++i)
    if (!(cfg->T_K[i] > 0) || !(cfg->x_h2o[i] >= 0 && cfg->x_h2o[i] <= 1) || !(cfg->p_atm[i] > 0))
      return sfail(c, RT_EINVAL, "rt_surrogate_train: invalid sample state");
  if (c->device < 0) return sfail(c, RT_EUNSUPPORTED, "host-only handle (RT_NO_DEVICE): the call needs a device");
  RT_SHIP(c, hipSetDevice(c->device));
  const bool timed = c->surrogate && c->surrogate->time_phases;  // kept across a new network
  free_surrogate(c);
  Surrogate& S = surrogate(c);
  S.time_phases = timed;
  S.n_nu = c->n_nu;
  S.n_chunks = (c->n_nu + kMlpWidth - 1) / kMlpWidth;
  S.T_min = cfg->T_min; S.T_max = cfg->T_max;
  S.x_min = cfg->x_min; S.x_max = cfg->x_max;
  S.p_min = cfg->p_min; S.p_max = cfg->p_max;
  S.check_cells = cfg->check_cells;
  S.tolerance = cfg->tolerance;
  S.check_seed = cfg->seed;
  if (rt_status s = alloc_params(c, S)) return s;
  hipStream_t s = c->stream;
  // initial weights: uniform +-sqrt(6 / (fan_in + fan_out)), zero biases
  SplitMix g{cfg->seed};
  for (int l = 0; l < kMlpLayers; ++l) {
    const int K = kMlpDims[l], N = kMlpDims[l + 1];
    std::vector<float> w((size_t)K * N), z((size_t)K * N, 0.f), zb(N, 0.f);
    const double a = std::sqrt(6.0 / (K + N));
    for (auto& v : w) v = (float)((2.0 * g.uniform() - 1.0) * a);
    RT_SHIP(c, hipMemcpy(S.w[l], w.data(), w.size() * 4, hipMemcpyHostToDevice));
    RT_SHIP(c, hipMemcpy(S.mw[l], z.data(), z.size() * 4, hipMemcpyHostToDevice));
    RT_SHIP(c, hipMemcpy(S.vw[l], z.data(), z.size() * 4, hipMemcpyHostToDevice));
    RT_SHIP(c, hipMemcpy(S.b[l], zb.data(), zb.size() * 4, hipMemcpyHostToDevice));
    RT_SHIP(c, hipMemcpy(S.mb[l], zb.data(), zb.size() * 4, hipMemcpyHostToDevice));
    RT_SHIP(c, hipMemcpy(S.vb[l], zb.data(), zb.size() * 4, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(to_bf16_kernel, dim3(grid1((int64_t)K * N)), dim3(256), 0, s, S.w[l], K,
                       N, S.wt[l], S.wk[l]);
  }
  // training spectra from the line sum over a grid of sample cells
  const int64_t ld_s = ((int64_t)S.n_chunks * kMlpWidth + dev::kKappaTilePoints - 1) /
                       dev::kKappaTilePoints * dev::kKappaTilePoints;
  double *dT = nullptr, *dx = nullptr, *dp = nullptr;
  float* Yall = nullptr;
  CellSet cs;
  int32_t* perm_d = nullptr;
  Acts a;
  auto cleanup = [&]() {
    dfree(dT); dfree(dx); dfree(dp); dfree(Yall); dfree(perm_d);
    dfree(cs.G); dfree(cs.beta); dfree(cs.theta); dfree(cs.lam2); dfree(cs.P);
    a.release();
  };
  auto fail = [&](rt_status st, const std::string& m) { cleanup(); return sfail(c, st, m); };
#define RT_TRY(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) return fail(RT_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)
  RT_TRY(dalloc(&dT, n)); RT_TRY(dalloc(&dx, n)); RT_TRY(dalloc(&dp, n));
  RT_TRY(dalloc(&cs.G, n)); RT_TRY(dalloc(&cs.beta, n)); RT_TRY(dalloc(&cs.theta, n));
  RT_TRY(dalloc(&cs.lam2, n)); RT_TRY(dalloc(&cs.P, n));
  RT_TRY(dalloc(&Yall, (int64_t)n * ld_s));
  RT_TRY(hipMemcpy(dT, cfg->T_K, n * 8, hipMemcpyHostToDevice));
  RT_TRY(hipMemcpy(dx, cfg->x_h2o, n * 8, hipMemcpyHostToDevice));
  RT_TRY(hipMemcpy(dp, cfg->p_atm, n * 8, hipMemcpyHostToDevice));
  RT_TRY(launch_cell_params_on(c, n, dT, dx, dp, cs, s));
  dev::KappaTile t;
  t.L = c->lines;
  t.C = cs;
  t.n_cells = n;
  t.n_nu = c->n_nu;
  t.K = c->K;
  t.have_E = c->have_E ? 1 : 0;
  t.out = Yall;
  t.ld_out = ld_s;
  t.col0 = 0;
  t.col_end = ld_s;
  RT_TRY(launch_kappa_tiles(c, t, (n + dev::kKappaCells - 1) / dev::kKappaCells, 0,
                            (int)(ld_s / dev::kKappaTilePoints), false, s));
  const int n_cols = S.n_chunks * kMlpWidth;
  hipLaunchKernelGGL(log_target_kernel, dim3(grid1((int64_t)n * ld_s)), dim3(256), 0, s, Yall,
                     (int64_t)n, ld_s, c->n_nu, dT, dx, dp);
  hipLaunchKernelGGL(col_stats_kernel, dim3(grid1(n_cols)), dim3(256), 0, s, Yall, (int64_t)n,
                     ld_s, n_cols, S.mean, S.stdv);
  hipLaunchKernelGGL(normalize_kernel, dim3(grid1((int64_t)n * ld_s)), dim3(256), 0, s, Yall,
                     (int64_t)n, ld_s, n_cols, S.mean, S.stdv);
  RT_TRY(hipGetLastError());
  // training
  const int M = cfg->batch;
  const int64_t n_rows = (int64_t)n * S.n_chunks;
  const int64_t steps_per_epoch = std::max<int64_t>(1, n_rows / M);
  const int64_t total_steps = steps_per_epoch * cfg->epochs;
  if (rt_status st = alloc_acts(c, a, M, true)) { cleanup(); return st; }
  RT_TRY(dalloc(&perm_d, steps_per_epoch * M));
  RT_TRY(hipMemsetAsync(a.step, 0, sizeof(int), s));
  const Box bx = make_box(S);
  std::vector<int32_t> perm(n_rows);
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  RT_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  RT_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed));
  {
    // one step: batch gather, forward, loss, backward, Adam, step++
    hipLaunchKernelGGL(gather_kernel, dim3(grid1((int64_t)M * kMlpWidth)), dim3(256), 0, cap,
                       perm_d, a.step, steps_per_epoch * M, M, dT, dx, dp, bx, Yall, ld_s, a.X0,
                       a.Y, a.row_chunk);
    forward(S, a, true, cap);
    hipLaunchKernelGGL(loss_grad_kernel, dim3(grid1((int64_t)M * kMlpWidth)), dim3(256), 0, cap,
                       a.P, a.Y, a.row_chunk, M, c->n_nu, a.dP, a.dPT, a.sse);
    backward(S, a, cap);
    adam(S, a, (int)total_steps, cfg->lr, cap);
  }
  hipError_t ce = hipStreamEndCapture(cap, &graph);
  if (ce == hipSuccess) ce = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (ce != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(cap);
    return fail(RT_EDEVICE, std::string("rt_surrogate_train: graph: ") + hipGetErrorString(ce));
  }
  SplitMix sh{cfg->seed ^ 0x5EED5EEDULL};
  double last_sse = 0;
  hipError_t re = hipSuccess;
  for (int ep = 0; ep < cfg->epochs && re == hipSuccess; ++ep) {
    for (int64_t i = 0; i < n_rows; ++i) perm[i] = (int32_t)i;
    for (int64_t i = n_rows - 1; i > 0; --i) {
      const int64_t j = (int64_t)(sh.uniform() * (double)(i + 1));
      std::swap(perm[i], perm[std::min(j, i)]);
    }
    // the permutation buffer is indexed by the global step modulo its size
    const int64_t base = (int64_t)ep * steps_per_epoch * M;
    std::vector<int32_t> rolled((size_t)steps_per_epoch * M);
    const int64_t span = steps_per_epoch * M;
    for (int64_t q = 0; q < span; ++q) rolled[(base + q) % span] = perm[q];
    re = hipMemcpyAsync(perm_d, rolled.data(), rolled.size() * 4, hipMemcpyHostToDevice, s);
    if (re == hipSuccess)
      re = hipMemsetAsync(a.sse, 0, (kAccDigits + 1) * sizeof(unsigned long long), s);
    if (re == hipSuccess) re = hipStreamSynchronize(s);
    for (int64_t st = 0; st < steps_per_epoch && re == hipSuccess; ++st)
      re = hipGraphLaunch(exec, s);
    if (re == hipSuccess) {
      hipLaunchKernelGGL(sse_value_kernel, dim3(1), dim3(1), 0, s, a.sse, a.sse_value);
      re = hipGetLastError();
    }
    if (re == hipSuccess)
      re = hipMemcpyAsync(&last_sse, a.sse_value, sizeof(double), hipMemcpyDeviceToHost, s);
    if (re == hipSuccess) re = hipStreamSynchronize(s);
  }
  (void)hipGraphExecDestroy(exec);
  (void)hipGraphDestroy(graph);
  (void)hipStreamDestroy(cap);
  if (re != hipSuccess) return fail(RT_EDEVICE, std::string("rt_surrogate_train: ") + hipGetErrorString(re));
  S.train_loss = last_sse / ((double)steps_per_epoch * M * kMlpWidth);
  if (final_loss) *final_loss = S.train_loss;
  pack_weights(S, s);
  if (hipStreamSynchronize(s) != hipSuccess) return fail(RT_EDEVICE, "rt_surrogate_train: packing failed");
  cleanup();
  S.trained = true;
#undef RT_TRY
  return RT_OK;
}

rt_status rt_surrogate_forward(rt_ctx c, int n_rows, const float* inputs, float* outputs) {
  if (!c || n_rows < 1 || !inputs || !outputs) return RT_EINVAL;
  if (!c->surrogate || !c->surrogate->trained) return sfail(c, RT_ESTATE, "rt_surrogate_forward: no surrogate");
  Surrogate& S = *c->surrogate;
  float* X0 = nullptr;
  float* P = nullptr;
  hipError_t e = dalloc(&X0, (int64_t)n_rows * 4);
  if (e == hipSuccess) e = dalloc(&P, (int64_t)n_rows * kMlpWidth);
  if (e == hipSuccess)
    e = hipMemcpyAsync(X0, inputs, (size_t)n_rows * 16, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) {
    launch_fused(c, S, n_rows, X0, P, c->stream, nullptr);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(outputs, P, (size_t)n_rows * kMlpWidth * 4, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  dfree(X0);
  dfree(P);
  if (e != hipSuccess) return sfail(c, RT_EDEVICE, std::string("rt_surrogate_forward: ") + hipGetErrorString(e));
  return RT_OK;
}

rt_status rt_surrogate_weights(rt_ctx c, float* out, int64_t n) {
  if (!c || !out) return RT_EINVAL;
  if (!c->surrogate || !c->surrogate->trained) return sfail(c, RT_ESTATE, "rt_surrogate_weights: no surrogate");
  Surrogate& S = *c->surrogate;
  if (n < S.param_count) return sfail(c, RT_EINVAL, "rt_surrogate_weights: buffer too small");
  int64_t off = 0;
  for (int l = 0; l < kMlpLayers; ++l) {
    const int64_t kn = (int64_t)kMlpDims[l] * kMlpDims[l + 1];
    RT_SHIP(c, hipMemcpy(out + off, S.w[l], kn * 4, hipMemcpyDeviceToHost));
    off += kn;
    RT_SHIP(c, hipMemcpy(out + off, S.b[l], kMlpDims[l + 1] * 4, hipMemcpyDeviceToHost));
    off += kMlpDims[l + 1];
  }
  return RT_OK;
}

rt_status rt_surrogate_time_phases(rt_ctx c, int on) {
  if (!c) return RT_EINVAL;
  surrogate(c).time_phases = on != 0;
  return RT_OK;
}

rt_status rt_surrogate_get_stats(rt_ctx c, rt_surrogate_stats* out) {
  if (!c || !out) return RT_EINVAL;
  if (!c->surrogate || !c->surrogate->trained) return sfail(c, RT_ESTATE, "rt_surrogate_get_stats: no surrogate");
  if (rt_status st = surrogate_finish_stats(c)) return st;
  const Surrogate& S = *c->surrogate;
  out->check_error = S.check_error;
  out->fallback_chunks = S.fallback_chunks;
  out->fallback_cells = S.fallback_cells;
  out->n_chunks = S.n_chunks;
  out->infer_ms = S.infer_ms;
  out->check_ms = S.check_ms;
  out->fallback_ms = S.fallback_ms;
  out->train_loss = S.train_loss;
  out->param_count = (double)S.param_count;
  out->exact_chunks = S.exact_chunks;
  return RT_OK;
}

// Blob: "RTLBLMLP", version 1, header ints/doubles, FP32 masters and the
// normalisation tables, FNV-1a 64 checksum of everything before it.
rt_status rt_surrogate_save(rt_ctx c, const char* path) {
  if (!c || !path) return RT_EINVAL;
  if (!c->surrogate || !c->surrogate->trained) return sfail(c, RT_ESTATE, "rt_surrogate_save: no surrogate");
  Surrogate& S = *c->surrogate;
  std::vector<char> blob;
  auto put = [&](const void* p, size_t n) {
    const char* b = static_cast<const char*>(p);
    blob.insert(blob.end(), b, b + n);
  };
  put("RTLBLMLP", 8);
  const int32_t hdr[4] = {1, S.n_nu, S.n_chunks, S.check_cells};
  put(hdr, sizeof(hdr));
  const double box[7] = {S.T_min, S.T_max, S.x_min, S.x_max, S.p_min, S.p_max, S.tolerance};
  put(box, sizeof(box));
  put(&S.check_seed, 8);
  for (int l = 0; l < kMlpLayers; ++l) {
    const int64_t kn = (int64_t)kMlpDims[l] * kMlpDims[l + 1];
    std::vector<float> w(kn), b(kMlpDims[l + 1]);
    RT_SHIP(c, hipMemcpy(w.data(), S.w[l], kn * 4, hipMemcpyDeviceToHost));
    RT_SHIP(c, hipMemcpy(b.data(), S.b[l], b.size() * 4, hipMemcpyDeviceToHost));
    put(w.data(), w.size() * 4);
    put(b.data(), b.size() * 4);
  }
  std::vector<float> mean((size_t)S.n_chunks * kMlpWidth), sd(mean.size());
  RT_SHIP(c, hipMemcpy(mean.data(), S.mean, mean.size() * 4, hipMemcpyDeviceToHost));
  RT_SHIP(c, hipMemcpy(sd.data(), S.stdv, sd.size() * 4, hipMemcpyDeviceToHost));
  put(mean.data(), mean.size() * 4);
  put(sd.data(), sd.size() * 4);
  const uint64_t h = fnv1a(blob.data(), blob.size());
  put(&h, 8);
  std::ofstream f(path, std::ios::binary | std::ios::trunc);
  f.write(blob.data(), (std::streamsize)blob.size());
  if (!f) return sfail(c, RT_EINVAL, "rt_surrogate_save: cannot write file");
  return RT_OK;
}

rt_status rt_surrogate_load(rt_ctx c, const char* path) {
  if (!c || !path) return RT_EINVAL;
  std::ifstream f(path, std::ios::binary);
  if (!f) return sfail(c, RT_EINVAL, "rt_surrogate_load: cannot read file");
  std::vector<char> blob((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
  if (blob.size() < 8 + 16 + 56 + 8 + 8 || std::memcmp(blob.data(), "RTLBLMLP", 8) != 0)
    return sfail(c, RT_EINVAL, "rt_surrogate_load: not a surrogate blob");
  uint64_t h;
  std::memcpy(&h, blob.data() + blob.size() - 8, 8);
  if (h != fnv1a(blob.data(), blob.size() - 8)) return sfail(c, RT_EINVAL, "rt_surrogate_load: checksum mismatch");
  size_t off = 8;
  int32_t hdr[4];
  std::memcpy(hdr, blob.data() + off, 16); off += 16;
  if (hdr[0] != 1) return sfail(c, RT_EINVAL, "rt_surrogate_load: unknown version");
  if (hdr[3] < 0 || hdr[3] > kMaxCheckCells)
    return sfail(c, RT_EINVAL, "rt_surrogate_load: sampled-cell count out of range");
  double box[7];
  std::memcpy(box, blob.data() + off, 56); off += 56;
  uint64_t seed;
  std::memcpy(&seed, blob.data() + off, 8); off += 8;
  int64_t need = 0;
  for (int l = 0; l < kMlpLayers; ++l) need += ((int64_t)kMlpDims[l] * kMlpDims[l + 1] + kMlpDims[l + 1]) * 4;
  need += 2LL * hdr[2] * kMlpWidth * 4;
  if ((int64_t)blob.size() != (int64_t)off + need + 8) return sfail(c, RT_EINVAL, "rt_surrogate_load: size mismatch");
  if (c->device < 0) return sfail(c, RT_EUNSUPPORTED, "host-only handle (RT_NO_DEVICE): the call needs a device");
  RT_SHIP(c, hipSetDevice(c->device));
  const bool timed = c->surrogate && c->surrogate->time_phases;  // kept across a new network
  free_surrogate(c);
  Surrogate& S = surrogate(c);
  S.time_phases = timed;
  S.n_nu = hdr[1]; S.n_chunks = hdr[2]; S.check_cells = hdr[3];
  S.T_min = box[0]; S.T_max = box[1]; S.x_min = box[2]; S.x_max = box[3];
  S.p_min = box[4]; S.p_max = box[5]; S.tolerance = box[6];
  S.check_seed = seed;
  if (rt_status st = alloc_params(c, S)) return st;
  for (int l = 0; l < kMlpLayers; ++l) {
    const int K = kMlpDims[l], N = kMlpDims[l + 1];
    RT_SHIP(c, hipMemcpy(S.w[l], blob.data() + off, (size_t)K * N * 4, hipMemcpyHostToDevice));
    off += (size_t)K * N * 4;
    RT_SHIP(c, hipMemcpy(S.b[l], blob.data() + off, (size_t)N * 4, hipMemcpyHostToDevice));
    off += (size_t)N * 4;
    hipLaunchKernelGGL(to_bf16_kernel, dim3(grid1((int64_t)K * N)), dim3(256), 0, c->stream,
                       S.w[l], K, N, S.wt[l], S.wk[l]);
  }
  RT_SHIP(c, hipMemcpy(S.mean, blob.data() + off, (size_t)S.n_chunks * kMlpWidth * 4, hipMemcpyHostToDevice));
  off += (size_t)S.n_chunks * kMlpWidth * 4;
  RT_SHIP(c, hipMemcpy(S.stdv, blob.data() + off, (size_t)S.n_chunks * kMlpWidth * 4, hipMemcpyHostToDevice));
  pack_weights(S, c->stream);
  RT_SHIP(c, hipStreamSynchronize(c->stream));
  S.trained = true;
  return RT_OK;
}

}  // extern "C"
