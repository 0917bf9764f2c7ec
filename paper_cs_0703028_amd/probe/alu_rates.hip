// alu_rates.hip -- issue-rate probe for the instruction classes the march and
// line-sum kernels are built from (gfx950): FP32 FMA, the hardware base-2
// exponential, the hardware reciprocal, and a 1:1 mix of exponential and FMA.
// Every lane runs 8 independent dependency chains so that issue rate, not
// latency, bounds the loop.  Prints one JSON line with wave-instructions per
// CU per cycle (at the 2.4 GHz peak clock) and lane-operations per second.
//
// Used to fix the operation-cost model behind the march roofline; the probe
// reads and writes only its own buffers.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CHECK(x)                                                              \
  do {                                                                        \
    hipError_t e_ = (x);                                                      \
    if (e_ != hipSuccess) {                                                   \
      std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));           \
      std::exit(1);                                                           \
    }                                                                         \
  } while (0)

constexpr int kChains = 8;

__global__ void k_fma(float* out, int iters, float b, float c) {
  float v[kChains];
  for (int i = 0; i < kChains; ++i) v[i] = threadIdx.x * 1e-3f + i;
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int i = 0; i < kChains; ++i) v[i] = fmaf(v[i], b, c);
  float s = 0;
  for (int i = 0; i < kChains; ++i) s += v[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void k_exp(float* out, int iters) {
  float v[kChains];
  for (int i = 0; i < kChains; ++i) v[i] = 0.1f * i + threadIdx.x * 1e-4f;
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int i = 0; i < kChains; ++i) v[i] = __builtin_amdgcn_exp2f(-v[i]);
  float s = 0;
  for (int i = 0; i < kChains; ++i) s += v[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void k_rcp(float* out, int iters) {
  float v[kChains];
  for (int i = 0; i < kChains; ++i) v[i] = 1.5f + 0.1f * i + threadIdx.x * 1e-4f;
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int i = 0; i < kChains; ++i) v[i] = __builtin_amdgcn_rcpf(-v[i]);
  float s = 0;
  for (int i = 0; i < kChains; ++i) s += v[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void k_mix(float* out, int iters, float b, float c) {
  float v[kChains], w[kChains];
  for (int i = 0; i < kChains; ++i) { v[i] = 0.1f * i; w[i] = threadIdx.x * 1e-3f + i; }
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int i = 0; i < kChains; ++i) {
      v[i] = __builtin_amdgcn_exp2f(-v[i]);
      w[i] = fmaf(w[i], b, c);
    }
  float s = 0;
  for (int i = 0; i < kChains; ++i) s += v[i] + w[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

int main() {
  int dev = 0;
  hipDeviceProp_t p;
  CHECK(hipGetDeviceProperties(&p, dev));
  const int cus = p.multiProcessorCount;
  const int blocks = cus * 16, threads = 256, iters = 4096;
  float* out;
  CHECK(hipMalloc(&out, sizeof(float) * blocks * threads));
  hipEvent_t a, b;
  CHECK(hipEventCreate(&a));
  CHECK(hipEventCreate(&b));
  const double waves = (double)blocks * threads / 64.0;
  auto run = [&](const char* name, int which, double instr_per_iter) {
    float best = 1e30f;
    for (int rep = 0; rep < 4; ++rep) {
      CHECK(hipEventRecord(a));
      if (which == 0) hipLaunchKernelGGL(k_fma, dim3(blocks), dim3(threads), 0, 0, out, iters, 0.999f, 1e-3f);
      if (which == 1) hipLaunchKernelGGL(k_exp, dim3(blocks), dim3(threads), 0, 0, out, iters);
      if (which == 2) hipLaunchKernelGGL(k_rcp, dim3(blocks), dim3(threads), 0, 0, out, iters);
      if (which == 3) hipLaunchKernelGGL(k_mix, dim3(blocks), dim3(threads), 0, 0, out, iters, 0.999f, 1e-3f);
      CHECK(hipGetLastError());
      CHECK(hipEventRecord(b));
      CHECK(hipEventSynchronize(b));
      float ms;
      CHECK(hipEventElapsedTime(&ms, a, b));
      if (rep > 0 && ms < best) best = ms;
    }
    const double instr = waves * iters * instr_per_iter;
    const double per_cu_cycle = instr / (best * 1e-3) / (cus * 2.4e9);
    std::printf("%s\"%s\": {\"ms\": %.4f, \"wave_instr_per_cu_cycle\": %.4f, \"lane_ops_per_s\": %.4e}",
                which ? ", " : "{", name, best, per_cu_cycle, instr * 64 / (best * 1e-3));
  };
  run("fma", 0, kChains);
  run("exp2", 1, kChains);
  run("rcp", 2, kChains);
  run("exp2+fma", 3, 2 * kChains);
  std::printf(", \"cus\": %d, \"arch\": \"%s\"}\n", cus, p.gcnArchName);
  CHECK(hipFree(out));
  return 0;
}
