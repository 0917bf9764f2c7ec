// arith.hip -- gfx950 FP32 arithmetic characterisation.
//
// The paper characterises the floating-point units of its GPUs with test
// vectors (its Table 2): rounding of sums and differences near a tie, whether
// a multiply-add rounds the product, sign and scaling symmetry and the error
// in ulp of products, overflow inside a composite expression, subnormals and
// NaNs across transfers.  The device side of the same experiments on gfx950
// is small: apply one named instruction (or a two-instruction composite kept
// in registers) element-wise and store the result bit for bit.  What the
// result should be, and its error in ulp, is worked out on the host from
// exact arithmetic.
#include "rt_internal.h"

namespace rt {
namespace {

// Two roundings: the product is rounded before the addition.
__device__ __forceinline__ float mul_then_add(float x, float y, float z) {
#pragma clang fp contract(off)
  const float p = x * y;
  return p + z;
}

template <int OP>
__device__ __forceinline__ float apply(float x, float y, float z) {
#pragma clang fp contract(off)
  switch (OP) {
    case RT_AR_COPY: return x;
    case RT_AR_ADD: return x + y;
    case RT_AR_SUB: return x - y;
    case RT_AR_MUL: return x * y;
    case RT_AR_FMA: return __builtin_fmaf(x, y, z);
    case RT_AR_MUL_ADD: return mul_then_add(x, y, z);
    case RT_AR_FMA_ERR: {  // x*y - round(x*y) when the multiply-add is fused
      const float p = x * y;
      return __builtin_fmaf(x, y, -p);
    }
    case RT_AR_ADD_SUB: return (x + y) - z;
    case RT_AR_SUB_SUB: return (x - y) - z;
    case RT_AR_DIV: return x / y;
    case RT_AR_EXP2: return __builtin_amdgcn_exp2f(x);
    case RT_AR_LOG2: return __builtin_amdgcn_logf(x);
    case RT_AR_RCP: return __builtin_amdgcn_rcpf(x);
    case RT_AR_RSQ: return __builtin_amdgcn_rsqf(x);
    case RT_AR_SQRT: return __builtin_amdgcn_sqrtf(x);
    default: return 0.f;
  }
}

template <int OP>
__global__ __launch_bounds__(256) void arith_kernel(const float* __restrict__ a,
                                                    const float* __restrict__ b,
                                                    const float* __restrict__ c,
                                                    float* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float x = a[i];
  const float y = b ? b[i] : 0.f;
  const float z = c ? c[i] : 0.f;
  out[i] = apply<OP>(x, y, z);
}

}  // namespace

int arith_operands(int op) {
  switch (op) {
    case RT_AR_COPY: case RT_AR_EXP2: case RT_AR_LOG2: case RT_AR_RCP: case RT_AR_RSQ:
    case RT_AR_SQRT:
      return 1;
    case RT_AR_ADD: case RT_AR_SUB: case RT_AR_MUL: case RT_AR_FMA_ERR: case RT_AR_DIV:
      return 2;
    case RT_AR_FMA: case RT_AR_MUL_ADD: case RT_AR_ADD_SUB: case RT_AR_SUB_SUB:
      return 3;
    default:
      return 0;
  }
}

hipError_t launch_arith(rt_ctx c, int op, const float* a, const float* b, const float* z,
                        float* out, int64_t n) {
  const int threads = 256;
  const int64_t blocks = (n + threads - 1) / threads;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 g((unsigned)blocks), t(threads);
#define RT_ARITH_CASE(OPV)                                                                 \
  case OPV:                                                                                \
    hipLaunchKernelGGL((arith_kernel<OPV>), g, t, 0, c->stream, a, b, z, out, n);          \
    break;
  switch (op) {
    RT_ARITH_CASE(RT_AR_COPY)
    RT_ARITH_CASE(RT_AR_ADD)
    RT_ARITH_CASE(RT_AR_SUB)
    RT_ARITH_CASE(RT_AR_MUL)
    RT_ARITH_CASE(RT_AR_FMA)
    RT_ARITH_CASE(RT_AR_MUL_ADD)
    RT_ARITH_CASE(RT_AR_FMA_ERR)
    RT_ARITH_CASE(RT_AR_ADD_SUB)
    RT_ARITH_CASE(RT_AR_SUB_SUB)
    RT_ARITH_CASE(RT_AR_DIV)
    RT_ARITH_CASE(RT_AR_EXP2)
    RT_ARITH_CASE(RT_AR_LOG2)
    RT_ARITH_CASE(RT_AR_RCP)
    RT_ARITH_CASE(RT_AR_RSQ)
    RT_ARITH_CASE(RT_AR_SQRT)
    default:
      return hipErrorInvalidValue;
  }
#undef RT_ARITH_CASE
  return hipGetLastError();
}

}  // namespace rt
