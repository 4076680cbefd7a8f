// ulp_ref.hip -- the platform's own math functions (HIP's device library,
// accurate to about 1 ulp, not correctly rounded) as elementwise maps with the
// launch shape of the correctly rounded kernels: 128-bit nontemporal loads and
// stores, 8 elements per thread per tile, a persistent grid.
//
// The paper's GPU results are ratios: correctly rounded throughput over the
// throughput of the same GPU's ~1-ulp library functions (Sec. III-C, Tables
// III and IV).  This library only serves that comparison in the benchmark; it
// is not part of libcr.
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace {

constexpr int BLOCK = 256;
constexpr int U = 2;

typedef float v4f_t __attribute__((ext_vector_type(4)));
typedef double v2d_t __attribute__((ext_vector_type(2)));

enum {
  F_EXPF = 0, F_EXP2F, F_EXP10F, F_EXPM1F, F_LOGF, F_LOG2F, F_LOG10F, F_LOG1PF, F_RSQRTF,
  F_SINF, F_COSF, F_SINCOSF, F_TANF, F_ASINF, F_ACOSF, F_ATANF, F_SINHF, F_COSHF, F_TANHF,
  F_EXP = 64, F_LOG = 65, F_EXP2 = 66
};

template <int F>
__device__ __forceinline__ float f32(float x) {
  switch (F) {
    case F_EXPF: return expf(x);
    case F_EXP2F: return exp2f(x);
    case F_EXP10F: return exp10f(x);
    case F_EXPM1F: return expm1f(x);
    case F_LOGF: return logf(x);
    case F_LOG2F: return log2f(x);
    case F_LOG10F: return log10f(x);
    case F_LOG1PF: return log1pf(x);
    case F_RSQRTF: return rsqrtf(x);
    case F_SINF: return sinf(x);
    case F_COSF: return cosf(x);
    case F_TANF: return tanf(x);
    case F_ASINF: return asinf(x);
    case F_ACOSF: return acosf(x);
    case F_ATANF: return atanf(x);
    case F_SINHF: return sinhf(x);
    case F_COSHF: return coshf(x);
    default: return tanhf(x);
  }
}

template <int F>
__global__ void __launch_bounds__(BLOCK) k_ref32(const float4* in, float4* out, long long n4) {
  for (long long t = blockIdx.x; t * BLOCK * U < n4; t += gridDim.x) {
#pragma unroll
    for (int u = 0; u < U; u++) {
      long long i = t * BLOCK * U + u * BLOCK + threadIdx.x;
      if (i < n4) {
        v4f_t v = __builtin_nontemporal_load(reinterpret_cast<const v4f_t*>(in + i));
        v4f_t r = {f32<F>(v.x), f32<F>(v.y), f32<F>(v.z), f32<F>(v.w)};
        __builtin_nontemporal_store(r, reinterpret_cast<v4f_t*>(out + i));
      }
    }
  }
}

__global__ void __launch_bounds__(BLOCK)
    k_ref_sincos(const float4* in, float4* os, float4* oc, long long n4) {
  for (long long t = blockIdx.x; t * BLOCK * U < n4; t += gridDim.x) {
#pragma unroll
    for (int u = 0; u < U; u++) {
      long long i = t * BLOCK * U + u * BLOCK + threadIdx.x;
      if (i < n4) {
        v4f_t v = __builtin_nontemporal_load(reinterpret_cast<const v4f_t*>(in + i));
        float s0, s1, s2, s3, c0, c1, c2, c3;
        sincosf(v.x, &s0, &c0);
        sincosf(v.y, &s1, &c1);
        sincosf(v.z, &s2, &c2);
        sincosf(v.w, &s3, &c3);
        v4f_t s = {s0, s1, s2, s3}, c = {c0, c1, c2, c3};
        __builtin_nontemporal_store(s, reinterpret_cast<v4f_t*>(os + i));
        __builtin_nontemporal_store(c, reinterpret_cast<v4f_t*>(oc + i));
      }
    }
  }
}

template <int F>
__global__ void __launch_bounds__(BLOCK) k_ref64(const double2* in, double2* out, long long n2) {
  for (long long t = blockIdx.x; t * BLOCK * 2 * U < n2; t += gridDim.x) {
#pragma unroll
    for (int u = 0; u < 2 * U; u++) {
      long long i = t * BLOCK * 2 * U + u * BLOCK + threadIdx.x;
      if (i < n2) {
        v2d_t v = __builtin_nontemporal_load(reinterpret_cast<const v2d_t*>(in + i));
        v2d_t r = F == F_EXP    ? v2d_t{exp(v.x), exp(v.y)}
                  : F == F_EXP2 ? v2d_t{exp2(v.x), exp2(v.y)}
                                : v2d_t{log(v.x), log(v.y)};
        __builtin_nontemporal_store(r, reinterpret_cast<v2d_t*>(out + i));
      }
    }
  }
}

int grid_for(long long units) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  long long g = (long long)cus * 32;
  long long tiles = (units + BLOCK * U - 1) / (BLOCK * U);
  return (int)(tiles < g ? (tiles > 0 ? tiles : 1) : g);
}

template <int F>
void launch32(const float* in, float* out, long long n4, hipStream_t s) {
  hipLaunchKernelGGL(k_ref32<F>, dim3(grid_for(n4)), dim3(BLOCK), 0, s,
                     reinterpret_cast<const float4*>(in), reinterpret_cast<float4*>(out), n4);
}

}  // namespace

// n elements (binary32 functions: n a multiple of 4, 16-byte aligned buffers;
// binary64: n even).  Returns 0, or -1 for an unknown function or a bad size.
extern "C" int cr_ref_eval(int f, const void* in, void* out, size_t n, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const float* a = (const float*)in;
  float* b = (float*)out;
  long long n4 = (long long)(n / 4);
  if (f < 64 && (n % 4)) return -1;
  switch (f) {
    case F_EXPF: launch32<F_EXPF>(a, b, n4, s); break;
    case F_EXP2F: launch32<F_EXP2F>(a, b, n4, s); break;
    case F_EXP10F: launch32<F_EXP10F>(a, b, n4, s); break;
    case F_EXPM1F: launch32<F_EXPM1F>(a, b, n4, s); break;
    case F_LOGF: launch32<F_LOGF>(a, b, n4, s); break;
    case F_LOG2F: launch32<F_LOG2F>(a, b, n4, s); break;
    case F_LOG10F: launch32<F_LOG10F>(a, b, n4, s); break;
    case F_LOG1PF: launch32<F_LOG1PF>(a, b, n4, s); break;
    case F_RSQRTF: launch32<F_RSQRTF>(a, b, n4, s); break;
    case F_SINF: launch32<F_SINF>(a, b, n4, s); break;
    case F_COSF: launch32<F_COSF>(a, b, n4, s); break;
    case F_TANF: launch32<F_TANF>(a, b, n4, s); break;
    case F_ASINF: launch32<F_ASINF>(a, b, n4, s); break;
    case F_ACOSF: launch32<F_ACOSF>(a, b, n4, s); break;
    case F_ATANF: launch32<F_ATANF>(a, b, n4, s); break;
    case F_SINHF: launch32<F_SINHF>(a, b, n4, s); break;
    case F_COSHF: launch32<F_COSHF>(a, b, n4, s); break;
    case F_TANHF: launch32<F_TANHF>(a, b, n4, s); break;
    case F_SINCOSF:
      hipLaunchKernelGGL(k_ref_sincos, dim3(grid_for(n4)), dim3(BLOCK), 0, s,
                         reinterpret_cast<const float4*>(a), reinterpret_cast<float4*>(b),
                         reinterpret_cast<float4*>(b + n), n4);
      break;
    case F_EXP:
    case F_EXP2:
    case F_LOG: {
      if (n % 2) return -1;
      long long n2 = (long long)(n / 2);
      auto k = f == F_EXP ? k_ref64<F_EXP> : (f == F_EXP2 ? k_ref64<F_EXP2> : k_ref64<F_LOG>);
      hipLaunchKernelGGL(k, dim3(grid_for(n2 / 2)), dim3(BLOCK), 0, s,
                         reinterpret_cast<const double2*>(in), reinterpret_cast<double2*>(out),
                         n2);
      break;
    }
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
