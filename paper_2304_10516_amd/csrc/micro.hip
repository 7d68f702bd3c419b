// Measurement kernels: the chip's attainable rates for the access patterns of
// the training step's phases, used as roofline denominators next to the
// vendor peaks.  None of them is part of the method; see include/dvnr_micro.h.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/dvnr_micro.h"

namespace {

// Integer finalizer of MurmurHash3 (fmix32): spreads consecutive counters over
// the whole 32-bit range, so that masked results address a table uniformly.
__device__ __forceinline__ uint32_t fmix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x85ebca6bu;
  x ^= x >> 13;
  x *= 0xc2b2ae35u;
  x ^= x >> 16;
  return x;
}

typedef float f4 __attribute__((ext_vector_type(4)));

// Streaming copy, four 16-byte elements per thread per iteration.
template <bool NT>
__global__ __launch_bounds__(256) void k_copy(const f4* __restrict__ src, f4* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * 256 * 4;
  for (int64_t i = (int64_t)blockIdx.x * 256 * 4 + threadIdx.x; i < n; i += stride) {
    f4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t j = i + 256 * u;
      if (j < n) v[u] = NT ? __builtin_nontemporal_load(src + j) : src[j];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t j = i + 256 * u;
      if (j < n) {
        if (NT)
          __builtin_nontemporal_store(v[u], dst + j);
        else
          dst[j] = v[u];
      }
    }
  }
}

// Random 4-byte loads: per thread `per_thread` lookups (a multiple of 8, eight
// in flight), addresses fmix32(counter ^ seed) & mask; the sum is stored so the
// loads stay live.
__global__ __launch_bounds__(256) void k_gather(const uint32_t* __restrict__ t, uint32_t mask, int per_thread,
                                                uint32_t seed, uint32_t* __restrict__ out) {
  const uint32_t tid = blockIdx.x * 256 + threadIdx.x;
  uint32_t acc = 0;
  for (int k = 0; k < per_thread; k += 8) {
    uint32_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = t[fmix32((tid * (uint32_t)per_thread + k + u) ^ seed) & mask];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u];
  }
  out[tid] = acc;
}

// Random fp32 atomic adds (no return value), `group` consecutive lanes adding
// to consecutive elements of one random group-aligned position.
__global__ __launch_bounds__(256) void k_atomic(float* __restrict__ t, uint32_t mask, int per_thread, int group,
                                                uint32_t seed) {
  const uint32_t tid = blockIdx.x * 256 + threadIdx.x;
  const uint32_t gid = tid / group, lane = tid % group;
  const uint32_t gmask = mask & ~(uint32_t)(group - 1);
  for (int k = 0; k < per_thread; ++k) {
    const uint32_t e = (fmix32((gid * (uint32_t)per_thread + k) ^ seed) & gmask) + lane;
    unsafeAtomicAdd(&t[e], 1.0f);
  }
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Back-to-back 16x16x32 bf16 MFMAs on eight independent accumulators per wave.
__global__ __launch_bounds__(256) void k_mfma_bf16(int iters, float* __restrict__ out) {
  bf16x8 a, b;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    a[k] = (__bf16)(1.0f + 0.001f * (float)(threadIdx.x + k));
    b[k] = (__bf16)(1.0f - 0.001f * (float)(threadIdx.x + 2 * k));
  }
  f4 c[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) c[j] = f4{0.f, 0.f, 0.f, 0.f};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) c[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c[j], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < 8; ++j) s += c[j][0] + c[j][1] + c[j][2] + c[j][3];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}

bool pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

}  // namespace

extern "C" {

int32_t dvnr_micro_copy(const void* src, void* dst, int64_t bytes, int32_t nontemporal, void* stream) {
  if (!src || !dst || bytes <= 0 || bytes % 16 || ((uintptr_t)src) % 16 || ((uintptr_t)dst) % 16) return 1;
  const int64_t n = bytes / 16;
  const int64_t per_wg = 256 * 4;
  const unsigned grid = (unsigned)((n + per_wg - 1) / per_wg < 65536 ? (n + per_wg - 1) / per_wg : 65536);
  if (nontemporal)
    hipLaunchKernelGGL(k_copy<true>, dim3(grid), dim3(256), 0, (hipStream_t)stream, (const f4*)src, (f4*)dst, n);
  else
    hipLaunchKernelGGL(k_copy<false>, dim3(grid), dim3(256), 0, (hipStream_t)stream, (const f4*)src, (f4*)dst, n);
  return hipGetLastError() == hipSuccess ? 0 : 3;
}

int32_t dvnr_micro_gather(const uint32_t* table, int64_t n_entries, int64_t n_threads, int32_t per_thread,
                          uint32_t seed, uint32_t* out, void* stream) {
  if (!table || !out || !pow2(n_entries) || n_entries > ((int64_t)1 << 32) || n_threads <= 0 ||
      n_threads % 256 || n_threads / 256 > 0x7fffffff || per_thread <= 0 || per_thread % 8)
    return 1;
  hipLaunchKernelGGL(k_gather, dim3((unsigned)(n_threads / 256)), dim3(256), 0, (hipStream_t)stream, table,
                     (uint32_t)(n_entries - 1), per_thread, seed, out);
  return hipGetLastError() == hipSuccess ? 0 : 3;
}

int32_t dvnr_micro_atomic(float* table, int64_t n_entries, int64_t n_threads, int32_t per_thread, int32_t group,
                          uint32_t seed, void* stream) {
  if (!table || !pow2(n_entries) || n_entries > ((int64_t)1 << 32) || n_threads <= 0 || n_threads % 256 ||
      n_threads / 256 > 0x7fffffff || per_thread <= 0 || !pow2(group) || group > 64 || group > n_entries)
    return 1;
  hipLaunchKernelGGL(k_atomic, dim3((unsigned)(n_threads / 256)), dim3(256), 0, (hipStream_t)stream, table,
                     (uint32_t)(n_entries - 1), per_thread, group, seed);
  return hipGetLastError() == hipSuccess ? 0 : 3;
}

int32_t dvnr_micro_mfma_bf16(int64_t n_workgroups, int32_t iters, float* out, void* stream) {
  if (!out || n_workgroups <= 0 || n_workgroups > 0x7fffffff || iters <= 0) return 1;
  hipLaunchKernelGGL(k_mfma_bf16, dim3((unsigned)n_workgroups), dim3(256), 0, (hipStream_t)stream, iters, out);
  return hipGetLastError() == hipSuccess ? 0 : 3;
}

}  // extern "C"
