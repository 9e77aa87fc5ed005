// mcrt_probes.hip -- memory-system probes (include/mcrt_probes.h): the
// access patterns of the life cycle's walks and tallies in isolation.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mcrt_probes.h"

namespace {

constexpr int kThreads = 256;
constexpr unsigned long long kPerThread = 64;  // ops per thread (gather, atomics)

// Finaliser of splitmix64 (Steele, Lea & Flood, OOPSLA 2014): a bijection
// of 64-bit words whose outputs look uniform for consecutive inputs.
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__global__ void __launch_bounds__(kThreads) k_stream_read(const float4* __restrict__ p, unsigned long long n4,
                                                          float* __restrict__ out) {
  float acc = 0.0f;
  const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
  for (unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; i < n4; i += stride) {
    const float4 v = p[i];
    acc += (v.x + v.y) + (v.z + v.w);
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = acc;  // keeps the loads
}

__global__ void __launch_bounds__(kThreads) k_gather(const float* __restrict__ t, unsigned long long mask,
                                                     float* __restrict__ out) {
  const unsigned long long tid = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x;
  float acc = 0.0f;
  for (unsigned long long k = 0; k < kPerThread; k += 4) {
    const unsigned long long b = tid * kPerThread + k;
    const float a0 = t[mix64(b) & mask], a1 = t[mix64(b + 1) & mask], a2 = t[mix64(b + 2) & mask],
                a3 = t[mix64(b + 3) & mask];
    acc += (a0 + a1) + (a2 + a3);
  }
  out[tid] = acc;
}

__global__ void __launch_bounds__(kThreads) k_atomic_scattered(double* t, unsigned long long mask) {
  const unsigned long long tid = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x;
  for (unsigned long long k = 0; k < kPerThread; ++k)
    __hip_atomic_fetch_add(t + (mix64(tid * kPerThread + k) & mask), 1.0, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void __launch_bounds__(kThreads) k_atomic_coalesced(double* t, unsigned long long mask) {
  const unsigned long long tid = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x;
  const unsigned long long wave = tid >> 6, lane = tid & 63ull;
  for (unsigned long long k = 0; k < kPerThread; ++k) {
    const unsigned long long base = (mix64(wave * kPerThread + k) & mask) & ~63ull;
    __hip_atomic_fetch_add(t + base + lane, 1.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

bool pow2(unsigned long long x) { return x && !(x & (x - 1)); }

}  // namespace

extern "C" int mcrt_probe(int kind, void* buf_dev, uint64_t buf_bytes, uint64_t n_ops, int reps, double* ms_host,
                          void* hip_stream) {
  if (!buf_dev || !ms_host || reps < 1 || n_ops == 0) return -1;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  unsigned long long elems = 0, blocks = 0;
  switch (kind) {  // arguments first: nothing touches the device before they pass
    case MCRT_PROBE_STREAM_READ:
      if (buf_bytes % 16) return -1;
      break;
    case MCRT_PROBE_GATHER:
      elems = buf_bytes / 4;
      if (buf_bytes % 4 || !pow2(elems) || elems < 64) return -1;
      break;
    case MCRT_PROBE_ATOMIC_SCATTERED:
    case MCRT_PROBE_ATOMIC_COALESCED:
      elems = buf_bytes / 8;
      if (buf_bytes % 8 || !pow2(elems) || elems < 64) return -1;
      break;
    default:
      return -1;
  }
  if (kind != MCRT_PROBE_STREAM_READ) {
    if (n_ops % (kPerThread * kThreads)) return -1;  // whole workgroups
    blocks = n_ops / (kPerThread * kThreads);
    if (blocks > (1ull << 31)) return -1;
  } else {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -3;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -3;
    blocks = (unsigned long long)cus * 16;  // a persistent grid-stride sweep
  }
  float* out = nullptr;
  if (hipMallocAsync(reinterpret_cast<void**>(&out), sizeof(float) * blocks * kThreads, st) != hipSuccess) return -3;
  hipEvent_t a = nullptr, b = nullptr;
  int rc = 0;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) rc = -3;
  for (int r = 0; r <= reps && rc == 0; ++r) {
    if (r == 1 && hipEventRecord(a, st) != hipSuccess) rc = -3;
    switch (kind) {
      case MCRT_PROBE_STREAM_READ:
        hipLaunchKernelGGL(k_stream_read, dim3((unsigned)blocks), dim3(kThreads), 0, st,
                           static_cast<const float4*>(buf_dev), (unsigned long long)(buf_bytes / 16), out);
        break;
      case MCRT_PROBE_GATHER:
        hipLaunchKernelGGL(k_gather, dim3((unsigned)blocks), dim3(kThreads), 0, st, static_cast<const float*>(buf_dev),
                           elems - 1, out);
        break;
      case MCRT_PROBE_ATOMIC_SCATTERED:
        hipLaunchKernelGGL(k_atomic_scattered, dim3((unsigned)blocks), dim3(kThreads), 0, st,
                           static_cast<double*>(buf_dev), elems - 1);
        break;
      default:
        hipLaunchKernelGGL(k_atomic_coalesced, dim3((unsigned)blocks), dim3(kThreads), 0, st,
                           static_cast<double*>(buf_dev), elems - 1);
        break;
    }
    if (hipGetLastError() != hipSuccess) rc = -3;
  }
  if (rc == 0 && hipEventRecord(b, st) != hipSuccess) rc = -3;
  if (rc == 0 && hipEventSynchronize(b) != hipSuccess) rc = -3;
  float ms = 0.0f;
  if (rc == 0 && hipEventElapsedTime(&ms, a, b) != hipSuccess) rc = -3;
  if (rc == 0) *ms_host = ms / reps;
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  (void)hipFreeAsync(out, st);
  return rc;
}
