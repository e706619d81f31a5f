// Streaming probes for the roofline's reference rates on the GPU at hand: a
// plain device copy and a read-only pass over a buffer, each at a launch
// shape the caller chooses (the benchmark sweeps shapes and keeps the best).
// They give the bandwidth a kernel that only streams can reach, next to the
// nominal 8 TB/s of HBM, and the counter calibration of the traffic figures
// (a copy of known size read and written once).  Not part of the solver's
// C-ABI.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace {

constexpr int kUnroll = 4;
// 16-byte word (a native vector type, as the nontemporal builtins take)
typedef unsigned int w16 __attribute__((ext_vector_type(4)));

// Each thread moves kUnroll 16-byte words per iteration, loads first, with
// a grid-stride loop; the tail (fewer than a full iteration) is done by the
// first threads one word at a time.
__global__ void probe_copy_kernel(const w16* __restrict__ src, w16* __restrict__ dst,
                                  size_t n) {
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nth = (size_t)gridDim.x * blockDim.x;
  const size_t body = n / (nth * kUnroll) * (nth * kUnroll);
  for (size_t i = tid; i < body; i += nth * kUnroll) {
    w16 v[kUnroll];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) v[k] = __builtin_nontemporal_load(src + i + k * nth);
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) __builtin_nontemporal_store(v[k], dst + i + k * nth);
  }
  for (size_t i = body + tid; i < n; i += nth) dst[i] = src[i];
}

__global__ void probe_read_kernel(const w16* __restrict__ src, size_t n, unsigned* sink,
                                  unsigned magic) {
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nth = (size_t)gridDim.x * blockDim.x;
  const size_t body = n / (nth * kUnroll) * (nth * kUnroll);
  unsigned acc = 0;
  for (size_t i = tid; i < body; i += nth * kUnroll) {
    w16 v[kUnroll];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) v[k] = __builtin_nontemporal_load(src + i + k * nth);
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) acc ^= v[k].x ^ v[k].y ^ v[k].z ^ v[k].w;
  }
  for (size_t i = body + tid; i < n; i += nth) acc ^= src[i].x ^ src[i].w;
  // never true for the probe's data (the caller passes a value no XOR of the
  // buffer can give); keeps the loads from being removed
  if (acc == magic) sink[0] = acc;
}

}  // namespace

extern "C" {

// Copy `bytes` (a multiple of 16, 16-byte aligned pointers) with `blocks`
// workgroups of `threads` threads on `stream`.  Returns a hipError_t value.
int clf_probe_copy(const void* src, void* dst, size_t bytes, int blocks, int threads,
                   void* stream) {
  if (!src || !dst || bytes % 16 != 0 || blocks < 1 || threads < 64 || threads > 1024 ||
      ((uintptr_t)src | (uintptr_t)dst) % 16 != 0)
    return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(probe_copy_kernel, dim3(blocks), dim3(threads), 0, (hipStream_t)stream,
                     (const w16*)src, (w16*)dst, bytes / 16);
  return (int)hipGetLastError();
}

// Read `bytes` once; `sink` (device, 4 bytes) is written only if the XOR of
// a thread's words equals `magic`.
int clf_probe_read(const void* src, size_t bytes, unsigned* sink, unsigned magic, int blocks,
                   int threads, void* stream) {
  if (!src || !sink || bytes % 16 != 0 || blocks < 1 || threads < 64 || threads > 1024 ||
      (uintptr_t)src % 16 != 0)
    return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(probe_read_kernel, dim3(blocks), dim3(threads), 0, (hipStream_t)stream,
                     (const w16*)src, bytes / 16, sink, magic);
  return (int)hipGetLastError();
}

}  // extern "C"
