// Streaming reference kernels: what plain HBM streaming reaches on the device,
// the yardstick beside the published peak for the sweep's roofline.  Each
// thread moves four 16-byte vectors per step (loads issued before stores);
// the grid strides over the buffer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mf {

constexpr int kStreamThreads = 256;
constexpr int kStreamUnroll = 4;
typedef uint32_t v4u __attribute__((ext_vector_type(4)));   // one 16-byte vector

// dst = src, n16 16-byte vectors.
template <bool NT>
__global__ void __launch_bounds__(kStreamThreads)
stream_copy_kernel(const v4u* __restrict__ src, v4u* __restrict__ dst, size_t n16) {
  const size_t step = static_cast<size_t>(gridDim.x) * kStreamThreads * kStreamUnroll;
  for (size_t base = static_cast<size_t>(blockIdx.x) * kStreamThreads * kStreamUnroll + threadIdx.x;
       base < n16; base += step) {
    v4u v[kStreamUnroll];
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u) {
      const size_t i = base + static_cast<size_t>(u) * kStreamThreads;
      if (i < n16) v[u] = NT ? __builtin_nontemporal_load(src + i) : src[i];
    }
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u) {
      const size_t i = base + static_cast<size_t>(u) * kStreamThreads;
      if (i < n16) {
        if (NT) __builtin_nontemporal_store(v[u], dst + i);
        else dst[i] = v[u];
      }
    }
  }
}

// Reads n16 16-byte vectors and writes one integer sum per workgroup to
// out[blockIdx.x] (so that the loads cannot be dropped).
template <bool NT>
__global__ void __launch_bounds__(kStreamThreads)
stream_read_kernel(const v4u* __restrict__ src, uint32_t* __restrict__ out, size_t n16) {
  __shared__ uint32_t red[kStreamThreads];
  const size_t step = static_cast<size_t>(gridDim.x) * kStreamThreads * kStreamUnroll;
  uint32_t acc = 0;
  for (size_t base = static_cast<size_t>(blockIdx.x) * kStreamThreads * kStreamUnroll + threadIdx.x;
       base < n16; base += step) {
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u) {
      const size_t i = base + static_cast<size_t>(u) * kStreamThreads;
      if (i < n16) {
        const v4u v = NT ? __builtin_nontemporal_load(src + i) : src[i];
        acc += v.x ^ v.y ^ v.z ^ v.w;
      }
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kStreamThreads / 2; s > 0; s >>= 1) {
    if (static_cast<int>(threadIdx.x) < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

}  // namespace mf
