// lcq_range.hpp -- NOA's range pass (section 2.1.3) for gfx950: the finite
// minimum and maximum of a field, then its parameters derived on the device.
// Shared by the plain quantizers and the fused compress path.
#pragma once
#include <hip/hip_runtime.h>

#include "lcq_math.hpp"
#include "lcq_tile.hpp"

namespace lcq {
constexpr int kMinmaxBlocks = 8192;  // range workgroups at most
}  // namespace lcq

namespace {

using namespace lcq;

// NOA pass 1: finite min / max of a contiguous share of the input.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_minmax(const T *in, uint64_t n, uint64_t share,
                                                   T *partials, uint64_t *clear,
                                                   uint64_t clear_count) {
  const uint64_t gtid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  const uint64_t gsize = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = gtid; i < clear_count; i += gsize) clear[i] = 0;
  const uint64_t b = min((uint64_t)blockIdx.x * share, n);
  const uint64_t e = min(b + share, n);
  T lo, hi;
  block_minmax<T>(in, b, e, lo, hi);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = lo;
    partials[2 * blockIdx.x + 1] = hi;
  }
}

// NOA pass 2: reduce the shares and derive the parameters.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_noa_params(const T *partials, int nparts, T eb_down,
                                                       DevParams *out) {
  T lo = (T)INFINITY, hi = (T)-INFINITY;
  // eight (min, max) pairs in flight per thread, then the rest one by one
  int i = threadIdx.x;
  for (; i + 7 * kBlock < nparts; i += 8 * kBlock) {
    T l[8], h[8];
#pragma unroll
    for (int u = 0; u < 8; u++) {
      l[u] = partials[2 * (i + u * kBlock)];
      h[u] = partials[2 * (i + u * kBlock) + 1];
    }
#pragma unroll
    for (int u = 0; u < 8; u++) {
      lo = fmin(lo, l[u]);
      hi = fmax(hi, h[u]);
    }
  }
  for (; i < nparts; i += kBlock) {
    lo = fmin(lo, partials[2 * i]);
    hi = fmax(hi, partials[2 * i + 1]);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o, 64));
    hi = fmax(hi, __shfl_xor(hi, o, 64));
  }
  __shared__ T s_lo[kWaves], s_hi[kWaves];
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_lo[wave] = lo;
    s_hi[wave] = hi;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int w = 1; w < kWaves; w++) {
    lo = fmin(lo, s_lo[w]);
    hi = fmax(hi, s_hi[w]);
  }
  *out = noa_params<T>(lo, hi, eb_down);
}

// Range pass of n values at d_in: per-workgroup (min, max) pairs into
// partials (2 * kMinmaxBlocks values of T), then the field's parameters into
// *out; the first kernel also zeroes clear[0..clear_count).
template <typename T>
void launch_noa_range(const T *d_in, uint64_t n, T *partials, uint64_t *clear,
                      uint64_t clear_count, T eb_down, DevParams *out, hipStream_t s) {
  // each workgroup reduces a contiguous share of whole 128-bit vectors
  const uint64_t W = 16 / sizeof(T);
  const uint64_t per = (uint64_t)kBlock * W * 8;  // >= 8 vectors per thread
  uint64_t nb = (n + per - 1) / per;
  nb = nb < 1 ? 1 : (nb > (uint64_t)kMinmaxBlocks ? kMinmaxBlocks : nb);
  uint64_t share = (n + nb - 1) / nb;
  share = (share + W - 1) / W * W;
  hipLaunchKernelGGL(k_minmax<T>, dim3((unsigned)nb), dim3(kBlock), 0, s, d_in, n, share,
                     partials, clear, clear_count);
  hipLaunchKernelGGL(k_noa_params<T>, dim3(1), dim3(kBlock), 0, s, partials, (int)nb, eb_down,
                     out);
}

}  // namespace
