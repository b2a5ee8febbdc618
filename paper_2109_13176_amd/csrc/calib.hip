// Roofline calibration kernels: the two reference rates the measurements of
// the mapping kernels are priced against on the device at hand.
//
//  * k_copy_bw: a plain device copy (16-byte streaming loads and stores),
//    the practical HBM rate and the scale for the FETCH_SIZE / WRITE_SIZE
//    counters (what they read for a copy of known size).
//  * k_atomic_peak: device-scope int32 atomic adds without return on
//    pseudo-random 64-byte lines, g lanes of a wave per line.  For g <= 16 the
//    g lanes add to g distinct words of the line; g = 64 puts four lanes on
//    each of the line's 16 words.  Every wave instruction therefore issues
//    64 / g line requests, which is the unit the memory side charges, so the
//    measured rate is reported both per lane update and per line request.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gvom.h"

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

// Block b copies the 1,024 16-byte elements 1024 b .. 1024 b + 1023: each
// lane loads four (256 apart) before it stores them, streaming (non-temporal)
// both ways.  This measured faster on the MI355X than grid-stride loops.
__global__ __launch_bounds__(256) void k_copy_bw(v4i* __restrict__ dst,
                                                 const v4i* __restrict__ src, int64_t n) {
  const int64_t base = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  v4i v[4];
#pragma unroll
  for (int k = 0; k < 4; k++)
    if (base + 256 * k < n) v[k] = __builtin_nontemporal_load(&src[base + 256 * k]);
#pragma unroll
  for (int k = 0; k < 4; k++)
    if (base + 256 * k < n) __builtin_nontemporal_store(v[k], &dst[base + 256 * k]);
}

// 32-bit mixing function (the finaliser of MurmurHash3 by Austin Appleby).
__device__ __forceinline__ uint32_t mix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

// Wave instruction k of global wave w: lane group j (64 / g groups) takes
// line mix(seed, w, k, j) mod n_lines; its lanes add 1 to their words.
__global__ __launch_bounds__(256) void k_atomic_peak(int32_t* __restrict__ tgt, uint32_t n_lines,
                                                     int32_t per_wave, int32_t g, uint32_t seed) {
  const int lane = threadIdx.x & 63;
  const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int grp = lane / g, sub = lane - grp * g;
  const int word = g >= 16 ? (sub & 15) : sub * (16 / g);
  for (int k = 0; k < per_wave; k++) {
    const uint32_t h = mix32(seed ^ mix32(wave * 0x9E3779B9u + (uint32_t)k * 0x7F4A7C15u + (uint32_t)grp));
    const uint32_t line = (uint32_t)(((uint64_t)h * n_lines) >> 32);
    __hip_atomic_fetch_add(&tgt[(int64_t)line * 16 + word], 1, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
  }
}

}  // namespace

extern "C" {

int32_t map_calib_copy(void* dst_dev, const void* src_dev, int64_t bytes, void* stream) {
  if (!dst_dev || !src_dev || bytes < 0 || (bytes & 15) ||
      (((uintptr_t)dst_dev | (uintptr_t)src_dev) & 15))
    return MAP_E_INVALID;
  if (bytes == 0) return MAP_OK;
  const int64_t n = bytes >> 4;
  const int64_t blocks = (n + 1023) / 1024;
  if (blocks > 0x7FFFFFFF) return MAP_E_INVALID;
  hipLaunchKernelGGL(k_copy_bw, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                     (v4i*)dst_dev, (const v4i*)src_dev, n);
  if (hipGetLastError() != hipSuccess) return MAP_E_DEVICE;
  return MAP_OK;
}

int32_t map_calib_atomic(int32_t* target_dev, int64_t n_words, int64_t n_waves,
                         int32_t per_wave, int32_t lanes_per_line, uint32_t seed, void* stream) {
  const int32_t g = lanes_per_line;
  if (!target_dev || n_words < 16 || n_words > (int64_t)0xFFFFFFFF * 16 || (n_words & 15) ||
      n_waves < 4 || n_waves > (1 << 24) || (n_waves & 3) || per_wave < 1 || per_wave > 4096 ||
      !(g == 1 || g == 2 || g == 4 || g == 8 || g == 16 || g == 64))
    return MAP_E_INVALID;
  // four waves per 256-thread block: n_waves is a multiple of 4
  hipLaunchKernelGGL(k_atomic_peak, dim3((unsigned)(n_waves / 4)), dim3(256), 0,
                     (hipStream_t)stream, target_dev, (uint32_t)(n_words / 16), per_wave, g, seed);
  if (hipGetLastError() != hipSuccess) return MAP_E_DEVICE;
  return MAP_OK;
}

}  // extern "C"
