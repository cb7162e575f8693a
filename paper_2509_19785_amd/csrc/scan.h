// Exclusive prefix sums of a host-known length: tile sums, then each tile
// scanned and offset by the sum of the tile sums before it (the block adds
// them itself while there are few tiles; beyond kScanDirectTiles a one-block
// scan of the tile sums runs in between). out may alias in.
#pragma once

#include <hip/hip_runtime.h>

#include "dev_util.h"

namespace tsnet {

constexpr int kTileScan = 2048;

template <typename T>
__global__ __launch_bounds__(256) void k_tile_sum(const T* __restrict__ in, int64_t N, T* tsum) {
  const int64_t base = (int64_t)blockIdx.x * kTileScan;
  T v = 0;
  for (int k2 = threadIdx.x; k2 < kTileScan; k2 += blockDim.x) {
    const int64_t i = base + k2;
    if (i < N) v += in[i];
  }
  v = wave_sum(v);
  __shared__ T sh[4];
  if (lane_id() == 0) sh[wave_id()] = v;
  __syncthreads();
  if (threadIdx.x == 0) tsum[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

template <typename T>
__global__ __launch_bounds__(1024) void k_scan_sums(T* tsum, int T_) {
  __shared__ T sh[17];
  T carry = 0;
  for (int base = 0; base < T_; base += 1024) {
    const int i = base + threadIdx.x;
    const T v = i < T_ ? tsum[i] : 0;
    T inc = wave_incl_scan(v);
    if (lane_id() == kWave - 1) sh[wave_id()] = inc;
    __syncthreads();
    if (threadIdx.x < kWave) {
      const T t = threadIdx.x < 16 ? sh[threadIdx.x] : 0;
      const T ti = wave_incl_scan(t);
      if (threadIdx.x < 16) sh[threadIdx.x] = ti - t;
      if (threadIdx.x == 15) sh[16] = ti;
    }
    __syncthreads();
    if (i < T_) tsum[i] = carry + inc - v + sh[wave_id()];
    carry += sh[16];
    __syncthreads();
  }
}

constexpr int kScanDirectTiles = 4096;

// out[i] = exclusive prefix of in; out[N] = total. tsum holds the exclusive
// prefix of the tile sums (SUMS_SCANNED) or the tile sums themselves, which
// the block then adds up for the tiles before its own.
template <typename T, bool SUMS_SCANNED>
__global__ __launch_bounds__(256) void k_scan_out(const T* __restrict__ in, int64_t N,
                                                  const T* __restrict__ tsum, T* out) {
  constexpr int per = kTileScan / 256;
  __shared__ T pre_sh[5];
  T pre = 0;
  if constexpr (SUMS_SCANNED) {
    pre = tsum[blockIdx.x];
  } else {
    for (int k = threadIdx.x; k < (int)blockIdx.x; k += 256) pre += tsum[k];
    pre = wave_sum(pre);
    if (lane_id() == 0) pre_sh[wave_id()] = pre;
    __syncthreads();
    pre = pre_sh[0] + pre_sh[1] + pre_sh[2] + pre_sh[3];
  }
  const int64_t first = (int64_t)blockIdx.x * kTileScan + threadIdx.x * per;
  T loc[per];
  T sum = 0;
#pragma unroll
  for (int q = 0; q < per; ++q) {
    const int64_t i = first + q;
    loc[q] = i < N ? in[i] : 0;
    sum += loc[q];
  }
  __shared__ T sh[5];
  T inc = wave_incl_scan(sum);
  if (lane_id() == kWave - 1) sh[wave_id()] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    T acc = 0;
    for (int w = 0; w < 4; ++w) {
      const T t = sh[w];
      sh[w] = acc;
      acc += t;
    }
  }
  __syncthreads();
  T run = pre + sh[wave_id()] + inc - sum;
#pragma unroll
  for (int q = 0; q < per; ++q) {
    const int64_t i = first + q;
    if (i < N) out[i] = run;
    run += loc[q];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 255) out[N] = run;
}

template <typename T>
__global__ void k_scan_empty(T* out) {
  if (threadIdx.x == 0) out[0] = 0;
}

// tsum needs ceil(N / kTileScan) entries; out needs N + 1. No memset: the
// calls may be captured into a graph.
template <typename T>
inline hipError_t exclusive_scan(const T* in, int64_t N, T* out, T* tsum, hipStream_t s) {
  const int tiles = (int)((N + kTileScan - 1) / kTileScan);
  if (tiles == 0) {
    hipLaunchKernelGGL(k_scan_empty<T>, dim3(1), dim3(64), 0, s, out);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_tile_sum<T>, dim3(tiles), dim3(256), 0, s, in, N, tsum);
  if (tiles <= kScanDirectTiles) {
    hipLaunchKernelGGL((k_scan_out<T, false>), dim3(tiles), dim3(256), 0, s, in, N, tsum, out);
  } else {
    hipLaunchKernelGGL(k_scan_sums<T>, dim3(1), dim3(1024), 0, s, tsum, tiles);
    hipLaunchKernelGGL((k_scan_out<T, true>), dim3(tiles), dim3(256), 0, s, in, N, tsum, out);
  }
  return hipGetLastError();
}

}  // namespace tsnet
