// Device helpers: wave64 reductions and scans, compensated sums, grid location.
#pragma once

#include <hip/hip_runtime.h>

#include "tsnet_internal.h"

namespace tsnet {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }
__device__ __forceinline__ int wave_id() { return threadIdx.x / kWave; }

// The dispatcher deals workgroups to the chip's 8 XCDs in turn (workgroup b
// to XCD b % 8), and each XCD has an L2 of its own. This renumbers the
// workgroups of a grid of nb so that XCD x takes one contiguous range of
// tiles (a bijection of [0, nb)): tiles that share cache lines, such as
// neighbouring columns of a digit-major count matrix or the adjacent output
// runs of a stable scatter, then meet in one L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int x = b % kXcds, q = b / kXcds, per = nb / kXcds, rem = nb % kXcds;
  return x * per + min(x, rem) + q;
}

// Cross-lane moves as DPP operand modifiers (VALU, no LDS traffic). Controls: row_shr:n / row_shl:n shift within rows of 16 lanes, row_bcast:15
// and :31 carry the last lane of a row (of rows 0-1) into the next row (rows
// 2-3), wave_shr:1 / wave_shl:1 shift by one lane across the whole wave.
// Lanes without a source keep `old`.
constexpr int kDppRowShr = 0x110;
constexpr int kDppRowShl1 = 0x101;
constexpr int kDppRowBcast15 = 0x142;
constexpr int kDppRowBcast31 = 0x143;
constexpr int kDppWaveShl1 = 0x130;
constexpr int kDppWaveShr1 = 0x138;

template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_i(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_f(float old, float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL,
                                                    ROWS, 0xF, false));
}

// Sum over the wave, in a fixed order, left in lane 63 (an inclusive prefix
// sum by DPP row shifts and row broadcasts; other lanes hold partial sums).
__device__ __forceinline__ float wave_sum_to_last(float v) {
  v += dpp_f<kDppRowShr | 1, 0xF>(0.f, v);
  v += dpp_f<kDppRowShr | 2, 0xF>(0.f, v);
  v += dpp_f<kDppRowShr | 4, 0xF>(0.f, v);
  v += dpp_f<kDppRowShr | 8, 0xF>(0.f, v);
  v += dpp_f<kDppRowBcast15, 0xA>(0.f, v);
  v += dpp_f<kDppRowBcast31, 0xC>(0.f, v);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, kWave));
  return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
  return v;
}

// Inclusive prefix sum across the wave.
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    T t = __shfl_up(v, o, kWave);
    if (l >= o) v += t;
  }
  return v;
}

// Exclusive block scan of one int per thread (blockDim.x <= 1024, multiple of 64).
// `sh` needs blockDim.x / 64 ints. Returns the exclusive prefix; *total gets the sum.
__device__ __forceinline__ int block_excl_scan(int v, int* sh, int* total) {
  const int nw = blockDim.x / kWave;
  int inc = wave_incl_scan(v);
  if (lane_id() == kWave - 1) sh[wave_id()] = inc;
  __syncthreads();
  if (threadIdx.x < kWave) {
    int t = threadIdx.x < nw ? sh[threadIdx.x] : 0;
    int ti = wave_incl_scan(t);
    if (threadIdx.x < nw) sh[threadIdx.x] = ti - t;
    if (threadIdx.x == nw - 1) sh[nw] = ti;
  }
  __syncthreads();
  int res = inc - v + sh[wave_id()];
  if (total) *total = sh[nw];
  __syncthreads();
  return res;
}

// Error-free transformation a + b = s + e (Knuth's TwoSum).
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Compensated FP32 accumulator: value = hi + lo.
struct CompSum {
  float hi = 0.f, lo = 0.f;
  __device__ __forceinline__ void add(float v) {
    float s, e;
    two_sum(hi, v, s, e);
    hi = s;
    lo += e;
  }
  __device__ __forceinline__ void merge(const CompSum& o) {
    float s, e;
    two_sum(hi, o.hi, s, e);
    hi = s;
    lo += e + o.lo;
  }
  __device__ __forceinline__ double value() const { return (double)hi + (double)lo; }
};

__device__ __forceinline__ CompSum wave_comp_sum(CompSum c) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    CompSum t;
    t.hi = __shfl_xor(c.hi, o, kWave);
    t.lo = __shfl_xor(c.lo, o, kWave);
    c.merge(t);
  }
  return c;
}

// Lagrange basis on the three nodes (t + 1/2) / 3 of a box, at local coordinate s.
// Denominators of the three cardinal polynomials: 2/9, -1/9, 2/9.
__device__ __forceinline__ void lagrange3(float s, float w[3]) {
  const float a = s - (1.0f / 6.0f), b = s - 0.5f, c = s - (5.0f / 6.0f);
  w[0] = 4.5f * b * c;
  w[1] = -9.0f * a * c;
  w[2] = 4.5f * a * b;
}

// Box of a point and its local coordinates in [0, 1]. NaN coordinates land in
// box 0 (the clamp absorbs them) so no index leaves the grid.
__device__ __forceinline__ void locate(const GridDesc& d, float x, float y, int& bx, int& by,
                                       float& s, float& t) {
  const float fx = (x - d.x0) / d.h;
  const float fy = (y - d.y0) / d.h;
  const float top = (float)(d.n_int - 1);
  const float cx = fminf(fmaxf(floorf(fx), 0.0f), top);
  const float cy = fminf(fmaxf(floorf(fy), 0.0f), top);
  bx = (int)cx;
  by = (int)cy;
  s = fx - cx;
  t = fy - cy;
}

// Loads that bypass the non-coherent per-CU cache: used where a block reads
// back values that its own threads wrote (the grid plan's descriptors).
template <typename T>
__device__ __forceinline__ T ld_coherent(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int graph_of(const int* goff, int G, int v) {
  int lo = 0, hi = G;  // goff[lo] <= v < goff[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (goff[mid] <= v) lo = mid; else hi = mid;
  }
  return lo;
}

}  // namespace tsnet
