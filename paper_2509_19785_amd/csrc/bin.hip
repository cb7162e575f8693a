// Binning of points by interpolation box and the spread to the nodes.
//
// Binning: stable LSD radix sort (9-bit digits: two passes cover the 2^18
// boxes of a 512 x 512 grid) of the global box id of every point. Tiles of 2048 points rank their digits in LDS with wave ballots, so
// no global atomics are needed and the order is deterministic (by box, then
// by vertex id). Pass 0 computes the keys from X; the last pass also gathers
// X into sorted order. box_off[b] is the first sorted slot of box b.
//
// Spread (Sec. 2.3): node charge w[c][a] = sum over the points of the node's
// box of L_tx(s) L_ty(t) q_c, q = (1, (x - cx) / half, (y - cy) / half).
// Every contribution is rounded to a 2^-28 grid and summed in 64-bit
// integers, so the totals do not depend on the summation order. Phase 1:
// one wave per range of 256 sorted points, a segmented wave reduction by box;
// boxes entirely inside the range are written directly, the box pieces at the
// two ends of the range are kept as partials. Phase 2: one wave per box adds
// the partials of boxes that span ranges and clears empty boxes.
#include <hip/hip_runtime.h>

#include "dev_util.h"
#include "scan.h"
#include "tsnet_internal.h"

namespace tsnet {

typedef unsigned long long u64;
constexpr int kBinTile = 2048;
constexpr int kDigitBits = kBinDigitBits;
constexpr int kDigits = 1 << kDigitBits;   // buckets per pass

__device__ __forceinline__ int box_key(const GridDesc& d, float x, float y) {
  int bx, by;
  float s, t;
  locate(d, x, y, bx, by, s, t);
  return d.box_base + by * d.n_int + bx;
}

// Pass 0: keys of tile `blockIdx.x` and its digit histogram.
__global__ __launch_bounds__(256) void k_bin_keys(const float2* __restrict__ X, int n,
                                                  const int* __restrict__ goff, int G,
                                                  const GridDesc* __restrict__ desc, int* keys,
                                                  int tiles, int* hist) {
  __shared__ int cnt[kDigits];
  for (int q = threadIdx.x; q < kDigits; q += 256) cnt[q] = 0;
  __syncthreads();
  const int base = blockIdx.x * kBinTile;
  for (int q = threadIdx.x; q < kBinTile; q += 256) {
    const int i = base + q;
    if (i < n) {
      const int g = G == 1 ? 0 : graph_of(goff, G, i);
      const float2 p = X[i];
      const int key = box_key(desc[g], p.x, p.y);
      keys[i] = key;
      atomicAdd(&cnt[key & (kDigits - 1)], 1);
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < kDigits; q += 256) hist[q * tiles + blockIdx.x] = cnt[q];
}

__global__ __launch_bounds__(256) void k_bin_hist(const int* __restrict__ keys, int n, int shift,
                                                  int tiles, int* hist) {
  __shared__ int cnt[kDigits];
  for (int q = threadIdx.x; q < kDigits; q += 256) cnt[q] = 0;
  __syncthreads();
  const int base = blockIdx.x * kBinTile;
  for (int q = threadIdx.x; q < kBinTile; q += 256) {
    const int i = base + q;
    if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & (kDigits - 1)], 1);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < kDigits; q += 256) hist[q * tiles + blockIdx.x] = cnt[q];
}

// Stable scatter of one pass. vin == nullptr means the payload is the index.
// When Xs != nullptr (last pass) X[payload] is written to Xs in sorted order.
__global__ __launch_bounds__(256) void k_bin_scatter(const int* __restrict__ kin,
                                                     const int* __restrict__ vin, int n, int shift,
                                                     int tiles, const int* __restrict__ offs,
                                                     int* kout, int* vout,
                                                     const float2* __restrict__ X, float2* Xs) {
  __shared__ int run[kDigits];
  __shared__ int wc[4][kDigits];
  const int tid = threadIdx.x, w = wave_id(), lane = lane_id();
  for (int d = tid; d < kDigits; d += 256) {
    run[d] = offs[d * tiles + blockIdx.x];
    for (int q = 0; q < 4; ++q) wc[q][d] = 0;
  }
  __syncthreads();
  const u64 lt = (1ull << lane) - 1ull;
  const int base = blockIdx.x * kBinTile;
  for (int round = 0; round < kBinTile / 256; ++round) {
    const int i = base + round * 256 + tid;
    const bool valid = i < n;
    int key = 0, val = 0, dg = 0;
    if (valid) {
      key = kin[i];
      val = vin ? vin[i] : i;
      dg = (key >> shift) & (kDigits - 1);
    }
    const u64 vb = __ballot(valid);
    u64 peers = valid ? vb : ~vb;
#pragma unroll
    for (int b = 0; b < kDigitBits; ++b) {
      const bool bit = (dg >> b) & 1;
      const u64 bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    const int rank_w = __popcll(peers & lt);
    if (valid && (peers & lt) == 0) wc[w][dg] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int pos = run[dg] + rank_w;
      for (int q = 0; q < w; ++q) pos += wc[q][dg];
      kout[pos] = key;
      vout[pos] = val;
      if (Xs) Xs[pos] = X[val];
    }
    __syncthreads();
    for (int d = tid; d < kDigits; d += 256) {
      run[d] += wc[0][d] + wc[1][d] + wc[2][d] + wc[3][d];
      for (int q = 0; q < 4; ++q) wc[q][d] = 0;
    }
    __syncthreads();
  }
}

// box_off[b] = first sorted slot with key >= b, for b in [0, btotal]
// (a binary search per box, so long runs of empty boxes cost nothing extra).
__global__ __launch_bounds__(256) void k_box_bounds(const int* __restrict__ skeys, int n,
                                                    const int* __restrict__ btotal, int* box_off) {
  const int B = *btotal;
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b <= B; b += gridDim.x * blockDim.x) {
    int lo = 0, hi = n;
    while (lo < hi) {
      const int m = (lo + hi) >> 1;
      if (skeys[m] < b) lo = m + 1; else hi = m;
    }
    box_off[b] = lo;
  }
}

hipError_t launch_bin(Problem& P, const float2* X, hipStream_t s) {
  const int n = P.n;
  const int tiles = (n + kBinTile - 1) / kBinTile;
  int bits = 1;
  while (((int64_t)1 << bits) < (int64_t)P.G * P.cap * P.cap) ++bits;
  const int passes = (bits + kDigitBits - 1) / kDigitBits;
  // pass p reads (kin, vin) and writes the final pair on the last pass, else
  // alternates between (keys_tmp, perm_tmp) and (keys, perm_tmp2); keys is
  // free once pass 0 has read it.
  int* kin = P.keys;
  int* vin = nullptr;
  hipLaunchKernelGGL(k_bin_keys, dim3(tiles), dim3(256), 0, s, X, n, P.goff_d, P.G, P.desc, P.keys,
                     tiles, P.bin_hist);
  for (int p = 0; p < passes; ++p) {
    const int shift = kDigitBits * p;
    if (p > 0)
      hipLaunchKernelGGL(k_bin_hist, dim3(tiles), dim3(256), 0, s, kin, n, shift, tiles, P.bin_hist);
    hipError_t e = exclusive_scan<int>(P.bin_hist, (int64_t)kDigits * tiles, P.bin_hist, P.bin_tsum, s);
    if (e != hipSuccess) return e;
    const bool last = p == passes - 1;
    int *kout, *vout;
    if (last) {
      kout = P.skeys;
      vout = P.perm;
    } else if (p % 2 == 0) {
      kout = P.keys_tmp;
      vout = P.perm_tmp;
    } else {
      kout = P.keys;
      vout = P.perm_tmp2;
    }
    hipLaunchKernelGGL(k_bin_scatter, dim3(tiles), dim3(256), 0, s, kin, vin, n, shift, tiles,
                       P.bin_hist, kout, vout, X, last ? P.xs : nullptr);
    kin = kout;
    vin = vout;
  }
  int bb = (P.G * P.cap * P.cap + 1 + 255) / 256;
  if (bb > 4096) bb = 4096;
  hipLaunchKernelGGL(k_box_bounds, dim3(bb), dim3(256), 0, s, P.skeys, n, P.btotal, P.box_off);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
constexpr int kRange = 256;  // sorted points per wave in spread phase 1
constexpr int kVals = 27;    // 9 nodes x 3 charges

__device__ __forceinline__ void node_store(float* out, int ng, int bx, int by, const long long* v) {
  const double inv = 1.0 / (double)kFixScale;
#pragma unroll
  for (int ty = 0; ty < 3; ++ty)
#pragma unroll
    for (int tx = 0; tx < 3; ++tx) {
      const size_t node = (size_t)(3 * by + ty) * ng + (3 * bx + tx);
      const int k = (ty * 3 + tx) * 3;
#pragma unroll
      for (int c = 0; c < 3; ++c) out[(size_t)c * ng * ng + node] = (float)((double)v[k + c] * inv);
    }
}

__device__ __forceinline__ int graph_of_box(const GridDesc* __restrict__ desc, int G, int key) {
  int lo = 0, hi = G;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (desc[mid].box_base <= key) lo = mid; else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(256) void k_spread_ranges(
    const float2* __restrict__ Xs, const int* __restrict__ skeys, int n,
    const int* __restrict__ box_off, const GridDesc* __restrict__ desc, int G, float* charges,
    size_t stride, int* head_box, int* tail_box, long long* head_val, long long* tail_val) {
  const int lane = lane_id();
  const u64 le = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  const int nranges = (n + kRange - 1) / kRange;
  const int nw = blockDim.x / kWave;
  for (int r = blockIdx.x * nw + wave_id(); r < nranges; r += gridDim.x * nw) {
    const int p0 = r * kRange;
    const int p1 = p0 + kRange < n ? p0 + kRange : n;
    if (lane == 0) {
      head_box[r] = -1;
      tail_box[r] = -1;
    }
    long long carry[kVals];
#pragma unroll
    for (int q = 0; q < kVals; ++q) carry[q] = 0;
    int carry_key = -1, carry_start = p0;
    for (int sp = p0; sp < p1; sp += kWave) {
      const int p = sp + lane;
      const bool valid = p < p1;
      const int key = valid ? skeys[p] : -2 - lane;
      long long v[kVals];
#pragma unroll
      for (int q = 0; q < kVals; ++q) v[q] = 0;
      int g = 0, bx = 0, by = 0;
      if (valid) {
        g = G == 1 ? 0 : graph_of_box(desc, G, key);
        const GridDesc d = desc[g];
        const int local = key - d.box_base;
        by = local / d.n_int;
        bx = local - by * d.n_int;
        const float2 x = Xs[p];
        const float s = (x.x - d.x0) / d.h - (float)bx;
        const float t = (x.y - d.y0) / d.h - (float)by;
        float lx[3], ly[3];
        lagrange3(s, lx);
        lagrange3(t, ly);
        const float inv_half = 1.0f / d.half;
        const float q1 = (x.x - d.cx) * inv_half, q2 = (x.y - d.cy) * inv_half;
#pragma unroll
        for (int ty = 0; ty < 3; ++ty)
#pragma unroll
          for (int tx = 0; tx < 3; ++tx) {
            const float w = ly[ty] * lx[tx];
            const int k = (ty * 3 + tx) * 3;
            v[k + 0] = __float2int_rn(fminf(fmaxf(w, -4.0f), 4.0f) * kFixScale);
            v[k + 1] = __float2int_rn(fminf(fmaxf(w * q1, -4.0f), 4.0f) * kFixScale);
            v[k + 2] = __float2int_rn(fminf(fmaxf(w * q2, -4.0f), 4.0f) * kFixScale);
          }
      }
      const int prev_key = __shfl_up(key, 1, kWave);
      const bool head = lane == 0 ? key != carry_key : key != prev_key;
      if (lane == 0 && !head) {
#pragma unroll
        for (int q = 0; q < kVals; ++q) v[q] += carry[q];
      }
      // segmented inclusive scan: (v, h) combine as h2 ? v2 : v1 + v2
      bool h = head;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const bool hh = __shfl_up(h, o, kWave);
        const bool take = lane >= o && !h;
#pragma unroll
        for (int q = 0; q < kVals; ++q) {
          const long long vv = __shfl_up(v[q], o, kWave);
          if (take) v[q] += vv;
        }
        if (lane >= o) h = h || hh;
      }
      const u64 heads = __ballot(head);
      const u64 hb = heads & le;
      const int seg_start = hb ? sp + 63 - __clzll(hb) : carry_start;
      // key of the next sorted point (lane 63 looks into the next step)
      int next_key = __shfl_down(key, 1, kWave);
      if (lane == kWave - 1) next_key = p + 1 < p1 ? skeys[p + 1] : -1;
      const bool last_pt = p == p1 - 1;
      const bool ends = valid && (last_pt || next_key != key);
      if (ends) {
        const GridDesc d = desc[g];
        const int bs = box_off[key], be = box_off[key + 1];
        float* out = charges + (size_t)g * stride;
        if (seg_start == bs && p == be - 1) {
          node_store(out, d.ng, bx, by, v);
        } else if (seg_start == p0) {
          head_box[r] = key;
#pragma unroll
          for (int q = 0; q < kVals; ++q) head_val[(size_t)r * kVals + q] = v[q];
        } else {
          tail_box[r] = key;
#pragma unroll
          for (int q = 0; q < kVals; ++q) tail_val[(size_t)r * kVals + q] = v[q];
        }
      }
      // the segment of lane 63 continues into the next step
#pragma unroll
      for (int q = 0; q < kVals; ++q) carry[q] = __shfl(v[q], kWave - 1, kWave);
      carry_key = __shfl(key, kWave - 1, kWave);
      carry_start = __shfl(seg_start, kWave - 1, kWave);
    }
  }
}

// Phase 2: empty boxes get zero nodes, boxes whose points span several
// ranges add up the head and tail partials of those ranges (integer sums, so
// the order does not matter). Boxes that phase 1 wrote whole are skipped.
// One thread per box; a box spanning more than kDenseRanges ranges (a dense
// cluster of points) is summed by its whole wave instead, lanes over ranges.
constexpr int kDenseRanges = 4;

__device__ __forceinline__ const long long* partial_of(int r, int b, const int* head_box,
                                                       const long long* head_val,
                                                       const long long* tail_val) {
  return head_box[r] == b ? head_val + (size_t)r * kVals : tail_val + (size_t)r * kVals;
}

__global__ __launch_bounds__(256) void k_spread_boxes(
    const int* __restrict__ box_off, const int* __restrict__ btotal,
    const GridDesc* __restrict__ desc, int G, float* charges, size_t stride,
    const int* __restrict__ head_box, const int* __restrict__ tail_box,
    const long long* __restrict__ head_val, const long long* __restrict__ tail_val) {
  const int B = *btotal;
  const int lane = lane_id();
  const int nwaves = gridDim.x * (blockDim.x / kWave);
  // every lane of a wave runs the same number of rounds (ballots below)
  for (int base = (blockIdx.x * (blockDim.x / kWave) + wave_id()) * kWave; base < B;
       base += nwaves * kWave) {
    const int b = base + lane;
    int r0 = 0, r1 = -1, bs = 0, be = 0;
    if (b < B) {
      bs = box_off[b];
      be = box_off[b + 1];
      if (be > bs) {
        r0 = bs / kRange;
        r1 = (be - 1) / kRange;
      }
    }
    const bool mine = b < B && !(be > bs && r0 == r1);  // not written whole by phase 1
    const bool dense = mine && r1 - r0 >= kDenseRanges;
    if (mine && !dense) {
      long long acc[kVals];
#pragma unroll
      for (int q = 0; q < kVals; ++q) acc[q] = 0;
      for (int r = r0; r <= r1; ++r) {
        const long long* src = partial_of(r, b, head_box, head_val, tail_val);
#pragma unroll
        for (int q = 0; q < kVals; ++q) acc[q] += src[q];
      }
      const int g = G == 1 ? 0 : graph_of_box(desc, G, b);
      const GridDesc d = desc[g];
      const int local = b - d.box_base;
      const int by = local / d.n_int, bx = local - by * d.n_int;
      node_store(charges + (size_t)g * stride, d.ng, bx, by, acc);
    }
    u64 todo = __ballot(dense);
    while (todo) {
      const int src_lane = __ffsll((long long)todo) - 1;
      todo &= todo - 1;
      const int bd = __shfl(b, src_lane, kWave);
      const int d0 = __shfl(r0, src_lane, kWave), d1 = __shfl(r1, src_lane, kWave);
      long long acc[kVals];
#pragma unroll
      for (int q = 0; q < kVals; ++q) acc[q] = 0;
      for (int r = d0 + lane; r <= d1; r += kWave) {
        const long long* src = partial_of(r, bd, head_box, head_val, tail_val);
#pragma unroll
        for (int q = 0; q < kVals; ++q) acc[q] += src[q];
      }
#pragma unroll
      for (int q = 0; q < kVals; ++q) acc[q] = wave_sum(acc[q]);
      if (lane == 0) {
        const int g = G == 1 ? 0 : graph_of_box(desc, G, bd);
        const GridDesc d = desc[g];
        const int local = bd - d.box_base;
        const int by = local / d.n_int, bx = local - by * d.n_int;
        node_store(charges + (size_t)g * stride, d.ng, bx, by, acc);
      }
    }
  }
}

hipError_t launch_spread(Problem& P, const float2* X, hipStream_t s) {
  (void)X;
  const int nranges = (P.n + kRange - 1) / kRange;
  int blocks = (nranges + 3) / 4;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_spread_ranges, dim3(blocks), dim3(256), 0, s, P.xs, P.skeys, P.n, P.box_off,
                     P.desc, P.G, P.charges, P.stride_charges, P.head_box, P.tail_box, P.head_val,
                     P.tail_val);
  int bblocks = (P.G * P.cap * P.cap + 255) / 256;
  if (bblocks > 8192) bblocks = 8192;
  hipLaunchKernelGGL(k_spread_boxes, dim3(bblocks), dim3(256), 0, s, P.box_off, P.btotal, P.desc,
                     P.G, P.charges, P.stride_charges, P.head_box, P.tail_box, P.head_val,
                     P.tail_val);
  return hipGetLastError();
}

}  // namespace tsnet
