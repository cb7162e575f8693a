// Binning of points by interpolation box and the spread to the nodes.
//
// Binning: stable LSD radix sort (10-bit digits: two passes cover the
// 2^18 + 1 boxes of a 512 x 512 grid and its far box) of the global box id
// of every point. Tiles of 2048 points rank their digits in LDS with wave
// ballots, so no global atomics are needed and the order is deterministic
// (by box, then by vertex id). Pass 0 computes the keys from X; the last
// pass also gathers X into sorted order. Per pass, the counts of the digits
// that occur are kept digit-major (one row per digit, one count per tile),
// turned into row prefixes one wave per row, and each scatter tile adds the
// digit bases itself. box_off[b] is the first sorted slot of box b.
//
// Spread (Sec. 2.3): node charge w[c][a] = sum over the points of the node's
// box of L_tx(s) L_ty(t) q_c, q = (1, (x - cx) / half, (y - cy) / half).
// The points of a box are contiguous after the sort. Phase 1 cuts the sorted
// points into ranges of 1024, one wave each, and sums every box's piece of a
// range in FP32 in a fixed order (a lane per short piece, the whole wave for a
// long one); whole boxes go straight to their nodes, the pieces at the two
// ends of a range are kept as partials. Phase 2 adds the partials of boxes
// that span ranges, in range order. Empty boxes keep the zeros written while
// the box offsets are found.
#include <hip/hip_runtime.h>

#include "dev_util.h"
#include "tsnet_internal.h"

namespace tsnet {

typedef unsigned long long u64;
constexpr int kBinTile = 2048;
constexpr int kBinRounds = kBinTile / 256;  // points per thread of a tile
constexpr int kDigitBits = kBinDigitBits;
constexpr int kDigits = 1 << kDigitBits;   // buckets per pass

// Digit values that occur in pass `shift` when the keys lie in [0, B): rows
// of the digit-major count matrix past them stay unwritten and unscanned.
__device__ __forceinline__ int digits_used(int B, int shift) {
  return min(kDigits, ((max(B, 1) - 1) >> shift) + 1);
}

// Bin of a coordinate under the far-point rule (the grid plan's function).
__device__ __forceinline__ int trim_bin_of(float v, float vmin, double s) {
  const double f = floor(((double)v - (double)vmin) * s);
  return f >= 0.0 ? (f < (double)(kTrimBins - 1) ? (int)f : kTrimBins - 1) : 0;
}

// Global box id of a point: its core box, or its graph's far box when the
// plan set far points apart and the point's bins leave the core bins.
__device__ __forceinline__ int box_key(const GridDesc& d, float x, float y) {
  if (d.trimmed) {
    const int bx = trim_bin_of(x, d.bmin_x, d.s_x), by = trim_bin_of(y, d.bmin_y, d.s_y);
    if (bx < d.lo_x || bx > d.hi_x || by < d.lo_y || by > d.hi_y) return far_key(d);
  }
  int bx, by;
  float s, t;
  locate(d, x, y, bx, by, s, t);
  return d.box_base + by * d.n_int + bx;
}

// Pass 0: keys of one tile and its digit histogram.
__global__ __launch_bounds__(256) void k_bin_keys(const float2* __restrict__ X, int n,
                                                  const int* __restrict__ vgraph, int G,
                                                  const GridDesc* __restrict__ desc, int* keys,
                                                  int tiles, const int* __restrict__ btotal,
                                                  int* hist) {
  __shared__ int cnt[kDigits];
  for (int q = threadIdx.x; q < kDigits; q += 256) cnt[q] = 0;
  __syncthreads();
  const int tile = xcd_tile(blockIdx.x, gridDim.x), base = tile * kBinTile;
  float2 p[kBinRounds];  // every load of the tile issued before any is used
#pragma unroll
  for (int r = 0; r < kBinRounds; ++r) p[r] = X[min(base + r * 256 + (int)threadIdx.x, n - 1)];
#pragma unroll
  for (int r = 0; r < kBinRounds; ++r) {
    const int i = base + r * 256 + threadIdx.x;
    if (i < n) {
      const int g = G == 1 ? 0 : vgraph[i];
      const int key = box_key(desc[g], p[r].x, p[r].y);
      keys[i] = key;
      atomicAdd(&cnt[key & (kDigits - 1)], 1);
    }
  }
  __syncthreads();
  const int D = digits_used(*btotal, 0);
  for (int q = threadIdx.x; q < D; q += 256) hist[q * tiles + tile] = cnt[q];
}

__global__ __launch_bounds__(256) void k_bin_hist(const int* __restrict__ keys, int n, int shift,
                                                  int tiles, const int* __restrict__ btotal,
                                                  int* hist) {
  __shared__ int cnt[kDigits];
  for (int q = threadIdx.x; q < kDigits; q += 256) cnt[q] = 0;
  __syncthreads();
  const int tile = xcd_tile(blockIdx.x, gridDim.x), base = tile * kBinTile;
  int k[kBinRounds];  // every load of the tile issued before any is used
#pragma unroll
  for (int r = 0; r < kBinRounds; ++r) k[r] = keys[min(base + r * 256 + (int)threadIdx.x, n - 1)];
#pragma unroll
  for (int r = 0; r < kBinRounds; ++r)
    if (base + r * 256 + (int)threadIdx.x < n) atomicAdd(&cnt[(k[r] >> shift) & (kDigits - 1)], 1);
  __syncthreads();
  const int D = digits_used(*btotal, shift);
  for (int q = threadIdx.x; q < D; q += 256) hist[q * tiles + tile] = cnt[q];
}

// Offsets of a pass, in two steps instead of a scan of the whole count
// matrix: here one wave per digit row replaces the row's counts (one per
// tile) by their exclusive prefix and writes the row total; the scatter adds
// the exclusive prefix of the row totals over the digits. Rows of digits that
// occur in no key are skipped.
constexpr int kRowBatch = 8;  // loads of a row in flight together, per lane
__global__ __launch_bounds__(256) void k_bin_rowscan(int* hist, int tiles, int shift,
                                                     const int* __restrict__ btotal, int* rtot) {
  const int q = blockIdx.x * (256 / kWave) + wave_id(), lane = lane_id();
  if (q >= digits_used(*btotal, shift)) return;
  int* row = hist + (size_t)q * tiles;
  int carry = 0;
  for (int t0 = 0; t0 < tiles; t0 += kRowBatch * kWave) {
    int v[kRowBatch];
#pragma unroll
    for (int j = 0; j < kRowBatch; ++j) {
      const int t = t0 + j * kWave + lane;
      v[j] = t < tiles ? row[t] : 0;
    }
#pragma unroll
    for (int j = 0; j < kRowBatch; ++j) {
      const int t = t0 + j * kWave + lane;
      const int inc = wave_incl_scan(v[j]);
      if (t < tiles) row[t] = carry + inc - v[j];
      carry += __builtin_amdgcn_readlane(inc, kWave - 1);
    }
  }
  if (lane == 0) rtot[q] = carry;
}

// Stable scatter of one pass. vin == nullptr means the payload is the index.
// When Xs != nullptr (last pass) X[payload] is written to Xs in sorted order.
__global__ __launch_bounds__(256) void k_bin_scatter(const int* __restrict__ kin,
                                                     const int* __restrict__ vin, int n, int shift,
                                                     int tiles, const int* __restrict__ btotal,
                                                     const int* __restrict__ rowpre,
                                                     const int* __restrict__ rtot,
                                                     int* kout, int* vout,
                                                     const float2* __restrict__ X, float2* Xs) {
  __shared__ int run[kDigits];
  __shared__ int wc[4][kDigits];
  __shared__ int sh[256 / kWave + 1];
  const int tid = threadIdx.x, w = wave_id(), lane = lane_id();
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int D = digits_used(*btotal, shift);  // digits past D occur in no key
  // first slot of every digit of this tile: the digit's base (the totals of
  // the digits below it) plus the tile's prefix within the digit's row
  constexpr int DPT = kDigits / 256;  // consecutive digits per thread
  int tot[DPT], pre[DPT], local = 0;
#pragma unroll
  for (int k = 0; k < DPT; ++k) {
    const int d = tid * DPT + k;
    tot[k] = d < D ? rtot[d] : 0;
    pre[k] = d < D ? rowpre[(size_t)d * tiles + tile] : 0;
    local += tot[k];
  }
  int dbase = block_excl_scan(local, sh, nullptr);
#pragma unroll
  for (int k = 0; k < DPT; ++k) {
    const int d = tid * DPT + k;
    run[d] = dbase + pre[k];
    dbase += tot[k];
    for (int q = 0; q < 4; ++q) wc[q][d] = 0;
  }
  __syncthreads();
  const u64 lt = (1ull << lane) - 1ull;
  const int base = tile * kBinTile;
  // the tile's keys and payloads (and on the last pass the X rows they name)
  // are loaded before the first round: one memory latency per tile, not one
  // per round
  int kr[kBinRounds], vr[kBinRounds];
#pragma unroll
  for (int r = 0; r < kBinRounds; ++r) {
    const int ic = min(base + r * 256 + tid, n - 1);
    kr[r] = kin[ic];
    vr[r] = vin ? vin[ic] : ic;
  }
  float2 xr[kBinRounds];
  if (Xs) {
#pragma unroll
    for (int r = 0; r < kBinRounds; ++r) xr[r] = X[vr[r]];
  }
#pragma unroll
  for (int round = 0; round < kBinRounds; ++round) {
    const int i = base + round * 256 + tid;
    const bool valid = i < n;
    const int key = kr[round], val = vr[round];
    const int dg = valid ? (key >> shift) & (kDigits - 1) : 0;
    const u64 vb = __ballot(valid);
    u64 peers = valid ? vb : ~vb;
#pragma unroll
    for (int b = 0; b < kDigitBits; ++b) {
      const bool bit = (dg >> b) & 1;
      const u64 bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    const int rank_w = __popcll(peers & lt);
    const bool leader = valid && (peers & lt) == 0;  // first lane of its digit in the wave
    if (leader) wc[w][dg] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int pos = run[dg] + rank_w;
      for (int q = 0; q < w; ++q) pos += wc[q][dg];
      kout[pos] = key;
      vout[pos] = val;
      if (Xs) Xs[pos] = xr[round];
    }
    __syncthreads();
    // only the digits of this round move on: each wave's leader adds its
    // count (integer sums, so the order of the adds does not matter) and
    // clears its own slot; the next round's first barrier orders these
    // against its reads
    if (leader) {
      atomicAdd(&run[dg], wc[w][dg]);
      wc[w][dg] = 0;
    }
  }
}

// box_off[b] = first sorted slot with key >= b, for b in [0, btotal]
// (a binary search per box, so long runs of empty boxes cost nothing extra).
// The same launch clears the charge grids of every graph with 16-byte stores,
// so the spread writes only the boxes that hold points.
__global__ __launch_bounds__(256) void k_box_bounds(const int* __restrict__ skeys, int n,
                                                    const int* __restrict__ btotal, int* box_off,
                                                    const GridDesc* __restrict__ desc, int G,
                                                    float* charges) {
  const int B = *btotal;
  const int t0 = blockIdx.x * blockDim.x + threadIdx.x, nt = gridDim.x * blockDim.x;
  for (int b = t0; b <= B; b += nt) {
    int lo = 0, hi = n;
    while (lo < hi) {
      const int m = (lo + hi) >> 1;
      if (skeys[m] < b) lo = m + 1; else hi = m;
    }
    box_off[b] = lo;
  }
  // the graphs' charge grids lie back to back in the pool (each part a
  // multiple of 64 floats): one flat sweep clears all of them
  const size_t len4 = (desc[G - 1].off_c + pool_elems(POOL_C, desc[G - 1].n_int)) / 4;
  float4* b4 = reinterpret_cast<float4*>(charges);
  for (size_t k = t0; k < len4; k += nt) b4[k] = make_float4(0.f, 0.f, 0.f, 0.f);
}

hipError_t launch_bin(Problem& P, const float2* X, hipStream_t s) {
  const int n = P.n;
  const int tiles = (n + kBinTile - 1) / kBinTile;
  int bits = 1;
  while (((int64_t)1 << bits) < (int64_t)P.G * ((int64_t)P.cap * P.cap + 1)) ++bits;
  const int passes = (bits + kDigitBits - 1) / kDigitBits;
  // pass p reads (kin, vin) and writes the final pair on the last pass, else
  // alternates between (keys_tmp, perm_tmp) and (keys, perm_tmp2); keys is
  // free once pass 0 has read it.
  int* kin = P.keys;
  int* vin = nullptr;
  hipLaunchKernelGGL(k_bin_keys, dim3(tiles), dim3(256), 0, s, X, n, P.vgraph, P.G, P.desc, P.keys,
                     tiles, P.btotal, P.bin_hist);
  for (int p = 0; p < passes; ++p) {
    const int shift = kDigitBits * p;
    if (p > 0)
      hipLaunchKernelGGL(k_bin_hist, dim3(tiles), dim3(256), 0, s, kin, n, shift, tiles, P.btotal,
                         P.bin_hist);
    hipLaunchKernelGGL(k_bin_rowscan, dim3(kDigits / (256 / kWave)), dim3(256), 0, s, P.bin_hist, tiles,
                       shift, P.btotal, P.bin_rtot);
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
                       P.btotal, P.bin_hist, P.bin_rtot, kout, vout, X, last ? P.xs : nullptr);
    kin = kout;
    vin = vout;
  }
  int bb = (int)(((int64_t)P.G * ((int64_t)P.cap * P.cap + 1) + 1 + 255) / 256);
  if (bb > 4096) bb = 4096;
  if (bb < 1024) bb = 1024;  // enough threads for the grid clearing
  hipLaunchKernelGGL(k_box_bounds, dim3(bb), dim3(256), 0, s, P.skeys, n, P.btotal, P.box_off,
                     P.desc, P.G, P.charges);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
constexpr int kVals = 27;        // 9 nodes x 3 charges
constexpr int kRange = kSpreadRange;
constexpr int kRangeWaves = 4;   // waves per block of phase 1
constexpr int kLongSeg = 64;     // segments this long are summed by the whole wave
constexpr int kSpreadBatch = 4;  // points loaded together by one lane

// Charges of the 9 nodes of box (bx, by): out[c][node], c = 1, x, y.
template <typename T>
__device__ __forceinline__ void node_store(float* out, int ng, int bx, int by, const T* v) {
#pragma unroll
  for (int ty = 0; ty < 3; ++ty)
#pragma unroll
    for (int tx = 0; tx < 3; ++tx) {
      const size_t node = (size_t)(3 * by + ty) * ng + (3 * bx + tx);
      const int k = (ty * 3 + tx) * 3;
#pragma unroll
      for (int c = 0; c < 3; ++c) out[(size_t)c * ng * ng + node] = (float)v[k + c];
    }
}

// Graph of global box id `key` among graphs [lo, hi) (key lies in one of them).
__device__ __forceinline__ int graph_of_box(const GridDesc* __restrict__ desc, int lo, int hi,
                                            int key) {
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (desc[mid].box_base <= key) lo = mid; else hi = mid;
  }
  return lo;
}

struct BoxAt {
  int g, bx, by;
  bool far;  // the graph's far box: its points are not spread
  GridDesc d;
};

__device__ __forceinline__ BoxAt box_at(const GridDesc* __restrict__ desc, int glo, int ghi,
                                        int key) {
  BoxAt b;
  b.g = ghi - glo == 1 ? glo : graph_of_box(desc, glo, ghi, key);
  b.d = desc[b.g];
  const int local = key - b.d.box_base;
  b.far = local == b.d.n_int * b.d.n_int;
  b.by = local / b.d.n_int;
  b.bx = local - b.by * b.d.n_int;
  return b;
}

__device__ __forceinline__ bool is_far_key(const GridDesc* __restrict__ desc, int g, int key) {
  return key == far_key(desc[g]);
}

// Adds the 27 node contributions of point x of box (bx, by), times w0, to acc
// (w0 = 0 for the padding of a batch).
__device__ __forceinline__ void add_point(const BoxAt& b, float2 x, float w0, float (&acc)[kVals]) {
  const GridDesc& d = b.d;
  const float s = (x.x - d.x0) * d.inv_h - (float)b.bx;
  const float t = (x.y - d.y0) * d.inv_h - (float)b.by;
  float lx[3], ly[3];
  lagrange3(s, lx);
  lagrange3(t, ly);
  const float inv_half = 1.0f / d.half;
  const float q1 = (x.x - d.cx) * inv_half, q2 = (x.y - d.cy) * inv_half;
#pragma unroll
  for (int ty = 0; ty < 3; ++ty)
#pragma unroll
    for (int tx = 0; tx < 3; ++tx) {
      const float w = w0 * ly[ty] * lx[tx];
      const int k = (ty * 3 + tx) * 3;
      acc[k + 0] += w;
      acc[k + 1] += w * q1;
      acc[k + 2] += w * q2;
    }
}

// Sorted points [a, a + stride * m) of one box, m batches of kSpreadBatch
// points `stride` apart, every point below `end` counted once.
__device__ __forceinline__ void add_points(const float2* __restrict__ Xs, const BoxAt& b, int a,
                                           int end, int stride, float (&acc)[kVals]) {
  for (int p = a; p < end; p += kSpreadBatch * stride) {
    float2 x[kSpreadBatch];
#pragma unroll
    for (int k = 0; k < kSpreadBatch; ++k) x[k] = Xs[min(p + k * stride, end - 1)];
#pragma unroll
    for (int k = 0; k < kSpreadBatch; ++k)
      add_point(b, x[k], p + k * stride < end ? 1.f : 0.f, acc);
  }
}

// Where the sum of segment s = [a, b) of range r goes: a whole box to its
// nodes, the first segment of the range to the head partial, the last one to
// the tail partial (a segment that is not a whole box touches an end of the
// range).
__device__ __forceinline__ void emit(const int* __restrict__ box_off, const BoxAt& bx, int key,
                                     int a, int b, int s, int r, float* charges,
                                     float* head_val, float* tail_val, const float (&v)[kVals]) {
  if (box_off[key] == a && box_off[key + 1] == b) {
    node_store(charges + bx.d.off_c, bx.d.ng, bx.bx, bx.by, v);
  } else {
    float* dst = (s == 0 ? head_val : tail_val) + (size_t)r * kVals;
#pragma unroll
    for (int q = 0; q < kVals; ++q) dst[q] = v[q];
  }
}

// Phase 1: one wave per range of `range` sorted points (a power of two, 64 to
// kRange, chosen per problem). The range splits into
// segments of equal box id (start positions collected in LDS). A lane sums a
// short segment by itself; a long one is summed by the whole wave (lanes
// stride over its points, then a DPP reduction). Every sum runs in a fixed
// order, so the charges are reproducible bit for bit.
__global__ __launch_bounds__(kRangeWaves * kWave) void k_spread_ranges(
    const float2* __restrict__ Xs, const int* __restrict__ skeys, int n,
    const int* __restrict__ box_off, const GridDesc* __restrict__ desc, int G, float* charges,
    int* head_box, int* tail_box, float* head_val, float* tail_val, int range) {
  __shared__ int seg_all[kRangeWaves][kRange + 1];
  int* seg = seg_all[wave_id()];
  const int lane = lane_id();
  const u64 below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
  const int nranges = (n + range - 1) / range;
  const int nw = gridDim.x * kRangeWaves;
  for (int r = blockIdx.x * kRangeWaves + wave_id(); r < nranges; r += nw) {
    const int p0 = r * range;
    const int p1 = p0 + range < n ? p0 + range : n;
    // the range's keys, all loads in flight together; the key before a
    // point comes from the neighbouring lane
    constexpr int kSteps = kRange / kWave;
    int kv[kSteps];
#pragma unroll
    for (int j = 0; j < kSteps; ++j) kv[j] = skeys[min(p0 + j * kWave + lane, p1 - 1)];
    int nseg = 0;
#pragma unroll
    for (int j = 0; j < kSteps; ++j) {
      const int p = p0 + j * kWave + lane;  // steps past the range end find no start
      const int carry = j > 0 ? __builtin_amdgcn_readlane(kv[j > 0 ? j - 1 : 0], kWave - 1) : -1;
      const int prev = dpp_i<kDppWaveShr1, 0xF>(carry, kv[j]);
      const bool start = p < p1 && (p == p0 || kv[j] != prev);
      const u64 m = __ballot(start);
      if (start) seg[nseg + __popcll(m & below)] = p;
      nseg += __popcll(m);
    }
    if (lane == 0) seg[nseg] = p1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // the graphs of the range's first and last points: every box of the
    // range belongs to a graph between them (keys are ordered by graph)
    const int k0 = __builtin_amdgcn_readfirstlane(kv[0]);
    const int kl = skeys[p1 - 1];
    const int g0 = G == 1 ? 0 : graph_of_box(desc, 0, G, k0);
    const int g1 = G == 1 ? 0 : graph_of_box(desc, g0, G, kl);
    if (lane == 0) {  // which end pieces of the range are partials
      const bool whole0 = box_off[k0] == p0 && box_off[k0 + 1] == seg[1];
      const bool wholel = box_off[kl] == seg[nseg - 1] && box_off[kl + 1] == p1;
      head_box[r] = (whole0 || is_far_key(desc, g0, k0)) ? -1 : k0;
      tail_box[r] = (nseg > 1 && !wholel && !is_far_key(desc, g1, kl)) ? kl : -1;
    }
    for (int s0 = 0; s0 < nseg; s0 += kWave) {
      const int s = s0 + lane;
      const bool mine = s < nseg;
      const int a = mine ? seg[s] : 0, b = mine ? seg[s + 1] : 0;
      if (mine && b - a < kLongSeg) {
        const int key = skeys[a];
        const BoxAt bx = box_at(desc, g0, g1 + 1, key);
        if (!bx.far) {  // far points are not spread
          float acc[kVals];
#pragma unroll
          for (int q = 0; q < kVals; ++q) acc[q] = 0.f;
          add_points(Xs, bx, a, b, 1, acc);
          emit(box_off, bx, key, a, b, s, r, charges, head_val, tail_val, acc);
        }
      }
      u64 todo = __ballot(mine && b - a >= kLongSeg);
      while (todo) {
        const int src = __ffsll((long long)todo) - 1;
        todo &= todo - 1;
        const int la = __shfl(a, src, kWave), lb = __shfl(b, src, kWave);
        const int key = skeys[la];
        const BoxAt bx = box_at(desc, g0, g1 + 1, key);
        if (bx.far) continue;  // uniform over the wave: far points are not spread
        float acc[kVals];
#pragma unroll
        for (int q = 0; q < kVals; ++q) acc[q] = 0.f;
        if (la + lane < lb) add_points(Xs, bx, la + lane, lb, kWave, acc);
#pragma unroll
        for (int q = 0; q < kVals; ++q) acc[q] = wave_sum_to_last(acc[q]);
        if (lane == kWave - 1)
          emit(box_off, bx, key, la, lb, s0 + src, r, charges, head_val, tail_val, acc);
      }
    }
  }
}

// Phase 2: boxes whose points span several ranges add up the partials of
// those ranges in FP64, in range order. Empty boxes keep the zeros the
// binning wrote; boxes that phase 1 wrote whole are skipped. One lane per box;
// a box spanning kDenseRanges ranges or more is summed by a wave of its own.
constexpr int kDenseRanges = 4;

__device__ __forceinline__ const float* partial_of(int r, int b, const int* head_box,
                                                   const float* head_val, const float* tail_val) {
  return head_box[r] == b ? head_val + (size_t)r * kVals : tail_val + (size_t)r * kVals;
}

// The whole wave sums the partials of dense box b (lanes over its ranges, lane
// sums in FP64 in range order, joined by a DPP reduction in a fixed order).
__device__ __forceinline__ void spread_dense_box(int b, const int* __restrict__ box_off,
                                                 const GridDesc* __restrict__ desc, int G,
                                                 float* charges,
                                                 const int* __restrict__ head_box,
                                                 const float* __restrict__ head_val,
                                                 const float* __restrict__ tail_val, int range) {
  const int lane = lane_id();
  const int r0 = box_off[b] / range, r1 = (box_off[b + 1] - 1) / range;
  double acc[kVals];
#pragma unroll
  for (int q = 0; q < kVals; ++q) acc[q] = 0.0;
  for (int r = r0 + lane; r <= r1; r += kWave) {
    const float* src = partial_of(r, b, head_box, head_val, tail_val);
#pragma unroll
    for (int q = 0; q < kVals; ++q) acc[q] += (double)src[q];
  }
  float tot[kVals];
#pragma unroll
  for (int q = 0; q < kVals; ++q) tot[q] = wave_sum_to_last((float)acc[q]);
  if (lane == kWave - 1) {
    const BoxAt bx = box_at(desc, 0, G, b);
    node_store(charges + bx.d.off_c, bx.d.ng, bx.bx, bx.by, tot);
  }
}

__global__ __launch_bounds__(256) void k_spread_boxes(
    const int* __restrict__ box_off, const int* __restrict__ btotal,
    const GridDesc* __restrict__ desc, int G, float* charges,
    const int* __restrict__ head_box, const float* __restrict__ head_val,
    const float* __restrict__ tail_val, int range) {
  const int B = *btotal;
  const int lane = lane_id();
  const int nwaves = gridDim.x * (blockDim.x / kWave);
  for (int base = (blockIdx.x * (blockDim.x / kWave) + wave_id()) * kWave; base < B;
       base += nwaves * kWave) {
    const int b = base + lane;
    int r0 = 0, r1 = -1, bs = 0, be = 0;
    if (b < B) {
      bs = box_off[b];
      be = box_off[b + 1];
      if (be > bs) {
        r0 = bs / range;
        r1 = (be - 1) / range;
      }
    }
    // holds points, not written whole by phase 1, not a far box
    const bool mine =
        b < B && be > bs && r0 != r1 && !is_far_key(desc, graph_of_box(desc, 0, G, b), b);
    if (mine && r1 - r0 < kDenseRanges) {
      double acc[kVals];
#pragma unroll
      for (int q = 0; q < kVals; ++q) acc[q] = 0.0;
      for (int r = r0; r <= r1; ++r) {
        const float* src = partial_of(r, b, head_box, head_val, tail_val);
#pragma unroll
        for (int q = 0; q < kVals; ++q) acc[q] += (double)src[q];
      }
      const BoxAt bx = box_at(desc, 0, G, b);
      node_store(charges + bx.d.off_c, bx.d.ng, bx.bx, bx.by, acc);
    }
  }
  // dense boxes (clustered points) are dealt to waves round-robin, one wave
  // per box: lanes over its ranges, lane sums (FP64, range order) joined by a
  // DPP reduction in a fixed order
  const int gw = blockIdx.x * (blockDim.x / kWave) + wave_id();
  for (int base = gw; base < B; base += nwaves * kWave) {
    const int bl = base + lane * nwaves;  // lane l checks box base + l * nwaves
    bool dense = false;
    if (bl < B) {
      const int bs = box_off[bl], be = box_off[bl + 1];
      dense = be > bs && (be - 1) / range - bs / range >= kDenseRanges &&
              !is_far_key(desc, graph_of_box(desc, 0, G, bl), bl);
    }
    u64 todo = __ballot(dense);
    while (todo) {
      const int src_lane = __ffsll((long long)todo) - 1;
      todo &= todo - 1;
      const int b = base + src_lane * nwaves;
      spread_dense_box(b, box_off, desc, G, charges, head_box, head_val, tail_val, range);
    }
  }
}

hipError_t launch_spread(Problem& P, const float2* X, hipStream_t s) {
  (void)X;
  const int nranges = (P.n + P.spread_range - 1) / P.spread_range;
  int blocks = (nranges + kRangeWaves - 1) / kRangeWaves;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_spread_ranges, dim3(blocks), dim3(kRangeWaves * kWave), 0, s, P.xs, P.skeys,
                     P.n, P.box_off, P.desc, P.G, P.charges, P.head_box,
                     P.tail_box, P.head_val, P.tail_val, P.spread_range);
  int bblocks = (int)(((int64_t)P.G * ((int64_t)P.cap * P.cap + 1) + 255) / 256);
  if (bblocks > 8192) bblocks = 8192;
  hipLaunchKernelGGL(k_spread_boxes, dim3(bblocks), dim3(256), 0, s, P.box_off, P.btotal, P.desc,
                     P.G, P.charges, P.head_box, P.head_val, P.tail_val,
                     P.spread_range);
  return hipGetLastError();
}

}  // namespace tsnet
