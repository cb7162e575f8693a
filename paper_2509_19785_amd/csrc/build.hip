// C0 of Algorithm 3 on the GPU: the affinities P of a graph batch.
//
//  1. validate the CSR (bounds, order, no self loops, symmetry, graph ranges);
//  2. partial BFS per source (Sec. 3.1): expand levels until k other vertices
//     are visited, cutting the last level by the tie key; one wave per source,
//     the visited set in an LDS hash table, the last level kept as a bounded
//     sorted list of the r smallest (key, id) pairs;
//  3. per-row FP64 bisection of the bandwidth so that the perplexity of
//     p_{.|i} (Eq. 3) is u, over the row's hop-distance level histogram;
//  4. symmetrisation (Eq. 2): a stable LSD radix sort of the selected pairs by
//     target gives every row its reverse entries in source order; rows are
//     merged with their own sorted entries, duplicates summed, and divided by
//     twice the number of non-empty rows of the graph.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <vector>

#include "dev_util.h"
#include "scan.h"
#include "tsnet_internal.h"

namespace tsnet {

typedef unsigned long long u64;

// ---------------------------------------------------------------------------
// 1. CSR validation. Bits of the flag word:
enum { BAD_INDPTR = 1, BAD_COL = 2, BAD_SELF = 4, BAD_ORDER = 8, BAD_SYM = 16, BAD_GRAPH = 32 };

__global__ __launch_bounds__(256) void k_check_indptr(const int64_t* __restrict__ indptr, int n,
                                                      int64_t num_arcs, unsigned* flag) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int64_t a = indptr[i], b = indptr[i + 1];
    bool bad = a < 0 || b < a || b > num_arcs;
    if (i == 0 && a != 0) bad = true;
    if (i == n - 1 && b != num_arcs) bad = true;
    if (bad) atomicOr(flag, (unsigned)BAD_INDPTR);
  }
}

// Run only once the row pointers are known to be sane.
__global__ __launch_bounds__(256) void k_check_cols(const int64_t* __restrict__ indptr,
                                                    const int* __restrict__ idx, int n,
                                                    const int* __restrict__ goff, int G,
                                                    unsigned* flag) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int g = G == 1 ? 0 : graph_of(goff, G, i);
    const int lo = goff[g], hi = goff[g + 1];
    unsigned bad = 0;
    int prev = -1;
    for (int64_t e = indptr[i]; e < indptr[i + 1]; ++e) {
      const int j = idx[e];
      if (j < 0 || j >= n) {
        bad |= BAD_COL;
        break;
      }
      if (j < lo || j >= hi) bad |= BAD_GRAPH;
      if (j == i) bad |= BAD_SELF;
      if (j <= prev) bad |= BAD_ORDER;
      prev = j;
      // symmetry: i must appear in row j (rows are sorted, so binary search)
      int64_t a = indptr[j], b = indptr[j + 1];
      while (a < b) {
        const int64_t m = (a + b) >> 1;
        if (idx[m] < i) a = m + 1; else b = m;
      }
      if (a >= indptr[j + 1] || idx[a] != i) bad |= BAD_SYM;
    }
    if (bad) atomicOr(flag, bad);
  }
}

// ---------------------------------------------------------------------------
// 2. Partial BFS with bounded selection of the last level.

__device__ __forceinline__ u64 mix64(u64 z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Tie key of candidate j seen from source i (SplitMix64 output function).
__device__ __forceinline__ u64 tie_key(int i, int j, u64 seed, int mode) {
  if (mode == TSNET_TIE_ID) return (u64)(unsigned)j;
  return mix64(seed ^ mix64(((u64)(unsigned)i << 32) | (u64)(unsigned)j));
}

__device__ __forceinline__ bool pair_lt(u64 ka, int ia, u64 kb, int ib) {
  return ka < kb || (ka == kb && ia < ib);
}

constexpr int kPend = 128;          // pending candidates before a merge
constexpr u64 kKeyMax = ~0ull;
constexpr int kIdMax = 0x7fffffff;

template <int KC>
struct BfsLds {
  static constexpr int kTS = 2 * KC;  // hash table slots (power of two)
  int hash[kTS];
  int vlist[KC + 1];                  // visited vertices in BFS order
  int fstart[KC + 1];                 // row start of each frontier vertex
  int dpre[KC + 1];                   // exclusive prefix of frontier degrees
  u64 tkey[KC];                       // sorted best candidates of the level
  int tid[KC];
  u64 pkey[kPend];
  int pid[kPend];
  u64 mkey[KC + kPend];
  int mid[KC + kPend];
  int wsum[1];
};

template <int KC>
__device__ __forceinline__ int hslot(int j) {
  constexpr int bits = __builtin_ctz(BfsLds<KC>::kTS);
  return (int)(((unsigned)j * 2654435769u) >> (32 - bits));
}

template <int KC>
__device__ bool hcontains(const BfsLds<KC>& L, int j) {
  constexpr int mask = BfsLds<KC>::kTS - 1;
  int p = hslot<KC>(j);
  for (int probe = 0; probe < BfsLds<KC>::kTS; ++probe) {
    const int v = L.hash[p];
    if (v == j) return true;
    if (v == -1) return false;
    p = (p + 1) & mask;
  }
  return false;
}

template <int KC>
__device__ void hinsert(BfsLds<KC>& L, int j) {
  constexpr int mask = BfsLds<KC>::kTS - 1;
  int p = hslot<KC>(j);
  for (int probe = 0; probe < BfsLds<KC>::kTS; ++probe) {
    const int prev = atomicCAS(&L.hash[p], -1, j);
    if (prev == -1 || prev == j) return;
    p = (p + 1) & mask;
  }
}

// Merge the pending candidates into the sorted list T (size tcount), keeping
// the r smallest distinct pairs. Returns the new size. One wave (the block).
template <int KC>
__device__ int merge_pending(BfsLds<KC>& L, int tcount, int pcount, int r) {
  const int lane = threadIdx.x;
  int p2 = 1;
  while (p2 < pcount) p2 <<= 1;
  for (int q = pcount + lane; q < p2; q += kWave) {
    L.pkey[q] = kKeyMax;
    L.pid[q] = kIdMax;
  }
  __syncthreads();
  // bitonic sort of the pending list, ascending
  for (int s = 2; s <= p2; s <<= 1) {
    for (int st = s >> 1; st > 0; st >>= 1) {
      for (int q = lane; q < p2 / 2; q += kWave) {
        const int i = 2 * q - (q & (st - 1));
        const int l = i + st;
        const bool up = (i & s) == 0;
        const u64 ka = L.pkey[i], kb = L.pkey[l];
        const int ia = L.pid[i], ib = L.pid[l];
        const bool gt = pair_lt(kb, ib, ka, ia);
        if (gt == up) {
          L.pkey[i] = kb;
          L.pid[i] = ib;
          L.pkey[l] = ka;
          L.pid[l] = ia;
        }
      }
      __syncthreads();
    }
  }
  // merge path: T elements go before equal pending elements
  for (int a = lane; a < tcount; a += kWave) {
    const u64 k = L.tkey[a];
    const int id = L.tid[a];
    int lo = 0, hi = pcount;  // first pending element not less than T[a]
    while (lo < hi) {
      const int m = (lo + hi) >> 1;
      if (pair_lt(L.pkey[m], L.pid[m], k, id)) lo = m + 1; else hi = m;
    }
    L.mkey[a + lo] = k;
    L.mid[a + lo] = id;
  }
  for (int b = lane; b < pcount; b += kWave) {
    const u64 k = L.pkey[b];
    const int id = L.pid[b];
    int lo = 0, hi = tcount;  // T elements not greater than pending[b]
    while (lo < hi) {
      const int m = (lo + hi) >> 1;
      if (!pair_lt(k, id, L.tkey[m], L.tid[m])) lo = m + 1; else hi = m;
    }
    L.mkey[b + lo] = k;
    L.mid[b + lo] = id;
  }
  __syncthreads();
  // drop repeats (equal neighbours after the merge) and keep the first r
  const int total = tcount + pcount;
  int kept = 0;
  for (int base = 0; base < total; base += kWave) {
    const int m = base + lane;
    bool keep = false;
    u64 k = 0;
    int id = 0;
    if (m < total) {
      k = L.mkey[m];
      id = L.mid[m];
      keep = m == 0 || L.mkey[m - 1] != k || L.mid[m - 1] != id;
    }
    const u64 bal = __ballot(keep);
    const int pos = kept + __popcll(bal & ((1ull << lane) - 1ull));
    __syncthreads();  // every read of this chunk is done before T is rewritten
    if (keep && pos < r) {
      L.tkey[pos] = k;
      L.tid[pos] = id;
    }
    kept += __popcll(bal);
  }
  __syncthreads();
  return kept < r ? kept : r;
}

template <int KC>
__global__ __launch_bounds__(64) void k_bfs_select(const int64_t* __restrict__ indptr,
                                                   const int* __restrict__ idx, int n, int k,
                                                   u64 seed, int mode, int* out_len,
                                                   int* out_nbr, uint16_t* out_dist) {
  __shared__ BfsLds<KC> L;
  const int lane = threadIdx.x;
  for (int src = blockIdx.x; src < n; src += gridDim.x) {
    for (int q = lane; q < BfsLds<KC>::kTS; q += kWave) L.hash[q] = -1;
    __syncthreads();
    if (lane == 0) {
      L.vlist[0] = src;
      hinsert<KC>(L, src);
    }
    __syncthreads();
    int nsel = 0, vcount = 1, lb = 0, le = 1, d = 0;
    while (nsel < k) {
      ++d;
      const int r = k - nsel;
      const int F = le - lb;
      // degree prefix of the frontier
      int carry = 0;
      for (int base = 0; base < F; base += kWave) {
        const int t = base + lane;
        int deg = 0;
        if (t < F) {
          const int f = L.vlist[lb + t];
          const int64_t a = indptr[f];
          deg = (int)(indptr[f + 1] - a);
          L.fstart[t] = (int)a;
        }
        const int inc = wave_incl_scan(deg);
        if (t < F) L.dpre[t] = carry + inc - deg;
        carry += __shfl(inc, kWave - 1, kWave);
      }
      if (lane == 0) L.dpre[F] = carry;
      __syncthreads();
      const int E = carry;
      int tcount = 0, pcount = 0;
      u64 thr_k = kKeyMax;
      int thr_i = kIdMax;
      for (int e0 = 0; e0 < E; e0 += kWave) {
        const int e = e0 + lane;
        bool take = false;
        u64 key = 0;
        int j = 0;
        if (e < E) {
          int lo = 0, hi = F;  // last t with dpre[t] <= e
          while (hi - lo > 1) {
            const int m = (lo + hi) >> 1;
            if (L.dpre[m] <= e) lo = m; else hi = m;
          }
          j = idx[L.fstart[lo] + (e - L.dpre[lo])];
          if (!hcontains<KC>(L, j)) {
            key = tie_key(src, j, seed, mode);
            take = pair_lt(key, j, thr_k, thr_i);
          }
        }
        const u64 bal = __ballot(take);
        const int pos = pcount + __popcll(bal & ((1ull << lane) - 1ull));
        if (take) {
          L.pkey[pos] = key;
          L.pid[pos] = j;
        }
        pcount += __popcll(bal);
        __syncthreads();
        if (pcount > kPend - kWave || (e0 + kWave >= E && pcount > 0)) {
          tcount = merge_pending<KC>(L, tcount, pcount, r);
          pcount = 0;
          if (tcount == r) {
            thr_k = L.tkey[r - 1];
            thr_i = L.tid[r - 1];
          }
        }
      }
      if (tcount == 0) break;  // the component is exhausted
      int* on = out_nbr + (size_t)src * k + nsel;
      uint16_t* od = out_dist + (size_t)src * k + nsel;
      for (int t = lane; t < tcount; t += kWave) {
        on[t] = L.tid[t];
        od[t] = (uint16_t)(d < 65535 ? d : 65535);
      }
      nsel += tcount;
      if (tcount == r) break;  // the last level was cut (or filled exactly)
      // the whole level was taken: it joins the visited set and is the next frontier
      for (int t = lane; t < tcount; t += kWave) {
        L.vlist[vcount + t] = L.tid[t];
        hinsert<KC>(L, L.tid[t]);
      }
      __syncthreads();
      lb = vcount;
      vcount += tcount;
      le = vcount;
    }
    if (lane == 0) out_len[src] = nsel;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// 3. Perplexity calibration, one wave per row, FP64 (Eq. 3).
//    H(beta) = ln S + beta A / S over levels (d_l, c_l), delta_l = d_l^2 - d_1^2.

constexpr int kLvl = kMaxK;  // level slots per wave

struct PerpLds {
  int lv_start[4][kLvl + 1];
  int lv_d[4][kLvl];
};

__device__ __forceinline__ double entropy_at(double beta, const int* lvd, const int* lvs, int L,
                                             double& S_out) {
  const int lane = lane_id();
  const double d1 = (double)lvd[0];
  double s = 0.0, a = 0.0;
  for (int l = lane; l < L; l += kWave) {
    const double dl = (double)lvd[l];
    const double delta = dl * dl - d1 * d1;
    const double c = (double)(lvs[l + 1] - lvs[l]);
    const double e = exp(-beta * delta);
    s += c * e;
    a += c * delta * e;
  }
  s = wave_sum(s);
  a = wave_sum(a);
  S_out = s;
  return log(s) + beta * a / s;
}

__global__ __launch_bounds__(256) void k_perplexity(const int* __restrict__ len,
                                                    const uint16_t* __restrict__ dist, int n,
                                                    int k, double u, double* pcond, double* beta,
                                                    int8_t* rstatus, unsigned* status) {
  __shared__ PerpLds S;
  const int w = wave_id(), lane = lane_id();
  int* lvs = S.lv_start[w];
  int* lvd = S.lv_d[w];
  const double target = log(u);
  const int nwaves = blockDim.x / kWave;
  for (int i = blockIdx.x * nwaves + w; i < n; i += gridDim.x * nwaves) {
    const int K = len[i];
    const uint16_t* di = dist + (size_t)i * k;
    double* pi = pcond + (size_t)i * k;
    if (K == 0) {
      if (lane == 0) {
        beta[i] = 0.0;
        rstatus[i] = 3;
        atomicOr(status, (unsigned)TSNET_STATUS_ROW_EMPTY);
      }
      continue;
    }
    // level boundaries: positions where the (ascending) distance changes
    int L = 0;
    for (int base = 0; base < K; base += kWave) {
      const int t = base + lane;
      const bool start = t < K && (t == 0 || di[t] != di[t - 1]);
      const u64 bal = __ballot(start);
      const int pos = L + __popcll(bal & ((1ull << lane) - 1ull));
      if (start) {
        lvs[pos] = t;
        lvd[pos] = di[t];
      }
      L += __popcll(bal);
    }
    if (lane == 0) lvs[L] = K;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int c1 = lvs[1] - lvs[0];
    int st;
    double b;
    if (L == 1 || u >= (double)K) {
      st = 1;
      b = 0.0;
      for (int t = lane; t < K; t += kWave) pi[t] = 1.0 / (double)K;
    } else if (u <= (double)c1) {
      st = 2;
      b = INFINITY;
      const int d1 = lvd[0];
      for (int t = lane; t < K; t += kWave) pi[t] = di[t] == d1 ? 1.0 / (double)c1 : 0.0;
    } else {
      st = 0;
      double S;
      double hi = 1.0;
      for (int guard = 0; guard < 1100 && entropy_at(hi, lvd, lvs, L, S) >= target; ++guard) hi *= 2.0;
      double lo = 0.0;
      for (int step = 0; step < 200; ++step) {
        if (hi - lo <= 1e-14 * hi) break;
        const double mid = 0.5 * (lo + hi);
        if (entropy_at(mid, lvd, lvs, L, S) > target) lo = mid; else hi = mid;
      }
      b = 0.5 * (lo + hi);
      (void)entropy_at(b, lvd, lvs, L, S);
      const double d1 = (double)lvd[0];
      for (int t = lane; t < K; t += kWave) {
        const double dt = (double)di[t];
        pi[t] = exp(-b * (dt * dt - d1 * d1)) / S;
      }
    }
    if (lane == 0) {
      beta[i] = b;
      rstatus[i] = (int8_t)st;
      if (st == 1) atomicOr(status, (unsigned)TSNET_STATUS_ROW_LOW);
      if (st == 2) atomicOr(status, (unsigned)TSNET_STATUS_ROW_HIGH);
    }
  }
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of (key, value) pairs, 8-bit digits.

__global__ __launch_bounds__(256) void k_radix_hist(const unsigned* __restrict__ keys, int N,
                                                    int shift, int tiles, int* hist) {
  __shared__ int cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int base = blockIdx.x * kRadixTile;
  for (int q = threadIdx.x; q < kRadixTile; q += 256) {
    const int i = base + q;
    if (i < N) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1);
  }
  __syncthreads();
  hist[threadIdx.x * tiles + blockIdx.x] = cnt[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_radix_scatter(const unsigned* __restrict__ kin,
                                                       const unsigned* __restrict__ vin, int N,
                                                       int shift, int tiles,
                                                       const int* __restrict__ offs,
                                                       unsigned* kout, unsigned* vout) {
  __shared__ int run[256];
  __shared__ int wc[4][256];
  const int tid = threadIdx.x, w = wave_id(), lane = lane_id();
  run[tid] = offs[tid * tiles + blockIdx.x];
  for (int q = 0; q < 4; ++q) wc[q][tid] = 0;
  __syncthreads();
  const u64 lt = (1ull << lane) - 1ull;
  const int base = blockIdx.x * kRadixTile;
  for (int round = 0; round < kRadixTile / 256; ++round) {
    const int i = base + round * 256 + tid;
    const bool valid = i < N;
    unsigned key = 0, val = 0;
    int dg = 256;  // invalid lanes use a digit of their own
    if (valid) {
      key = kin[i];
      val = vin[i];
      dg = (int)((key >> shift) & 255u);
    }
    // lanes match on validity first, then on each digit bit
    const u64 vb = __ballot(valid);
    u64 peers = valid ? vb : ~vb;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
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
    }
    __syncthreads();
    run[tid] += wc[0][tid] + wc[1][tid] + wc[2][tid] + wc[3][tid];
    for (int q = 0; q < 4; ++q) wc[q][tid] = 0;
    __syncthreads();
  }
}

// Sorts (keys, vals) by the low `bits` bits of the key; the result ends in
// (keys, vals) (ping-pong through kt, vt). Buffers of N entries; hist of 256 * tiles.
hipError_t radix_sort(unsigned* keys, unsigned* vals, unsigned* kt, unsigned* vt, int N, int bits,
                      int* hist, int* tsum, hipStream_t s) {
  const int tiles = (N + kRadixTile - 1) / kRadixTile;
  if (tiles == 0) return hipSuccess;
  unsigned *ka = keys, *va = vals, *kb = kt, *vb = vt;
  int passes = (bits + 7) / 8;
  if (passes % 2) ++passes;  // an even count leaves the result in (keys, vals)
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p;
    hipLaunchKernelGGL(k_radix_hist, dim3(tiles), dim3(256), 0, s, ka, N, shift, tiles, hist);
    hipError_t e = exclusive_scan<int>(hist, (int64_t)256 * tiles, hist, tsum, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_radix_scatter, dim3(tiles), dim3(256), 0, s, ka, va, N, shift, tiles, hist,
                       kb, vb);
    unsigned* t = ka;
    ka = kb;
    kb = t;
    t = va;
    va = vb;
    vb = t;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 4. Symmetrisation.

// Keys (target id, or n for unused slots) and values (slot index e = i*k + t).
__global__ __launch_bounds__(256) void k_pairs(const int* __restrict__ len,
                                               const int* __restrict__ nbr, int n, int k,
                                               unsigned* keys, unsigned* vals) {
  const int64_t N = (int64_t)n * k;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < N;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / k), t = (int)(e - (int64_t)i * k);
    keys[e] = t < len[i] ? (unsigned)nbr[e] : (unsigned)n;
    vals[e] = (unsigned)e;
  }
}

// trans_off[j] = first sorted slot with key >= j, for j in [0, n].
__global__ __launch_bounds__(256) void k_bounds(const unsigned* __restrict__ keys, int N, int n,
                                                int* off) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p <= N; p += gridDim.x * blockDim.x) {
    const int cur = p < N ? (int)keys[p] : n + 1;
    const int prev = p == 0 ? -1 : (int)keys[p - 1];
    for (int j = prev + 1; j <= cur && j <= n; ++j) off[j] = p;
  }
}

// Own entries of each row sorted by column (bitonic, one wave per row).
template <int KC>
__global__ __launch_bounds__(64) void k_sort_own(const int* __restrict__ len,
                                                 const int* __restrict__ nbr,
                                                 const double* __restrict__ pcond, int n, int k,
                                                 int* ocol, double* oval) {
  __shared__ int c[KC];
  __shared__ double v[KC];
  const int lane = threadIdx.x;
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const int K = len[i];
    int p2 = 1;
    while (p2 < K) p2 <<= 1;
    for (int t = lane; t < p2; t += kWave) {
      c[t] = t < K ? nbr[(size_t)i * k + t] : kIdMax;
      v[t] = t < K ? pcond[(size_t)i * k + t] : 0.0;
    }
    __syncthreads();
    for (int s2 = 2; s2 <= p2; s2 <<= 1) {
      for (int st = s2 >> 1; st > 0; st >>= 1) {
        for (int q = lane; q < p2 / 2; q += kWave) {
          const int a = 2 * q - (q & (st - 1));
          const int b = a + st;
          const bool up = (a & s2) == 0;
          if ((c[a] > c[b]) == up) {
            const int tc = c[a];
            c[a] = c[b];
            c[b] = tc;
            const double tv = v[a];
            v[a] = v[b];
            v[b] = tv;
          }
        }
        __syncthreads();
      }
    }
    for (int t = lane; t < K; t += kWave) {
      ocol[(size_t)i * k + t] = c[t];
      oval[(size_t)i * k + t] = v[t];
    }
    __syncthreads();
  }
}

// Source of reverse entry q of any row: the slot index divided by k.
__device__ __forceinline__ int rsrc(const unsigned* sv, int64_t q, int k) { return (int)(sv[q] / (unsigned)k); }

// Per row: mark own entries that also appear reversed; merged row length.
__global__ __launch_bounds__(256) void k_sym_count(const int* __restrict__ len,
                                                   const int* __restrict__ ocol, int n, int k,
                                                   const int* __restrict__ toff,
                                                   const unsigned* __restrict__ sv,
                                                   unsigned char* dup, int64_t* rowlen) {
  const int lane = lane_id();
  const int nwaves = blockDim.x / kWave;
  for (int i = blockIdx.x * nwaves + wave_id(); i < n; i += gridDim.x * nwaves) {
    const int K = len[i];
    const int64_t ta = toff[i], tb = toff[i + 1];
    int nd = 0;
    for (int t = lane; t < K; t += kWave) {
      const int cc = ocol[(size_t)i * k + t];
      int64_t a = ta, b = tb;
      while (a < b) {
        const int64_t m = (a + b) >> 1;
        if (rsrc(sv, m, k) < cc) a = m + 1; else b = m;
      }
      const bool d = a < tb && rsrc(sv, a, k) == cc;
      dup[(size_t)i * k + t] = d ? 1 : 0;
      nd += d ? 1 : 0;
    }
    nd = wave_sum(nd);
    if (lane == 0) rowlen[i] = (int64_t)K + (tb - ta) - nd;
  }
}

// Per row: write the merged, column-sorted entries with Eq. (2) values.
__global__ __launch_bounds__(256) void k_sym_fill(
    const int* __restrict__ len, const int* __restrict__ ocol, const double* __restrict__ oval,
    const unsigned char* __restrict__ dup, int n, int k, const int* __restrict__ toff,
    const unsigned* __restrict__ sv, const double* __restrict__ pcond,
    const int64_t* __restrict__ rowptr, const int* __restrict__ goff, int G,
    const double* __restrict__ denom, int* col, float* val) {
  __shared__ int dpre_s[4][kMaxK + 1];
  const int lane = lane_id(), w = wave_id();
  int* dpre = dpre_s[w];
  const int nwaves = blockDim.x / kWave;
  for (int i = blockIdx.x * nwaves + w; i < n; i += gridDim.x * nwaves) {
    const int K = len[i];
    const int64_t ta = toff[i], tb = toff[i + 1];
    const int64_t out0 = rowptr[i];
    const double inv = 1.0 / denom[G == 1 ? 0 : graph_of(goff, G, i)];
    // prefix count of duplicated own entries
    int carry = 0;
    for (int base = 0; base < K; base += kWave) {
      const int t = base + lane;
      const int dv = t < K ? (int)dup[(size_t)i * k + t] : 0;
      const int inc = wave_incl_scan(dv);
      if (t < K) dpre[t] = carry + inc - dv;
      carry += __shfl(inc, kWave - 1, kWave);
    }
    if (lane == 0) dpre[K] = carry;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // own entries
    for (int a = lane; a < K; a += kWave) {
      const int cc = ocol[(size_t)i * k + a];
      int64_t lo = ta, hi = tb;
      while (lo < hi) {
        const int64_t m = (lo + hi) >> 1;
        if (rsrc(sv, m, k) < cc) lo = m + 1; else hi = m;
      }
      double v = oval[(size_t)i * k + a];
      if (dup[(size_t)i * k + a]) v += pcond[sv[lo]];
      const int64_t pos = out0 + a + (lo - ta) - dpre[a];
      col[pos] = cc;
      val[pos] = (float)(v * inv);
    }
    // reverse-only entries
    for (int64_t q = ta + lane; q < tb; q += kWave) {
      const int s = rsrc(sv, q, k);
      int lo = 0, hi = K;  // own entries with column < s
      while (lo < hi) {
        const int m = (lo + hi) >> 1;
        if (ocol[(size_t)i * k + m] < s) lo = m + 1; else hi = m;
      }
      if (lo < K && ocol[(size_t)i * k + lo] == s) continue;  // merged into the own entry
      const int64_t pos = out0 + lo + (q - ta) - dpre[lo];
      col[pos] = s;
      val[pos] = (float)(pcond[sv[q]] * inv);
    }
  }
}

// Non-empty rows per graph -> denominators 2 n'_g.
__global__ __launch_bounds__(256) void k_denoms(const int* __restrict__ len,
                                                const int* __restrict__ goff, int G,
                                                double* denom) {
  const int g = blockIdx.x;
  int c = 0;
  for (int i = goff[g] + threadIdx.x; i < goff[g + 1]; i += blockDim.x) c += len[i] > 0 ? 1 : 0;
  c = wave_sum(c);
  __shared__ int sh[4];
  if (lane_id() == 0) sh[wave_id()] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int ne = sh[0] + sh[1] + sh[2] + sh[3];
    denom[g] = 2.0 * (double)(ne > 0 ? ne : 1);
  }
}

// ---------------------------------------------------------------------------
template <typename T>
static int tmalloc(T** p, size_t count) {
  if (count == 0) count = 1;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(e == hipErrorOutOfMemory ? TSNET_ENOMEM : TSNET_EHIP,
                std::string("hipMalloc in tsnet_build_P: ") + hipGetErrorString(e));
  }
  return TSNET_OK;
}

struct Scratch {
  std::vector<void*> ptrs;
  template <typename T>
  int get(T** p, size_t count) {
    int rc = tmalloc(p, count);
    if (!rc) ptrs.push_back(*p);
    return rc;
  }
  ~Scratch() {
    for (void* p : ptrs) (void)hipFree(p);
  }
};

#define BUILD_CHECK(expr)                                                            \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(TSNET_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
  } while (0)

template <int KC>
static void launch_bfs(Problem& P, const int64_t* indptr, const int* indices, uint64_t seed,
                       int mode, hipStream_t s) {
  const int blocks = P.n < 65536 ? P.n : 65536;
  hipLaunchKernelGGL(k_bfs_select<KC>, dim3(blocks), dim3(64), 0, s, indptr, indices, P.n, P.k,
                     (u64)seed, mode, P.cond_len, P.cond_nbr, P.cond_dist);
}

template <int KC>
static void launch_sort_own(Problem& P, const double* pcond, int* ocol, double* oval,
                            hipStream_t s) {
  const int blocks = P.n < 65536 ? P.n : 65536;
  hipLaunchKernelGGL(k_sort_own<KC>, dim3(blocks), dim3(64), 0, s, P.cond_len, P.cond_nbr, pcond,
                     P.n, P.k, ocol, oval);
}

int validate_csr(const int64_t* indptr, const int* indices, int n, int64_t num_arcs,
                 const int* goff_d, int G, hipStream_t s) {
  Scratch S;
  unsigned* flag = nullptr;
  int rc;
  if ((rc = S.get(&flag, 1))) return rc;
  BUILD_CHECK(hipMemsetAsync(flag, 0, sizeof(unsigned), s));
  const int vb = n / 256 + 1 < 8192 ? n / 256 + 1 : 8192;
  hipLaunchKernelGGL(k_check_indptr, dim3(vb), dim3(256), 0, s, indptr, n, num_arcs, flag);
  unsigned hflag = 0;
  BUILD_CHECK(hipMemcpyAsync(&hflag, flag, sizeof(unsigned), hipMemcpyDeviceToHost, s));
  BUILD_CHECK(hipStreamSynchronize(s));
  if (hflag) return fail(TSNET_EINVAL, "invalid CSR row pointers");
  if (num_arcs > 0) {
    hipLaunchKernelGGL(k_check_cols, dim3(vb), dim3(256), 0, s, indptr, indices, n, goff_d, G,
                       flag);
    BUILD_CHECK(hipMemcpyAsync(&hflag, flag, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    BUILD_CHECK(hipStreamSynchronize(s));
    if (hflag) {
      std::string why;
      if (hflag & BAD_COL) why += " column out of range;";
      if (hflag & BAD_GRAPH) why += " edge between graphs;";
      if (hflag & BAD_SELF) why += " self loop;";
      if (hflag & BAD_ORDER) why += " row not strictly ascending;";
      if (hflag & BAD_SYM) why += " not symmetric;";
      return fail(TSNET_EINVAL, "invalid CSR:" + why);
    }
  }
  return TSNET_OK;
}

int build_affinities(Problem& P, const int64_t* indptr, const int* indices, int64_t num_arcs,
                     double perplexity, uint64_t seed, int tie_mode, hipStream_t s) {
  const int n = P.n, k = P.k;
  const int64_t nk = (int64_t)n * k;
  Scratch S;
  int rc;
  if ((rc = validate_csr(indptr, indices, n, num_arcs, P.goff_d, P.G, s))) return rc;
  // persistent outputs
  if ((rc = tmalloc(&P.cond_len, n)) || (rc = tmalloc(&P.cond_nbr, nk)) ||
      (rc = tmalloc(&P.cond_dist, nk)) || (rc = tmalloc(&P.beta, n)) ||
      (rc = tmalloc(&P.rstatus, n)))
    return rc;
  // partial BFS
  if (k <= 128) launch_bfs<128>(P, indptr, indices, seed, tie_mode, s);
  else if (k <= 256) launch_bfs<256>(P, indptr, indices, seed, tie_mode, s);
  else if (k <= 512) launch_bfs<512>(P, indptr, indices, seed, tie_mode, s);
  else launch_bfs<1024>(P, indptr, indices, seed, tie_mode, s);
  BUILD_CHECK(hipGetLastError());
  // calibration
  double* pcond = nullptr;
  if ((rc = S.get(&pcond, nk))) return rc;
  {
    int blocks = (n + 3) / 4;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_perplexity, dim3(blocks), dim3(256), 0, s, P.cond_len, P.cond_dist, n, k,
                       perplexity, pcond, P.beta, P.rstatus, P.ctx->status);
    BUILD_CHECK(hipGetLastError());
  }
  // reverse lists: stable sort of all slots by target
  unsigned *keys, *vals, *kt, *vt;
  int *hist, *tsum, *toff;
  const int N = (int)nk;
  const int rtiles = (N + kRadixTile - 1) / kRadixTile;
  const int64_t hist_len = (int64_t)256 * rtiles;
  const int64_t tsum_len = (hist_len + kTileScan - 1) / kTileScan + (nk + kTileScan) / kTileScan + 8;
  if ((rc = S.get(&keys, nk)) || (rc = S.get(&vals, nk)) || (rc = S.get(&kt, nk)) ||
      (rc = S.get(&vt, nk)) || (rc = S.get(&hist, hist_len + 1)) || (rc = S.get(&tsum, tsum_len)) ||
      (rc = S.get(&toff, (size_t)n + 1)))
    return rc;
  {
    int blocks = (int)((nk + 255) / 256);
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_pairs, dim3(blocks), dim3(256), 0, s, P.cond_len, P.cond_nbr, n, k, keys,
                       vals);
    int bits = 1;
    while (((int64_t)1 << bits) <= n) ++bits;
    BUILD_CHECK(radix_sort(keys, vals, kt, vt, N, bits, hist, tsum, s));
    int bb = (N + 1 + 255) / 256;
    if (bb > 65536) bb = 65536;
    hipLaunchKernelGGL(k_bounds, dim3(bb), dim3(256), 0, s, keys, N, n, toff);
    BUILD_CHECK(hipGetLastError());
  }
  // own rows sorted by column
  int* ocol;
  double* oval;
  unsigned char* dup;
  int64_t *rowlen, *tsum64;
  double* denom;
  if ((rc = S.get(&ocol, nk)) || (rc = S.get(&oval, nk)) || (rc = S.get(&dup, nk)) ||
      (rc = S.get(&rowlen, (size_t)n + 1)) || (rc = S.get(&tsum64, (size_t)n / kTileScan + 8)) ||
      (rc = S.get(&denom, P.G)))
    return rc;
  if (k <= 128) launch_sort_own<128>(P, pcond, ocol, oval, s);
  else if (k <= 256) launch_sort_own<256>(P, pcond, ocol, oval, s);
  else if (k <= 512) launch_sort_own<512>(P, pcond, ocol, oval, s);
  else launch_sort_own<1024>(P, pcond, ocol, oval, s);
  BUILD_CHECK(hipGetLastError());
  int wb = (n + 3) / 4;
  if (wb > 16384) wb = 16384;
  hipLaunchKernelGGL(k_sym_count, dim3(wb), dim3(256), 0, s, P.cond_len, ocol, n, k, toff, vals,
                     dup, rowlen);
  if ((rc = tmalloc(&P.rowptr, (size_t)n + 1))) return rc;
  BUILD_CHECK(exclusive_scan<int64_t>(rowlen, n, P.rowptr, tsum64, s));
  int64_t nnz = 0;
  BUILD_CHECK(hipMemcpyAsync(&nnz, P.rowptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  BUILD_CHECK(hipStreamSynchronize(s));
  if (nnz < 0 || nnz >= ((int64_t)1 << 32)) return fail(TSNET_EINVAL, "P has too many nonzeros");
  P.nnz = nnz;
  if ((rc = tmalloc(&P.col, (size_t)nnz)) || (rc = tmalloc(&P.val, (size_t)nnz))) return rc;
  hipLaunchKernelGGL(k_denoms, dim3(P.G), dim3(256), 0, s, P.cond_len, P.goff_d, P.G, denom);
  hipLaunchKernelGGL(k_sym_fill, dim3(wb), dim3(256), 0, s, P.cond_len, ocol, oval, dup, n, k, toff,
                     vals, pcond, P.rowptr, P.goff_d, P.G, denom, P.col, P.val);
  BUILD_CHECK(hipGetLastError());
  BUILD_CHECK(hipStreamSynchronize(s));
  return TSNET_OK;
}

}  // namespace tsnet
