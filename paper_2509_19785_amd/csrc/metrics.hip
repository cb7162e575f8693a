// Layout quality metrics of Sec. 4.3: neighbourhood preservation with r = 2
// (Sec. 4.3.1) and stress (Sec. 4.3.2). The paper states the two formulas;
// the readings are the project's:
//
// Neighbourhood preservation of vertex v: N_G(v) = the vertices 1 or 2 hops
// from v (v excluded), k = |N_G(v)|; N_D(v) = the k vertices of v's graph
// nearest to v in the layout (v excluded), ranked by the FP32 squared
// distance dx*dx + dy*dy (every operation rounded on its own, no fused
// multiply-add), equal distances by increasing id. hits = |N_G & N_D|; the
// Jaccard ratio of the two sets is hits / (2k - hits). NP of a graph is its
// mean over the evaluated vertices with k > 0.
//
//  * N_G(v) is marked in a bitmap of the graph's vertices that the worker
//    (a wave, or a block for vertices with many 2-hop walks) owns; walking
//    the 2-hop paths a second time clears it again and counts the hits.
//  * N_D(v): the points are counting-sorted into a grid whose cell
//    boundaries are quantiles of each coordinate (about sqrt(n_g) cells per
//    axis, so cells follow the density of clustered layouts), with a
//    summed-area table of the cell counts. Cell membership is decided by
//    exact comparisons with the boundaries, so any boundaries give the same
//    result. The smallest square of cells around v's cell holding k others
//    bounds the k-th distance: a first radix select over that square finds
//    the k-th key there (key = squared-distance bits, id), whose distance
//    bounds the k-th nearest of the whole graph. Every point that can be
//    nearer lies in the cells meeting the disc of that radius (widened for
//    the FP32 rounding of the keys); a second radix select over those cells
//    gives the k-th smallest key, and a vertex is among the k nearest iff its
//    key is not above it.
//
// Stress over the ordered pairs (s, j), s a source, j != s reachable from s:
// d = hop distance, e = Euclidean distance in FP64 from the FP32 coordinates,
// per graph the pair count and the sums of (1 - e/d)^2, e/d and (e/d)^2.
// The distances come from a bit-parallel BFS of up to 64 sources at a time:
// each vertex holds the set of sources that have reached it, one level ORs
// in its neighbours' sets, and a source bit that appears at level L gives the
// pair its distance L. Each vertex adds its pairs into FP64 sums of its own
// in a fixed order, so the results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <string>
#include <vector>

#include "dev_util.h"
#include "scan.h"
#include "tsnet_internal.h"

namespace tsnet {

namespace {

typedef unsigned long long u64;
constexpr int kNpMaxGrid = 2048;       // cells per axis at most
constexpr int kNpHeavyWalks = 4096;    // 2-hop walks above which a vertex gets a whole block
constexpr int kNpLightWaves = 4;       // waves (one vertex each) per block of the light kernel
constexpr int kNpHeavyThreads = 1024;  // threads per vertex of the heavy kernel
constexpr int kStressSources = 64;     // sources per bit-parallel BFS
// The select over the square keeps going until the top 24 key bits (the
// squared distance to 15 mantissa bits) are fixed, so the radius it gives is
// within 2e-5 of the k-th distance in the square.
constexpr int kSquareExitShift = 40;

enum { NP_ERR_COORD = 1, NP_ERR_VERTEX = 2, NP_ERR_ORDER = 4, NP_ERR_SELECT = 8 };

// Squared layout distance in FP32 with one rounding per operation.
__device__ __forceinline__ float np_d2(float xw, float yw, float xv, float yv) {
#pragma clang fp contract(off)
  const float dx = xw - xv;
  const float dy = yw - yv;
  return dx * dx + dy * dy;
}

__device__ __forceinline__ u64 np_key(float d2, int w) {
  return ((u64)__float_as_uint(d2) << 32) | (u64)(unsigned)w;
}

struct NpDev {
  const int64_t* indptr;
  const int* indices;
  const float2* X;
  int n, G;
  const int* goff;      // [G+1]
  const int* gcell;     // [G] cells per axis
  const int* cbase;     // [G+1] first cell of each graph
  const int* sbase;     // [G] first summed-area entry of each graph
  const int* colbase;   // [G+1] first boundary (and summed-area column) of each graph
  float* bx;            // cell boundaries along x: G_g + 1 per graph, from colbase[g]
  float* by;            // the same along y
  int* cell_of;         // [n]
  int* cnt;             // [cells + 1] counts, then the fill cursors
  int* cstart;          // [cells + 1] first sorted point of each cell
  int* sat;             // summed-area tables, (G_g + 1)^2 per graph
  float4* sorted;       // [n] (x, y, id bits, 0) in cell order
  unsigned* skey;       // [n] sort keys (coordinate order, then graph)
  unsigned* sval;       // [n] vertex of each sorted key
  const int* verts;     // evaluated vertices (strictly increasing) or NULL for all
  int nv;               // number of evaluated vertices
  unsigned* bits;       // per-worker bitmaps of `words` words
  int words;
  int* ball;            // [nv]
  int* hits;            // [nv]
  int* err;             // [1] NP_ERR_* bits
};

__device__ __forceinline__ int np_graph(const NpDev& a, int v) {
  return a.G == 1 ? 0 : graph_of(a.goff, a.G, v);
}

// Cell along one axis: the largest c in [0, G_g - 1] with b[c] <= x, or 0.
__device__ __forceinline__ int qcell(const float* b, int Gg, double x) {
  int l = 1, h = Gg;  // the first index in [1, G_g) with b > x, else G_g
  while (l < h) {
    const int m = (l + h) >> 1;
    if ((double)b[m] > x) h = m; else l = m + 1;
  }
  return l - 1;
}

__global__ void k_fill_u32(unsigned* p, size_t count, unsigned v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ __launch_bounds__(256) void k_np_check(NpDev a) {
  bool bad = false;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += gridDim.x * blockDim.x) {
    const float2 p = a.X[v];
    if (!isfinite(p.x) || !isfinite(p.y)) bad = true;
  }
  if (bad) atomicOr(a.err, NP_ERR_COORD);
}

// Sort keys of one axis: the float bits mapped so that unsigned order is the
// order of the values.
__global__ __launch_bounds__(256) void k_np_axis_keys(NpDev a, int axis) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += gridDim.x * blockDim.x) {
    const float2 p = a.X[v];
    const unsigned u = __float_as_uint(axis ? p.y : p.x);
    a.skey[v] = u ^ ((u >> 31) ? 0xFFFFFFFFu : 0x80000000u);
    a.sval[v] = (unsigned)v;
  }
}

// After the sort by coordinate: the graph of each entry, for a stable sort by graph.
__global__ __launch_bounds__(256) void k_np_graph_keys(NpDev a) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += gridDim.x * blockDim.x)
    a.skey[i] = (unsigned)graph_of(a.goff, a.G, (int)a.sval[i]);
}

// Boundaries of graph g along one axis: b[c] = the coordinate of rank
// c n_g / G_g in the graph (b[0] its smallest, b[G_g] its largest).
__global__ __launch_bounds__(256) void k_np_bounds(NpDev a, int axis, int total) {
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < total; c += gridDim.x * blockDim.x) {
    const int g = graph_of(a.colbase, a.G, c);
    const int j = c - a.colbase[g], Gg = a.gcell[g];
    const int lo = a.goff[g], ng = a.goff[g + 1] - lo;
    const int pos = j == Gg ? lo + ng - 1 : lo + (int)((int64_t)j * ng / Gg);
    const float2 p = a.X[a.sval[pos]];
    (axis ? a.by : a.bx)[c] = axis ? p.y : p.x;
  }
}

__global__ __launch_bounds__(256) void k_np_cells(NpDev a) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += gridDim.x * blockDim.x) {
    const int g = np_graph(a, v);
    const int Gg = a.gcell[g], cb = a.colbase[g];
    const float2 x = a.X[v];
    const int cx = qcell(a.bx + cb, Gg, x.x), cy = qcell(a.by + cb, Gg, x.y);
    const int cell = a.cbase[g] + cy * Gg + cx;
    a.cell_of[v] = cell;
    atomicAdd(&a.cnt[cell], 1);
  }
}

__global__ __launch_bounds__(256) void k_np_scatter(NpDev a) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += gridDim.x * blockDim.x) {
    const int cell = a.cell_of[v];
    const int pos = a.cstart[cell] + atomicAdd(&a.cnt[cell], 1);
    const float2 x = a.X[v];
    a.sorted[pos] = make_float4(x.x, x.y, __int_as_float(v), 0.f);
  }
}

// Summed-area table of graph g: S[y][x] = points in cells [0, x) x [0, y),
// one thread per column x in [0, G_g], running down the rows. Row y's count
// of cells [0, x) is a difference of the cell starts.
__global__ __launch_bounds__(256) void k_np_sat(NpDev a, int total_cols) {
  constexpr int kB = 8;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < total_cols; c += gridDim.x * blockDim.x) {
    const int g = graph_of(a.colbase, a.G, c);
    const int x = c - a.colbase[g];
    const int Gg = a.gcell[g], cb = a.cbase[g];
    int* S = a.sat + a.sbase[g];
    int acc = 0;
    S[x] = 0;
    for (int y0 = 0; y0 < Gg; y0 += kB) {
      int d[kB];
#pragma unroll
      for (int q = 0; q < kB; ++q) {
        const int y = y0 + q;
        d[q] = y < Gg ? a.cstart[cb + y * Gg + x] - a.cstart[cb + y * Gg] : 0;
      }
#pragma unroll
      for (int q = 0; q < kB; ++q) {
        const int y = y0 + q;
        if (y < Gg) {
          acc += d[q];
          S[(size_t)(y + 1) * (Gg + 1) + x] = acc;
        }
      }
    }
  }
}

// Checks the evaluated list and sorts its entries into light and heavy work
// by the number of 2-hop walks deg(v) + sum over neighbours of their degree.
__global__ __launch_bounds__(256) void k_np_classify(NpDev a, int* light, int* heavy, int* counts) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < a.nv; i += gridDim.x * blockDim.x) {
    const int v = a.verts ? a.verts[i] : i;
    if (v < 0 || v >= a.n) {
      atomicOr(a.err, NP_ERR_VERTEX);
      continue;
    }
    if (a.verts && i + 1 < a.nv && a.verts[i + 1] <= v) atomicOr(a.err, NP_ERR_ORDER);
    const int64_t e0 = a.indptr[v], e1 = a.indptr[v + 1];
    int64_t walks = e1 - e0;
    for (int64_t e = e0; e < e1; ++e) {
      const int u = a.indices[e];
      walks += a.indptr[u + 1] - a.indptr[u];
    }
    if (walks > kNpHeavyWalks)
      heavy[atomicAdd(&counts[1], 1)] = i;
    else
      light[atomicAdd(&counts[0], 1)] = i;
  }
}

// ---- group primitives: a group is one wave (T = 64) or one block (T = 1024)
//
// Every value that steers a loop or a branch of the per-vertex work (the
// vertex index, k, the square radius, the segment totals, the selected
// bucket) is the same in all lanes by construction, and is passed through
// readfirstlane so that the compiler sees it as uniform too. Otherwise it may
// split the work loop per lane (lane 0 alone takes the path with the stores
// and the atomic that fetches the next vertex) and leave the other lanes in a
// loop that reads the next index from an inactive lane 0.
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

template <int T>
struct Grp;

template <>
struct Grp<kWave> {
  static __device__ __forceinline__ int tid() { return lane_id(); }
  static __device__ __forceinline__ void sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  static __device__ __forceinline__ int sum(int v, int*) { return uni(wave_sum(v)); }
  static __device__ __forceinline__ int bcast0(int v, int*) { return uni(v); }
  static __device__ __forceinline__ int excl_scan(int v, int*, int* total) {
    const int inc = wave_incl_scan(v);
    *total = uni(__shfl(inc, kWave - 1, kWave));
    return inc - v;
  }
  static __device__ __forceinline__ u64 max64(u64 v, int*) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
      const unsigned hi = __shfl_xor((unsigned)(v >> 32), o, kWave);
      const unsigned lo = __shfl_xor((unsigned)v, o, kWave);
      const u64 w = ((u64)hi << 32) | lo;
      v = w > v ? w : v;
    }
    return ((u64)(unsigned)uni((int)(v >> 32)) << 32) | (unsigned)uni((int)(unsigned)v);
  }
  // smallest r in [base, base + 64) with ok, or INT_MAX
  static __device__ __forceinline__ int first(bool ok, int r, int*) {
    const u64 m = __ballot(ok);
    return m ? uni(__shfl(r, __ffsll((long long)m) - 1, kWave)) : INT_MAX;
  }
};

template <>
struct Grp<kNpHeavyThreads> {
  static __device__ __forceinline__ int tid() { return threadIdx.x; }
  static __device__ __forceinline__ void sync() { __syncthreads(); }
  static __device__ __forceinline__ int sum(int v, int* red) {
    v = wave_sum(v);
    if (lane_id() == 0) red[wave_id()] = v;
    __syncthreads();
    int t = 0;
#pragma unroll
    for (int w = 0; w < kNpHeavyThreads / kWave; ++w) t += red[w];
    __syncthreads();
    return uni(t);
  }
  static __device__ __forceinline__ int bcast0(int v, int* red) {
    if (threadIdx.x == 0) red[0] = v;
    __syncthreads();
    v = uni(red[0]);
    __syncthreads();
    return v;
  }
  static __device__ __forceinline__ int excl_scan(int v, int* red, int* total) {
    int tot;
    const int ex = block_excl_scan(v, red, &tot);
    *total = uni(tot);
    return ex;
  }
  static __device__ __forceinline__ u64 max64(u64 v, int* red) {
    constexpr int NW = kNpHeavyThreads / kWave;
    v = Grp<kWave>::max64(v, nullptr);
    if (lane_id() == 0) {
      red[wave_id()] = (int)(unsigned)(v >> 32);
      red[NW + wave_id()] = (int)(unsigned)v;
    }
    __syncthreads();
    u64 m = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const u64 x = ((u64)(unsigned)red[w] << 32) | (unsigned)red[NW + w];
      m = x > m ? x : m;
    }
    __syncthreads();
    return ((u64)(unsigned)uni((int)(m >> 32)) << 32) | (unsigned)uni((int)(unsigned)m);
  }
  static __device__ __forceinline__ int first(bool ok, int r, int* red) {
    if (threadIdx.x == 0) red[0] = INT_MAX;
    __syncthreads();
    if (ok) atomicMin(&red[0], r);
    __syncthreads();
    const int f = uni(red[0]);
    __syncthreads();
    return f;
  }
};

// The positions of a batch of up to T index segments (segment t held by
// thread t) visited with all T threads of the group: the lengths' exclusive
// prefix goes through LDS and each position finds its segment by binary search.
template <int T, class ElemF>
__device__ __forceinline__ void seg_batch(int cnt, int64_t s0, int len, ElemF f, int* pre, int64_t* st,
                                          int* red) {
  const int t = Grp<T>::tid();
  int tot;
  const int ex = Grp<T>::excl_scan(t < cnt ? len : 0, red, &tot);
  pre[t] = ex;
  st[t] = s0;
  Grp<T>::sync();
  for (int q = t; q < tot; q += T) {
    int lo = 0, hi = cnt;  // pre[lo] <= q < pre[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (pre[mid] <= q) lo = mid; else hi = mid;
    }
    f(st[lo] + (q - pre[lo]));
  }
  Grp<T>::sync();
}

// nseg segments given by seg(j, start, len): kept in registers (one per
// thread) when they fit one batch, else computed again on every visit.
template <int T, class SegF>
struct SegSet {
  int nseg;
  SegF seg;
  int64_t s0 = 0;
  int len = 0;
  __device__ SegSet(int n_, SegF s_) : nseg(n_), seg(s_) {
    if (nseg <= T && Grp<T>::tid() < nseg) seg(Grp<T>::tid(), s0, len);
  }
  template <class ElemF>
  __device__ void each(ElemF f, int* pre, int64_t* st, int* red) {
    if (nseg <= T) {
      seg_batch<T>(nseg, s0, len, f, pre, st, red);
      return;
    }
    const int t = Grp<T>::tid();
    for (int base = 0; base < nseg; base += T) {
      const int cnt = min(T, nseg - base);
      int64_t b0 = 0;
      int bl = 0;
      if (t < cnt) seg(base + t, b0, bl);
      seg_batch<T>(cnt, b0, bl, f, pre, st, red);
    }
  }
};

template <int T>
struct NpLds {
  int hist[256];
  int pre[T];
  int64_t st[T];
  int red[2 * (kNpHeavyThreads / kWave) + 1];
  int bucket[3];
};

// The want-th smallest key K (want >= 1) among the points of `set` other
// than v, 8 bits at a time from the top; no early exit while shift >
// exit_shift. On return the keys of `set` among the want smallest are those
// with (key >> shift) <= lim. With exact, shift is 0 and lim is K itself (a
// last pass takes the largest key of the final bucket), so the test holds for
// any key, not only for those of `set`. Returns false if there are fewer
// than want keys.
template <int T, class Set>
__device__ bool radix_select(Set& set, const NpDev& a, int v, float xv, float yv, int want,
                             int exit_shift, bool exact, NpLds<T>& L, int& shift_out, u64& lim_out) {
  const int t = Grp<T>::tid();
  u64 prefix = 0, mask = 0;
  int shift = 56;
  while (true) {
    for (int b = t; b < 256; b += T) L.hist[b] = 0;
    Grp<T>::sync();
    set.each([&](int64_t pos) {
      const float4 rec = a.sorted[pos];
      const int w = __float_as_int(rec.z);
      if (w == v) return;
      const u64 key = np_key(np_d2(rec.x, rec.y, xv, yv), w);
      if ((key & mask) == prefix) atomicAdd(&L.hist[(key >> shift) & 255], 1);
    }, L.pre, L.st, L.red);
    if (t < kWave) {
      int c4[4], s = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        c4[q] = L.hist[4 * t + q];
        s += c4[q];
      }
      const int inc = wave_incl_scan(s);
      int below = inc - s;
      int hit = -1, hb = 0, hc = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (hit < 0 && below < want && want <= below + c4[q]) {
          hit = 4 * t + q;
          hb = below;
          hc = c4[q];
        }
        below += c4[q];
      }
      const int all = __shfl(inc, kWave - 1, kWave);
      if (hit >= 0) {  // exactly one lane
        L.bucket[0] = hit;
        L.bucket[1] = hb;
        L.bucket[2] = hc;
      }
      if (t == 0 && all < want) L.bucket[0] = -1;
    }
    Grp<T>::sync();
    const int bsel = uni(L.bucket[0]), bbelow = uni(L.bucket[1]), bcnt = uni(L.bucket[2]);
    Grp<T>::sync();
    if (bsel < 0) return false;
    prefix |= (u64)bsel << shift;
    mask |= (u64)255 << shift;
    want -= bbelow;
    if ((bcnt == want && shift <= exit_shift) || shift == 0) break;
    shift -= 8;
  }
  if (exact && shift > 0) {
    const u64 p = prefix >> shift;
    u64 m = 0;
    set.each([&](int64_t pos) {
      const float4 rec = a.sorted[pos];
      const int w = __float_as_int(rec.z);
      if (w == v) return;
      const u64 key = np_key(np_d2(rec.x, rec.y, xv, yv), w);
      if ((key >> shift) == p && key > m) m = key;
    }, L.pre, L.st, L.red);
    prefix = Grp<T>::max64(m, L.red);
    shift = 0;
  }
  shift_out = shift;
  lim_out = prefix >> shift;
  return true;
}

// One vertex per group; worker w takes entries w, w + W, ... of its list (W
// workers), and its bitmap is all zero between vertices. Nothing at the level
// of this loop depends on the lane: the results are stored by every lane
// (one address, one value), so the compiler keeps one loop for the wave.
template <int T>
__global__ __launch_bounds__(T == kWave ? kNpLightWaves * kWave : T) void k_np_eval(
    NpDev a, const int* list, const int* counts, int which) {
  constexpr int GPB = T == kWave ? kNpLightWaves : 1;
  __shared__ NpLds<T> lds_all[GPB];
  const int grp = T == kWave ? uni(wave_id()) : 0;
  NpLds<T>& L = lds_all[grp];
  const int t = Grp<T>::tid();
  const int worker = uni(blockIdx.x * GPB + grp), workers = uni(gridDim.x * GPB);
  unsigned* bm = a.bits + (size_t)worker * a.words;
  const int total = uni(counts[which]);
  for (int idx = worker; idx < total; idx += workers) {
    const int i = uni(list[idx]);
    const int v = uni(a.verts ? a.verts[i] : i);
    const int g = np_graph(a, v);
    const int ga = a.goff[g];
    const int64_t v0 = a.indptr[v];
    const int deg = (int)(a.indptr[v + 1] - v0);
    // walks: segment 0 is N(v), segment j >= 1 is N(j-th neighbour)
    auto walk_seg = [&](int j, int64_t& s0, int& len) {
      const int u = j == 0 ? v : a.indices[v0 + j - 1];
      s0 = a.indptr[u];
      len = (int)(a.indptr[u + 1] - s0);
    };
    SegSet<T, decltype(walk_seg)> walks(deg + 1, walk_seg);
    // pass 1: mark N_G(v), count its members
    int kl = 0;
    walks.each([&](int64_t pos) {
      const int u = a.indices[pos];
      if (u == v) return;
      const int lu = u - ga;
      const unsigned bit = 1u << (lu & 31);
      const unsigned old = atomicOr(&bm[lu >> 5], bit);
      kl += (old & bit) ? 0 : 1;
    }, L.pre, L.st, L.red);
    const int k = Grp<T>::sum(kl, L.red);
    if (k == 0) {
      a.ball[i] = 0;
      a.hits[i] = 0;
      continue;
    }
    const int Gg = a.gcell[g], cb = a.cbase[g];
    const float* bx = a.bx + a.colbase[g];
    const float* by = a.by + a.colbase[g];
    const int* S = a.sat + a.sbase[g];
    const float2 xv = a.X[v];
    const int cx = uni(qcell(bx, Gg, xv.x)), cy = uni(qcell(by, Gg, xv.y));
    // the smallest square of cells around v's cell that holds k others
    int r = INT_MAX;
    for (int base = 0; base < Gg && r == INT_MAX; base += T) {
      const int rr = base + t;
      bool ok = false;
      if (rr < Gg) {
        const int x1 = max(0, cx - rr), x2 = min(Gg - 1, cx + rr);
        const int y1 = max(0, cy - rr), y2 = min(Gg - 1, cy + rr);
        const int W = Gg + 1;
        const int c = S[(y2 + 1) * W + x2 + 1] - S[y1 * W + x2 + 1] - S[(y2 + 1) * W + x1] + S[y1 * W + x1];
        ok = c >= k + 1;
      }
      r = Grp<T>::first(ok, rr, L.red);
    }
    if (r == INT_MAX) r = Gg - 1;  // not reached: the whole grid holds n_g >= k + 1 points
    const int x1 = max(0, cx - r), x2 = min(Gg - 1, cx + r);
    const int y1 = max(0, cy - r), y2 = min(Gg - 1, cy + r);
    // phase A: the k-th smallest key in the square bounds the k-th distance
    auto square_seg = [&](int j, int64_t& s0, int& len) {
      const int row = cb + (y1 + j) * Gg;
      s0 = a.cstart[row + x1];
      len = a.cstart[row + x2 + 1] - (int)s0;
    };
    SegSet<T, decltype(square_seg)> square(y2 - y1 + 1, square_seg);
    int shift = 64;
    u64 lim = 0;
    bool okA = radix_select<T>(square, a, v, xv.x, xv.y, k, kSquareExitShift, false, L, shift, lim);
    bool okB = false;
    if (okA) {
      // an upper bound of the k-th key's squared distance (bits below `shift` set)
      const u64 ub = (lim << shift) | ((shift > 0) ? (~0ull >> (64 - shift)) : 0ull);
      const unsigned ubits = (unsigned)(ub >> 32);  // past +inf's bits the bound is +inf, not NaN
      const double d2 = ubits >= 0x7F800000u ? (double)INFINITY : (double)__uint_as_float(ubits);
      // a point whose FP32 key is at most that lies within rho (relative
      // rounding of the key below 1e-6, underflow below 1e-44)
      const double rho2 = d2 * (1.0 + 1e-5) + 1e-44;
      const double rho = sqrt(rho2);
      const double vx = xv.x, vy = xv.y;
      const int ylo = uni(qcell(by, Gg, vy - rho)), yhi = uni(qcell(by, Gg, vy + rho));
      // phase B: every point of the cells that meet the disc
      auto disc_seg = [&](int j, int64_t& s0, int& len) {
        const int c = ylo + j;
        const double dy = fmax(0.0, fmax((double)by[c] - vy, vy - (double)by[c + 1]));
        s0 = 0;
        len = 0;
        if (dy * dy > rho2) return;
        const double w = sqrt(rho2 - dy * dy);
        const int xl = qcell(bx, Gg, vx - w), xh = qcell(bx, Gg, vx + w);
        const int row = cb + c * Gg;
        s0 = a.cstart[row + xl];
        len = a.cstart[row + xh + 1] - (int)s0;
      };
      SegSet<T, decltype(disc_seg)> disc(yhi - ylo + 1, disc_seg);
      okB = radix_select<T>(disc, a, v, xv.x, xv.y, k, 64, true, L, shift, lim);
    }
    if (!okB) atomicOr(a.err, NP_ERR_SELECT);  // cannot happen: reported, nothing counted
    // pass 2: clear the bitmap, count the members among the k nearest
    int hl = 0;
    walks.each([&](int64_t pos) {
      const int u = a.indices[pos];
      if (u == v) return;
      const int lu = u - ga;
      const unsigned bit = 1u << (lu & 31);
      const unsigned old = atomicAnd(&bm[lu >> 5], ~bit);
      if (old & bit) {
        const float2 xu = a.X[u];
        const u64 key = np_key(np_d2(xu.x, xu.y, xv.x, xv.y), u);
        if (okB && (key >> shift) <= lim) ++hl;
      }
    }, L.pre, L.st, L.red);
    const int h = Grp<T>::sum(hl, L.red);
    a.ball[i] = k;
    a.hits[i] = h;
  }
}

// NP of graph g: the evaluated entries of g are a contiguous run of the
// (increasing) list; fixed-order FP64 sums of hits / (2k - hits) over k > 0.
__global__ __launch_bounds__(256) void k_np_mean(NpDev a, double* out) {
  __shared__ double rs[256];
  __shared__ int rc[256];
  const int g = blockIdx.x;
  int lo, hi;
  if (!a.verts) {
    lo = a.goff[g];
    hi = a.goff[g + 1];
  } else {
    auto lower = [&](int key) {
      int l = 0, h = a.nv;
      while (l < h) {
        const int m = (l + h) >> 1;
        if (a.verts[m] < key) l = m + 1; else h = m;
      }
      return l;
    };
    lo = lower(a.goff[g]);
    hi = lower(a.goff[g + 1]);
  }
  double s = 0.0;
  int c = 0;
  for (int i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    const int k = a.ball[i], h = a.hits[i];
    if (k > 0) {
      s += (double)h / (double)(2 * k - h);
      ++c;
    }
  }
  rs[threadIdx.x] = s;
  rc[threadIdx.x] = c;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      rs[threadIdx.x] += rs[threadIdx.x + o];
      rc[threadIdx.x] += rc[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[g] = rc[0] > 0 ? rs[0] / (double)rc[0] : NAN;
}

// ---- stress
struct StDev {
  const int64_t* indptr;
  const int* indices;
  const float2* X;
  int n, G;
  const int* goff;
  const int* src;   // sources of this batch
  int nsrc;
  u64* cur;         // [n] sources that reached each vertex
  u64* nxt;         // [n]
  double* acc;      // [n][4] pairs, sum (1 - r)^2, sum r, sum r^2 (r = e/d)
  int* flag;        // [2] level changed, bad source
};

__global__ __launch_bounds__(256) void k_st_clear(StDev a) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += gridDim.x * blockDim.x) a.cur[v] = 0;
}

__global__ void k_st_seed(StDev a) {
  const int i = threadIdx.x;
  if (i < a.nsrc) {
    const int s = a.src[i];
    if (s < 0 || s >= a.n) atomicOr(&a.flag[1], 1);
    else atomicOr(&a.cur[s], 1ull << i);
  }
}

__global__ __launch_bounds__(256) void k_st_level(StDev a, int level) {
  __shared__ double sx[kStressSources], sy[kStressSources];
  if (threadIdx.x < a.nsrc) {
    const int s = a.src[threadIdx.x];
    const float2 p = (s >= 0 && s < a.n) ? a.X[s] : make_float2(0.f, 0.f);
    sx[threadIdx.x] = p.x;
    sy[threadIdx.x] = p.y;
  }
  __syncthreads();
  const u64 full = a.nsrc == 64 ? ~0ull : ((1ull << a.nsrc) - 1);
  const double d = (double)level;
  for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < a.n; u += gridDim.x * blockDim.x) {
    const u64 c = a.cur[u];
    if (c == full) {
      a.nxt[u] = c;
      continue;
    }
    u64 nb = 0;
    const int64_t e1 = a.indptr[u + 1];
    for (int64_t e = a.indptr[u]; e < e1 && (nb | c) != full; ++e) nb |= a.cur[a.indices[e]];
    u64 nw = nb & ~c;
    a.nxt[u] = c | nw;
    if (!nw) continue;
    a.flag[0] = 1;
    const float2 xu = a.X[u];
    const double ux = xu.x, uy = xu.y;
    double cnt = 0.0, s1 = 0.0, sr = 0.0, sr2 = 0.0;
    while (nw) {
      const int b = __ffsll((long long)nw) - 1;
      nw &= nw - 1;
      const double dx = ux - sx[b], dy = uy - sy[b];
      const double rr = sqrt(dx * dx + dy * dy) / d;
      cnt += 1.0;
      s1 += (1.0 - rr) * (1.0 - rr);
      sr += rr;
      sr2 += rr * rr;
    }
    double* o = a.acc + (size_t)u * 4;
    o[0] += cnt;
    o[1] += s1;
    o[2] += sr;
    o[3] += sr2;
  }
}

// Per graph, fixed-order FP64 sums of the per-vertex sums, then the raw
// stress S1 / pairs and the stress at the best uniform scale
// (pairs - B^2 / C) / pairs (NaN without pairs; the raw value if C = 0).
__global__ __launch_bounds__(256) void k_st_sum(StDev a, double* out) {
  __shared__ double rs[4][256];
  const int g = blockIdx.x;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int v = a.goff[g] + threadIdx.x; v < a.goff[g + 1]; v += blockDim.x)
#pragma unroll
    for (int q = 0; q < 4; ++q) s[q] += a.acc[(size_t)v * 4 + q];
#pragma unroll
  for (int q = 0; q < 4; ++q) rs[q][threadIdx.x] = s[q];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o)
#pragma unroll
      for (int q = 0; q < 4; ++q) rs[q][threadIdx.x] += rs[q][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x < 4) out[(size_t)g * 6 + threadIdx.x] = rs[threadIdx.x][0];
  if (threadIdx.x == 0) {
    const double pairs = rs[0][0], s1 = rs[1][0], b = rs[2][0], c = rs[3][0];
    const double raw = pairs > 0.0 ? s1 / pairs : NAN;
    out[(size_t)g * 6 + 4] = raw;
    out[(size_t)g * 6 + 5] = pairs > 0.0 && c > 0.0 ? (pairs - b * b / c) / pairs : raw;
  }
}

__global__ __launch_bounds__(256) void k_fill_f64(double* p, size_t count) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// ---- host helpers
struct Owned {
  std::vector<void*> p;
  ~Owned() {
    for (void* q : p) (void)hipFree(q);
  }
  template <typename T>
  int alloc(T** ptr, size_t count, const char* what) {
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(ptr), count * sizeof(T));
    if (e != hipSuccess) {
      *ptr = nullptr;
      return fail(e == hipErrorOutOfMemory ? TSNET_ENOMEM : TSNET_EHIP,
                  std::string("hipMalloc (") + what + "): " + hipGetErrorString(e));
    }
    p.push_back(*ptr);
    return TSNET_OK;
  }
};

#define MET_HIP(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(TSNET_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
hipError_t to_dev(T* d, const std::vector<T>& h, hipStream_t s) {
  return hipMemcpyAsync(d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, s);
}

inline int grid_blocks(int64_t work, int per_block, int cap) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(cap, (work + per_block - 1) / per_block));
}

}  // namespace

int run_np(const int64_t* indptr, const int* indices, int n, const std::vector<int>& goff,
           const float* X, const int* verts, int nv, int* ball, int* hits, double* np_host,
           hipStream_t s) {
  const int G = (int)goff.size() - 1;
  // grid sizes (they depend on n_g only)
  std::vector<int> gcell(G), cbase(G + 1, 0), sbase(G, 0), colbase(G + 1, 0);
  int64_t cells = 0, satn = 0, maxng = 1;
  for (int g = 0; g < G; ++g) {
    const int ng = goff[g + 1] - goff[g];
    maxng = std::max<int64_t>(maxng, ng);
    const int Gg = (int)std::min<double>(kNpMaxGrid, std::max(1.0, std::ceil(std::sqrt((double)ng))));
    gcell[g] = Gg;
    sbase[g] = (int)satn;
    cells += (int64_t)Gg * Gg;
    satn += (int64_t)(Gg + 1) * (Gg + 1);
    cbase[g + 1] = (int)std::min<int64_t>(cells, INT_MAX);
    colbase[g + 1] = colbase[g] + Gg + 1;
  }
  if (cells >= INT_MAX / 2 || satn >= INT_MAX / 2) return fail(TSNET_EINVAL, "tsnet_np: graph too large");
  const int words = (int)((maxng + 31) / 32);
  // workers of the light kernel: as many as 512 MB of bitmaps allow, 256..8192
  const int64_t per_worker = (int64_t)words * 4;
  const int light_blocks = (int)std::max<int64_t>(
      64, std::min<int64_t>(2048, ((int64_t)512 << 20) / (per_worker * kNpLightWaves)));
  const int heavy_blocks = 256;
  const int64_t workers = std::max<int64_t>((int64_t)light_blocks * kNpLightWaves, heavy_blocks);
  const int rtiles = (n + kRadixTile - 1) / kRadixTile;
  const int64_t rhist_len = (int64_t)256 * rtiles;
  int gbits = 1;
  while ((1 << gbits) < G) ++gbits;
  Owned own;
  NpDev a;
  a.indptr = indptr;
  a.indices = indices;
  a.X = reinterpret_cast<const float2*>(X);
  a.n = n;
  a.G = G;
  a.verts = verts;
  a.nv = nv;
  a.words = words;
  a.ball = ball;
  a.hits = hits;
  int *goff_d, *gcell_d, *cbase_d, *sbase_d, *colbase_d, *tsum, *light, *heavy, *counts, *rhist, *rtsum;
  unsigned *kt, *vt;
  double* npd;
  int rc;
  if ((rc = own.alloc(&goff_d, G + 1, "offsets")) || (rc = own.alloc(&gcell_d, G, "grid")) ||
      (rc = own.alloc(&cbase_d, G + 1, "grid")) || (rc = own.alloc(&sbase_d, G, "grid")) ||
      (rc = own.alloc(&colbase_d, G + 1, "grid")) || (rc = own.alloc(&a.bx, colbase[G], "bounds")) ||
      (rc = own.alloc(&a.by, colbase[G], "bounds")) || (rc = own.alloc(&a.cell_of, n, "cells")) ||
      (rc = own.alloc(&a.cnt, cells + 1, "cells")) || (rc = own.alloc(&a.cstart, cells + 1, "cells")) ||
      (rc = own.alloc(&tsum, (cells + kTileScan) / kTileScan + 1, "scan")) ||
      (rc = own.alloc(&a.sat, satn, "summed-area tables")) ||
      (rc = own.alloc(&a.sorted, n, "sorted points")) || (rc = own.alloc(&a.skey, n, "sort")) ||
      (rc = own.alloc(&a.sval, n, "sort")) || (rc = own.alloc(&kt, n, "sort")) ||
      (rc = own.alloc(&vt, n, "sort")) || (rc = own.alloc(&rhist, rhist_len + 1, "sort")) ||
      (rc = own.alloc(&rtsum, (rhist_len + kTileScan) / kTileScan + 1, "sort")) ||
      (rc = own.alloc(&light, nv, "lists")) || (rc = own.alloc(&heavy, nv, "lists")) ||
      (rc = own.alloc(&counts, 8, "counters")) || (rc = own.alloc(&npd, G, "means")) ||
      (rc = own.alloc(&a.bits, (size_t)workers * words, "bitmaps")))
    return rc;
  a.err = counts + 2;
  a.goff = goff_d;
  a.gcell = gcell_d;
  a.cbase = cbase_d;
  a.sbase = sbase_d;
  a.colbase = colbase_d;
  MET_HIP(to_dev(goff_d, goff, s));
  MET_HIP(to_dev(gcell_d, gcell, s));
  MET_HIP(to_dev(cbase_d, cbase, s));
  MET_HIP(to_dev(sbase_d, sbase, s));
  MET_HIP(to_dev(colbase_d, colbase, s));
  const size_t nbits = (size_t)workers * words;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_blocks(nbits, 256, 8192)), dim3(256), 0, s, a.bits, nbits, 0u);
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_blocks(cells + 1, 256, 8192)), dim3(256), 0, s,
                     reinterpret_cast<unsigned*>(a.cnt), (size_t)cells + 1, 0u);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, reinterpret_cast<unsigned*>(counts), (size_t)8, 0u);
  MET_HIP(hipGetLastError());
  const int vb = grid_blocks(n, 256, 8192);
  hipLaunchKernelGGL(k_np_check, dim3(vb), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_np_classify, dim3(grid_blocks(nv, 256, 8192)), dim3(256), 0, s, a, light, heavy, counts);
  MET_HIP(hipGetLastError());
  int hc[3];
  MET_HIP(hipMemcpyAsync(hc, counts, sizeof(hc), hipMemcpyDeviceToHost, s));
  MET_HIP(hipStreamSynchronize(s));
  if (hc[2] & NP_ERR_COORD) return fail(TSNET_EINVAL, "tsnet_np: X holds a non-finite coordinate");
  if (hc[2] & NP_ERR_VERTEX) return fail(TSNET_EINVAL, "tsnet_np: a vertex id is out of range");
  if (hc[2] & NP_ERR_ORDER) return fail(TSNET_EINVAL, "tsnet_np: vertices must be strictly increasing");
  // cell boundaries: per axis, a sort by coordinate (then, stably, by graph)
  for (int axis = 0; axis < 2; ++axis) {
    hipLaunchKernelGGL(k_np_axis_keys, dim3(vb), dim3(256), 0, s, a, axis);
    MET_HIP(hipGetLastError());
    MET_HIP(radix_sort(a.skey, a.sval, kt, vt, n, 32, rhist, rtsum, s));
    if (G > 1) {
      hipLaunchKernelGGL(k_np_graph_keys, dim3(vb), dim3(256), 0, s, a);
      MET_HIP(hipGetLastError());
      MET_HIP(radix_sort(a.skey, a.sval, kt, vt, n, gbits, rhist, rtsum, s));
    }
    hipLaunchKernelGGL(k_np_bounds, dim3(grid_blocks(colbase[G], 256, 4096)), dim3(256), 0, s, a, axis,
                       colbase[G]);
    MET_HIP(hipGetLastError());
  }
  // counting sort into cells, cell starts, summed-area tables
  hipLaunchKernelGGL(k_np_cells, dim3(vb), dim3(256), 0, s, a);
  MET_HIP(hipGetLastError());
  MET_HIP(exclusive_scan<int>(a.cnt, cells, a.cstart, tsum, s));
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_blocks(cells + 1, 256, 8192)), dim3(256), 0, s,
                     reinterpret_cast<unsigned*>(a.cnt), (size_t)cells + 1, 0u);
  hipLaunchKernelGGL(k_np_scatter, dim3(vb), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_np_sat, dim3(grid_blocks(colbase[G], 256, 4096)), dim3(256), 0, s, a, colbase[G]);
  MET_HIP(hipGetLastError());
  if (hc[0] > 0)
    hipLaunchKernelGGL(k_np_eval<kWave>, dim3(std::min(light_blocks, (hc[0] + kNpLightWaves - 1) / kNpLightWaves)),
                       dim3(kNpLightWaves * kWave), 0, s, a, light, counts, 0);
  if (hc[1] > 0)
    hipLaunchKernelGGL(k_np_eval<kNpHeavyThreads>, dim3(std::min(heavy_blocks, hc[1])),
                       dim3(kNpHeavyThreads), 0, s, a, heavy, counts, 1);
  MET_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_np_mean, dim3(G), dim3(256), 0, s, a, npd);
  MET_HIP(hipGetLastError());
  int err = 0;
  MET_HIP(hipMemcpyAsync(&err, a.err, sizeof(int), hipMemcpyDeviceToHost, s));
  if (np_host) MET_HIP(hipMemcpyAsync(np_host, npd, sizeof(double) * G, hipMemcpyDeviceToHost, s));
  MET_HIP(hipStreamSynchronize(s));
  if (err & NP_ERR_SELECT) return fail(TSNET_EHIP, "tsnet_np: candidate search came up short");
  return TSNET_OK;
}

int run_stress(const int64_t* indptr, const int* indices, int n, const std::vector<int>& goff,
               const float* X, const int* sources, int nsrc, double* sums_host, int* levels_host,
               hipStream_t s) {
  const int G = (int)goff.size() - 1;
  Owned own;
  StDev a;
  a.indptr = indptr;
  a.indices = indices;
  a.X = reinterpret_cast<const float2*>(X);
  a.n = n;
  a.G = G;
  int *goff_d, *flag;
  double* out;
  int rc;
  if ((rc = own.alloc(&goff_d, G + 1, "offsets")) || (rc = own.alloc(&a.cur, n, "reached sets")) ||
      (rc = own.alloc(&a.nxt, n, "reached sets")) || (rc = own.alloc(&a.acc, (size_t)n * 4, "sums")) ||
      (rc = own.alloc(&flag, 2, "flags")) || (rc = own.alloc(&out, (size_t)G * 6, "sums")))
    return rc;
  a.goff = goff_d;
  a.flag = flag;
  MET_HIP(to_dev(goff_d, goff, s));
  hipLaunchKernelGGL(k_fill_f64, dim3(grid_blocks((int64_t)n * 4, 256, 8192)), dim3(256), 0, s, a.acc,
                     (size_t)n * 4);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, reinterpret_cast<unsigned*>(flag), (size_t)2, 0u);
  MET_HIP(hipGetLastError());
  const int vb = grid_blocks(n, 256, 8192);
  int64_t levels = 0;
  for (int b0 = 0; b0 < nsrc; b0 += kStressSources) {
    a.src = sources + b0;
    a.nsrc = std::min(kStressSources, nsrc - b0);
    hipLaunchKernelGGL(k_st_clear, dim3(vb), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_st_seed, dim3(1), dim3(kStressSources), 0, s, a);
    MET_HIP(hipGetLastError());
    for (int level = 1; level <= n; ++level) {
      hipLaunchKernelGGL(k_st_level, dim3(vb), dim3(256), 0, s, a, level);
      MET_HIP(hipGetLastError());
      int fl[2];
      MET_HIP(hipMemcpyAsync(fl, flag, sizeof(fl), hipMemcpyDeviceToHost, s));
      hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, reinterpret_cast<unsigned*>(flag), (size_t)1, 0u);
      MET_HIP(hipStreamSynchronize(s));
      if (fl[1]) return fail(TSNET_EINVAL, "tsnet_stress: a source id is out of range");
      std::swap(a.cur, a.nxt);
      ++levels;
      if (!fl[0]) break;
    }
  }
  hipLaunchKernelGGL(k_st_sum, dim3(G), dim3(256), 0, s, a, out);
  MET_HIP(hipGetLastError());
  MET_HIP(hipMemcpyAsync(sums_host, out, sizeof(double) * G * 6, hipMemcpyDeviceToHost, s));
  MET_HIP(hipStreamSynchronize(s));
  if (levels_host) *levels_host = (int)std::min<int64_t>(levels, INT_MAX);
  return TSNET_OK;
}

}  // namespace tsnet
