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
//  * N_D(v): the points are counting-sorted into a uniform grid of about one
//    point per cell (square cells over the graph's bounding box), with a
//    summed-area table of the cell counts. The smallest square of cells
//    around v's cell holding k others bounds the k-th distance; every point
//    that can be nearer lies in the cells of a disc around v (widened by one
//    cell plus a slack for the FP32 cell assignment). The k-th smallest key
//    (squared distance bits, id) over that disc is found by an 8-bit radix
//    select; a vertex is among the k nearest iff its key is not above it.
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
constexpr int kNpChunk = 1024;         // vertices per chunk of the bounding boxes
constexpr int kNpHeavyWalks = 4096;    // 2-hop walks above which a vertex gets a whole block
constexpr int kNpLightWaves = 4;       // waves (one vertex each) per block of the light kernel
constexpr int kNpHeavyThreads = 1024;  // threads per vertex of the heavy kernel
constexpr float kCellSlack = 1.002f;   // one cell plus the FP32 cell-assignment slack
constexpr int kStressSources = 64;     // sources per bit-parallel BFS

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
  const int* colbase;   // [G+1] first summed-area column of each graph
  float4* gparam;       // [G] (x0, y0, cells per unit length, unused)
  int* cell_of;         // [n]
  int* cnt;             // [cells + 1] counts, then the fill cursors
  int* cstart;          // [cells + 1] first sorted point of each cell
  int* sat;             // summed-area tables, (G_g + 1)^2 per graph
  float4* sorted;       // [n] (x, y, id bits, 0) in cell order
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

// Cell of a point: floor((x - x0) * cells per unit), clamped to the grid
// (NaN, from an overflowing difference with a zero scale, goes to cell 0).
__device__ __forceinline__ int np_cell1(float x, float x0, float inv, int Gg) {
  const float u = (x - x0) * inv;
  return u >= 0.f ? (int)fminf(u, (float)(Gg - 1)) : 0;
}

__device__ __forceinline__ void np_cell_xy(const float4& p, int Gg, float x, float y, int& cx, int& cy) {
  cx = np_cell1(x, p.x, p.z, Gg);
  cy = np_cell1(y, p.y, p.z, Gg);
}

__global__ void k_fill_u32(unsigned* p, size_t count, unsigned v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Bounding box of each chunk (one graph, up to kNpChunk vertices).
__global__ __launch_bounds__(256) void k_np_bbox(NpDev a, const int* cs, const int* ce, float4* part) {
  __shared__ float red[4][256 / kWave];
  const int c = blockIdx.x;
  float mnx = INFINITY, mny = INFINITY, mxx = -INFINITY, mxy = -INFINITY;
  bool bad = false;
  for (int v = cs[c] + threadIdx.x; v < ce[c]; v += blockDim.x) {
    const float2 p = a.X[v];
    if (!isfinite(p.x) || !isfinite(p.y)) bad = true;
    mnx = fminf(mnx, p.x);
    mny = fminf(mny, p.y);
    mxx = fmaxf(mxx, p.x);
    mxy = fmaxf(mxy, p.y);
  }
  if (bad) atomicOr(a.err, NP_ERR_COORD);
  mnx = wave_min(mnx);
  mny = wave_min(mny);
  mxx = wave_max(mxx);
  mxy = wave_max(mxy);
  if (lane_id() == 0) {
    red[0][wave_id()] = mnx;
    red[1][wave_id()] = mny;
    red[2][wave_id()] = mxx;
    red[3][wave_id()] = mxy;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 256 / kWave; ++w) {
      mnx = fminf(mnx, red[0][w]);
      mny = fminf(mny, red[1][w]);
      mxx = fmaxf(mxx, red[2][w]);
      mxy = fmaxf(mxy, red[3][w]);
    }
    part[c] = make_float4(mnx, mny, mxx, mxy);
  }
}

// Per graph: the box from its chunks and the cell size (square cells over the
// larger side). A zero or unusable span puts every point in cell (0, 0).
__global__ void k_np_plan(NpDev a, const int* gcb, const int* gce, const float4* part) {
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < a.G; g += gridDim.x * blockDim.x) {
    float mnx = INFINITY, mny = INFINITY, mxx = -INFINITY, mxy = -INFINITY;
    for (int c = gcb[g]; c < gce[g]; ++c) {
      const float4 p = part[c];
      mnx = fminf(mnx, p.x);
      mny = fminf(mny, p.y);
      mxx = fmaxf(mxx, p.z);
      mxy = fmaxf(mxy, p.w);
    }
    const float span = fmaxf(mxx - mnx, mxy - mny);
    float inv = span > 0.f ? (float)a.gcell[g] / span : 0.f;
    if (!isfinite(inv)) inv = 0.f;
    a.gparam[g] = make_float4(mnx, mny, inv, 0.f);
  }
}

__global__ __launch_bounds__(256) void k_np_cells(NpDev a) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += gridDim.x * blockDim.x) {
    const int g = np_graph(a, v);
    const int Gg = a.gcell[g];
    const float2 x = a.X[v];
    int cx, cy;
    np_cell_xy(a.gparam[g], Gg, x.x, x.y, cx, cy);
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

// Calls f(pos) for every position of nseg index segments with all T threads
// of the group: segments go T at a time through LDS (start, exclusive prefix
// of lengths), and each position finds its segment by binary search.
template <int T, class SegF, class ElemF>
__device__ __forceinline__ void for_segments(int nseg, SegF seg, ElemF f, int* pre, int64_t* st,
                                             int* red) {
  const int t = Grp<T>::tid();
  for (int base = 0; base < nseg; base += T) {
    const int cnt = min(T, nseg - base);
    int64_t s0 = 0;
    int len = 0;
    if (t < cnt) seg(base + t, s0, len);
    int tot;
    const int ex = Grp<T>::excl_scan(len, red, &tot);
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
}

template <int T>
struct NpLds {
  int hist[256];
  int pre[T];
  int64_t st[T];
  int red[kNpHeavyThreads / kWave + 1];
  int bucket[3];
};

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
    // pass 1: mark N_G(v), count its members
    int kl = 0;
    for_segments<T>(deg + 1, walk_seg, [&](int64_t pos) {
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
    // the smallest square of cells around v's cell that holds k others
    const float4 p = a.gparam[g];
    const int Gg = a.gcell[g], cb = a.cbase[g];
    const int* S = a.sat + a.sbase[g];
    const float2 xv = a.X[v];
    int cx, cy;
    np_cell_xy(p, Gg, xv.x, xv.y, cx, cy);
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
    // every point that can be among the k nearest lies within rho cells of v
    const float rho = 1.41421356f * ((float)r + kCellSlack) * 1.00001f;
    const int Ry = (int)floorf(rho + kCellSlack);
    const int ylo = max(0, cy - Ry), yhi = min(Gg - 1, cy + Ry);
    auto cand_seg = [&](int j, int64_t& s0, int& len) {
      const int y = ylo + j;
      const float dy = fmaxf(0.f, fabsf((float)(y - cy)) - kCellSlack);
      s0 = 0;
      len = 0;
      if (dy > rho) return;
      const int wx = (int)floorf(sqrtf(fmaxf(0.f, rho * rho - dy * dy)) + kCellSlack);
      const int x1 = max(0, cx - wx), x2 = min(Gg - 1, cx + wx);
      const int row = cb + y * Gg;
      s0 = a.cstart[row + x1];
      len = a.cstart[row + x2 + 1] - (int)s0;
    };
    // radix select of the k-th smallest key, 8 bits at a time from the top
    u64 prefix = 0, mask = 0;
    int want = k, shift = 56;
    while (true) {
      for (int b = t; b < 256; b += T) L.hist[b] = 0;
      Grp<T>::sync();
      for_segments<T>(yhi - ylo + 1, cand_seg, [&](int64_t pos) {
        const float4 rec = a.sorted[pos];
        const int w = __float_as_int(rec.z);
        if (w == v) return;
        const u64 key = np_key(np_d2(rec.x, rec.y, xv.x, xv.y), w);
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
      if (bsel < 0) {  // fewer candidates than k: cannot happen; reported, nothing counted
        atomicOr(a.err, NP_ERR_SELECT);
        prefix = 0;
        shift = 64;
        break;
      }
      prefix |= (u64)bsel << shift;
      mask |= (u64)255 << shift;
      want -= bbelow;
      if (bcnt == want || shift == 0) break;
      shift -= 8;
    }
    // a key is among the k nearest iff its bits above `shift` do not exceed the prefix's
    const u64 lim = shift >= 64 ? 0 : (prefix >> shift);
    // pass 2: clear the bitmap, count the members among the k nearest
    int hl = 0;
    for_segments<T>(deg + 1, walk_seg, [&](int64_t pos) {
      const int u = a.indices[pos];
      if (u == v) return;
      const int lu = u - ga;
      const unsigned bit = 1u << (lu & 31);
      const unsigned old = atomicAnd(&bm[lu >> 5], ~bit);
      if (old & bit) {
        const float2 xu = a.X[u];
        const u64 key = np_key(np_d2(xu.x, xu.y, xv.x, xv.y), u);
        if (shift < 64 && (key >> shift) <= lim) ++hl;
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
  // grid plan and chunks (host: the cell counts depend on n_g only)
  std::vector<int> gcell(G), cbase(G + 1, 0), sbase(G, 0), colbase(G + 1, 0);
  std::vector<int> cs, ce, gcb(G), gce(G);
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
    gcb[g] = (int)cs.size();
    for (int v = goff[g]; v < goff[g + 1]; v += kNpChunk) {
      cs.push_back(v);
      ce.push_back(std::min(goff[g + 1], v + kNpChunk));
    }
    gce[g] = (int)cs.size();
  }
  if (cells >= INT_MAX / 2 || satn >= INT_MAX / 2) return fail(TSNET_EINVAL, "tsnet_np: graph too large");
  const int nc = (int)cs.size();
  const int words = (int)((maxng + 31) / 32);
  // workers of the light kernel: as many as 512 MB of bitmaps allow, 256..8192 blocks' worth
  const int64_t per_worker = (int64_t)words * 4;
  const int light_blocks = (int)std::max<int64_t>(
      64, std::min<int64_t>(2048, ((int64_t)512 << 20) / (per_worker * kNpLightWaves)));
  const int heavy_blocks = 256;
  const int64_t workers = (int64_t)light_blocks * kNpLightWaves;
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
  int *goff_d, *gcell_d, *cbase_d, *sbase_d, *colbase_d, *cs_d, *ce_d, *gcb_d, *gce_d;
  int *tsum, *light, *heavy, *counts;
  float4 *gparam, *part;
  double* npd;
  int rc;
  if ((rc = own.alloc(&goff_d, G + 1, "offsets")) || (rc = own.alloc(&gcell_d, G, "grid")) ||
      (rc = own.alloc(&cbase_d, G + 1, "grid")) || (rc = own.alloc(&sbase_d, G, "grid")) ||
      (rc = own.alloc(&colbase_d, G + 1, "grid")) || (rc = own.alloc(&cs_d, nc, "chunks")) ||
      (rc = own.alloc(&ce_d, nc, "chunks")) || (rc = own.alloc(&gcb_d, G, "chunks")) ||
      (rc = own.alloc(&gce_d, G, "chunks")) || (rc = own.alloc(&gparam, G, "grid")) ||
      (rc = own.alloc(&part, nc, "boxes")) || (rc = own.alloc(&a.cell_of, n, "cells")) ||
      (rc = own.alloc(&a.cnt, cells + 1, "cells")) || (rc = own.alloc(&a.cstart, cells + 1, "cells")) ||
      (rc = own.alloc(&tsum, (cells + kTileScan) / kTileScan + 1, "scan")) ||
      (rc = own.alloc(&a.sat, satn, "summed-area tables")) ||
      (rc = own.alloc(&a.sorted, n, "sorted points")) || (rc = own.alloc(&light, nv, "lists")) ||
      (rc = own.alloc(&heavy, nv, "lists")) || (rc = own.alloc(&counts, 8, "counters")) ||
      (rc = own.alloc(&npd, G, "means")) ||
      (rc = own.alloc(&a.bits, (size_t)std::max<int64_t>(workers, heavy_blocks) * words, "bitmaps")))
    return rc;
  a.err = counts + 2;
  a.goff = goff_d;
  a.gcell = gcell_d;
  a.cbase = cbase_d;
  a.sbase = sbase_d;
  a.colbase = colbase_d;
  a.gparam = gparam;
  MET_HIP(to_dev(goff_d, goff, s));
  MET_HIP(to_dev(gcell_d, gcell, s));
  MET_HIP(to_dev(cbase_d, cbase, s));
  MET_HIP(to_dev(sbase_d, sbase, s));
  MET_HIP(to_dev(colbase_d, colbase, s));
  MET_HIP(to_dev(cs_d, cs, s));
  MET_HIP(to_dev(ce_d, ce, s));
  MET_HIP(to_dev(gcb_d, gcb, s));
  MET_HIP(to_dev(gce_d, gce, s));
  const size_t nbits = (size_t)std::max<int64_t>(workers, heavy_blocks) * words;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_blocks(nbits, 256, 8192)), dim3(256), 0, s, a.bits, nbits, 0u);
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_blocks(cells + 1, 256, 8192)), dim3(256), 0, s,
                     reinterpret_cast<unsigned*>(a.cnt), (size_t)cells + 1, 0u);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, reinterpret_cast<unsigned*>(counts), (size_t)8, 0u);
  MET_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_np_bbox, dim3(nc), dim3(256), 0, s, a, cs_d, ce_d, part);
  hipLaunchKernelGGL(k_np_plan, dim3(grid_blocks(G, 256, 1024)), dim3(256), 0, s, a, gcb_d, gce_d, part);
  hipLaunchKernelGGL(k_np_classify, dim3(grid_blocks(nv, 256, 8192)), dim3(256), 0, s, a, light, heavy, counts);
  MET_HIP(hipGetLastError());
  int hc[3];
  MET_HIP(hipMemcpyAsync(hc, counts, sizeof(hc), hipMemcpyDeviceToHost, s));
  MET_HIP(hipStreamSynchronize(s));
  if (hc[2] & NP_ERR_COORD) return fail(TSNET_EINVAL, "tsnet_np: X holds a non-finite coordinate");
  if (hc[2] & NP_ERR_VERTEX) return fail(TSNET_EINVAL, "tsnet_np: a vertex id is out of range");
  if (hc[2] & NP_ERR_ORDER) return fail(TSNET_EINVAL, "tsnet_np: vertices must be strictly increasing");
  // counting sort into cells, cell starts, summed-area tables
  hipLaunchKernelGGL(k_np_cells, dim3(grid_blocks(n, 256, 8192)), dim3(256), 0, s, a);
  MET_HIP(hipGetLastError());
  MET_HIP(exclusive_scan<int>(a.cnt, cells, a.cstart, tsum, s));
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_blocks(cells + 1, 256, 8192)), dim3(256), 0, s,
                     reinterpret_cast<unsigned*>(a.cnt), (size_t)cells + 1, 0u);
  hipLaunchKernelGGL(k_np_scatter, dim3(grid_blocks(n, 256, 8192)), dim3(256), 0, s, a);
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
