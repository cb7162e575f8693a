// Barnes-Hut quadtree sums of the repulsion (with Z) and entropy terms:
// C1 of BH-tsNET (Algorithm 1, the BH-SNE quadtree of Sec. 2.2) and C2 of
// BH-tsNET and FIt-tsNET (Algorithms 1-2, Eq. 7). The paper fixes neither
// the tree nor the opening test; the readings are the project's:
//
//  * Per graph, the bounding square (side = the larger extent, in FP64) is
//    cut into 2^32 cells per axis; a point's cell is floor((x - x_min) *
//    2^32 / side) in FP64. Its 64-bit code interleaves the cell bits, y above
//    x, so the 2-bit digit of level l is the l-th quadrant choice from the
//    root. 32 levels keep the leaves small when a few far points stretch the
//    square (the bulk of the layout then covers a tiny corner of it; with 16
//    levels whole clusters shared a leaf and were summed pair by pair).
//    Points are sorted by (graph, code, id) with stable radix sorts: the low
//    code word, the high code word, then the graph.
//  * The tree is the linear quadtree of the sorted codes: a node per
//    non-empty prefix of l digits whose parent holds two or more points;
//    leaves hold one point or sit at level 32. Sorted position p starts the
//    nodes of levels lmin(p)..lmax(p): lmin is one past the digits p shares
//    with p - 1 (0 at the graph's first point), lmax is one past the digits
//    it shares with p + 1 (at most 32, at least lmin). Numbering nodes by
//    (start, level) is a depth-first order, so a node's first child is the
//    next node and the node after its subtree is the first node starting at
//    its end: the traversal needs no stack.
//  * A node's centre of mass is its FP64 coordinate sum (a difference of
//    exclusive prefix sums over the sorted points) over its count.
//  * Point i walks the nodes of its graph in that order: a leaf adds its
//    points one by one (i itself left out); an inner node of width w = side /
//    2^l is a summary when w^2 < theta^2 ||X_i - c||^2 (FP64), adding its
//    count times the terms at c, else it is opened. theta <= 0.7 keeps a node
//    holding i from being a summary.
//  * Terms (FP32) at offset d, r2 = ||d||^2: z = 1 / (1 + r2) (sum z_i, and
//    Z = sum_i z_i per graph in FP64, fixed order), F_rep += z^2 d, F_ent +=
//    d / (eps + r2), and for the cost ln(eps + r2) (its per-vertex sum holds
//    the self term ln(eps), as the interpolated one does).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <string>

#include "dev_util.h"
#include "scan.h"
#include "tsnet_internal.h"

namespace tsnet {

struct QtParam {
  double x0, y0, side, scale;
};

// One node, 32 bytes: its sorted range, the first node after its subtree and
// its level, then its centre of mass (one record, so one line per visit).
struct __align__(32) QtNode {
  int4 b;      // (start, count, first node after the subtree, level)
  double2 c;   // centre of mass
};

struct QuadWs {
  int n = 0, G = 0, max_nodes = 0, gbits = 1;
  QtParam* gp = nullptr;     // [G]
  float4* part = nullptr;    // [num_chunks] bounding-box partials
  unsigned *key = nullptr, *val = nullptr, *kt = nullptr, *vt = nullptr;  // [n] sort
  int *rhist = nullptr, *rtsum = nullptr;
  unsigned long long* code = nullptr;  // [n] codes in sorted order
  float2* xs = nullptr;      // [n] X in sorted order
  double *px = nullptr, *py = nullptr;  // [n + 1] sorted X in FP64, then exclusive prefix sums
  double* dtsum = nullptr;
  int* base = nullptr;       // [n + 1] nodes starting at each position, then the first node index
  int* itsum = nullptr;
  QtNode* nodes = nullptr;   // [max_nodes]
  float* zv = nullptr;       // [n] sum_j z_ij per vertex
};

namespace {

constexpr int kQtLevels = 32;
constexpr double kQtCells = 4294967296.0;

__device__ __forceinline__ unsigned qt_coord(float x, double x0, double scale) {
#pragma clang fp contract(off)
  const double u = ((double)x - x0) * scale;
  return u >= 0.0 ? (u < kQtCells - 1.0 ? (unsigned)floor(u) : (unsigned)(kQtCells - 1.0)) : 0u;
}

__device__ __forceinline__ unsigned long long qt_spread(unsigned u) {  // bit b -> bit 2b
  unsigned long long v = u;
  v = (v | (v << 16)) & 0x0000FFFF0000FFFFull;
  v = (v | (v << 8)) & 0x00FF00FF00FF00FFull;
  v = (v | (v << 4)) & 0x0F0F0F0F0F0F0F0Full;
  v = (v | (v << 2)) & 0x3333333333333333ull;
  v = (v | (v << 1)) & 0x5555555555555555ull;
  return v;
}

__device__ __forceinline__ unsigned long long qt_code(float2 x, const QtParam& p) {
  return (qt_spread(qt_coord(x.y, p.y0, p.scale)) << 1) | qt_spread(qt_coord(x.x, p.x0, p.scale));
}

// digits shared by two different codes
__device__ __forceinline__ int qt_cpl(unsigned long long a, unsigned long long b) {
  return __clzll(a ^ b) >> 1;
}

struct QtDev {
  const float2* X;
  int n, G;
  const int* goff;
  QuadWs w;
};

__device__ __forceinline__ int qt_graph(const QtDev& a, int v) {
  return a.G == 1 ? 0 : graph_of(a.goff, a.G, v);
}

__global__ __launch_bounds__(256) void k_qt_bbox(QtDev a, const int* cs, const int* ce) {
  __shared__ float red[4][256 / kWave];
  const int c = blockIdx.x;
  float mnx = INFINITY, mny = INFINITY, mxx = -INFINITY, mxy = -INFINITY;
  for (int v = cs[c] + threadIdx.x; v < ce[c]; v += blockDim.x) {
    const float2 p = a.X[v];
    mnx = fminf(mnx, p.x);
    mny = fminf(mny, p.y);
    mxx = fmaxf(mxx, p.x);
    mxy = fmaxf(mxy, p.y);
  }
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
    a.w.part[c] = make_float4(mnx, mny, mxx, mxy);
  }
}

// One block per graph: its box from the chunk partials (block-strided, then
// a wave reduction), then the cell scale.
__global__ __launch_bounds__(256) void k_qt_plan(QtDev a, const GraphInfo* gi) {
  __shared__ float red[4][256 / kWave];
  const int g = blockIdx.x;
  float mnx = INFINITY, mny = INFINITY, mxx = -INFINITY, mxy = -INFINITY;
  for (int c = gi[g].chunk_begin + threadIdx.x; c < gi[g].chunk_end; c += blockDim.x) {
    const float4 p = a.w.part[c];
    mnx = fminf(mnx, p.x);
    mny = fminf(mny, p.y);
    mxx = fmaxf(mxx, p.z);
    mxy = fmaxf(mxy, p.w);
  }
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
    double side = fmax((double)mxx - (double)mnx, (double)mxy - (double)mny);
    if (!(side > 0.0) || !isfinite(side)) side = 1.0;
    QtParam q;
    q.x0 = mnx;
    q.y0 = mny;
    q.side = side;
    q.scale = kQtCells / side;
    a.w.gp[g] = q;
  }
}

// sort keys, first pass: the low code word of each vertex
__global__ __launch_bounds__(256) void k_qt_codes(QtDev a) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += gridDim.x * blockDim.x) {
    a.w.key[v] = (unsigned)qt_code(a.X[v], a.w.gp[qt_graph(a, v)]);
    a.w.val[v] = (unsigned)v;
  }
}

// second pass: the high code word of the vertex at each position
__global__ __launch_bounds__(256) void k_qt_high_keys(QtDev a) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < a.n; p += gridDim.x * blockDim.x) {
    const int v = (int)a.w.val[p];
    a.w.key[p] = (unsigned)(qt_code(a.X[v], a.w.gp[qt_graph(a, v)]) >> 32);
  }
}

__global__ __launch_bounds__(256) void k_qt_graph_keys(QtDev a) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < a.n; p += gridDim.x * blockDim.x)
    a.w.key[p] = (unsigned)graph_of(a.goff, a.G, (int)a.w.val[p]);
}

// Sorted position p (graph g's positions are goff[g]..goff[g+1]-1): its code,
// point and FP64 coordinates.
__global__ __launch_bounds__(256) void k_qt_sorted(QtDev a) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < a.n; p += gridDim.x * blockDim.x) {
    const int v = (int)a.w.val[p];
    const float2 x = a.X[v];
    a.w.code[p] = qt_code(x, a.w.gp[qt_graph(a, v)]);
    a.w.xs[p] = x;
    a.w.px[p] = x.x;
    a.w.py[p] = x.y;
  }
}

__device__ __forceinline__ void qt_levels(const QtDev& a, int p, int gs, int ge, int& lmin, int& lmax) {
  const unsigned long long c = a.w.code[p];
  if (p == gs) {
    lmin = 0;
  } else {
    const unsigned long long cp = a.w.code[p - 1];
    lmin = cp == c ? -1 : qt_cpl(cp, c) + 1;
  }
  int nxt = -1;
  if (p + 1 < ge) {
    const unsigned long long cn = a.w.code[p + 1];
    nxt = cn == c ? kQtLevels : qt_cpl(c, cn);
  }
  lmax = min(kQtLevels, max(lmin, nxt + 1));
}

__global__ __launch_bounds__(256) void k_qt_count(QtDev a) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < a.n; p += gridDim.x * blockDim.x) {
    const int g = qt_graph(a, p);
    int lmin, lmax;
    qt_levels(a, p, a.goff[g], a.goff[g + 1], lmin, lmax);
    a.w.base[p] = lmin < 0 ? 0 : lmax - lmin + 1;
  }
}

// The nodes starting at position p: end of each prefix run by a galloping
// search over the sorted codes, skip = first node at or after that end.
__global__ __launch_bounds__(256) void k_qt_nodes(QtDev a) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < a.n; p += gridDim.x * blockDim.x) {
    const int g = qt_graph(a, p);
    const int gs = a.goff[g], ge = a.goff[g + 1];
    int lmin, lmax;
    qt_levels(a, p, gs, ge, lmin, lmax);
    if (lmin < 0) continue;
    const unsigned long long c = a.w.code[p];
    const int b0 = a.w.base[p];
    const double sx = a.w.px[p], sy = a.w.py[p];
    int lo_hint = p + 1;
    for (int l = lmax; l >= lmin; --l) {  // deepest first: ends only grow going up
      int e;
      if (l == 0) {
        e = ge;
      } else {
        const int sh = 2 * (kQtLevels - l);
        const unsigned long long last = sh >= 64 ? ~0ull : (c | ((1ull << sh) - 1ull));
        // first q >= lo_hint with code[q] > last (ge if none): gallop from
        // lo_hint (most nodes are small), then bisect the last stride
        int lo = lo_hint, hi = lo_hint, stride = 1;
        while (hi < ge && a.w.code[hi] <= last) {
          lo = hi + 1;
          hi = lo + stride;
          stride <<= 1;
        }
        hi = min(hi, ge);
        while (lo < hi) {
          const int m = (lo + hi) >> 1;
          if (a.w.code[m] > last) hi = m; else lo = m + 1;
        }
        e = lo;
      }
      lo_hint = e;
      const int idx = b0 + (l - lmin);
      const int cnt = e - p;
      QtNode nd;
      nd.b = make_int4(p, cnt, a.w.base[e], l);
      nd.c = make_double2((a.w.px[e] - sx) / cnt, (a.w.py[e] - sy) / cnt);
      a.w.nodes[idx] = nd;
    }
  }
}

struct QtAcc {
  float z = 0.f, rx = 0.f, ry = 0.f, ex = 0.f, ey = 0.f, ln = 0.f;
  __device__ __forceinline__ void add(float dx, float dy, float c, float eps, int terms) {
    const float r2 = dx * dx + dy * dy;
    if (terms & QT_REP) {
      const float q = 1.f / (1.f + r2);
      z += c * q;
      const float q2 = c * q * q;
      rx += q2 * dx;
      ry += q2 * dy;
    }
    if (terms & QT_ENT) {
      const float u = c / (eps + r2);
      ex += u * dx;
      ey += u * dy;
    }
    if (terms & QT_LN) ln += c * logf(eps + r2);
  }
};

__global__ __launch_bounds__(256) void k_qt_traverse(QtDev a, double th2, float eps, int terms,
                                                     float4* rep_ent, float* zi, float* lnv) {
  for (int sp = blockIdx.x * blockDim.x + threadIdx.x; sp < a.n; sp += gridDim.x * blockDim.x) {
    const int g = qt_graph(a, sp);
    const int end = a.w.base[a.goff[g + 1]];
    const double side = a.w.gp[g].side;
    const float2 xi = a.w.xs[sp];
    QtAcc acc;
    int node = a.w.base[a.goff[g]];
    while (node < end) {
      // the whole record at once: the centre is not needed for a leaf, but
      // loading it with the rest costs no extra round trip (the empty asm
      // takes its registers, so both halves are in flight together)
      const int4* rp = reinterpret_cast<const int4*>(a.w.nodes + node);
      const int4 b = rp[0];
      const int4 h = rp[1];
      asm volatile("" ::"v"(h.x), "v"(h.y), "v"(h.z), "v"(h.w));
      if (b.y == 1 || b.w == kQtLevels) {  // leaf: its points one by one
        for (int q = b.x; q < b.x + b.y; ++q) {
          if (q == sp) continue;
          const float2 xq = a.w.xs[q];
          acc.add(xi.x - xq.x, xi.y - xq.y, 1.f, eps, terms);
        }
        node = b.z;
        continue;
      }
      const double2 cm = make_double2(__hiloint2double(h.y, h.x), __hiloint2double(h.w, h.z));
      const double dx = (double)xi.x - cm.x, dy = (double)xi.y - cm.y;
      const double wd = ldexp(side, -b.w);
      if (wd * wd < th2 * (dx * dx + dy * dy)) {
        acc.add((float)dx, (float)dy, (float)b.y, eps, terms);
        node = b.z;
      } else {
        ++node;
      }
    }
    const int v = (int)a.w.val[sp];
    float2* re = reinterpret_cast<float2*>(rep_ent) + 2 * (size_t)v;
    if (terms & QT_REP) {
      re[0] = make_float2(acc.rx, acc.ry);
      a.w.zv[v] = acc.z;
      if (zi) zi[v] = acc.z;
    }
    if (terms & QT_ENT) re[1] = make_float2(acc.ex, acc.ey);
    // as the interpolation does: the self term ln(eps) included, 0 for a one-vertex graph
    if (terms & QT_LN) lnv[v] = a.goff[g + 1] - a.goff[g] == 1 ? 0.f : acc.ln + logf(eps);
  }
}

// Z per chunk in FP64 (fixed order), then per graph over its chunks in order.
__global__ __launch_bounds__(256) void k_qt_zchunks(QtDev a, const int* cs, const int* ce, double* zpart) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int v = cs[c] + threadIdx.x; v < ce[c]; v += blockDim.x) s += (double)a.w.zv[v];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) zpart[c] = red[0];
}

// One block per graph: its chunk sums in a fixed order (block-strided, then a
// tree reduction).
__global__ __launch_bounds__(256) void k_qt_zgraphs(const GraphInfo* gi, const double* zpart, double* zg,
                                                    double* Z_out) {
  __shared__ double red[256];
  const int g = blockIdx.x;
  double z = 0.0;
  for (int c = gi[g].chunk_begin + threadIdx.x; c < gi[g].chunk_end; c += blockDim.x) z += zpart[c];
  red[threadIdx.x] = z;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    zg[g] = red[0];
    if (Z_out) Z_out[g] = red[0];
  }
}

template <typename T>
int qt_alloc(T** p, size_t count, const char* what) {
  if (count == 0) count = 1;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(e == hipErrorOutOfMemory ? TSNET_ENOMEM : TSNET_EHIP,
                std::string("hipMalloc (quadtree ") + what + "): " + hipGetErrorString(e));
  }
  return TSNET_OK;
}

int ensure_quadtree(Problem& P) {
  if (P.qt) return TSNET_OK;
  // each sorted position starts at most kQtLevels + 1 nodes; node indices are int
  if ((int64_t)(kQtLevels + 1) * P.n + 1 > INT_MAX)
    return fail(TSNET_EINVAL, "quadtree terms need n <= " + std::to_string((INT_MAX - 1) / (kQtLevels + 1)));
  QuadWs* w = new (std::nothrow) QuadWs;
  if (!w) return fail(TSNET_ENOMEM, "host allocation failed");
  P.qt = w;
  const int n = P.n;
  w->n = n;
  w->G = P.G;
  w->max_nodes = (kQtLevels + 1) * n + 1;
  while ((1 << w->gbits) < P.G) ++w->gbits;
  const int rtiles = (n + kRadixTile - 1) / kRadixTile;
  const int64_t rh = (int64_t)256 * rtiles;
  int rc;
  if ((rc = qt_alloc(&w->gp, P.G, "params")) || (rc = qt_alloc(&w->part, P.num_chunks, "boxes")) ||
      (rc = qt_alloc(&w->key, n, "sort")) || (rc = qt_alloc(&w->val, n, "sort")) ||
      (rc = qt_alloc(&w->kt, n, "sort")) || (rc = qt_alloc(&w->vt, n, "sort")) ||
      (rc = qt_alloc(&w->rhist, rh + 1, "sort")) ||
      (rc = qt_alloc(&w->rtsum, (rh + kTileScan) / kTileScan + 1, "sort")) ||
      (rc = qt_alloc(&w->code, n, "codes")) || (rc = qt_alloc(&w->xs, n, "points")) ||
      (rc = qt_alloc(&w->px, (size_t)n + 1, "sums")) || (rc = qt_alloc(&w->py, (size_t)n + 1, "sums")) ||
      (rc = qt_alloc(&w->dtsum, (size_t)n / kTileScan + 2, "sums")) ||
      (rc = qt_alloc(&w->base, (size_t)n + 1, "nodes")) ||
      (rc = qt_alloc(&w->itsum, (size_t)n / kTileScan + 2, "nodes")) ||
      (rc = qt_alloc(&w->nodes, (size_t)w->max_nodes, "nodes")) || (rc = qt_alloc(&w->zv, n, "z"))) {
    free_quadtree(P);
    return rc;
  }
  return TSNET_OK;
}

}  // namespace

void free_quadtree(Problem& P) {
  QuadWs* w = P.qt;
  if (!w) return;
  void* ptrs[] = {w->gp, w->part, w->key, w->val, w->kt, w->vt, w->rhist, w->rtsum, w->code,
                  w->xs, w->px, w->py, w->dtsum, w->base, w->itsum, w->nodes, w->zv};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  delete w;
  P.qt = nullptr;
}

#define QT_LAUNCH(expr)                                                                  \
  do {                                                                                   \
    expr;                                                                                \
    hipError_t e_ = hipGetLastError();                                                   \
    if (e_ != hipSuccess) return fail(TSNET_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

int run_quadtree(Problem& P, const float2* X, double theta, float eps, int terms, int with_zi,
                 double* Z_out, hipStream_t s) {
  int rc = ensure_quadtree(P);
  if (rc) return rc;
  QtDev a;
  a.X = X;
  a.n = P.n;
  a.G = P.G;
  a.goff = P.goff_d;
  a.w = *P.qt;
  const int n = P.n;
  const int vb = (int)std::max<int64_t>(1, std::min<int64_t>(8192, (n + 255) / 256));
  QT_LAUNCH(hipLaunchKernelGGL(k_qt_bbox, dim3(P.num_chunks), dim3(256), 0, s, a, P.chunk_start, P.chunk_end));
  QT_LAUNCH(hipLaunchKernelGGL(k_qt_plan, dim3(P.G), dim3(256), 0, s, a, P.ginfo));
  QT_LAUNCH(hipLaunchKernelGGL(k_qt_codes, dim3(vb), dim3(256), 0, s, a));
  hipError_t e = radix_sort(a.w.key, a.w.val, a.w.kt, a.w.vt, n, 32, a.w.rhist, a.w.rtsum, s);
  if (e != hipSuccess) return fail(TSNET_EHIP, std::string("quadtree sort: ") + hipGetErrorString(e));
  QT_LAUNCH(hipLaunchKernelGGL(k_qt_high_keys, dim3(vb), dim3(256), 0, s, a));
  e = radix_sort(a.w.key, a.w.val, a.w.kt, a.w.vt, n, 32, a.w.rhist, a.w.rtsum, s);
  if (e != hipSuccess) return fail(TSNET_EHIP, std::string("quadtree sort: ") + hipGetErrorString(e));
  if (P.G > 1) {
    QT_LAUNCH(hipLaunchKernelGGL(k_qt_graph_keys, dim3(vb), dim3(256), 0, s, a));
    e = radix_sort(a.w.key, a.w.val, a.w.kt, a.w.vt, n, a.w.gbits, a.w.rhist, a.w.rtsum, s);
    if (e != hipSuccess) return fail(TSNET_EHIP, std::string("quadtree sort: ") + hipGetErrorString(e));
  }
  QT_LAUNCH(hipLaunchKernelGGL(k_qt_sorted, dim3(vb), dim3(256), 0, s, a));
  e = exclusive_scan<double>(a.w.px, n, a.w.px, a.w.dtsum, s);
  if (e == hipSuccess) e = exclusive_scan<double>(a.w.py, n, a.w.py, a.w.dtsum, s);
  QT_LAUNCH(hipLaunchKernelGGL(k_qt_count, dim3(vb), dim3(256), 0, s, a));
  if (e == hipSuccess) e = exclusive_scan<int>(a.w.base, n, a.w.base, a.w.itsum, s);
  if (e != hipSuccess) return fail(TSNET_EHIP, std::string("quadtree scan: ") + hipGetErrorString(e));
  QT_LAUNCH(hipLaunchKernelGGL(k_qt_nodes, dim3(vb), dim3(256), 0, s, a));
  QT_LAUNCH(hipLaunchKernelGGL(k_qt_traverse, dim3(vb), dim3(256), 0, s, a, theta * theta, eps, terms,
                               P.rep_ent, with_zi ? P.zi : nullptr, P.lnv));
  if (terms & QT_REP) {
    QT_LAUNCH(hipLaunchKernelGGL(k_qt_zchunks, dim3(P.num_chunks), dim3(256), 0, s, a, P.chunk_start,
                                 P.chunk_end, P.zpart));
    QT_LAUNCH(hipLaunchKernelGGL(k_qt_zgraphs, dim3(P.G), dim3(256), 0, s, P.ginfo, P.zpart, P.zg, Z_out));
  }
  return TSNET_OK;
}

}  // namespace tsnet
