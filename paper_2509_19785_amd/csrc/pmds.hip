// Pivot MDS starting layout of a graph batch (Algorithms 1-3 start from it,
// as tsNET* does, Sec. 2.1 and Sec. 4.1; the method is the eigensolver of
// Brandes and Pich, Graph Drawing 2006). The paper gives no settings; these
// readings are the project's. Per graph g (vertices a..b-1, n_g of them):
//
//  1. k_g = min(pivots, n_g) pivots: the first is a + (mix64(seed ^ g) mod n_g)
//     (SplitMix64 finaliser); each further one maximises the hop distance to
//     the nearest pivot so far (unreachable = infinitely far), ties to the
//     smallest id. All graphs of the batch search from their j-th pivot in the
//     same level-synchronous BFS (frontier queues, one wave per frontier
//     vertex; the host reads the frontier size after each level).
//  2. D[j][v] = hop distance; a pair without a path takes 1 + the largest
//     finite distance of the graph's searches.
//  3. S = D^2 is double-centred, C_vj = -1/2 (S_vj - r_v - c_j + m), from exact
//     64-bit integer row and column sums of S.
//  4. The Gram matrix C^T C (k_g x k_g) in FP64: per chunk of 2048 vertices,
//     then per graph in chunk order (reproducible). Its two leading
//     eigenvectors come from a cyclic Jacobi solve on the host, each signed so
//     that sum_j (j + 1) e_j > 0 over the pivot order (by the entry of largest
//     magnitude if that sum is exactly 0).
//  5. X_v = (C_v . e1, C_v . e2) * scale / sqrt(lambda1 / n_g): the first axis
//     then has standard deviation `scale` (C is centred, so sum_v (C_v.e1)^2 =
//     lambda1). Fewer than two pivots or lambda1 = 0 give zeros.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <string>
#include <vector>

#include "dev_util.h"
#include "tsnet_internal.h"

namespace tsnet {

namespace {

typedef unsigned long long u64;
constexpr int kPmdsChunk = 2048;  // vertices per chunk of the sums and the Gram matrix
constexpr int kPmdsMaxPivots = 128;
constexpr int kGramStage = 32;    // vertices staged in LDS per round of the Gram kernel

__device__ __forceinline__ u64 pm_mix64(u64 z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct PmdsDev {
  const int64_t* indptr;
  const int* indices;
  int n, G, kmax;
  const int* goff;     // [G+1]
  const int* kg;       // [G] pivots per graph
  int* piv;            // [G][kmax]
  int* dist;           // [n] current search
  int* mind;           // [n] distance to the nearest pivot so far (INT_MAX: none reached)
  int* D;              // [kmax][n]
  u64* best;           // [G] next-pivot key
  int* maxd;           // [G] largest finite distance
  long long* rowsum;   // [n] sum_j D^2
  long long* colsum;   // [G][kmax] sum_v D^2
};

__device__ __forceinline__ int graph_of_v(const PmdsDev& a, int v) {
  return a.G == 1 ? 0 : graph_of(a.goff, a.G, v);
}

__global__ __launch_bounds__(256) void k_pmds_init(PmdsDev a, u64 seed) {
  const int t0 = blockIdx.x * blockDim.x + threadIdx.x, nt = gridDim.x * blockDim.x;
  for (int v = t0; v < a.n; v += nt) {
    a.mind[v] = INT_MAX;
    a.rowsum[v] = 0;
  }
  for (int g = t0; g < a.G; g += nt) {
    const int lo = a.goff[g], ng = a.goff[g + 1] - lo;
    for (int j = 0; j < a.kmax; ++j) {
      a.piv[(size_t)g * a.kmax + j] = -1;
      a.colsum[(size_t)g * a.kmax + j] = 0;
    }
    a.piv[(size_t)g * a.kmax] = lo + (int)(pm_mix64(seed ^ (u64)g) % (u64)ng);
    a.best[g] = 0;
    a.maxd[g] = 0;
  }
}

// Start of search j: every distance unknown, the j-th pivot of each graph
// (if it has one) at distance 0 in the first frontier; cur[g] = -1 otherwise.
__global__ __launch_bounds__(256) void k_pmds_sources(PmdsDev a, int j, int* cur) {
  const int t0 = blockIdx.x * blockDim.x + threadIdx.x, nt = gridDim.x * blockDim.x;
  for (int v = t0; v < a.n; v += nt) a.dist[v] = -1;
  for (int g = t0; g < a.G; g += nt) cur[g] = j < a.kg[g] ? a.piv[(size_t)g * a.kmax + j] : -1;
}

__global__ void k_pmds_mark_sources(PmdsDev a, const int* cur) {
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < a.G; g += gridDim.x * blockDim.x)
    if (cur[g] >= 0) a.dist[cur[g]] = 0;
}

// One BFS level: a wave per frontier vertex, lanes over its neighbours; a
// vertex joins the next frontier once (compare-and-swap on its distance).
__global__ __launch_bounds__(256) void k_pmds_expand(PmdsDev a, const int* cur, int count,
                                                     int level, int* next, int* next_count) {
  const int lane = lane_id();
  const u64 below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
  const int nw = gridDim.x * (blockDim.x / kWave);
  for (int f = blockIdx.x * (blockDim.x / kWave) + wave_id(); f < count; f += nw) {
    const int v = cur[f];  // the same for the whole wave
    if (v < 0) continue;
    const int64_t e1 = a.indptr[v + 1];
    for (int64_t e0 = a.indptr[v]; e0 < e1; e0 += kWave) {
      int u = -1;
      if (e0 + lane < e1) {
        u = a.indices[e0 + lane];
        if (a.dist[u] != -1 || atomicCAS(&a.dist[u], -1, level + 1) != -1) u = -1;
      }
      const u64 m = __ballot(u >= 0);
      if (m) {
        int base = 0;
        if (lane == 0) base = atomicAdd(next_count, __popcll(m));
        base = __shfl(base, 0, kWave);
        if (u >= 0) next[base + __popcll(m & below)] = u;
      }
    }
  }
}

// After search j: keep the distances, update the distance to the nearest
// pivot, and propose each graph's next pivot (largest distance, smallest id:
// the key packs (distance, ~local id) for a 64-bit maximum) and its largest
// finite distance. A wave whose vertices share one graph reduces first.
__global__ __launch_bounds__(256) void k_pmds_record(PmdsDev a, int j) {
  const int n = a.n;
  for (int base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
    const int v = base + threadIdx.x;
    const bool in = v < n;
    const int g = in ? graph_of_v(a, v) : -1;
    u64 key = 0;
    int dmax = 0;
    const bool act = in && j < a.kg[g];
    if (act) {
      const int d = a.dist[v];
      a.D[(size_t)j * n + v] = d;
      int md = a.mind[v];
      if (d >= 0 && d < md) md = d;
      a.mind[v] = md;
      dmax = d > 0 ? d : 0;
      const unsigned local = (unsigned)(v - a.goff[g]);
      key = ((u64)(unsigned)md << 32) | (u64)(0xFFFFFFFFu - local);
    }
    const int g0 = __shfl(g, 0, kWave);
    const bool uniform = __all(!in || g == g0) && g0 >= 0;
    if (uniform) {
      u64 k2 = key;
      int d2 = dmax;
#pragma unroll
      for (int o = kWave / 2; o > 0; o >>= 1) {
        const u64 ok = __shfl_xor(k2, o, kWave);
        const int od = __shfl_xor(d2, o, kWave);
        k2 = ok > k2 ? ok : k2;
        d2 = od > d2 ? od : d2;
      }
      if (lane_id() == 0 && j < a.kg[g0]) {
        atomicMax(&a.best[g0], k2);
        atomicMax(&a.maxd[g0], d2);
      }
    } else if (act) {
      atomicMax(&a.best[g], key);
      atomicMax(&a.maxd[g], dmax);
    }
  }
}

__global__ void k_pmds_next(PmdsDev a, int j) {
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < a.G; g += gridDim.x * blockDim.x) {
    if (j + 1 < a.kg[g]) {
      const unsigned local = 0xFFFFFFFFu - (unsigned)(a.best[g] & 0xFFFFFFFFull);
      a.piv[(size_t)g * a.kmax + j + 1] = a.goff[g] + (int)local;
    }
    a.best[g] = 0;
  }
}

// Unreachable pairs take 1 + the graph's largest finite distance; exact
// integer sums of D^2 per vertex and, per chunk (one graph), per pivot.
__global__ __launch_bounds__(256) void k_pmds_sums(PmdsDev a, const int* chunk_graph,
                                                   const int* chunk_start, const int* chunk_end) {
  __shared__ long long red[256 / kWave];
  const int c = blockIdx.x, g = chunk_graph[c];
  const int v0 = chunk_start[c], v1 = chunk_end[c], k = a.kg[g], n = a.n;
  const int far = a.maxd[g] + 1;
  for (int v = v0 + threadIdx.x; v < v1; v += blockDim.x) {
    long long rs = 0;
    for (int j = 0; j < k; ++j) {
      int d = a.D[(size_t)j * n + v];
      if (d < 0) {
        d = far;
        a.D[(size_t)j * n + v] = d;
      }
      rs += (long long)d * d;
    }
    a.rowsum[v] = rs;
  }
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    long long cs = 0;
    for (int v = v0 + threadIdx.x; v < v1; v += blockDim.x) {
      const long long d = a.D[(size_t)j * n + v];
      cs += d * d;
    }
    cs = wave_sum(cs);
    if (lane_id() == 0) red[wave_id()] = cs;
    __syncthreads();
    if (threadIdx.x == 0) {
      long long t = 0;
      for (int w = 0; w < (int)(blockDim.x / kWave); ++w) t += red[w];
      atomicAdd(reinterpret_cast<unsigned long long*>(&a.colsum[(size_t)g * a.kmax + j]),
                (unsigned long long)t);
    }
    __syncthreads();
  }
}

// C_vj of the double-centred squared distances.
__device__ __forceinline__ double c_entry(const PmdsDev& a, int v, int g, int j, int k, double ng) {
  const long long d = a.D[(size_t)j * a.n + v];
  const double s = (double)(d * d);
  const double r = (double)a.rowsum[v] / k;
  const double cj = (double)a.colsum[(size_t)g * a.kmax + j] / ng;
  return s - r - cj;  // the grand mean and the factor -1/2 are added by the caller
}

// Partial Gram matrix of one chunk: part[c][p][q] = sum_v C_vp C_vq, vertices
// staged kGramStage at a time in LDS. The 256 threads form a 16 x 16 grid;
// thread (tx, ty) owns entries p = tx + 16 a, q = ty + 16 b, a, b < KT.
template <int KT>
__global__ __launch_bounds__(256) void k_pmds_gram(PmdsDev a, const int* chunk_graph,
                                                   const int* chunk_start, const int* chunk_end,
                                                   const double* gmean, double* part) {
  extern __shared__ double cst[];  // [kGramStage][kmax]
  const int c = blockIdx.x, g = chunk_graph[c];
  const int v0 = chunk_start[c], v1 = chunk_end[c], k = a.kg[g];
  const double ng = (double)(a.goff[g + 1] - a.goff[g]), m = gmean[g];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[KT][KT];
#pragma unroll
  for (int i = 0; i < KT; ++i)
#pragma unroll
    for (int l = 0; l < KT; ++l) acc[i][l] = 0.0;
  for (int s0 = v0; s0 < v1; s0 += kGramStage) {
    const int ns = min(kGramStage, v1 - s0);
    for (int t = threadIdx.x; t < ns * k; t += blockDim.x) {
      const int vi = t / k, j = t - vi * k;
      cst[vi * a.kmax + j] = -0.5 * (c_entry(a, s0 + vi, g, j, k, ng) + m);
    }
    __syncthreads();
    for (int vi = 0; vi < ns; ++vi) {
      double cp[KT], cq[KT];
#pragma unroll
      for (int i = 0; i < KT; ++i) {
        const int p = tx + 16 * i, q = ty + 16 * i;
        cp[i] = p < k ? cst[vi * a.kmax + p] : 0.0;
        cq[i] = q < k ? cst[vi * a.kmax + q] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < KT; ++i)
#pragma unroll
        for (int l = 0; l < KT; ++l) acc[i][l] += cp[i] * cq[l];
    }
    __syncthreads();
  }
  double* out = part + (size_t)c * a.kmax * a.kmax;
#pragma unroll
  for (int i = 0; i < KT; ++i)
#pragma unroll
    for (int l = 0; l < KT; ++l) {
      const int p = tx + 16 * i, q = ty + 16 * l;
      if (p < k && q < k) out[p * a.kmax + q] = acc[i][l];
    }
}

// Per graph: the Gram matrix, chunk partials added in chunk order.
__global__ __launch_bounds__(256) void k_pmds_gram_sum(PmdsDev a, const int* gchunk_begin,
                                                       const int* gchunk_end, const double* part,
                                                       double* gram) {
  const int g = blockIdx.y, k = a.kg[g], kk = a.kmax * a.kmax;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < k * k; e += gridDim.x * blockDim.x) {
    const int p = e / k, q = e - p * k;
    double s = 0.0;
    for (int c = gchunk_begin[g]; c < gchunk_end[g]; ++c) s += part[(size_t)c * kk + p * a.kmax + q];
    gram[(size_t)g * kk + p * a.kmax + q] = s;
  }
}

// X_v = (C_v . w1, C_v . w2), w the scaled eigenvectors of the vertex's graph.
__global__ __launch_bounds__(256) void k_pmds_project(PmdsDev a, const double* gmean,
                                                      const double* w, float2* X) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += gridDim.x * blockDim.x) {
    const int g = graph_of_v(a, v), k = a.kg[g];
    const double ng = (double)(a.goff[g + 1] - a.goff[g]), m = gmean[g];
    const double* w1 = w + (size_t)g * 2 * a.kmax;
    const double* w2 = w1 + a.kmax;
    double y1 = 0.0, y2 = 0.0;
    for (int j = 0; j < k; ++j) {
      const double cv = -0.5 * (c_entry(a, v, g, j, k, ng) + m);
      y1 += cv * w1[j];
      y2 += cv * w2[j];
    }
    X[v] = make_float2((float)y1, (float)y2);
  }
}

// Cyclic Jacobi eigen-decomposition of a symmetric k x k matrix (row-major,
// destroyed); eigenvalues in w, eigenvectors in the columns of V.
void jacobi_eigen(std::vector<double>& A, int k, std::vector<double>& w, std::vector<double>& V) {
  V.assign((size_t)k * k, 0.0);
  for (int i = 0; i < k; ++i) V[(size_t)i * k + i] = 1.0;
  double total = 0.0;
  for (double x : A) total += x * x;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < k; ++p)
      for (int q = p + 1; q < k; ++q) off += A[(size_t)p * k + q] * A[(size_t)p * k + q];
    if (off <= 1e-30 * total || off == 0.0) break;
    for (int p = 0; p < k; ++p)
      for (int q = p + 1; q < k; ++q) {
        const double apq = A[(size_t)p * k + q];
        if (apq == 0.0) continue;
        const double app = A[(size_t)p * k + p], aqq = A[(size_t)q * k + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int r = 0; r < k; ++r) {  // A <- J^T A J on rows/columns p, q
          const double arp = A[(size_t)r * k + p], arq = A[(size_t)r * k + q];
          A[(size_t)r * k + p] = cs * arp - sn * arq;
          A[(size_t)r * k + q] = sn * arp + cs * arq;
        }
        for (int r = 0; r < k; ++r) {
          const double apr = A[(size_t)p * k + r], aqr = A[(size_t)q * k + r];
          A[(size_t)p * k + r] = cs * apr - sn * aqr;
          A[(size_t)q * k + r] = sn * apr + cs * aqr;
        }
        for (int r = 0; r < k; ++r) {
          const double vrp = V[(size_t)r * k + p], vrq = V[(size_t)r * k + q];
          V[(size_t)r * k + p] = cs * vrp - sn * vrq;
          V[(size_t)r * k + q] = sn * vrp + cs * vrq;
        }
      }
  }
  w.resize(k);
  for (int i = 0; i < k; ++i) w[i] = A[(size_t)i * k + i];
}

template <typename T>
int pm_alloc(std::vector<void*>& owned, T** p, size_t count) {
  if (count == 0) count = 1;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(e == hipErrorOutOfMemory ? TSNET_ENOMEM : TSNET_EHIP,
                std::string("hipMalloc in tsnet_pmds: ") + hipGetErrorString(e));
  }
  owned.push_back(*p);
  return TSNET_OK;
}

struct Owned {
  std::vector<void*> p;
  ~Owned() {
    for (void* q : p) (void)hipFree(q);
  }
};

#define PMDS_HIP(expr)                                                                  \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(TSNET_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

}  // namespace

int run_pmds(const int64_t* indptr, const int* indices, int n, const std::vector<int>& goff,
             int pivots, uint64_t seed, double scale, float* X, int* pivots_out, double* eig_host,
             int* levels_host, hipStream_t s) {
  const int G = (int)goff.size() - 1;
  std::vector<int> kg(G);
  int kmax = 0;
  for (int g = 0; g < G; ++g) {
    kg[g] = std::min(pivots, goff[g + 1] - goff[g]);
    kmax = std::max(kmax, kg[g]);
  }
  // chunks of at most kPmdsChunk vertices, never across graphs
  std::vector<int> cg, cs, ce, gb(G), ge(G);
  for (int g = 0; g < G; ++g) {
    gb[g] = (int)cg.size();
    for (int v = goff[g]; v < goff[g + 1]; v += kPmdsChunk) {
      cg.push_back(g);
      cs.push_back(v);
      ce.push_back(std::min(goff[g + 1], v + kPmdsChunk));
    }
    ge[g] = (int)cg.size();
  }
  const int nc = (int)cg.size();
  Owned own;
  PmdsDev a;
  a.indptr = indptr;
  a.indices = indices;
  a.n = n;
  a.G = G;
  a.kmax = kmax;
  int *goff_d, *kg_d, *piv, *dist, *mind, *D, *maxd, *cur, *nxt, *cnt, *chg, *chs, *che, *gbd, *ged;
  u64* best;
  long long *rowsum, *colsum;
  double *gmean, *part, *gram, *wd;
  int rc;
  if ((rc = pm_alloc(own.p, &goff_d, G + 1)) || (rc = pm_alloc(own.p, &kg_d, G)) ||
      (rc = pm_alloc(own.p, &piv, (size_t)G * kmax)) || (rc = pm_alloc(own.p, &dist, n)) ||
      (rc = pm_alloc(own.p, &mind, n)) || (rc = pm_alloc(own.p, &D, (size_t)kmax * n)) ||
      (rc = pm_alloc(own.p, &maxd, G)) || (rc = pm_alloc(own.p, &best, G)) ||
      (rc = pm_alloc(own.p, &cur, std::max(n, G))) || (rc = pm_alloc(own.p, &nxt, std::max(n, G))) ||
      (rc = pm_alloc(own.p, &cnt, 1)) || (rc = pm_alloc(own.p, &rowsum, n)) ||
      (rc = pm_alloc(own.p, &colsum, (size_t)G * kmax)) || (rc = pm_alloc(own.p, &chg, nc)) ||
      (rc = pm_alloc(own.p, &chs, nc)) || (rc = pm_alloc(own.p, &che, nc)) ||
      (rc = pm_alloc(own.p, &gbd, G)) || (rc = pm_alloc(own.p, &ged, G)) ||
      (rc = pm_alloc(own.p, &gmean, G)) || (rc = pm_alloc(own.p, &part, (size_t)nc * kmax * kmax)) ||
      (rc = pm_alloc(own.p, &gram, (size_t)G * kmax * kmax)) ||
      (rc = pm_alloc(own.p, &wd, (size_t)G * 2 * kmax)))
    return rc;
  PMDS_HIP(hipMemcpyAsync(goff_d, goff.data(), sizeof(int) * (G + 1), hipMemcpyHostToDevice, s));
  PMDS_HIP(hipMemcpyAsync(kg_d, kg.data(), sizeof(int) * G, hipMemcpyHostToDevice, s));
  PMDS_HIP(hipMemcpyAsync(chg, cg.data(), sizeof(int) * nc, hipMemcpyHostToDevice, s));
  PMDS_HIP(hipMemcpyAsync(chs, cs.data(), sizeof(int) * nc, hipMemcpyHostToDevice, s));
  PMDS_HIP(hipMemcpyAsync(che, ce.data(), sizeof(int) * nc, hipMemcpyHostToDevice, s));
  PMDS_HIP(hipMemcpyAsync(gbd, gb.data(), sizeof(int) * G, hipMemcpyHostToDevice, s));
  PMDS_HIP(hipMemcpyAsync(ged, ge.data(), sizeof(int) * G, hipMemcpyHostToDevice, s));
  a.goff = goff_d;
  a.kg = kg_d;
  a.piv = piv;
  a.dist = dist;
  a.mind = mind;
  a.D = D;
  a.best = best;
  a.maxd = maxd;
  a.rowsum = rowsum;
  a.colsum = colsum;
  const int vb = std::min(8192, n / 256 + 1), gbk = std::min(1024, G / 256 + 1);
  hipLaunchKernelGGL(k_pmds_init, dim3(std::max(vb, gbk)), dim3(256), 0, s, a, (u64)seed);
  PMDS_HIP(hipGetLastError());
  long long levels = 0;
  for (int j = 0; j < kmax; ++j) {
    hipLaunchKernelGGL(k_pmds_sources, dim3(std::max(vb, gbk)), dim3(256), 0, s, a, j, cur);
    hipLaunchKernelGGL(k_pmds_mark_sources, dim3(gbk), dim3(256), 0, s, a, cur);
    PMDS_HIP(hipGetLastError());
    int count = G, level = 0;
    int *c0 = cur, *c1 = nxt;
    while (count > 0) {
      PMDS_HIP(hipMemsetAsync(cnt, 0, sizeof(int), s));
      const int blocks = std::min(16384, (count + 3) / 4);
      hipLaunchKernelGGL(k_pmds_expand, dim3(blocks), dim3(256), 0, s, a, c0, count, level, c1, cnt);
      PMDS_HIP(hipGetLastError());
      PMDS_HIP(hipMemcpyAsync(&count, cnt, sizeof(int), hipMemcpyDeviceToHost, s));
      PMDS_HIP(hipStreamSynchronize(s));
      if (count < 0 || count > n) return fail(TSNET_EHIP, "tsnet_pmds: bad frontier size");
      std::swap(c0, c1);
      ++level;
      ++levels;
    }
    hipLaunchKernelGGL(k_pmds_record, dim3(vb), dim3(256), 0, s, a, j);
    hipLaunchKernelGGL(k_pmds_next, dim3(gbk), dim3(256), 0, s, a, j);
    PMDS_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_pmds_sums, dim3(nc), dim3(256), 0, s, a, chg, chs, che);
  PMDS_HIP(hipGetLastError());
  // grand means (exact integer totals)
  std::vector<long long> colsum_h((size_t)G * kmax);
  PMDS_HIP(hipMemcpyAsync(colsum_h.data(), colsum, sizeof(long long) * G * kmax,
                          hipMemcpyDeviceToHost, s));
  PMDS_HIP(hipStreamSynchronize(s));
  std::vector<double> gmean_h(G);
  for (int g = 0; g < G; ++g) {
    long long t = 0;
    for (int j = 0; j < kg[g]; ++j) t += colsum_h[(size_t)g * kmax + j];
    gmean_h[g] = (double)t / ((double)(goff[g + 1] - goff[g]) * kg[g]);
  }
  PMDS_HIP(hipMemcpyAsync(gmean, gmean_h.data(), sizeof(double) * G, hipMemcpyHostToDevice, s));
  const size_t lds = sizeof(double) * kGramStage * kmax;
  if (kmax <= 64)
    hipLaunchKernelGGL(k_pmds_gram<4>, dim3(nc), dim3(256), lds, s, a, chg, chs, che, gmean, part);
  else
    hipLaunchKernelGGL(k_pmds_gram<8>, dim3(nc), dim3(256), lds, s, a, chg, chs, che, gmean, part);
  PMDS_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_pmds_gram_sum, dim3(std::max(1, (kmax * kmax + 255) / 256), G), dim3(256), 0,
                     s, a, gbd, ged, part, gram);
  PMDS_HIP(hipGetLastError());
  std::vector<double> gram_h((size_t)G * kmax * kmax);
  PMDS_HIP(hipMemcpyAsync(gram_h.data(), gram, sizeof(double) * gram_h.size(),
                          hipMemcpyDeviceToHost, s));
  PMDS_HIP(hipStreamSynchronize(s));
  std::vector<double> w_h((size_t)G * 2 * kmax, 0.0);
  for (int g = 0; g < G; ++g) {
    const int k = kg[g];
    double l1 = 0.0, l2 = 0.0;
    if (k >= 2) {
      std::vector<double> A((size_t)k * k), wv, V;
      for (int p = 0; p < k; ++p)
        for (int q = 0; q < k; ++q) A[(size_t)p * k + q] = gram_h[(size_t)g * kmax * kmax + p * kmax + q];
      jacobi_eigen(A, k, wv, V);
      std::vector<int> ord(k);
      for (int i = 0; i < k; ++i) ord[i] = i;
      std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return wv[x] > wv[y]; });
      l1 = wv[ord[0]];
      l2 = wv[ord[1]];
      const double ng = (double)(goff[g + 1] - goff[g]);
      const double f = l1 > 0.0 ? scale / std::sqrt(l1 / ng) : 0.0;
      for (int ax = 0; ax < 2; ++ax) {
        const int col = ord[ax];
        double t = 0.0;
        for (int i = 0; i < k; ++i) t += (double)(i + 1) * V[(size_t)i * k + col];
        if (t == 0.0) {
          int imax = 0;
          for (int i = 1; i < k; ++i)
            if (std::fabs(V[(size_t)i * k + col]) > std::fabs(V[(size_t)imax * k + col])) imax = i;
          t = V[(size_t)imax * k + col];
        }
        const double sg = t >= 0.0 ? 1.0 : -1.0;
        for (int i = 0; i < k; ++i) w_h[(size_t)g * 2 * kmax + ax * kmax + i] = sg * f * V[(size_t)i * k + col];
      }
    }
    if (eig_host) {
      eig_host[2 * g] = l1;
      eig_host[2 * g + 1] = l2;
    }
  }
  PMDS_HIP(hipMemcpyAsync(wd, w_h.data(), sizeof(double) * w_h.size(), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_pmds_project, dim3(vb), dim3(256), 0, s, a, gmean, wd,
                     reinterpret_cast<float2*>(X));
  PMDS_HIP(hipGetLastError());
  if (pivots_out) {
    // [G][pivots] with -1 past k_g (kmax <= pivots)
    std::vector<int> ph((size_t)G * kmax), po((size_t)G * pivots, -1);
    PMDS_HIP(hipMemcpyAsync(ph.data(), piv, sizeof(int) * ph.size(), hipMemcpyDeviceToHost, s));
    PMDS_HIP(hipStreamSynchronize(s));
    for (int g = 0; g < G; ++g)
      for (int j = 0; j < kg[g]; ++j) po[(size_t)g * pivots + j] = ph[(size_t)g * kmax + j];
    PMDS_HIP(hipMemcpyAsync(pivots_out, po.data(), sizeof(int) * po.size(), hipMemcpyHostToDevice, s));
  }
  PMDS_HIP(hipStreamSynchronize(s));
  if (levels_host) *levels_host = (int)levels;
  return TSNET_OK;
}

}  // namespace tsnet
