// Attractive KL term (Eq. 6, first sum) over the sparse P, fused with the
// gradient assembly:
//   G_i = 4 l_kl (F_attr,i - F_rep,i / Z) + (l_c / n) X_i - (l_r / n^2) F_ent,i.
//
// One wave per row, lanes over the row's nonzeros (four per lane in flight),
// the loads of the wave's next rows issued ahead of time.
// Rows are visited longest first within each graph, graphs in order (an
// order fixed once per problem): the few very long rows of hub vertices
// start early instead of forming a tail, and in a batch the waves in flight
// gather x_j from one graph at a time (P is block-diagonal), so X stays in
// cache.
// The row sum is a fixed wave reduction, so results are reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <numeric>
#include <string>
#include <vector>

#include "dev_util.h"
#include "tsnet_internal.h"

namespace tsnet {

static int attract_grid(Problem& P);

int build_row_order(Problem& P) {
  std::vector<int64_t> rp(P.n + 1);
  hipError_t e = hipMemcpy(rp.data(), P.rowptr, sizeof(int64_t) * (P.n + 1), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(TSNET_EHIP, std::string("row order: ") + hipGetErrorString(e));
  std::vector<int> order(P.n);
  std::iota(order.begin(), order.end(), 0);
  for (int g = 0; g < P.G; ++g)
    std::stable_sort(order.begin() + P.goff[g], order.begin() + P.goff[g + 1], [&](int a, int b) {
      return rp[a + 1] - rp[a] > rp[b + 1] - rp[b];
    });
  if (hipMalloc(&P.row_order, sizeof(int) * P.n) != hipSuccess)
    return fail(TSNET_ENOMEM, "row order allocation");
  e = hipMemcpy(P.row_order, order.data(), sizeof(int) * P.n, hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(TSNET_EHIP, std::string("row order: ") + hipGetErrorString(e));
  return attract_grid(P);
}

struct AttrParams {
  float lkl4, lc, lr;
};

// Entries per lane loaded together in one round (a row of up to 256 entries
// takes one round trip for its columns and one for their x_j).
constexpr int kRowBatch = 4;

// Columns and values of the first kRowBatch * 64 entries of row [a, b), lane
// `lane` taking a + lane + 64 u. Indices are clamped into the row, or to entry
// 0 for an empty row (the arrays hold one element or more), so the loads are
// unconditional. Entries past b get weight 0 and column 0: what was read
// there may belong to no row (P with no entries holds one unset element).
__device__ __forceinline__ void row_batch(const int* __restrict__ col, const float* __restrict__ val,
                                          int a, int b, int lane, int (&j)[kRowBatch],
                                          float (&p)[kRowBatch]) {
#pragma unroll
  for (int u = 0; u < kRowBatch; ++u) {
    const int e = max(min(a + lane + u * kWave, b - 1), 0);
    j[u] = col[e];
    p[u] = val[e];
  }
#pragma unroll
  for (int u = 0; u < kRowBatch; ++u)
    if (a + lane + u * kWave >= b) {
      j[u] = 0;
      p[u] = 0.f;
    }
}

__device__ __forceinline__ void row_terms(float2 xi, const float2 (&xj)[kRowBatch],
                                          const float (&p)[kRowBatch], float& fx, float& fy) {
#pragma unroll
  for (int u = 0; u < kRowBatch; ++u) {
    const float dx = xi.x - xj[u].x, dy = xi.y - xj[u].y;
    const float w = p[u] * __builtin_amdgcn_rcpf(1.0f + dx * dx + dy * dy);
    fx += w * dx;
    fy += w * dy;
  }
}

// A wave takes rows t, t + S, t + 2S, ... of the row order (S waves in the
// grid) through a three-stage software pipeline, so that the chain of
// dependent loads of a row (row id -> row bounds -> columns -> x_j) is not
// waited out row by row: while the x_j of row t are gathered, the columns of
// row t + S, the bounds of row t + 2S and the id of row t + 3S are in flight.
// Rows past n are read at the clamped index n - 1 and never written. Entry
// offsets are 32-bit (P holds fewer than 2^31 entries); the weight uses the
// hardware reciprocal (1 ulp), as the tiled kernel does.
__global__ __launch_bounds__(256) void k_attract(
    const float2* __restrict__ X, const int64_t* __restrict__ rowptr, const int* __restrict__ col,
    const float* __restrict__ val, const int* __restrict__ order, int n,
    const int* __restrict__ vgraph, int G, const GraphInfo* __restrict__ gi,
    const double* __restrict__ zg, const float4* __restrict__ rep_ent, AttrParams ap, float2* Gout,
    float2* Fattr) {
  const int lane = lane_id();
  const int nwaves = blockDim.x / kWave;
  const int S = gridDim.x * nwaves;
  int t = blockIdx.x * nwaves + wave_id();
  if (t >= n) return;
  auto row_at = [&](int64_t q) { return order[q < n ? q : n - 1]; };
  // row t: bounds, x_i, graph and first batch
  int i0 = row_at(t);
  int a0 = (int)rowptr[i0], b0 = (int)rowptr[i0 + 1];
  float2 x0 = X[i0];
  int g0 = G == 1 ? 0 : vgraph[i0];
  int j0[kRowBatch];
  float p0[kRowBatch];
  row_batch(col, val, a0, b0, lane, j0, p0);
  // row t + S: bounds; row t + 2S: id
  int i1 = row_at((int64_t)t + S);
  int a1 = (int)rowptr[i1], b1 = (int)rowptr[i1 + 1];
  float2 x1 = X[i1];
  int g1 = G == 1 ? 0 : vgraph[i1];
  int i2 = row_at((int64_t)t + 2 * (int64_t)S);
  for (; t < n; t += S) {
    // row t: gathers and the terms of its assembly
    float2 xj[kRowBatch];
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u) xj[u] = X[j0[u]];
    const float4 re = rep_ent[i0];
    const double Z = zg[g0];
    const float inv_n = gi[g0].inv_n, inv_n2 = gi[g0].inv_n2;
    // the next rows' loads, in flight while row t is summed
    int j1[kRowBatch];
    float p1[kRowBatch];
    row_batch(col, val, a1, b1, lane, j1, p1);
    const int a2 = (int)rowptr[i2], b2 = (int)rowptr[i2 + 1];
    const float2 x2 = X[i2];
    const int g2 = G == 1 ? 0 : vgraph[i2];
    const int i3 = row_at((int64_t)t + 3 * (int64_t)S);

    float fx = 0.f, fy = 0.f;
    row_terms(x0, xj, p0, fx, fy);
    // entries past the first batch of a long row (not pipelined)
    for (int e0 = a0 + lane + kRowBatch * kWave; e0 < b0; e0 += kRowBatch * kWave) {
      int j[kRowBatch];
      float p[kRowBatch];
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u) {
        const int e = min(e0 + u * kWave, b0 - 1);
        j[u] = col[e];
        p[u] = val[e];
      }
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u)
        if (e0 + u * kWave >= b0) p[u] = 0.f;
      float2 xk[kRowBatch];
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u) xk[u] = X[j[u]];
      row_terms(x0, xk, p, fx, fy);
    }
    fx = wave_sum(fx);
    fy = wave_sum(fy);
    if (lane == 0) {
      const float inv_z = Z > 0.0 ? (float)(1.0 / Z) : 0.0f;
      const float2 r = make_float2(re.x, re.y), en = make_float2(re.z, re.w);
      const float cn = ap.lc * inv_n, rn = ap.lr * inv_n2;
      float2 o;
      o.x = ap.lkl4 * (fx - r.x * inv_z) + cn * x0.x - rn * en.x;
      o.y = ap.lkl4 * (fy - r.y * inv_z) + cn * x0.y - rn * en.y;
      Gout[i0] = o;
      if (Fattr) Fattr[i0] = make_float2(fx, fy);
    }
    i0 = i1;
    a0 = a1;
    b0 = b1;
    x0 = x1;
    g0 = g1;
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u) {
      j0[u] = j1[u];
      p0[u] = p1[u];
    }
    i1 = i2;
    a1 = a2;
    b1 = b2;
    x1 = x2;
    g1 = g2;
    i2 = i3;
  }
}

// The grid of the row attraction is what the device holds at once: its waves
// then sweep the row order together, so the x_j they gather belong to the
// rows of one or two graphs and stay in L2. A larger grid would start its
// later blocks at the head of the order while the first ones are near the
// end, and the waves in flight would gather from all of X.
static int attract_grid(Problem& P) {
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_attract),
                                                     256, 0);
  if (e != hipSuccess) return fail(TSNET_EHIP, std::string("attraction grid: ") + hipGetErrorString(e));
  P.attract_blocks = std::max(1, cus * per_cu);
  return TSNET_OK;
}

hipError_t launch_attract(Problem& P, const float2* X, const tsnet_params& prm, float2* G,
                          float2* F_attr, hipStream_t s) {
  AttrParams ap;
  ap.lkl4 = (float)(4.0 * prm.lambda_kl);
  ap.lc = (float)prm.lambda_c;
  ap.lr = (float)prm.lambda_r;
  int blocks = (P.n + 3) / 4;
  if (blocks > P.attract_blocks) blocks = P.attract_blocks;
  hipLaunchKernelGGL(k_attract, dim3(blocks), dim3(256), 0, s, X, P.rowptr, P.col, P.val,
                     P.row_order, P.n, P.vgraph, P.G, P.ginfo, P.zg, P.rep_ent, ap, G, F_attr);
  return hipGetLastError();
}

}  // namespace tsnet
