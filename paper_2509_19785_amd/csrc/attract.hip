// Attractive KL term (Eq. 6, first sum) over the sparse P, fused with the
// gradient assembly:
//   G_i = 4 l_kl (F_attr,i - F_rep,i / Z) + (l_c / n) X_i - (l_r / n^2) F_ent,i.
//
// One wave per row, lanes over the row's nonzeros (two per lane in flight).
// Rows are visited longest first (an order fixed once per problem), so the
// few very long rows of hub vertices start early instead of forming a tail.
// The row sum is a fixed wave reduction, so results are reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <numeric>
#include <string>
#include <vector>

#include "dev_util.h"
#include "tsnet_internal.h"

namespace tsnet {

int build_row_order(Problem& P) {
  std::vector<int64_t> rp(P.n + 1);
  hipError_t e = hipMemcpy(rp.data(), P.rowptr, sizeof(int64_t) * (P.n + 1), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(TSNET_EHIP, std::string("row order: ") + hipGetErrorString(e));
  std::vector<int> order(P.n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return rp[a + 1] - rp[a] > rp[b + 1] - rp[b];
  });
  if (hipMalloc(&P.row_order, sizeof(int) * P.n) != hipSuccess)
    return fail(TSNET_ENOMEM, "row order allocation");
  e = hipMemcpy(P.row_order, order.data(), sizeof(int) * P.n, hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(TSNET_EHIP, std::string("row order: ") + hipGetErrorString(e));
  return TSNET_OK;
}

struct AttrParams {
  float lkl4, lc, lr;
};

__global__ __launch_bounds__(256) void k_attract(
    const float2* __restrict__ X, const int64_t* __restrict__ rowptr, const int* __restrict__ col,
    const float* __restrict__ val, const int* __restrict__ order, int n,
    const int* __restrict__ goff, int G, const GraphInfo* __restrict__ gi,
    const double* __restrict__ zg, const float4* __restrict__ rep_ent, AttrParams ap, float2* Gout,
    float2* Fattr) {
  const int lane = lane_id();
  const int nwaves = blockDim.x / kWave;
  for (int t = blockIdx.x * nwaves + wave_id(); t < n; t += gridDim.x * nwaves) {
    const int i = order[t];
    const int64_t a = rowptr[i], b = rowptr[i + 1];
    const float2 xi = X[i];
    float fx = 0.f, fy = 0.f;
    int64_t e = a + lane;
    for (; e + kWave < b; e += 2 * kWave) {
      const int j0 = col[e], j1 = col[e + kWave];
      const float p0 = val[e], p1 = val[e + kWave];
      const float2 x0 = X[j0], x1 = X[j1];
      const float dx0 = xi.x - x0.x, dy0 = xi.y - x0.y;
      const float dx1 = xi.x - x1.x, dy1 = xi.y - x1.y;
      const float w0 = p0 / (1.0f + dx0 * dx0 + dy0 * dy0);
      const float w1 = p1 / (1.0f + dx1 * dx1 + dy1 * dy1);
      fx += w0 * dx0 + w1 * dx1;
      fy += w0 * dy0 + w1 * dy1;
    }
    if (e < b) {
      const int j = col[e];
      const float p = val[e];
      const float2 xj = X[j];
      const float dx = xi.x - xj.x, dy = xi.y - xj.y;
      const float w = p / (1.0f + dx * dx + dy * dy);
      fx += w * dx;
      fy += w * dy;
    }
    fx = wave_sum(fx);
    fy = wave_sum(fy);
    if (lane == 0) {
      const int g = G == 1 ? 0 : graph_of(goff, G, i);
      const double Z = zg[g];
      const float inv_z = Z > 0.0 ? (float)(1.0 / Z) : 0.0f;
      const float4 re = rep_ent[i];
      const float2 r = make_float2(re.x, re.y), en = make_float2(re.z, re.w);
      const float cn = ap.lc * gi[g].inv_n, rn = ap.lr * gi[g].inv_n2;
      float2 o;
      o.x = ap.lkl4 * (fx - r.x * inv_z) + cn * xi.x - rn * en.x;
      o.y = ap.lkl4 * (fy - r.y * inv_z) + cn * xi.y - rn * en.y;
      Gout[i] = o;
      if (Fattr) Fattr[i] = make_float2(fx, fy);
    }
  }
}

hipError_t launch_attract(Problem& P, const float2* X, const tsnet_params& prm, float2* G,
                          float2* F_attr, hipStream_t s) {
  AttrParams ap;
  ap.lkl4 = (float)(4.0 * prm.lambda_kl);
  ap.lc = (float)prm.lambda_c;
  ap.lr = (float)prm.lambda_r;
  int blocks = (P.n + 3) / 4;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_attract, dim3(blocks), dim3(256), 0, s, X, P.rowptr, P.col, P.val,
                     P.row_order, P.n, P.goff_d, P.G, P.ginfo, P.zg, P.rep_ent, ap, G, F_attr);
  return hipGetLastError();
}

}  // namespace tsnet
