// Far points: the points the grid plan set apart (the last box of their
// graph after the binning sort) meet the core through the node grid.
//
// Between a far point o and a core point j the kernel is interpolated in j's
// argument only, K(X_o - X_j) ~ sum_b K(X_o - y_b) L_b(X_j), y_b the nodes.
// That gives two node-level sums per far point, with the same approximation
// in both directions:
//  - o's own sums: S_c(o) = sum_b K(X_o - y_b) w_c(b) over the node charges
//    w_c (charges 1, (x - cx) / half, (y - cy) / half of the spread), plus the
//    exact sums over the other far points of the graph;
//  - o's charges at the nodes: pot_c(a) += K(y_a - X_o) q_c(o) for every node
//    a, added after the FFT and before the gather, so every core point picks
//    them up through its Lagrange weights.
// Then, as in the gather, F_rep = (x_o - c) S[K2,1] - half S[K2,x],
// F_ent = (x_o - c) S[Ke,1] - half S[Ke,x], Z_o = S[K1,1] (no self term) and
// the ln sum S[Kln,1] + ln(eps) (the self term the cost removes for every
// point). Far-far terms are added in direct form, K (X_o - X_o').
//
// One launch, blocks (j, g): j < nbx take far points j, j + nbx, ... of graph
// g (a block sums over all nodes of the graph), j >= nbx sweep the graph's
// nodes with its far points staged in LDS (four threads per node, each over
// every fourth far point). Every sum runs in a fixed order.
// Kernel values use the hardware reciprocal (1 ulp).
#include <hip/hip_runtime.h>

#include <cmath>

#include "dev_util.h"
#include "tsnet_internal.h"

namespace tsnet {

constexpr int kFarThreads = 512;
constexpr int kFarBatch = 512;  // far points staged in LDS at a time (node role)
constexpr int kFarNodes = 16;   // nodes a thread loads ahead per step (far-point role)
constexpr int kFarSums = 14;    // 8 node channels + 6 far-far direct sums
constexpr int kFarParts = 4;    // threads per node in the node role
constexpr int kFarNodesPerBlock = kFarThreads / kFarParts;

struct FarArgs {
  const GridDesc* desc;
  const int* box_off;
  const float2* xs;
  const int* perm;
  const float* charges;
  float* pot;
  float4* rep_ent;
  float* slot_z;
  float* slot_ln;
  float eps;
  int with_ln;
  int nbx;
};

__global__ __launch_bounds__(kFarThreads) void k_far(FarArgs A) {
  __shared__ float4 fp[kFarBatch];
  __shared__ double red[kFarThreads / kWave][kFarSums];
  __shared__ float nsum[kFarParts][8][kFarNodesPerBlock];
  const int g = blockIdx.y;
  const GridDesc d = A.desc[g];
  if (!d.trimmed) return;
  const int fk = far_key(d);
  const int fs = A.box_off[fk], fe = A.box_off[fk + 1];
  const int F = fe - fs;
  if (F == 0) return;
  const int ng = d.ng;
  const int nodes = ng * ng;
  const float inv_half = 1.0f / d.half;
  const int tid = threadIdx.x;
  if ((int)blockIdx.x < A.nbx) {
    // ---- far points' own sums
    const float* w = A.charges + d.off_c;  // [3][ng][ng]
    for (int p = fs + blockIdx.x; p < fe; p += A.nbx) {
      const float2 xo = A.xs[p];
      float acc[kFarSums];
#pragma unroll
      for (int k = 0; k < kFarSums; ++k) acc[k] = 0.f;
      // kFarNodes nodes per step, all their charges loaded before any is used.
      // The thread's nodes advance by kFarThreads: their row and column are
      // carried along (a division per node would cost a third of the loop)
      const int sy = kFarThreads / ng, sx = kFarThreads - sy * ng;
      int ay = tid / ng, ax = tid - ay * ng;
      for (int a0 = tid; a0 < nodes; a0 += kFarNodes * kFarThreads) {
        float w1[kFarNodes], wx[kFarNodes], wy[kFarNodes];
#pragma unroll
        for (int u = 0; u < kFarNodes; ++u) {
          const int a = min(a0 + u * kFarThreads, nodes - 1);
          w1[u] = w[a];
          wx[u] = w[nodes + a];
          wy[u] = w[2 * nodes + a];
        }
#pragma unroll
        for (int u = 0; u < kFarNodes; ++u) {
          const int a = a0 + u * kFarThreads;
          if (a < nodes) {
            const float dx = xo.x - (d.x0 + ((float)ax + 0.5f) * d.spacing);
            const float dy = xo.y - (d.y0 + ((float)ay + 0.5f) * d.spacing);
            const float r2 = dx * dx + dy * dy;
            const float k1 = __builtin_amdgcn_rcpf(1.0f + r2);
            const float k2 = k1 * k1;
            const float ke = __builtin_amdgcn_rcpf(A.eps + r2);
            acc[0] += k2 * w1[u];
            acc[1] += k2 * wx[u];
            acc[2] += k2 * wy[u];
            acc[3] += k1 * w1[u];
            acc[4] += ke * w1[u];
            acc[5] += ke * wx[u];
            acc[6] += ke * wy[u];
            if (A.with_ln) acc[7] += logf(A.eps + r2) * w1[u];
          }
          ax += sx;
          ay += sy;
          if (ax >= ng) {
            ax -= ng;
            ++ay;
          }
        }
      }
      for (int q = fs + tid; q < fe; q += kFarThreads) {
        if (q == p) continue;
        const float2 xq = A.xs[q];
        const float dx = xo.x - xq.x, dy = xo.y - xq.y;
        const float r2 = dx * dx + dy * dy;
        const float k1 = __builtin_amdgcn_rcpf(1.0f + r2);
        const float k2 = k1 * k1;
        const float ke = __builtin_amdgcn_rcpf(A.eps + r2);
        acc[8] += k2 * dx;
        acc[9] += k2 * dy;
        acc[10] += ke * dx;
        acc[11] += ke * dy;
        acc[12] += k1;
        if (A.with_ln) acc[13] += logf(A.eps + r2);
      }
#pragma unroll
      for (int k = 0; k < kFarSums; ++k) {
        const float v = wave_sum(acc[k]);
        if (lane_id() == 0) red[wave_id()][k] = (double)v;
      }
      __syncthreads();
      if (tid == 0) {
        double S[kFarSums];
#pragma unroll
        for (int k = 0; k < kFarSums; ++k) {
          S[k] = 0.0;
          for (int wv = 0; wv < kFarThreads / kWave; ++wv) S[k] += red[wv][k];
        }
        const double xt = (double)xo.x - (double)d.cx, yt = (double)xo.y - (double)d.cy;
        const double hf = (double)d.half;
        const float4 re = make_float4((float)(xt * S[0] - hf * S[1] + S[8]),
                                      (float)(yt * S[0] - hf * S[2] + S[9]),
                                      (float)(xt * S[4] - hf * S[5] + S[10]),
                                      (float)(yt * S[4] - hf * S[6] + S[11]));
        A.rep_ent[A.perm[p]] = re;
        A.slot_z[p] = (float)(S[3] + S[12]);
        if (A.with_ln) A.slot_ln[p] = (float)(S[7] + S[13] + (double)logf(A.eps));
      }
      __syncthreads();
    }
    return;
  }
  // ---- far charges at the nodes: kFarParts threads per node, each over
  // every kFarParts-th far point, their sums joined in part order
  const int j = blockIdx.x - A.nbx;
  const int nbn = gridDim.x - A.nbx;
  const int part = tid / kFarNodesPerBlock, lt = tid - part * kFarNodesPerBlock;
  float2* pl = reinterpret_cast<float2*>(A.pot + d.off_p);  // 4 planes of ng^2
  const int sweep = nbn * kFarNodesPerBlock;
  for (int base = j * kFarNodesPerBlock; base < nodes; base += sweep) {  // uniform over the block
    const int a = base + lt;
    const bool active = a < nodes;
    const int ay = active ? a / ng : 0, ax = active ? a - ay * ng : 0;
    const float nx = d.x0 + ((float)ax + 0.5f) * d.spacing;
    const float ny = d.y0 + ((float)ay + 0.5f) * d.spacing;
    float acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = 0.f;
    for (int b0 = 0; b0 < F; b0 += kFarBatch) {
      const int nb = min(kFarBatch, F - b0);
      __syncthreads();
      if (tid < nb) {
        const float2 xq = A.xs[fs + b0 + tid];
        fp[tid] = make_float4(xq.x, xq.y, (xq.x - d.cx) * inv_half, (xq.y - d.cy) * inv_half);
      }
      __syncthreads();
      if (active) {
        for (int q = part; q < nb; q += kFarParts) {
          const float4 o = fp[q];
          const float dx = nx - o.x, dy = ny - o.y;
          const float r2 = dx * dx + dy * dy;
          const float k1 = __builtin_amdgcn_rcpf(1.0f + r2);
          const float k2 = k1 * k1;
          const float ke = __builtin_amdgcn_rcpf(A.eps + r2);
          acc[CH_K2_1] += k2;
          acc[CH_K2_X] += k2 * o.z;
          acc[CH_K2_Y] += k2 * o.w;
          acc[CH_K1_1] += k1;
          acc[CH_KE_1] += ke;
          acc[CH_KE_X] += ke * o.z;
          acc[CH_KE_Y] += ke * o.w;
          if (A.with_ln) acc[CH_KLN_1] += logf(A.eps + r2);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) nsum[part][k][lt] = acc[k];
    __syncthreads();
    if (part == 0 && active) {
#pragma unroll
      for (int pr = 0; pr < kPotCh / 2; ++pr) {
        float2 v = pl[(size_t)pr * nodes + a];
#pragma unroll
        for (int q = 0; q < kFarParts; ++q) {
          v.x += nsum[q][2 * pr][lt];
          v.y += nsum[q][2 * pr + 1][lt];
        }
        pl[(size_t)pr * nodes + a] = v;
      }
    }
  }
}

hipError_t launch_far(Problem& P, int far_trim, float eps, int with_ln, hipStream_t s) {
  // blocks per graph and role: one per far point at G = 1 (4 t at most),
  // fewer per graph in a batch, at least 16
  int nbx = 16384 / P.G;
  if (nbx > 4 * far_trim) nbx = 4 * far_trim;
  if (nbx > 256) nbx = 256;
  if (nbx < 16) nbx = 16;
  FarArgs A;
  A.desc = P.desc;
  A.box_off = P.box_off;
  A.xs = P.xs;
  A.perm = P.perm;
  A.charges = P.charges;
  A.pot = P.pot;
  A.rep_ent = P.rep_ent;
  A.slot_z = P.slot_z;
  A.slot_ln = P.slot_ln;
  A.eps = eps;
  A.with_ln = with_ln;
  A.nbx = nbx;
  hipLaunchKernelGGL(k_far, dim3(3 * nbx, P.G), dim3(kFarThreads), 0, s, A);  // nbx far-point blocks, 2 nbx node blocks
  return hipGetLastError();
}

}  // namespace tsnet
