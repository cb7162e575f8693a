// Per-evaluation kernels of the L-tsNET gradient: bounding box and grid plan,
// gather of the node potentials back to the points, Z reduction, the vertex
// move and the cost. Binning and spread live in bin.hip, the attraction in
// attract.hip, the convolution in fft.hip.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

#include "dev_util.h"
#include "tsnet_internal.h"

namespace tsnet {

// ---------------------------------------------------------------------------
// Bounding box per chunk (k_bbox_part, the bounds of every chunk to
// part[chunk]); then one wave per graph reduces its chunks and starts the
// graph's descriptor (join_bbox, in k_bbox_join or, for a single graph the
// far-point rule may apply to, in the blocks of k_trim_hist, which saves a
// launch; in a batch each such block would wait on its own join): the box,
// the bin scales of the far-point rule and whether that rule can apply
// (t = min(far_trim, n / 64) >= 1 and a positive width). The grid itself is
// planned by k_trim_plan.
//
// Partial results pass between blocks through a kernel boundary, never
// through a last-block counter: on this GPU a device-wide fence writes back
// and invalidates the L2 of the block's XCD, and one per block cost more than
// the work it guards.
constexpr int kPartBatch = 8;  // chunk partials a lane of the final reduction loads at once

constexpr int kBboxThreads = 256;
constexpr int kBboxPer = kChunk / kBboxThreads;  // points per thread, loaded together

// Per chunk: the bounding box of its finite points, NaN in part[c].x when the
// chunk holds a non-finite coordinate.
__global__ __launch_bounds__(kBboxThreads) void k_bbox_part(const float2* __restrict__ X,
                                                            const int* __restrict__ chunk_start,
                                                            const int* __restrict__ chunk_end,
                                                            float4* part) {
  __shared__ float red[kBboxThreads / kWave][4];
  __shared__ int bad_s;
  const int c = blockIdx.x;
  if (threadIdx.x == 0) bad_s = 0;
  __syncthreads();
  float xmn = FLT_MAX, xmx = -FLT_MAX, ymn = FLT_MAX, ymx = -FLT_MAX;
  int bad = 0;
  {
    const int i0 = chunk_start[c] + threadIdx.x, i1 = chunk_end[c];
    float2 p[kBboxPer];
#pragma unroll
    for (int u = 0; u < kBboxPer; ++u) p[u] = X[min(i0 + u * kBboxThreads, i1 - 1)];
#pragma unroll
    for (int u = 0; u < kBboxPer; ++u) {
      if (i0 + u * kBboxThreads >= i1) continue;
      if (!(isfinite(p[u].x) && isfinite(p[u].y))) {
        bad = 1;
        continue;
      }
      xmn = fminf(xmn, p[u].x);
      xmx = fmaxf(xmx, p[u].x);
      ymn = fminf(ymn, p[u].y);
      ymx = fmaxf(ymx, p[u].y);
    }
  }
  xmn = wave_min(xmn);
  xmx = wave_max(xmx);
  ymn = wave_min(ymn);
  ymx = wave_max(ymx);
  if (bad) atomicOr(&bad_s, 1);
  if (lane_id() == 0) {
    red[wave_id()][0] = xmn;
    red[wave_id()][1] = xmx;
    red[wave_id()][2] = ymn;
    red[wave_id()][3] = ymx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBboxThreads / kWave; ++w) {
      xmn = fminf(xmn, red[w][0]);
      xmx = fmaxf(xmx, red[w][1]);
      ymn = fminf(ymn, red[w][2]);
      ymx = fmaxf(ymx, red[w][3]);
    }
    part[c] = make_float4(bad_s ? NAN : xmn, xmx, ymn, ymx);
  }
}

// A graph's box from its chunks, and the far-point rule's parameters (bins,
// trimming count), computed by one whole wave (every lane gets the result;
// min and max do not depend on the order, so any wave anywhere gets the same).
__device__ GridDesc join_bbox(const float4* __restrict__ part, const GraphInfo& gg,
                              const PlanParams& pp) {
  float a = FLT_MAX, b = -FLT_MAX, e = FLT_MAX, f = -FLT_MAX;
  int nonfinite = 0;
  const int c1 = gg.chunk_end;
  for (int k0 = gg.chunk_begin + lane_id(); k0 < c1; k0 += kPartBatch * kWave) {
    float4 q[kPartBatch];  // the batch's loads in flight together
#pragma unroll
    for (int j = 0; j < kPartBatch; ++j)
      q[j] = k0 + j * kWave < c1 ? part[k0 + j * kWave]
                                 : make_float4(FLT_MAX, -FLT_MAX, FLT_MAX, -FLT_MAX);
#pragma unroll
    for (int j = 0; j < kPartBatch; ++j) {
      if (isnan(q[j].x)) nonfinite = 1;
      if (q[j].y >= q[j].x) {  // chunk had at least one finite point
        a = fminf(a, q[j].x);
        b = fmaxf(b, q[j].y);
        e = fminf(e, q[j].z);
        f = fmaxf(f, q[j].w);
      }
    }
  }
  a = wave_min(a);
  b = wave_max(b);
  e = wave_min(e);
  f = wave_max(f);
  nonfinite = __any(nonfinite);
  if (!(b >= a)) {  // no finite point at all
    a = b = e = f = 0.f;
  }
  GridDesc d = {};
  d.bmin_x = a;
  d.bmax_x = b;
  d.bmin_y = e;
  d.bmax_y = f;
  d.flags = nonfinite ? TSNET_STATUS_NONFINITE : 0;
  const double wx = (double)b - (double)a, wy = (double)f - (double)e;
  d.s_x = wx > 0.0 ? (double)kTrimBins / wx : 0.0;
  d.s_y = wy > 0.0 ? (double)kTrimBins / wy : 0.0;
  const int t = min(pp.far_trim, gg.n / kTrimMinPoints);
  d.trim_t = t;
  d.trimmed = (t >= 1 && fmax(wx, wy) > 0.0 && !nonfinite) ? 1 : 0;
  return d;
}

// One wave per graph: join_bbox into the graph's descriptor. For a single
// graph the far-point rule may apply to, k_trim_hist does this itself.
__global__ __launch_bounds__(256) void k_bbox_join(const float4* __restrict__ part,
                                                   const GraphInfo* __restrict__ gi, int G,
                                                   PlanParams pp, GridDesc* desc) {
  const int g = blockIdx.x * (256 / kWave) + wave_id();
  if (g >= G) return;
  const GridDesc d = join_bbox(part, gi[g], pp);
  if (lane_id() == 0) desc[g] = d;
}

hipError_t launch_bbox_plan(Problem& P, const float2* X, const PlanParams& pp, bool with_hist,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_bbox_part, dim3(P.num_chunks), dim3(kBboxThreads), 0, s, X, P.chunk_start,
                     P.chunk_end, P.bbox_part);
  if (!(with_hist && P.G == 1))  // else the histogram's blocks join the box (one launch fewer)
    hipLaunchKernelGGL(k_bbox_join, dim3((P.G + 3) / 4), dim3(256), 0, s, P.bbox_part, P.ginfo, P.G,
                       pp, P.desc);
  return hipGetLastError();
}

// Bin of coordinate v among kTrimBins equal bins from v_min (s = kTrimBins /
// width), in FP64: floor((v - v_min) s), the last bin closed. A product of a
// difference, so no contraction changes it.
__device__ __forceinline__ int trim_bin(float v, float vmin, double s) {
  const double f = floor(((double)v - (double)vmin) * s);
  return f >= 0.0 ? (f < (double)(kTrimBins - 1) ? (int)f : kTrimBins - 1) : 0;
}

// Per cpb consecutive chunks of a graph the far-point rule may apply to (cpb
// > 1 only for a single graph, whose chunks are all its own): bin counts of
// both axes in LDS, added to the graph's counts (integer atomics, so the
// counts do not depend on the order).
constexpr int kTrimThreads = 1024;
constexpr int kTrimChunksSingle = 4;

__global__ __launch_bounds__(kTrimThreads) void k_trim_hist(
    const float2* __restrict__ X, const int* __restrict__ chunk_graph,
    const int* __restrict__ chunk_start, const int* __restrict__ chunk_end, int nc, int cpb,
    int join, const float4* __restrict__ part, const GraphInfo* __restrict__ gi, PlanParams pp,
    GridDesc* desc, int* hist) {
  __shared__ int hx[kTrimBins], hy[kTrimBins];
  __shared__ GridDesc dsh;
  const int c0 = blockIdx.x * cpb, c1 = min(c0 + cpb, nc);
  const int g = chunk_graph[c0];
  if (join) {
    // the graph's box, joined by the first wave of every block (the same in
    // each); the block of the graph's first chunk starts its descriptor
    if (wave_id() == 0) {
      const GraphInfo gg = gi[g];
      const GridDesc dj = join_bbox(part, gg, pp);
      if (lane_id() == 0) {
        dsh = dj;
        if (c0 == gg.chunk_begin) desc[g] = dj;
      }
    }
  } else if (threadIdx.x == 0) {
    dsh = desc[g];
  }
  __syncthreads();
  const GridDesc d = dsh;
  if (!d.trimmed) return;
  for (int b = threadIdx.x; b < kTrimBins; b += kTrimThreads) hx[b] = hy[b] = 0;
  __syncthreads();
  const int i0 = chunk_start[c0], i1 = chunk_end[c1 - 1];
  constexpr int U = 4;  // points per thread loaded together
  for (int base = i0; base < i1; base += U * kTrimThreads) {
    float2 p[U];
#pragma unroll
    for (int u = 0; u < U; ++u) p[u] = X[min(base + u * kTrimThreads + (int)threadIdx.x, i1 - 1)];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (base + u * kTrimThreads + (int)threadIdx.x < i1) {
        atomicAdd(&hx[trim_bin(p[u].x, d.bmin_x, d.s_x)], 1);
        atomicAdd(&hy[trim_bin(p[u].y, d.bmin_y, d.s_y)], 1);
      }
    }
  }
  __syncthreads();
  int* h = hist + (size_t)g * 2 * kTrimBins;
  for (int b = threadIdx.x; b < kTrimBins; b += kTrimThreads) {
    if (hx[b]) atomicAdd(&h[b], hx[b]);
    if (hy[b]) atomicAdd(&h[kTrimBins + b], hy[b]);
  }
}

// Grid plan, one block per graph (Sec. 2.3 leaves the interval count, the
// node placement and the covered region open). Where the far-point rule may
// apply: lo = bin of the (t+1)-th smallest coordinate, hi = bin of the
// (t+1)-th largest, per axis; when the core bins' region is at most half the
// bounding box's larger side, the grid covers that region and the points
// outside it are far. Otherwise the grid covers the bounding box. Then
// span = larger side (floor kSpanFloor), n_int = ceil(span / h_target)
// clamped to [min, max] and rounded up to a power of two, h = span / n_int,
// grid centred on the region. Decisions in FP64 with every operation rounded
// on its own (no contraction), so the far points and the grid are those of
// the same rule evaluated anywhere else in IEEE FP64. The counts are cleared
// for the next call. Then k_plan_pools (one block; for a single graph the
// plan's own block) sizes the grid buffers, fits them into the workspace
// pools and numbers the boxes.
constexpr int kPlanThreads = 256;
constexpr int kPlanBins = kTrimBins / kPlanThreads;  // consecutive bins per thread

__device__ void plan_pools_block(GridDesc* desc, int G, const PlanParams& pp, int* btotal,
                                 unsigned* status);

__global__ __launch_bounds__(kPlanThreads) void k_trim_plan(GridDesc* desc, int* hist,
                                                             PlanParams pp, unsigned* status,
                                                             int* single_btotal) {
  __shared__ int sh[kPlanThreads / kWave + 1];
  __shared__ int bounds[4];  // lo_x, hi_x, lo_y, hi_y
  const int g = blockIdx.x;
  GridDesc d = desc[g];
  if (d.trimmed) {  // uniform over the block
    int* h = hist + (size_t)g * 2 * kTrimBins;
    const int t = d.trim_t;
    for (int axis = 0; axis < 2; ++axis) {
      int* ha = h + axis * kTrimBins;
      int v[kPlanBins];
      int local = 0;
#pragma unroll
      for (int k = 0; k < kPlanBins; ++k) {
        v[k] = ha[threadIdx.x * kPlanBins + k];
        local += v[k];
      }
#pragma unroll
      for (int k = 0; k < kPlanBins; ++k) ha[threadIdx.x * kPlanBins + k] = 0;
      int total;
      int cum = block_excl_scan(local, sh, &total);
      const int want_lo = t + 1, want_hi = total - t;  // first bins reaching these counts
#pragma unroll
      for (int k = 0; k < kPlanBins; ++k) {
        const int before = cum;
        cum += v[k];
        if (before < want_lo && cum >= want_lo) bounds[2 * axis] = threadIdx.x * kPlanBins + k;
        if (before < want_hi && cum >= want_hi) bounds[2 * axis + 1] = threadIdx.x * kPlanBins + k;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double xlo = d.bmin_x, xhi = d.bmax_x, ylo = d.bmin_y, yhi = d.bmax_y;
    int trim = 0;
    if (d.trimmed) {
      const double wx = __dsub_rn((double)d.bmax_x, (double)d.bmin_x);
      const double wy = __dsub_rn((double)d.bmax_y, (double)d.bmin_y);
      const double qx = wx / kTrimBins, qy = wy / kTrimBins;  // exact: a power of two
      d.lo_x = bounds[0];
      d.hi_x = bounds[1];
      d.lo_y = bounds[2];
      d.hi_y = bounds[3];
      const double cw = __dmul_rn((double)(d.hi_x - d.lo_x + 1), qx);
      const double ch = __dmul_rn((double)(d.hi_y - d.lo_y + 1), qy);
      if (2.0 * fmax(cw, ch) <= fmax(wx, wy)) {
        trim = 1;
        xlo = __dadd_rn((double)d.bmin_x, __dmul_rn((double)d.lo_x, qx));
        xhi = __dadd_rn((double)d.bmin_x, __dmul_rn((double)(d.hi_x + 1), qx));
        ylo = __dadd_rn((double)d.bmin_y, __dmul_rn((double)d.lo_y, qy));
        yhi = __dadd_rn((double)d.bmin_y, __dmul_rn((double)(d.hi_y + 1), qy));
      }
    }
    d.trimmed = trim;
    int flags = d.flags;
    double span = fmax(__dsub_rn(xhi, xlo), __dsub_rn(yhi, ylo));
    if (!(span >= kSpanFloor)) span = kSpanFloor;
    const double q = span / pp.h_target;
    int nint;
    if (!(q <= (double)pp.max_int)) {
      nint = pp.max_int;
      flags |= TSNET_STATUS_GRID_CAPPED;
    } else {
      nint = (int)ceil(q);
      if (nint < pp.min_int) nint = pp.min_int;
    }
    int p2 = 1;
    while (p2 < nint) p2 <<= 1;
    nint = p2 < pp.max_int ? p2 : pp.max_int;
    const double h = span / nint;
    const double cx = __dmul_rn(0.5, __dadd_rn(xlo, xhi)), cy = __dmul_rn(0.5, __dadd_rn(ylo, yhi));
    const double half = __dmul_rn(__dmul_rn(0.5, (double)nint), h);
    d.x0 = (float)__dsub_rn(cx, half);
    d.y0 = (float)__dsub_rn(cy, half);
    d.h = (float)h;
    d.inv_h = (float)(1.0 / h);
    d.cx = (float)cx;
    d.cy = (float)cy;
    d.half = (float)half;
    d.spacing = (float)(h / kNodes);
    d.n_int = nint;
    d.ng = kNodes * nint;
    d.M = 2 * kNodes * nint;
    d.box_base = 0;
    d.flags = flags;
    desc[g] = d;
    if (flags) atomicOr(status, (unsigned)flags);
  }
  if (single_btotal) {  // a single graph: this block also fits the pools (no second launch)
    __syncthreads();
    plan_pools_block(desc, 1, pp, single_btotal, status);
  }
}

// The grid buffers every graph needs, before and after fitting them into the
// workspace pools, then the box ids and pool offsets of every graph (one
// block: one graph per thread and step). Descriptors are read past the
// non-coherent cache: the block may have written them itself.
__device__ void plan_pools_block(GridDesc* desc, int G, const PlanParams& pp, int* btotal,
                                 unsigned* status) {
  __shared__ unsigned long long red_need[POOL_KINDS][kPlanThreads / kWave];
  size_t need[POOL_KINDS] = {0, 0, 0, 0, 0};
  for (int gg = threadIdx.x; gg < G; gg += kPlanThreads) {
    const int ni = ld_coherent(&desc[gg].n_int);
    for (int k = 0; k < POOL_KINDS; ++k) need[k] += pool_elems(k, ni);
  }
  for (int k = 0; k < POOL_KINDS; ++k) {
    const unsigned long long v = wave_sum((unsigned long long)need[k]);
    if (lane_id() == 0) red_need[k][wave_id()] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 0; k < POOL_KINDS; ++k) {
      need[k] = 0;
      for (int w = 0; w < kPlanThreads / kWave; ++w) need[k] += red_need[k][w];
    }
    if (pp.need) {
      for (int k = 0; k < POOL_KINDS; ++k) pp.need[k] = need[k];
      __threadfence_system();
    }
    bool short_pool = false;
    for (int k = 0; k < POOL_KINDS; ++k) short_pool |= need[k] > pp.cap[k];
    if (short_pool) {
      // while a pool is short, the largest grid (the lowest graph id among
      // equals) is halved per axis over the same region
      const unsigned raised = TSNET_STATUS_WORKSPACE | TSNET_STATUS_GRID_CAPPED;
      for (;;) {
        bool fits = true;
        for (int k = 0; k < POOL_KINDS; ++k) fits &= need[k] <= pp.cap[k];
        if (fits) break;
        int big = -1, bn = 1;
        for (int gg = 0; gg < G; ++gg) {
          const int ni = ld_coherent(&desc[gg].n_int);  // this thread's own stores included
          if (ni > bn) {
            bn = ni;
            big = gg;
          }
        }
        if (big < 0) break;  // every grid is down to one box: nothing left to give
        GridDesc d2 = desc[big];
        const double span = (double)d2.h * d2.n_int;
        const int nn = d2.n_int / 2;
        for (int k = 0; k < POOL_KINDS; ++k) need[k] += pool_elems(k, nn) - pool_elems(k, d2.n_int);
        const double h2 = span / nn;
        const double half2 = 0.5 * nn * h2;
        d2.x0 = (float)((double)d2.cx - half2);
        d2.y0 = (float)((double)d2.cy - half2);
        d2.h = (float)h2;
        d2.inv_h = (float)(1.0 / h2);
        d2.half = (float)half2;
        d2.spacing = (float)(h2 / kNodes);
        d2.n_int = nn;
        d2.ng = kNodes * nn;
        d2.M = 2 * kNodes * nn;
        d2.flags |= (int)raised;
        desc[big] = d2;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // stored before it is read again
      }
      atomicOr(status, raised);
    }
  }
  __syncthreads();
  // box ids and pool offsets: exclusive prefix sums over the graphs in order,
  // kPlanThreads graphs per step
  __shared__ int carry_box;
  __shared__ unsigned long long carry_off[POOL_KINDS];
  __shared__ int sh_scan[kPlanThreads / kWave + 1];
  if (threadIdx.x == 0) {
    carry_box = 0;
    for (int k = 0; k < POOL_KINDS; ++k) carry_off[k] = 0;
  }
  __syncthreads();
  for (int base = 0; base < G; base += kPlanThreads) {
    const int gg = base + threadIdx.x;
    const int ni = gg < G ? ld_coherent(&desc[gg].n_int) : 0;
    int tot;
    const int bx = block_excl_scan(gg < G ? ni * ni + 1 : 0, sh_scan, &tot);
    size_t off[POOL_KINDS];
    unsigned long long tot_k[POOL_KINDS];
    for (int k = 0; k < POOL_KINDS; ++k) {
      // pool parts are multiples of 64 elements: scan them in units of 64
      int t64;
      const int u = block_excl_scan(gg < G ? (int)(pool_elems(k, ni) / 64) : 0, sh_scan, &t64);
      off[k] = (size_t)carry_off[k] + (size_t)u * 64;
      tot_k[k] = (unsigned long long)t64 * 64;
    }
    if (gg < G) {
      desc[gg].box_base = carry_box + bx;
      desc[gg].off_c = off[POOL_C];
      desc[gg].off_q = off[POOL_Q];
      desc[gg].off_k = off[POOL_K];
      desc[gg].off_o = off[POOL_O];
      desc[gg].off_p = off[POOL_P];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      carry_box += tot;
      for (int k = 0; k < POOL_KINDS; ++k) carry_off[k] += tot_k[k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *btotal = carry_box;
}

__global__ __launch_bounds__(kPlanThreads) void k_plan_pools(GridDesc* desc, int G, PlanParams pp,
                                                              int* btotal, unsigned* status) {
  plan_pools_block(desc, G, pp, btotal, status);
}

hipError_t launch_trim_plan(Problem& P, const float2* X, const PlanParams& pp, bool with_hist,
                            hipStream_t s) {
  if (with_hist) {
    const int cpb = P.G == 1 ? kTrimChunksSingle : 1;
    hipLaunchKernelGGL(k_trim_hist, dim3((P.num_chunks + cpb - 1) / cpb), dim3(kTrimThreads), 0, s, X,
                       P.chunk_graph, P.chunk_start, P.chunk_end, P.num_chunks, cpb,
                       P.G == 1 ? 1 : 0, P.bbox_part, P.ginfo, pp, P.desc, P.trim_hist);
  }
  hipLaunchKernelGGL(k_trim_plan, dim3(P.G), dim3(kPlanThreads), 0, s, P.desc, P.trim_hist, pp,
                     P.ctx->status, P.G == 1 ? P.btotal : nullptr);
  if (P.G > 1)
    hipLaunchKernelGGL(k_plan_pools, dim3(1), dim3(kPlanThreads), 0, s, P.desc, P.G, pp, P.btotal,
                       P.ctx->status);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// phi = the 8 potential channels at x, interpolated from the 3 x 3 nodes of
// box (bx, by): the Lagrange weights of the point times the node values (the
// potentials are 4 planes, one per channel pair, of ng^2 float2 nodes).
__device__ __forceinline__ void gather_box(const float* __restrict__ pg, const GridDesc& d,
                                           float2 x, int by, int bx, float (&phi)[8]) {
  const float s = (x.x - d.x0) * d.inv_h - (float)bx;
  const float t = (x.y - d.y0) * d.inv_h - (float)by;
  float lx[3], ly[3];
  lagrange3(s, lx);
  lagrange3(t, ly);
#pragma unroll
  for (int k = 0; k < 8; ++k) phi[k] = 0.f;
  const float2* pl = reinterpret_cast<const float2*>(pg);
  const size_t plane = (size_t)d.ng * d.ng;
#pragma unroll
  for (int ty = 0; ty < 3; ++ty) {
    const size_t row = (size_t)(3 * by + ty) * d.ng + 3 * bx;
#pragma unroll
    for (int tx = 0; tx < 3; ++tx) {
      const float w = ly[ty] * lx[tx];
#pragma unroll
      for (int pr = 0; pr < kPotCh / 2; ++pr) {
        const float2 v = pl[pr * plane + row + tx];
        phi[2 * pr] += w * v.x;
        phi[2 * pr + 1] += w * v.y;
      }
    }
  }
}

// Gather (Sec. 2.3 / Sec. 3.3): interpolate the 8 node potentials to every
// point in sorted order (coordinates and box ids come from the binning, so a
// wave reads few nodes), then form
//   F_rep = (x - c) phi[K2,1] - phi[K2,x],  F_ent = (x - c) phi[Ke,1] - phi[Ke,x],
//   Z_i = phi[K1,1] - 1 (the self term K1(0) = 1),
// and write them at the vertex of the slot (F_rep and F_ent as one 16-byte
// record, Z_i only when it is asked for). Far points (the last box of their
// graph) were summed by k_far: their F_rep and F_ent are in place, their Z_i
// and ln sum come from slot_z and slot_ln.
// kGatherSplit blocks of kGatherThreads per chunk, each taking one part of
// its sorted slots (several blocks of a CU keep more points in flight than one
// large block, which the gather's registers would make the only one). Each
// block also sums the Z_i of its part (compensated FP32, in sorted order) into
// zpart[chunk * kGatherSplit + part]; k_zsum then adds every graph's part sums
// in FP64 (fixed order, so Z is reproducible) into zg and Z_out.
constexpr int kGatherThreads = 256;
static_assert(kGatherSplit * kGatherThreads * 2 == kChunk, "two points per thread");

__global__ __launch_bounds__(kGatherThreads) void k_gather(
    const float2* __restrict__ xs, const int* __restrict__ skeys, const int* __restrict__ perm,
    const int* __restrict__ chunk_graph, const int* __restrict__ chunk_start,
    const int* __restrict__ chunk_end, const GridDesc* __restrict__ desc,
    const GraphInfo* __restrict__ gi, int G, const float* __restrict__ pot,
    const float* __restrict__ slot_z, const float* __restrict__ slot_ln, float4* rep_ent,
    float* zi, float* lnv, double* zpart) {
  constexpr int NW = kGatherThreads / kWave;
  __shared__ float sh_hi[NW], sh_lo[NW];
  const int c = blockIdx.x / kGatherSplit, part = blockIdx.x - c * kGatherSplit;
  const int g = chunk_graph[c];
  const GridDesc d = desc[g];
  const float* pg = pot + d.off_p;
  const bool single = gi[g].n == 1;
  CompSum zs;
  // the thread's points of the part, their slot data loaded together
  // (clamped into the chunk) before any is used
  constexpr int PPT = 2;
  const int cs = chunk_start[c], pe = chunk_end[c];
  const int pa = cs + part * (PPT * kGatherThreads) + threadIdx.x;
  float2 xv[PPT];
  int kv[PPT], iv[PPT];
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    const int q = max(min(pa + u * kGatherThreads, pe - 1), cs);
    xv[u] = xs[q];
    kv[u] = skeys[q];
    iv[u] = perm[q];
  }
  // the box of each point (n_int is a power of two: the plan rounds up to
  // one and only halves it); far points, the last box of their graph, take
  // their sums from k_far
  const int lg = __builtin_ctz((unsigned)d.n_int), far_local = d.n_int * d.n_int;
  int loc[PPT];
  bool act[PPT];
  // whether, for each u, the wave's interpolated points share one box (the
  // common case in sorted order): their node potentials then have one
  // address per wave and come through the scalar cache. One decision for
  // all u, so that either way every point's loads are in flight together.
  bool uni = true;
  int kb[PPT];
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    loc[u] = kv[u] - d.box_base;
    act[u] = pa + u * kGatherThreads < pe && loc[u] != far_local;
    const unsigned long long m = __ballot(act[u]);
    kb[u] = m ? __builtin_amdgcn_readlane(loc[u], __ffsll((long long)m) - 1) : 0;
    uni = uni && __ballot(act[u] && loc[u] != kb[u]) == 0;
  }
  auto point = [&](int u, int by, int bx) {
    const int p = pa + u * kGatherThreads;
    if (p >= pe) return;
    if (!act[u]) {
      const float z = slot_z[p];
      if (zi) zi[iv[u]] = z;
      if (lnv) lnv[iv[u]] = slot_ln[p];
      zs.add(z);
      return;
    }
    const float2 x = xv[u];
    float phi[8];
    gather_box(pg, d, x, by, bx, phi);
    const float xt = x.x - d.cx, yt = x.y - d.cy;
    float2 r = make_float2(xt * phi[CH_K2_1] - d.half * phi[CH_K2_X],
                           yt * phi[CH_K2_1] - d.half * phi[CH_K2_Y]);
    float2 e = make_float2(xt * phi[CH_KE_1] - d.half * phi[CH_KE_X],
                           yt * phi[CH_KE_1] - d.half * phi[CH_KE_Y]);
    float z = phi[CH_K1_1] - 1.0f;
    if (single) {
      r = make_float2(0.f, 0.f);
      e = make_float2(0.f, 0.f);
      z = 0.f;
    }
    const int i = iv[u];
    rep_ent[i] = make_float4(r.x, r.y, e.x, e.y);  // one scattered 16-byte store
    if (zi) zi[i] = z;
    if (lnv) lnv[i] = single ? 0.f : phi[CH_KLN_1];
    zs.add(z);
  };
  if (uni) {
#pragma unroll
    for (int u = 0; u < PPT; ++u) point(u, kb[u] >> lg, kb[u] & (d.n_int - 1));
  } else {
#pragma unroll
    for (int u = 0; u < PPT; ++u) point(u, loc[u] >> lg, loc[u] & (d.n_int - 1));
  }
  zs = wave_comp_sum(zs);
  if (lane_id() == 0) {
    sh_hi[wave_id()] = zs.hi;
    sh_lo[wave_id()] = zs.lo;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double v = 0.0;
    for (int w = 0; w < NW; ++w) v += (double)sh_hi[w] + (double)sh_lo[w];
    zpart[blockIdx.x] = v;
  }
}

// One wave per graph: Z = the graph's part sums added in FP64 in chunk and
// part order.
__global__ __launch_bounds__(256) void k_zsum(const double* __restrict__ zpart,
                                              const GraphInfo* __restrict__ gi, int G, double* zg,
                                              double* Z_out) {
  const int g = blockIdx.x * (256 / kWave) + wave_id();
  if (g >= G) return;
  double z = 0.0;
  const int c1 = gi[g].chunk_end * kGatherSplit;
  for (int k0 = gi[g].chunk_begin * kGatherSplit + lane_id(); k0 < c1; k0 += kPartBatch * kWave) {
    double q[kPartBatch];  // the batch's loads in flight together
#pragma unroll
    for (int j = 0; j < kPartBatch; ++j) q[j] = k0 + j * kWave < c1 ? zpart[k0 + j * kWave] : 0.0;
#pragma unroll
    for (int j = 0; j < kPartBatch; ++j) z += q[j];
  }
  z = wave_sum(z);
  if (lane_id() == 0) {
    zg[g] = z;
    if (Z_out) Z_out[g] = z;
  }
}

hipError_t launch_gather(Problem& P, const float2* X, int with_ln, int with_zi, double* Z_out,
                         hipStream_t s) {
  (void)X;
  const int nb = P.num_chunks;
  hipLaunchKernelGGL(k_gather, dim3(nb * kGatherSplit), dim3(kGatherThreads), 0, s, P.xs, P.skeys, P.perm, P.chunk_graph,
                     P.chunk_start, P.chunk_end, P.desc, P.ginfo, P.G, P.pot,
                     P.slot_z, P.slot_ln, P.rep_ent, with_zi ? P.zi : nullptr, with_ln ? P.lnv : nullptr, P.zpart);
  hipLaunchKernelGGL(k_zsum, dim3((P.G + 3) / 4), dim3(256), 0, s, P.zpart, P.ginfo, P.G, P.zg, Z_out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Vertex move with momentum and gains (t-SNE's update; the paper only says
// "move each vertex along the gradient").
struct StepK {
  float eta, mu, min_gain, up, down;
};

// The step of one vertex (gains, momentum update, move).
__device__ __forceinline__ void step_vertex(float2& x, float2& u, float2& k, float2 g, float eta,
                                            const StepK& sk) {
  k.x = ((g.x > 0.f) != (u.x > 0.f)) ? k.x + sk.up : k.x * sk.down;
  k.y = ((g.y > 0.f) != (u.y > 0.f)) ? k.y + sk.up : k.y * sk.down;
  k.x = fmaxf(k.x, sk.min_gain);
  k.y = fmaxf(k.y, sk.min_gain);
  u.x = sk.mu * u.x - eta * k.x * g.x;
  u.y = sk.mu * u.y - eta * k.y * g.y;
  x.x += u.x;
  x.y += u.y;
}

__device__ __forceinline__ float step_eta(const StepK& sk, const GraphInfo* __restrict__ gi,
                                          const int* __restrict__ vgraph, int G, int i) {
  return sk.eta > 0.f ? sk.eta : gi[G == 1 ? 0 : vgraph[i]].lr;
}

__global__ __launch_bounds__(256) void k_step(float2* X, float2* upd, float2* gains,
                                              const float2* __restrict__ Gr, int n,
                                              const int* __restrict__ vgraph, int G,
                                              const GraphInfo* __restrict__ gi, StepK sk) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    float2 u = upd[i], k = gains[i], x = X[i];
    step_vertex(x, u, k, Gr[i], step_eta(sk, gi, vgraph, G, i), sk);
    gains[i] = k;
    upd[i] = u;
    X[i] = x;
  }
}

// The same step, two vertices per thread with 16-byte loads and stores (the
// four arrays 16-byte aligned); the last vertex of an odd n by one thread.
__global__ __launch_bounds__(256) void k_step_pairs(float4* X, float4* upd, float4* gains,
                                                    const float4* __restrict__ Gr, int n,
                                                    const int* __restrict__ vgraph, int G,
                                                    const GraphInfo* __restrict__ gi, StepK sk) {
  const int np = n / 2;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < np; p += gridDim.x * blockDim.x) {
    const float4 g = Gr[p];
    float4 u = upd[p], k = gains[p], x = X[p];
    float2 x0 = make_float2(x.x, x.y), x1 = make_float2(x.z, x.w);
    float2 u0 = make_float2(u.x, u.y), u1 = make_float2(u.z, u.w);
    float2 k0 = make_float2(k.x, k.y), k1 = make_float2(k.z, k.w);
    step_vertex(x0, u0, k0, make_float2(g.x, g.y), step_eta(sk, gi, vgraph, G, 2 * p), sk);
    step_vertex(x1, u1, k1, make_float2(g.z, g.w), step_eta(sk, gi, vgraph, G, 2 * p + 1), sk);
    gains[p] = make_float4(k0.x, k0.y, k1.x, k1.y);
    upd[p] = make_float4(u0.x, u0.y, u1.x, u1.y);
    X[p] = make_float4(x0.x, x0.y, x1.x, x1.y);
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    const int i = n - 1;
    float2* X2 = reinterpret_cast<float2*>(X);
    float2* u2 = reinterpret_cast<float2*>(upd);
    float2* k2 = reinterpret_cast<float2*>(gains);
    float2 u = u2[i], k = k2[i], x = X2[i];
    step_vertex(x, u, k, reinterpret_cast<const float2*>(Gr)[i], step_eta(sk, gi, vgraph, G, i), sk);
    k2[i] = k;
    u2[i] = u;
    X2[i] = x;
  }
}

hipError_t launch_step(Problem& P, float2* X, float2* upd, float2* gains, const float2* G,
                       const tsnet_step_params& sp, int iter, hipStream_t s) {
  StepK sk;
  sk.eta = (float)sp.eta;
  sk.mu = (float)(iter < sp.momentum_switch_iter ? sp.momentum_early : sp.momentum_late);
  sk.min_gain = (float)sp.min_gain;
  sk.up = (float)sp.gain_up;
  sk.down = (float)sp.gain_down;
  const bool a16 = ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(upd) |
                     reinterpret_cast<uintptr_t>(gains) | reinterpret_cast<uintptr_t>(G)) & 15) == 0;
  if (a16) {
    int blocks = (P.n / 2 + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_step_pairs, dim3(blocks), dim3(256), 0, s, reinterpret_cast<float4*>(X),
                       reinterpret_cast<float4*>(upd), reinterpret_cast<float4*>(gains),
                       reinterpret_cast<const float4*>(G), P.n, P.vgraph, P.G, P.ginfo, sk);
  } else {
    int blocks = (P.n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_step, dim3(blocks), dim3(256), 0, s, X, upd, gains, G, P.n, P.vgraph, P.G,
                       P.ginfo, sk);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Cost of Eq. (1), entropy in the kernel form -l_r / (4 n^2) sum ln(eps + r^2):
//  per row: sum_j p_ij (ln p_ij + ln(1 + r_ij^2)) over p > 0 and sum_j p_ij;
//  per chunk: compensated sums of those, of ||X_i||^2 and of the interpolated
//  sum_j ln(eps + r_ij^2) (self term ln eps included);
//  per graph (k_cost_join): C_KL = l_kl (S_pl + S_p ln Z) with the Z the
//  gather reduced, C_CMP, C_ENT, total.
__global__ __launch_bounds__(256) void k_cost_rows(const float2* __restrict__ X,
                                                   const int64_t* __restrict__ rowptr,
                                                   const int* __restrict__ col,
                                                   const float* __restrict__ val, int n,
                                                   float2* rowv) {
  const int lane = lane_id();
  const int nwaves = blockDim.x / kWave;
  for (int i = blockIdx.x * nwaves + wave_id(); i < n; i += gridDim.x * nwaves) {
    const float2 xi = X[i];
    float s1 = 0.f, s2 = 0.f;
    for (int64_t e = rowptr[i] + lane; e < rowptr[i + 1]; e += kWave) {
      const float p = val[e];
      if (p > 0.f) {
        const float2 xj = X[col[e]];
        const float dx = xi.x - xj.x, dy = xi.y - xj.y;
        s1 += p * (logf(p) + log1pf(dx * dx + dy * dy));
        s2 += p;
      }
    }
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    if (lane == 0) rowv[i] = make_float2(s1, s2);
  }
}

struct CostK {
  double lkl, lc, lr, log_eps;
};

__global__ __launch_bounds__(256) void k_cost_reduce(
    const float2* __restrict__ X, const float2* __restrict__ rowv, const float* __restrict__ lnv,
    const int* __restrict__ chunk_start, const int* __restrict__ chunk_end, double* part) {
  constexpr int NQ = kCostTerms;
  __shared__ float sh[NQ][2][4];
  const int c = blockIdx.x;
  CompSum acc[NQ];
  for (int i = chunk_start[c] + threadIdx.x; i < chunk_end[c]; i += blockDim.x) {
    const float2 rv = rowv[i];
    const float2 x = X[i];
    acc[0].add(rv.x);
    acc[1].add(rv.y);
    acc[2].add(x.x * x.x + x.y * x.y);
    acc[3].add(lnv[i]);
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    acc[q] = wave_comp_sum(acc[q]);
    if (lane_id() == 0) {
      sh[q][0][wave_id()] = acc[q].hi;
      sh[q][1][wave_id()] = acc[q].lo;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 0; q < NQ; ++q) {
      double v = 0.0;
      for (int w = 0; w < 4; ++w) v += (double)sh[q][0][w] + (double)sh[q][1][w];
      part[(size_t)c * NQ + q] = v;
    }
  }
}

// One wave per graph: the chunk sums in chunk order, then the cost terms.
__global__ __launch_bounds__(256) void k_cost_join(const double* __restrict__ part,
                                                   const double* __restrict__ zg,
                                                   const GraphInfo* __restrict__ gi, int G,
                                                   CostK ck, double* cost) {
  constexpr int NQ = kCostTerms;
  const int g = blockIdx.x * (256 / kWave) + wave_id();
  if (g >= G) return;
  {
    double s[NQ] = {0, 0, 0, 0};
    for (int k = gi[g].chunk_begin + lane_id(); k < gi[g].chunk_end; k += kWave)
      for (int q = 0; q < NQ; ++q) s[q] += part[(size_t)k * NQ + q];
    for (int q = 0; q < NQ; ++q) s[q] = wave_sum(s[q]);
    if (lane_id() != 0) return;
    const double n = (double)gi[g].n;
    const double Z = zg[g];
    const double kl = (n > 1 && Z > 0) ? ck.lkl * (s[0] + s[1] * log(Z)) : 0.0;
    const double cm = ck.lc / (2.0 * n) * s[2];
    const double en = n > 1 ? -ck.lr / (4.0 * n * n) * (s[3] - n * ck.log_eps) : 0.0;
    cost[g * 4 + 0] = kl;
    cost[g * 4 + 1] = cm;
    cost[g * 4 + 2] = en;
    cost[g * 4 + 3] = kl + cm + en;
  }
}

hipError_t launch_cost(Problem& P, const float2* X, const tsnet_params& prm, double* cost,
                       hipStream_t s) {
  int blocks = (P.n + 3) / 4;
  if (blocks > 8192) blocks = 8192;
  // rows' KL sums go to the storage of rep_ent (unused by the cost path)
  float2* rowv = reinterpret_cast<float2*>(P.rep_ent);
  hipLaunchKernelGGL(k_cost_rows, dim3(blocks), dim3(256), 0, s, X, P.rowptr, P.col, P.val, P.n,
                     rowv);
  CostK ck{prm.lambda_kl, prm.lambda_c, prm.lambda_r, log(prm.eps_r)};
  hipLaunchKernelGGL(k_cost_reduce, dim3(P.num_chunks), dim3(256), 0, s, X, rowv, P.lnv,
                     P.chunk_start, P.chunk_end, P.cost_part);
  hipLaunchKernelGGL(k_cost_join, dim3((P.G + 3) / 4), dim3(256), 0, s, P.cost_part, P.zg, P.ginfo,
                     P.G, ck, cost);
  return hipGetLastError();
}

// The two halves of the packed (F_rep, F_ent) records into the caller's arrays.
__global__ __launch_bounds__(256) void k_split_terms(const float4* __restrict__ re, int n,
                                                     float2* F_rep, float2* F_ent) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const float4 v = re[i];
    if (F_rep) F_rep[i] = make_float2(v.x, v.y);
    if (F_ent) F_ent[i] = make_float2(v.z, v.w);
  }
}

hipError_t launch_copy_terms(Problem& P, float2* F_rep, float2* F_ent, float* Z_i, hipStream_t s) {
  if ((F_rep || F_ent) && P.n > 0) {
    int blocks = (P.n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_split_terms, dim3(blocks), dim3(256), 0, s, P.rep_ent, P.n, F_rep, F_ent);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (Z_i) {
    hipError_t e = hipMemcpyAsync(Z_i, P.zi, sizeof(float) * P.n, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

}  // namespace tsnet
