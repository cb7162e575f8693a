// Exact O(n^2) FP64 gradient: the tsNET evaluation over the same sparse P,
// used as the comparison baseline for the interpolation path.
//
// Per row i of graph g (all j of g, j != i):
//   Z_i = sum w_ij, F_rep,i = sum w_ij^2 (X_i - X_j), F_ent,i = sum (X_i - X_j) / (eps + r^2)
// with w = 1 / (1 + r^2) (Sec. 2.1, Eq. 6 and Eq. 8); then the sparse
// F_attr,i = sum_j p_ij w_ij (X_i - X_j) and the assembled gradient.
// Both reciprocals of a pair come from one: 1 / ((1 + r^2)(eps + r^2)),
// refined by two Newton steps from the hardware estimate.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "dev_util.h"
#include "tsnet_internal.h"

namespace tsnet {

constexpr int kDirRows = 2;     // rows per thread
constexpr int kDirTile = 512;   // j points staged in LDS per step

__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

// terms[r][5] = {Z_i, F_rep x, F_rep y, F_ent x, F_ent y} (zonly: Z_i only).
__global__ __launch_bounds__(256) void k_direct_pairs(const double2* __restrict__ X, int n,
                                                      const int* __restrict__ rows, int nrows,
                                                      const int* __restrict__ goff, int G,
                                                      double eps, int zonly, double* terms) {
  __shared__ double2 tile[kDirTile];
  const int r0 = blockIdx.x * blockDim.x * kDirRows;
  int ri[kDirRows], lo[kDirRows], hi[kDirRows];
  double2 xi[kDirRows];
  double z[kDirRows], rx[kDirRows], ry[kDirRows], ex[kDirRows], ey[kDirRows];
  int jmin = 0x7fffffff, jmax = 0;
#pragma unroll
  for (int q = 0; q < kDirRows; ++q) {
    const int r = r0 + q * blockDim.x + threadIdx.x;
    ri[q] = r < nrows ? (rows ? rows[r] : r) : -1;
    if (ri[q] >= n) ri[q] = -1;  // ids outside the problem are not evaluated
    if (ri[q] >= 0) {
      const int g = G == 1 ? 0 : graph_of(goff, G, ri[q]);
      lo[q] = goff[g];
      hi[q] = goff[g + 1];
      xi[q] = X[ri[q]];
    } else {
      lo[q] = hi[q] = 0;
      xi[q] = make_double2(0.0, 0.0);
    }
    z[q] = rx[q] = ry[q] = ex[q] = ey[q] = 0.0;
  }
  // j range of the block: union of its rows' graphs
  __shared__ int sh_lo, sh_hi;
  if (threadIdx.x == 0) {
    sh_lo = 0x7fffffff;
    sh_hi = 0;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kDirRows; ++q)
    if (ri[q] >= 0) {
      atomicMin(&sh_lo, lo[q]);
      atomicMax(&sh_hi, hi[q]);
    }
  __syncthreads();
  jmin = sh_lo;
  jmax = sh_hi;
  for (int j0 = jmin; j0 < jmax; j0 += kDirTile) {
    const int nt = jmax - j0 < kDirTile ? jmax - j0 : kDirTile;
    for (int t = threadIdx.x; t < nt; t += blockDim.x) tile[t] = X[j0 + t];
    __syncthreads();
    for (int t = 0; t < nt; ++t) {
      const double2 xj = tile[t];
      const int j = j0 + t;
#pragma unroll
      for (int q = 0; q < kDirRows; ++q) {
        if (j < lo[q] || j >= hi[q]) continue;
        const double dx = xi[q].x - xj.x, dy = xi[q].y - xj.y;
        const double r2 = fma(dx, dx, dy * dy);
        const double a = 1.0 + r2;
        if (zonly) {
          z[q] += rcp_nr(a);
        } else {
          const double b = eps + r2;
          const double inv = rcp_nr(a * b);
          const double w = inv * b;
          const double ke = inv * a;
          z[q] += w;
          const double w2 = w * w;
          rx[q] = fma(w2, dx, rx[q]);
          ry[q] = fma(w2, dy, ry[q]);
          ex[q] = fma(ke, dx, ex[q]);
          ey[q] = fma(ke, dy, ey[q]);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < kDirRows; ++q) {
    const int r = r0 + q * blockDim.x + threadIdx.x;
    if (r >= nrows) continue;
    // remove the j = i term, evaluated the same way (its displacement is zero)
    double self;
    if (zonly) {
      self = rcp_nr(1.0);
    } else {
      const double inv = rcp_nr(1.0 * eps);
      self = inv * eps;
    }
    double* o = terms + (size_t)r * 5;
    if (ri[q] < 0) {
      o[0] = o[1] = o[2] = o[3] = o[4] = __builtin_nan("");
      continue;
    }
    o[0] = z[q] - self;
    if (!zonly) {
      o[1] = rx[q];
      o[2] = ry[q];
      o[3] = ex[q];
      o[4] = ey[q];
    }
  }
}

// Z per graph from per-row Z_i (terms[.][0]) in row order; rows are all n vertices.
__global__ __launch_bounds__(256) void k_direct_z(const double* __restrict__ terms,
                                                  const int* __restrict__ goff, int G,
                                                  double* zg, double* Z_out) {
  const int g = blockIdx.x;
  __shared__ double sh[4];
  double acc = 0.0;
  for (int i = goff[g] + threadIdx.x; i < goff[g + 1]; i += blockDim.x) acc += terms[(size_t)i * 5];
  acc = wave_sum(acc);
  if (lane_id() == 0) sh[wave_id()] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double z = sh[0] + sh[1] + sh[2] + sh[3];
    zg[g] = z;
    if (Z_out) Z_out[g] = z;
  }
}

struct DirParams {
  double lkl4, lc, lr;
};

// Sparse attraction in FP64 and the assembled gradient, one wave per row.
__global__ __launch_bounds__(256) void k_direct_attr(
    const double2* __restrict__ X, int n, const int64_t* __restrict__ rowptr,
    const int* __restrict__ col, const float* __restrict__ val, const int* __restrict__ rows, int nrows,
    const int* __restrict__ goff, int G, const GraphInfo* __restrict__ gi,
    const double* __restrict__ zg, const double* __restrict__ pairs, DirParams dp, double2* Gout,
    double* terms) {
  const int lane = lane_id();
  const int nwaves = blockDim.x / kWave;
  for (int r = blockIdx.x * nwaves + wave_id(); r < nrows; r += gridDim.x * nwaves) {
    const int i = rows ? rows[r] : r;
    if (i < 0 || i >= n) {
      if (lane == 0) {
        Gout[r] = make_double2(__builtin_nan(""), __builtin_nan(""));
        if (terms)
          for (int q = 0; q < 7; ++q) terms[(size_t)r * 7 + q] = __builtin_nan("");
      }
      continue;
    }
    const double2 xi = X[i];
    double fx = 0.0, fy = 0.0;
    for (int64_t e = rowptr[i] + lane; e < rowptr[i + 1]; e += kWave) {
      const double2 xj = X[col[e]];
      const double dx = xi.x - xj.x, dy = xi.y - xj.y;
      const double pw = (double)val[e] / (1.0 + dx * dx + dy * dy);
      fx += pw * dx;
      fy += pw * dy;
    }
    fx = wave_sum(fx);
    fy = wave_sum(fy);
    if (lane == 0) {
      const int g = G == 1 ? 0 : graph_of(goff, G, i);
      const double Z = zg[g];
      const double ng = (double)gi[g].n;
      const double* pt = pairs + (size_t)r * 5;
      const double iz = Z > 0.0 ? 1.0 / Z : 0.0;
      double2 out;
      out.x = dp.lkl4 * (fx - pt[1] * iz) + dp.lc / ng * xi.x - dp.lr / (ng * ng) * pt[3];
      out.y = dp.lkl4 * (fy - pt[2] * iz) + dp.lc / ng * xi.y - dp.lr / (ng * ng) * pt[4];
      Gout[r] = out;
      if (terms) {
        double* t = terms + (size_t)r * 7;
        t[0] = fx;
        t[1] = fy;
        t[2] = pt[1];
        t[3] = pt[2];
        t[4] = pt[3];
        t[5] = pt[4];
        t[6] = pt[0];
      }
    }
  }
}

hipError_t launch_direct(Problem& P, const double2* X, const tsnet_params& prm, double2* G,
                         double* Z_out, const int* rows, int nrows, double* terms, double* pairs,
                         hipStream_t s) {
  const int per_block = 256 * kDirRows;
  // pairs: [nrows][5] row sums, then (with rows) [n][5] for the Z pass; sized by the caller
  double* zrows = rows ? pairs + (size_t)nrows * 5 : pairs;
  if (rows) {
    hipLaunchKernelGGL(k_direct_pairs, dim3((P.n + per_block - 1) / per_block), dim3(256), 0, s, X,
                       P.n, nullptr, P.n, P.goff_d, P.G, prm.eps_r, 1, zrows);
    hipLaunchKernelGGL(k_direct_pairs, dim3((nrows + per_block - 1) / per_block), dim3(256), 0, s,
                       X, P.n, rows, nrows, P.goff_d, P.G, prm.eps_r, 0, pairs);
  } else {
    hipLaunchKernelGGL(k_direct_pairs, dim3((P.n + per_block - 1) / per_block), dim3(256), 0, s, X,
                       P.n, nullptr, P.n, P.goff_d, P.G, prm.eps_r, 0, pairs);
  }
  hipLaunchKernelGGL(k_direct_z, dim3(P.G), dim3(256), 0, s, zrows, P.goff_d, P.G, P.zg, Z_out);
  DirParams dp{4.0 * prm.lambda_kl, prm.lambda_c, prm.lambda_r};
  int blocks = (nrows + 3) / 4;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_direct_attr, dim3(blocks), dim3(256), 0, s, X, P.n, P.rowptr, P.col, P.val, rows,
                     nrows, P.goff_d, P.G, P.ginfo, P.zg, pairs, dp, G, terms);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free entry point: the per-row pair sums live in a
// file-scope device array of kStaticScratchDoubles doubles (16 MiB), one copy
// per GPU for the life of the process. Host code never passes the array's
// name to a kernel: its device address comes from hipGetSymbolAddress, once
// per device with that device current, and is kept per device.
__device__ __align__(256) double scratch[kStaticScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

int static_scratch(int device, double** out) {
  if (device < 0 || device >= kMaxDevices) return fail(TSNET_EINVAL, "device id out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = 0;
    TSNET_HIP(hipGetDevice(&cur));
    TSNET_HIP(hipSetDevice(device));
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr)
      return fail(TSNET_EHIP, std::string("static scratch address: ") + hipGetErrorString(e));
    g_scratch_ptr[device] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[device];
  return TSNET_OK;
}

}  // namespace tsnet
