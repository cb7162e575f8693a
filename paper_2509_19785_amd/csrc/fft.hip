// FFT-accelerated node-to-node convolution (Sec. 2.3; Algorithm 3, "compute
// the sums ... using FFT-accelerated interpolation").
//
// Per graph the node grid is N_g x N_g (N_g = 3 n_int); the linear convolution
// with each kernel is embedded in an M x M circulant, M = 2 N_g = 3 * 2^b. The
// kernels are even in both axes, so their 2-D spectra are real.
//
//  rows_fwd: real rows -> half spectra. Charge rows pack (q0 + i q1) and
//            (q2 + i 0); kernel rows pack (K2 + i K1) and (Ke + i Kln) and are
//            generated on the fly (rows r and M - r coincide, so M/2 + 1 rows).
//  cols:     per frequency column: kernel columns (real, mirrored) -> real
//            kernel spectra; each charge column -> spectrum; products; inverse
//            column transforms of the 7 (8 with ln) outputs, rows < N_g kept.
//  rows_inv: pairs of output channels share one complex inverse row transform
//            (u + i v); the first N_g values of each row are the potentials,
//            scaled by 1 / M^2, stored node-major with 8 channels per node.
//
// All transforms are one Stockham autosort FFT over LDS with radix-4 passes,
// one radix-2 pass when b is odd, and a final radix-3 pass.
#include <hip/hip_runtime.h>

#include <cmath>

#include "dev_util.h"
#include "tsnet_internal.h"

namespace tsnet {

constexpr int kFftLds = 65536;  // bytes of LDS per block for every FFT kernel

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// nb sequences of length L (= 3 * 2^b, L | kMaxM) starting in `a`; `b` is the
// ping-pong buffer. sign = -1 forward, +1 inverse (unnormalised). Returns the
// buffer holding the result. Must be reached by every thread of the block.
__device__ float2* block_fft(float2* a, float2* b, int nb, int L, const float2* __restrict__ tw,
                             int sign) {
  int p2 = L / 3;
  int Ns = 1;
  const float s3 = 0.86602540378443864676f * (float)(-sign);  // sin(2 pi / 3) with direction
  while (Ns < L) {
    int R;
    if (p2 >= 4) {
      R = 4;
      p2 >>= 2;
    } else if (p2 == 2) {
      R = 2;
      p2 = 1;
    } else {
      R = 3;
    }
    const int nbut = L / R;
    const int tstep = kMaxM / (Ns * R);
    const int total = nb * nbut;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
      const int sq = idx / nbut;
      const int j = idx - sq * nbut;
      const float2* in = a + sq * L;
      float2* out = b + sq * L;
      const int k = j & (Ns - 1);  // Ns is a power of two before every pass
      float2 v[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (r < R) {
          float2 x = in[j + r * nbut];
          if (r > 0 && k > 0) {
            float2 w = tw[k * r * tstep];
            if (sign > 0) w.y = -w.y;
            x = cmul(x, w);
          }
          v[r] = x;
        }
      }
      const int base = (j - k) * R + k;
      if (R == 4) {
        const float2 t0 = make_float2(v[0].x + v[2].x, v[0].y + v[2].y);
        const float2 t1 = make_float2(v[0].x - v[2].x, v[0].y - v[2].y);
        const float2 t2 = make_float2(v[1].x + v[3].x, v[1].y + v[3].y);
        float2 t3 = make_float2(v[1].x - v[3].x, v[1].y - v[3].y);
        // multiply by -i (forward) or +i (inverse)
        t3 = sign < 0 ? make_float2(t3.y, -t3.x) : make_float2(-t3.y, t3.x);
        out[base] = make_float2(t0.x + t2.x, t0.y + t2.y);
        out[base + Ns] = make_float2(t1.x + t3.x, t1.y + t3.y);
        out[base + 2 * Ns] = make_float2(t0.x - t2.x, t0.y - t2.y);
        out[base + 3 * Ns] = make_float2(t1.x - t3.x, t1.y - t3.y);
      } else if (R == 2) {
        out[base] = make_float2(v[0].x + v[1].x, v[0].y + v[1].y);
        out[base + Ns] = make_float2(v[0].x - v[1].x, v[0].y - v[1].y);
      } else {
        const float2 t1 = make_float2(v[1].x + v[2].x, v[1].y + v[2].y);
        const float2 t2 = make_float2(v[1].x - v[2].x, v[1].y - v[2].y);
        const float2 m = make_float2(v[0].x - 0.5f * t1.x, v[0].y - 0.5f * t1.y);
        // n = sign * i * sin(2pi/3) * t2: forward -i s t2, inverse +i s t2
        const float2 nn = make_float2(s3 * t2.y, -s3 * t2.x);
        out[base] = make_float2(v[0].x + t1.x, v[0].y + t1.y);
        out[base + Ns] = make_float2(m.x + nn.x, m.y + nn.y);
        out[base + 2 * Ns] = make_float2(m.x - nn.x, m.y - nn.y);
      }
    }
    __syncthreads();
    float2* t = a;
    a = b;
    b = t;
    Ns *= R;
  }
  return a;
}

struct FftArgs {
  const GridDesc* desc;
  const float2* tw;
  const float* charges;
  size_t s_charges;
  float2* qspec;
  size_t s_qspec;
  float* kspec;
  size_t s_kspec;
  float2* ospec;
  size_t s_ospec;
  float* pot;
  size_t s_pot;
  float eps;
  int with_ln;
};

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fft_rows_fwd(FftArgs A) {
  extern __shared__ float2 lds[];
  const int g = blockIdx.y;
  const GridDesc d = A.desc[g];
  const int M = d.M, ng = d.ng, Mh = M / 2 + 1;
  const int capc = kFftLds / 16;  // complex values per ping-pong buffer
  float2* bufA = lds;
  float2* bufB = lds + capc;
  const int J = capc / (2 * M) > 0 ? capc / (2 * M) : 1;
  const int jobs = ng + Mh;
  const float* ch = A.charges + (size_t)g * A.s_charges;
  float2* qs = A.qspec + (size_t)g * A.s_qspec;
  float* ks = A.kspec + (size_t)g * A.s_kspec;
  const float sp = d.spacing;
  for (int j0 = blockIdx.x * J; j0 < jobs; j0 += gridDim.x * J) {
    const int nj = jobs - j0 < J ? jobs - j0 : J;
    for (int idx = threadIdx.x; idx < nj * 2 * M; idx += blockDim.x) {
      const int jl = idx / (2 * M);
      const int rem = idx - jl * 2 * M;
      const int sq = rem / M, x = rem - sq * M;
      const int job = j0 + jl;
      float2 v;
      if (job < ng) {
        const int ry = job;
        if (x < ng) {
          const size_t o = (size_t)ry * ng + x;
          v = sq == 0 ? make_float2(ch[o], ch[(size_t)ng * ng + o])
                      : make_float2(ch[2 * (size_t)ng * ng + o], 0.f);
        } else {
          v = make_float2(0.f, 0.f);
        }
      } else {
        const int ry = job - ng;
        const int xi = x < M - x ? x : M - x;
        const float dy = (float)ry * sp, dx = (float)xi * sp;
        const float r2 = dy * dy + dx * dx;
        if (sq == 0) {
          const float w = 1.0f / (1.0f + r2);
          v = make_float2(w * w, w);
        } else {
          v = make_float2(1.0f / (A.eps + r2), A.with_ln ? logf(A.eps + r2) : 0.f);
        }
      }
      bufA[jl * 2 * M + sq * M + x] = v;
    }
    __syncthreads();
    const float2* res = block_fft(bufA, bufB, nj * 2, M, A.tw, -1);
    for (int idx = threadIdx.x; idx < nj * Mh; idx += blockDim.x) {
      const int jl = idx / Mh;
      const int k = idx - jl * Mh;
      const int km = k == 0 ? 0 : M - k;
      const float2* s0 = res + jl * 2 * M;
      const float2* s1 = s0 + M;
      const int job = j0 + jl;
      const float2 a = s0[k], ar = s0[km];
      if (job < ng) {
        const int ry = job;
        // Q0 = (A_k + conj A_{M-k}) / 2,  Q1 = -i (A_k - conj A_{M-k}) / 2
        const float2 q0 = make_float2(0.5f * (a.x + ar.x), 0.5f * (a.y - ar.y));
        const float2 q1 = make_float2(0.5f * (a.y + ar.y), -0.5f * (a.x - ar.x));
        qs[((size_t)0 * ng + ry) * Mh + k] = q0;
        qs[((size_t)1 * ng + ry) * Mh + k] = q1;
        qs[((size_t)2 * ng + ry) * Mh + k] = s1[k];
      } else {
        const int ry = job - ng;
        const float2 b = s1[k], br = s1[km];
        ks[((size_t)0 * Mh + ry) * Mh + k] = 0.5f * (a.x + ar.x);
        ks[((size_t)1 * Mh + ry) * Mh + k] = 0.5f * (a.y + ar.y);
        ks[((size_t)2 * Mh + ry) * Mh + k] = 0.5f * (b.x + br.x);
        ks[((size_t)3 * Mh + ry) * Mh + k] = 0.5f * (b.y + br.y);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fft_cols(FftArgs A) {
  extern __shared__ float2 lds[];
  const int g = blockIdx.y;
  const GridDesc d = A.desc[g];
  const int M = d.M, ng = d.ng, Mh = M / 2 + 1;
  int nc = kFftLds / (40 * M);
  if (nc < 1) nc = 1;
  float* khat = reinterpret_cast<float*>(lds);           // [4][nc][M]
  float2* B0 = lds + (size_t)2 * nc * M;                  // after 4 nc M floats
  float2* B1 = B0 + (size_t)nc * M;
  float2* B2 = B1 + (size_t)nc * M;
  const float2* qs = A.qspec + (size_t)g * A.s_qspec;
  const float* ks = A.kspec + (size_t)g * A.s_kspec;
  float2* os = A.ospec + (size_t)g * A.s_ospec;
  const int nout0 = A.with_ln ? 4 : 3;
  for (int c0 = blockIdx.x * nc; c0 < Mh; c0 += gridDim.x * nc) {
    const int ncc = Mh - c0 < nc ? Mh - c0 : nc;
    // kernel spectra: two packed real columns per transform
    for (int pair = 0; pair < 2; ++pair) {
      for (int idx = threadIdx.x; idx < ncc * M; idx += blockDim.x) {
        const int y = idx / ncc, col = idx - y * ncc;
        const int ry = y < M - y ? y : M - y;
        const size_t o = (size_t)ry * Mh + c0 + col;
        B0[col * M + y] = make_float2(ks[(size_t)(2 * pair) * Mh * Mh + o],
                                      ks[(size_t)(2 * pair + 1) * Mh * Mh + o]);
      }
      __syncthreads();
      const float2* r = block_fft(B0, B1, ncc, M, A.tw, -1);
      for (int idx = threadIdx.x; idx < ncc * M; idx += blockDim.x) {
        const float2 v = r[idx];
        khat[(size_t)(2 * pair) * nc * M + idx] = v.x;
        khat[(size_t)(2 * pair + 1) * nc * M + idx] = v.y;
      }
      __syncthreads();
    }
    for (int c = 0; c < 3; ++c) {
      for (int idx = threadIdx.x; idx < ncc * M; idx += blockDim.x) {
        const int y = idx / ncc, col = idx - y * ncc;
        B0[col * M + y] = y < ng ? qs[((size_t)c * ng + y) * Mh + c0 + col] : make_float2(0.f, 0.f);
      }
      __syncthreads();
      const float2* Q = block_fft(B0, B1, ncc, M, A.tw, -1);
      float2* fr = Q == B0 ? B1 : B0;
      const int nout = c == 0 ? nout0 : 2;
      for (int t = 0; t < nout; ++t) {
        int o, kk;
        if (c == 0) {
          const int oo[4] = {CH_K2_1, CH_K1_1, CH_KE_1, CH_KLN_1};
          const int kq[4] = {0, 1, 2, 3};
          o = oo[t];
          kk = kq[t];
        } else {
          o = t == 0 ? (c == 1 ? CH_K2_X : CH_K2_Y) : (c == 1 ? CH_KE_X : CH_KE_Y);
          kk = t == 0 ? 0 : 2;
        }
        const float* kh = khat + (size_t)kk * nc * M;
        for (int idx = threadIdx.x; idx < ncc * M; idx += blockDim.x) {
          const float2 q = Q[idx];
          const float kv = kh[idx];
          fr[idx] = make_float2(kv * q.x, kv * q.y);
        }
        __syncthreads();
        const float2* r = block_fft(fr, B2, ncc, M, A.tw, +1);
        for (int idx = threadIdx.x; idx < ncc * ng; idx += blockDim.x) {
          const int y = idx / ncc, col = idx - y * ncc;
          os[((size_t)o * ng + y) * Mh + c0 + col] = r[col * M + y];
        }
        __syncthreads();
      }
    }
  }
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fft_rows_inv(FftArgs A) {
  extern __shared__ float2 lds[];
  const int g = blockIdx.y;
  const GridDesc d = A.desc[g];
  const int M = d.M, ng = d.ng, Mh = M / 2 + 1;
  const int capc = kFftLds / 16;
  float2* bufA = lds;
  float2* bufB = lds + capc;
  const int J = capc / M;
  const int jobs = ng * 4;
  const float2* os = A.ospec + (size_t)g * A.s_ospec;
  float* pg = A.pot + (size_t)g * A.s_pot;
  const float scale = 1.0f / ((float)M * (float)M);
  for (int j0 = blockIdx.x * J; j0 < jobs; j0 += gridDim.x * J) {
    const int nj = jobs - j0 < J ? jobs - j0 : J;
    for (int idx = threadIdx.x; idx < nj * M; idx += blockDim.x) {
      const int jl = idx / M, k = idx - jl * M;
      const int job = j0 + jl;
      const int ry = job >> 2, pr = job & 3;
      const int o0 = 2 * pr, o1 = 2 * pr + 1;
      const bool conj_ = k > M / 2;
      const int kk = conj_ ? M - k : k;
      float2 f0 = os[((size_t)o0 * ng + ry) * Mh + kk];
      float2 f1 = (o1 == CH_KLN_1 && !A.with_ln) ? make_float2(0.f, 0.f)
                                                  : os[((size_t)o1 * ng + ry) * Mh + kk];
      if (conj_) {
        f0.y = -f0.y;
        f1.y = -f1.y;
      }
      bufA[jl * M + k] = make_float2(f0.x - f1.y, f0.y + f1.x);
    }
    __syncthreads();
    const float2* res = block_fft(bufA, bufB, nj, M, A.tw, +1);
    for (int idx = threadIdx.x; idx < nj * ng; idx += blockDim.x) {
      const int jl = idx / ng, x = idx - jl * ng;
      const int job = j0 + jl;
      const int ry = job >> 2, pr = job & 3;
      const float2 v = res[jl * M + x];
      *reinterpret_cast<float2*>(pg + ((size_t)ry * ng + x) * kPotCh + 2 * pr) =
          make_float2(v.x * scale, v.y * scale);
    }
    __syncthreads();
  }
}

hipError_t launch_fft_conv(Problem& P, float eps, int with_ln, hipStream_t s) {
  FftArgs A;
  A.desc = P.desc;
  A.tw = P.ctx->twiddle;
  A.charges = P.charges;
  A.s_charges = P.stride_charges;
  A.qspec = P.qspec;
  A.s_qspec = P.stride_qspec;
  A.kspec = P.kspec;
  A.s_kspec = P.stride_kspec;
  A.ospec = P.ospec;
  A.s_ospec = P.stride_ospec;
  A.pot = P.pot;
  A.s_pot = P.stride_pot;
  A.eps = eps;
  A.with_ln = with_ln;
  const int bx = P.G >= 64 ? 4 : (P.G >= 8 ? 32 : 256);
  hipLaunchKernelGGL(k_fft_rows_fwd, dim3(bx, P.G), dim3(256), kFftLds, s, A);
  hipLaunchKernelGGL(k_fft_cols, dim3(bx, P.G), dim3(256), kFftLds, s, A);
  hipLaunchKernelGGL(k_fft_rows_inv, dim3(bx, P.G), dim3(256), kFftLds, s, A);
  return hipGetLastError();
}

}  // namespace tsnet
