// FFT-accelerated node-to-node convolution (Sec. 2.3; Algorithm 3, "compute
// the sums ... using FFT-accelerated interpolation").
//
// Per graph the node grid is N_g x N_g (N_g = 3 n_int); the linear convolution
// with each kernel is embedded in an M x M circulant, M = 2 N_g = 3 * 2^b. The
// kernels are even in both axes, so their 2-D spectra are real. Every
// transform runs along contiguous memory; tiled transposes sit between the
// row and column stages:
//
//  rows_fwd:  real rows -> half spectra Qr[c][y][kx] (charges 1, x, y packed
//             as q0 + i q1 and q2) and Kr[k][y][kx] (kernels generated on the
//             fly, packed as K2 + i K1 and Ke + i Kln; rows y and M - y
//             coincide, so only y <= M/2).
//  transpose: Qr -> Qt[c][kx][y], Kr -> Kt[k][kx][y].
//  cols:      per frequency column kx: the mirrored kernel columns give the
//             real kernel spectra (kept in registers); each charge column is
//             transformed (kept in registers), multiplied by its kernels and
//             transformed back; rows < N_g of the 7 (8 with ln) outputs go to
//             Ot[o][kx][y].
//  transpose: Ot -> Or[o][y][kx].
//  rows_inv:  two output channels share one complex inverse row transform
//             (u + i v); the first N_g values of each row, times 1 / M^2, are
//             the node potentials, stored as 4 planes (one per channel pair) of
//             N_g x N_g float2 nodes, so each row transform writes contiguously.
//
// The transforms are Stockham autosort FFTs over LDS (fft_core.h): radix-16
// passes (the last power-of-two pass 8, 4 or 2) and one radix-12 pass, each
// butterfly an in-register DFT; every pass reads the buffer into registers,
// synchronises and writes back in place. Each block owns one padded LDS
// buffer of C::Elems complex values and the first M / 2 twiddles of its
// transform length (copied from the context's table once per block);
// sequences of length M share a block up to C::Elems / M at a time (fewer
// when there are fewer sequences than blocks, so small grids stay spread).
#include <hip/hip_runtime.h>

#include <cmath>

#include "dev_util.h"
#include "fft_core.h"
#include "tsnet_internal.h"

namespace tsnet {

// A size class of the transform kernels: buffer length E complex values and
// T threads per block, so every thread holds E / T slots in registers (12 in
// both classes). The small class takes every length up to 3072 (512
// intervals); the large class only 6144 (1024 intervals), with twice the
// threads and 75 KB of LDS per block. Each kernel is instantiated per class
// and a block returns at once when its graph's length belongs to the other.
template <int E, int T>
struct FftCfg {
  static constexpr int Elems = E;              // complex values per transform buffer
  static constexpr int Threads = T;
  static constexpr int Buf = E + E / 16;       // the buffer, padded (one spare slot per 16)
  static constexpr int Lds = (Buf + E / 2) * 8;  // bytes of LDS per block: buffer + half twiddles
  static constexpr int PerThread = E / T;      // register slots per thread
  __device__ static bool handles(int M) { return E > kFftSmallM ? M > kFftSmallM : M <= kFftSmallM; }
};
using FftSmall = FftCfg<kFftSmallM, 256>;
using FftLarge = FftCfg<kMaxM, 512>;
constexpr int kColBatch = 4;  // loads in flight per thread in the column stage
static_assert(FftSmall::PerThread % kColBatch == 0 && FftLarge::PerThread % kColBatch == 0,
              "whole batches");

// e^{-2 pi i m / L}, 0 <= m < L, from the half table th[r] = e^{-2 pi i r / L},
// r < L / 2 (the second half is the negated first half).
template <int L>
__device__ __forceinline__ float2 twh(const float2* th, int m) {
  constexpr int h = L / 2;
  const bool hi = m >= h;
  const float2 t = th[hi ? m - h : m];
  return hi ? make_float2(-t.x, -t.y) : t;
}

// One Stockham pass of radix R over sub-length NS, in place: every thread
// reads and transforms its butterflies into registers, the block
// synchronises, then the results are written back to the same buffer.
// Index arithmetic as in fft_pass (fft_core.h); where the input stride L/R
// and the output stride NS are multiples of 16 the padded addresses are a
// base plus constant offsets. INV: inverse transform (conjugate twiddles),
// fixed at compile time so the sign folds into the arithmetic.
template <int R, int L, int NS, bool INV, class C>
__device__ __forceinline__ void pass_ip(float2* buf, int nb, const float2* th) {
  constexpr float sgn = INV ? 1.f : -1.f;
  constexpr int nbut = L / R;
  constexpr int tstep = L / (NS * R);
  constexpr int BPT = (C::Elems / R + C::Threads - 1) / C::Threads;
  constexpr bool in_lin = nbut % 16 == 0;
  constexpr bool out_lin = NS % 16 == 0 || (NS == 1 && R == 16);
  const int total = nb * nbut;
  float2 v[BPT][R];
  int ob[BPT];
#pragma unroll
  for (int u = 0; u < BPT; ++u) {
    const int idx = threadIdx.x + u * C::Threads;
    ob[u] = -1;
    if (idx < total) {
      const int sq = idx / nbut, j = idx - sq * nbut, k = j & (NS - 1);
      const int ib = sq * L + j;
      if constexpr (in_lin) {
        const float2* p = buf + fft_pad(ib);
#pragma unroll
        for (int r = 0; r < R; ++r) v[u][r] = p[r * (nbut + nbut / 16)];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) v[u][r] = buf[fft_pad(ib + r * nbut)];
      }
      if (k > 0) {  // k r tstep < NS R tstep = L
#pragma unroll
        for (int r = 1; r < R; ++r) {
          float2 w = twh<L>(th, k * r * tstep);
          if constexpr (INV) w.y = -w.y;
          v[u][r] = fmulc(v[u][r], w);
        }
      }
      small_dft<R>(v[u], sgn);
      ob[u] = sq * L + (j - k) * R + k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < BPT; ++u) {
    if (ob[u] < 0) continue;
    if constexpr (out_lin) {
      float2* p = buf + fft_pad(ob[u]);
#pragma unroll
      for (int r = 0; r < R; ++r) p[r * (NS + NS / 16)] = v[u][r];
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) buf[fft_pad(ob[u] + r * NS)] = v[u][r];
    }
  }
  __syncthreads();
}

// The passes of fft_plan for a length known at compile time.
template <int L, int NS, int P2, bool INV, class C>
struct FftPasses {
  __device__ __forceinline__ static void run(float2* buf, int nb, const float2* th) {
    if constexpr (P2 > 1) {
      constexpr int R = P2 >= 16 ? 16 : P2;
      pass_ip<R, L, NS, INV, C>(buf, nb, th);
      FftPasses<L, NS * R, P2 / R, INV, C>::run(buf, nb, th);
    } else {
      pass_ip<L / NS, L, NS, INV, C>(buf, nb, th);  // the radix-12 (6, 3) pass
    }
  }
};

// One length and direction per function, not inlined into the callers: the
// kernels pick the length at run time (it comes from the grid plan on the
// device), and inlining every length into one body inflates the register
// allocation.
template <int L, bool INV, class C>
__device__ __noinline__ void fft_len(float2* buf, int nb, const float2* th) {
  constexpr int p2 = L / 3;
  constexpr int r3 = p2 >= 4 ? 12 : (p2 == 2 ? 6 : 3);
  FftPasses<L, 1, p2 / (r3 / 3), INV, C>::run(buf, nb, th);
}

template <bool INV, class C>
__device__ void block_fft_dir(float2* buf, int nb, int L, const float2* th) {
  if constexpr (C::Elems > kFftSmallM) {  // the large class has one length
    fft_len<C::Elems, INV, C>(buf, nb, th);
  } else {
    switch (L) {
      case 3072: fft_len<3072, INV, C>(buf, nb, th); break;
      case 1536: fft_len<1536, INV, C>(buf, nb, th); break;
      case 768: fft_len<768, INV, C>(buf, nb, th); break;
      case 384: fft_len<384, INV, C>(buf, nb, th); break;
      case 192: fft_len<192, INV, C>(buf, nb, th); break;
      case 96: fft_len<96, INV, C>(buf, nb, th); break;
      case 48: fft_len<48, INV, C>(buf, nb, th); break;
      case 24: fft_len<24, INV, C>(buf, nb, th); break;
      case 12: fft_len<12, INV, C>(buf, nb, th); break;
      default: fft_len<6, INV, C>(buf, nb, th); break;
    }
  }
}

// nb sequences of length L (= 6 * 2^a <= C::Elems, nb L <= C::Elems) at
// buf[pad(s L + i)], transformed in place; th is the half twiddle table of
// length L in LDS. sgn = -1 forward, +1 inverse (unnormalised). Must be
// reached by every thread of the block.
template <class C>
__device__ __forceinline__ void block_fft(float2* buf, int nb, int L, const float2* th, float sgn) {
  if (sgn > 0.f)
    block_fft_dir<true, C>(buf, nb, L, th);
  else
    block_fft_dir<false, C>(buf, nb, L, th);
}

// The first half of the twiddles of length M from the context table (length
// kMaxM) into LDS.
__device__ __forceinline__ void load_twiddles(float2* th, const float2* __restrict__ tw, int M) {
  const int step = kMaxM / M;
  for (int m = threadIdx.x; m < (M >> 1); m += blockDim.x) th[m] = tw[m * step];
}

// Sequences per block iteration for `jobs` sequences of length M: as many as
// the buffer holds, but few enough that the jobs still reach about one block
// per compute unit (256), or every block of a smaller grid. Small transforms
// then keep many blocks busy instead of a few full ones; at M = 1536 the
// column stage measured faster with 2 columns per block (385 blocks) than
// with 1 (769 blocks), so the target is the CU count, not the grid.
template <class C>
__device__ __forceinline__ int fft_pack(int M, int jobs) {
  constexpr int kSpreadBlocks = 256;
  const int smax = C::Elems / M;
  const int target = (int)gridDim.x < kSpreadBlocks ? (int)gridDim.x : kSpreadBlocks;
  const int want = jobs / target;
  return want < 1 ? 1 : (want < smax ? want : smax);
}

struct FftArgs {
  const GridDesc* desc;
  const float2* tw;
  // pools; every graph's part starts at its GridDesc offsets
  const float* charges;
  float2* qr;   // [3][ng][Mh]
  float2* qt;   // [3][Mh][ng]
  float* kr;    // [4][Mh][Mh]
  float* kt;    // [4][Mh][Mh] transposed
  float2* ot;   // [8][Mh][ng]
  float2* orr;  // [8][ng][Mh]
  float* pot;
  float eps;
  int with_ln;
};

// ---------------------------------------------------------------------------
// Row transforms of the charges and kernels. Sequence s of a graph:
//   s < 2 ng:        charge row s / 2, part s % 2 (0: q0 + i q1, 1: q2)
//   otherwise:       kernel row (s - 2 ng) / 2 in [0, M/2], part (0: K2 + i K1, 1: Ke + i Kln)
template <class C>
__global__ __launch_bounds__(C::Threads, 4) void k_fft_rows_fwd(FftArgs A) {
  extern __shared__ float2 lds[];
  const int g = blockIdx.y;
  const GridDesc d = A.desc[g];
  const int M = d.M, ng = d.ng, Mh = M / 2 + 1;
  if (!C::handles(M)) return;  // the other size class transforms this graph
  float2* bufA = lds;
  float2* twl = lds + C::Buf;  // half twiddle table
  load_twiddles(twl, A.tw, M);
  const int nseq = 2 * ng + 2 * Mh;
  const int S = fft_pack<C>(M, nseq);  // sequences per block iteration
  const float* ch = A.charges + d.off_c;
  float2* qs = A.qr + d.off_q;
  float* ks = A.kr + d.off_k;
  const float sp = d.spacing;
  for (int s0 = blockIdx.x * S; s0 < nseq; s0 += gridDim.x * S) {
    const int ns = nseq - s0 < S ? nseq - s0 : S;
    if (s0 + ns <= 2 * ng) {
      // charge rows only: every load is issued before any is used
      float2 vin[C::PerThread];
#pragma unroll
      for (int q = 0; q < C::PerThread; ++q) {
        const int idx = threadIdx.x + q * C::Threads;
        vin[q] = make_float2(0.f, 0.f);
        if (idx >= ns * M) continue;
        const int sl = idx / M, x = idx - sl * M;
        const int sq = s0 + sl;
        const int ry = sq >> 1, part = sq & 1;
        if (x < ng) {
          const size_t o = (size_t)ry * ng + x;
          vin[q] = part == 0 ? make_float2(ch[o], ch[(size_t)ng * ng + o])
                             : make_float2(ch[2 * (size_t)ng * ng + o], 0.f);
        }
      }
#pragma unroll
      for (int q = 0; q < C::PerThread; ++q) {
        const int idx = threadIdx.x + q * C::Threads;
        if (idx < ns * M) bufA[fft_pad(idx)] = vin[q];
      }
    } else {
      for (int idx = threadIdx.x; idx < ns * M; idx += blockDim.x) {
        const int sl = idx / M, x = idx - sl * M;
        const int sq = s0 + sl;
        float2 v;
        if (sq < 2 * ng) {
          const int ry = sq >> 1, part = sq & 1;
          if (x < ng) {
            const size_t o = (size_t)ry * ng + x;
            v = part == 0 ? make_float2(ch[o], ch[(size_t)ng * ng + o])
                          : make_float2(ch[2 * (size_t)ng * ng + o], 0.f);
          } else {
            v = make_float2(0.f, 0.f);
          }
        } else {  // kernel rows, generated
          const int t = sq - 2 * ng;
          const int ry = t >> 1, part = t & 1;
          const int xi = x < M - x ? x : M - x;
          const float dy = (float)ry * sp, dx = (float)xi * sp;
          const float r2 = dy * dy + dx * dx;
          if (part == 0) {
            const float w = 1.0f / (1.0f + r2);
            v = make_float2(w * w, w);
          } else {
            v = make_float2(1.0f / (A.eps + r2), A.with_ln ? logf(A.eps + r2) : 0.f);
          }
        }
        bufA[fft_pad(idx)] = v;
      }
    }
    __syncthreads();
    block_fft<C>(bufA, ns, M, twl, -1.f);
    const float2* res = bufA;
    for (int idx = threadIdx.x; idx < ns * Mh; idx += blockDim.x) {
      const int sl = idx / Mh, k = idx - sl * Mh;
      const int km = k == 0 ? 0 : M - k;
      const float2 a = res[fft_pad(sl * M + k)], ar = res[fft_pad(sl * M + km)];
      const int sq = s0 + sl;
      if (sq < 2 * ng) {
        const int ry = sq >> 1, part = sq & 1;
        if (part == 0) {
          // Q0 = (A_k + conj A_{M-k}) / 2,  Q1 = -i (A_k - conj A_{M-k}) / 2
          qs[((size_t)0 * ng + ry) * Mh + k] = make_float2(0.5f * (a.x + ar.x), 0.5f * (a.y - ar.y));
          qs[((size_t)1 * ng + ry) * Mh + k] = make_float2(0.5f * (a.y + ar.y), -0.5f * (a.x - ar.x));
        } else {
          qs[((size_t)2 * ng + ry) * Mh + k] = a;
        }
      } else {
        const int t = sq - 2 * ng;
        const int ry = t >> 1, part = t & 1;
        // real spectra of the two packed even rows
        ks[((size_t)(2 * part) * Mh + ry) * Mh + k] = 0.5f * (a.x + ar.x);
        ks[((size_t)(2 * part + 1) * Mh + ry) * Mh + k] = 0.5f * (a.y + ar.y);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Tiled transposes in[b][r][c] -> out[b][c][r], r < R, c < C (sizes per graph).
// Blocks b0, b0 + nblk, ... of the launch take kTrTiles consecutive tiles of
// 32 x 32 at a time: every thread issues its loads of all of them (clamped
// into the array, unconditional) before any is used, then the tiles go
// through LDS and out along the other axis.
constexpr int kTrTiles = 2;

template <typename T>
__device__ __forceinline__ void transpose_tiles(const T* __restrict__ in, T* out, int R, int C,
                                                int nb, T (*tile)[32][33], int b0, int nblk) {
  const int tilesR = (R + 31) / 32, tilesC = (C + 31) / 32;
  const int per = tilesR * tilesC;
  const int total = nb * per;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
  const size_t last = (size_t)nb * R * C - 1;
  for (int t0 = b0 * kTrTiles; t0 < total; t0 += nblk * kTrTiles) {
    T v[kTrTiles][4];
#pragma unroll
    for (int u = 0; u < kTrTiles; ++u) {
      const int t = min(t0 + u, total - 1);
      const int b = t / per, rem = t - b * per;
      const int tr = rem / tilesC, tc = rem - tr * tilesC;
      const int c = min(tc * 32 + tx, C - 1);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int r = min(tr * 32 + ty + 8 * k, R - 1);
        v[u][k] = in[min((size_t)b * R * C + (size_t)r * C + c, last)];
      }
    }
#pragma unroll
    for (int u = 0; u < kTrTiles; ++u)
#pragma unroll
      for (int k = 0; k < 4; ++k) tile[u][ty + 8 * k][tx] = v[u][k];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kTrTiles; ++u) {
      const int t = t0 + u;
      if (t >= total) break;
      const int b = t / per, rem = t - b * per;
      const int tr = rem / tilesC, tc = rem - tr * tilesC;
      T* ob = out + (size_t)b * R * C;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int c = tc * 32 + ty + 8 * k, r = tr * 32 + tx;
        if (r < R && c < C) ob[(size_t)c * R + r] = tile[u][tx][ty + 8 * k];
      }
    }
    __syncthreads();
  }
}

// which = 0: Qr -> Qt (the first half of the blocks) and Kr -> Kt (the
// second half), one launch; which = 2: Ot -> Or.
__global__ __launch_bounds__(256) void k_fft_transpose(FftArgs A, int which) {
  const int g = blockIdx.y;
  const GridDesc d = A.desc[g];
  const int ng = d.ng, Mh = d.M / 2 + 1;
  __shared__ float2 tc[kTrTiles][32][33];
  if (which == 0) {
    const int half = gridDim.x / 2;
    if ((int)blockIdx.x < half) {
      transpose_tiles<float2>(A.qr + d.off_q, A.qt + d.off_q, ng, Mh, 3, tc,
                              blockIdx.x, half);
    } else {
      float (*tf)[32][33] = reinterpret_cast<float (*)[32][33]>(&tc[0][0][0]);
      transpose_tiles<float>(A.kr + d.off_k, A.kt + d.off_k, Mh, Mh, 4, tf,
                             blockIdx.x - half, gridDim.x - half);
    }
  } else {
    transpose_tiles<float2>(A.ot + d.off_o, A.orr + d.off_o, Mh, ng,
                            A.with_ln ? 8 : 7, tc, blockIdx.x, gridDim.x);
  }
}

// The products of a column group: output channel, kernel (K2, K1, Ke, Kln)
// and charge (1, x, y) of each, in the order the column stage forms them.
__device__ __forceinline__ void product_of(int t, int& o, int& kk, int& c) {
  switch (t) {
    case 0: o = CH_K2_1; kk = 0; c = 0; break;
    case 1: o = CH_K1_1; kk = 1; c = 0; break;
    case 2: o = CH_KE_1; kk = 2; c = 0; break;
    case 3: o = CH_K2_X; kk = 0; c = 1; break;
    case 4: o = CH_KE_X; kk = 2; c = 1; break;
    case 5: o = CH_K2_Y; kk = 0; c = 2; break;
    case 6: o = CH_KE_Y; kk = 2; c = 2; break;
    default: o = CH_KLN_1; kk = 3; c = 0; break;
  }
}

// Column stage for a column group whose every transform fits the buffer at
// once (8 ncc M <= C::Elems: small grids of a single graph, one column per
// block): the two kernel-spectrum transforms run as one batch, the three
// charge transforms as another and the 7 (8 with ln) inverse transforms of
// the products as a third, instead of one call per transform. Each
// transform is the same sequence of passes as in the unbatched path, so
// the results are the same bit for bit.
template <class C>
__device__ __noinline__ void cols_batched(const FftArgs& A, float2* B0, const float2* twl,
                                             int M, int ng, int Mh, int c0, int ncc,
                                             const float2* qt, const float* kt, float2* ot) {
  constexpr int PB = (C::PerThread + 7) / 8;  // a thread's elements of one column group
  const int tot = ncc * M;
  const int nout = A.with_ln ? 8 : 7;
  // kernel spectra, pair p at sequences [p ncc, (p + 1) ncc)
  for (int e = threadIdx.x; e < 2 * tot; e += C::Threads) {
    const int pair = e >= tot, r = e - pair * tot;
    const int col = r / M, y = r - col * M;
    const int ry = y < M - y ? y : M - y;
    const size_t o = (size_t)(c0 + col) * Mh + ry;
    B0[fft_pad(e)] = make_float2(kt[(size_t)(2 * pair) * Mh * Mh + o], kt[(size_t)(2 * pair + 1) * Mh * Mh + o]);
  }
  __syncthreads();
  block_fft<C>(B0, 2 * ncc, M, twl, -1.f);
  float kh[4][PB];
#pragma unroll
  for (int q = 0; q < PB; ++q) {
    const int idx = threadIdx.x + q * C::Threads;
    const float2 v0 = idx < tot ? B0[fft_pad(idx)] : make_float2(0.f, 0.f);
    const float2 v1 = idx < tot ? B0[fft_pad(tot + idx)] : make_float2(0.f, 0.f);
    kh[0][q] = v0.x;
    kh[1][q] = v0.y;
    kh[2][q] = v1.x;
    kh[3][q] = v1.y;
  }
  __syncthreads();
  // charges 1, x, y at sequences [c ncc, (c + 1) ncc)
  for (int e = threadIdx.x; e < 3 * tot; e += C::Threads) {
    const int c = e / tot, r = e - c * tot;
    const int col = r / M, y = r - col * M;
    B0[fft_pad(e)] = y < ng ? qt[((size_t)c * Mh + c0 + col) * ng + y] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  block_fft<C>(B0, 3 * ncc, M, twl, -1.f);
  float2 qh[3][PB];
#pragma unroll
  for (int q = 0; q < PB; ++q) {
    const int idx = threadIdx.x + q * C::Threads;
#pragma unroll
    for (int c = 0; c < 3; ++c)
      qh[c][q] = idx < tot ? B0[fft_pad(c * tot + idx)] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  // products, output t at sequences [t ncc, (t + 1) ncc), then one inverse batch
  for (int t = 0; t < nout; ++t) {
    int o, kk, c;
    product_of(t, o, kk, c);
#pragma unroll
    for (int q = 0; q < PB; ++q) {
      const int idx = threadIdx.x + q * C::Threads;
      if (idx >= tot) continue;
      const float kv = kk == 0 ? kh[0][q] : (kk == 1 ? kh[1][q] : (kk == 2 ? kh[2][q] : kh[3][q]));
      const float2 qv = c == 0 ? qh[0][q] : (c == 1 ? qh[1][q] : qh[2][q]);
      B0[fft_pad(t * tot + idx)] = make_float2(kv * qv.x, kv * qv.y);
    }
  }
  __syncthreads();
  block_fft<C>(B0, nout * ncc, M, twl, +1.f);
  for (int e = threadIdx.x; e < nout * ncc * ng; e += C::Threads) {
    const int t = e / (ncc * ng), r = e - t * (ncc * ng);
    const int col = r / ng, y = r - col * ng;
    int o, kk, c;
    product_of(t, o, kk, c);
    ot[((size_t)o * Mh + c0 + col) * ng + y] = B0[fft_pad(t * tot + col * M + y)];
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
template <class C>
__global__ __launch_bounds__(C::Threads, 3) void k_fft_cols(FftArgs A) {
  extern __shared__ float2 lds[];
  const int g = blockIdx.y;
  const GridDesc d = A.desc[g];
  const int M = d.M, ng = d.ng, Mh = M / 2 + 1;
  if (!C::handles(M)) return;  // the other size class transforms this graph
  const int S = fft_pack<C>(M, Mh);  // columns per block iteration
  float2* B0 = lds;
  float2* twl = lds + C::Buf;  // half twiddle table
  load_twiddles(twl, A.tw, M);
  const float2* qt = A.qt + d.off_q;
  const float* kt = A.kt + d.off_k;
  float2* ot = A.ot + d.off_o;
  const int nout0 = A.with_ln ? 4 : 3;
  if (8 * S * M <= C::Elems) {  // every transform of a column group fits at once
    for (int c0 = blockIdx.x * S; c0 < Mh; c0 += gridDim.x * S)
      cols_batched<C>(A, B0, twl, M, ng, Mh, c0, Mh - c0 < S ? Mh - c0 : S, qt, kt, ot);
    return;
  }
  for (int c0 = blockIdx.x * S; c0 < Mh; c0 += gridDim.x * S) {
    const int ncc = Mh - c0 < S ? Mh - c0 : S;
    const int tot = ncc * M;
    float kh[4][C::PerThread];
    // kernel spectra: two packed real columns per transform, kept in registers
    for (int pair = 0; pair < 2; ++pair) {
      // loads in groups of kColBatch in flight (registers are scarce here)
#pragma unroll 1
      for (int q0 = 0; q0 < C::PerThread; q0 += kColBatch) {
        float2 t[kColBatch];
#pragma unroll
        for (int j = 0; j < kColBatch; ++j) {
          const int idx = threadIdx.x + (q0 + j) * C::Threads;
          if (idx >= tot) continue;
          const int col = idx / M, y = idx - col * M;
          const int ry = y < M - y ? y : M - y;
          const size_t o = (size_t)(c0 + col) * Mh + ry;
          t[j] = make_float2(kt[(size_t)(2 * pair) * Mh * Mh + o], kt[(size_t)(2 * pair + 1) * Mh * Mh + o]);
        }
#pragma unroll
        for (int j = 0; j < kColBatch; ++j) {
          const int idx = threadIdx.x + (q0 + j) * C::Threads;
          if (idx < tot) B0[fft_pad(idx)] = t[j];
        }
      }
      __syncthreads();
      block_fft<C>(B0, ncc, M, twl, -1.f);
      const float2* r = B0;
#pragma unroll
      for (int q = 0; q < C::PerThread; ++q) {
        const int idx = threadIdx.x + q * C::Threads;
        const float2 v = idx < tot ? r[fft_pad(idx)] : make_float2(0.f, 0.f);
        kh[2 * pair][q] = v.x;
        kh[2 * pair + 1][q] = v.y;
      }
      __syncthreads();
    }
    for (int c = 0; c < 3; ++c) {
#pragma unroll 1
      for (int q0 = 0; q0 < C::PerThread; q0 += kColBatch) {
        float2 t[kColBatch];
#pragma unroll
        for (int j = 0; j < kColBatch; ++j) {
          const int idx = threadIdx.x + (q0 + j) * C::Threads;
          const int col = idx / M, y = idx - col * M;
          t[j] = (idx < tot && y < ng) ? qt[((size_t)c * Mh + c0 + col) * ng + y] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int j = 0; j < kColBatch; ++j) {
          const int idx = threadIdx.x + (q0 + j) * C::Threads;
          if (idx < tot) B0[fft_pad(idx)] = t[j];
        }
      }
      __syncthreads();
      block_fft<C>(B0, ncc, M, twl, -1.f);
      const float2* Q = B0;
      float2 qh[C::PerThread];
#pragma unroll
      for (int q = 0; q < C::PerThread; ++q) {
        const int idx = threadIdx.x + q * C::Threads;
        qh[q] = idx < tot ? Q[fft_pad(idx)] : make_float2(0.f, 0.f);
      }
      __syncthreads();
      const int nout = c == 0 ? nout0 : 2;
      for (int t = 0; t < nout; ++t) {
        int o, kk;
        if (c == 0) {
          o = t == 0 ? CH_K2_1 : (t == 1 ? CH_K1_1 : (t == 2 ? CH_KE_1 : CH_KLN_1));
          kk = t;
        } else {
          o = t == 0 ? (c == 1 ? CH_K2_X : CH_K2_Y) : (c == 1 ? CH_KE_X : CH_KE_Y);
          kk = t == 0 ? 0 : 2;
        }
#pragma unroll
        for (int q = 0; q < C::PerThread; ++q) {
          const int idx = threadIdx.x + q * C::Threads;
          if (idx < tot) {
            const float kv = kk == 0 ? kh[0][q] : (kk == 1 ? kh[1][q] : (kk == 2 ? kh[2][q] : kh[3][q]));
            B0[fft_pad(idx)] = make_float2(kv * qh[q].x, kv * qh[q].y);
          }
        }
        __syncthreads();
        block_fft<C>(B0, ncc, M, twl, +1.f);
        const float2* r = B0;
        for (int idx = threadIdx.x; idx < ncc * ng; idx += blockDim.x) {
          const int col = idx / ng, y = idx - col * ng;
          ot[((size_t)o * Mh + c0 + col) * ng + y] = r[fft_pad(col * M + y)];
        }
        __syncthreads();
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Inverse rows: job (row y, pair p) transforms F_{2p} + i F_{2p+1}.
template <class C>
__global__ __launch_bounds__(C::Threads) void k_fft_rows_inv(FftArgs A) {
  extern __shared__ float2 lds[];
  const int g = blockIdx.y;
  const GridDesc d = A.desc[g];
  const int M = d.M, ng = d.ng, Mh = M / 2 + 1;
  if (!C::handles(M)) return;  // the other size class transforms this graph
  float2* bufA = lds;
  float2* twl = lds + C::Buf;  // half twiddle table
  load_twiddles(twl, A.tw, M);
  const int jobs = ng * 4;
  const int S = fft_pack<C>(M, jobs);
  const float2* orr = A.orr + d.off_o;
  float* pg = A.pot + d.off_p;
  const float scale = 1.0f / ((float)M * (float)M);
  for (int j0 = blockIdx.x * S; j0 < jobs; j0 += gridDim.x * S) {
    const int nj = jobs - j0 < S ? jobs - j0 : S;
    // every load of the block's jobs is issued before any is used
    float2 f0[C::PerThread], f1[C::PerThread];
#pragma unroll
    for (int q = 0; q < C::PerThread; ++q) {
      const int idx = threadIdx.x + q * C::Threads;
      f0[q] = f1[q] = make_float2(0.f, 0.f);
      if (idx >= nj * M) continue;
      const int jl = idx / M, k = idx - jl * M;
      const int job = j0 + jl;
      const int ry = job >> 2, pr = job & 3;
      const int o0 = 2 * pr, o1 = 2 * pr + 1;
      const int kk = k > M / 2 ? M - k : k;
      f0[q] = orr[((size_t)o0 * ng + ry) * Mh + kk];
      if (!(o1 == CH_KLN_1 && !A.with_ln)) f1[q] = orr[((size_t)o1 * ng + ry) * Mh + kk];
    }
#pragma unroll
    for (int q = 0; q < C::PerThread; ++q) {
      const int idx = threadIdx.x + q * C::Threads;
      if (idx >= nj * M) continue;
      const int k = idx - (idx / M) * M;
      float2 a = f0[q], b = f1[q];
      if (k > M / 2) {  // conjugate half of the Hermitian spectra
        a.y = -a.y;
        b.y = -b.y;
      }
      bufA[fft_pad(idx)] = make_float2(a.x - b.y, a.y + b.x);
    }
    __syncthreads();
    block_fft<C>(bufA, nj, M, twl, +1.f);
    const float2* res = bufA;
    for (int idx = threadIdx.x; idx < nj * ng; idx += blockDim.x) {
      const int jl = idx / ng, x = idx - jl * ng;
      const int job = j0 + jl;
      const int ry = job >> 2, pr = job & 3;
      const float2 v = res[fft_pad(jl * M + x)];
      // plane pr of the potentials: contiguous float2 per node
      reinterpret_cast<float2*>(pg)[(size_t)pr * ng * ng + (size_t)ry * ng + x] =
          make_float2(v.x * scale, v.y * scale);
    }
    __syncthreads();
  }
}

hipError_t launch_fft_conv(Problem& P, float eps, int with_ln, int max_intervals, hipStream_t s) {
  FftArgs A;
  A.desc = P.desc;
  A.tw = P.ctx->twiddle;
  A.charges = P.charges;
  A.qr = P.qspec;
  A.qt = P.qspec_t;
  A.kr = P.kspec;
  A.kt = P.kspec_t;
  A.ot = P.ospec_t;
  A.orr = P.ospec;
  A.pot = P.pot;
  A.eps = eps;
  A.with_ln = with_ln;
  const int bx = P.G >= 64 ? 4 : (P.G >= 8 ? 32 : 1024);
  const int tb = P.G >= 64 ? 64 : (P.G >= 8 ? 256 : 2048);  // transpose blocks per graph
  // the large class only where the plan may give a graph 1024 intervals
  const bool large = max_intervals > kFftSmallM / (2 * kNodes);
  hipLaunchKernelGGL(k_fft_rows_fwd<FftSmall>, dim3(bx, P.G), dim3(FftSmall::Threads), FftSmall::Lds,
                     s, A);
  if (large)
    hipLaunchKernelGGL(k_fft_rows_fwd<FftLarge>, dim3(bx, P.G), dim3(FftLarge::Threads),
                       FftLarge::Lds, s, A);
  hipLaunchKernelGGL(k_fft_transpose, dim3(2 * tb, P.G), dim3(256), 0, s, A, 0);
  // the column kernel's registers hold three of its blocks per CU: in a batch
  // of 256 graphs, three blocks per graph fill the chip in one round where
  // four would take a second, mostly idle one
  const int cbx = P.G >= 64 ? 3 : bx;
  hipLaunchKernelGGL(k_fft_cols<FftSmall>, dim3(cbx, P.G), dim3(FftSmall::Threads), FftSmall::Lds,
                     s, A);
  if (large)
    hipLaunchKernelGGL(k_fft_cols<FftLarge>, dim3(bx, P.G), dim3(FftLarge::Threads), FftLarge::Lds,
                       s, A);
  hipLaunchKernelGGL(k_fft_transpose, dim3(tb, P.G), dim3(256), 0, s, A, 2);
  hipLaunchKernelGGL(k_fft_rows_inv<FftSmall>, dim3(bx, P.G), dim3(FftSmall::Threads), FftSmall::Lds,
                     s, A);
  if (large)
    hipLaunchKernelGGL(k_fft_rows_inv<FftLarge>, dim3(bx, P.G), dim3(FftLarge::Threads),
                       FftLarge::Lds, s, A);
  return hipGetLastError();
}

// Allows the large class its dynamic LDS (more than 64 KB per block); false
// when the device cannot give it, and then grids stay at 512 intervals.
bool fft_large_init() {
  int dev = 0, lim = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
      lim < FftLarge::Lds)
    return false;
  const void* ks[3] = {reinterpret_cast<const void*>(k_fft_rows_fwd<FftLarge>),
                       reinterpret_cast<const void*>(k_fft_cols<FftLarge>),
                       reinterpret_cast<const void*>(k_fft_rows_inv<FftLarge>)};
  for (const void* k : ks)
    if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, FftLarge::Lds) !=
        hipSuccess)
      return false;
  return true;
}

}  // namespace tsnet
