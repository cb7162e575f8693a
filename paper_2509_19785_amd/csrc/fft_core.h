// Building blocks of the LDS FFT: small DFTs in registers and one Stockham
// pass. Header-only and usable on the host, so the index arithmetic can be
// checked against a plain DFT without a GPU.
//
// A transform of length L = 3 * 2^b runs as power-of-two passes of radix
// 16 (the last one 8, 4 or 2) followed by one pass of radix 12 (6 or 3 for
// the shortest lengths). Pass p with radix R over sub-length Ns (the product
// of the radices before it, a power of two) maps
//   in[j + r L/R] * w_L^{r k (L/(Ns R))}, k = j mod Ns, r < R
// through an R-point DFT to out[(j - k) R + k + r Ns] (Stockham autosort).
// Buffers are addressed through pad(i) = i + i / 16: the strided writes of
// the first pass then fall into distinct LDS banks.
#pragma once

#include <hip/hip_runtime.h>

namespace tsnet {

__host__ __device__ __forceinline__ int fft_pad(int i) { return i + (i >> 4); }

__host__ __device__ __forceinline__ float2 fmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ __forceinline__ float2 faddc(float2 a, float2 b) {
  return make_float2(a.x + b.x, a.y + b.y);
}
__host__ __device__ __forceinline__ float2 fsubc(float2 a, float2 b) {
  return make_float2(a.x - b.x, a.y - b.y);
}
// a * (sgn i): forward transforms use sgn = -1
__host__ __device__ __forceinline__ float2 fmuli(float2 a, float sgn) {
  return make_float2(-sgn * a.y, sgn * a.x);
}

// e^{sgn 2 pi i m / N} for the small N of the in-register DFTs (exact
// values of cos and sin at multiples of pi / 8 and pi / 6).
template <int N>
__host__ __device__ __forceinline__ float2 wconst(int m, float sgn) {
  m %= N;
  if constexpr (N == 16) {
    constexpr float c[16] = {1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
                             0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
                             -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f,
                             0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f};
    constexpr float s[16] = {0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f,
                             1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
                             0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
                             -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f};
    return make_float2(c[m], sgn * s[m]);
  } else if constexpr (N == 8) {
    constexpr float c[8] = {1.0f, 0.70710678118654752f, 0.0f, -0.70710678118654752f,
                            -1.0f, -0.70710678118654752f, 0.0f, 0.70710678118654752f};
    constexpr float s[8] = {0.0f, 0.70710678118654752f, 1.0f, 0.70710678118654752f,
                            0.0f, -0.70710678118654752f, -1.0f, -0.70710678118654752f};
    return make_float2(c[m], sgn * s[m]);
  } else if constexpr (N == 12) {
    constexpr float c[12] = {1.0f, 0.86602540378443865f, 0.5f, 0.0f, -0.5f, -0.86602540378443865f,
                             -1.0f, -0.86602540378443865f, -0.5f, 0.0f, 0.5f, 0.86602540378443865f};
    constexpr float s[12] = {0.0f, 0.5f, 0.86602540378443865f, 1.0f, 0.86602540378443865f, 0.5f,
                             0.0f, -0.5f, -0.86602540378443865f, -1.0f, -0.86602540378443865f, -0.5f};
    return make_float2(c[m], sgn * s[m]);
  } else {  // N == 6
    static_assert(N == 6, "no table for this N");
    constexpr float c[6] = {1.0f, 0.5f, -0.5f, -1.0f, -0.5f, 0.5f};
    constexpr float s[6] = {0.0f, 0.86602540378443865f, 0.86602540378443865f, 0.0f,
                            -0.86602540378443865f, -0.86602540378443865f};
    return make_float2(c[m], sgn * s[m]);
  }
}

__host__ __device__ __forceinline__ void dft2(float2& a, float2& b) {
  const float2 t = a;
  a = faddc(t, b);
  b = fsubc(t, b);
}

// 4-point DFT of (a, b, c, d) in place, natural order.
__host__ __device__ __forceinline__ void dft4(float2& a, float2& b, float2& c, float2& d, float sgn) {
  const float2 t0 = faddc(a, c), t1 = fsubc(a, c);
  const float2 t2 = faddc(b, d), t3 = fmuli(fsubc(b, d), sgn);
  a = faddc(t0, t2);
  c = fsubc(t0, t2);
  b = faddc(t1, t3);
  d = fsubc(t1, t3);
}

// 3-point DFT in place, natural order.
__host__ __device__ __forceinline__ void dft3(float2& a, float2& b, float2& c, float sgn) {
  const float s3 = 0.86602540378443865f;
  const float2 t1 = faddc(b, c), t2 = fsubc(b, c);
  const float2 m = make_float2(a.x - 0.5f * t1.x, a.y - 0.5f * t1.y);
  const float2 nn = make_float2(-sgn * s3 * t2.y, sgn * s3 * t2.x);  // sgn i s3 t2
  a = faddc(a, t1);
  b = faddc(m, nn);
  c = fsubc(m, nn);
}

// R-point DFT of v[0..R) in place, natural order. R in {2, 3, 4, 6, 8, 12, 16}.
// Composite R = A * B: n = B n1 + n2, k = k1 + A k2; A-point DFTs over n1,
// twiddles w_R^{n2 k1}, B-point DFTs over n2.
template <int R>
__host__ __device__ __forceinline__ void small_dft(float2* v, float sgn) {
  if constexpr (R == 2) {
    dft2(v[0], v[1]);
  } else if constexpr (R == 3) {
    dft3(v[0], v[1], v[2], sgn);
  } else if constexpr (R == 4) {
    dft4(v[0], v[1], v[2], v[3], sgn);
  } else {
    constexpr int A = (R == 6) ? 2 : 4;  // first factor
    constexpr int B = R / A;             // second factor: 3, 2, 3, 4
    float2 y[A][B];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) {
      float2 t[4];
#pragma unroll
      for (int n1 = 0; n1 < A; ++n1) t[n1] = v[B * n1 + n2];
      if constexpr (A == 2) dft2(t[0], t[1]);
      else dft4(t[0], t[1], t[2], t[3], sgn);
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1)
        y[k1][n2] = (n2 * k1 == 0) ? t[k1] : fmulc(t[k1], wconst<R>(n2 * k1, sgn));
    }
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
      float2 t[4];
#pragma unroll
      for (int n2 = 0; n2 < B; ++n2) t[n2] = y[k1][n2];
      if constexpr (B == 2) dft2(t[0], t[1]);
      else if constexpr (B == 3) dft3(t[0], t[1], t[2], sgn);
      else dft4(t[0], t[1], t[2], t[3], sgn);
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) v[k1 + A * k2] = t[k2];
    }
  }
}

// One Stockham pass of radix R over nb sequences of length L held at
// in[pad(s L + i)]; butterflies idx = first, first + stride, ... (the thread
// index and the block size on the GPU). tw[m] = e^{-2 pi i m / L}; sgn = -1
// forward, +1 inverse.
template <int R>
__host__ __device__ __forceinline__ void fft_pass(const float2* in, float2* out, int nb, int L, int Ns,
                                                  const float2* tw, float sgn, int first, int stride) {
  const int nbut = L / R;
  const int tstep = L / (Ns * R);
  const int total = nb * nbut;
  for (int idx = first; idx < total; idx += stride) {
    const int sq = idx / nbut;
    const int j = idx - sq * nbut;
    const int k = j & (Ns - 1);
    const int ib = sq * L + j;
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = in[fft_pad(ib + r * nbut)];
    if (k > 0) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        float2 w = tw[k * r * tstep];
        if (sgn > 0.f) w.y = -w.y;
        v[r] = fmulc(v[r], w);
      }
    }
    small_dft<R>(v, sgn);
    const int ob = sq * L + (j - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) out[fft_pad(ob + r * Ns)] = v[r];
  }
}

// The radices of a transform of length L = 3 * 2^b (b >= 1), in pass order.
// Returns the number of passes (at most 4 for L <= 3 * 2^10).
__host__ __device__ __forceinline__ int fft_plan(int L, int* radix) {
  int p2 = L / 3;
  const int r3 = p2 >= 4 ? 12 : (p2 == 2 ? 6 : 3);
  p2 /= r3 / 3;
  int np = 0;
  while (p2 > 1) {
    const int r = p2 >= 16 ? 16 : p2;
    radix[np++] = r;
    p2 /= r;
  }
  radix[np++] = r3;
  return np;
}

}  // namespace tsnet
