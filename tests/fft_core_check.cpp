// Host check of the FFT building blocks of the library (fft_core.h: the small
// in-register DFTs, the Stockham pass index arithmetic, the pass plan and the
// padded addressing) against a plain O(L^2) DFT in double, for every
// transform length the interpolation grid can take. Exit status 0 when every
// relative L2 error is below 1e-6.
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>
#include "fft_core.h"
using namespace tsnet;

template <int R>
void run_pass(const float2* in, float2* out, int nb, int L, int Ns, const float2* tw, float sgn) {
  fft_pass<R>(in, out, nb, L, Ns, tw, sgn, 0, 1);
}
void dispatch(int R, const float2* in, float2* out, int nb, int L, int Ns, const float2* tw, float sgn) {
  switch (R) {
    case 2: run_pass<2>(in, out, nb, L, Ns, tw, sgn); break;
    case 3: run_pass<3>(in, out, nb, L, Ns, tw, sgn); break;
    case 4: run_pass<4>(in, out, nb, L, Ns, tw, sgn); break;
    case 6: run_pass<6>(in, out, nb, L, Ns, tw, sgn); break;
    case 8: run_pass<8>(in, out, nb, L, Ns, tw, sgn); break;
    case 12: run_pass<12>(in, out, nb, L, Ns, tw, sgn); break;
    case 16: run_pass<16>(in, out, nb, L, Ns, tw, sgn); break;
    default: printf("bad radix %d\n", R);
  }
}
int main() {
  std::mt19937 rng(1);
  std::normal_distribution<float> nd;
  int bad = 0;
  for (int L : {6, 12, 24, 48, 96, 192, 384, 768, 1536, 3072, 6144}) {  // every M = 6 n_int
    for (float sgn : {-1.f, 1.f}) {
      const int nb = 3;
      std::vector<float2> tw(L);
      for (int m = 0; m < L; ++m) {
        const double a = 2 * M_PI * m / L;
        tw[m] = make_float2((float)cos(a), (float)-sin(a));
      }
      const int pl = fft_pad(nb * L) + 16;
      std::vector<float2> A(pl), B(pl);
      std::vector<double> xr(nb * L), xi(nb * L);
      for (int i = 0; i < nb * L; ++i) {
        xr[i] = nd(rng); xi[i] = nd(rng);
        A[fft_pad(i)] = make_float2((float)xr[i], (float)xi[i]);
      }
      int radix[8];
      const int np = fft_plan(L, radix);
      float2 *a = A.data(), *b = B.data();
      int Ns = 1;
      for (int p = 0; p < np; ++p) {
        dispatch(radix[p], a, b, nb, L, Ns, tw.data(), sgn);
        std::swap(a, b);
        Ns *= radix[p];
      }
      double err = 0, ref = 0;
      for (int s = 0; s < nb; ++s)
        for (int k = 0; k < L; ++k) {
          double sr = 0, si = 0;
          for (int n = 0; n < L; ++n) {
            const double ang = sgn * 2 * M_PI * (double)((long)n * k % L) / L;
            const double c = cos(ang), sn = sin(ang);
            sr += xr[s * L + n] * c - xi[s * L + n] * sn;
            si += xr[s * L + n] * sn + xi[s * L + n] * c;
          }
          const float2 g = a[fft_pad(s * L + k)];
          err += (g.x - sr) * (g.x - sr) + (g.y - si) * (g.y - si);
          ref += sr * sr + si * si;
        }
      const double rel = sqrt(err / ref);
      printf("L=%5d sgn=%+.0f passes=%d [", L, sgn, np);
      for (int p = 0; p < np; ++p) printf("%d%s", radix[p], p + 1 < np ? " " : "");
      printf("] rel err %.2e\n", rel);
      if (!(rel < 1e-6)) bad++;
    }
  }
  printf(bad ? "FAILED %d\n" : "all ok\n", bad);
  return bad;
}
