// Host check of the FP64 planner under AddressSanitizer and
// UndefinedBehaviorSanitizer (built and run by tests/test_planner_sanitized.py
// with g++, CPU only).  Exercises every planner routine over the sizes the
// library plans for and prints "key value" lines that the test compares with
// the FP64 oracle.
#include <cmath>
#include <cstdio>
#include <vector>

#include "planner.h"

int main() {
  const double pi = 3.14159265358979323846;
  // Section 3.1: Gauss-Jacobi(0,1) rule for k dk on [0, pi n / 2]
  const int Ms[] = {1, 2, 5, 16, 48, 64, 96, 256, 512};
  for (int M : Ms) {
    std::vector<double> k, w;
    ftkplan::radial_rule(M, pi * 64.0, k, w);
    double sw = 0.0, m3 = 0.0;
    for (int i = 0; i < M; ++i) {
      sw += w[i];
      m3 += w[i] * k[i] * k[i] * k[i];
    }
    std::printf("rule %d %.17g %.17g %.17g %.17g\n", M, sw, m3, k.front(), k.back());
  }
  // Bessel functions by the backward recurrence, orders up to 64
  const double zs[] = {0.0, 1e-3, 0.5, 3.0, 12.5, 25.1, 40.0};
  for (double z : zs) {
    std::vector<double> J(65);
    ftkplan::bessel_orders(64, z, J.data());
    double s = J[0] * J[0];
    for (int l = 1; l <= 64; ++l) s += 2.0 * J[l] * J[l];
    std::printf("bessel %.17g %.17g %.17g %.17g\n", z, J[0], J[3], s);
  }
  // Section 4.5: modal SVD and eps-truncation at every shift radius of the
  // ragged workload (2 to 8 px, W in the paper's units = half that)
  const double epss[] = {1e-2, 1e-3, 1e-5};
  for (int twoR = 2; twoR <= 16; ++twoR) {
    const double Rpx = 0.5 * twoR;
    for (double eps : epss) {
      const ftkplan::Truncation t = ftkplan::truncate(pi * Rpx, eps);
      double s2 = 0.0;
      for (const auto& term : t.terms) s2 += term.sigma * term.sigma;
      // factor products u(x) Sigma v(y) of the terms with l >= 0 at one
      // point, through both Nystrom forms (independent of the vectors' signs)
      double uv = 0.0;
      for (const auto& term : t.terms) {
        if (term.ell < 0) continue;
        const ftkplan::ModalSVD& m = t.svds[term.ell];
        uv += m.u(term.eta, 0.7 * m.X) * m.sigma_v(term.eta, 0.3);
      }
      std::printf("trunc %.17g %.17g %zu %d %.17g %.17g %.17g\n", Rpx, eps, t.terms.size(), t.L, t.sigma_next,
                  s2, uv);
    }
  }
  // NUFFT spreading kernel and FFT lengths
  const int ns[] = {8, 32, 64, 96, 128, 192, 1024};
  for (int n : ns) {
    const ftkplan::SpreadKernel sk = ftkplan::spread_kernel(n, 8);
    std::printf("spread %d %d %.17g %.17g\n", n, sk.nf, sk.ft(0.0), sk.ft(0.5 * pi * n));
  }
  const int ls[] = {1, 2, 7, 64, 100, 385, 2049, 4096, 4097, 9000};
  for (int L : ls) std::printf("fft %d %d %d\n", L, ftkplan::fft_size(L), ftkplan::fft_supported(L) ? 1 : 0);
  std::vector<double> A = {4, 1, 2, 1, 3, 0, 2, 0, 5, 1, 1, 1}, sig, U, V;
  ftkplan::jacobi_svd(4, 3, A, sig, U, V);
  std::printf("svd %.17g %.17g %.17g\n", sig[0], sig[1], sig[2]);
  return 0;
}
