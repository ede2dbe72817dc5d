// Host-side FP64 planning for the FTK path: radial quadrature, Bessel
// functions, the per-mode operator SVD of the translation kernel, its
// eps-truncation, and the NUFFT spreading-kernel tables.  Plain C++17, no
// device code; everything here is image independent and runs once per plan.
#pragma once

#include <cstdint>
#include <vector>

namespace ftkplan {

// Gauss-Jacobi(alpha=0, beta=1) rule on [0, len] for the measure k dk
// (Section 3.1 of the paper).  nodes/weights have M entries, ascending.
void radial_rule(int M, double len, std::vector<double>& nodes, std::vector<double>& weights);

// J_l(z) for l = 0..lmax at one z >= 0 (Miller backward recurrence,
// normalised by J_0 + 2 sum J_2k = 1).  out has lmax+1 entries.
void bessel_orders(int lmax, double z, double* out);

// Same quantity from the trapezoid rule on the integral representation
// J_l(z) = (1/2 pi) int exp(i (z sin a - l a)) da; used as a self-check.
double bessel_integral(int l, double z);

// k-side weight of the operator SVD (Section 4.5, the remark on alternative
// weight functions): p(y) = c sum_j alpha_j exp(-beta_j y^2), y = k / Kmax,
// alpha_j >= 0 (not all 0), beta_j >= 0, with c such that its mean over the
// unit disk is 1 (int_0^1 p(y) y dy = 1/2).  Empty: p = 1, the paper's weight.
struct Weight {
  std::vector<double> alpha, beta;
  double c = 1.0;
  bool empty() const { return alpha.empty(); }
  double operator()(double y) const;
};
// Checks the terms and sets c; throws std::invalid_argument on bad terms.
Weight make_weight(const double* alpha, const double* beta, int nterms);

// Modal SVD of J_l(x y) on x in [0, X] (x dx) and y in [0, 1] (p(y) y dy).
struct ModalSVD {
  int ell = 0;
  int P = 0;
  double X = 0;
  std::vector<double> sigma;  // P, descending
  std::vector<double> U;      // P x P, column eta = left vector (x side), U[i*P + eta]
  std::vector<double> V;      // P x P, column eta = right vector (y side), V[j*P + eta]
  std::vector<double> xn, xw, yn, yw;  // yw: quadrature weights times p(y_j)
  // Sigma_eta v_eta(y), Nystrom through the x side (no division by Sigma).
  double sigma_v(int eta, double y) const;
  // u_eta(x), Nystrom through the y side.
  double u(int eta, double x) const;
};

ModalSVD modal_svd(int ell, double X, const Weight& weight = Weight());

struct Term {
  int ell;
  int eta;
  double sigma;
};

struct Truncation {
  std::vector<Term> terms;         // ordered by (ell, eta), ell from -L..L
  std::vector<ModalSVD> svds;      // index ell = 0..L
  double sigma_next = 0;           // largest discarded singular value
  int L = 0;                       // largest |ell| kept
};

// Keep every Sigma_eta(l) > eps; scan |l| = 0, 1, ... until Sigma_1(l) <= eps.
Truncation truncate(double X, double eps, const Weight& weight = Weight());

// One-sided Jacobi SVD of a dense m x n (m >= n) row-major matrix A.
// On exit: sigma (n, descending), U (m x n, row-major), V (n x n, row-major).
void jacobi_svd(int m, int n, std::vector<double> A, std::vector<double>& sigma,
                std::vector<double>& U, std::vector<double>& V);

// NUFFT (type 2) spreading kernel: phi(z) = exp(beta (sqrt(1 - z^2) - 1)),
// |z| < 1.  Phi(s) = int psi(t) e^{i s t} dt with psi(t) = phi(t / alpha).
struct SpreadKernel {
  int w = 8;          // width in fine-grid points
  double beta = 0;    // shape
  int nf = 0;         // fine grid size (oversampled)
  double h = 0;       // fine grid spacing 2 pi / nf
  double alpha = 0;   // half width in t: w h / 2
  double ft(double s) const;  // Phi(s)
};
SpreadKernel spread_kernel(int n, int w);

// Smallest length >= n of the form 2^a 3^b that the device FFT supports
// (at most 4096); 0 when n > 4096.
int fft_size(int n);
bool fft_supported(int L);

}  // namespace ftkplan
