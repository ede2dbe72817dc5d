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

// Contrast transfer function for the joint translation-CTF factorisation
// (Section 7.1, other 2D kernels): the isotropic weak-phase model
//   C(y; tau) = -(sqrt(1 - A^2) sin chi + A cos chi),
//   chi = pi lambda tau s^2 - (pi / 2) Cs lambda^3 s^4,  s = y / (2 pixel),
// y = k / Kmax, s in 1/Angstrom, lambda, Cs, tau and the pixel in Angstrom;
// tau (defocus) ranges over [tmin, tmax] with the uniform measure of mass 1.
struct Ctf {
  bool on = false;
  double lambda = 0, cs = 0, amp = 0, pixel = 1, tmin = 0, tmax = 0;
  double chi(double y, double tau) const;
  double operator()(double y, double tau) const;
};
// Checks the parameters (throws std::invalid_argument); cs in millimetres.
Ctf make_ctf(double wavelength_A, double cs_mm, double amplitude_contrast, double pixel_A, double tmin_A,
             double tmax_A);

// Modal SVD of the kernel K_l(x, tau; y) = J_l(x y) C(y; tau) from L2(p(y) y dy)
// on [0, 1] to L2(x dx dtau) on [0, X] x [tmin, tmax] (without a CTF: C = 1
// and no tau, the translation kernel of Section 4.5).
struct ModalSVD {
  int ell = 0;
  int P = 0;   // x nodes
  int Pt = 1;  // tau nodes (1 without a CTF)
  int Py = 0;  // y nodes (P without a CTF)
  double X = 0;
  Ctf ctf;
  std::vector<double> sigma;  // Py, descending
  std::vector<double> U;      // (P Pt) x Py: row i Pt + t (x_i, tau_t), column eta = left vector
  std::vector<double> V;      // Py x Py, column eta = right vector (y side), V[j*Py + eta]
  std::vector<double> xn, xw, tn, tw, yn, yw;  // yw: quadrature weights times p(y_j)
  double kernel(double x, double y, double tau) const;
  // Sigma_eta v_eta(y), Nystrom through the x side (no division by Sigma).
  double sigma_v(int eta, double y) const;
  // u_eta(x, tau), Nystrom through the y side.
  double u(int eta, double x, double tau = 0.0) const;
};

ModalSVD modal_svd(int ell, double X, const Weight& weight = Weight());
ModalSVD ctf_modal_svd(int ell, double X, const Ctf& ctf);

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
// With ctf.on the modal SVDs are those of the joint kernel (the weight is
// then not used).
Truncation truncate(double X, double eps, const Weight& weight = Weight(), const Ctf& ctf = Ctf());

// One-sided Jacobi SVD of a dense m x n (m >= n) row-major matrix A.
// On exit: sigma (n, descending), U (m x n, row-major), V (n x n, row-major).
void jacobi_svd(int m, int n, std::vector<double> A, std::vector<double>& sigma,
                std::vector<double>& U, std::vector<double>& V);
// The same for m much larger than n: Householder QR first, one-sided Jacobi
// on the n x n triangle, U = Q U_R.
void qr_jacobi_svd(int m, int n, const std::vector<double>& A, std::vector<double>& sigma,
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
