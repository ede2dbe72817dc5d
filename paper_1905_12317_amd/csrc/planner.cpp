// FP64 host planning for the FTK path.  See planner.h.
#include "planner.h"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <stdexcept>
#include <string>
#include <thread>

namespace ftkplan {

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

// Cyclic Jacobi eigenvalue iteration on a dense symmetric n x n matrix
// (row-major).  Returns eigenvalues in w and eigenvectors as columns of Z.
void sym_eig(int n, std::vector<double> A, std::vector<double>& w, std::vector<double>& Z) {
  Z.assign(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i) Z[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < n - 1; ++p) {
      for (int q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        double app = A[p * n + p], aqq = A[q * n + q];
        // below rounding of the diagonal: the pair is already decoupled
        if (std::fabs(apq) <= 1e-18 * (std::fabs(app) + std::fabs(aqq))) continue;
        rotated = true;
        double theta = (aqq - app) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // rows p, q
          double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // columns p, q
          double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double zkp = Z[k * n + p], zkq = Z[k * n + q];
          Z[k * n + p] = c * zkp - s * zkq;
          Z[k * n + q] = s * zkp + c * zkq;
        }
      }
    }
    if (!rotated) break;
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = A[i * n + i];
}

// Gauss rule from the three-term recurrence of the orthonormal polynomials
// b_{k+1} p_{k+1} = (t - a_k) p_k - b_k p_{k-1}, p_0 = 1/sqrt(mu0)
// (Golub-Welsch), nodes polished by Newton on p_M, weights from the
// Christoffel sum w = 1 / sum_k p_k(t)^2.  a has M entries, b has M+1
// (b[0] unused, b[M] used for p_M).
void gauss_rule(int M, const std::vector<double>& a, const std::vector<double>& b, double mu0,
                std::vector<double>& t, std::vector<double>& wt) {
  std::vector<double> J(static_cast<size_t>(M) * M, 0.0);
  for (int k = 0; k < M; ++k) {
    J[k * M + k] = a[k];
    if (k + 1 < M) J[k * M + k + 1] = J[(k + 1) * M + k] = b[k + 1];
  }
  std::vector<double> ev, Z;
  sym_eig(M, J, ev, Z);
  std::sort(ev.begin(), ev.end());
  t = ev;
  wt.assign(M, 0.0);
  const double p0 = 1.0 / std::sqrt(mu0);
  for (int i = 0; i < M; ++i) {
    double x = t[i];
    for (int it = 0; it < 6; ++it) {
      double pm1 = 0.0, p = p0, dpm1 = 0.0, dp = 0.0;
      for (int k = 0; k < M; ++k) {
        double pn = ((x - a[k]) * p - (k > 0 ? b[k] * pm1 : 0.0)) / b[k + 1];
        double dpn = (p + (x - a[k]) * dp - (k > 0 ? b[k] * dpm1 : 0.0)) / b[k + 1];
        pm1 = p; p = pn; dpm1 = dp; dp = dpn;
      }
      if (dp == 0.0) break;
      double step = p / dp;
      x -= step;
      if (std::fabs(step) < 1e-17) break;
    }
    t[i] = x;
    double s = 0.0, pm1 = 0.0, p = p0;
    for (int k = 0; k < M; ++k) {
      s += p * p;
      double pn = ((x - a[k]) * p - (k > 0 ? b[k] * pm1 : 0.0)) / b[k + 1];
      pm1 = p; p = pn;
    }
    wt[i] = 1.0 / s;
  }
}

void legendre_rule01(int M, std::vector<double>& z, std::vector<double>& wz) {
  std::vector<double> a(M, 0.0), b(M + 1, 0.0);
  for (int k = 1; k <= M; ++k) b[k] = k / std::sqrt(4.0 * k * k - 1.0);
  std::vector<double> t, wt;
  gauss_rule(M, a, b, 2.0, t, wt);
  z.resize(M); wz.resize(M);
  for (int i = 0; i < M; ++i) { z[i] = 0.5 * (t[i] + 1.0); wz[i] = 0.5 * wt[i]; }
}

}  // namespace

void radial_rule(int M, double len, std::vector<double>& nodes, std::vector<double>& weights) {
  // Jacobi(0,1) recurrence: a_k = 1/((2k+1)(2k+3)), b_k = sqrt(k(k+1))/(2k+1),
  // mu0 = int_{-1}^{1} (1+t) dt = 2.
  std::vector<double> a(M), b(M + 1, 0.0);
  for (int k = 0; k < M; ++k) a[k] = 1.0 / ((2.0 * k + 1.0) * (2.0 * k + 3.0));
  for (int k = 1; k <= M; ++k) b[k] = std::sqrt(double(k) * (k + 1)) / (2.0 * k + 1.0);
  std::vector<double> t, wt;
  gauss_rule(M, a, b, 2.0, t, wt);
  nodes.resize(M); weights.resize(M);
  const double h = 0.5 * len;
  for (int i = 0; i < M; ++i) {
    nodes[i] = h * (1.0 + t[i]);
    weights[i] = h * h * wt[i];
  }
}

void bessel_orders(int lmax, double z, double* out) {
  for (int k = 0; k <= lmax; ++k) out[k] = 0.0;
  if (z < 1e-6) {
    // leading series terms; the next term is O(z^4) relative
    double term = 1.0;
    for (int k = 0; k <= lmax; ++k) {
      if (k > 0) term *= 0.5 * z / k;
      out[k] = term * (1.0 - 0.25 * z * z / (k + 1));
      if (term < 1e-300) break;
    }
    return;
  }
  const double top = std::max<double>(lmax, z);
  int N = static_cast<int>(top + 30.0 + 2.0 * std::sqrt(40.0 * top + 1.0));
  N += (N & 1);
  double fp1 = 0.0, f = 1e-30, sum = 0.0;
  // f holds f_k; walk k = N .. 1 producing f_{k-1}
  for (int k = N; k >= 1; --k) {
    double fm1 = (2.0 * k / z) * f - fp1;
    fp1 = f;
    f = fm1;
    int km1 = k - 1;
    if (km1 <= lmax) out[km1] = f;
    if (km1 > 0 && (km1 % 2) == 0) sum += 2.0 * f;
    if (std::fabs(f) > 1e250) {
      f *= 1e-250; fp1 *= 1e-250; sum *= 1e-250;
      for (int j = km1; j <= lmax; ++j) out[j] *= 1e-250;
    }
  }
  sum += f;  // f_0
  for (int k = 0; k <= lmax; ++k) out[k] /= sum;
}

double bessel_integral(int l, double z) {
  int P = 2 * (std::abs(l) + static_cast<int>(z) + 48);
  double s = 0.0;
  for (int p = 0; p < P; ++p) {
    double a = 2.0 * kPi * p / P;
    s += std::cos(l * a - z * std::sin(a));
  }
  return s / P;
}

void jacobi_svd(int m, int n, std::vector<double> A, std::vector<double>& sigma,
                std::vector<double>& U, std::vector<double>& V) {
  std::vector<double> Vw(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i) Vw[i * n + i] = 1.0;
  // columns whose norm^2 is below this floor carry nothing above rounding of
  // the largest singular value; rotating them cannot converge further
  double fro2 = 0.0;
  for (double v : A) fro2 += v * v;
  const double floor2 = 1e-30 * fro2;
  // attainable orthogonality of m-vectors in double (as in one-sided Jacobi codes)
  const double tol = 4.0 * std::sqrt(static_cast<double>(m)) * 2.220446049250313e-16;
  for (int sweep = 0; sweep < 80; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < n - 1; ++p) {
      for (int q = p + 1; q < n; ++q) {
        double al = 0, be = 0, ga = 0;
        for (int i = 0; i < m; ++i) {
          double x = A[i * n + p], y = A[i * n + q];
          al += x * x; be += y * y; ga += x * y;
        }
        if (ga == 0.0 || std::fabs(ga) <= tol * std::sqrt(al * be)) continue;
        if (al < floor2 && be < floor2) continue;
        rotated = true;
        double zeta = (be - al) / (2.0 * ga);
        double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
        for (int i = 0; i < m; ++i) {
          double x = A[i * n + p], y = A[i * n + q];
          A[i * n + p] = c * x - s * y;
          A[i * n + q] = s * x + c * y;
        }
        for (int i = 0; i < n; ++i) {
          double x = Vw[i * n + p], y = Vw[i * n + q];
          Vw[i * n + p] = c * x - s * y;
          Vw[i * n + q] = s * x + c * y;
        }
      }
    }
    if (!rotated) break;
  }
  std::vector<double> nrm(n);
  for (int j = 0; j < n; ++j) {
    double s = 0;
    for (int i = 0; i < m; ++i) s += A[i * n + j] * A[i * n + j];
    nrm[j] = std::sqrt(s);
  }
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return nrm[a] > nrm[b]; });
  sigma.resize(n);
  U.assign(static_cast<size_t>(m) * n, 0.0);
  V.assign(static_cast<size_t>(n) * n, 0.0);
  for (int jj = 0; jj < n; ++jj) {
    int j = order[jj];
    sigma[jj] = nrm[j];
    double inv = nrm[j] > 0 ? 1.0 / nrm[j] : 0.0;
    for (int i = 0; i < m; ++i) U[i * n + jj] = A[i * n + j] * inv;
    for (int i = 0; i < n; ++i) V[i * n + jj] = Vw[i * n + j];
  }
}

void qr_jacobi_svd(int m, int n, const std::vector<double>& A, std::vector<double>& sigma, std::vector<double>& U,
                   std::vector<double>& V) {
  // column-major copy; Householder vectors kept below the diagonal
  std::vector<double> Cm(static_cast<size_t>(m) * n);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) Cm[static_cast<size_t>(j) * m + i] = A[static_cast<size_t>(i) * n + j];
  std::vector<double> beta(n, 0.0), diag(n, 0.0);
  for (int k = 0; k < n; ++k) {
    double* ck = &Cm[static_cast<size_t>(k) * m];
    double nrm2 = 0.0;
    for (int i = k; i < m; ++i) nrm2 += ck[i] * ck[i];
    const double nrm = std::sqrt(nrm2);
    if (nrm == 0.0) {
      diag[k] = 0.0;
      continue;
    }
    const double alpha = ck[k] > 0 ? -nrm : nrm;
    ck[k] -= alpha;  // v = x - alpha e_k, stored in place
    double vv = 0.0;
    for (int i = k; i < m; ++i) vv += ck[i] * ck[i];
    beta[k] = vv > 0.0 ? 2.0 / vv : 0.0;
    for (int j = k + 1; j < n; ++j) {
      double* cj = &Cm[static_cast<size_t>(j) * m];
      double d = 0.0;
      for (int i = k; i < m; ++i) d += ck[i] * cj[i];
      d *= beta[k];
      for (int i = k; i < m; ++i) cj[i] -= d * ck[i];
    }
    diag[k] = alpha;
  }
  std::vector<double> R(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i) {
    R[static_cast<size_t>(i) * n + i] = diag[i];
    for (int j = i + 1; j < n; ++j) R[static_cast<size_t>(i) * n + j] = Cm[static_cast<size_t>(j) * m + i];
  }
  std::vector<double> UR;
  jacobi_svd(n, n, std::move(R), sigma, UR, V);
  // U = H_0 ... H_{n-1} [U_R; 0], column by column
  U.assign(static_cast<size_t>(m) * n, 0.0);
  std::vector<double> w(m);
  for (int c = 0; c < n; ++c) {
    std::fill(w.begin(), w.end(), 0.0);
    for (int i = 0; i < n; ++i) w[i] = UR[static_cast<size_t>(i) * n + c];
    for (int k = n - 1; k >= 0; --k) {
      if (beta[k] == 0.0) continue;
      const double* vk = &Cm[static_cast<size_t>(k) * m];
      double d = 0.0;
      for (int i = k; i < m; ++i) d += vk[i] * w[i];
      d *= beta[k];
      for (int i = k; i < m; ++i) w[i] -= d * vk[i];
    }
    for (int i = 0; i < m; ++i) U[static_cast<size_t>(i) * n + c] = w[i];
  }
}

double Ctf::chi(double y, double tau) const {
  const double s = y / (2.0 * pixel);
  const double s2 = s * s;
  return kPi * lambda * tau * s2 - 0.5 * kPi * cs * lambda * lambda * lambda * s2 * s2;
}

double Ctf::operator()(double y, double tau) const {
  if (!on) return 1.0;
  const double c = chi(y, tau);
  return -(std::sqrt(1.0 - amp * amp) * std::sin(c) + amp * std::cos(c));
}

Ctf make_ctf(double wavelength_A, double cs_mm, double amplitude_contrast, double pixel_A, double tmin_A,
             double tmax_A) {
  for (double v : {wavelength_A, cs_mm, amplitude_contrast, pixel_A, tmin_A, tmax_A})
    if (!std::isfinite(v)) throw std::invalid_argument("ctf: non-finite parameter");
  if (wavelength_A < 0.0 || wavelength_A > 1.0) throw std::invalid_argument("ctf: wavelength must be in [0, 1] A");
  if (cs_mm < 0.0 || cs_mm > 100.0) throw std::invalid_argument("ctf: Cs must be in [0, 100] mm");
  if (amplitude_contrast < 0.0 || amplitude_contrast > 1.0)
    throw std::invalid_argument("ctf: amplitude contrast must be in [0, 1]");
  if (!(pixel_A > 0.0) || pixel_A > 100.0) throw std::invalid_argument("ctf: pixel size must be in (0, 100] A");
  if (!(tmax_A > tmin_A) || std::fabs(tmin_A) > 1e6 || std::fabs(tmax_A) > 1e6)
    throw std::invalid_argument("ctf: defocus range must satisfy tmin < tmax, |tau| <= 1e6 A");
  Ctf c;
  c.on = true;
  c.lambda = wavelength_A;
  c.cs = cs_mm * 1e7;
  c.amp = amplitude_contrast;
  c.pixel = pixel_A;
  c.tmin = tmin_A;
  c.tmax = tmax_A;
  return c;
}

double ModalSVD::kernel(double x, double y, double tau) const {
  std::vector<double> J(ell + 1);
  bessel_orders(ell, x * y, J.data());
  return J[ell] * ctf(y, tau);
}

double ModalSVD::sigma_v(int eta, double y) const {
  std::vector<double> J(ell + 1);
  std::vector<double> c(Pt, 1.0);
  if (ctf.on)
    for (int t = 0; t < Pt; ++t) c[t] = ctf(y, tn[t]) * std::sqrt(tw[t]);
  double s = 0.0;
  for (int i = 0; i < P; ++i) {
    bessel_orders(ell, xn[i] * y, J.data());
    for (int t = 0; t < Pt; ++t) s += std::sqrt(xw[i]) * c[t] * J[ell] * U[static_cast<size_t>(i * Pt + t) * Py + eta];
  }
  return s;
}

double ModalSVD::u(int eta, double x, double tau) const {
  std::vector<double> J(ell + 1);
  double s = 0.0;
  for (int j = 0; j < Py; ++j) {
    bessel_orders(ell, x * yn[j], J.data());
    s += std::sqrt(yw[j]) * J[ell] * ctf(yn[j], tau) * V[static_cast<size_t>(j) * Py + eta];
  }
  return s / sigma[eta];
}

double Weight::operator()(double y) const {
  if (alpha.empty()) return 1.0;
  double s = 0.0;
  for (size_t j = 0; j < alpha.size(); ++j) s += alpha[j] * std::exp(-beta[j] * y * y);
  return c * s;
}

Weight make_weight(const double* alpha, const double* beta, int nterms) {
  Weight w;
  if (nterms <= 0) return w;
  if (!alpha || !beta) throw std::invalid_argument("weight: NULL terms");
  double total = 0.0, amax = 0.0;
  for (int j = 0; j < nterms; ++j) {
    const double a = alpha[j], b = beta[j];
    if (!std::isfinite(a) || !std::isfinite(b) || a < 0.0 || b < 0.0)
      throw std::invalid_argument("weight: alpha and beta must be finite and >= 0");
    // int_0^1 a exp(-b y^2) y dy
    total += b > 0.0 ? a * (-std::expm1(-b)) / (2.0 * b) : 0.5 * a;
    amax = std::max(amax, a);
    w.alpha.push_back(a);
    w.beta.push_back(b);
  }
  if (!(amax > 0.0) || !(total > 0.0)) throw std::invalid_argument("weight: every alpha is 0");
  w.c = 0.5 / total;
  return w;
}

ModalSVD modal_svd(int ell, double X, const Weight& weight) {
  if (ell < 0) throw std::invalid_argument("modal_svd: ell >= 0 expected");
  ModalSVD r;
  r.ell = ell;
  r.X = X;
  r.P = static_cast<int>(std::ceil(X)) + 32;
  r.Py = r.P;
  const int P = r.P;
  radial_rule(P, X, r.xn, r.xw);
  radial_rule(P, 1.0, r.yn, r.yw);
  if (!weight.empty())
    for (int j = 0; j < P; ++j) r.yw[j] *= weight(r.yn[j]);
  std::vector<double> K(static_cast<size_t>(P) * P);
  std::vector<double> J(ell + 1);
  for (int i = 0; i < P; ++i)
    for (int j = 0; j < P; ++j) {
      bessel_orders(ell, r.xn[i] * r.yn[j], J.data());
      K[i * P + j] = std::sqrt(r.xw[i]) * J[ell] * std::sqrt(r.yw[j]);
    }
  jacobi_svd(P, P, std::move(K), r.sigma, r.U, r.V);
  return r;
}

ModalSVD ctf_modal_svd(int ell, double X, const Ctf& ctf) {
  if (ell < 0) throw std::invalid_argument("ctf_modal_svd: ell >= 0 expected");
  ModalSVD r;
  r.ell = ell;
  r.X = X;
  r.ctf = ctf;
  // x nodes as the translation SVD; tau nodes for the phase range of chi at
  // Nyquist over the defocus range; y nodes for the oscillation of C in y
  double chimax = 0.0;
  for (int i = 0; i <= 256; ++i)
    for (double t : {ctf.tmin, ctf.tmax}) chimax = std::max(chimax, std::fabs(ctf.chi(i / 256.0, t)));
  const double dchi = kPi * ctf.lambda * (ctf.tmax - ctf.tmin) / (4.0 * ctf.pixel * ctf.pixel);
  r.P = static_cast<int>(std::ceil(X)) + 32;
  r.Pt = static_cast<int>(std::ceil(dchi)) + 12;
  r.Py = r.P + static_cast<int>(std::ceil(2.0 * chimax)) + 24;
  const int P = r.P, Pt = r.Pt, Py = r.Py;
  radial_rule(P, X, r.xn, r.xw);
  radial_rule(Py, 1.0, r.yn, r.yw);
  legendre_rule01(Pt, r.tn, r.tw);  // weights of mass 1
  for (int t = 0; t < Pt; ++t) r.tn[t] = ctf.tmin + r.tn[t] * (ctf.tmax - ctf.tmin);
  if (P * Pt < Py) throw std::invalid_argument("ctf_modal_svd: fewer shift-side than k-side nodes");
  std::vector<double> C(static_cast<size_t>(Pt) * Py);
  for (int t = 0; t < Pt; ++t)
    for (int j = 0; j < Py; ++j) C[static_cast<size_t>(t) * Py + j] = ctf(r.yn[j], r.tn[t]);
  std::vector<double> A(static_cast<size_t>(P) * Pt * Py);
  std::vector<double> J(ell + 1);
  for (int i = 0; i < P; ++i)
    for (int j = 0; j < Py; ++j) {
      bessel_orders(ell, r.xn[i] * r.yn[j], J.data());
      for (int t = 0; t < Pt; ++t)
        A[static_cast<size_t>(i * Pt + t) * Py + j] =
            std::sqrt(r.xw[i] * r.tw[t]) * J[ell] * C[static_cast<size_t>(t) * Py + j] * std::sqrt(r.yw[j]);
    }
  qr_jacobi_svd(P * Pt, Py, A, r.sigma, r.U, r.V);
  return r;
}

Truncation truncate(double X, double eps, const Weight& weight, const Ctf& ctf) {
  Truncation tr;
  std::vector<int> keep_count;
  // modes in batches, one thread each (the CTF kernel's SVDs are the costly ones)
  const int batch = ctf.on ? std::max(1u, std::min(16u, std::thread::hardware_concurrency())) : 1;
  bool done = false;
  for (int ell0 = 0; ell0 < 4096 && !done; ell0 += batch) {
    std::vector<ModalSVD> got(batch);
    if (batch == 1) {
      got[0] = modal_svd(ell0, X, weight);
    } else {
      std::vector<std::thread> th;
      std::vector<std::string> err(batch);
      for (int b = 0; b < batch; ++b)
        th.emplace_back([&, b] {
          try {
            got[b] = ctf_modal_svd(ell0 + b, X, ctf);
          } catch (const std::exception& ex) {
            err[b] = ex.what();
          }
        });
      for (auto& t : th) t.join();
      for (const auto& e : err)
        if (!e.empty()) throw std::invalid_argument(e);
    }
    for (int b = 0; b < batch; ++b) {
      ModalSVD& s = got[b];
      if (s.sigma[0] <= eps) {
        tr.sigma_next = std::max(tr.sigma_next, s.sigma[0]);
        done = true;
        break;
      }
      int h = 0;
      const int ns = static_cast<int>(s.sigma.size());
      while (h < ns && s.sigma[h] > eps) ++h;
      if (h < ns) tr.sigma_next = std::max(tr.sigma_next, s.sigma[h]);
      keep_count.push_back(h);
      tr.svds.push_back(std::move(s));
    }
  }
  tr.L = static_cast<int>(keep_count.size()) - 1;
  for (int ell = -tr.L; ell <= tr.L; ++ell) {
    const ModalSVD& s = tr.svds[std::abs(ell)];
    for (int e = 0; e < keep_count[std::abs(ell)]; ++e) tr.terms.push_back({ell, e, s.sigma[e]});
  }
  return tr;
}

double SpreadKernel::ft(double s) const {
  static thread_local std::vector<double> z, wz;
  if (z.empty()) legendre_rule01(160, z, wz);
  double acc = 0.0;
  for (size_t i = 0; i < z.size(); ++i) {
    double zz = z[i];
    double phi = std::exp(beta * (std::sqrt(std::max(0.0, 1.0 - zz * zz)) - 1.0));
    acc += wz[i] * phi * std::cos(s * alpha * zz);
  }
  return 2.0 * alpha * acc;
}

bool fft_supported(int L) {
  if (L < 2 || L > 4096) return false;
  while (L % 2 == 0) L /= 2;
  while (L % 3 == 0) L /= 3;
  return L == 1;
}

int fft_size(int n) {
  for (int L = std::max(n, 2); L <= 4096; ++L)
    if (fft_supported(L)) return L;
  return 0;  // beyond the largest supported length
}

SpreadKernel spread_kernel(int n, int w) {
  SpreadKernel k;
  k.w = w;
  k.beta = 2.30 * w;
  k.nf = fft_size(2 * n);
  k.h = 2.0 * kPi / k.nf;
  k.alpha = 0.5 * w * k.h;
  return k;
}

}  // namespace ftkplan
