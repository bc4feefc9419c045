// FP64 formation of the small 1-D operators on the host: finite-difference
// generators (Section 4.1), the matrix exponential E = exp(c A) of a small
// dense matrix (Section 2: the d exponentials are precomputed once for a
// constant step), and Gauss-Hermite nodes, weights and transform matrices
// (Section 3).  None of this is on the per-step path.
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "../../include/mumode.h"

namespace {

typedef std::complex<double> cd;

// C = A B, n x n complex, column-major.
void matmul(int n, const cd* A, const cd* B, cd* C) {
  for (int j = 0; j < n; ++j) {
    cd* c = C + (size_t)j * n;
    for (int i = 0; i < n; ++i) c[i] = 0.0;
    for (int k = 0; k < n; ++k) {
      const cd b = B[k + (size_t)j * n];
      if (b == 0.0) continue;
      const cd* a = A + (size_t)k * n;
      for (int i = 0; i < n; ++i) c[i] += a[i] * b;
    }
  }
}

double norm1(int n, const cd* A) {
  double m = 0.0;
  for (int j = 0; j < n; ++j) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += std::abs(A[i + (size_t)j * n]);
    m = std::max(m, s);
  }
  return m;
}

// Orthonormal Hermite functions phi_0..phi_{kmax-1} at x (three-term
// recurrence normalised for H_k exp(-x^2/2)).
void hermite_values(int kmax, double x, double* phi) {
  phi[0] = std::pow(M_PI, -0.25) * std::exp(-0.5 * x * x);
  if (kmax > 1) phi[1] = std::sqrt(2.0) * x * phi[0];
  for (int k = 1; k + 1 < kmax; ++k)
    phi[k + 1] = std::sqrt(2.0 / (k + 1)) * x * phi[k] - std::sqrt((double)k / (k + 1)) * phi[k - 1];
}

// Number of eigenvalues below x of the symmetric tridiagonal Jacobi matrix of
// the Hermite recurrence (zero diagonal, off-diagonal sqrt(k/2)), by the
// Sturm sequence of its leading principal minors.
int sturm_count(int m, double x) {
  int cnt = 0;
  double q = -x;
  if (q < 0) ++cnt;
  for (int k = 1; k < m; ++k) {
    const double b2 = 0.5 * k;
    if (q == 0.0) q = 1e-300;
    q = -x - b2 / q;
    if (q < 0) ++cnt;
  }
  return cnt;
}

}  // namespace

extern "C" {

mm_status mm_fd2_matrix(int n, double a, double b, int bc, double* out) {
  if (!out) return MM_ERR_ARG;
  if (n < 1 || n > 65536 || !(b > a)) return MM_ERR_SHAPE;
  if (bc != 0 && bc != 1) return MM_ERR_ARG;
  if (bc == 1 && n < 3) return MM_ERR_SHAPE;
  const double h = bc == 0 ? (b - a) / (n + 1) : (b - a) / n;
  const double s = 1.0 / (h * h);
  std::memset(out, 0, sizeof(double) * (size_t)n * n);
  for (int j = 0; j < n; ++j) {
    out[j + (size_t)j * n] = -2.0 * s;
    if (j > 0) out[j + (size_t)(j - 1) * n] = s;
    if (j + 1 < n) out[j + (size_t)(j + 1) * n] = s;
  }
  if (bc == 1) {
    out[0 + (size_t)(n - 1) * n] += s;
    out[(n - 1) + 0] += s;
  }
  return MM_OK;
}

mm_status mm_expm(int n, const double* A, double c_re, double c_im, double* out) {
  if (!A || !out) return MM_ERR_ARG;
  if (n < 1 || n > 4096) return MM_ERR_SHAPE;
  const size_t nn = (size_t)n * n;
  const cd c(c_re, c_im);
  std::vector<cd> X(nn), T(nn), W(nn);
  for (size_t e = 0; e < nn; ++e) {
    const cd v = c * cd(A[2 * e], A[2 * e + 1]);
    if (!std::isfinite(v.real()) || !std::isfinite(v.imag())) return MM_ERR_NONFINITE;
    X[e] = v;
  }
  // scaling: ||X / 2^s||_1 <= 1/2
  const double nrm = norm1(n, X.data());
  int s = 0;
  if (nrm > 0.5) s = (int)std::ceil(std::log2(nrm / 0.5));
  const double sc = std::ldexp(1.0, -s);
  for (auto& v : X) v *= sc;
  // Taylor polynomial of degree 18 by Horner's rule: the truncation error
  // for ||X|| <= 1/2 is below 0.5^19 / 19! ~ 1.6e-23.
  const int deg = 18;
  for (size_t e = 0; e < nn; ++e) T[e] = 0.0;
  for (int i = 0; i < n; ++i) T[i + (size_t)i * n] = 1.0;
  for (int k = deg; k >= 1; --k) {
    matmul(n, X.data(), T.data(), W.data());
    const double f = 1.0 / k;
    for (size_t e = 0; e < nn; ++e) T[e] = W[e] * f;
    for (int i = 0; i < n; ++i) T[i + (size_t)i * n] += 1.0;
  }
  // squaring
  for (int k = 0; k < s; ++k) {
    matmul(n, T.data(), T.data(), W.data());
    T.swap(W);
  }
  for (size_t e = 0; e < nn; ++e) {
    out[2 * e] = T[e].real();
    out[2 * e + 1] = T[e].imag();
  }
  return MM_OK;
}

mm_status mm_hermite_nodes(int m, double* X, double* w) {
  if (!X) return MM_ERR_ARG;
  if (m < 1 || m > 4096) return MM_ERR_SHAPE;
  // Gershgorin bound of the Jacobi matrix
  const double R = 2.0 * std::sqrt(0.5 * (m - 1)) + 1.0;
  std::vector<double> phi(m + 1);
  for (int k = 0; k < m; ++k) {
    // k-th eigenvalue (ascending) by bisection on the Sturm count
    double lo = -R, hi = R;
    for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(lo)); ++it) {
      const double mid = 0.5 * (lo + hi);
      if (sturm_count(m, mid) > k) hi = mid;
      else lo = mid;
    }
    double x = 0.5 * (lo + hi);
    // Newton polish on phi_m(x) = 0, phi_m' = sqrt(2m) phi_{m-1} - x phi_m
    for (int it = 0; it < 3; ++it) {
      hermite_values(m + 1, x, phi.data());
      const double f = phi[m];
      const double fp = std::sqrt(2.0 * m) * phi[m - 1] - x * phi[m];
      if (fp == 0.0) break;
      const double dx = f / fp;
      if (std::fabs(dx) > 1e-6 * std::max(1.0, std::fabs(x))) break;
      x -= dx;
    }
    X[k] = x;
  }
  if (w) {
    for (int k = 0; k < m; ++k) {
      hermite_values(m, X[k], phi.data());
      w[k] = 1.0 / (m * phi[m - 1] * phi[m - 1]);
    }
  }
  return MM_OK;
}

mm_status mm_hermite_matrices(int m, double* Phi, double* Psi) {
  if (m < 1 || m > 4096) return MM_ERR_SHAPE;
  std::vector<double> X(m), w(m), phi(m);
  mm_status st = mm_hermite_nodes(m, X.data(), w.data());
  if (st != MM_OK) return st;
  for (int l = 0; l < m; ++l) {
    hermite_values(m, X[l], phi.data());
    for (int k = 0; k < m; ++k) {
      if (Phi) Phi[k + (size_t)l * m] = phi[k] * w[l];   // Phi[k, l]
      if (Psi) Psi[l + (size_t)k * m] = phi[k];          // Psi[l, k]
    }
  }
  return MM_OK;
}

mm_status mm_hermite_ho_exponential(int m, double tau, double* out) {
  if (!out) return MM_ERR_ARG;
  if (m < 1 || m > 4096) return MM_ERR_SHAPE;
  if (!std::isfinite(tau)) return MM_ERR_ARG;
  std::vector<double> Phi((size_t)m * m), Psi((size_t)m * m);
  mm_status st = mm_hermite_matrices(m, Phi.data(), Psi.data());
  if (st != MM_OK) return st;
  // E = Psi diag(exp(-i tau (k + 1/2))) Phi: Hermite function k is an
  // eigenfunction of -1/2 (d^2 - x^2) with eigenvalue k + 1/2 (Section 3)
  std::vector<cd> ph(m);
  for (int k = 0; k < m; ++k) ph[k] = std::exp(cd(0.0, -tau * (k + 0.5)));
  for (int j = 0; j < m; ++j)
    for (int i = 0; i < m; ++i) {
      cd acc = 0.0;
      for (int k = 0; k < m; ++k) acc += Psi[i + (size_t)k * m] * ph[k] * Phi[k + (size_t)j * m];
      out[2 * (i + (size_t)j * m)] = acc.real();
      out[2 * (i + (size_t)j * m) + 1] = acc.imag();
    }
  return MM_OK;
}

mm_status mm_schrodinger_fd_hamiltonian(int n, double a, double b, double omega2, double* out) {
  if (!out) return MM_ERR_ARG;
  if (!std::isfinite(omega2)) return MM_ERR_ARG;
  mm_status st = mm_fd2_matrix(n, a, b, 0, out);
  if (st != MM_OK) return st;
  // H = -1/2 D2 + (omega2 / 2) diag(x^2) on the interior nodes x_j = a + j h
  const double h = (b - a) / (n + 1);
  for (size_t e = 0; e < (size_t)n * n; ++e) out[e] *= -0.5;
  for (int j = 0; j < n; ++j) {
    const double x = a + (j + 1) * h;
    out[j + (size_t)j * n] += 0.5 * omega2 * x * x;
  }
  return MM_OK;
}

mm_status mm_schrodinger_fd_exponential(int n, double a, double b, double omega2, double tau, double* out) {
  if (!out) return MM_ERR_ARG;
  if (!std::isfinite(tau)) return MM_ERR_ARG;
  if (n < 1 || n > 4096) return MM_ERR_SHAPE;
  std::vector<double> H((size_t)n * n), Hc(2 * (size_t)n * n, 0.0);
  mm_status st = mm_schrodinger_fd_hamiltonian(n, a, b, omega2, H.data());
  if (st != MM_OK) return st;
  for (size_t e = 0; e < H.size(); ++e) Hc[2 * e] = H[e];
  // i psi_t = H psi  =>  psi(tau) = exp(-i tau H) psi(0)
  return mm_expm(n, Hc.data(), 0.0, -tau, out);
}

mm_status mm_hermite_ho_generator(int m, double* out) {
  if (!out) return MM_ERR_ARG;
  if (m < 1 || m > 4096) return MM_ERR_SHAPE;
  std::vector<double> Phi((size_t)m * m), Psi((size_t)m * m);
  mm_status st = mm_hermite_matrices(m, Phi.data(), Psi.data());
  if (st != MM_OK) return st;
  // (i/2)(d^2 - x^2) phi_k = -i (k + 1/2) phi_k (Section 3), so in nodal
  // space the generator is Psi diag(-i (k + 1/2)) Phi (purely imaginary)
  for (int j = 0; j < m; ++j)
    for (int i = 0; i < m; ++i) {
      double acc = 0.0;
      for (int k = 0; k < m; ++k) acc += Psi[i + (size_t)k * m] * (k + 0.5) * Phi[k + (size_t)j * m];
      out[2 * (i + (size_t)j * m)] = 0.0;
      out[2 * (i + (size_t)j * m) + 1] = -acc;
    }
  return MM_OK;
}

mm_status mm_fd2_periodic_order(int n, double a, double b, int order, double* out) {
  if (!out) return MM_ERR_ARG;
  if (order < 2 || order > 16 || (order & 1)) return MM_ERR_ARG;
  const int m = order / 2;
  if (n < 2 * m + 1 || n > 65536 || !(b > a)) return MM_ERR_SHAPE;
  const double h = (b - a) / n;
  // w_k = 2 (-1)^(k+1) (m!)^2 / (k^2 (m-k)! (m+k)!), w_0 = -2 sum w_k
  std::vector<double> w(m + 1, 0.0);
  for (int k = 1; k <= m; ++k) {
    double r = 1.0;   // (m!)^2 / ((m-k)! (m+k)!) = prod_{i=1..k} (m-i+1)/(m+i)
    for (int i = 1; i <= k; ++i) r *= (double)(m - i + 1) / (double)(m + i);
    w[k] = 2.0 * ((k & 1) ? 1.0 : -1.0) * r / ((double)k * k);
    w[0] -= 2.0 * w[k];
  }
  std::memset(out, 0, sizeof(double) * (size_t)n * n);
  const double s2 = 1.0 / (h * h);
  for (int i = 0; i < n; ++i) {
    out[i + (size_t)i * n] += w[0] * s2;
    for (int k = 1; k <= m; ++k) {
      out[i + (size_t)((i + k) % n) * n] += w[k] * s2;
      out[i + (size_t)((i - k + n) % n) * n] += w[k] * s2;
    }
  }
  return MM_OK;
}

mm_status mm_fourier_d2(int n, double a, double b, double* out) {
  if (!out) return MM_ERR_ARG;
  if (n < 2 || n > 65536 || !(b > a)) return MM_ERR_SHAPE;
  // closed form of the periodic spectral second derivative on [0, 2 pi)
  // (h = 2 pi / n), scaled by (2 pi / L)^2 for the interval [a, b)
  const double h = 2.0 * M_PI / n;
  const double sc = (2.0 * M_PI / (b - a)) * (2.0 * M_PI / (b - a));
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      double v;
      if (i == j) {
        v = (n % 2 == 0) ? -M_PI * M_PI / (3.0 * h * h) - 1.0 / 6.0 : -M_PI * M_PI / (3.0 * h * h) + 1.0 / 12.0;
      } else {
        const int k = i - j;
        const double sg = (k & 1) ? -1.0 : 1.0;
        const double sn = std::sin(0.5 * k * h);
        v = (n % 2 == 0) ? -sg / (2.0 * sn * sn) : -sg * std::cos(0.5 * k * h) / (2.0 * sn * sn);
      }
      out[i + (size_t)j * n] = sc * v;
    }
  return MM_OK;
}

mm_status mm_pipe_flow_operators(int n_r, int n_z, double r_min, double r_max, double z_max, double alpha,
                                 double* A_r, double* A_z) {
  if (!A_r || !A_z) return MM_ERR_ARG;
  if (n_r < 3 || n_z < 3 || n_r > 65536 || n_z > 65536) return MM_ERR_SHAPE;
  if (!(r_min > 0.0) || !(r_max > r_min) || !(z_max > 0.0) || !std::isfinite(alpha)) return MM_ERR_ARG;
  std::memset(A_r, 0, sizeof(double) * (size_t)n_r * n_r);
  std::memset(A_z, 0, sizeof(double) * (size_t)n_z * n_z);
  // r: nodes r_min + i h (i = 0..n-1), Neumann at both ends by mirrored
  // ghost values (c_{-1} = c_1, c_n = c_{n-2})
  const double hr = (r_max - r_min) / (n_r - 1);
  for (int i = 0; i < n_r; ++i) {
    const double r = r_min + i * hr;
    const double lo = alpha * (1.0 / (hr * hr) - 0.5 / (hr * r));   // coefficient of c_{i-1}
    const double hi = alpha * (1.0 / (hr * hr) + 0.5 / (hr * r));   // coefficient of c_{i+1}
    const int il = i == 0 ? 1 : i - 1;
    const int ih = i == n_r - 1 ? n_r - 2 : i + 1;
    A_r[i + (size_t)i * n_r] += -2.0 * alpha / (hr * hr);
    A_r[i + (size_t)il * n_r] += lo;
    A_r[i + (size_t)ih * n_r] += hi;
  }
  // z: nodes j h (j = 1..n), c = 0 at z = 0, Neumann at z_max (c_{n+1} = c_{n-1})
  const double hz = z_max / n_z;
  for (int j = 0; j < n_z; ++j) {
    const double z = (j + 1) * hz;
    const double sv = 2.0 + std::tanh(4.0 * (z - 2.5)) - std::tanh(4.0 * (z - 5.0));
    const double lo = alpha / (hz * hz) + 0.5 * sv / hz;
    const double hi = alpha / (hz * hz) - 0.5 * sv / hz;
    A_z[j + (size_t)j * n_z] += -2.0 * alpha / (hz * hz);
    if (j > 0) A_z[j + (size_t)(j - 1) * n_z] += lo;
    const int jh = j == n_z - 1 ? n_z - 2 : j + 1;
    A_z[j + (size_t)jh * n_z] += hi;
  }
  return MM_OK;
}

mm_status mm_nonuniform_neumann_d2(int n, const double* x, double* M, double* w) {
  if (n < 2 || n > 4096 || !x || !M) return MM_ERR_ARG;
  for (int j = 0; j + 1 < n; ++j)
    if (!(x[j + 1] > x[j]) || !std::isfinite(x[j]) || !std::isfinite(x[j + 1])) return MM_ERR_SHAPE;
  // dual-cell widths: half of each neighbouring cell
  std::vector<double> wd(n, 0.0);
  for (int j = 0; j + 1 < n; ++j) {
    const double h = x[j + 1] - x[j];
    wd[j] += 0.5 * h;
    wd[j + 1] += 0.5 * h;
  }
  std::memset(M, 0, sizeof(double) * (size_t)n * n);
  // M = W^-1/2 S W^-1/2, S the stiffness of the fluxes (u_{j+1} - u_j) / h_j;
  // no flux through the ends (homogeneous Neumann)
  for (int j = 0; j + 1 < n; ++j) {
    const double c = 1.0 / (x[j + 1] - x[j]);
    const double off = c / std::sqrt(wd[j] * wd[j + 1]);
    M[(size_t)j * n + j] -= c / wd[j];
    M[(size_t)(j + 1) * n + (j + 1)] -= c / wd[j + 1];
    M[(size_t)(j + 1) * n + j] = off;
    M[(size_t)j * n + (j + 1)] = off;
  }
  if (w) std::memcpy(w, wd.data(), sizeof(double) * n);
  return MM_OK;
}

}  // extern "C"
