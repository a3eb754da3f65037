// Host FP64 finisher: Cholesky, symmetric eigendecomposition and the CVA
// generalized symmetric-definite solve from class moments.
//
// The paper's C implementation calls a generalized symmetric-definite
// eigensolver on the within- and between-class matrices (Section 4); this
// file solves the same problem, S_b w = lambda (S_w + ridge I) w, by the
// textbook reduction: Cholesky S_w = L L^T, then the ordinary symmetric
// problem for L^-1 S_b L^-T, then w = L^-T u.  Because
// S_b = D D^T with D = [sqrt(n_k) (m_k - m)] (B x K), the nonzero part of
// that symmetric problem is also the one of the K x K Gram matrix
// E^T E with E = L^-1 D: if E^T E u' = s u' then u = E u' / sqrt(s) is a
// unit eigenvector of E E^T with the same eigenvalue.  The smaller of the
// two problems is solved.
#include "finisher.h"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <numeric>
#include <vector>

#include "cvamx.h"

namespace cvamx {

// The O(n^3) loops of the eigensolver are built twice, for AVX2 + FMA
// processors and for the baseline, and the loader picks one at run time.
#define CVX_HOST_SIMD __attribute__((target_clones("arch=haswell", "default")))

int cholesky_lower(int n, const double* A, double* L) {
  std::fill(L, L + (size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    const double ajj = A[(size_t)j * n + j];
    double s = ajj;
    for (int k = 0; k < j; ++k) s -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
    // A pivot that lost all but ~13 digits of its diagonal entry is treated
    // as zero: S_w is then singular to working precision.
    if (!std::isfinite(s) || !(s > 1e-13 * std::fabs(ajj))) return CVAMX_E_NOT_PD;
    const double d = std::sqrt(s);
    L[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double t = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      L[(size_t)i * n + j] = t / d;
    }
  }
  return 0;
}

// Householder reduction of the full symmetric matrix T (in place) to
// tridiagonal form, accumulating the reflectors into Q so that the input
// equals Q T Q^T.
CVX_HOST_SIMD static void tridiagonalize(int n, double* T, double* Q) {
  std::vector<double> v(n), p(n), w(n);
  for (int k = 0; k + 2 < n; ++k) {
    double xx = 0.0;
    for (int i = k + 1; i < n; ++i) xx += T[(size_t)i * n + k] * T[(size_t)i * n + k];
    if (xx == 0.0) continue;
    const double xnorm = std::sqrt(xx);
    const double x0 = T[(size_t)(k + 1) * n + k];
    const double alpha = (x0 > 0.0) ? -xnorm : xnorm;
    for (int i = k + 1; i < n; ++i) v[i] = T[(size_t)i * n + k];
    v[k + 1] -= alpha;
    double vtv = 0.0;
    for (int i = k + 1; i < n; ++i) vtv += v[i] * v[i];
    if (vtv == 0.0) continue;
    const double beta = 2.0 / vtv;
    double pv = 0.0;
    for (int i = k + 1; i < n; ++i) {
      double s = 0.0;
      for (int j = k + 1; j < n; ++j) s += T[(size_t)i * n + j] * v[j];
      p[i] = beta * s;
      pv += p[i] * v[i];
    }
    const double half = 0.5 * beta * pv;
    for (int i = k + 1; i < n; ++i) w[i] = p[i] - half * v[i];
    for (int i = k + 1; i < n; ++i)
      for (int j = k + 1; j < n; ++j)
        T[(size_t)i * n + j] -= v[i] * w[j] + w[i] * v[j];
    T[(size_t)(k + 1) * n + k] = alpha;
    T[(size_t)k * n + (k + 1)] = alpha;
    for (int i = k + 2; i < n; ++i) {
      T[(size_t)i * n + k] = 0.0;
      T[(size_t)k * n + i] = 0.0;
    }
    for (int r = 0; r < n; ++r) {
      double s = 0.0;
      for (int j = k + 1; j < n; ++j) s += Q[(size_t)r * n + j] * v[j];
      s *= beta;
      for (int j = k + 1; j < n; ++j) Q[(size_t)r * n + j] -= s * v[j];
    }
  }
}

// sqrt(x^2 + z^2): the plain formula where the squares can neither
// overflow nor lose precision to underflow, std::hypot otherwise.
static inline double norm2(double x, double z) {
  const double ax = std::fabs(x), az = std::fabs(z);
  const double big = ax > az ? ax : az;
  if (big > 1e-150 && big < 1e150) return std::sqrt(x * x + z * z);
  return std::hypot(x, z);
}

// Implicit symmetric QR steps with a Wilkinson shift on the tridiagonal T
// (stored dense), deflating negligible off-diagonal entries, with the
// rotations accumulated into Zt = Q^T (row i of Zt is column i of Q, so a
// rotation of two columns of Q touches two contiguous rows).
CVX_HOST_SIMD static int tridiagonal_qr(int n, double* T, double* Zt) {
  const int maxit = 60 * n + 100;
  int it = 0;
  int m = n - 1;
  auto at = [&](int i, int j) -> double& { return T[(size_t)i * n + j]; };
  while (m > 0) {
    for (int i = 0; i < m; ++i) {
      if (std::fabs(at(i + 1, i)) <= DBL_EPSILON * (std::fabs(at(i, i)) + std::fabs(at(i + 1, i + 1)))) {
        at(i + 1, i) = 0.0;
        at(i, i + 1) = 0.0;
      }
    }
    while (m > 0 && at(m, m - 1) == 0.0) --m;
    if (m == 0) break;
    int l = m - 1;
    while (l > 0 && at(l, l - 1) != 0.0) --l;
    if (++it > maxit) return CVAMX_E_NUMERIC;
    const double a = at(m - 1, m - 1), b = at(m, m - 1), c = at(m, m);
    const double d = 0.5 * (a - c);
    const double den = d + std::copysign(norm2(d, b), d);
    const double mu = (den != 0.0) ? c - b * b / den : c - std::fabs(b);
    double x = at(l, l) - mu;
    double z = at(l + 1, l);
    for (int k = l; k < m; ++k) {
      const double r = norm2(x, z);
      const double cs = (r == 0.0) ? 1.0 : x / r;
      const double sn = (r == 0.0) ? 0.0 : -z / r;
      const int lo = std::max(l, k - 1), hi = std::min(m, k + 2);
      for (int j = lo; j <= hi; ++j) {
        const double t1 = at(k, j), t2 = at(k + 1, j);
        at(k, j) = cs * t1 - sn * t2;
        at(k + 1, j) = sn * t1 + cs * t2;
      }
      for (int i = lo; i <= hi; ++i) {
        const double t1 = at(i, k), t2 = at(i, k + 1);
        at(i, k) = cs * t1 - sn * t2;
        at(i, k + 1) = sn * t1 + cs * t2;
      }
      double* __restrict__ z1 = Zt + (size_t)k * n;
      double* __restrict__ z2 = z1 + n;
      for (int i = 0; i < n; ++i) {
        const double q1 = z1[i], q2 = z2[i];
        z1[i] = cs * q1 - sn * q2;
        z2[i] = sn * q1 + cs * q2;
      }
      if (k + 1 < m) {
        x = at(k + 1, k);
        z = at(k + 2, k);
      }
    }
  }
  return 0;
}

int sym_eig_desc(int n, const double* A, double* w, double* V) {
  std::vector<double> T((size_t)n * n), Q((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) {
      T[(size_t)i * n + j] = A[(size_t)i * n + j];
      T[(size_t)j * n + i] = A[(size_t)i * n + j];
    }
  for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
  if (n > 2) tridiagonalize(n, T.data(), Q.data());
  std::vector<double> Zt((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Zt[(size_t)j * n + i] = Q[(size_t)i * n + j];
  const int st = tridiagonal_qr(n, T.data(), Zt.data());
  if (st != 0) return st;
  std::vector<int> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
    return T[(size_t)a * n + a] > T[(size_t)b * n + b];
  });
  for (int j = 0; j < n; ++j) {
    w[j] = T[(size_t)ord[j] * n + ord[j]];
    for (int i = 0; i < n; ++i) V[(size_t)i * n + j] = Zt[(size_t)ord[j] * n + i];
  }
  return 0;
}

void sign_rule(int rows, int nc, double* W) {
  for (int j = 0; j < nc; ++j) {
    int best = 0;
    double bv = -1.0;
    for (int i = 0; i < rows; ++i) {
      const double a = std::fabs(W[(size_t)i * nc + j]);
      if (a > bv) {
        bv = a;
        best = i;
      }
    }
    if (W[(size_t)best * nc + j] < 0.0)
      for (int i = 0; i < rows; ++i) W[(size_t)i * nc + j] = -W[(size_t)i * nc + j];
  }
}

int cva_solve(int K, int B, const double* cnt, const double* cm, const double* Sw,
              double ridge, int nc, double* W, double* eig, double* mean,
              double* Sb_out, std::string* err) {
  const int C = std::min(K - 1, B);
  if (K < 2 || B < 1 || nc < 1 || nc > C || !(ridge >= 0.0)) {
    if (err) *err = "cva_solve: need K >= 2, B >= 1, 1 <= n_comp <= min(K-1, B), ridge >= 0";
    return CVAMX_E_INVALID_ARG;
  }
  double N = 0.0;
  for (int k = 0; k < K; ++k) {
    if (!(cnt[k] > 0.0)) {
      if (err) *err = "cva_solve: class " + std::to_string(k) + " has no training weight";
      return CVAMX_E_EMPTY_CLASS;
    }
    N += cnt[k];
  }
  std::vector<double> m(B, 0.0);
  for (int k = 0; k < K; ++k)
    for (int b = 0; b < B; ++b) m[b] += cnt[k] * cm[(size_t)k * B + b];
  for (int b = 0; b < B; ++b) m[b] /= N;

  std::vector<double> A((size_t)B * B), L((size_t)B * B);
  for (int i = 0; i < B; ++i)
    for (int j = 0; j < B; ++j)
      A[(size_t)i * B + j] = 0.5 * (Sw[(size_t)i * B + j] + Sw[(size_t)j * B + i]) + (i == j ? ridge : 0.0);
  if (cholesky_lower(B, A.data(), L.data()) != 0) {
    if (err) *err = "cva_solve: S_w + ridge I is not positive definite";
    return CVAMX_E_NOT_PD;
  }
  // E = L^-1 D, D[:, k] = sqrt(n_k) (m_k - m)
  std::vector<double> E((size_t)B * K);
  for (int k = 0; k < K; ++k) {
    const double sq = std::sqrt(cnt[k]);
    for (int i = 0; i < B; ++i) {
      double t = sq * (cm[(size_t)k * B + i] - m[i]);
      for (int j = 0; j < i; ++j) t -= L[(size_t)i * B + j] * E[(size_t)j * K + k];
      E[(size_t)i * K + k] = t / L[(size_t)i * B + i];
    }
  }
  std::vector<double> U((size_t)B * nc), lam(nc);
  bool done = false;
  if (K <= B) {
    std::vector<double> G((size_t)K * K), s(K), V((size_t)K * K);
    for (int a = 0; a < K; ++a)
      for (int b = 0; b < K; ++b) {
        double t = 0.0;
        for (int i = 0; i < B; ++i) t += E[(size_t)i * K + a] * E[(size_t)i * K + b];
        G[(size_t)a * K + b] = t;
      }
    const int st = sym_eig_desc(K, G.data(), s.data(), V.data());
    if (st != 0) {
      if (err) *err = "cva_solve: eigensolver did not converge";
      return st;
    }
    if (s[0] > 0.0 && s[C - 1] > 1e-10 * s[0]) {
      for (int j = 0; j < nc; ++j) {
        const double inv = 1.0 / std::sqrt(s[j]);
        for (int i = 0; i < B; ++i) {
          double t = 0.0;
          for (int a = 0; a < K; ++a) t += E[(size_t)i * K + a] * V[(size_t)a * K + j];
          U[(size_t)i * nc + j] = t * inv;
        }
        lam[j] = s[j];
      }
      done = true;
    }
  }
  if (!done) {
    std::vector<double> M((size_t)B * B), s(B), V((size_t)B * B);
    for (int i = 0; i < B; ++i)
      for (int j = 0; j < B; ++j) {
        double t = 0.0;
        for (int a = 0; a < K; ++a) t += E[(size_t)i * K + a] * E[(size_t)j * K + a];
        M[(size_t)i * B + j] = t;
      }
    const int st = sym_eig_desc(B, M.data(), s.data(), V.data());
    if (st != 0) {
      if (err) *err = "cva_solve: eigensolver did not converge";
      return st;
    }
    for (int j = 0; j < nc; ++j) {
      for (int i = 0; i < B; ++i) U[(size_t)i * nc + j] = V[(size_t)i * B + j];
      lam[j] = s[j];
    }
  }
  // W = L^-T U (back substitution)
  std::vector<double> Wt((size_t)B * nc);
  for (int j = 0; j < nc; ++j) {
    for (int i = B - 1; i >= 0; --i) {
      double t = U[(size_t)i * nc + j];
      for (int r = i + 1; r < B; ++r) t -= L[(size_t)r * B + i] * Wt[(size_t)r * nc + j];
      Wt[(size_t)i * nc + j] = t / L[(size_t)i * B + i];
    }
  }
  sign_rule(B, nc, Wt.data());
  std::copy(Wt.begin(), Wt.end(), W);
  std::copy(lam.begin(), lam.end(), eig);
  if (mean) std::copy(m.begin(), m.end(), mean);
  if (Sb_out) {
    for (int i = 0; i < B; ++i)
      for (int j = 0; j < B; ++j) {
        double t = 0.0;
        for (int k = 0; k < K; ++k)
          t += cnt[k] * (cm[(size_t)k * B + i] - m[i]) * (cm[(size_t)k * B + j] - m[j]);
        Sb_out[(size_t)i * B + j] = t;
      }
  }
  return 0;
}

}  // namespace cvamx

extern "C" int cva_solve_moments(const int64_t* counts, const double* class_means,
                                 const double* Sw, int32_t K, int32_t B, double ridge,
                                 int32_t n_comp, double* W, double* eigvals, double* mean) {
  if (!counts || !class_means || !Sw || !W || !eigvals) return CVAMX_E_INVALID_ARG;
  if (K < 2 || K > CVAMX_MAX_CLASSES || B < 1 || B > CVAMX_MAX_BANDS) return CVAMX_E_INVALID_ARG;
  std::vector<double> c(K);
  for (int k = 0; k < K; ++k) c[k] = (double)counts[k];
  return cvamx::cva_solve(K, B, c.data(), class_means, Sw, ridge, n_comp, W, eigvals, mean,
                          nullptr, nullptr);
}

extern "C" int cvamx_sym_eig(int32_t n, const double* A, double* w, double* V) {
  if (!A || !w || !V || n < 1 || n > 4096) return CVAMX_E_INVALID_ARG;
  const int st = cvamx::sym_eig_desc(n, A, w, V);
  if (st != 0) return st;
  cvamx::sign_rule(n, n, V);
  return 0;
}
