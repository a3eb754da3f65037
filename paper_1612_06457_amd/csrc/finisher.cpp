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

// Right-looking: after column j is final, its outer product is taken from
// the trailing rows at once (independent updates along each row, which
// vectorise), rather than one dot product per entry.
CVX_HOST_SIMD int cholesky_lower(int n, const double* A, double* L) {
  std::vector<double> S((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k <= i; ++k) S[(size_t)i * n + k] = A[(size_t)i * n + k];
  std::fill(L, L + (size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    const double ajj = A[(size_t)j * n + j];
    const double s = S[(size_t)j * n + j];
    // A pivot that lost all but ~13 digits of its diagonal entry is treated
    // as zero: S_w is then singular to working precision.
    if (!std::isfinite(s) || !(s > 1e-13 * std::fabs(ajj))) return CVAMX_E_NOT_PD;
    const double d = std::sqrt(s), inv = 1.0 / d;
    L[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) L[(size_t)i * n + j] = S[(size_t)i * n + j] * inv;
    for (int i = j + 1; i < n; ++i) {
      const double lij = L[(size_t)i * n + j];
      double* __restrict__ si = S.data() + (size_t)i * n;
      const double* __restrict__ lk = L + j;
      for (int k = j + 1; k <= i; ++k) si[k] -= lij * lk[(size_t)k * n];
    }
  }
  return 0;
}

// Householder reduction of the full symmetric matrix T (in place) to
// tridiagonal form, accumulating the reflectors into Q so that the input
// equals Q T Q^T.
// With Q null the reflectors are kept instead: row k of Vh holds v_k
// (entries k + 1 .. n - 1) and bk[k] its 2 / v^T v (0: no reflection), and
// the input equals H_0 H_1 ... T ... H_1 H_0 with H_k = I - bk[k] v_k v_k^T.
CVX_HOST_SIMD static void tridiagonalize(int n, double* T, double* Q, double* Vh = nullptr,
                                         double* bk = nullptr) {
  std::vector<double> v(n), p(n), w(n);
  if (bk) std::fill(bk, bk + n, 0.0);
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
    if (!Q) {
      for (int j = k + 1; j < n; ++j) Vh[(size_t)k * n + j] = v[j];
      bk[k] = beta;
      continue;
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

// Implicit symmetric QR steps with a Wilkinson shift on the tridiagonal
// matrix with diagonal d and off-diagonal e (e[i] couples i and i + 1),
// deflating negligible off-diagonal entries.  Each step chases the bulge
// down the unreduced block with Givens rotations of rows and columns
// (k, k + 1), updating the few entries they touch; the rotations are
// accumulated into Zt = Q^T (row i of Zt is column i of Q, so a rotation of
// two columns of Q touches two contiguous rows), or not at all when Zt is
// null.  The eigenvalues are left in d.
CVX_HOST_SIMD static int tridiagonal_qr(int n, double* d, double* e, double* Zt) {
  const int maxit = 60 * n + 100;
  int it = 0;
  int m = n - 1;
  while (m > 0) {
    for (int i = 0; i < m; ++i)
      if (std::fabs(e[i]) <= DBL_EPSILON * (std::fabs(d[i]) + std::fabs(d[i + 1]))) e[i] = 0.0;
    while (m > 0 && e[m - 1] == 0.0) --m;
    if (m == 0) break;
    int l = m - 1;
    while (l > 0 && e[l - 1] != 0.0) --l;
    if (++it > maxit) return CVAMX_E_NUMERIC;
    const double a = d[m - 1], b = e[m - 1], c = d[m];
    const double dd = 0.5 * (a - c);
    const double den = dd + std::copysign(norm2(dd, b), dd);
    const double mu = (den != 0.0) ? c - b * b / den : c - std::fabs(b);
    double x = d[l] - mu;
    double z = e[l];
    for (int k = l; k < m; ++k) {
      const double r = norm2(x, z);
      const double cs = (r == 0.0) ? 1.0 : x / r;
      const double sn = (r == 0.0) ? 0.0 : z / r;
      if (k > l) e[k - 1] = r;
      // rows k, k + 1 of the 2 x 2 block, then its columns
      const double p = d[k], q = e[k], t = d[k + 1];
      const double r00 = cs * p + sn * q, r01 = cs * q + sn * t;
      const double r10 = -sn * p + cs * q, r11 = -sn * q + cs * t;
      d[k] = cs * r00 + sn * r01;
      e[k] = cs * r10 + sn * r11;
      d[k + 1] = -sn * r10 + cs * r11;
      if (k + 1 < m) {
        // the rotation of rows k, k + 1 moves part of e[k + 1] into the
        // bulge at (k, k + 2)
        z = sn * e[k + 1];
        e[k + 1] = cs * e[k + 1];
        x = e[k];
      }
      if (Zt) {
        double* __restrict__ z1 = Zt + (size_t)k * n;
        double* __restrict__ z2 = z1 + n;
        for (int i = 0; i < n; ++i) {
          const double q1 = z1[i], q2 = z2[i];
          z1[i] = cs * q1 + sn * q2;
          z2[i] = -sn * q1 + cs * q2;
        }
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
  std::vector<double> d(n), e(n, 0.0);
  for (int i = 0; i < n; ++i) d[i] = T[(size_t)i * n + i];
  for (int i = 0; i + 1 < n; ++i) e[i] = T[(size_t)(i + 1) * n + i];
  const int st = tridiagonal_qr(n, d.data(), e.data(), Zt.data());
  if (st != 0) return st;
  std::vector<int> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return d[a] > d[b]; });
  for (int j = 0; j < n; ++j) {
    w[j] = d[ord[j]];
    for (int i = 0; i < n; ++i) V[(size_t)i * n + j] = Zt[(size_t)ord[j] * n + i];
  }
  return 0;
}

// Solve (T - sigma I) x = b in place for the tridiagonal T (diagonal d,
// off-diagonal e), by Gaussian elimination with partial pivoting (the
// factor gains a second superdiagonal); a pivot of zero is replaced by tiny.
static void tri_shifted_solve(int n, const double* d, const double* e, double sigma, double tiny, double* x) {
  std::vector<double> u0(n), u1(n, 0.0), u2(n, 0.0), l(n, 0.0);
  std::vector<char> sw(n, 0);
  u0[0] = d[0] - sigma;
  if (n > 1) u1[0] = e[0];
  for (int i = 0; i + 1 < n; ++i) {
    const double c = e[i], an = d[i + 1] - sigma, bn = (i + 2 < n) ? e[i + 1] : 0.0;
    if (std::fabs(u0[i]) >= std::fabs(c)) {
      if (u0[i] == 0.0) u0[i] = tiny;
      const double m = c / u0[i];
      l[i] = m;
      u0[i + 1] = an - m * u1[i];
      u1[i + 1] = bn - m * u2[i];
    } else {
      const double m = u0[i] / c;
      l[i] = m;
      sw[i] = 1;
      const double r1 = u1[i], r2 = u2[i];
      u0[i] = c;
      u1[i] = an;
      u2[i] = bn;
      u0[i + 1] = r1 - m * an;
      u1[i + 1] = r2 - m * bn;
    }
  }
  if (u0[n - 1] == 0.0) u0[n - 1] = tiny;
  for (int i = 0; i + 1 < n; ++i) {
    if (sw[i]) std::swap(x[i], x[i + 1]);
    x[i + 1] -= l[i] * x[i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double t = x[i];
    if (i + 1 < n) t -= u1[i] * x[i + 1];
    if (i + 2 < n) t -= u2[i] * x[i + 2];
    x[i] = t / u0[i];
  }
}

int sym_eig_top(int n, const double* A, int k, double* w, double* V) {
  if (k < 1 || k > n) return CVAMX_E_INVALID_ARG;
  if (n <= 2 || 4 * k > n) {
    // small or most of the spectrum: the full decomposition
    std::vector<double> wf(n), Vf((size_t)n * n);
    const int st = sym_eig_desc(n, A, wf.data(), Vf.data());
    if (st != 0) return st;
    for (int i = 0; i < n; ++i) {
      w[i] = wf[i];
      for (int j = 0; j < k; ++j) V[(size_t)i * k + j] = Vf[(size_t)i * n + j];
    }
    return 0;
  }
  std::vector<double> T((size_t)n * n), Vh((size_t)n * n, 0.0), bk(n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) {
      T[(size_t)i * n + j] = A[(size_t)i * n + j];
      T[(size_t)j * n + i] = A[(size_t)i * n + j];
    }
  tridiagonalize(n, T.data(), nullptr, Vh.data(), bk.data());
  std::vector<double> d(n), e(n, 0.0);
  for (int i = 0; i < n; ++i) d[i] = T[(size_t)i * n + i];
  for (int i = 0; i + 1 < n; ++i) e[i] = T[(size_t)(i + 1) * n + i];
  double tnorm = 0.0;   // 1-norm of the tridiagonal
  for (int i = 0; i < n; ++i)
    tnorm = std::max(tnorm, std::fabs(d[i]) + (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(e[i]) : 0.0));
  std::vector<double> dq(d), eq(e);
  const int st = tridiagonal_qr(n, dq.data(), eq.data(), nullptr);
  if (st != 0) return st;
  std::copy(dq.begin(), dq.end(), w);
  std::sort(w, w + n, [](double a, double b) { return a > b; });
  if (tnorm == 0.0) {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < k; ++j) V[(size_t)i * k + j] = i == j ? 1.0 : 0.0;
    return 0;
  }
  // eigenvectors of the tridiagonal by inverse iteration: vectors whose
  // eigenvalues lie within 1e-3 |T| of each other form a cluster and are
  // kept orthogonal to one another (modified Gram-Schmidt in every step),
  // and their shifts are kept at least 10 eps |T| apart
  const double ortol = 1e-3 * tnorm, pertol = 10.0 * DBL_EPSILON * tnorm, tiny = DBL_EPSILON * tnorm;
  std::vector<double> X((size_t)k * n), x(n);
  int c0 = 0;
  double prev = 0.0;
  for (int j = 0; j < k; ++j) {
    double sigma = w[j];
    if (j > 0 && w[j - 1] - w[j] > ortol) c0 = j;
    if (j > c0 && sigma > prev - pertol) sigma = prev - pertol;
    prev = sigma;
    for (int i = 0; i < n; ++i) x[i] = 1.0 + 0.25 * (double)((7 * i + 3 * j) % 11) / 11.0;
    for (int it = 0; it < 5; ++it) {
      tri_shifted_solve(n, d.data(), e.data(), sigma, tiny, x.data());
      for (int c = c0; c < j; ++c) {
        const double* xc = X.data() + (size_t)c * n;
        double dot = 0.0;
        for (int i = 0; i < n; ++i) dot += xc[i] * x[i];
        for (int i = 0; i < n; ++i) x[i] -= dot * xc[i];
      }
      double nrm = 0.0;
      for (int i = 0; i < n; ++i) nrm += x[i] * x[i];
      nrm = std::sqrt(nrm);
      if (!(nrm > 0.0) || !std::isfinite(nrm)) return CVAMX_E_NUMERIC;
      for (int i = 0; i < n; ++i) x[i] /= nrm;
    }
    std::copy(x.begin(), x.end(), X.begin() + (size_t)j * n);
  }
  // back to the input's basis: y = H_0 H_1 ... H_{n-3} x
  for (int j = 0; j < k; ++j) {
    double* y = X.data() + (size_t)j * n;
    for (int r = n - 3; r >= 0; --r) {
      if (bk[r] == 0.0) continue;
      const double* v = Vh.data() + (size_t)r * n;
      double dot = 0.0;
      for (int i = r + 1; i < n; ++i) dot += v[i] * y[i];
      dot *= bk[r];
      for (int i = r + 1; i < n; ++i) y[i] -= dot * v[i];
    }
    for (int i = 0; i < n; ++i) V[(size_t)i * k + j] = y[i];
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

CVX_HOST_SIMD int cva_solve(int K, int B, const double* cnt, const double* cm, const double* Sw,
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
  // E = L^-1 D, D[:, k] = sqrt(n_k) (m_k - m): forward substitution by
  // rows, all K columns at once
  std::vector<double> E((size_t)B * K), sq(K);
  for (int k = 0; k < K; ++k) sq[k] = std::sqrt(cnt[k]);
  for (int i = 0; i < B; ++i) {
    double* __restrict__ ei = E.data() + (size_t)i * K;
    for (int k = 0; k < K; ++k) ei[k] = sq[k] * (cm[(size_t)k * B + i] - m[i]);
    for (int j = 0; j < i; ++j) {
      const double lij = L[(size_t)i * B + j];
      const double* __restrict__ ej = E.data() + (size_t)j * K;
      for (int k = 0; k < K; ++k) ei[k] -= lij * ej[k];
    }
    const double inv = 1.0 / L[(size_t)i * B + i];
    for (int k = 0; k < K; ++k) ei[k] *= inv;
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
  // W = L^-T U: back substitution by rows, all nc columns at once
  std::vector<double> Wt((size_t)B * nc);
  for (int i = B - 1; i >= 0; --i) {
    double* __restrict__ wi = Wt.data() + (size_t)i * nc;
    for (int j = 0; j < nc; ++j) wi[j] = U[(size_t)i * nc + j];
    for (int r = i + 1; r < B; ++r) {
      const double lri = L[(size_t)r * B + i];
      const double* __restrict__ wr = Wt.data() + (size_t)r * nc;
      for (int j = 0; j < nc; ++j) wi[j] -= lri * wr[j];
    }
    const double inv = 1.0 / L[(size_t)i * B + i];
    for (int j = 0; j < nc; ++j) wi[j] *= inv;
  }
  sign_rule(B, nc, Wt.data());
  std::copy(Wt.begin(), Wt.end(), W);
  std::copy(lam.begin(), lam.end(), eig);
  if (mean) std::copy(m.begin(), m.end(), mean);
  if (Sb_out) {
    // S_b = sum_k n_k (m_k - m)(m_k - m)^T, one rank-one update per class
    std::fill(Sb_out, Sb_out + (size_t)B * B, 0.0);
    std::vector<double> dk(B);
    for (int k = 0; k < K; ++k) {
      for (int i = 0; i < B; ++i) dk[i] = cm[(size_t)k * B + i] - m[i];
      for (int i = 0; i < B; ++i) {
        const double a = cnt[k] * dk[i];
        double* __restrict__ row = Sb_out + (size_t)i * B;
        for (int j = 0; j < B; ++j) row[j] += a * dk[j];
      }
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

extern "C" int cvamx_sym_eig_top(int32_t n, const double* A, int32_t k, double* w, double* V) {
  if (!A || !w || !V || n < 1 || n > 4096 || k < 1 || k > n) return CVAMX_E_INVALID_ARG;
  const int st = cvamx::sym_eig_top(n, A, k, w, V);
  if (st != 0) return st;
  cvamx::sign_rule(n, k, V);
  return 0;
}

extern "C" int cvamx_sym_eig(int32_t n, const double* A, double* w, double* V) {
  if (!A || !w || !V || n < 1 || n > 4096) return CVAMX_E_INVALID_ARG;
  const int st = cvamx::sym_eig_desc(n, A, w, V);
  if (st != 0) return st;
  cvamx::sign_rule(n, n, V);
  return 0;
}
