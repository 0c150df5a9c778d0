// Small dense linear algebra for the GCRO-DR cycle problems (host, float64).
#include "host_la.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <numeric>
#include <type_traits>

namespace gir {
namespace la {

using cd = std::complex<double>;

double givens_lsq(const double* H, int ldh, int j, double beta, double* y) {
  if (j <= 0) return std::fabs(beta);
  std::vector<double> R((size_t)(j + 1) * j, 0.0);
  std::vector<double> cs(j), sn(j), g(j + 1, 0.0);
  g[0] = beta;
  for (int c = 0; c < j; ++c) {
    std::vector<double> h(j + 2, 0.0);
    for (int i = 0; i <= c + 1; ++i) h[i] = H[(size_t)c * ldh + i];
    for (int i = 0; i < c; ++i) {
      const double t = cs[i] * h[i] + sn[i] * h[i + 1];
      h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
      h[i] = t;
    }
    const double a = h[c], b = h[c + 1];
    const double r = std::hypot(a, b);
    double cc = 1.0, ss = 0.0;
    if (r != 0.0) {
      cc = a / r;
      ss = b / r;
    }
    cs[c] = cc;
    sn[c] = ss;
    h[c] = cc * a + ss * b;
    g[c + 1] = -ss * g[c];
    g[c] = cc * g[c];
    for (int i = 0; i <= c; ++i) R[(size_t)c * (j + 1) + i] = h[i];
  }
  for (int i = j - 1; i >= 0; --i) {
    double s = g[i];
    for (int t = i + 1; t < j; ++t) s -= R[(size_t)t * (j + 1) + i] * y[t];
    const double d = R[(size_t)i * (j + 1) + i];
    y[i] = (d != 0.0) ? s / d : 0.0;
  }
  return std::fabs(g[j]);
}

bool qr_thin(const double* A, int lda, int m, int k, double* Q, double* R) {
  std::vector<double> W((size_t)m * k);
  for (int c = 0; c < k; ++c)
    for (int i = 0; i < m; ++i) W[(size_t)c * m + i] = A[(size_t)c * lda + i];
  std::vector<double> vs((size_t)m * k, 0.0), betas(k, 0.0);
  bool ok = true;
  for (int c = 0; c < k; ++c) {
    double* x = &W[(size_t)c * m];
    double nrm = 0.0;
    for (int i = c; i < m; ++i) nrm += x[i] * x[i];
    nrm = std::sqrt(nrm);
    double* v = &vs[(size_t)c * m];
    if (nrm == 0.0) {
      ok = false;
      betas[c] = 0.0;
      continue;
    }
    const double alpha = (x[c] >= 0.0) ? -nrm : nrm;
    for (int i = c; i < m; ++i) v[i] = x[i];
    v[c] -= alpha;
    double vn = 0.0;
    for (int i = c; i < m; ++i) vn += v[i] * v[i];
    betas[c] = (vn > 0.0) ? 2.0 / vn : 0.0;
    for (int cc = c; cc < k; ++cc) {
      double* y = &W[(size_t)cc * m];
      double d = 0.0;
      for (int i = c; i < m; ++i) d += v[i] * y[i];
      d *= betas[c];
      for (int i = c; i < m; ++i) y[i] -= d * v[i];
    }
  }
  // R and the thin Q = H_0 ... H_{k-1} [I; 0]
  for (int c = 0; c < k; ++c)
    for (int i = 0; i < k; ++i) R[(size_t)c * k + i] = (i <= c) ? W[(size_t)c * m + i] : 0.0;
  for (int c = 0; c < k; ++c)
    for (int i = 0; i < m; ++i) Q[(size_t)c * m + i] = (i == c) ? 1.0 : 0.0;
  for (int h = k - 1; h >= 0; --h) {
    const double* v = &vs[(size_t)h * m];
    for (int c = 0; c < k; ++c) {
      double* q = &Q[(size_t)c * m];
      double d = 0.0;
      for (int i = h; i < m; ++i) d += v[i] * q[i];
      d *= betas[h];
      for (int i = h; i < m; ++i) q[i] -= d * v[i];
    }
  }
  // non-negative diagonal of R
  for (int i = 0; i < k; ++i) {
    if (R[(size_t)i * k + i] < 0.0) {
      for (int c = i; c < k; ++c) R[(size_t)c * k + i] = -R[(size_t)c * k + i];
      for (int r = 0; r < m; ++r) Q[(size_t)i * m + r] = -Q[(size_t)i * m + r];
    }
    if (R[(size_t)i * k + i] == 0.0) ok = false;
  }
  return ok;
}

bool cholesky_upper(const double* G, int k, double* R) {
  std::fill(R, R + (size_t)k * k, 0.0);
  for (int j = 0; j < k; ++j) {
    double s = G[(size_t)j * k + j];
    for (int t = 0; t < j; ++t) s -= R[(size_t)j * k + t] * R[(size_t)j * k + t];
    if (!(s > 0.0)) return false;
    const double d = std::sqrt(s);
    R[(size_t)j * k + j] = d;
    for (int c = j + 1; c < k; ++c) {
      double v = G[(size_t)c * k + j];
      for (int t = 0; t < j; ++t) v -= R[(size_t)j * k + t] * R[(size_t)c * k + t];
      R[(size_t)c * k + j] = v / d;
    }
  }
  return true;
}

void inv_upper(const double* R, int k, double* Rinv) {
  std::vector<double> X((size_t)k * k, 0.0);
  for (int c = 0; c < k; ++c) {
    // solve R x = e_c
    for (int i = k - 1; i >= 0; --i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int t = i + 1; t < k; ++t) s -= R[(size_t)t * k + i] * X[(size_t)c * k + t];
      X[(size_t)c * k + i] = s / R[(size_t)i * k + i];
    }
  }
  std::memcpy(Rinv, X.data(), sizeof(double) * (size_t)k * k);
}

// ---------------------------------------------------------------------------
// eigenproblem: complex Hessenberg reduction, single-shift QR, back substitution
// ---------------------------------------------------------------------------
namespace {

inline void givens_c(cd x, cd y, double& c, cd& s) {
  const double ax = std::abs(x), ay = std::abs(y);
  if (ay == 0.0) {
    c = 1.0;
    s = 0.0;
    return;
  }
  if (ax == 0.0) {
    c = 0.0;
    s = std::conj(y) / ay;
    return;
  }
  const double r = std::hypot(ax, ay);
  c = ax / r;
  s = (x / ax) * std::conj(y) / r;
}

}  // namespace

namespace {

// Real Schur form T = Z^T A Z of a real matrix (T quasi upper triangular:
// 1 x 1 blocks for the real eigenvalues, 2 x 2 blocks for the complex
// conjugate pairs): Householder reduction to upper Hessenberg form, then
// Francis double-shift QR sweeps (3-element reflectors chasing the bulge,
// a 2-element reflector at the end of the window; an ad hoc shift on the
// 10th and 20th iteration without deflation), every 2 x 2 block with real
// eigenvalues split into two 1 x 1 blocks.  Z is not accumulated: its
// factors (the reflectors, in the order applied) are kept, and vector(e)
// forms only the eigenvectors asked for: back substitution on T (2 x 2
// blocks solved directly), then Z applied factor by factor.
struct SchurR {
  struct Refl {
    int k;       // first row / column
    int len;     // 2 or 3
    double v[3];
    double beta;  // P = I - beta v v^T (0: identity)
  };
  int N = 0;
  std::vector<double> T;   // column-major
  std::vector<double> hv;  // Hessenberg reflector c: hv[c * N + i] for i > c
  std::vector<double> hb;
  std::vector<Refl> refl;
  std::vector<cd> w;       // eigenvalues, in the order of T's diagonal
  double small = 0.0;

  double& t(int i, int j) { return T[(size_t)j * N + i]; }
  double t(int i, int j) const { return T[(size_t)j * N + i]; }

  // P u = alpha e_1 for u of length len (beta = 0 when u = 0)
  static Refl house(int k, int len, const double* u) {
    Refl r{k, len, {0.0, 0.0, 0.0}, 0.0};
    double nrm = 0.0;
    for (int i = 0; i < len; ++i) nrm += u[i] * u[i];
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) return r;
    const double alpha = (u[0] >= 0.0) ? -nrm : nrm;
    for (int i = 0; i < len; ++i) r.v[i] = u[i];
    r.v[0] -= alpha;
    double vn = 0.0;
    for (int i = 0; i < len; ++i) vn += r.v[i] * r.v[i];
    r.beta = (vn > 0.0) ? 2.0 / vn : 0.0;
    return r;
  }

  // T <- P T P on rows k .. k+len-1 (columns c0 .. N-1) and columns
  // k .. k+len-1 (rows 0 .. r1); the transformation is recorded.  The length
  // is a template argument so that the short loops unroll (the same
  // operations in the same order).
  template <int L>
  void apply_len(const Refl& p, int c0, int r1) {
    double* tk = T.data() + p.k;  // row k of column 0
    for (int j = c0; j < N; ++j) {
      double* col = tk + (size_t)j * N;
      double d = 0.0;
      for (int i = 0; i < L; ++i) d += p.v[i] * col[i];
      d *= p.beta;
      for (int i = 0; i < L; ++i) col[i] -= d * p.v[i];
    }
    double* ck = T.data() + (size_t)p.k * N;  // column k
    for (int i = 0; i <= r1; ++i) {
      double d = 0.0;
      for (int q = 0; q < L; ++q) d += ck[(size_t)q * N + i] * p.v[q];
      d *= p.beta;
      for (int q = 0; q < L; ++q) ck[(size_t)q * N + i] -= d * p.v[q];
    }
  }
  void apply(const Refl& p, int c0, int r1) {
    if (p.beta == 0.0) return;
    if (p.len == 3)
      apply_len<3>(p, c0, r1);
    else
      apply_len<2>(p, c0, r1);
    refl.push_back(p);
  }

  bool factor(const double* A, int n) {
    N = n;
    T.assign(A, A + (size_t)N * N);
    hv.assign((size_t)N * N, 0.0);
    hb.assign(N, 0.0);
    refl.clear();
    refl.reserve((size_t)N * 48);
    w.assign(N, cd(0.0));
    // Householder reduction to upper Hessenberg form
    for (int c = 0; c + 2 < N; ++c) {
      double nrm = 0.0;
      for (int i = c + 1; i < N; ++i) nrm += t(i, c) * t(i, c);
      nrm = std::sqrt(nrm);
      if (nrm == 0.0) continue;
      const double x0 = t(c + 1, c);
      const double alpha = (x0 >= 0.0) ? -nrm : nrm;
      double* v = &hv[(size_t)c * N];
      for (int i = c + 1; i < N; ++i) v[i] = t(i, c);
      v[c + 1] -= alpha;
      double vn = 0.0;
      for (int i = c + 1; i < N; ++i) vn += v[i] * v[i];
      if (vn == 0.0) continue;
      const double beta = 2.0 / vn;
      hb[c] = beta;
      for (int j = 0; j < N; ++j) {
        double d = 0.0;
        for (int i = c + 1; i < N; ++i) d += v[i] * t(i, j);
        d *= beta;
        for (int i = c + 1; i < N; ++i) t(i, j) -= d * v[i];
      }
      for (int i = 0; i < N; ++i) {
        double d = 0.0;
        for (int j = c + 1; j < N; ++j) d += t(i, j) * v[j];
        d *= beta;
        for (int j = c + 1; j < N; ++j) t(i, j) -= d * v[j];
      }
      for (int i = c + 2; i < N; ++i) t(i, c) = 0.0;
    }
    double tn = 0.0;
    for (int j = 0; j < N; ++j)
      for (int i = 0; i < N; ++i) tn = std::max(tn, std::fabs(t(i, j)));
    const double eps = std::numeric_limits<double>::epsilon();
    small = std::max(tn, 1e-300) * eps;
    int hi = N - 1;
    int iter = 0, total = 0;
    while (hi >= 0) {
      // deflation: the active window is l .. hi
      int l = hi;
      while (l > 0) {
        const double sub = std::fabs(t(l, l - 1));
        double dsum = std::fabs(t(l - 1, l - 1)) + std::fabs(t(l, l));
        if (dsum == 0.0) dsum = tn;
        if (sub <= eps * dsum) {
          t(l, l - 1) = 0.0;
          break;
        }
        --l;
      }
      if (l == hi) {
        w[hi] = t(hi, hi);
        --hi;
        iter = 0;
        continue;
      }
      if (l == hi - 1) {
        // a 2 x 2 block: a complex pair stays, real eigenvalues are split
        const double a = t(hi - 1, hi - 1), b = t(hi - 1, hi), c = t(hi, hi - 1),
                     d = t(hi, hi);
        const double p = 0.5 * (a - d);
        const double disc = p * p + b * c;
        if (disc >= 0.0) {
          const double sq = std::sqrt(disc);
          const double l1 = 0.5 * (a + d) + (p >= 0.0 ? sq : -sq);
          // an eigenvector of the block for l1, the larger of two forms
          double u[2] = {b, l1 - a};
          const double u2[2] = {l1 - d, c};
          if (std::hypot(u2[0], u2[1]) > std::hypot(u[0], u[1])) {
            u[0] = u2[0];
            u[1] = u2[1];
          }
          apply(house(hi - 1, 2, u), hi - 1, hi);
          t(hi, hi - 1) = 0.0;
          w[hi - 1] = t(hi - 1, hi - 1);
          w[hi] = t(hi, hi);
        } else {
          const double re = 0.5 * (a + d), im = std::sqrt(-disc);
          w[hi - 1] = cd(re, im);
          w[hi] = cd(re, -im);
        }
        hi -= 2;
        iter = 0;
        continue;
      }
      if (++total > 100 * N) return false;
      ++iter;
      double s, q;
      if (iter == 10 || iter == 20) {
        const double ex = std::fabs(t(hi, hi - 1)) + std::fabs(t(hi - 1, hi - 2));
        s = 1.5 * ex;
        q = ex * ex;
      } else {
        s = t(hi - 1, hi - 1) + t(hi, hi);
        q = t(hi - 1, hi - 1) * t(hi, hi) - t(hi - 1, hi) * t(hi, hi - 1);
      }
      // the first column of (T - r1)(T - r2) on the window
      double x = t(l, l) * t(l, l) + t(l, l + 1) * t(l + 1, l) - s * t(l, l) + q;
      double y = t(l + 1, l) * (t(l, l) + t(l + 1, l + 1) - s);
      double z = t(l + 1, l) * t(l + 2, l + 1);
      for (int k = l; k <= hi - 2; ++k) {
        const double u[3] = {x, y, z};
        apply(house(k, 3, u), std::max(l, k - 1), std::min(k + 3, hi));
        if (k > l) {
          t(k + 1, k - 1) = 0.0;
          t(k + 2, k - 1) = 0.0;
        }
        x = t(k + 1, k);
        y = t(k + 2, k);
        if (k < hi - 2) z = t(k + 3, k);
      }
      const double u[2] = {x, y};
      apply(house(hi - 1, 2, u), hi - 2, hi);
      t(hi, hi - 2) = 0.0;
    }
    return true;
  }

  cd value(int e) const { return w[e]; }

  // the unit eigenvector of eigenvalue e
  void vector(int e, cd* out) const {
    std::vector<cd> x(N, cd(0.0));
    const cd lam = w[e];
    int top;  // the last row already set
    if (e > 0 && t(e, e - 1) != 0.0) {
      // second row of a complex 2 x 2 block
      top = e - 1;
    } else if (e + 1 < N && t(e + 1, e) != 0.0) {
      top = e;
    } else {
      top = -1;
    }
    int r;
    if (top >= 0) {
      // the block's own eigenvector, the larger of two forms
      const double a = t(top, top), b = t(top, top + 1), c = t(top + 1, top),
                   d = t(top + 1, top + 1);
      cd u0 = b, u1 = lam - a;
      const cd v0 = lam - d, v1 = c;
      if (std::norm(v0) + std::norm(v1) > std::norm(u0) + std::norm(u1)) {
        u0 = v0;
        u1 = v1;
      }
      x[top] = u0;
      x[top + 1] = u1;
      r = top - 1;
    } else {
      x[e] = 1.0;
      r = e - 1;
    }
    const int last = (top >= 0) ? top + 1 : e;
    while (r >= 0) {
      if (r > 0 && t(r, r - 1) != 0.0) {
        // rows r-1, r form a 2 x 2 block: solve it for both
        cd s1 = 0.0, s2 = 0.0;
        for (int q = r + 1; q <= last; ++q) {
          s1 += t(r - 1, q) * x[q];
          s2 += t(r, q) * x[q];
        }
        const cd m11 = t(r - 1, r - 1) - lam, m12 = t(r - 1, r), m21 = t(r, r - 1),
                 m22 = t(r, r) - lam;
        cd det = m11 * m22 - m12 * m21;
        if (std::abs(det) < small * small) det = small * small;
        x[r - 1] = (-s1 * m22 + m12 * s2) / det;
        x[r] = (-m11 * s2 + m21 * s1) / det;
        r -= 2;
      } else {
        cd s = 0.0;
        for (int q = r + 1; q <= last; ++q) s += t(r, q) * x[q];
        cd den = t(r, r) - lam;
        if (std::abs(den) < small) den = small;
        x[r] = -s / den;
        r -= 1;
      }
    }
    // Z = H_0 .. H_{N-3} P_1 .. P_R: the sweep reflectors last to first,
    // then the Hessenberg reflectors last to first
    auto replay = [&](const Refl& p, auto len) {
      constexpr int L = decltype(len)::value;
      cd* xk = x.data() + p.k;
      cd d = 0.0;
      for (int i = 0; i < L; ++i) d += p.v[i] * xk[i];
      d *= p.beta;
      for (int i = 0; i < L; ++i) xk[i] -= d * p.v[i];
    };
    for (size_t q = refl.size(); q-- > 0;) {
      const Refl& p = refl[q];
      if (p.beta == 0.0) continue;
      if (p.len == 3)
        replay(p, std::integral_constant<int, 3>{});
      else
        replay(p, std::integral_constant<int, 2>{});
    }
    for (int c = N - 3; c >= 0; --c) {
      if (hb[c] == 0.0) continue;
      const double* v = &hv[(size_t)c * N];
      cd d = 0.0;
      for (int i = c + 1; i < N; ++i) d += v[i] * x[i];
      d *= hb[c];
      for (int i = c + 1; i < N; ++i) x[i] -= d * v[i];
    }
    double nrm = 0.0;
    for (int i = 0; i < N; ++i) nrm += std::norm(x[i]);
    nrm = std::sqrt(nrm);
    for (int i = 0; i < N; ++i) out[i] = (nrm > 0.0) ? x[i] / nrm : x[i];
  }
};

}  // namespace

bool eig_real(const double* A, int N, std::vector<cd>& w, std::vector<cd>& V) {
  w.assign(N, cd(0.0));
  V.assign((size_t)N * N, cd(0.0));
  if (N == 0) return true;
  SchurR sc;
  if (!sc.factor(A, N)) return false;
  for (int e = 0; e < N; ++e) {
    w[e] = sc.value(e);
    sc.vector(e, &V[(size_t)e * N]);
  }
  return true;
}

int harmonic_ritz(const double* G, const double* M, int rows, int cols, int k, double* P) {
  if (cols <= 0 || k <= 0) return 0;
  std::vector<double> Q((size_t)rows * cols), R((size_t)cols * cols);
  if (!qr_thin(G, rows, rows, cols, Q.data(), R.data())) return 0;
  // N = G^T M (cols x cols)
  std::vector<double> Nm((size_t)cols * cols, 0.0);
  for (int j = 0; j < cols; ++j)
    for (int i = 0; i < cols; ++i) {
      double s = 0.0;
      for (int r = 0; r < rows; ++r) s += G[(size_t)i * rows + r] * M[(size_t)j * rows + r];
      Nm[(size_t)j * cols + i] = s;
    }
  // X = N R^-1 : solve X R = N column by column (forward in columns)
  std::vector<double> X((size_t)cols * cols, 0.0);
  for (int j = 0; j < cols; ++j) {
    for (int i = 0; i < cols; ++i) {
      double s = Nm[(size_t)j * cols + i];
      for (int t = 0; t < j; ++t) s -= X[(size_t)t * cols + i] * R[(size_t)j * cols + t];
      X[(size_t)j * cols + i] = s / R[(size_t)j * cols + j];
    }
  }
  // T = R^-T X : solve R^T T = X (forward substitution on rows)
  std::vector<double> Tm((size_t)cols * cols, 0.0);
  for (int j = 0; j < cols; ++j) {
    for (int i = 0; i < cols; ++i) {
      double s = X[(size_t)j * cols + i];
      for (int t = 0; t < i; ++t) s -= R[(size_t)i * cols + t] * Tm[(size_t)j * cols + t];
      Tm[(size_t)j * cols + i] = s / R[(size_t)i * cols + i];
    }
  }
  SchurR sc;
  if (!sc.factor(Tm.data(), cols)) return 0;
  std::vector<cd> mu(cols), wv(cols);
  for (int e = 0; e < cols; ++e) mu[e] = sc.value(e);
  // order: largest |mu| first (smallest |theta|), stable in index
  std::vector<int> ord(cols);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(),
                   [&](int a, int b) { return std::abs(mu[a]) > std::abs(mu[b]); });
  std::vector<bool> used(cols, false);
  int kout = 0;
  auto back = [&](const cd* wv, std::vector<cd>& z) {
    // z = R^-1 w
    z.assign(cols, cd(0.0));
    for (int i = cols - 1; i >= 0; --i) {
      cd s = wv[i];
      for (int t = i + 1; t < cols; ++t) s -= R[(size_t)t * cols + i] * z[t];
      z[i] = s / R[(size_t)i * cols + i];
    }
  };
  std::vector<cd> z;
  for (int oi = 0; oi < cols && kout < k; ++oi) {
    const int idx = ord[oi];
    if (used[idx]) continue;
    const cd m = mu[idx];
    const double am = std::abs(m);
    const bool is_complex = std::abs(m.imag()) > 1e3 * 2.220446049250313e-16 * am && am > 0.0;
    used[idx] = true;
    sc.vector(idx, wv.data());
    back(wv.data(), z);
    if (is_complex) {
      if (kout + 2 > k) break;
      int partner = -1;
      double best = 0.0;
      for (int t = 0; t < cols; ++t) {
        if (used[t]) continue;
        const double dd = std::abs(mu[t] - std::conj(m));
        if (partner < 0 || dd < best) {
          partner = t;
          best = dd;
        }
      }
      if (partner >= 0) used[partner] = true;
      for (int i = 0; i < cols; ++i) P[(size_t)kout * cols + i] = z[i].real();
      for (int i = 0; i < cols; ++i) P[(size_t)(kout + 1) * cols + i] = z[i].imag();
      kout += 2;
    } else {
      // rotate the phase so that the largest component is real
      int imax = 0;
      for (int i = 1; i < cols; ++i)
        if (std::abs(z[i]) > std::abs(z[imax])) imax = i;
      const cd ph = (std::abs(z[imax]) > 0.0) ? std::conj(z[imax]) / std::abs(z[imax]) : cd(1.0);
      for (int i = 0; i < cols; ++i) P[(size_t)kout * cols + i] = (z[i] * ph).real();
      kout += 1;
    }
  }
  return kout;
}

}  // namespace la
}  // namespace gir
