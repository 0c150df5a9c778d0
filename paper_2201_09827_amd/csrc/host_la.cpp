// Small dense linear algebra for the GCRO-DR cycle problems (host, float64).
#include "host_la.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <numeric>

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

// Complex Schur form T = Z^H A Z of a real matrix: Householder reduction to
// upper Hessenberg form (real arithmetic), then single-shift QR with
// Wilkinson shifts (an
// exceptional shift every 11th iteration).  Z is not accumulated: its
// factors (the reflectors and every sweep's rotations) are kept, and
// vector(e) forms only the eigenvectors asked for (back substitution on T,
// then Z applied factor by factor), which costs far less than carrying Z
// through every sweep when a few vectors are wanted.
struct SchurC {
  struct Rot {
    int k;
    double c;
    cd s;
  };
  int N = 0;
  std::vector<cd> T;          // column-major
  std::vector<double> hv;     // reflector c: hv[c * N + i] for i > c (real: A is real)
  std::vector<double> hb;     // its beta (0: no reflection)
  std::vector<Rot> rots;      // in the order they were applied
  double small = 0.0;

  cd& t(int i, int j) { return T[(size_t)j * N + i]; }
  const cd& t(int i, int j) const { return T[(size_t)j * N + i]; }

  bool factor(const double* A, int n) {
    N = n;
    // Householder reduction to upper Hessenberg form in real arithmetic
    std::vector<double> H(A, A + (size_t)N * N);
    auto h = [&](int i, int j) -> double& { return H[(size_t)j * N + i]; };
    hv.assign((size_t)N * N, 0.0);
    hb.assign(N, 0.0);
    rots.clear();
    for (int c = 0; c + 2 < N; ++c) {
      double nrm = 0.0;
      for (int i = c + 1; i < N; ++i) nrm += h(i, c) * h(i, c);
      nrm = std::sqrt(nrm);
      if (nrm == 0.0) continue;
      const double x0 = h(c + 1, c);
      const double alpha = (x0 >= 0.0) ? -nrm : nrm;
      double* v = &hv[(size_t)c * N];
      for (int i = c + 1; i < N; ++i) v[i] = h(i, c);
      v[c + 1] -= alpha;
      double vn = 0.0;
      for (int i = c + 1; i < N; ++i) vn += v[i] * v[i];
      if (vn == 0.0) continue;
      const double beta = 2.0 / vn;
      hb[c] = beta;
      // H = (I - beta v v^T) H (I - beta v v^T)
      for (int j = 0; j < N; ++j) {
        double d = 0.0;
        for (int i = c + 1; i < N; ++i) d += v[i] * h(i, j);
        d *= beta;
        for (int i = c + 1; i < N; ++i) h(i, j) -= d * v[i];
      }
      for (int i = 0; i < N; ++i) {
        double d = 0.0;
        for (int j = c + 1; j < N; ++j) d += h(i, j) * v[j];
        d *= beta;
        for (int j = c + 1; j < N; ++j) h(i, j) -= d * v[j];
      }
      for (int i = c + 2; i < N; ++i) h(i, c) = 0.0;
    }
    T.assign((size_t)N * N, cd(0.0));
    for (size_t i = 0; i < (size_t)N * N; ++i) T[i] = H[i];
    const double eps = std::numeric_limits<double>::epsilon();
    int hi = N - 1;
    int iter = 0, total = 0;
    while (hi > 0) {
      int l = hi;
      while (l > 0) {
        const double sub = std::abs(t(l, l - 1));
        const double dsum = std::abs(t(l - 1, l - 1)) + std::abs(t(l, l));
        if (sub <= eps * (dsum > 0.0 ? dsum : 1.0)) {
          t(l, l - 1) = 0.0;
          break;
        }
        --l;
      }
      if (l == hi) {
        --hi;
        iter = 0;
        continue;
      }
      if (++total > 100 * N) return false;
      ++iter;
      const cd a = t(hi - 1, hi - 1), b = t(hi - 1, hi), c = t(hi, hi - 1), d = t(hi, hi);
      cd mu;
      if (iter % 11 == 10) {
        mu = d + std::abs(t(hi, hi - 1));  // exceptional shift
      } else {
        const cd tr = a + d;
        const cd det = a * d - b * c;
        const cd disc = std::sqrt(tr * tr * 0.25 - det);
        const cd m1 = tr * 0.5 + disc, m2 = tr * 0.5 - disc;
        mu = (std::abs(m1 - d) < std::abs(m2 - d)) ? m1 : m2;
      }
      cd x = t(l, l) - mu;
      cd y = t(l + 1, l);
      for (int k = l; k < hi; ++k) {
        double cc;
        cd s;
        givens_c(x, y, cc, s);
        // rows k, k+1, then columns k, k+1
        for (int j = std::max(l, k - 1); j < N; ++j) {
          const cd t1 = t(k, j), t2 = t(k + 1, j);
          t(k, j) = cc * t1 + s * t2;
          t(k + 1, j) = -std::conj(s) * t1 + cc * t2;
        }
        const int rmax = std::min(k + 2, hi);
        for (int i = 0; i <= rmax; ++i) {
          const cd t1 = t(i, k), t2 = t(i, k + 1);
          t(i, k) = cc * t1 + std::conj(s) * t2;
          t(i, k + 1) = -s * t1 + cc * t2;
        }
        rots.push_back({k, cc, s});
        if (k + 1 < hi) {
          x = t(k + 1, k);
          y = t(k + 2, k);
        }
      }
    }
    double tn = 0.0;
    for (int j = 0; j < N; ++j)
      for (int i = 0; i <= j; ++i) tn = std::max(tn, std::abs(t(i, j)));
    small = std::max(tn, 1e-300) * eps;
    return true;
  }

  cd value(int e) const { return t(e, e); }

  // the unit eigenvector of eigenvalue e: T x = lambda x by back
  // substitution (x_e = 1), then Z x
  void vector(int e, cd* out) const {
    std::vector<cd> x(N, cd(0.0));
    x[e] = 1.0;
    const cd lam = t(e, e);
    for (int r = e - 1; r >= 0; --r) {
      cd s = 0.0;
      for (int q = r + 1; q <= e; ++q) s += t(r, q) * x[q];
      cd den = t(r, r) - lam;
      if (std::abs(den) < small) den = small;
      x[r] = -s / den;
    }
    // Z = P_0 .. P_{N-3} G_1 .. G_R: the rotations last to first, then the
    // reflectors last to first
    for (size_t q = rots.size(); q-- > 0;) {
      const Rot& g = rots[q];
      const cd x1 = x[g.k], x2 = x[g.k + 1];
      x[g.k] = g.c * x1 - g.s * x2;
      x[g.k + 1] = std::conj(g.s) * x1 + g.c * x2;
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
  SchurC sc;
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
  SchurC sc;
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
