// Test driver for the host small-problem routines (host_la.cpp), built with
// g++ and the address and undefined-behaviour sanitizers by
// tests/test_host_la.py.  Reads commands from stdin, one per line, and
// prints the results as whitespace-separated numbers (%.17g):
//   givens j ldh beta H[ldh*j]         -> res y[j]
//   qr m k A[m*k]                      -> ok Q[m*k] R[k*k]
//   chol k G[k*k]                      -> ok R[k*k]
//   invu k R[k*k]                      -> Rinv[k*k]
//   eig N A[N*N]                       -> ok w[N] as (re im), V[N*N] as (re im)
//   hritz rows cols k G[rows*cols] M[rows*cols] -> kout P[cols*kout]
// All matrices column-major, as in host_la.h.
#include <complex>
#include <cstdio>
#include <iostream>
#include <string>
#include <vector>

#include "host_la.h"

namespace {

std::vector<double> read_vec(size_t n) {
  std::vector<double> v(n);
  for (auto& x : v) std::cin >> x;
  return v;
}

void put(double x) { std::printf("%.17g ", x); }

void put_vec(const double* v, size_t n) {
  for (size_t i = 0; i < n; ++i) put(v[i]);
}

}  // namespace

int main() {
  std::string cmd;
  while (std::cin >> cmd) {
    if (cmd == "givens") {
      int j, ldh;
      double beta;
      std::cin >> j >> ldh >> beta;
      auto H = read_vec((size_t)ldh * j);
      std::vector<double> y(j > 0 ? j : 1);
      const double res = gir::la::givens_lsq(H.data(), ldh, j, beta, y.data());
      put(res);
      put_vec(y.data(), j);
    } else if (cmd == "qr") {
      int m, k;
      std::cin >> m >> k;
      auto A = read_vec((size_t)m * k);
      std::vector<double> Q((size_t)m * k), R((size_t)k * k);
      const bool ok = gir::la::qr_thin(A.data(), m, m, k, Q.data(), R.data());
      put(ok ? 1 : 0);
      put_vec(Q.data(), Q.size());
      put_vec(R.data(), R.size());
    } else if (cmd == "chol") {
      int k;
      std::cin >> k;
      auto G = read_vec((size_t)k * k);
      std::vector<double> R((size_t)k * k);
      const bool ok = gir::la::cholesky_upper(G.data(), k, R.data());
      put(ok ? 1 : 0);
      put_vec(R.data(), R.size());
    } else if (cmd == "invu") {
      int k;
      std::cin >> k;
      auto R = read_vec((size_t)k * k);
      std::vector<double> Ri((size_t)k * k);
      gir::la::inv_upper(R.data(), k, Ri.data());
      put_vec(Ri.data(), Ri.size());
    } else if (cmd == "eig") {
      int N;
      std::cin >> N;
      auto A = read_vec((size_t)N * N);
      std::vector<std::complex<double>> w, V;
      const bool ok = gir::la::eig_real(A.data(), N, w, V);
      put(ok ? 1 : 0);
      for (int i = 0; i < N; ++i) {
        put(i < (int)w.size() ? w[i].real() : 0.0);
        put(i < (int)w.size() ? w[i].imag() : 0.0);
      }
      for (size_t i = 0; i < (size_t)N * N; ++i) {
        put(i < V.size() ? V[i].real() : 0.0);
        put(i < V.size() ? V[i].imag() : 0.0);
      }
    } else if (cmd == "hritz") {
      int rows, cols, k;
      std::cin >> rows >> cols >> k;
      auto G = read_vec((size_t)rows * cols);
      auto M = read_vec((size_t)rows * cols);
      std::vector<double> P((size_t)cols * (k > 0 ? k : 1));
      const int kout = gir::la::harmonic_ritz(G.data(), M.data(), rows, cols, k, P.data());
      put(kout);
      put_vec(P.data(), (size_t)cols * (kout > 0 ? kout : 0));
    } else {
      std::fprintf(stderr, "unknown command %s\n", cmd.c_str());
      return 2;
    }
    std::printf("\n");
    std::fflush(stdout);
  }
  return 0;
}
