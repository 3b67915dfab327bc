// Host-side eigen-decomposition of small dense symmetric matrices by the
// cyclic Jacobi method (used on the k x k Lanczos tridiagonal, k <= 64).
#pragma once

#include <cmath>
#include <vector>

namespace xl {

// A: k x k symmetric, row-major, overwritten.  On return ev[i] are the
// eigenvalues (unsorted) and column i of V (row-major k x k) the matching
// unit eigenvector.  Returns false if the sweeps did not converge.
inline bool jacobi_eig(int k, std::vector<double> &A, std::vector<double> &V, std::vector<double> &ev) {
  V.assign((size_t)k * k, 0.0);
  for (int i = 0; i < k; ++i) V[(size_t)i * k + i] = 1.0;
  double frob = 0.0;
  for (double a : A) frob += a * a;
  bool conv = false;
  for (int sweep = 0; sweep < 64 && !conv; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < k; ++p)
      for (int q = p + 1; q < k; ++q) off += A[(size_t)p * k + q] * A[(size_t)p * k + q];
    if (off <= 1e-32 * frob) {
      conv = true;
      break;
    }
    for (int p = 0; p < k; ++p) {
      for (int q = p + 1; q < k; ++q) {
        const double apq = A[(size_t)p * k + q];
        if (apq == 0.0) continue;
        const double th = (A[(size_t)q * k + q] - A[(size_t)p * k + p]) / (2.0 * apq);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        // A <- J^T A J, J = rotation in the (p, q) plane
        for (int r = 0; r < k; ++r) {
          const double arp = A[(size_t)r * k + p], arq = A[(size_t)r * k + q];
          A[(size_t)r * k + p] = cs * arp - sn * arq;
          A[(size_t)r * k + q] = sn * arp + cs * arq;
        }
        for (int r = 0; r < k; ++r) {
          const double apr = A[(size_t)p * k + r], aqr = A[(size_t)q * k + r];
          A[(size_t)p * k + r] = cs * apr - sn * aqr;
          A[(size_t)q * k + r] = sn * apr + cs * aqr;
        }
        for (int r = 0; r < k; ++r) {
          const double vrp = V[(size_t)r * k + p], vrq = V[(size_t)r * k + q];
          V[(size_t)r * k + p] = cs * vrp - sn * vrq;
          V[(size_t)r * k + q] = sn * vrp + cs * vrq;
        }
      }
    }
  }
  ev.resize(k);
  for (int i = 0; i < k; ++i) ev[i] = A[(size_t)i * k + i];
  return conv;
}

}  // namespace xl
