// Host-side eigenvalues of the k x k Lanczos tridiagonal (k <= 64) by the
// implicit QL iteration with Wilkinson shifts, keeping only the last row of the
// accumulated rotations: the last component of every Ritz vector, which is all
// the residual bounds beta_k |s_k| need.  O(k^2) work.
#pragma once

#include <cmath>
#include <vector>

namespace xl {

// d: diagonal (k), e: off-diagonal (k - 1).  On return ev[i] are the
// eigenvalues (unsorted) and zl[i] the last component of the matching unit
// eigenvector.  Returns false if an eigenvalue took more than 60 QL steps.
inline bool tridiag_eig_last(int k, const std::vector<double> &d, const std::vector<double> &e,
                             std::vector<double> &ev, std::vector<double> &zl) {
  ev.assign(d.begin(), d.begin() + k);
  std::vector<double> off(k, 0.0);
  for (int i = 0; i + 1 < k; ++i) off[i] = e[i];
  zl.assign(k, 0.0);
  if (k > 0) zl[k - 1] = 1.0;
  for (int l = 0; l < k; ++l) {
    for (int iter = 0;; ++iter) {
      // the first negligible off-diagonal entry at or after l splits the matrix
      int m = l;
      for (; m + 1 < k; ++m) {
        const double scale = std::fabs(ev[m]) + std::fabs(ev[m + 1]);
        if (std::fabs(off[m]) <= 2.3e-16 * scale) break;
      }
      if (m == l) break;
      if (iter == 60) return false;
      // Wilkinson shift from the leading 2 x 2 block of the unreduced part
      double g = (ev[l + 1] - ev[l]) / (2.0 * off[l]);
      double r = std::sqrt(g * g + 1.0);
      g = ev[m] - ev[l] + off[l] / (g + (g >= 0.0 ? r : -r));
      double s = 1.0, c = 1.0, p = 0.0;
      bool deflated = false;
      // chase the bulge from the bottom of the block up to l with Givens rotations
      for (int i = m - 1; i >= l; --i) {
        const double f = s * off[i], b = c * off[i];
        r = std::sqrt(f * f + g * g);  // entries are energies: no overflow
        off[i + 1] = r;
        if (r == 0.0) {
          ev[i + 1] -= p;
          off[m] = 0.0;
          deflated = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = ev[i + 1] - p;
        r = (ev[i] - g) * s + 2.0 * c * b;
        p = s * r;
        ev[i + 1] = g + p;
        g = c * r - b;
        // the rotation acts on columns i, i+1 of the eigenvector matrix; keep its last row
        const double zi = zl[i], zi1 = zl[i + 1];
        zl[i + 1] = s * zi + c * zi1;
        zl[i] = c * zi - s * zi1;
      }
      if (deflated) continue;
      ev[l] -= p;
      off[l] = g;
      off[m] = 0.0;
    }
  }
  return true;
}

}  // namespace xl
