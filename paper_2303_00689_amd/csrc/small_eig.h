// Host-side eigenvalues of the k x k Lanczos tridiagonal (k <= SMALL_EIG_MAX)
// by the implicit QL iteration with Wilkinson shifts: the published method of
// Bowdler, Martin, Reinsch and Wilkinson, "The QR and QL algorithms for
// symmetric matrices", Numer. Math. 11 (1968) 293-306 (Handbook for Automatic
// Computation II/3; EISPACK tql2), written here from that description.  The one
// change is that only the last row of the accumulated rotations is kept: the
// last component of every Ritz vector, which is all the residual bounds
// beta_k |s_k| need.  O(k^2) work, fixed-size arrays, no allocation.
#pragma once

#include <cmath>

namespace xl {

constexpr int SMALL_EIG_MAX = 64;

// d: diagonal (k), e: off-diagonal (k - 1).  On return ev[i] are the
// eigenvalues (unsorted) and zl[i] the last component of the matching unit
// eigenvector.  Returns false if k is out of range or an eigenvalue took more
// than 60 QL steps.
inline bool tridiag_eig_last(int k, const double *d, const double *e, double *ev, double *zl) {
  if (k < 1 || k > SMALL_EIG_MAX) return false;
  double off[SMALL_EIG_MAX];
  for (int i = 0; i < k; ++i) {
    ev[i] = d[i];
    off[i] = i + 1 < k ? e[i] : 0.0;
    zl[i] = 0.0;
  }
  zl[k - 1] = 1.0;
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

// Spectral bounds of a symmetric n x n matrix from its Gershgorin interval
// g[0..1] and K Lanczos steps ab[2 j] = alpha_j, ab[2 j + 1] = beta_j: the
// extreme Ritz values widened by their residual bounds beta_k |s_k| and by
// 1e-3 of the Ritz spread, clipped to the Gershgorin interval.  The
// Gershgorin interval is kept alone if the Lanczos data are not finite, if
// the small solve fails, or if the Krylov space closed (beta_j ~ 0) before
// spanning all n dimensions: its Ritz values are then eigenvalues, but the
// eigenvalues outside it are not seen.  Returns false if g is not finite.
inline bool bounds_from_lanczos(const double g[2], const double *ab, int K, int n, double lohi[2]) {
  if (!std::isfinite(g[0]) || !std::isfinite(g[1])) return false;
  lohi[0] = g[0];
  lohi[1] = g[1];
  if (K < 1 || K > SMALL_EIG_MAX) return true;
  const double scale = std::fmax(std::fabs(g[0]), std::fabs(g[1]));
  int k = K;
  for (int j = 0; j < K; ++j) {
    if (!std::isfinite(ab[2 * j]) || !std::isfinite(ab[2 * j + 1])) return true;  // keep Gershgorin
    if (ab[2 * j + 1] <= 1e-12 * scale) {
      // invariant subspace: the Ritz values are eigenvalues, and all of them
      // only if the subspace is the whole space
      if (j + 1 < n) return true;
      k = j + 1;
      break;
    }
  }
  double dg[SMALL_EIG_MAX], od[SMALL_EIG_MAX], th[SMALL_EIG_MAX], zl[SMALL_EIG_MAX];
  for (int j = 0; j < k; ++j) {
    dg[j] = ab[2 * j];
    od[j] = ab[2 * j + 1];
  }
  if (!tridiag_eig_last(k, dg, od, th, zl)) return true;
  int imin = 0, imax = 0;
  for (int i = 1; i < k; ++i) {
    if (th[i] < th[imin]) imin = i;
    if (th[i] > th[imax]) imax = i;
  }
  const double bk = ab[2 * (k - 1) + 1];
  const double rmin = bk * std::fabs(zl[imin]);
  const double rmax = bk * std::fabs(zl[imax]);
  const double margin = 1e-3 * (th[imax] - th[imin]) + 1e-12 * scale;
  lohi[0] = std::fmax(g[0], th[imin] - rmin - margin);
  lohi[1] = std::fmin(g[1], th[imax] + rmax + margin);
  return true;
}

}  // namespace xl
