"""The host solver behind the Lanczos spectral bounds: implicit QL on a
symmetric tridiagonal matrix that keeps only the last row of the eigenvector
matrix.  A small C++ driver built with g++ against the library's header runs it
on seeded tridiagonals (dense spectra, clusters, split blocks, 1x1 and 2x2),
and numpy's dense eigensolver is the reference for the eigenvalues and for the
last components of the unit eigenvectors (compared in absolute value, so the
sign of each eigenvector does not matter)."""

import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "paper_2303_00689_amd", "csrc", "small_eig.h")

DRIVER = r'''
#include "small_eig.h"
#include <cstdio>
#include <vector>
// stdin: count, then per case k, d[0..k), e[0..k-1); stdout: ok flag, eigenvalues, last components
int main() {
  int cases;
  if (scanf("%d", &cases) != 1) return 1;
  for (int t = 0; t < cases; ++t) {
    int k;
    if (scanf("%d", &k) != 1) return 1;
    std::vector<double> d(k), e(k, 0.0), ev(k), zl(k);
    for (auto &x : d) if (scanf("%lf", &x) != 1) return 1;
    for (int i = 0; i + 1 < k; ++i) if (scanf("%lf", &e[i]) != 1) return 1;
    const bool ok = xl::tridiag_eig_last(k, d.data(), e.data(), ev.data(), zl.data());
    printf("%d", ok ? 1 : 0);
    for (int i = 0; i < k; ++i) printf(" %.17g %.17g", ev[i], zl[i]);
    printf("\n");
  }
  return 0;
}
'''


def _cases():
    rng = np.random.default_rng(7)
    out = [(np.array([3.5]), np.array([])), (np.array([1.0, 2.0]), np.array([0.5]))]
    for k in (3, 8, 16, 32, 48, 64):
        out.append((10.0 * rng.standard_normal(k), 3.0 + rng.standard_normal(k - 1)))
    # a Lanczos-like tridiagonal of a spectrum with clusters
    out.append((np.repeat([-20.0, 0.0, 15.0], 10) + 1e-3 * rng.standard_normal(30),
                1e-2 * rng.random(29)))
    # exact splits: zero couplings make independent blocks
    d = rng.standard_normal(20)
    e = rng.standard_normal(19)
    e[[4, 11]] = 0.0
    out.append((d, e))
    # equal diagonal (degenerate start of the shift)
    out.append((np.full(12, 2.0), np.ones(11)))
    return out


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("eig")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True)
    return str(exe)


def test_ql_matches_dense_eigensolver(driver):
    cases = _cases()
    inp = [str(len(cases))]
    for d, e in cases:
        inp.append(str(len(d)))
        inp.append(" ".join(repr(float(x)) for x in d))
        inp.append(" ".join(repr(float(x)) for x in e))
    res = subprocess.run([driver], input="\n".join(inp) + "\n", capture_output=True, text=True, check=True)
    lines = res.stdout.strip().splitlines()
    assert len(lines) == len(cases)
    for (d, e), line in zip(cases, lines):
        vals = line.split()
        assert vals[0] == "1"
        k = len(d)
        got = np.array(vals[1:], dtype=float).reshape(k, 2)
        T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
        w, V = np.linalg.eigh(T)
        scale = max(1.0, np.abs(w).max())
        order = np.argsort(got[:, 0])
        assert np.abs(got[order, 0] - w).max() <= 1e-13 * scale * k
        # last components: unique up to sign for simple eigenvalues; within a
        # cluster compare the sum of squares, which is basis independent
        zl = np.abs(got[order, 1])
        ref = np.abs(V[-1, :])
        gaps = np.diff(w)
        simple = np.ones(k, bool)
        simple[:-1] &= gaps > 1e-6 * scale
        simple[1:] &= gaps > 1e-6 * scale
        assert np.abs(zl[simple] - ref[simple]).max(initial=0.0) <= 1e-10
        assert abs(np.sum(zl ** 2) - 1.0) <= 1e-12 * k
