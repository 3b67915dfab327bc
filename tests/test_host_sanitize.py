"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Every source of the library is compiled with the sanitizers on the host
pass (device code is built but never launched, so no GPU is needed), with a
small C++ test program that exercises what the host side does on its own:

* the implicit-QL solve of the Lanczos tridiagonal on the seeded cases of
  tests/test_host_eig.py plus the largest order and an order past it;
* the spectral bounds from Gershgorin and Lanczos data, checked against
  numpy: the bounds hold the whole spectrum, lie inside the Gershgorin
  interval, and fall back to it for non-finite data, a Krylov space that
  closes early, or a step count out of range;
* argument validation of every entry point (null handle, null pointers,
  sizes and settings out of range), which must answer XLBOMD_E_ARG before
  any HIP call;
* the tile table: validation, ordering by n_max, first-match lookup.

A sanitizer finding aborts the test program with a non-zero status and its
report on stderr, which the test shows.
"""

import os
import shutil
import subprocess

import numpy as np
import pytest

from test_host_eig import _cases

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2303_00689_amd", "csrc")
SOURCES = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))   # every source of the library
HIPCC = "/opt/rocm/bin/hipcc"
E_ARG = -1

DRIVER = r'''
#include "../../include/xlbomd.h"
#include "common.h"
#include "small_eig.h"
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

static int eig_mode() {
  int cases;
  if (scanf("%d", &cases) != 1) return 1;
  for (int t = 0; t < cases; ++t) {
    int k;
    if (scanf("%d", &k) != 1 || k < 1) return 1;
    std::vector<double> d(k), e(k, 0.0), ev(k), zl(k);
    for (auto &x : d) if (scanf("%lf", &x) != 1) return 1;
    for (int i = 0; i + 1 < k; ++i) if (scanf("%lf", &e[i]) != 1) return 1;
    const bool ok = xl::tridiag_eig_last(k, d.data(), e.data(), ev.data(), zl.data());
    printf("%d", ok ? 1 : 0);
    for (int i = 0; i < k && ok; ++i) printf(" %.17g %.17g", ev[i], zl[i]);
    printf("\n");
  }
  return 0;
}

// stdin: count, then per case g0 g1 K n and 2 K Lanczos coefficients (alpha, beta)
static int bounds_mode() {
  int cases;
  if (scanf("%d", &cases) != 1) return 1;
  for (int t = 0; t < cases; ++t) {
    double g[2];
    int K, n, nab;
    if (scanf("%lf %lf %d %d %d", &g[0], &g[1], &K, &n, &nab) != 5 || nab < 0) return 1;
    // exactly nab values on the heap, so a read past them is an ASan report
    double *ab = new double[nab > 0 ? nab : 1];
    for (int i = 0; i < nab; ++i) if (scanf("%lf", &ab[i]) != 1) return 1;
    double lohi[2] = {NAN, NAN};
    const bool ok = xl::bounds_from_lanczos(g, ab, K, n, lohi);
    printf("%d %.17g %.17g\n", ok ? 1 : 0, lohi[0], lohi[1]);
    delete[] ab;
  }
  return 0;
}

static xlbomd_system good_system(const double *oc, const float *noise) {
  xlbomd_system s;
  memset(&s, 0, sizeof(s));
  s.n_atoms = 2;
  s.n_elec = 8.0;
  s.onecenter = oc;
  s.noise55 = noise;
  return s;
}

static xlbomd_params good_params() {
  xlbomd_params p;
  memset(&p, 0, sizeof(p));
  p.prec = XLBOMD_FP64;
  p.T_e = 3000.0;
  p.m = 4;
  p.dt = 0.5;
  p.kernel_c = 1.0;
  return p;
}

#define REPORT(name, expr) printf("%s %d\n", name, (int)(expr))

static int api_mode() {
  double oc[10] = {0};
  float noise[55] = {0};
  double buf[64] = {0};
  int ibuf[4] = {0};
  xlbomd_handle h = (xlbomd_handle)0x1;  // must be overwritten with NULL on failure
  xlbomd_system s = good_system(oc, noise);
  xlbomd_params p = good_params();
  REPORT("create_null_sys", xlbomd_create(nullptr, &p, nullptr, &h));
  REPORT("create_null_prm", xlbomd_create(&s, nullptr, nullptr, &h));
  REPORT("create_null_out", xlbomd_create(&s, &p, nullptr, nullptr));
  struct SysCase { const char *name; void (*edit)(xlbomd_system &); };
  const SysCase sys_cases[] = {
    {"atoms_0", [](xlbomd_system &x) { x.n_atoms = 0; }},
    {"atoms_8192", [](xlbomd_system &x) { x.n_atoms = 8192; }},
    {"onecenter_null", [](xlbomd_system &x) { x.onecenter = nullptr; }},
    {"noise_null", [](xlbomd_system &x) { x.noise55 = nullptr; }},
    {"n_elec_0", [](xlbomd_system &x) { x.n_elec = 0.0; }},
    {"n_elec_2n", [](xlbomd_system &x) { x.n_elec = 16.0; }},
    {"n_elec_nan", [](xlbomd_system &x) { x.n_elec = NAN; }},
  };
  for (const auto &c : sys_cases) {
    xlbomd_system x = good_system(oc, noise);
    c.edit(x);
    h = (xlbomd_handle)0x1;
    const int st = xlbomd_create(&x, &p, nullptr, &h);
    printf("create_%s %d\n", c.name, st);
    if (st == XLBOMD_E_ARG && h != nullptr) printf("create_%s_handle_not_cleared 0\n", c.name);
  }
  struct PrmCase { const char *name; void (*edit)(xlbomd_params &); };
  const PrmCase prm_cases[] = {
    {"T_e_0", [](xlbomd_params &q) { q.T_e = 0.0; }},
    {"T_e_nan", [](xlbomd_params &q) { q.T_e = NAN; }},
    {"m_neg", [](xlbomd_params &q) { q.m = -1; }},
    {"m_33", [](xlbomd_params &q) { q.m = 33; }},
    {"prec_7", [](xlbomd_params &q) { q.prec = (xlbomd_precision)7; }},
    {"prec_neg", [](xlbomd_params &q) { q.prec = (xlbomd_precision)-1; }},
    {"kernel_c_0", [](xlbomd_params &q) { q.kernel_c = 0.0; }},
    {"kernel_c_inf", [](xlbomd_params &q) { q.kernel_c = INFINITY; }},
    {"w0_limit_neg", [](xlbomd_params &q) { q.w0_limit = -1.0; }},
    {"w0_limit_nan", [](xlbomd_params &q) { q.w0_limit = NAN; }},
    {"T_ion_limit_neg", [](xlbomd_params &q) { q.T_ion_limit = -1.0; }},
  };
  for (const auto &c : prm_cases) {
    xlbomd_params q = good_params();
    c.edit(q);
    h = (xlbomd_handle)0x1;
    printf("create_%s %d\n", c.name, (int)xlbomd_create(&s, &q, nullptr, &h));
  }
  xlbomd_md_state st;
  memset(&st, 0, sizeof(st));
  xlbomd_report rep;
  xlbomd_scf_params sp;
  memset(&sp, 0, sizeof(sp));
  REPORT("destroy", xlbomd_destroy(nullptr));
  REPORT("n_orb", xlbomd_n_orb(nullptr) == 0 ? XLBOMD_E_ARG : 0);
  REPORT("last_error", strcmp(xlbomd_last_error(nullptr), "null handle") == 0 ? XLBOMD_E_ARG : 0);
  REPORT("set_geometry", xlbomd_set_geometry(nullptr, buf));
  REPORT("hcore", xlbomd_hcore(nullptr, buf));
  REPORT("fock", xlbomd_fock(nullptr, buf, buf + 16, 1));
  REPORT("fermi_dm", xlbomd_fermi_dm(nullptr, buf, buf + 1, buf + 16, buf + 2));
  REPORT("spectral_bounds", xlbomd_spectral_bounds(nullptr, buf, buf + 2));
  REPORT("noalloc_null_F", xlbomd_spectral_bounds_noalloc(nullptr, 4, nullptr, buf));
  REPORT("noalloc_null_lohi", xlbomd_spectral_bounds_noalloc(buf, 4, nullptr, nullptr));
  REPORT("noalloc_n_0", xlbomd_spectral_bounds_noalloc(buf, 0, nullptr, buf + 2));
  REPORT("noalloc_n_max", xlbomd_spectral_bounds_noalloc(buf, XLBOMD_SPECTRAL_BOUNDS_NOALLOC_MAX_N + 1,
                                                          nullptr, buf + 2));
  REPORT("dm_response", xlbomd_dm_response(nullptr, buf, buf + 16));
  REPORT("krylov_kernel", xlbomd_krylov_kernel(nullptr, buf, buf + 16, 4, 0.0, buf + 32, ibuf, buf + 48));
  REPORT("forces", xlbomd_forces(nullptr, buf, buf + 16, buf + 32, buf + 48));
  REPORT("integrate", xlbomd_integrate(nullptr, &st));
  REPORT("step", xlbomd_step(nullptr, &st, 1, &rep));
  REPORT("step_langevin", xlbomd_step_langevin(nullptr, &st, 1, 0.01, 300.0, buf, &rep));
  REPORT("ensemble_null", xlbomd_ensemble_step(nullptr, &st, 1, 1, &rep));
  REPORT("ensemble_count_neg", xlbomd_ensemble_step(&h, &st, -1, 1, &rep));
  REPORT("ensemble_steps_neg", xlbomd_ensemble_step(&h, &st, 1, -1, &rep));
  REPORT("md_init", xlbomd_md_init(nullptr, &st));
  REPORT("scf", xlbomd_scf(nullptr, buf, &sp, nullptr, 0, nullptr));
  REPORT("matmul", xlbomd_matmul(nullptr, buf, buf + 16, buf + 32, 0, 1));
  REPORT("profile", xlbomd_profile(nullptr, 1));
  REPORT("profile_read", xlbomd_profile_read(nullptr, buf));
  xlbomd_overlap_model ov = {0.08, 1.4, 0.4}, bad_ov = {0.08, 1.4, 0.0};
  REPORT("overlap", xlbomd_overlap(nullptr, &ov, buf));
  REPORT("overlap_null_model", xlbomd_overlap(nullptr, nullptr, buf));
  REPORT("lowdin", xlbomd_lowdin(nullptr, buf, buf + 16, ibuf));
  REPORT("fermi_dm_nonorth", xlbomd_fermi_dm_nonorth(nullptr, buf, buf + 16, buf + 32, buf + 48, nullptr));
  REPORT("dm_response_nonorth", xlbomd_dm_response_nonorth(nullptr, buf, buf + 16, buf + 32));
  REPORT("pulay_forces", xlbomd_pulay_forces(nullptr, &ov, buf, buf + 16, buf + 32, buf + 48));
  REPORT("pulay_forces_bad_model", xlbomd_pulay_forces(nullptr, &bad_ov, buf, buf + 16, buf + 32, buf + 48));
  double us = 0.0;
  REPORT("time_gemm_n_0", xlbomd_time_gemm(0, 0, 0, 1, 1, nullptr, &us));
  REPORT("time_gemm_prec_4", xlbomd_time_gemm(256, 4, 0, 1, 1, nullptr, &us));
  REPORT("time_gemm_sym_2", xlbomd_time_gemm(256, 0, 2, 1, 1, nullptr, &us));
  REPORT("time_gemm_family_auto", xlbomd_time_gemm(256, 0, 0, 0, 1, nullptr, &us));
  REPORT("time_gemm_family_5", xlbomd_time_gemm(256, 0, 0, 5, 1, nullptr, &us));
  REPORT("time_gemm_medium_fp64", xlbomd_time_gemm(256, 0, 0, 3, 1, nullptr, &us));
  REPORT("time_gemm_reps_0", xlbomd_time_gemm(256, 0, 0, 1, 0, nullptr, &us));
  REPORT("time_gemm_us_null", xlbomd_time_gemm(256, 0, 0, 1, 1, nullptr, nullptr));
  REPORT("time_gemm_large_ragged", xlbomd_time_gemm(400, 1, 0, 2, 1, nullptr, &us));
  REPORT("time_gemm_medium_fp16_ragged", xlbomd_time_gemm(400, 3, 1, 3, 1, nullptr, &us));
  return 0;
}

// stdin: row count and rows, then query count and (prec, sym, n) queries;
// stdout: the status of the install, then one family per query
static int tiles_mode() {
  int count;
  if (scanf("%d", &count) != 1) return 1;
  std::vector<int> rows(4 * (count > 0 ? count : 0) + 1);
  for (int i = 0; i < 4 * count; ++i) if (scanf("%d", &rows[i]) != 1) return 1;
  // the rows live in a heap block of exactly 4 count ints (plus one guard the
  // table must never read as a row)
  int *exact = new int[4 * (count > 0 ? count : 0) + 1];
  memcpy(exact, rows.data(), sizeof(int) * rows.size());
  printf("%d\n", (int)xlbomd_set_tile_table(count > 0 ? exact : nullptr, count));
  delete[] exact;
  int q;
  if (scanf("%d", &q) != 1) return 1;
  for (int i = 0; i < q; ++i) {
    int prec, sym, n;
    if (scanf("%d %d %d", &prec, &sym, &n) != 3) return 1;
    printf("%d\n", xl::table_family(prec, sym, n));
  }
  return 0;
}

int main(int argc, char **argv) {
  if (argc < 2) return 2;
  if (!strcmp(argv[1], "eig")) return eig_mode();
  if (!strcmp(argv[1], "bounds")) return bounds_mode();
  if (!strcmp(argv[1], "api")) return api_mode();
  if (!strcmp(argv[1], "tiles")) return tiles_mode();
  return 2;
}
'''


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which(HIPCC) is None:
        pytest.skip("hipcc not installed")
    d = tmp_path_factory.mktemp("sanitize")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    # device code is built as for the library (the host pass needs its
    # fat binaries to link) but never launched; the sanitizers go on the host
    # pass alone
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-w",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer", "-I", CSRC]
    jobs, objs = [], []
    for f in SOURCES + [str(src)]:
        obj = str(d / (os.path.basename(f).split(".")[0] + ".o"))
        args = [HIPCC] + flags + ["-x", "hip", "-c", os.path.join(CSRC, f), "-o", obj]
        jobs.append(subprocess.Popen(args, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
        objs.append(obj)
    for j in jobs:
        _, err = j.communicate()
        assert j.returncode == 0, err[-4000:]
    exe = d / "drv"
    res = subprocess.run([HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
                          "-fsanitize=undefined"] + objs +
                         ["-o", str(exe), "-L/opt/rocm/lib", "-lhipsolver", "-Wl,-rpath,/opt/rocm/lib"],
                         capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-4000:]
    return str(exe)


def run(driver, mode, text=""):
    env = dict(os.environ)
    # leaks of the HIP runtime's own start-up are not this library's
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    res = subprocess.run([driver, mode], input=text, capture_output=True, text=True, env=env, timeout=120)
    assert res.returncode == 0, res.stderr[-4000:]
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr[-4000:]
    return res.stdout.split("\n")


def test_ql_cases_are_clean_and_correct(driver):
    rng = np.random.default_rng(11)
    cases = _cases()
    cases.append((rng.standard_normal(64), rng.standard_normal(63)))   # the largest order
    inp = [str(len(cases) + 1)]
    for d, e in cases:
        inp += [str(len(d)), " ".join(repr(float(x)) for x in d), " ".join(repr(float(x)) for x in e)]
    inp += ["65", " ".join(["1.0"] * 65), " ".join(["0.5"] * 64)]       # past the fixed arrays
    lines = run(driver, "eig", "\n".join(inp) + "\n")
    for (d, e), line in zip(cases, lines):
        vals = line.split()
        assert vals[0] == "1"
        k = len(d)
        got = np.sort(np.array(vals[1:], dtype=float).reshape(k, 2)[:, 0])
        w = np.linalg.eigvalsh(np.diag(d) + np.diag(e, 1) + np.diag(e, -1))
        assert np.abs(got - w).max() <= 1e-13 * max(1.0, np.abs(w).max()) * k
    assert lines[len(cases)].strip() == "0"


def lanczos(A, v, K):
    """K Lanczos steps with full reorthogonalisation: (alpha, beta) pairs."""
    n = A.shape[0]
    Q = np.zeros((n, K + 1))
    Q[:, 0] = v / np.linalg.norm(v)
    ab = []
    for j in range(K):
        w = A @ Q[:, j]
        a = Q[:, j] @ w
        w -= Q[:, : j + 1] @ (Q[:, : j + 1].T @ w)
        w -= Q[:, : j + 1] @ (Q[:, : j + 1].T @ w)
        b = np.linalg.norm(w)
        ab += [a, b]
        if b == 0.0:
            ab += [0.0, 0.0] * (K - j - 1)
            break
        Q[:, j + 1] = w / b
    return np.array(ab)


def gershgorin(A):
    r = np.abs(A).sum(axis=1) - np.abs(np.diag(A))
    return float((np.diag(A) - r).min()), float((np.diag(A) + r).max())


def bounds_cases():
    rng = np.random.default_rng(5)
    out = []
    # a Fock-like spectrum: a dense band and two outliers; the Lanczos data
    # converge at both ends well within K steps
    n = 48
    Qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.concatenate([np.linspace(-30.0, 10.0, n - 2), [-45.0, 25.0]])
    A = (Qm * lam) @ Qm.T
    A = 0.5 * (A + A.T)
    out.append(("converged", A, lanczos(A, rng.standard_normal(n), 40), 40, n))
    # a random symmetric matrix with every step of the Krylov space (K = n)
    n = 24
    B = rng.standard_normal((n, n))
    B = B + B.T
    out.append(("full", B, lanczos(B, rng.standard_normal(n), n), n, n))
    # a start vector in a 3-dimensional invariant subspace: the space closes
    # at j = 3 < n and only the Gershgorin interval is safe
    D = np.diag(np.arange(10.0))
    v = np.zeros(10)
    v[:3] = 1.0
    out.append(("closed_early", D, lanczos(D, v, 6), 6, 10))
    # a 4 x 4 matrix closed after all 4 dimensions: exact eigenvalues
    C = np.diag([1.0, 2.0, 3.0, 4.0]) + 0.1
    out.append(("closed_full", C, lanczos(C, np.ones(4) + np.arange(4.0), 4), 4, 4))
    return out


def test_spectral_bounds_hold_the_spectrum(driver):
    cases = bounds_cases()
    inp = [str(len(cases) + 5)]
    for _, A, ab, K, n in cases:
        g = gershgorin(A)
        inp.append(f"{g[0]!r} {g[1]!r} {K} {n} {len(ab)} " + " ".join(repr(float(x)) for x in ab))
    ab = lanczos(cases[0][1], np.ones(cases[0][4]), 40)
    g = g_first = gershgorin(cases[0][1])
    bad = ab.copy()
    bad[7] = np.nan
    inp.append(f"{g[0]!r} {g[1]!r} 40 48 80 " + " ".join(repr(float(x)) for x in bad))   # NaN in the data
    inp.append(f"{g[0]!r} {g[1]!r} 0 48 0")                                             # no steps
    inp.append(f"{g[0]!r} {g[1]!r} 65 48 0")                                            # too many steps
    inp.append(f"nan {g[1]!r} 40 48 80 " + " ".join(repr(float(x)) for x in ab))       # Gershgorin not finite
    inp.append(f"{g[0]!r} inf 40 48 80 " + " ".join(repr(float(x)) for x in ab))
    lines = run(driver, "bounds", "\n".join(inp) + "\n")
    for (name, A, ab, K, n), line in zip(cases, lines):
        ok, lo, hi = line.split()
        lo, hi = float(lo), float(hi)
        w = np.linalg.eigvalsh(A)
        g = gershgorin(A)
        print(f"{name}: [{lo:.6f}, {hi:.6f}] spectrum [{w[0]:.6f}, {w[-1]:.6f}] Gershgorin [{g[0]:.3f}, {g[1]:.3f}]")
        assert ok == "1"
        assert g[0] <= lo <= w[0] and w[-1] <= hi <= g[1]
        if name == "closed_early":
            assert (lo, hi) == g
        else:
            # tight: the widening is 1e-3 of the spread plus the residual bounds
            assert w[0] - lo <= 2e-3 * (w[-1] - w[0]) and hi - w[-1] <= 2e-3 * (w[-1] - w[0])
    rest = lines[len(cases):len(cases) + 5]
    for line in rest[:3]:
        ok, lo, hi = line.split()
        assert ok == "1" and (float(lo), float(hi)) == g_first
    assert rest[3].split()[0] == "0" and rest[4].split()[0] == "0"


def test_every_entry_point_rejects_bad_arguments_before_hip(driver):
    lines = [ln for ln in run(driver, "api") if ln.strip()]
    assert len(lines) == 64          # every call of the test program reported
    for line in lines:
        name, st = line.split()
        assert int(st) == E_ARG, f"{name} returned {st}"


def test_tile_table_orders_and_matches_rows(driver):
    rows = [[1, 0, 500, 2], [0, 1, 300, 1], [1, 0, 200, 1], [1, 0, 200, 2], [3, 1, 4096, 1]]
    queries = [(1, 0, 150), (1, 0, 200), (1, 0, 201), (1, 0, 500), (1, 0, 501), (0, 1, 300), (0, 0, 100),
               (3, 1, 4096), (3, 1, 4097), (2, 0, 100)]
    text = [str(len(rows))] + [" ".join(map(str, r)) for r in rows]
    text += [str(len(queries))] + [" ".join(map(str, q)) for q in queries]
    out = [ln for ln in run(driver, "tiles", "\n".join(text) + "\n") if ln.strip()]
    assert out[0] == "0"
    # sorted by n_max, ties in the caller's order, first match wins, none: auto (0)
    assert [int(x) for x in out[1:]] == [1, 1, 2, 2, 0, 1, 0, 1, 0, 0]
    for bad in ([[4, 0, 100, 1]], [[0, 2, 100, 1]], [[0, 0, 0, 1]], [[0, 0, 100, 5]], [[0, 0, 100, -1]]):
        text = ["1", " ".join(map(str, bad[0])), "1", "0 0 50"]
        out = [ln for ln in run(driver, "tiles", "\n".join(text) + "\n") if ln.strip()]
        assert out == [str(E_ARG), "0"]
    for count in (-1, 257):
        out = [ln for ln in run(driver, "tiles", f"{count}\n" + "0 0 100 1\n" * max(count, 0) + "0\n")
               if ln.strip()]
        assert out == [str(E_ARG)]
    # an empty table is allowed and makes every lookup auto
    out = [ln for ln in run(driver, "tiles", "0\n1\n1 0 100\n") if ln.strip()]
    assert out == ["0", "0"]
