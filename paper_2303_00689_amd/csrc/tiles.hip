// The tile table (which GEMM kernel family serves a product of a given order,
// precision and output kind) and the timing call an autotuner fills it from.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <shared_mutex>

#include "../../include/xlbomd.h"
#include "common.h"

namespace xl {
namespace {

struct TileRow {
  int prec, sym, n_max, family;
};
std::shared_mutex table_mutex;
TileRow table_rows[XLBOMD_TILE_TABLE_MAX];
int table_count = 0;

}  // namespace

bool family_runs(int prec, int fam, int n) {
  if (fam == GEMM_AUTO || fam == GEMM_SMALL) return n >= 1;
  // medium tiles: a ragged last k panel (n % 32 != 0) for BF16x3 and BF16x6
  // only; FP16x3's ragged instantiation would spill
  if (fam == GEMM_MEDIUM)
    return prec >= 1 && prec <= 3 && n % (prec == 3 ? 32 : 4) == 0 && n >= 128 && n <= 32767;
  if (fam == GEMM_COMPACT) return prec >= 0 && prec <= 3 && n % 4 == 0 && n >= (prec == 0 ? 4 : 64) && n <= 32767;
  if (fam != GEMM_LARGE) return false;
  if (prec == 0) return n % 16 == 0 && n >= 128 && n <= 23170;
  if (prec >= 1 && prec <= 3) return n % 32 == 0 && n >= 128 && n <= 32767;
  return false;
}

int table_family(int prec, int sym, int n) {
  std::shared_lock<std::shared_mutex> lock(table_mutex);
  for (int i = 0; i < table_count; ++i) {
    const TileRow &r = table_rows[i];
    if (r.prec == prec && r.sym == sym && n <= r.n_max) return r.family;
  }
  return GEMM_AUTO;
}

}  // namespace xl

extern "C" xlbomd_status xlbomd_set_tile_table(const int *rows, int count) {
  if (count < 0 || count > XLBOMD_TILE_TABLE_MAX || (count > 0 && !rows)) return XLBOMD_E_ARG;
  xl::TileRow tmp[XLBOMD_TILE_TABLE_MAX];
  for (int i = 0; i < count; ++i) {
    const int *r = rows + 4 * i;
    if (r[0] < 0 || r[0] > 3 || (r[1] != 0 && r[1] != 1) || r[2] < 1 || r[3] < xl::GEMM_AUTO ||
        r[3] > xl::GEMM_COMPACT)
      return XLBOMD_E_ARG;
    tmp[i] = {r[0], r[1], r[2], r[3]};
  }
  // first matching row wins: order by n_max, keeping the caller's order on ties
  std::stable_sort(tmp, tmp + count, [](const xl::TileRow &a, const xl::TileRow &b) { return a.n_max < b.n_max; });
  std::unique_lock<std::shared_mutex> lock(xl::table_mutex);
  std::copy(tmp, tmp + count, xl::table_rows);
  xl::table_count = count;
  return XLBOMD_OK;
}

extern "C" xlbomd_status xlbomd_time_gemm(int n, int prec, int sym, int family, int reps, void *stream,
                                          double *us) {
  if (n < 1 || prec < 0 || prec > 3 || (sym != 0 && sym != 1) || reps < 1 || !us ||
      (family < xl::GEMM_SMALL || family > xl::GEMM_COMPACT) ||
      !xl::family_runs(prec, family, n))
    return XLBOMD_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t bytes = (size_t)n * n * (prec == 0 ? 8 : 4);
  void *A = nullptr, *B = nullptr, *Cm = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  xlbomd_status st = XLBOMD_E_HIP;
  if (hipMalloc(&A, bytes) == hipSuccess && hipMalloc(&B, bytes) == hipSuccess &&
      hipMalloc(&Cm, bytes) == hipSuccess && hipEventCreate(&e0) == hipSuccess &&
      hipEventCreate(&e1) == hipSuccess && hipMemsetAsync(A, 0x3c, bytes, s) == hipSuccess &&
      hipMemsetAsync(B, 0x3c, bytes, s) == hipSuccess) {
    xl::GemmArgs g{};
    g.n = n;
    g.nprod = 1;
    g.A[0] = A;
    g.B[0] = B;
    g.out = Cm;
    g.alpha = 1.0;
    g.sym = sym;
    g.family = family;
    auto launch = [&]() {
      if (prec == 0)
        xl::gemm_f64(g, s);
      else
        xl::gemm_split(g, prec, s);
    };
    launch();  // warm-up: code object loading, clocks
    float ms = 0.f;
    if (hipEventRecord(e0, s) == hipSuccess) {
      for (int r = 0; r < reps; ++r) launch();
      if (hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
          hipGetLastError() == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) {
        *us = 1e3 * (double)ms / reps;
        st = XLBOMD_OK;
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (A) (void)hipFree(A);
  if (B) (void)hipFree(B);
  if (Cm) (void)hipFree(Cm);
  return st;
}
