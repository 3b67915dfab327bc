// Workgroup -> output-tile map for the GEMM kernels, aware of the eight XCDs
// of the MI355X.
//
// Workgroups are dispatched to the XCDs round-robin by workgroup id, and each
// XCD has its own L2.  The map first gives every XCD one contiguous range of
// logical tile indices (XCD x receives ids x, x + 8, x + 16, ... and runs them
// in that order).  Logical tiles are then ordered in groups of G tile rows,
// column by column inside a group, so the workgroups resident on one XCD at
// the same time share a few A row panels and B column panels through its L2.
// With sym != 0 only the upper triangle (bj >= bi) is enumerated.
#pragma once

#include <hip/hip_runtime.h>

namespace xl {

constexpr int NXCD = 8;

__host__ __device__ inline int tile_count(int T, int sym) { return sym ? T * (T + 1) / 2 : T * T; }

__host__ __device__ inline void tile_of(int w, int T, int sym, int G, int &bi, int &bj) {
  const int B = tile_count(T, sym);
  // XCD-contiguous logical index
  const int q = B / NXCD, r = B % NXCD;
  const int x = w % NXCD, k = w / NXCD;
  int l = (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
  // row group containing l
  int r0 = 0;
  while (true) {
    const int r1 = r0 + G < T ? r0 + G : T;
    const int h = r1 - r0;
    const int size = sym ? h * (h + 1) / 2 + h * (T - r1) : h * T;
    if (l < size) {
      if (!sym) {
        bj = l / h;
        bi = r0 + l % h;
      } else if (l < h * (h + 1) / 2) {
        // leading triangle: column c holds rows r0 .. r0 + c
        int c = 0;
        while ((c + 1) * (c + 2) / 2 <= l) ++c;
        bj = r0 + c;
        bi = r0 + (l - c * (c + 1) / 2);
      } else {
        const int m = l - h * (h + 1) / 2;
        bj = r1 + m / h;
        bi = r0 + m % h;
      }
      return;
    }
    l -= size;
    r0 = r1;
  }
}

// Symmetric outputs on rectangular tiles of 2h x h (TI tile rows of 2h, TJ
// tile columns of h): tile (I, J) holds entries with j >= i exactly when
// J >= 2 I, so those are the tiles enumerated, row by row, after the same
// XCD-contiguous remap as tile_of.
__host__ __device__ inline int tile_count_rect_sym(int TI, int TJ) {
  int c = 0;
  for (int I = 0; I < TI; ++I) c += TJ - 2 * I > 0 ? TJ - 2 * I : 0;
  return c;
}

__host__ __device__ inline void tile_of_rect_sym(int w, int TI, int TJ, int &bi, int &bj) {
  const int B = tile_count_rect_sym(TI, TJ);
  const int q = B / NXCD, r = B % NXCD;
  const int x = w % NXCD, k = w / NXCD;
  int l = (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
  for (int I = 0; I < TI; ++I) {
    const int cnt = TJ - 2 * I > 0 ? TJ - 2 * I : 0;
    if (l < cnt) {
      bi = I;
      bj = 2 * I + l;
      return;
    }
    l -= cnt;
  }
  bi = bj = 0;  // not reached for w < tile_count_rect_sym
}

}  // namespace xl
