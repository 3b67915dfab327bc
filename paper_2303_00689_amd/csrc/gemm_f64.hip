// FP64 MFMA GEMM with fused epilogue for the Fermi-operator and response chains.
//
// Tile 64 x 64 per workgroup of 256 threads (4 wavefronts of 64 lanes in a
// 2 x 2 arrangement, 32 x 32 each = 2 x 2 blocks of v_mfma_f64_16x16x4).  The
// K dimension advances by 16 through double-buffered LDS panels; the next
// panel is fetched into registers while the current one feeds the MFMAs.
//
// Operand layout for v_mfma_f64_16x16x4f64 (one double per lane):
//   A (16 x 4): lane l holds A[l % 16][l / 16]
//   B (4 x 16): lane l holds B[l / 16][l % 16]
//   D (16 x 16): lane l holds D[l / 16 + 4 * q][l % 16], q = 0..3
// LDS panels are stored k-major (As[k][m], Bs[k][n]) so that both fragments
// are read as 16 consecutive doubles per lane group.
#include "common.h"
#include "tile_map.h"

namespace xl {
namespace {

constexpr int TILE_GROUP = 8;  // tile rows per L2-sharing group

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64;
constexpr int BK = 16;

__global__ __launch_bounds__(256) void k_gemm_f64(GemmArgs p, int T) {
  const int n = p.n;
  int bi, bj;
  tile_of(blockIdx.x, T, p.sym, TILE_GROUP, bi, bj);
  const int i0 = bi * BM, j0 = bj * BM;
  __shared__ double As[2][BK][BM];
  __shared__ double Bs[2][BK][BM];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;

  d4 acc[2][2];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[r][c] = d4{0.0, 0.0, 0.0, 0.0};

  const int kt_per = (n + BK - 1) / BK;
  const int ktiles = kt_per * p.nprod;

  // A panel rows k (16) x cols m (64): thread -> (k = tid / 16, m = 4 * (tid % 16))
  const int la_k = tid >> 4, la_m = (tid & 15) * 4;
  // B panel, normal: same mapping; transposed: rows j (64) x 16 k: (j = tid / 4, k = 4 * (tid % 4))
  const int lbt_j = tid >> 2, lbt_k = (tid & 3) * 4;

  // Unconditional loads from clamped in-bounds addresses (n % 4 == 0, so a
  // group of four consecutive columns is either all in range or all out);
  // the zeroing select happens in store(), after the MFMAs of the current
  // panel, so that the loads of the next panel stay in flight during them.
  typedef double dd2 __attribute__((ext_vector_type(2)));
  dd2 ua[2], ub[2];
  bool oka = true, okb = true;
  auto load = [&](int kt) {
    const int prod = kt / kt_per;
    const int k0 = (kt - prod * kt_per) * BK;
    const double *A = (const double *)p.A[prod];
    const double *B = (const double *)p.B[prod];
    {
      const int k = k0 + la_k, m = i0 + la_m;
      oka = k < n && m < n;
      const double *src = A + (size_t)(k < n ? k : n - 1) * n + (m < n ? m : n - 4);
      ua[0] = *(const dd2 *)src;
      ua[1] = *(const dd2 *)(src + 2);
    }
    if (!p.btrans) {
      const int k = k0 + la_k, j = j0 + la_m;
      okb = k < n && j < n;
      const double *src = B + (size_t)(k < n ? k : n - 1) * n + (j < n ? j : n - 4);
      ub[0] = *(const dd2 *)src;
      ub[1] = *(const dd2 *)(src + 2);
    } else {
      const int j = j0 + lbt_j, k = k0 + lbt_k;
      okb = k < n && j < n;
      const double *src = B + (size_t)(j < n ? j : n - 1) * n + (k < n ? k : n - 4);
      ub[0] = *(const dd2 *)src;
      ub[1] = *(const dd2 *)(src + 2);
    }
  };
  auto store = [&](int buf) {
    const double ra[4] = {oka ? ua[0][0] : 0.0, oka ? ua[0][1] : 0.0, oka ? ua[1][0] : 0.0, oka ? ua[1][1] : 0.0};
    const double rb[4] = {okb ? ub[0][0] : 0.0, okb ? ub[0][1] : 0.0, okb ? ub[1][0] : 0.0, okb ? ub[1][1] : 0.0};
#pragma unroll
    for (int q = 0; q < 4; ++q) As[buf][la_k][la_m + q] = ra[q];
    if (!p.btrans) {
#pragma unroll
      for (int q = 0; q < 4; ++q) Bs[buf][la_k][la_m + q] = rb[q];
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) Bs[buf][lbt_k + q][lbt_j] = rb[q];
    }
  };

  load(0);
  store(0);
  __syncthreads();
  for (int kt = 0; kt < ktiles; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < ktiles) load(kt + 1);
    // fragments of k-step kk + 4 are read while the MFMAs of step kk run
    double fa0, fa1, fb0, fb1;
    auto frags = [&](int kk) {
      const int kr = kk + (lane >> 4);
      fa0 = As[buf][kr][wm + (lane & 15)];
      fa1 = As[buf][kr][wm + 16 + (lane & 15)];
      fb0 = Bs[buf][kr][wn + (lane & 15)];
      fb1 = Bs[buf][kr][wn + 16 + (lane & 15)];
    };
    frags(0);
    __builtin_amdgcn_iglp_opt(0);  // interleave the LDS reads with the MFMAs
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const double a0 = fa0, a1 = fa1, b0 = fb0, b1 = fb1;
      if (kk + 4 < BK) frags(kk + 4);
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    if (kt + 1 < ktiles) store(buf ^ 1);
    __syncthreads();
  }

  const double *C1 = (const double *)p.C1;
  const double *C2 = (const double *)p.C2;
  double *out = (double *)p.out;
  const bool mirror = p.sym && (bi != bj);
#pragma unroll
  for (int r = 0; r < 2; ++r) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int j = j0 + wn + c * 16 + (lane & 15);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = i0 + wm + r * 16 + (lane >> 4) + 4 * q;
        if (i < n && j < n) {
          const size_t off = (size_t)i * n + j;
          double x = p.alpha * acc[r][c][q];
          if (C1) x += p.beta1 * C1[off];
          if (C2) x += p.beta2 * C2[off];
          if (i == j) x += p.gamma;
          out[off] = x;
          if (mirror) out[(size_t)j * n + i] = x;
        }
      }
    }
  }
}

}  // namespace

void gemm_f64(const GemmArgs &a, hipStream_t s) {
  const int T = (a.n + BM - 1) / BM;
  const int blocks = a.sym ? T * (T + 1) / 2 : T * T;
  hipLaunchKernelGGL(k_gemm_f64, dim3(blocks), dim3(256), 0, s, a, T);
}

}  // namespace xl
