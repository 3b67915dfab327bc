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

// ---------------------------------------------------------------------------
// Compact FP64 GEMM for small orders: 32 x 32 tiles, four waves of one 16 x 16
// block each, so an order gives four times the workgroups of the 64 x 64
// kernel (its products are latency-bound there, and more workgroups keep more
// compute units busy).  Same conventions as k_gemm_f64: K advances by 16
// through double-buffered LDS panels, loads from clamped in-bounds addresses
// (n % 4 == 0: a pair of consecutive columns is all in range or all out),
// zeroed after the loads.
constexpr int CM = 32;

__global__ __launch_bounds__(256) void k_gemm_f64_c32(GemmArgs p, int T) {
  const int n = p.n;
  int bi, bj;
  tile_of(blockIdx.x, T, p.sym, TILE_GROUP, bi, bj);
  const int i0 = bi * CM, j0 = bj * CM;
  __shared__ double As[2][BK][CM];
  __shared__ double Bs[2][BK][CM];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave >> 1) * 16, wn = (wave & 1) * 16;
  d4 acc = d4{0.0, 0.0, 0.0, 0.0};
  const int kt_per = (n + BK - 1) / BK;
  const int ktiles = kt_per * p.nprod;
  // A panel (and B not transposed) k (16) x m (32): thread -> (k = tid / 16, m = 2 (tid % 16));
  // B transposed, rows j (32) x 16 k: thread -> (j = tid / 8, k = 2 (tid % 8))
  const int la_k = tid >> 4, la_m = (tid & 15) * 2;
  const int lbt_j = tid >> 3, lbt_k = (tid & 7) * 2;
  typedef double dd2 __attribute__((ext_vector_type(2)));
  dd2 ua, ub;
  bool oka = true, okb = true;
  auto load = [&](int kt) {
    const int prod = kt / kt_per;
    const int k0 = (kt - prod * kt_per) * BK;
    const double *A = (const double *)p.A[prod];
    const double *B = (const double *)p.B[prod];
    {
      const int k = k0 + la_k, m = i0 + la_m;
      oka = k < n && m < n;
      ua = *(const dd2 *)(A + (size_t)(k < n ? k : n - 1) * n + (m < n ? m : n - 2));
    }
    if (!p.btrans) {
      const int k = k0 + la_k, j = j0 + la_m;
      okb = k < n && j < n;
      ub = *(const dd2 *)(B + (size_t)(k < n ? k : n - 1) * n + (j < n ? j : n - 2));
    } else {
      const int j = j0 + lbt_j, k = k0 + lbt_k;
      okb = k < n && j < n;
      ub = *(const dd2 *)(B + (size_t)(j < n ? j : n - 1) * n + (k < n ? k : n - 2));
    }
  };
  auto store = [&](int buf) {
    As[buf][la_k][la_m] = oka ? ua[0] : 0.0;
    As[buf][la_k][la_m + 1] = oka ? ua[1] : 0.0;
    if (!p.btrans) {
      Bs[buf][la_k][la_m] = okb ? ub[0] : 0.0;
      Bs[buf][la_k][la_m + 1] = okb ? ub[1] : 0.0;
    } else {
      Bs[buf][lbt_k][lbt_j] = okb ? ub[0] : 0.0;
      Bs[buf][lbt_k + 1][lbt_j] = okb ? ub[1] : 0.0;
    }
  };

  load(0);
  store(0);
  __syncthreads();
  for (int kt = 0; kt < ktiles; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < ktiles) load(kt + 1);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(As[buf][kr][wm + (lane & 15)], Bs[buf][kr][wn + (lane & 15)], acc,
                                                 0, 0, 0);
    }
    if (kt + 1 < ktiles) store(buf ^ 1);
    __syncthreads();
  }

  const double *C1 = (const double *)p.C1;
  const double *C2 = (const double *)p.C2;
  double *out = (double *)p.out;
  const bool mirror = p.sym && (bi != bj);
  const int j = j0 + wn + (lane & 15);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = i0 + wm + (lane >> 4) + 4 * q;
    if (i < n && j < n) {
      const size_t off = (size_t)i * n + j;
      double x = p.alpha * acc[q];
      if (C1) x += p.beta1 * C1[off];
      if (C2) x += p.beta2 * C2[off];
      if (i == j) x += p.gamma;
      out[off] = x;
      if (mirror) out[(size_t)j * n + i] = x;
    }
  }
}

// ---------------------------------------------------------------------------
// Large-tile FP64 GEMM: 128 x 128 tiles, four waves of 64 x 64 (4 x 4 blocks
// of v_mfma_f64_16x16x4f64), two workgroups per compute unit.  Against the
// 64 x 64 kernel the workgroup reads half the operand bytes per flop from L2.
//
// K advances by 16.  The panels stream into LDS by buffer loads, two stages
// in separate LDS arrays, so the loads of panel k + 1 need no wait before the
// reads of panel k; the one barrier per panel is where a panel's loads are
// complete and the stage read before it is free.
//   A panel (and B when not transposed): 16 k rows of 128 doubles, each row
//     one 1 KB load instruction, rows padded to 1152 bytes so that the four
//     k rows one fragment read touches fall on different banks;
//   B transposed: 128 rows j of 16 k values (128 bytes), eight rows per load
//     instruction, 16-byte chunk c of row j at position c ^ (j & 7) ^ ((j >> 3) & 1).
// n % 16 == 0 is required (every k panel full); rows and columns past n are
// read clamped and never stored.
typedef __attribute__((address_space(3))) void lds_void_t;

constexpr int FT = 128;                 // tile edge
constexpr int FK = 16;                  // k panel
constexpr int FROW = 144;               // doubles per padded k row (1152 bytes)
constexpr int FSTAGE = 2 * FK * FROW;   // doubles per stage (A rows, then B rows): 36 KB
constexpr int F_GROUP = 4;              // tile rows per L2-sharing group
constexpr int F_BUF_WORD3 = 0x00020000;  // raw buffer descriptor word 3

__device__ inline int swz8(int r, int c) { return c ^ (r & 7) ^ ((r >> 3) & 1); }

// TN = 128: square tiles (tile_of; symmetric outputs mirror off-diagonal
// tiles).  TN = 64: 128 x 64 tiles for symmetric outputs, enumerated by
// tile_of_rect_sym; each entry with j >= i is written and, for j > i,
// mirrored, so every entry is written once.  TI, TJ: tile rows, columns.
template <int BTRANS, int TN>
__device__ __forceinline__ void gemm_f64_big_body(GemmArgs p, int TI, int TJ) {
  constexpr int WNC = TN / 2;   // wave tile columns
  constexpr int NCB = WNC / 16;  // 16-column blocks per wave
  const int n = p.n;
  int bi, bj;
  if (TN == FT)
    tile_of(blockIdx.x, TI, p.sym, F_GROUP, bi, bj);
  else
    tile_of_rect_sym(blockIdx.x, TI, TJ, bi, bj);
  const int i0 = bi * FT, j0 = bj * TN;
  // a stage holds the A rows (padded) and the B panel; 128 x 64 tiles need
  // only half the B space, which lets three workgroups share a CU's LDS
  constexpr int STAGE = TN == FT ? FSTAGE : FK * FROW + FK * TN;
  __shared__ double sa[STAGE];
  __shared__ double sb[STAGE];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * WNC;

  d4 acc[4][NCB];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < NCB; ++c) acc[r][c] = d4{0.0, 0.0, 0.0, 0.0};

  const int kt_per = n / FK;
  const int ktiles = kt_per * p.nprod;
  const int nbytes = (int)(8u * (unsigned)n * (unsigned)n);  // buffer range (n <= 23170)

  // Loads.  A (and normal B when TN = 128): wave w loads k rows 4 w .. 4 w + 3,
  // lane -> 16 bytes at column 2 lane of the tile (clamped to n - 2).
  // Normal B when TN = 64: 64-double k rows, two per instruction (wave w:
  // rows 4 w .. 4 w + 3), lane -> row lane / 32 of the pair, physical 16-byte
  // chunk lane % 32, which holds logical chunk (lane % 32) ^ (8 (row & 1)).
  // Transposed B: wave w loads tile rows j = (TN / 4) w .., eight per
  // instruction, lane -> row lane / 8, physical chunk lane % 8.
  int colA = i0 + 2 * lane;
  colA = colA < n ? colA : n - 2;
  int colB = j0 + 2 * lane;
  if (TN == 64) colB = j0 + 2 * ((lane & 31) ^ (8 * ((lane >> 5) & 1)));
  colB = colB < n ? colB : n - 2;
  const int lr = lane >> 3, lpc = lane & 7;
  constexpr int TQ = TN / 32;  // transposed-B load instructions per wave
  unsigned toff[TQ];
#pragma unroll
  for (int q = 0; q < TQ; ++q) {
    int j = j0 + (TN / 4) * wave + 8 * q + lr;
    j = j < n ? j : n - 1;
    // stage row (TN / 4) w + 8 q + lr: logical chunk lpc ^ lr ^ (q & 1) (2 doubles)
    toff[q] = 8u * ((unsigned)j * (unsigned)n + 2u * (unsigned)(lpc ^ lr ^ (q & 1)));
  }
  auto issue = [&](int kt, double *st) {
    const int prod = kt / kt_per;
    const int k0 = (kt - prod * kt_per) * FK;
    const __amdgpu_buffer_rsrc_t ra =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p.A[prod]), (short)0, nbytes, F_BUF_WORD3);
    const __amdgpu_buffer_rsrc_t rb =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p.B[prod]), (short)0, nbytes, F_BUF_WORD3);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = k0 + 4 * wave + q;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (lds_void_t *)&st[(4 * wave + q) * FROW], 16,
                                               8u * ((unsigned)k * (unsigned)n + (unsigned)colA), 0, 0, 0);
    }
    if (!BTRANS && TN == FT) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = k0 + 4 * wave + q;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, (lds_void_t *)&st[(FK + 4 * wave + q) * FROW], 16,
                                                 8u * ((unsigned)k * (unsigned)n + (unsigned)colB), 0, 0, 0);
      }
    } else if (!BTRANS) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int k = k0 + 4 * wave + 2 * q + (lane >> 5);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, (lds_void_t *)&st[FK * FROW + (4 * wave + 2 * q) * 64], 16,
                                                 8u * ((unsigned)k * (unsigned)n + (unsigned)colB), 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int q = 0; q < TQ; ++q)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, (lds_void_t *)&st[FK * FROW + ((TN / 4) * wave + 8 * q) * 16],
                                                 16, toff[q], 8u * (unsigned)k0, 0, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
  };

  const int fl = lane & 15, fk = lane >> 4;
  // fragments of k step kk: A[kk + fk][wm + 16 r + fl], B[kk + fk][wn + 16 c + fl]
  auto frags = [&](const double *st, int kk, double (&a)[4], double (&b)[NCB]) {
#pragma unroll
    for (int r = 0; r < 4; ++r) a[r] = st[(kk + fk) * FROW + wm + 16 * r + fl];
#pragma unroll
    for (int c = 0; c < NCB; ++c) {
      if (!BTRANS && TN == FT) {
        b[c] = st[(FK + kk + fk) * FROW + wn + 16 * c + fl];
      } else if (!BTRANS) {
        const int row = kk + fk, col = wn + 16 * c + fl;
        b[c] = st[FK * FROW + row * 64 + 2 * ((col >> 1) ^ (8 * (row & 1))) + (col & 1)];
      } else {
        const int j = wn + 16 * c + fl, k = kk + fk;
        b[c] = st[FK * FROW + j * 16 + 2 * swz8(j, k >> 1) + (k & 1)];
      }
    }
  };
  auto panel = [&](const double *st) {
    double a[4], b[NCB];
    frags(st, 0, a, b);
#pragma unroll
    for (int kk = 0; kk < FK; kk += 4) {
      double an[4], bn[NCB];
      if (kk + 4 < FK) frags(st, kk + 4, an, bn);
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < NCB; ++c)
          acc[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r], b[c], acc[r][c], 0, 0, 0);
      if (kk + 4 < FK) {
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] = an[q];
#pragma unroll
        for (int q = 0; q < NCB; ++q) b[q] = bn[q];
      }
    }
  };

  // Panel kt + 1 loads into one stage while panel kt is read from the other.
  // At the top of each panel: this wave's loads of panel kt are complete once
  // vmcnt drains (the compiler does not wait for them by itself), and the
  // barrier makes every wave's part visible and frees the stage of panel
  // kt - 1 for the loads of panel kt + 1.
  issue(0, sa);
  for (int kt = 0; kt < ktiles; ++kt) {
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __syncthreads();
    if (kt + 1 < ktiles) issue(kt + 1, (kt & 1) ? sa : sb);
    panel((kt & 1) ? sb : sa);
  }

  const double *C1 = (const double *)p.C1;
  const double *C2 = (const double *)p.C2;
  double *out = (double *)p.out;
  const bool mirror = p.sym && (bi != bj);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
#pragma unroll
    for (int c = 0; c < NCB; ++c) {
      const int j = j0 + wn + c * 16 + fl;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = i0 + wm + r * 16 + fk + 4 * q;
        if (i < n && j < n && (TN == FT || j >= i)) {
          const size_t off = (size_t)i * n + j;
          double x = p.alpha * acc[r][c][q];
          if (C1) x += p.beta1 * C1[off];
          if (C2) x += p.beta2 * C2[off];
          if (i == j) x += p.gamma;
          out[off] = x;
          if (TN == FT ? mirror : j > i) out[(size_t)j * n + i] = x;
        }
      }
    }
  }
}

template <int BTRANS>
__global__ __launch_bounds__(256, 2) void k_gemm_f64_big(GemmArgs p, int TI, int TJ) {
  gemm_f64_big_body<BTRANS, FT>(p, TI, TJ);
}

// the 128 x 64 tiles of symmetric outputs: 52 KB of LDS and 104 VGPRs, so
// three workgroups share a CU and the 729 tiles at n = 3360 run in one round
template <int BTRANS>
__global__ __launch_bounds__(256, 3) void k_gemm_f64_half(GemmArgs p, int TI, int TJ) {
  gemm_f64_big_body<BTRANS, 64>(p, TI, TJ);
}

}  // namespace

void gemm_f64(const GemmArgs &a, hipStream_t s) {
  // the requested family, else the tile table's, else 128-row tiles from
  // n = 1024 on (n % 16 == 0; the buffer range limits n to 23170)
  int fam = a.family != GEMM_AUTO ? a.family : table_family(0, a.sym, a.n);
  if (!family_runs(0, fam, a.n)) fam = GEMM_AUTO;
  if (fam == GEMM_COMPACT) {
    const int Tc = (a.n + CM - 1) / CM;
    hipLaunchKernelGGL(k_gemm_f64_c32, dim3(a.sym ? Tc * (Tc + 1) / 2 : Tc * Tc), dim3(256), 0, s, a, Tc);
    return;
  }
  const bool large = fam == GEMM_AUTO ? (a.n % 16 == 0 && a.n >= 1024 && a.n <= 23170) : fam == GEMM_LARGE;
  if (large) {
    const int TI = (a.n + FT - 1) / FT;
    if (a.sym) {
      // symmetric outputs: 128 x 64 tiles, twice as many for an even load over the CUs
      const int TJ = (a.n + 63) / 64;
      const int blocks = tile_count_rect_sym(TI, TJ);
      if (a.btrans)
        hipLaunchKernelGGL((k_gemm_f64_half<1>), dim3(blocks), dim3(256), 0, s, a, TI, TJ);
      else
        hipLaunchKernelGGL((k_gemm_f64_half<0>), dim3(blocks), dim3(256), 0, s, a, TI, TJ);
    } else {
      const int blocks = tile_count(TI, 0);
      if (a.btrans)
        hipLaunchKernelGGL((k_gemm_f64_big<1>), dim3(blocks), dim3(256), 0, s, a, TI, TI);
      else
        hipLaunchKernelGGL((k_gemm_f64_big<0>), dim3(blocks), dim3(256), 0, s, a, TI, TI);
    }
    return;
  }
  const int T = (a.n + BM - 1) / BM;
  const int blocks = a.sym ? T * (T + 1) / 2 : T * T;
  hipLaunchKernelGGL(k_gemm_f64, dim3(blocks), dim3(256), 0, s, a, T);
}

}  // namespace xl
