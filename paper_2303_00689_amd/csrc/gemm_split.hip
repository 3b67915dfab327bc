// Split-precision MFMA GEMM on FP32 storage for the Fermi-operator and
// response chains.
//
// Every FP32 operand value x is split in registers into low-precision parts,
//   BF16X3: x ~ h + l,           products h*h + h*l + l*h            (3 MFMA)
//   BF16X6: x ~ h + l + l2,      + l*l + h*l2 + l2*h                 (6 MFMA)
//   FP16X3: x ~ h + l / 2^11,    h*h into one accumulator, h*l + l*h into a
//           second one that is scaled by 2^-11 at the end (the scaling keeps
//           the low parts of small entries out of the FP16 subnormal range)
// each part rounded to nearest-even, and the products accumulate in FP32 on
// v_mfma_f32_16x16x32_{bf16,f16}.
//
// Three kernels share these conventions:
//  * k_gemm_split_bf16x3 (BF16x3) and k_gemm_split_lds (BF16x6, FP16x3):
//    128 x 128 tiles, any n with n % 4 == 0;
//  * k_gemm_split_big (n % 32 == 0, large n): 224 x 224 tiles for full
//    outputs, 160 x 160 for symmetric ones (FP16x3: 160 x 160 for both), and
//    k_gemm_split_mid, the same kernel at 128 x 128 tiles and two workgroups
//    per compute unit (n % 4 == 0; FP16x3 n % 32 == 0).
//
// Tile 128 x 128 per workgroup of 256 threads (2 x 2 wavefronts of 64 x 64,
// i.e. 4 x 4 MFMA blocks of 16 x 16 each).  K advances by 32 through
// double-buffered LDS panels.  Both panels are stored k-fastest (row-major
// [m][k] and [n][k]), which is what the MFMA operand layout wants:
//   A (16 x 32): lane l holds A[l % 16][8 (l / 16) .. 8 (l / 16) + 7]
//   B (32 x 16): lane l holds B[8 (l / 16) .. + 7][l % 16]
//   D (16 x 16): lane l holds D[4 (l / 16) + q][l % 16], q = 0..3
// so operand rows are read straight from memory: op(A) = A for the symmetric
// A operands of the chains, and op(B) = B^T, which is B for a symmetric B and
// the requested transpose when btrans = 1.
#include "common.h"
#include "tile_map.h"

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <utility>

namespace xl {
namespace {

constexpr int TILE_GROUP = 4;  // tile rows per L2-sharing group

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));

constexpr int TM = 128;
constexpr int TK = 32;
constexpr int PITCH = TK + 8;  // 16-bit elements per LDS row (padding breaks bank aliasing)

template <int MODE>
struct Parts {
  static constexpr int P = (MODE == 1) ? 3 : 2;
};

__device__ inline unsigned short bf16_bits(float x) {
  __bf16 b = (__bf16)x;  // round to nearest even
  return __builtin_bit_cast(unsigned short, b);
}
__device__ inline float bf16_val(unsigned short u) {
  return __builtin_bit_cast(float, (unsigned)u << 16);
}
__device__ inline unsigned short f16_bits(float x) {
  _Float16 h = (_Float16)x;
  return __builtin_bit_cast(unsigned short, h);
}
__device__ inline float f16_val(unsigned short u) {
  return (float)__builtin_bit_cast(_Float16, u);
}

template <int MODE>
__device__ inline void split(float x, unsigned short *out) {
  if (MODE == 2) {
    const unsigned short h = f16_bits(x);
    out[0] = h;
    out[1] = f16_bits((x - f16_val(h)) * 2048.0f);
  } else {
    const unsigned short h = bf16_bits(x);
    const float r = x - bf16_val(h);
    const unsigned short l = bf16_bits(r);
    out[0] = h;
    out[1] = l;
    if (MODE == 1) out[2] = bf16_bits(r - bf16_val(l));
  }
}

__device__ inline f4 mfma(us8 a, us8 b, f4 c, bool f16) {
  if (f16)
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a), __builtin_bit_cast(h8, b), c, 0,
                                                  0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0,
                                                 0, 0);
}

// STAGES = 2 keeps the raw rows of two panels in registers (see below); it is
// used where the register budget still allows two waves per SIMD.
template <int MODE, int STAGES>
__device__ __forceinline__ void gemm_split_body(GemmArgs p, int T) {
  constexpr int P = Parts<MODE>::P;
  constexpr bool F16 = (MODE == 2);
  const int n = p.n;
  int bi, bj;
  tile_of(blockIdx.x, T, p.sym, TILE_GROUP, bi, bj);
  const int i0 = bi * TM, j0 = bj * TM;
  // [buffer][part][row][k]
  __shared__ unsigned short As[2][P][TM][PITCH];
  __shared__ unsigned short Bs[2][P][TM][PITCH];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;

  f4 acc[4][4];
  f4 acc2[F16 ? 4 : 1][F16 ? 4 : 1];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = f4{0.f, 0.f, 0.f, 0.f};
  if (F16) {
#pragma unroll
    for (int r = 0; r < (F16 ? 4 : 1); ++r)
#pragma unroll
      for (int c = 0; c < (F16 ? 4 : 1); ++c) acc2[r][c] = f4{0.f, 0.f, 0.f, 0.f};
  }

  const int kt_per = (n + TK - 1) / TK;
  const int ktiles = kt_per * p.nprod;
  // loader: 128 rows x 32 floats per operand; thread -> row tid / 2, 16 floats at 16 * (tid % 2)
  const int lrow = tid >> 1, lk = (tid & 1) * 16;
  // Two register stages: the raw rows of panel kt + 2 are loaded while panel
  // kt feeds the MFMAs and panel kt + 1 is split into LDS, so every global
  // load has about two panels of MFMA work to arrive.  The zeroing select and
  // the split happen in store(), after the loads of the later panel have been
  // issued.
  struct Stage {
    f4 xa[4], xb[4];
    bool vla, vlb, vk[4];
  };
  Stage s0, s1;
  (void)s1;

  // Loads are unconditional (clamped in-bounds addresses), so no branch
  // separates them and the compiler can keep all of them in flight.
  auto load = [&](int kt, Stage &st) {
    const int prod = kt / kt_per;
    const int k0 = (kt - prod * kt_per) * TK + lk;
    const float *A = (const float *)p.A[prod];
    const float *B = (const float *)p.B[prod];
    const int ia = i0 + lrow, jb = j0 + lrow;
    st.vla = ia < n;
    st.vlb = jb < n;
    const size_t ra_off = (size_t)(st.vla ? ia : n - 1) * n;
    const size_t rb_off = (size_t)(st.vlb ? jb : n - 1) * n;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k = k0 + 4 * v;
      st.vk[v] = k < n;
      const int kc = st.vk[v] ? k : n - 4;
      st.xa[v] = *(const f4 *)(A + ra_off + kc);
      st.xb[v] = *(const f4 *)(B + rb_off + kc);
    }
  };
  auto store = [&](int buf, const Stage &st) {
    // eight values at a time: select, split, one 16-byte LDS write per part
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      unsigned short pa[P][8], pb[P][8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int v = 2 * h + e / 4, q4 = e % 4;
        const float fa = (st.vla && st.vk[v]) ? st.xa[v][q4] : 0.0f;
        const float fb = (st.vlb && st.vk[v]) ? st.xb[v][q4] : 0.0f;
        unsigned short t[3];
        split<MODE>(fa, t);
#pragma unroll
        for (int q = 0; q < P; ++q) pa[q][e] = t[q];
        split<MODE>(fb, t);
#pragma unroll
        for (int q = 0; q < P; ++q) pb[q][e] = t[q];
      }
#pragma unroll
      for (int q = 0; q < P; ++q) {
        *(us8 *)&As[buf][q][lrow][lk + 8 * h] =
            us8{pa[q][0], pa[q][1], pa[q][2], pa[q][3], pa[q][4], pa[q][5], pa[q][6], pa[q][7]};
        *(us8 *)&Bs[buf][q][lrow][lk + 8 * h] =
            us8{pb[q][0], pb[q][1], pb[q][2], pb[q][3], pb[q][4], pb[q][5], pb[q][6], pb[q][7]};
      }
    }
  };
  const int fr = lane & 15, fk = 8 * (lane >> 4);
  auto compute = [&](int buf) {
    // B fragments for the four column blocks, then one row block of A at a time
    us8 b[P][4];
#pragma unroll
    for (int q = 0; q < P; ++q)
#pragma unroll
      for (int c = 0; c < 4; ++c) b[q][c] = *(const us8 *)&Bs[buf][q][wn + 16 * c + fr][fk];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      us8 a[P];
#pragma unroll
      for (int q = 0; q < P; ++q) a[q] = *(const us8 *)&As[buf][q][wm + 16 * r + fr][fk];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (MODE == 2) {
          acc[r][c] = mfma(a[0], b[0][c], acc[r][c], true);
          acc2[r][c] = mfma(a[0], b[1][c], acc2[r][c], true);
          acc2[r][c] = mfma(a[1], b[0][c], acc2[r][c], true);
        } else {
          // small terms first
          if (MODE == 1) {
            acc[r][c] = mfma(a[1], b[1][c], acc[r][c], false);
            acc[r][c] = mfma(a[0], b[2][c], acc[r][c], false);
            acc[r][c] = mfma(a[2], b[0][c], acc[r][c], false);
          }
          acc[r][c] = mfma(a[0], b[1][c], acc[r][c], false);
          acc[r][c] = mfma(a[1], b[0][c], acc[r][c], false);
          acc[r][c] = mfma(a[0], b[0][c], acc[r][c], false);
        }
      }
    }
  };

  if constexpr (STAGES == 2) {
    load(0, s0);
    if (ktiles > 1) load(1, s1);
    store(0, s0);
    __syncthreads();
    for (int kt = 0; kt < ktiles; kt += 2) {
      // panel kt from buffer 0; stage 0 is free again
      if (kt + 2 < ktiles) load(kt + 2, s0);
      compute(0);
      if (kt + 1 < ktiles) store(1, s1);
      __syncthreads();
      if (kt + 1 >= ktiles) break;
      // panel kt + 1 from buffer 1; stage 1 is free again
      if (kt + 3 < ktiles) load(kt + 3, s1);
      compute(1);
      if (kt + 2 < ktiles) store(0, s0);
      __syncthreads();
    }
  } else {
    load(0, s0);
    store(0, s0);
    __syncthreads();
    for (int kt = 0; kt < ktiles; ++kt) {
      const int buf = kt & 1;
      if (kt + 1 < ktiles) load(kt + 1, s0);
      compute(buf);
      if (kt + 1 < ktiles) store(buf ^ 1, s0);
      __syncthreads();
    }
  }

  const float *C1 = (const float *)p.C1;
  const float *C2 = (const float *)p.C2;
  float *out = (float *)p.out;
  const bool mirror = p.sym && (bi != bj);
  const float alpha = (float)p.alpha, b1 = (float)p.beta1, b2 = (float)p.beta2, gam = (float)p.gamma;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = j0 + wn + 16 * c + fr;
      const int ib = i0 + wm + 16 * r + 4 * (lane >> 4);
      float v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = ib + q;
        float accv = acc[r][c][q];
        if (MODE == 2) accv += acc2[r][c][q] * (1.0f / 2048.0f);
        float x = alpha * accv;
        if (i < n && j < n) {
          const size_t off = (size_t)i * n + j;
          if (C1) x += b1 * C1[off];
          if (C2) x += b2 * C2[off];
          if (i == j) x += gam;
          out[off] = x;
        }
        v[q] = x;
      }
      if (mirror && j < n && ib < n) {
        // four consecutive rows -> four consecutive columns of row j (ib % 4 == 0, n % 4 == 0)
        *(f4 *)(out + (size_t)j * n + ib) = f4{v[0], v[1], v[2], v[3]};
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Split GEMM with direct-to-LDS operand panels (gfx950 global_load_lds).
//
// The FP32 panels (128 rows x 32 k of A and of B) stream into LDS without
// passing through registers, two stages deep, so the loads of panel kt + 1
// are in flight while panel kt feeds the MFMAs.  Every wave splits the FP32
// values of its own fragments into BF16/FP16 parts right before the MFMAs.
// Within an LDS row (eight 16-byte chunks) chunk kc sits at position
// kc ^ (r & 7) ^ ((r >> 3) & 1), which puts the 16 rows a fragment read
// touches on distinct bank groups.  A direct load writes lane i's 16 bytes at
// (wave-uniform base) + 16 i, so each load instruction fills eight rows.
typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) const void gbl_void_t;

constexpr int LROW = 32;                 // floats per LDS row (one k panel)
constexpr int LSTAGE = 2 * TM * LROW;     // floats per stage (A then B)

__device__ inline int swz(int r, int kc) { return kc ^ (r & 7) ^ ((r >> 3) & 1); }

template <int MODE>
__device__ inline void split8(const float (&x)[8], us8 (&o)[3]) {
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    unsigned short t[3];
    split<MODE>(x[v], t);
    o[0][v] = t[0];
    o[1][v] = t[1];
    if (MODE == 1) o[2][v] = t[2];
  }
}

template <int MODE>
__device__ __forceinline__ void gemm_split_lds_body(GemmArgs p, int T) {
  constexpr int P = Parts<MODE>::P;
  constexpr bool F16 = (MODE == 2);
  const int n = p.n;
  int bi, bj;
  tile_of(blockIdx.x, T, p.sym, TILE_GROUP, bi, bj);
  const int i0 = bi * TM, j0 = bj * TM;
  __shared__ float stage[2][LSTAGE];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;          // waves 0..3 compute, wave 4 loads
  const bool producer = wave == 4;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;

  f4 acc[4][4];
  f4 acc2[F16 ? 4 : 1][F16 ? 4 : 1];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = f4{0.f, 0.f, 0.f, 0.f};
  if (F16) {
#pragma unroll
    for (int r = 0; r < (F16 ? 4 : 1); ++r)
#pragma unroll
      for (int c = 0; c < (F16 ? 4 : 1); ++c) acc2[r][c] = f4{0.f, 0.f, 0.f, 0.f};
  }

  const int kt_per = (n + TK - 1) / TK;
  const int ktiles = kt_per * p.nprod;
  const bool edge_rows = (i0 + TM > n) || (j0 + TM > n);

  // producer: 16 load instructions per operand fill the 128 rows of a panel;
  // lane -> row 8 j + lane / 8, physical chunk lane % 8
  const int lr = lane >> 3, lpc = lane & 7;
  auto issue = [&](int kt, int st) {
    const int prod = kt / kt_per;
    const int k0 = (kt - prod * kt_per) * TK;
    const float *A = (const float *)p.A[prod];
    const float *B = (const float *)p.B[prod];
#pragma unroll 4
    for (int j = 0; j < TM / 8; ++j) {
      const int r = 8 * j + lr;
      const int kc = swz(r, lpc);
      int k = k0 + 4 * kc;
      k = k < n ? k : n - 4;
      const int ia = i0 + r < n ? i0 + r : n - 1;
      const int jb = j0 + r < n ? j0 + r : n - 1;
      __builtin_amdgcn_global_load_lds((gbl_void_t *)(A + (size_t)ia * n + k),
                                       (lds_void_t *)&stage[st][8 * j * LROW], 16, 0, 0);
      __builtin_amdgcn_global_load_lds((gbl_void_t *)(B + (size_t)jb * n + k),
                                       (lds_void_t *)&stage[st][TM * LROW + 8 * j * LROW], 16, 0, 0);
    }
  };

  const int fr = lane & 15, fq = lane >> 4;  // fragment row, k group (8 values)
  // eight FP32 values row r, k 8 fq .. 8 fq + 7 of a stage operand, zeroed
  // outside the matrix on edge tiles and on a partial last k panel
  auto fetch = [&](const float *base, int r, int rlim, int klim, bool edge, float (&x)[8]) {
    const f4 lo = *(const f4 *)(base + r * LROW + 4 * swz(r, 2 * fq));
    const f4 hi = *(const f4 *)(base + r * LROW + 4 * swz(r, 2 * fq + 1));
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      x[v] = lo[v];
      x[4 + v] = hi[v];
    }
    if (edge) {
      const bool rv = r < rlim;
      const bool k0v = 8 * fq < klim, k1v = 8 * fq + 4 < klim;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        x[v] = (rv && k0v) ? x[v] : 0.0f;
        x[4 + v] = (rv && k1v) ? x[4 + v] : 0.0f;
      }
    }
  };
  auto compute = [&](int st, int kt) {
    const int prod = kt / kt_per;
    const int k0 = (kt - prod * kt_per) * TK;
    const int klim = n - k0;  // valid k of this panel: [0, klim)
    const bool edge = edge_rows || klim < TK;
    const float *sa = &stage[st][0];
    const float *sb = &stage[st][TM * LROW];
    us8 b[4][3];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      float x[8];
      fetch(sb, wn + 16 * c + fr, n - j0, klim, edge, x);
      split8<MODE>(x, b[c]);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float x[8];
      us8 a[3];
      fetch(sa, wm + 16 * r + fr, n - i0, klim, edge, x);
      split8<MODE>(x, a);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (MODE == 2) {
          acc[r][c] = mfma(a[0], b[c][0], acc[r][c], true);
          acc2[r][c] = mfma(a[0], b[c][1], acc2[r][c], true);
          acc2[r][c] = mfma(a[1], b[c][0], acc2[r][c], true);
        } else {
          if (MODE == 1) {
            acc[r][c] = mfma(a[1], b[c][1], acc[r][c], false);
            acc[r][c] = mfma(a[0], b[c][2], acc[r][c], false);
            acc[r][c] = mfma(a[2], b[c][0], acc[r][c], false);
          }
          acc[r][c] = mfma(a[0], b[c][1], acc[r][c], false);
          acc[r][c] = mfma(a[1], b[c][0], acc[r][c], false);
          acc[r][c] = mfma(a[0], b[c][0], acc[r][c], false);
        }
      }
    }
  };

  // The producer wave loads panel kt + 1 into the other stage (and waits for
  // its own loads) while the four compute waves work on panel kt; the one
  // barrier per panel hands the stages over.  Only the producer ever has
  // loads in flight, so no wait for them lands in the compute waves.
  if (producer) {
    issue(0, 0);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
  }
  __syncthreads();
  for (int kt = 0; kt < ktiles; ++kt) {
    if (producer) {
      if (kt + 1 < ktiles) issue(kt + 1, (kt + 1) & 1);
      __builtin_amdgcn_s_waitcnt(0x0F70);
    } else {
      compute(kt & 1, kt);
    }
    __syncthreads();
  }
  if (producer) return;

  const float *C1 = (const float *)p.C1;
  const float *C2 = (const float *)p.C2;
  float *out = (float *)p.out;
  const bool mirror = p.sym && (bi != bj);
  const float alpha = (float)p.alpha, b1 = (float)p.beta1, b2 = (float)p.beta2, gam = (float)p.gamma;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = j0 + wn + 16 * c + fr;
      const int ib = i0 + wm + 16 * r + 4 * (lane >> 4);
      float v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = ib + q;
        float accv = acc[r][c][q];
        if (MODE == 2) accv += acc2[r][c][q] * (1.0f / 2048.0f);
        float x = alpha * accv;
        if (i < n && j < n) {
          const size_t off = (size_t)i * n + j;
          if (C1) x += b1 * C1[off];
          if (C2) x += b2 * C2[off];
          if (i == j) x += gam;
          out[off] = x;
        }
        v[q] = x;
      }
      if (mirror && j < n && ib < n) *(f4 *)(out + (size_t)j * n + ib) = f4{v[0], v[1], v[2], v[3]};
    }
  }
}

template <int MODE>
__global__ __launch_bounds__(320) void k_gemm_split_lds(GemmArgs p, int T) {
  gemm_split_lds_body<MODE>(p, T);
}

// ---------------------------------------------------------------------------
// Large-tile split GEMM (BF16 splits, n % 32 == 0): 2 x 2 waves of BNB x BNB
// MFMA blocks of 16, one workgroup per compute unit.  BNB = 7 gives 224 x 224
// tiles (full outputs: 225 tiles at the 3360 orbitals of the 840-atom
// cluster), BNB = 5 gives 160 x 160 tiles (symmetric outputs: 231 upper
// tiles there), so either fills the 256 compute units in one round.
//
// The larger wave tiles cut the bytes moved per MFMA against 64 x 64 waves.
// Each wave loads its own A rows straight from global memory into registers
// (the two waves sharing them both load them: L2 hits), and the four waves
// stream the B panels (B rows x 32 k) into LDS with buffer loads, 3 or 4
// stages deep, so LDS carries only B.  Every fragment of the next k panel is
// loaded under the MFMAs of the current one.  Each wave splits its fragments
// into BF16 parts on read.
// BF16 parts of eight FP32 values, two at a time: v_cvt_pk_bf16_f32 rounds a
// pair to nearest even, and each rounded part goes back to FP32 by a shift
// or a mask of its half of the packed word.
typedef float f2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
__device__ inline unsigned cvt_pk_bf16(float a, float b) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector((f2){a, b}, bf2));
}
// FP16 parts of a pair, rounded to nearest even
typedef _Float16 h2v __attribute__((ext_vector_type(2)));
__device__ inline unsigned cvt_pk_f16(float a, float b) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector((f2){a, b}, h2v));
}
template <int MODE>
__device__ inline void split8_pk(const float (&x)[8], us8 (&o)[3]) {
  typedef unsigned u4 __attribute__((ext_vector_type(4)));
  u4 h, l, l2;
  if (MODE == 2) {
    // FP16 parts, the low part scaled by 2^11 (out of the subnormal range)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float a = x[2 * v], b = x[2 * v + 1];
      const unsigned hp = cvt_pk_f16(a, b);
      const h2v hv = __builtin_bit_cast(h2v, hp);
      h[v] = hp;
      l[v] = cvt_pk_f16((a - (float)hv[0]) * 2048.0f, (b - (float)hv[1]) * 2048.0f);
    }
    o[0] = __builtin_bit_cast(us8, h);
    o[1] = __builtin_bit_cast(us8, l);
    return;
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const float a = x[2 * v], b = x[2 * v + 1];
    const unsigned hp = cvt_pk_bf16(a, b);
    const float ra = a - __builtin_bit_cast(float, hp << 16);
    const float rb = b - __builtin_bit_cast(float, hp & 0xffff0000u);
    const unsigned lp = cvt_pk_bf16(ra, rb);
    h[v] = hp;
    l[v] = lp;
    if (MODE == 1) {
      const float sa = ra - __builtin_bit_cast(float, lp << 16);
      const float sb = rb - __builtin_bit_cast(float, lp & 0xffff0000u);
      l2[v] = cvt_pk_bf16(sa, sb);
    }
  }
  o[0] = __builtin_bit_cast(us8, h);
  o[1] = __builtin_bit_cast(us8, l);
  if (MODE == 1) o[2] = __builtin_bit_cast(us8, l2);
}

constexpr int BIG_GROUP = 3;          // tile rows per L2-sharing group
constexpr int BUF_DWORD3 = 0x00020000;  // raw buffer descriptor word 3 (32-bit data format)

template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
// f(std::integral_constant<int, i>) for i = 0 .. N - 1, each i a compile-time constant
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// BNB MFMA blocks of 16 per wave tile edge: 7 (224-row tiles), 5 (160) or 4
// (128); STAGES k panels of B in LDS.  RAGGED: n % 32 != 0 (n % 4 == 0), the
// last k panel runs past n: its A values there are zeroed after loads from a
// valid address (the row's first column), so every load is still issued and
// the counted waits below stay exact, and B's values there (the next row's,
// or zeros past the buffer's range) multiply those zeros.
template <int MODE, int BNB, int STAGES, bool RAGGED = false>
__device__ __forceinline__ void gemm_split_big_body(GemmArgs p, int T) {
  // every split; FP16x3 keeps its scaled cross terms in a second accumulator,
  // which fits the 160- and 128-row tiles, not the 224-row ones
  static_assert(MODE >= 0 && MODE <= 2, "split mode");
  static_assert(MODE != 2 || BNB <= 5, "FP16x3: the second accumulator needs BNB <= 5");
  static_assert(STAGES >= 2 && STAGES <= 4, "2 to 4 LDS stages");
  constexpr int BW = 16 * BNB;           // wave tile edge
  constexpr int BT = 2 * BW;             // tile edge
  constexpr int BSTAGE = BT * LROW;      // floats per stage: BT rows of B x 32 k
  constexpr int LPW = BT / 32;           // load instructions per wave per panel (8 rows each)
  const int n = p.n;
  int bi, bj;
  tile_of(blockIdx.x, T, p.sym, BIG_GROUP, bi, bj);
  const int i0 = bi * BT, j0 = bj * BT;
  __shared__ float stg[STAGES][BSTAGE];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  const int wm = (wave >> 1) * BW, wn = (wave & 1) * BW;
  const int fr = lane & 15, fq = lane >> 4;  // fragment row, k group (8 values)

  // FP16x3: the cross terms h l + l h, scaled by 2^11, accumulate in acc2
  constexpr int NB2 = MODE == 2 ? BNB : 1;
  f4 acc[BNB][BNB], acc2[NB2][NB2];
#pragma unroll
  for (int r = 0; r < BNB; ++r)
#pragma unroll
    for (int c = 0; c < BNB; ++c) acc[r][c] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int r = 0; r < NB2; ++r)
#pragma unroll
    for (int c = 0; c < NB2; ++c) acc2[r][c] = f4{0.f, 0.f, 0.f, 0.f};

  // Unless RAGGED, n is a multiple of 32 and every k panel is full.  Rows
  // past n are read clamped to row n - 1: they only reach output rows and
  // columns past n, which are not stored.
  const int kt_per = RAGGED ? (n + TK - 1) / TK : n / TK;
  const int ktiles = kt_per * p.nprod;

  // B panels: buffer loads to LDS, the BT rows x 32 k of a panel shared by the
  // four waves (BT / 4 rows each, eight per instruction; lane -> row lane / 8,
  // physical chunk lane % 8 holding logical chunk swz(row, lane % 8)).  The
  // lane's byte offset of each load row is computed once (n^2 FP32 values fit
  // in 32 bits for n <= 32767) and the k panel is the scalar offset.
  const int lr = lane >> 3, lpc = lane & 7;
  unsigned roff[LPW];
#pragma unroll
  for (int j = 0; j < LPW; ++j) {
    const int R = wave * (BT / 4) + 8 * j + lr;  // stage row
    int g = j0 + R;
    g = g < n ? g : n - 1;
    roff[j] = 4u * ((unsigned)g * (unsigned)n + 4u * (unsigned)swz(R, lpc));
  }
  const int nbytes = (int)(4u * (unsigned)n * (unsigned)n);  // buffer range (n <= 32767)
  auto issueB = [&](int kt, float *st) {
    const int prod = kt / kt_per;
    const unsigned kb = 4u * (unsigned)((kt - prod * kt_per) * TK);
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p.B[prod]), (short)0, nbytes, BUF_DWORD3);
#pragma unroll
    for (int j = 0; j < LPW; ++j)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void_t *)&st[(wave * (BT / 4) + 8 * j) * LROW], 16,
                                               roff[j], kb, 0, 0);
  };
  // A fragments straight from global memory into registers: row block r of
  // this lane is row i0 + wm + 16 r + fr, k values 8 fq .. 8 fq + 7 of the panel
  unsigned aoff[BNB];
#pragma unroll
  for (int r = 0; r < BNB; ++r) {
    int g = i0 + wm + 16 * r + fr;
    g = g < n ? g : n - 1;
    aoff[r] = 4u * ((unsigned)g * (unsigned)n + 8u * (unsigned)fq);
  }
  auto loadA = [&](int kt, int r, float (&x)[8]) {
    const int prod = kt / kt_per;
    const char *base = (const char *)p.A[prod] + aoff[r] + 4 * (kt - prod * kt_per) * TK;
    if (RAGGED) {
      // k of this lane's first value; n % 4 == 0, so each group of four is
      // wholly below n or wholly past it
      const int kl = (kt - prod * kt_per) * TK + 8 * fq;
      const bool okl = kl < n, okh = kl + 4 < n;
      const char *row0 = (const char *)p.A[prod] + (aoff[r] - 32u * (unsigned)fq);
      const f4 lo = *(const f4 *)(okl ? base : row0);
      const f4 hi = *(const f4 *)(okh ? base + 16 : row0);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        x[v] = okl ? lo[v] : 0.f;
        x[4 + v] = okh ? hi[v] : 0.f;
      }
    } else {
      const f4 lo = *(const f4 *)base;
      const f4 hi = *(const f4 *)(base + 16);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        x[v] = lo[v];
        x[4 + v] = hi[v];
      }
    }
  };
  // eight FP32 values of B stage row r, k 8 fq .. 8 fq + 7 of panel kt
  // (RAGGED: zero past n, whatever the stage holds there)
  auto fetch = [&](const float *st, int r, float (&x)[8], int kt) {
    const f4 lo = *(const f4 *)(st + r * LROW + 4 * swz(r, 2 * fq));
    const f4 hi = *(const f4 *)(st + r * LROW + 4 * swz(r, 2 * fq + 1));
    bool okl = true, okh = true;
    if (RAGGED) {
      const int kl = (kt % kt_per) * TK + 8 * fq;
      okl = kl < n;
      okh = kl + 4 < n;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      x[v] = okl ? lo[v] : 0.f;
      x[4 + v] = okh ? hi[v] : 0.f;
    }
  };
  // the product terms of row block r and column block c, small terms first
  auto mma = [&](int r, int c, const us8 (&a)[3], const us8 (&bc)[3]) {
    if (MODE == 2) {
      acc[r][c] = mfma(a[0], bc[0], acc[r][c], true);
      acc2[r % NB2][c % NB2] = mfma(a[0], bc[1], acc2[r % NB2][c % NB2], true);
      acc2[r % NB2][c % NB2] = mfma(a[1], bc[0], acc2[r % NB2][c % NB2], true);
      return;
    }
    if (MODE == 1) {
      acc[r][c] = mfma(a[1], bc[1], acc[r][c], false);
      acc[r][c] = mfma(a[0], bc[2], acc[r][c], false);
      acc[r][c] = mfma(a[2], bc[0], acc[r][c], false);
    }
    acc[r][c] = mfma(a[0], bc[1], acc[r][c], false);
    acc[r][c] = mfma(a[1], bc[0], acc[r][c], false);
    acc[r][c] = mfma(a[0], bc[0], acc[r][c], false);
  };
  constexpr int TERMS = (MODE == 1) ? 6 : 3;
  constexpr int RM = BNB * TERMS;                    // MFMAs per row block
  constexpr int SPLIT_VALU = MODE == 1 ? 44 : (MODE == 2 ? 32 : 24);  // VALU instructions of one split8_pk

  // Software pipeline over k panels, a full panel ahead: panel p of B lives
  // in stage p % STAGES, and while panel k is multiplied from registers, the
  // next panel's A fragments come from global memory and its B fragments from
  // LDS, and panel k + STAGES streams into the stage panel k has left.
  // Registers: raw A of a panel (block r is refilled with the next panel's
  // block r once split), split A of the row block being multiplied (a) and of
  // the next one (an), split B of the current panel (b) and of the next (bn),
  // raw B blocks of the next panel (xb).  Per row block the next panel's loads
  // go first, then the block's MFMAs interleaved with the splits of fragments
  // loaded at least one row block earlier.  Per accumulator the MFMA sequence
  // over k is fixed, so the result does not depend on this schedule.
  float xa[BNB][8], xb[BNB][8];
  us8 b[BNB][3], bn[BNB][3], a[3];
#pragma unroll
  for (int s0 = 0; s0 < STAGES; ++s0)
    if (s0 < ktiles) issueB(s0, stg[s0]);
#pragma unroll
  for (int r = 0; r < BNB; ++r) loadA(0, r, xa[r]);
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): every prologue load has landed
  __syncthreads();
#pragma unroll
  for (int c = 0; c < BNB; ++c) {
    float x[8];
    fetch(stg[0], wn + 16 * c + fr, x, 0);
    split8_pk<MODE>(x, b[c]);
  }
  split8_pk<MODE>(xa[0], a);
  // every read of stage 0 is done before any wave loads into it (the compiler
  // does not wait for buffer loads to LDS or count them at barriers)
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
  __syncthreads();
  for (int kt = 0; kt < ktiles; ++kt) {
    float *nxt = stg[(kt + 1) % STAGES];  // panel kt + 1, landed
    const bool steady = kt + STAGES < ktiles;
    if (steady) issueB(kt + STAGES, stg[kt % STAGES]);
    // the next panel's A (the last panel reloads itself: in bounds, unused)
    const int ka = kt + 1 < ktiles ? kt + 1 : kt;
    __builtin_amdgcn_sched_barrier(0);
    static_for<BNB>([&](auto rc) {
      constexpr int r = decltype(rc)::value;
      // the next panel's A block r and B block r + 1 (B blocks 0 and 1 in row
      // block 0); the last panel reads a stage not loaded again (in bounds,
      // values unused), so that no branch separates the reads from their uses
      constexpr int nreads = (r == 0 ? 2 : 0) + (r + 1 < BNB ? 2 : 0);
      loadA(ka, r, xa[r]);
      if (r == 0) fetch(nxt, wn + fr, xb[0], kt + 1);
      if (r + 1 < BNB) fetch(nxt, wn + 16 * (r + 1) + fr, xb[r + 1 < BNB ? r + 1 : 0], kt + 1);
      // splits under this row block's MFMAs: the A block multiplied next (the
      // next panel's block 0 in the last row block) and the B block(s) loaded
      // at least one row block earlier
      us8 an[3];
      split8_pk<MODE>(r + 1 < BNB ? xa[r + 1 < BNB ? r + 1 : 0] : xa[0], an);
      constexpr int nsplit = 1 + (r >= 1 ? 1 : 0) + (r == BNB - 1 ? 1 : 0);
      if (r >= 1) split8_pk<MODE>(xb[r >= 1 ? r - 1 : 0], bn[r >= 1 ? r - 1 : 0]);
      if (r == BNB - 1) split8_pk<MODE>(xb[BNB - 1], bn[BNB - 1]);
#pragma unroll
      for (int c = 0; c < BNB; ++c) mma(r, c, a, b[c]);
      constexpr int per = (nsplit * SPLIT_VALU + RM - 1) / RM;
      __builtin_amdgcn_sched_group_barrier(0x020, 2, 0);                    // VMEM read
      if (nreads) __builtin_amdgcn_sched_group_barrier(0x100, nreads, 0);  // DS read
#pragma unroll
      for (int q = 0; q < RM; ++q) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);    // MFMA
        __builtin_amdgcn_sched_group_barrier(0x002, per, 0);  // VALU
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int q = 0; q < 3; ++q) a[q] = an[q];
    });
#pragma unroll
    for (int c = 0; c < BNB; ++c)
#pragma unroll
      for (int q = 0; q < 3; ++q) b[c][q] = bn[c][q];
    // Panel kt + 2 must have landed before the next iteration reads it, and
    // every read of panel kt + 1 must be done before its stage is reloaded.
    // Loads complete in issue order: B(kt + 2) was issued at iteration
    // kt + 2 - STAGES (earlier ones in the prologue, which waited for all),
    // and after it came 2 BNB A loads per iteration and LPW B loads per later
    // iteration.  Near the end, with fewer B loads after it, the wait keeps
    // only this iteration's A loads in flight.
    constexpr int NA = 2 * BNB + (STAGES - 2) * (LPW + 2 * BNB);
    constexpr int NE = 2 * BNB;
    static_assert(NA < 64, "vmcnt holds 6 bits");
    if (steady)
      __builtin_amdgcn_s_waitcnt((NA & 15) | ((NA >> 4) << 14) | 0x0070);  // vmcnt(NA) lgkmcnt(0)
    else
      __builtin_amdgcn_s_waitcnt((NE & 15) | ((NE >> 4) << 14) | 0x0070);  // vmcnt(NE) lgkmcnt(0)
    __syncthreads();
  }

  const float *C1 = (const float *)p.C1;
  const float *C2 = (const float *)p.C2;
  float *out = (float *)p.out;
  const bool mirror = p.sym && (bi != bj);
  const float alpha = (float)p.alpha, b1 = (float)p.beta1, b2 = (float)p.beta2, gam = (float)p.gamma;
#pragma unroll
  for (int r = 0; r < BNB; ++r) {
#pragma unroll
    for (int c = 0; c < BNB; ++c) {
      const int j = j0 + wn + 16 * c + fr;
      const int ib = i0 + wm + 16 * r + 4 * fq;
      float v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = ib + q;
        const float a = MODE == 2 ? acc[r][c][q] + acc2[r % NB2][c % NB2][q] * (1.0f / 2048.0f) : acc[r][c][q];
        float x = alpha * a;
        if (i < n && j < n) {
          const size_t off = (size_t)i * n + j;
          if (C1) x += b1 * C1[off];
          if (C2) x += b2 * C2[off];
          if (i == j) x += gam;
          out[off] = x;
        }
        v[q] = x;
      }
      if (mirror && j < n && ib < n) *(f4 *)(out + (size_t)j * n + ib) = f4{v[0], v[1], v[2], v[3]};
    }
  }
}

// 224-row tiles (BNB = 7) keep four B stages in LDS (115 KB), 160-row tiles three (61 KB)
template <int MODE, int BNB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_gemm_split_big(GemmArgs p,
                                                                                                   int T) {
  gemm_split_big_body<MODE, BNB, BNB == 7 ? 4 : 3>(p, T);
}
// 128-row tiles (BNB = 4): three B stages (49 KB) and at most 256 registers,
// so two workgroups share a compute unit and a second wave per SIMD hides
// the first one's memory waits
template <int MODE, bool RAGGED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_gemm_split_mid(GemmArgs p,
                                                                                                  int T) {
  gemm_split_big_body<MODE, 4, 3, RAGGED>(p, T);
}
// 64-row tiles (BNB = 2) for small orders: 24 KB of LDS and few registers,
// so several workgroups share a compute unit
template <int MODE, bool RAGGED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_gemm_split_compact(GemmArgs p,
                                                                                                   int T) {
  gemm_split_big_body<MODE, 2, 3, RAGGED>(p, T);
}

// BF16x3, the response-chain mode of the mixed-precision step: two register
// stages at two waves per SIMD
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_gemm_split_bf16x3(GemmArgs p,
                                                                                                  int T) {
  gemm_split_body<0, 2>(p, T);
}

}  // namespace

// whether gemm_split runs the large-tile kernel for this product (the rule below)
static bool split_runs_large(int prec, int sym, int n) {
  const int edge = sym || prec == 3 ? 160 : 224;
  const int T = (n + edge - 1) / edge;
  int fam = table_family(prec, sym, n);
  if (!family_runs(prec, fam, n)) fam = GEMM_AUTO;
  if (fam == GEMM_AUTO) return family_runs(prec, GEMM_LARGE, n) && tile_count(T, sym) >= 192;
  return fam == GEMM_LARGE;
}

bool split_sum_by_transpose(int prec, int n) {
  if (prec != 1 && prec != 2) return false;
  const int T = (n + 223) / 224;
  return T * T <= 256 && split_runs_large(prec, 0, n) && split_runs_large(prec, 1, n);
}

void gemm_split(const GemmArgs &a, int prec, hipStream_t s) {
  // large tiles (224 rows for full outputs, 160 for symmetric ones) need
  // n % 32 == 0 and pay once they give at least 3/4 of a workgroup per
  // compute unit (192 of the 256); below that the 128-row tiles fill the chip
  // better
  // the requested family, else the tile table's, else the rule above
  // FP16x3 takes 160-row tiles for full outputs too (its second accumulator)
  const int edge = a.sym || prec == 3 ? 160 : 224;
  const int T = (a.n + edge - 1) / edge;
  const int blocks = tile_count(T, a.sym);
  int fam = a.family != GEMM_AUTO ? a.family : table_family(prec, a.sym, a.n);
  if (!family_runs(prec, fam, a.n)) fam = GEMM_AUTO;
  if (fam == GEMM_COMPACT) {
    const int Tc = (a.n + 63) / 64;
    const int bc = tile_count(Tc, a.sym);
    const bool rag = a.n % 32 != 0;
#define XL_COMPACT(M)                                                                              \
  if (rag)                                                                                         \
    hipLaunchKernelGGL((k_gemm_split_compact<M, true>), dim3(bc), dim3(256), 0, s, a, Tc);         \
  else                                                                                             \
    hipLaunchKernelGGL((k_gemm_split_compact<M, false>), dim3(bc), dim3(256), 0, s, a, Tc);
    if (prec == 3) {
      XL_COMPACT(2)
    } else if (prec == 2) {
      XL_COMPACT(1)
    } else {
      XL_COMPACT(0)
    }
#undef XL_COMPACT
    return;
  }
  if (fam == GEMM_MEDIUM) {
    const int Tm = (a.n + 127) / 128;
    const int bm = tile_count(Tm, a.sym);
    const bool rag = a.n % 32 != 0;
    if (prec == 3) {
      // n % 32 == 0 (family_runs): the ragged FP16x3 instantiation would spill
      hipLaunchKernelGGL((k_gemm_split_mid<2, false>), dim3(bm), dim3(256), 0, s, a, Tm);
    } else if (prec == 2) {
      if (rag)
        hipLaunchKernelGGL((k_gemm_split_mid<1, true>), dim3(bm), dim3(256), 0, s, a, Tm);
      else
        hipLaunchKernelGGL((k_gemm_split_mid<1, false>), dim3(bm), dim3(256), 0, s, a, Tm);
    } else {
      if (rag)
        hipLaunchKernelGGL((k_gemm_split_mid<0, true>), dim3(bm), dim3(256), 0, s, a, Tm);
      else
        hipLaunchKernelGGL((k_gemm_split_mid<0, false>), dim3(bm), dim3(256), 0, s, a, Tm);
    }
    return;
  }
  const bool big = fam == GEMM_AUTO ? (family_runs(prec, GEMM_LARGE, a.n) && blocks >= 192) : fam == GEMM_LARGE;
  if (big) {
    if (prec == 3) {
      hipLaunchKernelGGL((k_gemm_split_big<2, 5>), dim3(blocks), dim3(256), 0, s, a, T);
    } else if (a.sym) {
      if (prec == 2)
        hipLaunchKernelGGL((k_gemm_split_big<1, 5>), dim3(blocks), dim3(256), 0, s, a, T);
      else
        hipLaunchKernelGGL((k_gemm_split_big<0, 5>), dim3(blocks), dim3(256), 0, s, a, T);
    } else {
      if (prec == 2)
        hipLaunchKernelGGL((k_gemm_split_big<1, 7>), dim3(blocks), dim3(256), 0, s, a, T);
      else
        hipLaunchKernelGGL((k_gemm_split_big<0, 7>), dim3(blocks), dim3(256), 0, s, a, T);
    }
    return;
  }
  const int Ts = (a.n + TM - 1) / TM;
  const int nb = a.sym ? Ts * (Ts + 1) / 2 : Ts * Ts;
  switch (prec) {
    // the three-part split (and the FP16 split with its second accumulator)
    // run the direct-to-LDS kernel; BF16x3 the register-staged one, whose
    // single split per element is cheaper than splitting on every read
    case 2: hipLaunchKernelGGL(k_gemm_split_lds<1>, dim3(nb), dim3(320), 0, s, a, Ts); break;
    case 3: hipLaunchKernelGGL(k_gemm_split_lds<2>, dim3(nb), dim3(320), 0, s, a, Ts); break;
    default: hipLaunchKernelGGL(k_gemm_split_bf16x3, dim3(nb), dim3(256), 0, s, a, Ts); break;
  }
}

}  // namespace xl
