// Overlap matrix of a non-orthogonal sp basis and its Pulay force term
// (Methods section 3, eqs. 17-21; forces eqs. 37, 39, 41).
//
// The overlap is the synthetic one of the library's model: unit atom blocks,
// and for A != B the angular structure of the hopping block (s-s: s;
// s_A-p_B: s l; p_A-s_B: -s l; p_A-p_B: s l l^T, l = (R_B - R_A)/R) with the
// radial factor s(R) = s0 exp(-(R - r0)/lam).
#include <hip/hip_runtime.h>

#include "common.h"

namespace xl {
namespace {

struct OvlGeo {
  double r, l[3], s, ds;  // distance, unit vector A -> B, s(R), s'(R)
};

__device__ inline OvlGeo ovl_geo(const double *R, int A, int B, const OverlapSys &ov) {
  OvlGeo g;
  double d[3];
  for (int k = 0; k < 3; ++k) d[k] = R[3 * B + k] - R[3 * A + k];
  g.r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  for (int k = 0; k < 3; ++k) g.l[k] = d[k] / g.r;
  g.s = ov.s0 * exp(-(g.r - ov.r0) / ov.lam);
  g.ds = -g.s / ov.lam;
  return g;
}

// S: one thread per ordered atom pair (A, B), B fastest, writing the 4 x 4
// block as four 32-byte row pieces (consecutive threads, consecutive pieces)
__global__ __launch_bounds__(256) void k_overlap(int N, const double *R, OverlapSys ov, double *S) {
  const size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (idx >= (size_t)N * N) return;
  const int A = (int)(idx / N), B = (int)(idx % N);
  const size_t n = 4 * (size_t)N;
  double blk[4][4];
  if (A == B) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) blk[i][j] = i == j ? 1.0 : 0.0;
  } else {
    const OvlGeo g = ovl_geo(R, A, B, ov);
    blk[0][0] = g.s;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      blk[0][1 + j] = g.s * g.l[j];
      blk[1 + j][0] = -g.s * g.l[j];
#pragma unroll
      for (int i = 0; i < 3; ++i) blk[1 + i][1 + j] = g.s * g.l[i] * g.l[j];
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double *row = S + (4 * (size_t)A + i) * n + 4 * (size_t)B;
    *(double2 *)row = double2{blk[i][0], blk[i][1]};
    *(double2 *)(row + 2) = double2{blk[i][2], blk[i][3]};
  }
}

// Pulay force term F_I = Tr[Q S_{R_I}] with Q = S^-1 F P given transposed (Qt):
// one wavefront per atom I, lane b taking partners B = b, b + 64, ... in that
// order, then a fixed butterfly over the lanes (deterministic).  For the block
// (I, B), d = R_B - R_I and dS_IB/dR_I = -dS_IB/dd, so
//   F_I = -sum_B sum_ij (Q + Q^T)_{4I+i, 4B+j} dS_IB[i][j] / dd.
__global__ __launch_bounds__(256) void k_pulay(int N, const double *R, OverlapSys ov, const double *Qt,
                                               double *frc) {
  const int I = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (I >= N) return;
  const size_t n = 4 * (size_t)N;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int B = lane; B < N; B += 64) {
    if (B == I) continue;
    const OvlGeo g = ovl_geo(R, I, B, ov);
    // M_ij = Q_{4I+i, 4B+j} + Q_{4B+j, 4I+i} = Qt_{4B+j, 4I+i} + Qt_{4I+i, 4B+j}
    double M[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double *ri = Qt + (4 * (size_t)I + i) * n + 4 * (size_t)B;
      const double2 a = *(const double2 *)ri, b = *(const double2 *)(ri + 2);
      M[i][0] = a.x;
      M[i][1] = a.y;
      M[i][2] = b.x;
      M[i][3] = b.y;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double *rj = Qt + (4 * (size_t)B + j) * n + 4 * (size_t)I;
#pragma unroll
      for (int i = 0; i < 4; ++i) M[i][j] += rj[i];
    }
    // derivative blocks with respect to d_k: r' = l_k, l_i' = (delta_ik - l_i l_k) / r
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double dl[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) dl[i] = ((i == k ? 1.0 : 0.0) - g.l[i] * g.l[k]) / g.r;
      const double dsk = g.ds * g.l[k];
      double t = M[0][0] * dsk;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double dsl = dsk * g.l[j] + g.s * dl[j];  // d(s l_j)/dd_k
        t += (M[0][1 + j] - M[1 + j][0]) * dsl;
#pragma unroll
        for (int i = 0; i < 3; ++i)
          t += M[1 + i][1 + j] * (dsk * g.l[i] * g.l[j] + g.s * (dl[i] * g.l[j] + g.l[i] * dl[j]));
      }
      acc[k] -= t;
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc[k] += __shfl_xor(acc[k], o, 64);
  if (lane == 0) {
    frc[3 * I + 0] = acc[0];
    frc[3 * I + 1] = acc[1];
    frc[3 * I + 2] = acc[2];
  }
}

}  // namespace

void overlap_matrix(int n_atoms, const double *R, const OverlapSys &ov, double *S, hipStream_t s) {
  const size_t threads = (size_t)n_atoms * n_atoms;
  hipLaunchKernelGGL(k_overlap, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, n_atoms, R, ov, S);
}

void pulay_forces(int n_atoms, const double *R, const OverlapSys &ov, const double *Qt, double *frc,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_pulay, dim3((n_atoms + 3) / 4), dim3(256), 0, s, n_atoms, R, ov, Qt, frc);
}

}  // namespace xl
