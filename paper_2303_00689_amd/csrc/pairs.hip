// Atom-pair kernels: Fock build F = h + G(P) (eqs. 3, 6, 17), h(R), and the
// eq. 37 forces with the pair-decomposed parts of the shadow energy (eq. 13).
//
// Work is organised in tiles of 16 x 16 atom pairs (upper triangle of atom
// tiles, 256 threads, one thread per pair A < B).  The R-independent factor
// noise_AB of every two-centre block is stored tile-major in groups of four
// integrals, as float4 elements
//   noise_t4[(tilepair * 14 + q) * 256 + slot] = noise[4q .. 4q + 3],
//   slot = 16 * a_local + b_local (the 56th value is a zero pad),
// so that a tile's 55 values reach each thread in 14 loads of 16 bytes, each
// a fully coalesced 4 KiB row of the workgroup.  W_AB is formed in registers
// as gamma(R) * (J[k] + noise_amp * noise[k]).
//
// Per-atom sums over all partners (the two-centre Coulomb term of the
// diagonal blocks, the force on each atom) are reduced deterministically:
// every tile pair writes one partial per (partner tile, atom) and a second
// kernel adds the partials of each atom in a fixed order.
#include "common.h"

#include <cmath>

namespace xl {
namespace {

constexpr int TA = 16;

// packed orbital pairs of one atom (row-major upper triangle of the 4x4 block)
__device__ constexpr int PM[10] = {0, 0, 0, 0, 1, 1, 1, 2, 2, 3};
__device__ constexpr int PN[10] = {0, 1, 2, 3, 1, 2, 3, 2, 3, 3};

__host__ __device__ constexpr int pidx55(int r, int c) {  // r <= c
  return r * 10 - r * (r - 1) / 2 + (c - r);
}

__device__ inline void tri_tile(int bid, int T, int &ta, int &tb) {
  int r = 0, start = 0;
  while (start + (T - r) <= bid) {
    start += T - r;
    ++r;
  }
  ta = r;
  tb = r + (bid - start);
}

constexpr int NQ = 14;  // float4 groups of the 55 noise values (one pad)

__global__ void k_repack(int N, int T, const float *src, float4 *dst) {
  const int tp = blockIdx.x;
  int ta, tb;
  tri_tile(tp, T, ta, tb);
  const int slot = threadIdx.x;
  const int A = ta * TA + slot / TA, B = tb * TA + slot % TA;
  const bool valid = A < N && B < N && A < B;
  const size_t p = valid ? ((size_t)A * N - (size_t)A * (A + 1) / 2 + (B - A - 1)) : 0;
  for (int q = 0; q < NQ; ++q) {
    float v[4];
    for (int e = 0; e < 4; ++e) {
      const int k = 4 * q + e;
      v[e] = valid && k < 55 ? src[p * 55 + k] : 0.0f;
    }
    dst[((size_t)tp * NQ + q) * 256 + slot] = float4{v[0], v[1], v[2], v[3]};
  }
}

// the 55 noise values of the calling thread's pair (14 loads of 16 bytes)
__device__ inline void load_noise(const float *noise_t, int tp, int slot, float nz[4 * NQ]) {
  const float4 *src = reinterpret_cast<const float4 *>(noise_t) + (size_t)tp * NQ * 256 + slot;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const float4 v = src[(size_t)q * 256];
    nz[4 * q] = v.x;
    nz[4 * q + 1] = v.y;
    nz[4 * q + 2] = v.z;
    nz[4 * q + 3] = v.w;
  }
}

struct PairGeo {
  double r, l[3], gamma, dgamma, t, dt;
};

__device__ inline PairGeo pair_geo(const PairSys &ps, int A, int B) {
  PairGeo g;
  double d[3];
  for (int k = 0; k < 3; ++k) d[k] = ps.R[3 * B + k] - ps.R[3 * A + k];
  const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  g.r = sqrt(r2);
  for (int k = 0; k < 3; ++k) g.l[k] = d[k] / g.r;
  const double s2 = r2 + ps.coul_a * ps.coul_a;
  const double is = 1.0 / sqrt(s2);
  g.gamma = ps.coul_k * is;
  g.dgamma = -ps.coul_k * g.r * is * is * is;
  g.t = ps.t0 * exp(-(g.r - ps.r0_hop) / ps.lam_hop);
  g.dt = -g.t / ps.lam_hop;
  return g;
}

// F off-diagonal atom blocks and Coulomb partials.  A workgroup takes one
// 16 x 16 atom-tile pair (ta <= tb), one thread per atom pair.
//   1. the packed diagonal density blocks of its 32 atoms (off-diagonal
//      entries doubled, -zsub at ss for h alone) into LDS;
//   2. per pair the 10 x 10 two-centre block W_AB in registers, the exchange
//      block G_AB = -1/2 sum P_AB W_AB and the Coulomb sums of A over B's
//      packed density and of B over A's;
//   3. the Coulomb sums reduced per atom over the tile's 16 partners, one
//      partial per (atom, partner tile): part[(atom * T + tile) * 10 + r];
//   4. the 64 x 64 block of F in LDS, written to F row by row and, transposed,
//      to the mirrored position, 512 contiguous bytes per row.  On a diagonal
//      tile pair (ta == tb) only blocks of distinct atoms are written; the
//      diagonal atom blocks are k_fock_diag's.
constexpr int FT = 4 * TA;       // F rows (and columns) of a tile: 64
constexpr int FTP = FT + 1;      // padded LDS row of the staged block (doubles)
// LDS row of the Coulomb sums, one per packed pair (doubles): 261 rather than
// 256 puts the ten rows that the lanes of one reduction read on different banks
constexpr int CRS = 261;
// staged block entry (row, col): columns rotated by row / 2 within the row, so
// that the 4 x 4 block stores and the row and column reads of the F store
// phase spread over the LDS banks
__device__ inline int ft_at(int row, int col) { return row * FTP + ((col + (row >> 1)) & (FT - 1)); }

__global__ __launch_bounds__(256) void k_fock_pairs(PairSys ps, int n, const double *P, double zsub,
                                                     int include_h, double *F, double *part) {
  const int N = ps.n_atoms, T = ps.n_tiles;
  const int tp = blockIdx.x;
  int ta, tb;
  tri_tile(tp, T, ta, tb);
  const int slot = threadIdx.x, al = slot / TA, bl = slot % TA;
  const int A = ta * TA + al, B = tb * TA + bl;
  const bool valid = A < N && B < N && (ta < tb || al < bl);

  // LDS, reused by the phases: packed diagonals (phase 1-2), Coulomb sums
  // (phase 3), the staged F block (phase 4)
  __shared__ double sh[2 * 10 * CRS];
  double *spk = sh + 2 * 10 * CRS - 32 * 10;  // [32][10]: A atoms 0..15, B atoms 16..31 (top of sh)
  double *shA = sh, *shB = sh + 10 * CRS;     // [10][CRS] each
  double *ft = sh;                            // [FT][FTP]

  for (int v = slot; v < 320; v += 256) {
    const int q = v / 10, r = v % 10;
    const int X = q < TA ? ta * TA + q : tb * TA + (q - TA);
    double x = 0.0;
    if (X < N) {
      const int m = PM[r], c = PN[r];
      x = P ? P[(size_t)(4 * X + m) * n + 4 * X + c] : 0.0;
      if (m != c) x *= 2.0;
      if (r == 0) x -= zsub;
    }
    spk[q * 10 + r] = x;
  }
  __syncthreads();

  double cA[10], cB[10], G[4][4];
#pragma unroll
  for (int r = 0; r < 10; ++r) cA[r] = cB[r] = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) G[i][j] = 0.0;

  if (valid) {
    const PairGeo g = pair_geo(ps, A, B);
    double Pab[4][4], pA[10], pB[10];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) Pab[i][j] = P ? P[(size_t)(4 * A + i) * n + 4 * B + j] : 0.0;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
      pA[r] = spk[al * 10 + r];
      pB[r] = spk[(TA + bl) * 10 + r];
    }
    float nz[4 * NQ];
    load_noise(ps.noise_t, tp, slot, nz);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
#pragma unroll
      for (int c = r; c < 10; ++c) {
        const int k = pidx55(r, c);
        const double w = g.gamma * (ps.j55[k] + ps.noise_amp * (double)nz[k]);
        // position (r, c): r is A's orbital pair, c is B's
        cA[r] += w * pB[c];
        cB[c] += w * pA[r];
        {
          const int mu = PM[r], nu = PN[r], la = PM[c], si = PN[c];
          G[mu][la] -= 0.5 * w * Pab[nu][si];
          if (la != si) G[mu][si] -= 0.5 * w * Pab[nu][la];
          if (mu != nu) G[nu][la] -= 0.5 * w * Pab[mu][si];
          if (mu != nu && la != si) G[nu][si] -= 0.5 * w * Pab[mu][la];
        }
        if (r != c) {  // mirrored position (c, r)
          cA[c] += w * pB[r];
          cB[r] += w * pA[c];
          const int mu = PM[c], nu = PN[c], la = PM[r], si = PN[r];
          G[mu][la] -= 0.5 * w * Pab[nu][si];
          if (la != si) G[mu][si] -= 0.5 * w * Pab[nu][la];
          if (mu != nu) G[nu][la] -= 0.5 * w * Pab[mu][si];
          if (mu != nu && la != si) G[nu][si] -= 0.5 * w * Pab[mu][la];
        }
      }
    }
    if (include_h) {
      const double t = g.t;
      G[0][0] += t;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        G[0][1 + j] += t * g.l[j];
        G[1 + j][0] -= t * g.l[j];
#pragma unroll
        for (int i = 0; i < 3; ++i) G[1 + i][1 + j] += t * g.l[i] * g.l[j];
      }
    }
  }
  __syncthreads();  // every read of the packed diagonals is done
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    shA[r * CRS + slot] = cA[r];
    shB[r * CRS + slot] = cB[r];
  }
  __syncthreads();
  if (slot < 160) {
    const int x = slot / 10, r = slot % 10;
    double row = 0.0, col = 0.0;
    for (int q = 0; q < TA; ++q) {
      row += shA[r * CRS + x * TA + q];  // atom ta*16+x as A, over partners b
      col += shB[r * CRS + q * TA + x];  // atom tb*16+x as B, over partners a
    }
    if (ta == tb) {
      const int X = ta * TA + x;
      if (X < N) part[((size_t)X * T + ta) * 10 + r] = row + col;
    } else {
      const int XA = ta * TA + x, XB = tb * TA + x;
      if (XA < N) part[((size_t)XA * T + tb) * 10 + r] = row;
      if (XB < N) part[((size_t)XB * T + ta) * 10 + r] = col;
    }
  }
  __syncthreads();  // the Coulomb sums are read; the block is staged over them
  // On a diagonal tile pair the pairs a < b fill the upper blocks and their
  // transposes the lower ones (each LDS word written by one thread only); the
  // diagonal atom blocks are left out below.
  if (ta != tb || valid) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        ft[ft_at(4 * al + i, 4 * bl + j)] = G[i][j];
        if (ta == tb) ft[ft_at(4 * bl + j, 4 * al + i)] = G[i][j];
      }
  }
  __syncthreads();
  // 8 threads per row, two consecutive columns per store: 128 contiguous
  // bytes of a row per store instruction, for the block and for its transpose
  // (a column of the staged block)
  const int k8 = slot & 7;
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
    const int row = pass * 32 + (slot >> 3);
    const int ra = ta * TA + row / 4;  // atom of block row `row` (tile ta)
    const int rb = tb * TA + row / 4;  // atom of transposed row `row` (tile tb)
    const size_t ga = ((size_t)4 * ta * TA + row) * n + (size_t)4 * tb * TA;
    const size_t gb = ((size_t)4 * tb * TA + row) * n + (size_t)4 * ta * TA;
#pragma unroll
    for (int s8 = 0; s8 < 4; ++s8) {
      const int cc = 16 * s8 + 2 * k8;  // two consecutive columns of one atom
      const int ca = tb * TA + cc / 4, cb = ta * TA + cc / 4;
      if (ra < N && ca < N && (ta != tb || ra != ca))
        *(double2 *)(F + ga + cc) = double2{ft[ft_at(row, cc)], ft[ft_at(row, cc + 1)]};
      if (ta != tb && rb < N && cb < N)
        *(double2 *)(F + gb + cc) = double2{ft[ft_at(cc, row)], ft[ft_at(cc + 1, row)]};
    }
  }
}

// one-centre two-electron block of atom A from its spin-summed density block
__device__ inline void onecenter_G(const double *oc, const double Pd[4][4], double G1[4][4]) {
  const double gss = oc[0], gsp = oc[1], gpp = oc[2], gp2 = oc[3], hsp = oc[4];
  const double hpp = 0.5 * (gpp - gp2);
  const double pss = Pd[0][0], pxx = Pd[1][1], pyy = Pd[2][2], pzz = Pd[3][3];
  G1[0][0] = 0.5 * pss * gss + (pxx + pyy + pzz) * (gsp - 0.5 * hsp);
  const double pp[3] = {pxx, pyy, pzz};
  for (int i = 0; i < 3; ++i) {
    double v = pss * (gsp - 0.5 * hsp) + 0.5 * pp[i] * gpp;
    for (int j = 0; j < 3; ++j)
      if (j != i) v += pp[j] * (gp2 - 0.5 * hpp);
    G1[1 + i][1 + i] = v;
    G1[0][1 + i] = G1[1 + i][0] = 0.5 * Pd[0][1 + i] * (3.0 * hsp - gsp);
    for (int j = 0; j < 3; ++j)
      if (j != i) G1[1 + i][1 + j] = 0.5 * Pd[1 + i][1 + j] * (3.0 * hpp - gp2);
  }
}

// Diagonal atom blocks: the one-centre part (eq. 6 with the one-centre
// integrals), the two-centre Coulomb sums over all partners, and h's on-site
// terms.  One wavefront per atom: lane l adds the partials of partner tiles
// l, l + 64, ... in that order, then a fixed butterfly over the lanes.
__global__ __launch_bounds__(256) void k_fock_diag(PairSys ps, int n, const double *P, int include_h,
                                                   const double *part, double *F) {
  const int N = ps.n_atoms, T = ps.n_tiles;
  const int A = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (A >= N) return;
  double coul[10];
#pragma unroll
  for (int r = 0; r < 10; ++r) coul[r] = 0.0;
  for (int t = lane; t < T; t += 64) {
    const double *pp = part + ((size_t)A * T + t) * 10;
#pragma unroll
    for (int r = 0; r < 10; ++r) coul[r] += pp[r];
  }
#pragma unroll
  for (int r = 0; r < 10; ++r)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) coul[r] += __shfl_xor(coul[r], o, 64);
  if (lane >= 16) return;
  // lane 4 i + j writes element (i, j) of the block, the value of the upper
  // element (lo, hi) for both (i, j) and (j, i): like the pair blocks, the
  // diagonal blocks take P's upper triangle, so F is symmetric for any P
  const int i = lane >> 2, j = lane & 3;
  const int lo = i < j ? i : j, hi = i < j ? j : i;
  double Pd[4][4], G1[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) Pd[a][b] = P ? P[(size_t)(4 * A + a) * n + 4 * A + b] : 0.0;
  onecenter_G(ps.onecenter + 5 * A, Pd, G1);
  // (lo, hi) differ by lane: pick by compare-and-select with constant
  // indices, so that G1 and coul stay in registers
  double c = 0.0, g = 0.0;
#pragma unroll
  for (int r = 0; r < 10; ++r)
    if (PM[r] == lo && PN[r] == hi) c = coul[r];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = a; b < 4; ++b)
      if (a == lo && b == hi) g = G1[a][b];
  double v = g + c;
  if (include_h && i == j) v += (i == 0) ? ps.eps_s : ps.eps_p;
  F[(size_t)(4 * A + i) * n + 4 * A + j] = v;
}

// ---- forces and pair energies
// pk3 = [p0 | x | q] packed diagonal blocks, q = P0 - X/2, each N x 10
__global__ __launch_bounds__(256) void k_force_pairs(PairSys ps, int n, const double *P0,
                                                      const double *X, const double *pk3,
                                                      double *fpart, double *epart) {
  const int N = ps.n_atoms, T = ps.n_tiles;
  const int tp = blockIdx.x;
  int ta, tb;
  tri_tile(tp, T, ta, tb);
  const int slot = threadIdx.x, al = slot / TA, bl = slot % TA;
  const int A = ta * TA + al, B = tb * TA + bl;
  const bool valid = A < N && B < N && (ta < tb || al < bl);
  __shared__ double shf[3][256];
  __shared__ double she[5][4];
  double dE[3] = {0.0, 0.0, 0.0};
  double e_hop = 0.0, e_core = 0.0, e_ee = 0.0, e_nn = 0.0, e_rep = 0.0;
  if (valid) {
    const PairGeo g = pair_geo(ps, A, B);
    double Pab[4][4], Qab[4][4], Xab[4][4];
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        const size_t off = (size_t)(4 * A + i) * n + 4 * B + j;
        Pab[i][j] = P0[off];
        Xab[i][j] = X[off];
        Qab[i][j] = Pab[i][j] - 0.5 * Xab[i][j];
      }
    const double *p0A = pk3 + A * 10, *p0B = pk3 + B * 10;
    const double *xA = pk3 + (size_t)N * 10 + A * 10, *xB = pk3 + (size_t)N * 10 + B * 10;
    const double *qA = pk3 + (size_t)2 * N * 10 + A * 10, *qB = pk3 + (size_t)2 * N * 10 + B * 10;
    // hopping: E = 2 t phi(l), phi = P_ss + (a - b).l + l^T C l
    double phi = Pab[0][0], gv[3];
    for (int j = 0; j < 3; ++j) {
      phi += (Pab[0][1 + j] - Pab[1 + j][0]) * g.l[j];
      gv[j] = Pab[0][1 + j] - Pab[1 + j][0];
    }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        phi += Pab[1 + i][1 + j] * g.l[i] * g.l[j];
        gv[i] += Pab[1 + i][1 + j] * g.l[j];
        gv[j] += Pab[1 + i][1 + j] * g.l[i];
      }
    e_hop = 2.0 * g.t * phi;
    const double gl = gv[0] * g.l[0] + gv[1] * g.l[1] + gv[2] * g.l[2];
    for (int k = 0; k < 3; ++k)
      dE[k] = 2.0 * g.dt * phi * g.l[k] + 2.0 * g.t / g.r * (gv[k] - gl * g.l[k]);
    // terms linear in W, evaluated with the base block b = J + noise_amp * noise
    float nz[4 * NQ];
    load_noise(ps.noise_t, tp, slot, nz);
    const double Z = ps.z_core;
    double bcore = 0.0, bee = 0.0, bnn = 0.0;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
#pragma unroll
      for (int c = r; c < 10; ++c) {
        const int k = pidx55(r, c);
        const double b = ps.j55[k] + ps.noise_amp * (double)nz[k];
        // position (r, c)
        double ex = 0.0;
        {
          const int mu = PM[r], nu = PN[r], la = PM[c], si = PN[c];
          ex += Qab[mu][la] * Xab[nu][si];
          if (la != si) ex += Qab[mu][si] * Xab[nu][la];
          if (mu != nu) ex += Qab[nu][la] * Xab[mu][si];
          if (mu != nu && la != si) ex += Qab[nu][si] * Xab[mu][la];
        }
        double core = (c == 0 ? p0A[r] : 0.0) + (r == 0 ? p0B[c] : 0.0);
        double ee = qA[r] * xB[c] + xA[r] * qB[c] - ex;
        if (r != c) {
          const int mu = PM[c], nu = PN[c], la = PM[r], si = PN[r];
          double ex2 = Qab[mu][la] * Xab[nu][si];
          if (la != si) ex2 += Qab[mu][si] * Xab[nu][la];
          if (mu != nu) ex2 += Qab[nu][la] * Xab[mu][si];
          if (mu != nu && la != si) ex2 += Qab[nu][si] * Xab[mu][la];
          core += (r == 0 ? p0A[c] : 0.0) + (c == 0 ? p0B[r] : 0.0);
          ee += qA[c] * xB[r] + xA[c] * qB[r] - ex2;
        }
        bcore -= Z * core * b;
        bee += ee * b;
        if (r == 0 && c == 0) bnn += Z * Z * b;
      }
    }
    e_core = g.gamma * bcore;
    e_ee = g.gamma * bee;
    e_nn = g.gamma * bnn;
    e_rep = ps.a_rep * exp(-(g.r - ps.r0_rep) / ps.rho_rep);
    const double dr = g.dgamma * (bcore + bee + bnn) - e_rep / ps.rho_rep;
    for (int k = 0; k < 3; ++k) dE[k] += dr * g.l[k];
  }
  // dE = dE_pair/dR_B: the force on B is -dE and the force on A is +dE
  for (int k = 0; k < 3; ++k) shf[k][slot] = dE[k];
  // block energy sums
  double ev[5] = {e_hop, e_core, e_ee, e_nn, e_rep};
  for (int q = 0; q < 5; ++q) {
    double v = ev[q];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if ((slot & 63) == 0) she[q][slot >> 6] = v;
  }
  __syncthreads();
  if (slot < 5) epart[(size_t)tp * 5 + slot] = she[slot][0] + she[slot][1] + she[slot][2] + she[slot][3];
  if (slot < 48) {
    const int x = slot / 3, k = slot % 3;
    double row = 0.0, col = 0.0;
    for (int q = 0; q < TA; ++q) {
      row += shf[k][x * TA + q];
      col -= shf[k][q * TA + x];
    }
    if (ta == tb) {
      const int Xa = ta * TA + x;
      if (Xa < N) fpart[((size_t)ta * N + Xa) * 3 + k] = row + col;
    } else {
      const int XA = ta * TA + x, XB = tb * TA + x;
      if (XA < N) fpart[((size_t)tb * N + XA) * 3 + k] = row;
      if (XB < N) fpart[((size_t)ta * N + XB) * 3 + k] = col;
    }
  }
}

__global__ void k_zero(size_t m, double *p) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < m; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// one thread per (atom, packed orbital pair)
__global__ void k_pack3(int N, int n, const double *P0, const double *X, double *pk3) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= 10 * N) return;
  const int A = v / 10, r = v % 10;
  const int m = PM[r], q = PN[r];
  const size_t off = (size_t)(4 * A + m) * n + 4 * A + q;
  const double f = (m != q) ? 2.0 : 1.0;
  pk3[v] = f * P0[off];
  pk3[(size_t)N * 10 + v] = f * X[off];
  pk3[(size_t)2 * N * 10 + v] = f * (P0[off] - 0.5 * X[off]);
}

// per-atom: total force, and per-atom energies (on-site h, one-centre ee).
// One wavefront per atom: lane l adds the force partials of partner tiles
// l, l + 64, ... in that order, then a fixed butterfly over the lanes.
__global__ __launch_bounds__(256) void k_force_atoms(PairSys ps, int n, const double *P0, const double *X,
                                                     const double *fpart, double *frc, double *eatom) {
  const int A = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int N = ps.n_atoms;
  if (A >= N) return;
  double f[3] = {0.0, 0.0, 0.0};
  for (int t = lane; t < ps.n_tiles; t += 64)
#pragma unroll
    for (int k = 0; k < 3; ++k) f[k] += fpart[((size_t)t * N + A) * 3 + k];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) f[k] += __shfl_xor(f[k], o, 64);
  if (lane != 0) return;
#pragma unroll
  for (int k = 0; k < 3; ++k) frc[3 * A + k] = f[k];  // partials already hold -dE/dR of their pairs
  double Xd[4][4], G1[4][4];
  double e_on = 0.0, e_1c = 0.0;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) Xd[i][j] = X[(size_t)(4 * A + i) * n + 4 * A + j];
  onecenter_G(ps.onecenter + 5 * A, Xd, G1);
  for (int i = 0; i < 4; ++i) {
    const size_t di = (size_t)(4 * A + i) * n + 4 * A + i;
    e_on += (i == 0 ? ps.eps_s : ps.eps_p) * P0[di];
    for (int j = 0; j < 4; ++j) {
      const size_t off = (size_t)(4 * A + i) * n + 4 * A + j;
      e_1c += (P0[off] - 0.5 * X[off]) * G1[i][j];
    }
  }
  eatom[2 * A] = e_on;
  eatom[2 * A + 1] = e_1c;
}

// e[0] = Tr[h P0] = on-site + hop + core; e[1] = Tr[(P0 - X/2) G(X)] = 1c + ee;
// e[2] = V_nn = nn + rep.  Fixed-order sums.
__global__ void k_energy_final(int ntp, const double *epart, int N, const double *eatom, double *e) {
  __shared__ double sh[7][256];
  double s[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int t = threadIdx.x; t < ntp; t += 256)
    for (int q = 0; q < 5; ++q) s[q] += epart[(size_t)t * 5 + q];
  for (int a = threadIdx.x; a < N; a += 256) {
    s[5] += eatom[2 * a];
    s[6] += eatom[2 * a + 1];
  }
  for (int q = 0; q < 7; ++q) sh[q][threadIdx.x] = s[q];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o)
      for (int q = 0; q < 7; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    e[0] = sh[5][0] + sh[0][0] + sh[1][0];
    e[1] = sh[6][0] + sh[2][0];
    e[2] = sh[3][0] + sh[4][0];
  }
}

}  // namespace

size_t noise_tile_floats(int n_atoms) {
  const int T = (n_atoms + TA - 1) / TA;
  return (size_t)T * (T + 1) / 2 * 4 * NQ * 256;
}

void repack_noise(int n_atoms, const float *src, float *dst, hipStream_t s) {
  const int T = (n_atoms + TA - 1) / TA;
  hipLaunchKernelGGL(k_repack, dim3(T * (T + 1) / 2), dim3(256), 0, s, n_atoms, T, src,
                     reinterpret_cast<float4 *>(dst));
}

void fock(const PairSys &ps, const double *P, double *F, int include_h, double *part, hipStream_t s) {
  const int N = ps.n_atoms, n = 4 * N, T = ps.n_tiles;
  if (N > 1)
    hipLaunchKernelGGL(k_fock_pairs, dim3(T * (T + 1) / 2), dim3(256), 0, s, ps, n, P,
                       include_h ? ps.z_core : 0.0, include_h, F, part);
  else
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, s, (size_t)10 * N * T, part);
  hipLaunchKernelGGL(k_fock_diag, dim3((N + 3) / 4), dim3(256), 0, s, ps, n, P, include_h, part, F);
}

void hcore(const PairSys &ps, double *H, double *part, hipStream_t s) {
  // h = F(P = 0) with the core attraction carried by the packed "-z at ss" density
  fock(ps, nullptr, H, 1, part, s);
}

size_t force_partial_doubles(int n_atoms) {
  const int T = (n_atoms + TA - 1) / TA;
  return (size_t)T * n_atoms * 3;
}
size_t energy_partial_doubles(int n_atoms) {
  const int T = (n_atoms + TA - 1) / TA;
  return (size_t)T * (T + 1) / 2 * 5 + 2 * (size_t)n_atoms;
}

void forces(const PairSys &ps, const double *P0, const double *X, double *frc, double *e,
            double *pk3, double *fpart, double *epart, hipStream_t s) {
  const int N = ps.n_atoms, n = 4 * N, T = ps.n_tiles;
  const int ntp = T * (T + 1) / 2;
  double *eatom = epart + (size_t)ntp * 5;
  hipLaunchKernelGGL(k_pack3, dim3((10 * N + 255) / 256), dim3(256), 0, s, N, n, P0, X, pk3);
  if (N > 1) {
    hipLaunchKernelGGL(k_force_pairs, dim3(ntp), dim3(256), 0, s, ps, n, P0, X, pk3, fpart, epart);
  } else {
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, s, (size_t)3 * N * T, fpart);
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, s, (size_t)5 * ntp, epart);
  }
  hipLaunchKernelGGL(k_force_atoms, dim3((N + 3) / 4), dim3(256), 0, s, ps, n, P0, X, fpart, frc, eatom);
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(256), 0, s, ntp, epart, N, eatom, e);
}

}  // namespace xl
