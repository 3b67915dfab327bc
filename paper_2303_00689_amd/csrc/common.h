// Internal declarations shared by the HIP translation units of libxlbomd.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace xl {

// ---------------------------------------------------------------- GEMM (FP64)
// out = alpha * sum_p op(A_p) op(B_p) + beta1 * C1 + beta2 * C2 + gamma * I
// op(A) reads A as its transpose (A^T tiles are contiguous rows of A), which is
// A itself for the symmetric operands of the Fermi-operator and response chains.
// op(B) is B (btrans = 0) or B^T (btrans = 1) in the FP64 kernels.  The split
// kernels read B by rows whatever btrans says, i.e. op(B) = B^T: a caller
// passes a symmetric B there (op(B) = B), or B^T to get A B.  sym = 1 computes only tiles with
// tile_row <= tile_col and writes each one also to the mirrored position; it is
// valid when the result is symmetric (products of commuting symmetric matrices,
// A B + B A, and the final product of a response level).  out must not alias an
// A or B operand; it may alias C1 or C2.
struct GemmArgs {
  int n;
  int nprod;               // 1 or 2
  const void *A[2];
  const void *B[2];
  int btrans;
  const void *C1, *C2;     // nullable
  void *out;
  double alpha, beta1, beta2, gamma;
  int sym;
  int family;              // GEMM_AUTO: the tile table, else the built-in rule
};
// Kernel families of an n x n product.  FP64: GEMM_SMALL = 64 x 64 tiles,
// GEMM_LARGE = 128 x 128 (128 x 64 over the upper triangle for symmetric
// outputs; n % 16 == 0, n <= 23170).  Split: GEMM_SMALL = 128 x 128 tiles,
// GEMM_LARGE = 224 x 224 full / 160 x 160 symmetric (FP16x3: 160 x 160 for
// both; n % 32 == 0, n <= 32767), GEMM_MEDIUM = the large-tile kernel with
// 128 x 128 tiles at two workgroups per compute unit (n % 4 == 0, a ragged
// last k panel when n % 32 != 0; FP16x3 n % 32 == 0).  A family that cannot run n falls back to
// the built-in rule.
// GEMM_COMPACT: small tiles for small orders, four times the workgroups of
// the next family up: split, the large-tile kernel at 64 x 64 (2 x 2 MFMA
// blocks per wave, n % 4 == 0, n >= 64); FP64, 32 x 32 tiles (n % 4 == 0).
enum { GEMM_AUTO = 0, GEMM_SMALL = 1, GEMM_LARGE = 2, GEMM_MEDIUM = 3, GEMM_COMPACT = 4 };
// The tile table's family for a product of order n (prec 0 = FP64, 1..3 as
// below), or GEMM_AUTO when no row matches.
int table_family(int prec, int sym, int n);
// Whether family fam can run an n x n product in precision prec.
bool family_runs(int prec, int fam, int n);
void gemm_f64(const GemmArgs &a, hipStream_t s);
// Split-precision GEMM on FP32 storage (prec: 1 = BF16x3, 2 = BF16x6, 3 = FP16x3).
void gemm_split(const GemmArgs &a, int prec, hipStream_t s);
// Whether A B + B A (A, B symmetric, split precision prec) is cheaper as one
// full-output product 2 A B and the in-place transpose average than as one
// two-product launch over the upper triangle: where both run the large tiles
// (224 rows full, 160 symmetric; BF16x3 and BF16x6) and the 224-row tiles of
// the full output fit one round of the 256 compute units, the full-output
// tiles' higher MFMA rate outweighs the extra pass over the result.
bool split_sum_by_transpose(int prec, int n);

// ------------------------------------------------------------- BLAS-1 (FP64 or FP32)
// Elementwise kernels operate on n*n matrices of the given element type
// (is32 = 0: double, 1: float).  Scalars marked "_dev" are read from device memory.
void axpby(int n2, double a, const void *x, double b, const void *y, void *out, int is32, hipStream_t s);
// out = a*x + b*y + g*I, with a, b, g taken from device scalars (null -> host value)
void axpbyI_dev(int n, const double *a_dev, double a, const void *x, const double *b_dev, double b,
                const void *y, const double *g_dev, double g, void *out, int is32, hipStream_t s);
// out = scale * in, converted (scale applied in FP64 before the rounding to out's type)
void convert(int n2, const void *in, int in32, void *out, int out32, hipStream_t s, double scale = 1.0);
// out = 2 (H + s M) - sub, FP64 out; H, M FP32 (is32) or FP64; s a device
// scalar; sub FP64 or null (then nothing is subtracted)
void canon_out(int n2, const void *H, const void *M, const double *s_dev, const double *sub, double *out,
               int is32, hipStream_t s);
// out = in^T (n x n, FP64 in, FP32 out)
void convert_t(int n, const double *in, float *out, hipStream_t s);
// out = sum_{j<4} a_j X_j + g I (null X_j skipped; out may alias an X_j)
void poly_comb(int n, const void *const X[4], const double a[4], double g, void *out, int is32,
               hipStream_t s);
void symmetrize(int n, void *M, int is32, hipStream_t s);
// out = a + b (FP64 a, FP32 b, FP64 out; out may alias a) and out32 = FP32(out) if non-null
void add_mixed(int n2, const double *a, const float *b, double *out, float *out32, hipStream_t s);
// out = sum_j coef[j] * M_j (coef on device), j < k <= 40, FP64
void lincomb_dev(int n2, int k, const double *const *M, const double *coef, double *out, hipStream_t s);

// Deterministic FP64 reductions into device scalars.
// dots: res[i] = <X_i, Y_i> (Frobenius) for i < k <= 16; every X_i, Y_i 16-byte aligned
// (library buffers, or halves of them at offsets of 4 n^2 bytes with n = 4 N_atoms)
void dots(int n2, int k, const void *const *X, const void *const *Y, double *res, int is32,
          double *partials, hipStream_t s);
// Gram-Schmidt update out = v - sum_{j<k} c_j V_j (1 <= k <= 32; c: k device
// doubles; Vs: device array of k device pointers; out must not alias v or a
// V_j) and, in the same pass, res[j] = <V_j, out> for j < k (self = 0) or
// res[0] = <out, out> (self = 1)
void orth_dots(int n2, int k, const double *v, const double *const *Vs, const double *c, double *out, int self,
               double *res, double *partials, hipStream_t s);
// res[0] = trace(M)
void trace(int n, const void *M, double *res, int is32, double *partials, hipStream_t s);
// Gershgorin bounds of a symmetric matrix: res[0] = min(F_ii - r_i), res[1] = max(F_ii + r_i)
void gershgorin(int n, const double *F, double *res, double *partials, hipStream_t s);
// the fixed unit start vector of the Lanczos steps into row 0 of Q (n values)
void lanczos_start(int n, double *Q, hipStream_t s);
// k Lanczos steps on symmetric F from the unit vector in row 0 of Q
// ((k + 1) x n); w: n scratch; ab: 2k device doubles (alpha_j, beta_j)
void lanczos(int n, int k, const double *F, double *Q, double *w, double *ab, hipStream_t s);
int reduce_partials_capacity();

// ------------------------------------------------------------- pair kernels
struct PairSys {
  int n_atoms;
  int n_tiles;             // atom tiles of 16
  const double *R;         // n_atoms x 3
  const double *onecenter; // n_atoms x 5
  const float *noise_t;    // tile-major noise, float4 groups [tilepair][14][256][4], 16-byte aligned
  const double *j55;       // device, 55
  double eps_s, eps_p, t0, r0_hop, lam_hop, coul_k, coul_a, noise_amp, z_core, a_rep, r0_rep,
      rho_rep;
};
void repack_noise(int n_atoms, const float *noise_host_layout_dev, float *noise_t, hipStream_t s);
size_t noise_tile_floats(int n_atoms);
// F = [h +] G(P); partial: scratch of n_atoms * n_tiles * 10 doubles
void fock(const PairSys &ps, const double *P, double *F, int include_h, double *partial, hipStream_t s);
void hcore(const PairSys &ps, double *H, double *partial, hipStream_t s);
// forces (n_atoms x 3) and energy parts e[0..2] = Tr[hP0], Tr[(P0-X/2)G(X)], Vnn (device)
void forces(const PairSys &ps, const double *P0, const double *X, double *frc, double *e,
            double *pk3, double *fpart, double *epart, hipStream_t s);
size_t force_partial_doubles(int n_atoms);
size_t energy_partial_doubles(int n_atoms);

// ------------------------------------------------- non-orthogonal basis
// radial constants of the synthetic overlap s(R) = s0 exp(-(R - r0)/lam)
struct OverlapSys {
  double s0, r0, lam;
};
// S (4 n_atoms square, row-major): unit atom blocks, hopping-shaped off-site blocks
void overlap_matrix(int n_atoms, const double *R, const OverlapSys &ov, double *S, hipStream_t s);
// frc (n_atoms x 3) = Tr[Q S_{R_I}] for Q = S^-1 F P, given as Qt = Q^T
void pulay_forces(int n_atoms, const double *R, const OverlapSys &ov, const double *Qt, double *frc,
                  hipStream_t s);

// ------------------------------------------------------------- scalar kernels
// Chemical-potential and Krylov scalar steps (one thread), see the .hip file.
// tol_n: a trace within tol_n of n_occ takes no shift (dmu = 0)
void mu_series_solve(const double *tau, double n_occ, double beta, double tol_n, double *out, hipStream_t s);
void mu_newton(const double *t01, double n_occ, double beta, double tol_n, double *out, hipStream_t s);
void krylov_solve(int k, const double *O, const double *rhs, double *coef, double *resid2,
                  const double *k_rank, hipStream_t s);

// ------------------------------------------------------------- MD kernels
void x_verlet(int n2, const double *const *Xk, const double *Y, double kappa, double alpha,
              const double *c, double *out, hipStream_t s);
// BAOAB (Leimkuhler-Matthews) before the force evaluation: half kick, half
// drift, V <- c1 V + c2 xi, half drift
void baoab_pre(int n3, double *R, double *V, const double *A, double dt, double c1, double c2,
               const double *xi, hipStream_t s);
void kick_drift(int n3, double *R, double *V, const double *A, double dt, int drift,
                hipStream_t s);
void accel(int n3, const double *frc, double inv_mass_conv, double *A, hipStream_t s);

}  // namespace xl

#define XL_CHECK_LAUNCH() (void)0
