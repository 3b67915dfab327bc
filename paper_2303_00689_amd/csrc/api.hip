// C ABI of libxlbomd: handle, workspace and the host orchestration of the
// hot path.  Every arithmetic step runs in the kernels of gemm_*.hip,
// blas1.hip and pairs.hip; this file only sequences them, keeps the chain
// cache and moves a few scalars between host and device.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include <hipsolver/hipsolver.h>

#include "../../include/xlbomd.h"
#include "common.h"
#include "small_eig.h"

using namespace xl;

namespace {

constexpr int LMAX = 24;     // maximum number of recursion levels
constexpr int MMAX = 32;     // maximum Krylov rank
constexpr double KB = 8.617333262e-5;           // eV / K
constexpr double ACC = 9.648533e-3;             // (eV / (Angstrom amu)) -> Angstrom / fs^2
constexpr int LANCZOS_K = 32;                 // Lanczos steps for the spectral bounds
// Start interval and least depth of the Fermi chain.  For the degree-9 start
// followed by L doubling levels, the largest deviation from the Fermi function
// and from its derivative over |v| <= vb (scalar recursion in FP64) is
//   L = 1..4: 1e-2 .. 4e-11 already for vb >= 0.4 (the start's truncation error,
//             and that of its derivative, is not yet squared away);
//   L >= 5:   <= 4e-14 for every vb up to 1.68 (1.85 at L = 6),
// so the chain takes L >= 5 and |v| <= 1.6.
constexpr double VMAX = 1.6;
constexpr int LMIN = 5;
// Taylor coefficients of tanh(v) / v in powers of v^2 (degree-9 start)
constexpr double TC0 = 1.0, TC1 = -1.0 / 3.0, TC2 = 2.0 / 15.0, TC3 = -17.0 / 315.0,
                 TC4 = 62.0 / 2835.0;

// device scalar slots
enum Slot {
  S_LOHI = 0,      // 2
  S_TAU = 4,       // 8: tau_0..tau_5
  S_MU1 = 16,      // 5: dmu, c, 2/(1+c), flag, 1-c
  S_T01 = 28,      // 2: Tr D1, Tr D1(I-D1)
  S_TRM = 48,      // Tr M
  S_TRR = 50,      // Tr R (response)
  S_CAN = 52,      // -Tr R / Tr M
  S_TRD = 54,      // final trace of D
  S_FIX = 56,      // first-order trace correction coefficient (+1: mu_shift's own step)
  S_ENT = 59,      // entropy S/k_B
  S_TRP = 58,      // trace of the returned P
  S_ENER = 60,     // 3 energies
  S_DOTS = 64,     // 40 dots
  S_KO = 128,      // Krylov O, 32 x 32 (row stride 32)
  S_KRHS = 1152,   // 32
  S_KCOEF = 1184,  // 32
  S_KRES = 1216,   // 3: resid^2, ||W0||^2, singular
  S_ORTH = 1220,   // 33 orthogonalisation coefficients
  S_LANC = 1280,   // 2 * LANCZOS_K: alpha_j, beta_j
  S_KCTL = 1344,   // Krylov control: |v|^2, |source|^2, scale, breakdown rank (-1: none)
  S_TOTAL = 1352
};

// s = -scale tr / Tr M, the chemical-potential term of the canonical response
__global__ void k_canon(const double *tr, const double *trM, double scale, double *out) {
  if (threadIdx.x) return;
  *out = (*trM > 0.0) ? -scale * (*tr) / (*trM) : 0.0;
}

// first-order chemical-potential correction of the stored chain result:
// P = 2 (D + c M) with c = (n_occ - Tr D) / Tr M, written in FP64.  dD/dmu =
// beta M, so this is the exact derivative step that makes Tr P = 2 n_occ.  A
// Tr M at or below tol (the storage's trace resolution; 0 for FP64) carries no
// information, so no step is taken.
__global__ void k_trace_fix(const double *trD, const double *trM, double n_occ, double tol, double *c) {
  if (threadIdx.x) return;
  *c = (*trM > tol) ? (n_occ - *trD) / *trM : 0.0;
}
template <typename T>
__global__ void k_finalize_P(size_t n2, const T *D, const T *M, const double *c, double *P) {
  const double cv = *c;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n2;
       i += (size_t)gridDim.x * blockDim.x)
    P[i] = 2.0 * ((double)D[i] + cv * (double)M[i]);
}

// electronic entropy S/k_B = -sum [f ln f + (1-f) ln(1-f)] over one-spin levels
// (eq. 4) with f from eq. 7, written through x = beta (eps - mu) as
// ln(1 + e^-|x|) + |x| e^-|x| / (1 + e^-|x|), which is exact and cannot overflow
__global__ void k_entropy_partial(int n, const double *eps, double mu, double beta, double *part) {
  double v = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double ax = fabs(beta * (eps[i] - mu));
    const double e = exp(-ax);
    v += log1p(e) + ax * e / (1.0 + e);
  }
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  __shared__ double sh[4];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}
__global__ void k_sum_fixed(int m, const double *part, double *out) {
  if (threadIdx.x) return;
  double s = 0.0;
  for (int i = 0; i < m; ++i) s += part[i];
  *out = s;
}

// copy the dots results into row k of O and rhs; <W_k, W_k> is the squared
// norm of the next Krylov source
__global__ void k_store_orow(int k, const double *d, double *O, double *rhs, double *src_sq) {
  if (threadIdx.x) return;
  for (int j = 0; j <= k; ++j) {
    O[k * 32 + j] = d[j];
    O[j * 32 + k] = d[j];
  }
  rhs[k] = d[k + 1];
  *src_sq = d[k];
}

// normalisation of Krylov direction k on the device: scale = 1/|v| unless
// |v| <= 1e-12 |source| (breakdown: the rank is recorded, later directions get
// scale 0 and the solve uses the leading basis only)
__global__ void k_kscale(int k, double *ctl) {
  if (threadIdx.x) return;
  if (ctl[3] >= 0.0) {
    ctl[2] = 0.0;
    return;
  }
  const double nv = sqrt(ctl[0]);
  if (nv > 1e-12 * sqrt(ctl[1])) {
    ctl[2] = 1.0 / nv;
  } else {
    ctl[2] = 0.0;
    ctl[3] = k;
  }
}
__global__ void k_kinit(double *ctl, double w0sq) {
  if (threadIdx.x) return;
  ctl[0] = 0.0;
  ctl[1] = w0sq;
  ctl[2] = 0.0;
  ctl[3] = -1.0;
}

inline void cheb_lin(double lmax, double &a, double &b, double &e0) {
  // a + b*lambda minimising max |1 - lambda (a + b lambda)| on [1, lmax]
  const double d = lmax - 1.0;
  if (d < 1e-12) {
    a = 1.0;
    b = 0.0;
    e0 = d;
    return;
  }
  const double s = (lmax + 1.0) / d;
  const double t2 = 2.0 * s * s - 1.0;
  const double c2 = 8.0 / (d * d) / t2;
  const double c1 = -8.0 * (lmax + 1.0) / (d * d) / t2;
  a = -c1;
  b = -c2;
  e0 = 1.0 / t2;
}

}  // namespace

struct xlbomd_ctx {
  int N = 0, n = 0;
  size_t n2 = 0;
  double n_elec = 0, n_occ = 0, beta = 0;
  xlbomd_params prm{};
  xlbomd_model model{};
  hipStream_t s = nullptr;
  int device = 0;               // the device current at create
  int prec = 0;                 // precision as requested at create
  int prec_dm = 0, prec_rs = 0; // Fermi chain + mu shift / response chains
  int is32 = 0, rs32 = 0;       // FP32 storage of the Fermi-chain / response-chain matrices
  size_t esz = 8;
  std::string err;
  bool geom = false;
  // device buffers
  double *R = nullptr, *onecenter = nullptr, *j55 = nullptr;
  float *noise_t = nullptr;
  double *part = nullptr, *pk3 = nullptr, *fpart = nullptr, *epart = nullptr;
  double *dscal = nullptr, *red = nullptr, *frc = nullptr;
  double *lq = nullptr, *lw = nullptr;  // Lanczos vectors ((K+1) x n) and product
  const double **dptr = nullptr;  // device pointer arrays (for lincomb / orth)
  // chain storage (chain element type)
  void *Yc[LMAX + 1] = {}, *Zc[LMAX] = {};
  void *Vst = nullptr, *Pst = nullptr, *Sst = nullptr, *S2st = nullptr, *Bst = nullptr;
  void *D = nullptr, *M = nullptr;
  double shift_c = 1.0;  // prod c_k of the last chemical-potential shift
  bool fix_pending = false;  // mu_shift left a first-order step in slot S_FIX + 1
  // response-precision copies of the cached chain (alias the above when the
  // two chains share a precision), made on the first response after a chain
  void *Yr[LMAX] = {};
  void *Vr = nullptr, *Pr = nullptr, *Sr = nullptr, *S2r = nullptr, *Br = nullptr, *Mr = nullptr;
  void *Wr = nullptr;  // W = 2^(L/2) Qs prod_i Z_i, response precision (Qs: see mu_shift)
  bool resp_copy = false;
  bool resp_ready = false;
  void *w[8] = {};
  int L = 0;
  int Lalloc = 0;  // chain levels with storage (grown on demand up to LMAX)
  int mu_passes = 0;
  bool chain_valid = false;
  bool chain_nonorth = false;  // the cached chain is of F_perp (xlbomd_fermi_dm_nonorth)
  double mu_chain = 0.0;
  // Trace tolerance of the chemical-potential passes.  With FP32 storage of the
  // Fermi chain, Tr D and Tr D(I - D) carry the chain's rounding; in a strongly
  // gapped state Tr D(I - D) = sum f(1 - f) falls to that level and a Newton
  // step on it chases noise, while any mu in the gap gives the same D to that
  // precision.  A trace within trace_tol of N_occ therefore takes no shift and
  // the FP64 first-order correction of the result finishes.  0 with FP64
  // storage.
  double trace_tol = 0.0;
  // FP64 work
  double *f64[6] = {};
  double *Vk[MMAX] = {}, *Wk[MMAX] = {};
  int kalloc = 0;
  // non-orthogonal basis: four FP64 n x n work matrices, allocated by the
  // first call that needs them
  double *no_w[4] = {};
  // entropy diagnostic: FP64 eigenvalues of F (library eigenvalue solve)
  hipsolverHandle_t solver = nullptr;
  double *eig = nullptr, *eig_work = nullptr;
  int *eig_info = nullptr;
  int eig_lwork = 0;
  // stats and optional per-launch timing (HIP events on the handle's stream)
  long long n_gemm = 0;
  bool prof = false;
  std::vector<hipEvent_t> evpool;
  struct Rec { int cls; int ev; double work; };
  std::vector<Rec> recs;
};

namespace {

xlbomd_status fail(xlbomd_ctx *c, xlbomd_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return st;
}

#define HIPCHK(c, x)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess)                                                                \
      return fail(c, XLBOMD_E_HIP, "%s failed: %s", #x, hipGetErrorString(e_));          \
  } while (0)

bool dev_alloc(void **p, size_t bytes) { return hipMalloc(p, bytes) == hipSuccess; }

// kernel classes of the timing hooks: GEMMs by precision and output kind (each
// class is one kernel at a given n), then the pair passes
enum {
  PC_GEMM64 = 0,      // + sym: FP64 full / symmetric output
  PC_GEMMS = 2,       // + 2 (prec - 1) + sym: BF16x3, BF16x6, FP16x3 split, full / symmetric
  PC_FOCK = 8,
  PC_FORCE = 9,
  PC_N = 10
};

int prof_begin(xlbomd_ctx *c) {
  if (!c->prof) return -1;
  const int e = (int)c->recs.size() * 2;
  if (e + 2 > (int)c->evpool.size()) return -1;
  hipEventRecord(c->evpool[e], c->s);
  return e;
}
void prof_end(xlbomd_ctx *c, int e, int cls, double work) {
  if (e < 0) return;
  hipEventRecord(c->evpool[e + 1], c->s);
  c->recs.push_back({cls, e, work});
}

// ------------------------------------------------------------------ GEMM helper
void mm_p(xlbomd_ctx *c, int prec, const void *A, const void *B, void *out, double alpha, int sym,
        const void *C1 = nullptr, double b1 = 0.0, const void *C2 = nullptr, double b2 = 0.0,
        double gamma = 0.0, int btrans = 0, const void *A2 = nullptr, const void *B2 = nullptr) {
  GemmArgs g{};
  g.n = c->n;
  g.nprod = A2 ? 2 : 1;
  g.A[0] = A;
  g.B[0] = B;
  g.A[1] = A2;
  g.B[1] = B2;
  g.btrans = btrans;
  g.C1 = C1;
  g.C2 = C2;
  g.out = out;
  g.alpha = alpha;
  g.beta1 = b1;
  g.beta2 = b2;
  g.gamma = gamma;
  g.sym = sym;
  const int e = prof_begin(c);
  if (prec == XLBOMD_FP64)
    gemm_f64(g, c->s);
  else
    gemm_split(g, prec, c->s);
  // profiled work: executed MFMA flops (a split product runs 3 or 6 MFMA products)
  const double n = (double)c->n;
  const double parts = prec == XLBOMD_FP64 ? 1.0 : (prec == XLBOMD_BF16X6 ? 6.0 : 3.0);
  const int cls = (prec == XLBOMD_FP64 ? PC_GEMM64 : PC_GEMMS + 2 * (prec - 1)) + (sym ? 1 : 0);
  prof_end(c, e, cls, parts * g.nprod * (sym ? 1.0 : 2.0) * n * n * n);
  ++c->n_gemm;
}

// GEMM in the Fermi-chain precision
void mm(xlbomd_ctx *c, const void *A, const void *B, void *out, double alpha, int sym,
        const void *C1 = nullptr, double b1 = 0.0, const void *C2 = nullptr, double b2 = 0.0,
        double gamma = 0.0, int btrans = 0, const void *A2 = nullptr, const void *B2 = nullptr) {
  mm_p(c, c->prec_dm, A, B, out, alpha, sym, C1, b1, C2, b2, gamma, btrans, A2, B2);
}
// GEMM in the response-chain precision
void mr(xlbomd_ctx *c, const void *A, const void *B, void *out, double alpha, int sym,
        const void *C1 = nullptr, double b1 = 0.0, const void *C2 = nullptr, double b2 = 0.0,
        double gamma = 0.0, int btrans = 0, const void *A2 = nullptr, const void *B2 = nullptr) {
  mm_p(c, c->prec_rs, A, B, out, alpha, sym, C1, b1, C2, b2, gamma, btrans, A2, B2);
}

PairSys pairsys(xlbomd_ctx *c);

// algorithmic HBM bytes of one pair pass: the FP32 noise blocks, two n x n FP64
// matrices read or written (P and F, or P0 and X)
// Algorithmic HBM bytes of the pair passes.  Both read the 55 FP32 noise
// values of every atom pair (220 B) and, of each symmetric n x n input, only
// the atom blocks on and above the diagonal (16 doubles per block).  The Fock
// build writes all of F; the force pass writes O(N) values.
double fock_bytes(xlbomd_ctx *c) {
  const double np = 0.5 * c->N * (c->N - 1.0);
  return 220.0 * np + 128.0 * (np + c->N) + 8.0 * (double)c->n2;
}
double force_bytes(xlbomd_ctx *c) {
  const double np = 0.5 * c->N * (c->N - 1.0);
  return 220.0 * np + 2.0 * 128.0 * (np + c->N);
}

void fock_t(xlbomd_ctx *c, const double *P, double *F, int include_h) {
  const int e = prof_begin(c);
  fock(pairsys(c), P, F, include_h, c->part, c->s);
  prof_end(c, e, PC_FOCK, fock_bytes(c));
}

PairSys pairsys(xlbomd_ctx *c) {
  PairSys p{};
  p.n_atoms = c->N;
  p.n_tiles = (c->N + 15) / 16;
  p.R = c->R;
  p.onecenter = c->onecenter;
  p.noise_t = c->noise_t;
  p.j55 = c->j55;
  const xlbomd_model &m = c->model;
  p.eps_s = m.eps_s;
  p.eps_p = m.eps_p;
  p.t0 = m.t0;
  p.r0_hop = m.r0_hop;
  p.lam_hop = m.lam_hop;
  p.coul_k = m.coul_k;
  p.coul_a = m.coul_a;
  p.noise_amp = m.noise_amp;
  p.z_core = m.z_core;
  p.a_rep = m.a_rep;
  p.r0_rep = m.r0_rep;
  p.rho_rep = m.rho_rep;
  return p;
}

xlbomd_status get_scalars(xlbomd_ctx *c, int slot, int cnt, double *out) {
  HIPCHK(c, hipMemcpyAsync(out, c->dscal + slot, sizeof(double) * cnt, hipMemcpyDeviceToHost, c->s));
  HIPCHK(c, hipStreamSynchronize(c->s));
  return XLBOMD_OK;
}
// two groups of slots behind one synchronisation
xlbomd_status get_scalars2(xlbomd_ctx *c, int slot1, int cnt1, double *out1, int slot2, int cnt2, double *out2) {
  HIPCHK(c, hipMemcpyAsync(out1, c->dscal + slot1, sizeof(double) * cnt1, hipMemcpyDeviceToHost, c->s));
  return get_scalars(c, slot2, cnt2, out2);
}

// Newton-Schulz stopping bound (a-priori error of each inverse).  In FP64 the
// relative error of every level's inverse passes unamplified into Y for the
// levels near mu, so L levels at 3e-12 keep D within ~1e-11 of the exact
// Fermi matrix.
double eps_for_prec(int prec) {
  switch (prec) {
    case XLBOMD_FP64: return 3e-12;
    case XLBOMD_BF16X6: return 1e-8;
    case XLBOMD_FP16X3: return 1e-7;
    default: return 1e-6;
  }
}

inline void split_prec(int prec, int &dm, int &rs) {
  switch (prec) {
    case XLBOMD_DM64_BF16X3: dm = XLBOMD_FP64; rs = XLBOMD_BF16X3; break;
    case XLBOMD_DM64_BF16X6: dm = XLBOMD_FP64; rs = XLBOMD_BF16X6; break;
    case XLBOMD_DM64_FP16X3: dm = XLBOMD_FP64; rs = XLBOMD_FP16X3; break;
    default: dm = rs = prec; break;
  }
}

// Bounds [lo, hi] on the spectrum of the symmetric F.  K Lanczos steps give
// Ritz values theta_min, theta_max and their residual norms
// r = beta_K |s_K| (s the Ritz vector of the tridiagonal); the bounds are
// theta -/+ (r + 1e-3 (theta_max - theta_min)), clipped to the Gershgorin
// interval, which is rigorous but much wider for large clusters.  The chain
// depth L grows with log2 of the bound, so each factor of two saved is one
// recursion level less in the density matrix and in every response.  The
// Lanczos start vector (row 0 of lq) is written once at create.
xlbomd_status spectral_bounds(xlbomd_ctx *c, const double *F, double lohi[2], double *gersh = nullptr) {
  const int n = c->n;
  gershgorin(n, F, c->dscal + S_LOHI, c->red, c->s);
  const int K = std::min(LANCZOS_K, n);
  lanczos(n, K, F, c->lq, c->lw, c->dscal + S_LANC, c->s);
  double g[2], ab[2 * LANCZOS_K];
  xlbomd_status st = get_scalars2(c, S_LOHI, 2, g, S_LANC, 2 * K, ab);
  if (st) return st;
  if (!bounds_from_lanczos(g, ab, K, n, lohi)) return fail(c, XLBOMD_E_NONFINITE, "non-finite Fock matrix");
  if (gersh) {
    gersh[0] = g[0];
    gersh[1] = g[1];
  }
  return XLBOMD_OK;
}

// ------------------------------------------------------------------ Fermi chain
// D = (exp(beta (F - mu I)) + I)^-1 (one spin) by the centred tanh-doubling
// recursion Y_{i+1} = 2 Y_i (I + 4 Y_i^2)^-1 started from a degree-9 Taylor
// polynomial of tanh at v = -beta (F - mu)/2^(L+1); D = I/2 + Y_L.  The inverse
// of every level is a Newton-Schulz iteration started from the best linear
// polynomial of T = I + 4 Y^2 on its spectral interval; in the FP64 chain of
// the mixed modes that iteration runs in split precision and Y_{i+1} takes one
// FP64 residual correction instead.
// Storage of chain levels Lalloc .. L - 1 (Y up to Y_L); levels are kept once allocated.
bool ensure_levels(xlbomd_ctx *c, int L) {
  const size_t mb = c->n2 * c->esz, m4 = c->n2 * 4;
  for (int i = c->Lalloc; i < L; ++i) {
    if (!c->Yc[i + 1] && !dev_alloc(&c->Yc[i + 1], mb)) return false;
    if (!c->Zc[i] && !dev_alloc(&c->Zc[i], mb)) return false;
    if (c->resp_copy && !c->Yr[i] && !dev_alloc(&c->Yr[i], m4)) return false;
  }
  if (L > c->Lalloc) c->Lalloc = L;
  return true;
}

xlbomd_status run_chain(xlbomd_ctx *c, const double *F, double mu, double lo, double hi) {
  const int n = c->n;
  c->resp_ready = false;
  const double beta = c->beta;
  const double rho = beta * std::max(hi - mu, mu - lo) / 2.0;
  int L = (int)std::ceil(std::log2(std::max(rho / VMAX, 1.0)));
  if (L < LMIN) L = LMIN;
  if (L > LMAX) return fail(c, XLBOMD_E_ARG, "spectral range too wide (needs %d levels)", L);
  if (!ensure_levels(c, L)) return fail(c, XLBOMD_E_NOMEM, "no memory for %d chain levels", L);
  c->L = L;
  const double vb = std::min(rho / std::ldexp(1.0, L), VMAX);
  const double sc = -beta / std::ldexp(1.0, L + 1);
  void *V = c->Vst, *S = c->Sst, *S2 = c->S2st, *B = c->Bst, *P = c->Pst;
  // V = sc (F - mu I), in chain precision
  if (c->is32) {
    convert((int)c->n2, F, 0, c->w[0], 1, c->s);
    axpbyI_dev(n, nullptr, sc, c->w[0], nullptr, 0.0, nullptr, nullptr, -sc * mu, V, 1, c->s);
  } else {
    axpbyI_dev(n, nullptr, sc, F, nullptr, 0.0, nullptr, nullptr, -sc * mu, V, 0, c->s);
  }
  mm(c, V, V, S, 1.0, 1);                                   // S = V^2
  mm(c, S, S, S2, 1.0, 1);                                  // S2 = S^2
  axpbyI_dev(n, nullptr, TC3, S, nullptr, TC4, S2, nullptr, TC2, B, c->is32, c->s);  // c2 + c3 S + c4 S2
  mm(c, S2, B, P, 1.0, 1, S, TC1, nullptr, 0.0, TC0);       // P = c0 + c1 S + S2 B
  mm(c, V, P, c->Yc[0], 0.5, 1);                            // Y0 = V P / 2
  const double vb2 = vb * vb;
  double yb = 0.5 * vb * (TC0 + vb2 * (TC1 + vb2 * (TC2 + vb2 * (TC3 + vb2 * TC4))));
  const double eps = eps_for_prec(c->prec_dm);
  const bool mixed = c->prec_dm == XLBOMD_FP64 && c->resp_copy;
  const int n2i = (int)c->n2;
  for (int i = 0; i < L; ++i) {
    void *Y = c->Yc[i];
    void *Si = c->w[1], *E = c->w[2], *Za = c->w[3], *Zb = c->w[4];
    mm(c, Y, Y, Si, 1.0, 1);
    double a, b, e0;
    cheb_lin(1.0 + 4.0 * yb * yb, a, b, e0);
    if (mixed) {
      // Split-precision inverse Z ~ T^-1 to ~sqrt(eps) by Newton-Schulz (it
      // corrects itself: start in BF16x3, steps in BF16x6); the FP64 accuracy
      // comes from one residual correction of Y_{i+1} below.
      const size_t half = c->n2 * 4;
      void *S32 = c->w[5], *E32 = (char *)c->w[5] + half, *Za32 = c->w[6], *Zb32 = (char *)c->w[6] + half,
           *C32 = c->w[7];
      convert(n2i, Si, 0, S32, 1, c->s);
      mm_p(c, XLBOMD_BF16X3, S32, S32, E32, -16.0 * b, 1, S32, -(4.0 * a + 8.0 * b), nullptr, 0.0, 1.0 - a - b);
      mm_p(c, XLBOMD_BF16X3, S32, E32, Za32, 4.0 * b, 1, S32, 4.0 * b, E32, a + b, a + b);
      // Steps of order 2, Z <- Z (I + E), or 3, Z <- Z (I + E + E^2) with
      // E' = E E + E: two or three products for error e^2 or e^3.  Each step
      // takes order 2 if that reaches the target, else order 3.  Only the
      // residual E = I - T Z is a cancellation (BF16x6); the correction
      // products act on a quantity of size e and run in BF16x3, adding
      // ~2e-5 e to the error.
      double el = e0 * e0 + 2e-5;  // + BF16x3 rounding
      const double target = std::sqrt(eps);
      for (int it = 0; it < 8 && el > target; ++it) {
        mm_p(c, XLBOMD_BF16X6, S32, Za32, E32, -4.0, 1, Za32, -1.0, nullptr, 0.0, 1.0);  // E = I - T Z
        const double e1 = el;
        if (el * el + 1e-7 + 2e-5 * e1 > target) {
          mm_p(c, XLBOMD_BF16X3, E32, E32, Zb32, 1.0, 1, E32, 1.0);                   // E' = E E + E
          std::swap(E32, Zb32);
          el = el * el * el;
        } else {
          el = el * el;
        }
        el += 1e-7 + 2e-5 * e1;
        mm_p(c, XLBOMD_BF16X3, Za32, E32, Zb32, 1.0, 1, Za32, 1.0);                   // Z + Z E
        std::swap(Za32, Zb32);
      }
      // Y_{i+1} = 2 T^-1 Y by one residual correction of the split solve
      // Y0 = 2 Z Y: R = 2 Y - T Y0 in FP64 (a cancellation), Y_{i+1} = Y0 + Z R,
      // which leaves (I - Z T)(Y0 - 2 T^-1 Y), the square of the split error
      // (Y0 and Z R in BF16x6: with Y0 in BF16x3 the 840-atom D moves 1.1e-10
      // from the exact Fermi matrix, errors near mu growing by 2^(L-i)).
      // Z and Y0 are functions of the FP32-rounded S and Y, so T Y0 is
      // symmetric only to ~1e-7 and R is not symmetric: R is formed in full,
      // and the split GEMM (which takes its second operand transposed) gets R^T.
      // Y32 (the FP32 Y_i, kept as the response's copy) is the previous level's
      // by-product, except at level 0
      void *Y32 = c->Yr[i], *Yn32 = E32, *Yn = Za, *R = E;
      if (i == 0) convert(n2i, Y, 0, Y32, 1, c->s);
      mm_p(c, XLBOMD_BF16X6, Za32, Y32, Yn32, 2.0, 1);         // Y0 = 2 Z Y
      convert(n2i, Yn32, 1, Yn, 0, c->s);
      mm(c, Si, Yn, R, -4.0, 0, Yn, -1.0, Y, 2.0);             // R = 2 Y - Y0 - 4 S Y0 in FP64
      convert_t(n, (const double *)R, (float *)E32, c->s);
      mm_p(c, XLBOMD_BF16X6, Za32, E32, C32, 1.0, 0);          // Z R
      // Y0 + Z R, with its FP32 copy for the next level.  Z R is symmetric only
      // to ~1e-13 relative; every level rebuilds Y_{i+1} from the symmetric Y0,
      // so only the last one (which gives D) is symmetrised.
      add_mixed(n2i, (const double *)Yn, (const float *)C32, (double *)c->Yc[i + 1],
                i + 1 < L ? (float *)c->Yr[i + 1] : nullptr, c->s);
      if (i + 1 == L) symmetrize(n, c->Yc[L], 0, c->s);
      // the FP32 Z_i is what the response needs
      convert(n2i, Za32, 1, c->Zc[i], 1, c->s);
    } else {
      // E0 = I - a T - b T^2 with T = I + 4S, T^2 = I + 8S + 16 S^2
      mm(c, Si, Si, E, -16.0 * b, 1, Si, -(4.0 * a + 8.0 * b), nullptr, 0.0, 1.0 - a - b);
      // Z1 = Z0 (I + E0), Z0 = (a + b) I + 4 b S
      mm(c, Si, E, Za, 4.0 * b, 1, Si, 4.0 * b, E, a + b, a + b);
      // steps of order 2 (Z + Z E) where that reaches the level's target,
      // else of order 3 (Z + Z E' with E' = E E + E: three products for e^3).
      // The later levels amplify this level's error by up to 2^(L-1-i) for
      // states near mu; eps is set for up to five of them, and deeper chains
      // (cold systems) tighten the target of their early levels to match.
      const double eps_i = eps * std::ldexp(1.0, std::min(0, 5 - (L - 1 - i)));
      void *E2 = c->w[5];
      double el = e0 * e0;
      for (int it = 0; it < 8 && el > eps_i; ++it) {
        mm(c, Si, Za, E, -4.0, 1, Za, -1.0, nullptr, 0.0, 1.0);   // E = I - T Z
        const void *Ec = E;
        if (el * el > eps_i) {
          mm(c, E, E, E2, 1.0, 1, E, 1.0);                        // E' = E E + E
          Ec = E2;
          el = el * el * el;
        } else {
          el = el * el;
        }
        mm(c, Za, Ec, Zb, 1.0, 1, Za, 1.0);                       // Z <- Z + Z E
        std::swap(Za, Zb);
      }
    }
    if (!mixed) {
      // keep Z_i in the cache
      if (Za != c->w[3]) std::swap(c->w[3], c->w[4]);
      std::swap(c->Zc[i], c->w[3]);
      mm(c, Y, c->Zc[i], c->Yc[i + 1], 2.0, 1);
    }
    yb = 2.0 * yb / (1.0 + 4.0 * yb * yb);
  }
  // D = I/2 + Y_L
  axpbyI_dev(n, nullptr, 1.0, c->Yc[L], nullptr, 0.0, nullptr, nullptr, 0.5, c->D, c->is32, c->s);
  c->mu_chain = mu;
  return XLBOMD_OK;
}

// Exact chemical-potential shift: D(mu + dmu) = D (c I + (1 - c) D)^-1 with
// c = exp(-beta dmu), applied in passes.  Pass 1 solves the trace series
// sum_k (1-c)^k Tr[D (I-D)^k] = N_occ (k < 6); every later pass is a Newton step
// dmu = (N_occ - Tr D) / (beta Tr D(I-D)).  Each pass is clamped to
// |beta dmu| <= 0.3 and is followed by its exact shift, so a poor warm start
// costs a few shifts instead of a new chain.  Leaves D, M = D(I - D) and
// shift_c = prod c_k (the response's Qs follows from it and D); *dmu_out gets
// the total.
// Returns XLBOMD_E_NOCONV (without changing mu) if the passes run out.
xlbomd_status mu_shift(xlbomd_ctx *c, double *dmu_out) {
  const int n = c->n, i32 = c->is32;
  c->resp_ready = false;
  hipStream_t s = c->s;
  xlbomd_status st;
  void *D = c->D, *D2 = c->w[0], *D3 = c->w[1], *Mx = c->w[2], *Nx = c->w[3], *N2 = c->w[4],
       *MN = c->w[5], *N3 = c->w[6];
  mm(c, D, D, D2, 1.0, 1);
  mm(c, D, D2, D3, 1.0, 1);
  axpby((int)c->n2, 1.0, D, -1.0, D2, Mx, i32, s);                                  // M
  axpbyI_dev(n, nullptr, -1.0, D, nullptr, 0.0, nullptr, nullptr, 1.0, Nx, i32, s);  // N = I - D
  axpbyI_dev(n, nullptr, -2.0, D, nullptr, 1.0, D2, nullptr, 1.0, N2, i32, s);      // N^2
  axpbyI_dev(n, nullptr, 1.0, D, nullptr, -2.0, D2, nullptr, 0.0, MN, i32, s);      // D - 2D^2
  axpby((int)c->n2, 1.0, MN, 1.0, D3, MN, i32, s);                                  // + D^3
  {
    const void *Xs[4] = {D, D2, D3, nullptr};
    const double a[4] = {-3.0, 3.0, -1.0, 0.0};
    poly_comb(n, Xs, a, 1.0, N3, i32, s);                                           // N^3
  }
  trace(n, D, c->dscal + S_TAU, i32, c->red, s);
  trace(n, Mx, c->dscal + S_TAU + 1, i32, c->red, s);
  {
    // Tr D N^k for k = 2..5 as Frobenius products of symmetric matrices
    const void *X[4] = {Mx, Mx, MN, MN};
    const void *Y[4] = {Nx, N2, N2, N3};
    dots((int)c->n2, 4, X, Y, c->dscal + S_TAU + 2, i32, c->red, s);
  }
  mu_series_solve(c->dscal + S_TAU, c->n_occ, c->beta, c->trace_tol, c->dscal + S_MU1, s);
  // Each pass shifts D exactly to D(mu + dmu) = D Q^-1, Q = c I + (1 - c) D,
  // c = exp(-beta dmu): pass 0 with dmu from the trace series, later passes
  // with a (clamped) Newton step on Tr D.  A large step inverts Q by
  // Newton-Schulz; the passes end with a small step taken as a truncated
  // series in D.  The shifts compose: c multiplies.
  double dmu_total = 0.0, cprod = 1.0;
  bool done = false, wide = false;
  c->mu_passes = 0;
  for (int pass = 0; pass < 8 && !done; ++pass) {
    double mres[5];
    bool have_d3 = pass == 0;  // D2 = D^2 (and D3 = D^3 in pass 0) are current
    if (pass > 0) {
      // Newton step from Tr D and Tr D(I - D)
      void *Mt = c->w[1];
      mm(c, D, D, D2, 1.0, 1);
      axpby((int)c->n2, 1.0, D, -1.0, D2, Mt, i32, s);
      trace(n, D, c->dscal + S_T01, i32, c->red, s);
      trace(n, Mt, c->dscal + S_T01 + 1, i32, c->red, s);
      mu_newton(c->dscal + S_T01, c->n_occ, c->beta, c->trace_tol, c->dscal + S_MU1, s);
    }
    if ((st = get_scalars(c, S_MU1, 5, mres))) return st;
    c->mu_passes = pass + 1;
    const bool clamped = mres[3] != 0.0;
    const double cc = mres[1];
    // The series step ends the passes.  After pass 0 (trace series with k < 6)
    // Tr D misses N_occ by O((1 - c)^6), after a Newton pass by O(dmu^2); the
    // first-order trace correction applied afterwards leaves the square of
    // that, so pass 0 may take the series for |1 - c| up to 8e-2, a Newton pass
    // for |1 - c| up to 1e-3.
    const double ser_max = pass == 0 ? 8e-2 : 1e-3;
    if (!clamped && std::fabs(1.0 - cc) <= ser_max) {
      wide = std::fabs(1.0 - cc) > 1e-3;
      // D Q^-1 = (1/c) sum_{k<=K} (-r)^k D^(k+1), r = (1 - c)/c, with K the
      // least order whose remainder |r|^(K+1) / (1 - |r|) is below 1e-13 (K <= 15)
      const double r = (1.0 - cc) / cc, ar = std::fabs(r);
      int K = 0;
      for (double rem = ar; K < 15 && rem / (1.0 - ar) > 1e-13; rem *= ar) ++K;
      const int deg = K + 1;
      double p[17] = {};  // p[j]: coefficient of D^j
      for (int k = 0; k <= K; ++k) p[k + 1] = std::pow(-r, k) / cc;
      void *D4 = c->w[2];
      if (!have_d3 && deg >= 3) mm(c, D, D2, D3, 1.0, 1);
      if (deg >= 4) mm(c, D2, D2, D4, 1.0, 1);
      if (deg <= 4) {
        const void *Xs[4] = {D, D2, deg >= 3 ? D3 : nullptr, deg >= 4 ? D4 : nullptr};
        const double a[4] = {p[1], p[2], p[3], p[4]};
        poly_comb(n, Xs, a, 0.0, D, i32, s);  // D <- D Q^-1 in place
      } else {
        // Horner in D^4 over blocks B_m = sum_{i<4} p[4m+i] D^i (the top block
        // also takes p[4H+4] D^4): p(D) = B_0 + D^4 (B_1 + D^4 (.. + D^4 B_H))
        const int H = (deg - 1) / 4;
        const void *Xs[4] = {D, D2, D3, D4};
        void *acc = c->w[3], *blk = c->w[4], *nxt = c->w[5];
        {
          const double a[4] = {p[4 * H + 1], p[4 * H + 2], p[4 * H + 3], 4 * H + 4 <= 16 ? p[4 * H + 4] : 0.0};
          poly_comb(n, Xs, a, p[4 * H], acc, i32, s);
        }
        for (int m = H - 1; m >= 0; --m) {
          const double a[4] = {p[4 * m + 1], p[4 * m + 2], p[4 * m + 3], 0.0};
          poly_comb(n, Xs, a, p[4 * m], blk, i32, s);
          void *out = m == 0 ? D : nxt;
          mm(c, D4, acc, out, 1.0, 1, blk, 1.0);
          std::swap(acc, nxt);
        }
      }
      done = true;
    } else {
      // inverse of Q (spectrum in [min(c,1), max(c,1)]) by Newton-Schulz from
      // the Chebyshev-optimal linear start Z0 = z0 I + z1 D; the first step
      // Z1 = Z0 (2I - Q Z0) is a cubic polynomial in D
      const double lmin = std::min(cc, 1.0), kap = std::max(cc, 1.0) / lmin;
      double ca, cb, e0;
      cheb_lin(kap, ca, cb, e0);
      const double z0 = ca / lmin + cb * cc / (lmin * lmin), z1 = cb * (1.0 - cc) / (lmin * lmin);
      const double p0 = 2.0 - cc * z0, p1 = -((1.0 - cc) * z0 + cc * z1), p2 = -(1.0 - cc) * z1;
      void *Za, *Zb, *E;
      if (have_d3) {
        const void *Xs[4] = {D, D2, D3, nullptr};
        const double co[4] = {z0 * p1 + z1 * p0, z0 * p2 + z1 * p1, z1 * p2, 0.0};
        Za = c->w[2];
        Zb = c->w[3];
        E = c->w[4];
        poly_comb(n, Xs, co, z0 * p0, Za, i32, s);
      } else {
        void *Z0 = c->w[2], *Pp = c->w[1];
        const void *X0s[4] = {D, nullptr, nullptr, nullptr};
        const double c0[4] = {z1, 0.0, 0.0, 0.0};
        poly_comb(n, X0s, c0, z0, Z0, i32, s);
        const void *X1s[4] = {D, D2, nullptr, nullptr};
        const double c1[4] = {p1, p2, 0.0, 0.0};
        poly_comb(n, X1s, c1, p0, Pp, i32, s);  // 2I - Q Z0
        mm(c, Z0, Pp, c->w[3], 1.0, 1);
        Za = c->w[3];
        Zb = c->w[2];
        E = c->w[1];
      }
      double e = e0 * e0;
      const double eps = eps_for_prec(c->prec_dm);
      for (int it = 0; it < 8 && e > eps; ++it) {
        mm(c, D, Za, E, -(1.0 - cc), 1, Za, -cc, nullptr, 0.0, 1.0);  // E = I - Q Z
        mm(c, Za, E, Zb, 1.0, 1, Za, 1.0);                            // Z <- Z + Z E
        std::swap(Za, Zb);
        e = e * e;
      }
      void *Dn = (Za == c->w[2]) ? c->w[3] : c->w[2];
      mm(c, D, Za, Dn, 1.0, 1);
      axpby((int)c->n2, 1.0, Dn, 0.0, nullptr, D, i32, s);
    }
    dmu_total += mres[0];
    cprod *= cc;
  }
  if (!done) return XLBOMD_E_NOCONV;
  c->shift_c = cprod;
  c->fix_pending = wide;
  // M, and D^2, D^3 of the first-order step below, enter D only multiplied by a
  // trace correction f <~ 1e-7, and the response (of split precision in the
  // mixed modes) takes M as it is: with a split response they are products in
  // the response precision (relative error <~ 2e-5, so <~ 2e-12 in D); an FP64
  // response keeps them FP64.
  const bool lowM = c->prec_dm == XLBOMD_FP64 && c->resp_copy;
  const size_t half = c->n2 * 4;
  void *D32 = c->w[3], *P2_32 = (char *)c->w[3] + half, *P3_32 = c->w[4];
  if (lowM) convert((int)c->n2, D, 0, D32, 1, s);
  auto dsq = [&](void *out) {  // out = D^2
    if (lowM) {
      mm_p(c, c->prec_rs, D32, D32, P2_32, 1.0, 1);
      convert((int)c->n2, P2_32, 1, out, 0, s);
    } else {
      mm(c, D, D, out, 1.0, 1);
    }
  };
  if (wide) {
    // A wide series step leaves Tr D off N_occ by up to ~1e-7 Tr M.  Step to the
    // trace to first order, x = beta dmu by f = (N_occ - Tr D) / Tr M (slot
    // S_FIX + 1): D += f M and M += f dM/dx, dM/dx = D - 3 D^2 + 2 D^3, so that
    // D, M and the response's Qs (c <- c e^-f, after the host reads f) describe
    // one chemical potential up to O(f^2).
    void *D2n = c->w[0], *D3n = c->w[1], *Tn = c->w[2];
    dsq(D2n);
    axpby((int)c->n2, 1.0, D, -1.0, D2n, c->M, i32, s);
    if (lowM) {
      mm_p(c, c->prec_rs, D32, P2_32, P3_32, 1.0, 1);
      convert((int)c->n2, P3_32, 1, D3n, 0, s);
    } else {
      mm(c, D, D2n, D3n, 1.0, 1);
    }
    trace(n, c->M, c->dscal + S_TRM, i32, c->red, s);
    trace(n, D, c->dscal + S_TRD, i32, c->red, s);
    hipLaunchKernelGGL(k_trace_fix, dim3(1), dim3(64), 0, s, c->dscal + S_TRD, c->dscal + S_TRM, c->n_occ,
                       c->trace_tol, c->dscal + S_FIX + 1);
    const void *Xs[4] = {D, D2n, D3n, nullptr};
    const double a[4] = {1.0, -3.0, 2.0, 0.0};
    poly_comb(n, Xs, a, 0.0, Tn, i32, s);
    axpbyI_dev(n, nullptr, 1.0, D, c->dscal + S_FIX + 1, 0.0, c->M, nullptr, 0.0, D, i32, s);
    axpbyI_dev(n, nullptr, 1.0, c->M, c->dscal + S_FIX + 1, 0.0, Tn, nullptr, 0.0, c->M, i32, s);
  } else if (lowM) {
    dsq(c->w[0]);
    axpby((int)c->n2, 1.0, D, -1.0, c->w[0], c->M, i32, s);  // M = D - D^2
  } else {
    mm(c, D, D, c->M, -1.0, 1, D, 1.0);                       // M = D - D^2
  }
  trace(n, c->M, c->dscal + S_TRM, i32, c->red, s);
  trace(n, D, c->dscal + S_TRD, i32, c->red, s);
  *dmu_out = dmu_total;
  return XLBOMD_OK;
}

// Response-side factors of the cached chain, made once per chain on its first
// response.  In the eigenbasis of F, level i of the tanh-doubling recursion maps
// a response entry (a, b) by the divided difference of y -> 2y / (1 + 4y^2):
//   2 z_a z_b (1 - 4 y_a y_b),   z = 1 / (1 + 4 y^2),  y = eigenvalues of Y_i,
// and the chemical-potential shift D Q^-1 maps it by qs_a qs_b (qs the
// eigenvalues of Qs).  These are Hadamard factors, so they commute: the z-parts
// and qs collect into W = 2^(L/2) Qs Z_0 ... Z_(L-1) (L products, once per chain)
// and each level keeps only K -> K - 4 Y_i K Y_i (two products per response).
// The shift D -> D Q^-1, Q = c I + (1 - c) D, inverts to Q^-1 = (I - (1 - c) D')/c
// in terms of the shifted D', and shifts compose (c multiplies), so
// Qs = sqrt(c) Q^-1 = (I - (1 - c) D) / sqrt(c) with the cached D and c = shift_c.
void prepare_response(xlbomd_ctx *c) {
  const int n = c->n, n2 = (int)c->n2, L = c->L;
  hipStream_t s = c->s;
  const double rs = 1.0 / std::sqrt(c->shift_c), qa = -(1.0 - c->shift_c) * rs;
  const void *Q = c->w[0];
  // the FP64 chain with split Newton-Schulz keeps its Z_i in FP32
  const bool zc32 = c->prec_dm == XLBOMD_FP64 && c->resp_copy;
  if (c->resp_copy) {
    // the mixed chain leaves its FP32 Y_i in Yr already
    if (!zc32)
      for (int i = 0; i < L; ++i) convert(n2, c->Yc[i], c->is32, c->Yr[i], 1, s);
    convert(n2, c->Vst, c->is32, c->Vr, 1, s);
    convert(n2, c->Pst, c->is32, c->Pr, 1, s);
    convert(n2, c->Sst, c->is32, c->Sr, 1, s);
    convert(n2, c->S2st, c->is32, c->S2r, 1, s);
    convert(n2, c->Bst, c->is32, c->Br, 1, s);
    convert(n2, c->M, c->is32, c->Mr, 1, s);
    convert(n2, c->D, c->is32, c->w[1], 1, s);
    axpbyI_dev(n, nullptr, qa, c->w[1], nullptr, 0.0, nullptr, nullptr, rs, c->w[0], 1, s);
  } else {
    axpbyI_dev(n, nullptr, qa, c->D, nullptr, 0.0, nullptr, nullptr, rs, c->w[0], c->is32, s);
  }
  // W <- sqrt(2) Z_i W for i < L (commuting symmetric factors: symmetric products)
  const void *Wa = Q;
  for (int i = 0; i < L; ++i) {
    const void *Zi = c->Zc[i];
    if (c->resp_copy && !zc32) {
      convert(n2, c->Zc[i], c->is32, c->w[1], 1, s);
      Zi = c->w[1];
    }
    void *dst = i == L - 1 ? c->Wr : (Wa == c->w[2] ? c->w[3] : c->w[2]);
    mr(c, Zi, Wa, dst, std::sqrt(2.0), 1);
    Wa = dst;
  }
  c->resp_ready = true;
}

// canonical response of the cached chain to F1 (FP64, spin-summed F1): P1 = 2 D1,
// or P1 = 2 D1 - sub when sub is given (the Krylov kernel's J V = P1[G(V)] - V)
xlbomd_status response(xlbomd_ctx *c, const double *F1, double *P1, const double *sub = nullptr) {
  const int n = c->n, i32 = c->rs32, L = c->L;
  hipStream_t s = c->s;
  // the Fermi-chain cache itself, or its response-precision copy
  if (!c->resp_ready) prepare_response(c);
  const bool cp = c->resp_copy;
  void *const *Yr = cp ? c->Yr : c->Yc;
  void *Vr = cp ? c->Vr : c->Vst, *Pr = cp ? c->Pr : c->Pst, *Sr = cp ? c->Sr : c->Sst;
  void *S2r = cp ? c->S2r : c->S2st, *Br = cp ? c->Br : c->Bst;
  void *Mr = cp ? c->Mr : c->M, *Wr = c->Wr;
  const double sc = -c->beta / std::ldexp(1.0, L + 1);
  void *V1 = c->w[0], *dS = c->w[1], *dS2 = c->w[2], *Y1 = c->w[3], *G = c->w[4], *H = c->w[5],
       *Y1b = c->w[6];
  if (i32) {
    convert((int)c->n2, F1, 0, V1, 1, s, sc);
  } else {
    axpby((int)c->n2, sc, F1, 0.0, nullptr, V1, 0, s);
  }
  if (i32 && split_sum_by_transpose(c->prec_rs, n)) {
    // A B + B A = (2 A B + (2 A B)^T) / 2 for symmetric A, B (V1 and dS are
    // symmetric: F1, and the average itself)
    mr(c, Vr, V1, dS, 2.0, 0);                                                          // V V1 + V1 V
    symmetrize(n, dS, 1, s);
    mr(c, Sr, dS, dS2, 2.0, 0);                                                         // S dS + dS S
    symmetrize(n, dS2, 1, s);
  } else {
    mr(c, Vr, V1, dS, 1.0, 1, nullptr, 0.0, nullptr, 0.0, 0.0, 0, V1, Vr);          // V V1 + V1 V
    mr(c, Sr, dS, dS2, 1.0, 1, nullptr, 0.0, nullptr, 0.0, 0.0, 0, dS, Sr);          // S dS + dS S
  }
  void *dB = c->w[7], *dP = G;
  axpby((int)c->n2, TC3, dS, TC4, dS2, dB, i32, s);                                       // dB
  // dP = c1 dS + dS2 B + S2 dB (symmetric as a sum: S2 B = B S2)
  mr(c, dS2, Br, dP, 1.0, 1, dS, TC1, nullptr, 0.0, 0.0, 0, S2r, dB);
  mr(c, V1, Pr, Y1, 0.5, 1, nullptr, 0.0, nullptr, 0.0, 0.0, 0, Vr, dP);          // (V1 P + V dP)/2
  // Level i maps a response K to K - 4 Y_i K Y_i (its z-part is in W): G = Y_i K,
  // then Y_i G^T = Y_i K Y_i, symmetric, with K added in the epilogue.
  for (int i = 0; i < L; ++i) {
    mr(c, Yr[i], Y1, G, 1.0, 0);                                                         // G = Y_i K
    mr(c, Yr[i], G, Y1b, -4.0, 1, Y1, 1.0, nullptr, 0.0, 0.0, 1);                        // K - 4 Y_i K Y_i
    std::swap(Y1, Y1b);
  }
  // the z-parts of all levels and the chemical-potential shift: W K W
  mr(c, Wr, Y1, G, 1.0, 0);
  mr(c, Wr, G, H, 1.0, 1, nullptr, 0.0, nullptr, 0.0, 0.0, 1);
  // canonical projection: R - (Tr R / Tr M) M.  An FP64 response takes Tr R
  // from the exact trace of the fixed-mu derivative, Tr f'(F)[F1] =
  // -beta <M, F1> = 2^(L+1) <M, V1> (V1 = sc F1): a product of two accurate
  // matrices, where the trace of the computed R sums n rounded diagonal
  // entries, which the division by Tr M (small when few states lie near mu)
  // amplifies.  A split response keeps the trace of its own R: its error
  // along M (the FP32 chain's own chemical potential) then cancels, and
  // Tr P1 = 0 holds to rounding.
  double tr_scale = 1.0;
  if (c->prec_rs == XLBOMD_FP64) {
    const void *a[1] = {Mr}, *b[1] = {V1};
    dots((int)c->n2, 1, a, b, c->dscal + S_TRR, i32, c->red, s);
    tr_scale = std::ldexp(1.0, L + 1);
  } else {
    trace(n, H, c->dscal + S_TRR, i32, c->red, s);
  }
  hipLaunchKernelGGL(k_canon, dim3(1), dim3(64), 0, s, c->dscal + S_TRR, c->dscal + S_TRM, tr_scale,
                     c->dscal + S_CAN);
  // P1 = 2 (R + s M), s = -Tr R / Tr M, straight into the caller's FP64 buffer
  canon_out((int)c->n2, H, Mr, c->dscal + S_CAN, sub, P1, i32, s);
  return XLBOMD_OK;
}

// One pass of the density matrix at given spectral bounds: chain, chemical-
// potential shift (bisection with new chains when the warm start is far off),
// first-order trace correction into P.  fx: S_FIX, mu_shift's own first-order
// step, Tr P; trd: Tr D before the first-order correction.
xlbomd_status fermi_pass(xlbomd_ctx *c, const double *F, const double lohi[2], double &mu, double *P, double fx[3],
                         double trdm[2]) {
  const int n = c->n;
  xlbomd_status st;
  bool cold = !std::isfinite(mu);
  bool converged = false;
  double bracket = 0.4 / c->beta;
  for (int attempt = 0; attempt < 4 && !converged; ++attempt) {
    if (cold) {
      // bisection on Tr D(mu) with full chains until the bracket is within
      // 0.4/beta; a retry after the shift passes ran out bisects 10x tighter,
      // so that they start closer
      double a = lohi[0], b = lohi[1];
      while (b - a > bracket) {
        const double mid = 0.5 * (a + b);
        if ((st = run_chain(c, F, mid, lohi[0], lohi[1]))) return st;
        trace(n, c->D, c->dscal + S_TRD, c->is32, c->red, c->s);
        double tr;
        if ((st = get_scalars(c, S_TRD, 1, &tr))) return st;
        if (tr < c->n_occ)
          a = mid;
        else
          b = mid;
      }
      mu = 0.5 * (a + b);
      cold = false;
      bracket *= 0.1;
    }
    if ((st = run_chain(c, F, mu, lohi[0], lohi[1]))) return st;
    double dmu = 0.0;
    st = mu_shift(c, &dmu);
    if (st == XLBOMD_E_NOCONV) {
      // far from the warm start: bisection with full chains, then try again
      cold = true;
      continue;
    }
    if (st) return st;
    mu += dmu;
    converged = true;
  }
  if (!converged) return fail(c, XLBOMD_E_NOCONV, "chemical potential search did not converge");
  c->chain_valid = true;
  c->resp_ready = false;
  hipLaunchKernelGGL(k_trace_fix, dim3(1), dim3(64), 0, c->s, c->dscal + S_TRD, c->dscal + S_TRM, c->n_occ,
                     c->trace_tol, c->dscal + S_FIX);
  {
    size_t blocks = std::min<size_t>((c->n2 + 255) / 256, 8192);
    if (c->is32)
      hipLaunchKernelGGL(k_finalize_P<float>, dim3(blocks), dim3(256), 0, c->s, c->n2, (const float *)c->D,
                         (const float *)c->M, c->dscal + S_FIX, P);
    else
      hipLaunchKernelGGL(k_finalize_P<double>, dim3(blocks), dim3(256), 0, c->s, c->n2, (const double *)c->D,
                         (const double *)c->M, c->dscal + S_FIX, P);
  }
  trace(n, P, c->dscal + S_TRP, 0, c->red, c->s);
  // Tr M, Tr D; S_FIX, first-order step of mu_shift, S_TRP
  HIPCHK(c, hipMemcpyAsync(trdm, c->dscal + S_TRM, sizeof(double), hipMemcpyDeviceToHost, c->s));
  return get_scalars2(c, S_TRD, 1, trdm + 1, S_FIX, 3, fx);
}

// A sound chain leaves (a) an electron-count defect |N_occ - Tr D| for the
// first-order trace correction of O((1 - c)^6) or O(dmu^2) times
// Tr D(I - D), far below DEFECT_MAX N_occ, and (b) every eigenvalue of D in
// [0, 1], so Tr D(I - D) >= 0 up to rounding (of the storage: trace_tol with
// FP32).  A chain that fails either is off, e.g. for an eigenvalue of F
// outside the spectral bounds that the chain's start polynomial and a-priori
// Newton-Schulz counts were set for.
constexpr double DEFECT_MAX = 1e-6;
bool chain_sound(const xlbomd_ctx *c, const double tm[2]) {
  return std::fabs(c->n_occ - tm[1]) <= DEFECT_MAX * c->n_occ + c->trace_tol &&
         tm[0] >= -(1e-9 * c->n_occ + 4.0 * c->trace_tol);
}

xlbomd_status fermi(xlbomd_ctx *c, const double *F, double *mu_io, double *P, bool sync_check) {
  c->chain_nonorth = false;
  double lohi[2], gersh[2];
  xlbomd_status st = spectral_bounds(c, F, lohi, gersh);
  if (st) return st;
  double mu = *mu_io, fx[3], tm[2] = {0.0, 0.0};  // tm: Tr M, Tr D
  if ((st = fermi_pass(c, F, lohi, mu, P, fx, tm))) return st;
  if (!chain_sound(c, tm)) {
    // once more on the rigorous Gershgorin interval, from the same warm start
    mu = *mu_io;
    if ((st = fermi_pass(c, F, gersh, mu, P, fx, tm))) return st;
    if (!chain_sound(c, tm))
      return fail(c, XLBOMD_E_NOCONV, "density matrix inconsistent (Tr D - N_occ %.3e, Tr D(I-D) %.3e)",
                  tm[1] - c->n_occ, tm[0]);
  }
  if (c->fix_pending) {
    mu += fx[1] / c->beta;
    c->shift_c *= std::exp(-fx[1]);
    c->fix_pending = false;
  }
  mu += fx[0] / c->beta;
  *mu_io = mu;
  if (sync_check) {
    const double tr = fx[2];
    if (!std::isfinite(tr)) return fail(c, XLBOMD_E_NONFINITE, "non-finite density matrix");
    if (std::fabs(tr - c->n_elec) > 1e-9 * c->n_elec + 4.0 * c->trace_tol)
      return fail(c, XLBOMD_E_NOCONV,
                  "trace %.15g differs from N_e %.15g (Tr D %.15g, Tr D(I-D) %.3e, first-order step %.3e, "
                  "%d levels, %d mu passes)",
                  tr, c->n_elec, tm[1], tm[0], fx[0], c->L, c->mu_passes);
  }
  return XLBOMD_OK;
}

xlbomd_status ensure_krylov(xlbomd_ctx *c, int m) {
  while (c->kalloc < m) {
    const int k = c->kalloc;
    if (!dev_alloc((void **)&c->Vk[k], c->n2 * 8) || !dev_alloc((void **)&c->Wk[k], c->n2 * 8))
      return fail(c, XLBOMD_E_NOMEM, "Krylov workspace allocation failed");
    ++c->kalloc;
    // the basis pointers live on the device for orth_dots / lincomb; uploading
    // them once here keeps pageable copies out of the step
    if (c->kalloc == m &&
        hipMemcpy(c->dptr, c->Vk, sizeof(double *) * c->kalloc, hipMemcpyHostToDevice) != hipSuccess)
      return fail(c, XLBOMD_E_HIP, "Krylov pointer upload failed");
  }
  return XLBOMD_OK;
}

xlbomd_status krylov(xlbomd_ctx *c, const double *X, const double *P0, int m, double tol, double *Y,
                     int *rank_out, double *rel_out, double *w0_out) {
  hipStream_t s = c->s;
  const int n2 = (int)c->n2;
  xlbomd_status st;
  if (m < 0 || m > MMAX) return fail(c, XLBOMD_E_ARG, "m must be in [0, %d]", MMAX);
  if (!c->chain_valid) return fail(c, XLBOMD_E_STATE, "no Fermi chain cached");
  if ((st = ensure_krylov(c, m))) return st;
  double *W0 = c->f64[0], *v = c->f64[1], *tmp = c->f64[2], *F1 = c->f64[3];
  axpby(n2, 1.0, P0, -1.0, X, W0, 0, s);
  {
    const void *a[1] = {W0};
    dots(n2, 1, a, a, c->dscal + S_KRES + 1, 0, c->red, s);
  }
  double nw0sq;
  if ((st = get_scalars(c, S_KRES + 1, 1, &nw0sq))) return st;
  if (w0_out) *w0_out = std::sqrt(nw0sq);
  if (rank_out) *rank_out = 0;
  if (rel_out) *rel_out = 0.0;
  if (m == 0) {
    // original XL-BOMD: the scaled-identity kernel K = -c I
    axpby(n2, -c->prm.kernel_c, W0, 0.0, nullptr, Y, 0, s);
    if (rel_out) *rel_out = nw0sq > 0.0 ? 1.0 : 0.0;
    return XLBOMD_OK;
  }
  axpby(n2, 0.0, W0, 0.0, nullptr, Y, 0, s);
  if (!(nw0sq > 0.0)) return XLBOMD_OK;
  // The basis is built without host round trips: normalisation and the
  // breakdown test run on the device (k_kscale), and the host reads the
  // residual once at the end (per direction only when tol > 0 asks for an
  // early stop).
  double *ctl = c->dscal + S_KCTL;
  hipLaunchKernelGGL(k_kinit, dim3(1), dim3(64), 0, s, ctl, nw0sq);
  const double *src = W0;
  int k = 0;
  double rel = 1.0;
  double kres[3] = {0.0, 0.0, 0.0};
  for (; k < m;) {
    // classical Gram-Schmidt applied twice; the sweeps read the previous W (or
    // W0) in place and write the two work vectors in turn.  The first sweep's
    // update also forms the second sweep's coefficients <V_j, v>, and the
    // second's the squared norm, in the same pass over the elements.
    const double *cur = src;
    if (k > 0) {
      const void *xs[MMAX], *ys[MMAX];
      for (int j = 0; j < k; ++j) {
        xs[j] = c->Vk[j];
        ys[j] = cur;
      }
      for (int j0 = 0; j0 < k; j0 += 16)
        dots(n2, std::min(16, k - j0), xs + j0, ys + j0, c->dscal + S_ORTH + j0, 0, c->red, s);
      orth_dots(n2, k, cur, c->dptr, c->dscal + S_ORTH, v, 0, c->dscal + S_ORTH, c->red, s);
      orth_dots(n2, k, v, c->dptr, c->dscal + S_ORTH, tmp, 1, ctl, c->red, s);
      cur = tmp;
    } else {
      const void *a[1] = {cur};
      dots(n2, 1, a, a, ctl, 0, c->red, s);
    }
    hipLaunchKernelGGL(k_kscale, dim3(1), dim3(64), 0, s, k, ctl);
    axpbyI_dev(c->n, ctl + 2, 0.0, cur, nullptr, 0.0, nullptr, nullptr, 0.0, c->Vk[k], 0, s);
    // W_k = J V_k = P1[G(V_k)] - V_k
    fock_t(c, c->Vk[k], F1, 0);
    if ((st = response(c, F1, c->Wk[k], c->Vk[k]))) return st;
    {
      const void *xs[MMAX + 1], *ys[MMAX + 1];
      for (int j = 0; j <= k; ++j) {
        xs[j] = c->Wk[k];
        ys[j] = c->Wk[j];
      }
      xs[k + 1] = c->Wk[k];
      ys[k + 1] = W0;
      const int tot = k + 2;
      for (int j0 = 0; j0 < tot; j0 += 16)
        dots(n2, std::min(16, tot - j0), xs + j0, ys + j0, c->dscal + S_DOTS + j0, 0, c->red, s);
    }
    hipLaunchKernelGGL(k_store_orow, dim3(1), dim3(64), 0, s, k, c->dscal + S_DOTS, c->dscal + S_KO,
                       c->dscal + S_KRHS, ctl + 1);
    ++k;
    krylov_solve(k, c->dscal + S_KO, c->dscal + S_KRHS, c->dscal + S_KCOEF, c->dscal + S_KRES, ctl + 3, s);
    src = c->Wk[k - 1];
    if (tol > 0.0) {
      double kc[4];
      if ((st = get_scalars2(c, S_KRES, 3, kres, S_KCTL, 4, kc))) return st;
      rel = std::sqrt(std::max(kres[0], 0.0) / nw0sq);
      if (rel < tol || kc[3] >= 0.0) break;
    }
  }
  double kc[4];
  if ((st = get_scalars2(c, S_KRES, 3, kres, S_KCTL, 4, kc))) return st;
  rel = std::sqrt(std::max(kres[0], 0.0) / nw0sq);
  const int rank = kc[3] >= 0.0 ? std::min(k, (int)kc[3]) : k;
  if (k > 0) {
    lincomb_dev(n2, k, c->dptr, c->dscal + S_KCOEF, Y, s);
  }
  if (rank_out) *rank_out = rank;
  if (rel_out) *rel_out = rel;
  return XLBOMD_OK;
}

xlbomd_status energy_forces(xlbomd_ctx *c, const double *P0, const double *X, double *frc,
                            double e[3]) {
  const int ev = prof_begin(c);
  forces(pairsys(c), P0, X, frc, c->dscal + S_ENER, c->pk3, c->fpart, c->epart, c->s);
  prof_end(c, ev, PC_FORCE, force_bytes(c));
  if (e) return get_scalars(c, S_ENER, 3, e);
  return XLBOMD_OK;
}

// S/k_B of the Fermi occupations of F at mu, from FP64 eigenvalues of F
xlbomd_status entropy(xlbomd_ctx *c, const double *F, double mu, double *S) {
  const int n = c->n;
  if (!c->solver) {
    if (hipsolverCreate(&c->solver) != HIPSOLVER_STATUS_SUCCESS)
      return fail(c, XLBOMD_E_HIP, "hipsolverCreate failed");
    int lwork = 0;
    if (hipsolverDnDsyevd_bufferSize(c->solver, HIPSOLVER_EIG_MODE_NOVECTOR, HIPSOLVER_FILL_MODE_LOWER, n,
                                     c->f64[2], n, c->f64[3], &lwork) != HIPSOLVER_STATUS_SUCCESS)
      return fail(c, XLBOMD_E_HIP, "syevd buffer query failed");
    c->eig_lwork = lwork;
    if (!dev_alloc((void **)&c->eig, sizeof(double) * n) ||
        !dev_alloc((void **)&c->eig_work, sizeof(double) * std::max(lwork, 1)) ||
        !dev_alloc((void **)&c->eig_info, sizeof(int)))
      return fail(c, XLBOMD_E_NOMEM, "eigenvalue workspace allocation failed");
  }
  hipsolverSetStream(c->solver, c->s);
  double *Fw = c->f64[2];
  HIPCHK(c, hipMemcpyAsync(Fw, F, c->n2 * 8, hipMemcpyDeviceToDevice, c->s));
  if (hipsolverDnDsyevd(c->solver, HIPSOLVER_EIG_MODE_NOVECTOR, HIPSOLVER_FILL_MODE_LOWER, n, Fw, n, c->eig,
                        c->eig_work, c->eig_lwork, c->eig_info) != HIPSOLVER_STATUS_SUCCESS)
    return fail(c, XLBOMD_E_HIP, "syevd failed");
  const int nb = std::min((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_entropy_partial, dim3(nb), dim3(256), 0, c->s, n, c->eig, mu, c->beta, c->red);
  hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(64), 0, c->s, nb, c->red, c->dscal + S_ENT);
  return get_scalars(c, S_ENT, 1, S);
}

// ------------------------------------------------------ non-orthogonal basis
// Methods section 3: F_perp = Z^T F Z (eq. 18), the Fermi matrix of F_perp
// (eq. 19), D0 = Z D0_perp Z^T (eq. 20) for any Z with Z^T S Z = I (eq. 21);
// the response transforms the same way (eq. 36); the Pulay term is eq. 41.
// Every transform is an FP64 GEMM (out = A^T op(B)): with U = Z^T M,
// Z^T M Z = Z^T U^T for a symmetric M, and with V = M Z^T, Z M Z^T = V^T Z^T.
xlbomd_status ensure_nonorth(xlbomd_ctx *c) {
  for (auto &p : c->no_w)
    if (!p && !dev_alloc((void **)&p, c->n2 * 8))
      return fail(c, XLBOMD_E_NOMEM, "non-orthogonal work matrices: allocation failed");
  return XLBOMD_OK;
}

// out = Z^T M Z for a symmetric M (U: work)
void congruence_t(xlbomd_ctx *c, const double *Z, const double *M, double *U, double *out) {
  mm_p(c, XLBOMD_FP64, Z, M, U, 1.0, 0);
  mm_p(c, XLBOMD_FP64, Z, U, out, 1.0, 1, nullptr, 0.0, nullptr, 0.0, 0.0, 1);
}
// out = Z M Z^T for a symmetric M (U: work)
void congruence(xlbomd_ctx *c, const double *Z, const double *M, double *U, double *out) {
  mm_p(c, XLBOMD_FP64, M, Z, U, 1.0, 0, nullptr, 0.0, nullptr, 0.0, 0.0, 1);
  mm_p(c, XLBOMD_FP64, U, Z, out, 1.0, 1, nullptr, 0.0, nullptr, 0.0, 0.0, 1);
}

// Z = S^(-1/2), the symmetric choice of eq. 21, by the coupled Newton-Schulz
// iteration (Higham, "Functions of Matrices", SIAM 2008, section 6.3), which
// takes only products of matrices that commute with S: with Y_0 = S / c and
// Z_0 = I, D_k = (I - Z_k Y_k) / 2, Y_{k+1} = Y_k + Y_k D_k, Z_{k+1} = Z_k + D_k Z_k,
// Z_k -> (S / c)^(-1/2).  c is the middle of the spectral bounds of S, so the
// eigenvalues of S / c lie in (0, 2) and ||I - S / c|| < 1.  The GEMM writes
// D directly, so ||D||_F has no cancellation; after the update that follows a
// ||2 D||_F <= 1e-8 sqrt(n) the error is of order the square of that.
xlbomd_status lowdin(xlbomd_ctx *c, const double *S, double *Z, int *iters) {
  xlbomd_status st = ensure_nonorth(c);
  if (st) return st;
  double lohi[2];
  if ((st = spectral_bounds(c, S, lohi))) return st;
  if (!(lohi[0] > 0.0))
    return fail(c, XLBOMD_E_ARG, "overlap matrix not positive definite (spectral lower bound %.3e)", lohi[0]);
  const int n = c->n, n2 = (int)c->n2;
  const double sc = 0.5 * (lohi[0] + lohi[1]);
  double *Y[2] = {c->no_w[0], c->no_w[1]}, *Zk[2] = {Z, c->no_w[3]}, *D = c->no_w[2];
  axpby(n2, 1.0 / sc, S, 0.0, nullptr, Y[0], 0, c->s);
  axpbyI_dev(n, nullptr, 0.0, nullptr, nullptr, 0.0, nullptr, nullptr, 1.0, Zk[0], 0, c->s);
  const double tol = 1e-8 * std::sqrt((double)n);
  int cur = 0, it = 0;
  for (;; ++it) {
    if (it == 60) return fail(c, XLBOMD_E_NOCONV, "Newton-Schulz inverse square root: no convergence");
    mm_p(c, XLBOMD_FP64, Zk[cur], Y[cur], D, -0.5, 1, nullptr, 0.0, nullptr, 0.0, 0.5);
    const void *dd[1] = {D};
    dots(n2, 1, dd, dd, c->dscal + S_DOTS, 0, c->red, c->s);
    mm_p(c, XLBOMD_FP64, Y[cur], D, Y[1 - cur], 1.0, 1, Y[cur], 1.0);
    mm_p(c, XLBOMD_FP64, D, Zk[cur], Zk[1 - cur], 1.0, 1, Zk[cur], 1.0);
    cur = 1 - cur;
    double e2;
    if ((st = get_scalars(c, S_DOTS, 1, &e2))) return st;
    const double e = 2.0 * std::sqrt(e2);
    if (!std::isfinite(e)) return fail(c, XLBOMD_E_NONFINITE, "non-finite Newton-Schulz residual");
    if (e <= tol) break;
  }
  axpby(n2, 1.0 / std::sqrt(sc), Zk[cur], 0.0, nullptr, Z, 0, c->s);
  if (iters) *iters = it + 1;
  return XLBOMD_OK;
}

}  // namespace

// ====================================================================== ABI
extern "C" {

const char *xlbomd_last_error(xlbomd_handle h) { return h ? h->err.c_str() : "null handle"; }
int xlbomd_n_orb(xlbomd_handle h) { return h ? h->n : 0; }

xlbomd_status xlbomd_destroy(xlbomd_handle c) {
  if (!c) return XLBOMD_E_ARG;
  hipStreamSynchronize(c->s);
  auto f = [](void *p) {
    if (p) hipFree(p);
  };
  f(c->R);
  f(c->onecenter);
  f(c->j55);
  f(c->noise_t);
  f(c->part);
  f(c->pk3);
  f(c->fpart);
  f(c->epart);
  f(c->dscal);
  f(c->red);
  f(c->frc);
  f(c->dptr);
  f(c->lq);
  f(c->lw);
  for (auto &p : c->Yc) f(p);
  for (auto &p : c->Zc) f(p);
  f(c->Vst);
  f(c->Pst);
  f(c->Sst);
  f(c->S2st);
  f(c->Bst);
  f(c->D);
  f(c->M);
  for (auto &p : c->w) f(p);
  for (auto &p : c->f64) f(p);
  if (c->resp_copy) {
    for (auto &p : c->Yr) f(p);
    f(c->Vr);
    f(c->Pr);
    f(c->Sr);
    f(c->S2r);
    f(c->Br);
    f(c->Mr);
  }
  f(c->Wr);
  for (int k = 0; k < c->kalloc; ++k) {
    f(c->Vk[k]);
    f(c->Wk[k]);
  }
  for (auto e : c->evpool) hipEventDestroy(e);
  if (c->solver) hipsolverDestroy(c->solver);
  f(c->eig);
  f(c->eig_work);
  f(c->eig_info);
  for (auto &p : c->no_w) f(p);
  delete c;
  return XLBOMD_OK;
}

xlbomd_status xlbomd_create(const xlbomd_system *sys, const xlbomd_params *prm, void *stream,
                            xlbomd_handle *out) {
  if (!sys || !prm || !out) return XLBOMD_E_ARG;
  *out = nullptr;
  // n = 4 n_atoms <= 32764: element counts n^2 stay below 2^30 (32-bit in the
  // element-wise kernels) and n within the split GEMM's 16-bit tile indexing
  if (sys->n_atoms < 1 || sys->n_atoms > 8191 || !sys->onecenter || (sys->n_atoms > 1 && !sys->noise55))
    return XLBOMD_E_ARG;
  const double n = 4.0 * sys->n_atoms;
  if (!(sys->n_elec > 0.0) || !(sys->n_elec < 2.0 * n)) return XLBOMD_E_ARG;
  // the precision is read as the int a C caller stores: in C++ a load of an
  // enum outside its enumerators' range is undefined, and the range test on
  // such a load may be dropped
  static_assert(sizeof(xlbomd_precision) == sizeof(int), "precision is an int-sized enum");
  int prec_raw;
  std::memcpy(&prec_raw, &prm->prec, sizeof prec_raw);
  if (!(prm->T_e > 0.0) || prm->m < 0 || prm->m > MMAX || prec_raw < 0 || prec_raw > 6 ||
      !(prm->kernel_c > 0.0) || !std::isfinite(prm->kernel_c) || !(prm->w0_limit >= 0.0) ||
      !(prm->T_ion_limit >= 0.0))
    return XLBOMD_E_ARG;
  xlbomd_ctx *c = new xlbomd_ctx();
  c->N = sys->n_atoms;
  c->n = 4 * c->N;
  c->n2 = (size_t)c->n * c->n;
  c->n_elec = sys->n_elec;
  c->n_occ = 0.5 * sys->n_elec;
  c->prm = *prm;
  c->model = sys->model;
  c->s = (hipStream_t)stream;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return XLBOMD_E_HIP;
  }
  c->beta = 1.0 / (KB * prm->T_e);
  c->prec = prm->prec;
  split_prec(prm->prec, c->prec_dm, c->prec_rs);
  c->is32 = c->prec_dm != XLBOMD_FP64;
  c->rs32 = c->prec_rs != XLBOMD_FP64;
  c->resp_copy = c->prec_dm != c->prec_rs;
  c->esz = c->is32 ? 4 : 8;
  c->trace_tol = !c->is32 ? 0.0 : (c->prec_dm == XLBOMD_BF16X3 ? 2e-6 : 2e-7) * c->n;
  const int N = c->N, T = (N + 15) / 16;
  bool ok = true;
  auto A = [&](void **p, size_t bytes) { ok = ok && dev_alloc(p, bytes); };
  A((void **)&c->R, sizeof(double) * 3 * N);
  A((void **)&c->onecenter, sizeof(double) * 5 * N);
  A((void **)&c->j55, sizeof(double) * 55);
  A((void **)&c->noise_t, sizeof(float) * std::max<size_t>(noise_tile_floats(N), 1));
  A((void **)&c->part, sizeof(double) * 10 * (size_t)N * T);
  A((void **)&c->pk3, sizeof(double) * 30 * N);
  A((void **)&c->fpart, sizeof(double) * std::max<size_t>(force_partial_doubles(N), 1));
  A((void **)&c->epart, sizeof(double) * (energy_partial_doubles(N) + 8));
  A((void **)&c->dscal, sizeof(double) * S_TOTAL);
  A((void **)&c->red, sizeof(double) * (reduce_partials_capacity() + 2 * (size_t)c->n));
  A((void **)&c->frc, sizeof(double) * 3 * N);
  A((void **)&c->dptr, sizeof(double *) * 64);
  A((void **)&c->lq, sizeof(double) * (LANCZOS_K + 1) * (size_t)c->n);
  A((void **)&c->lw, sizeof(double) * (size_t)c->n);
  const size_t mb = c->n2 * c->esz;
  A(&c->Yc[0], mb);  // levels beyond the first are allocated as chains need them
  A(&c->Vst, mb);
  A(&c->Pst, mb);
  A(&c->Sst, mb);
  A(&c->S2st, mb);
  A(&c->Bst, mb);
  A(&c->D, mb);
  A(&c->M, mb);
  for (auto &p : c->w) A(&p, c->n2 * 8);  // work matrices hold either element type
  for (auto &p : c->f64) A((void **)&p, c->n2 * 8);
  if (c->resp_copy) {
    const size_t m4 = c->n2 * 4;
    A(&c->Vr, m4);
    A(&c->Pr, m4);
    A(&c->Sr, m4);
    A(&c->S2r, m4);
    A(&c->Br, m4);
    A(&c->Mr, m4);
  }
  A(&c->Wr, c->resp_copy ? c->n2 * 4 : mb);
  if (!ok) {
    xlbomd_destroy(c);
    return XLBOMD_E_NOMEM;
  }
  if (hipMemcpy(c->onecenter, sys->onecenter, sizeof(double) * 5 * N, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->j55, sys->model.j55, sizeof(double) * 55, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(c->dscal, 0, sizeof(double) * S_TOTAL) != hipSuccess) {
    xlbomd_destroy(c);
    return XLBOMD_E_HIP;
  }
  lanczos_start(c->n, c->lq, c->s);
  if (N > 1) {
    const size_t npair = (size_t)N * (N - 1) / 2;
    float *tmp = nullptr;
    if (!dev_alloc((void **)&tmp, sizeof(float) * npair * 55)) {
      xlbomd_destroy(c);
      return XLBOMD_E_NOMEM;
    }
    bool copied = hipMemcpy(tmp, sys->noise55, sizeof(float) * npair * 55, hipMemcpyHostToDevice) == hipSuccess;
    if (copied) {
      repack_noise(N, tmp, c->noise_t, c->s);
      copied = hipStreamSynchronize(c->s) == hipSuccess;
    }
    hipFree(tmp);
    if (!copied) {
      xlbomd_destroy(c);
      return XLBOMD_E_HIP;
    }
  }
  if (hipGetLastError() != hipSuccess) {
    xlbomd_destroy(c);
    return XLBOMD_E_HIP;
  }
  *out = c;
  return XLBOMD_OK;
}

xlbomd_status xlbomd_set_geometry(xlbomd_handle c, const double *R) {
  if (!c || !R) return XLBOMD_E_ARG;
  HIPCHK(c, hipMemcpyAsync(c->R, R, sizeof(double) * 3 * c->N, hipMemcpyDeviceToDevice, c->s));
  c->geom = true;
  c->chain_valid = false;
  return XLBOMD_OK;
}

xlbomd_status xlbomd_hcore(xlbomd_handle c, double *H) {
  if (!c || !H) return XLBOMD_E_ARG;
  if (!c->geom) return fail(c, XLBOMD_E_STATE, "positions not set");
  hcore(pairsys(c), H, c->part, c->s);
  HIPCHK(c, hipGetLastError());
  return XLBOMD_OK;
}

xlbomd_status xlbomd_fock(xlbomd_handle c, const double *P, double *F, int include_h) {
  if (!c || !P || !F || P == F) return c ? fail(c, XLBOMD_E_ARG, "bad fock arguments") : XLBOMD_E_ARG;
  if (!c->geom) return fail(c, XLBOMD_E_STATE, "positions not set");
  fock_t(c, P, F, include_h ? 1 : 0);
  HIPCHK(c, hipGetLastError());
  return XLBOMD_OK;
}

xlbomd_status xlbomd_fermi_dm(xlbomd_handle c, const double *F, double *mu, double *P,
                              double *entropy) {
  if (!c || !F || !mu || !P || F == P) return c ? fail(c, XLBOMD_E_ARG, "bad fermi_dm arguments") : XLBOMD_E_ARG;
  xlbomd_status st = fermi(c, F, mu, P, true);
  if (st) return st;
  if (entropy && (st = ::entropy(c, F, *mu, entropy))) return st;
  HIPCHK(c, hipGetLastError());
  return XLBOMD_OK;
}

xlbomd_status xlbomd_spectral_bounds(xlbomd_handle c, const double *F, double *lohi) {
  if (!c || !F || !lohi) return c ? fail(c, XLBOMD_E_ARG, "bad spectral_bounds arguments") : XLBOMD_E_ARG;
  xlbomd_status st = spectral_bounds(c, F, lohi);
  if (st) return st;
  HIPCHK(c, hipGetLastError());
  return XLBOMD_OK;
}

xlbomd_status xlbomd_dm_response(xlbomd_handle c, const double *F1, double *P1) {
  if (!c || !F1 || !P1 || F1 == P1) return c ? fail(c, XLBOMD_E_ARG, "bad response arguments") : XLBOMD_E_ARG;
  if (!c->chain_valid) return fail(c, XLBOMD_E_STATE, "no Fermi chain cached");
  xlbomd_status st = response(c, F1, P1);
  if (st) return st;
  HIPCHK(c, hipGetLastError());
  return XLBOMD_OK;
}

xlbomd_status xlbomd_krylov_kernel(xlbomd_handle c, const double *X, const double *P0, int m, double tol,
                                   double *Y, int *rank, double *relres) {
  if (!c || !X || !P0 || !Y) return XLBOMD_E_ARG;
  xlbomd_status st = krylov(c, X, P0, m, tol, Y, rank, relres, nullptr);
  if (st) return st;
  HIPCHK(c, hipStreamSynchronize(c->s));
  return XLBOMD_OK;
}

xlbomd_status xlbomd_forces(xlbomd_handle c, const double *P0, const double *X, double *frc,
                            double *energy) {
  if (!c || !P0 || !X || !frc) return XLBOMD_E_ARG;
  if (!c->geom) return fail(c, XLBOMD_E_STATE, "positions not set");
  double e[3];
  xlbomd_status st = energy_forces(c, P0, X, frc, e);
  if (st) return st;
  if (energy) {
    energy[0] = e[0];
    energy[1] = e[1];
    energy[2] = e[2];
    energy[3] = e[0] + e[1] + e[2];
  }
  return XLBOMD_OK;
}

// an MD state with every buffer present and its ring slot inside the history
static bool overlap_ok(const xlbomd_overlap_model *ov) {
  return ov && std::isfinite(ov->s0) && std::isfinite(ov->r0) && ov->lam > 0.0 && std::isfinite(ov->lam);
}

xlbomd_status xlbomd_overlap(xlbomd_handle c, const xlbomd_overlap_model *ov, double *S) {
  if (!c || !S || !overlap_ok(ov)) return c ? fail(c, XLBOMD_E_ARG, "bad overlap arguments") : XLBOMD_E_ARG;
  if (!c->geom) return fail(c, XLBOMD_E_STATE, "positions not set");
  overlap_matrix(c->N, c->R, OverlapSys{ov->s0, ov->r0, ov->lam}, S, c->s);
  HIPCHK(c, hipGetLastError());
  return XLBOMD_OK;
}

xlbomd_status xlbomd_lowdin(xlbomd_handle c, const double *S, double *Z, int *iterations) {
  if (!c || !S || !Z || S == Z) return c ? fail(c, XLBOMD_E_ARG, "bad lowdin arguments") : XLBOMD_E_ARG;
  xlbomd_status st = lowdin(c, S, Z, iterations);
  if (st) return st;
  HIPCHK(c, hipGetLastError());
  return XLBOMD_OK;
}

xlbomd_status xlbomd_fermi_dm_nonorth(xlbomd_handle c, const double *F, const double *Z, double *mu, double *P,
                                      double *entropy) {
  if (!c || !F || !Z || !mu || !P || P == F || P == Z)
    return c ? fail(c, XLBOMD_E_ARG, "bad fermi_dm_nonorth arguments") : XLBOMD_E_ARG;
  xlbomd_status st = ensure_nonorth(c);
  if (st) return st;
  double *U = c->no_w[0], *Fp = c->no_w[1], *Pp = c->no_w[2];
  congruence_t(c, Z, F, U, Fp);
  if ((st = fermi(c, Fp, mu, Pp, true))) return st;
  c->chain_nonorth = true;
  if (entropy && (st = ::entropy(c, Fp, *mu, entropy))) return st;
  congruence(c, Z, Pp, U, P);
  HIPCHK(c, hipGetLastError());
  return XLBOMD_OK;
}

xlbomd_status xlbomd_dm_response_nonorth(xlbomd_handle c, const double *F1, const double *Z, double *P1) {
  if (!c || !F1 || !Z || !P1 || P1 == F1 || P1 == Z)
    return c ? fail(c, XLBOMD_E_ARG, "bad dm_response_nonorth arguments") : XLBOMD_E_ARG;
  if (!c->chain_valid || !c->chain_nonorth)
    return fail(c, XLBOMD_E_STATE, "no chain of xlbomd_fermi_dm_nonorth cached");
  xlbomd_status st = ensure_nonorth(c);
  if (st) return st;
  double *U = c->no_w[0], *F1p = c->no_w[1], *P1p = c->no_w[2];
  congruence_t(c, Z, F1, U, F1p);
  if ((st = response(c, F1p, P1p))) return st;
  congruence(c, Z, P1p, U, P1);
  HIPCHK(c, hipGetLastError());
  return XLBOMD_OK;
}

xlbomd_status xlbomd_pulay_forces(xlbomd_handle c, const xlbomd_overlap_model *ov, const double *F,
                                  const double *P, const double *Z, double *frc) {
  if (!c || !F || !P || !Z || !frc || !overlap_ok(ov))
    return c ? fail(c, XLBOMD_E_ARG, "bad pulay_forces arguments") : XLBOMD_E_ARG;
  if (!c->geom) return fail(c, XLBOMD_E_STATE, "positions not set");
  xlbomd_status st = ensure_nonorth(c);
  if (st) return st;
  double *U = c->no_w[0], *FSi = c->no_w[1], *Qt = c->no_w[2];
  mm_p(c, XLBOMD_FP64, Z, F, U, 1.0, 0);                                           // Z^T F
  mm_p(c, XLBOMD_FP64, U, Z, FSi, 1.0, 0, nullptr, 0.0, nullptr, 0.0, 0.0, 1);     // F Z Z^T = F S^-1
  mm_p(c, XLBOMD_FP64, P, FSi, Qt, 1.0, 0);                                        // P F S^-1 = Q^T
  pulay_forces(c->N, c->R, OverlapSys{ov->s0, ov->r0, ov->lam}, Qt, frc, c->s);
  HIPCHK(c, hipGetLastError());
  return XLBOMD_OK;
}

static bool state_ok(const xlbomd_md_state *st) {
  return st && st->R && st->V && st->A && st->X && st->Y && st->head >= 0 && st->head < 7;
}

xlbomd_status xlbomd_integrate(xlbomd_handle c, xlbomd_md_state *st) {
  if (!c || !state_ok(st)) return XLBOMD_E_ARG;
  const int n2 = (int)c->n2;
  const double *Xk[7];
  for (int k = 0; k < 7; ++k) Xk[k] = st->X + (size_t)((st->head + k) % 7) * c->n2;
  const int nh = (st->head + 6) % 7;
  x_verlet(n2, Xk, st->Y, c->prm.kappa, c->prm.alpha, c->prm.c, st->X + (size_t)nh * c->n2, c->s);
  st->head = nh;
  kick_drift(3 * c->N, st->R, st->V, st->A, c->prm.dt, 1, c->s);
  HIPCHK(c, hipGetLastError());
  return XLBOMD_OK;
}

static xlbomd_status evaluate_state(xlbomd_ctx *c, xlbomd_md_state *st, double e[3], int *rank,
                                    double *rel, double *w0, double *S = nullptr) {
  xlbomd_status s;
  if ((s = xlbomd_set_geometry(c, st->R))) return s;
  const double *X = st->X + (size_t)st->head * c->n2;
  double *F = c->f64[5];
  double *P0 = c->f64[4];
  fock_t(c, X, F, 1);
  // P0 lives in f64[4] only until the Krylov call, which reuses it: keep a copy in Vk? use Wk slots
  // warm start: linear extrapolation of mu from the last two steps
  double mu = st->mu;
  if (std::isfinite(st->mu) && std::isfinite(st->mu_prev)) mu = 2.0 * st->mu - st->mu_prev;
  if ((s = fermi(c, F, &mu, P0, true))) return s;
  st->mu_prev = st->mu;
  st->mu = mu;
  if (S && (s = entropy(c, F, mu, S))) return s;
  // forces first (Krylov reuses f64[0..4])
  if ((s = energy_forces(c, P0, X, c->frc, e))) return s;
  accel(3 * c->N, c->frc, ACC / c->model.mass, st->A, c->s);
  double *P0k = c->f64[5];  // F no longer needed
  HIPCHK(c, hipMemcpyAsync(P0k, P0, c->n2 * 8, hipMemcpyDeviceToDevice, c->s));
  if ((s = krylov(c, X, P0k, c->prm.m, c->prm.krylov_tol, st->Y, rank, rel, w0))) return s;
  return XLBOMD_OK;
}

xlbomd_status xlbomd_md_init(xlbomd_handle c, xlbomd_md_state *st) {
  if (!c || !state_ok(st)) return XLBOMD_E_ARG;
  st->mu_prev = NAN;
  // replicate X(t0) into every history slot
  const double *X0 = st->X + (size_t)st->head * c->n2;
  for (int k = 1; k < 7; ++k)
    HIPCHK(c, hipMemcpyAsync(st->X + (size_t)((st->head + k) % 7) * c->n2, X0, c->n2 * 8,
                             hipMemcpyDeviceToDevice, c->s));
  double e[3];
  int rank;
  double rel, w0;
  return evaluate_state(c, st, e, &rank, &rel, &w0);
}

// the steps of xlbomd_step and xlbomd_step_langevin (xi == nullptr: NVE)
static xlbomd_status md_steps(xlbomd_ctx *c, xlbomd_md_state *st, int n_steps, xlbomd_report *rep,
                              double c1, double c2, const double *xi) {
  if (!state_ok(st)) return XLBOMD_E_ARG;
  const bool t_guard = c->prm.T_ion_limit > 0.0;
  const int dof = std::max(3 * c->N - 3, 1);
  std::vector<double> V;
  for (int k = 0; k < n_steps; ++k) {
    xlbomd_status s;
    // a failing step leaves its status in its report
    auto stop = [&](xlbomd_status why) {
      if (rep) rep[k].status = why;
      return why;
    };
    if (xi) {
      const double *Xk[7];
      for (int j = 0; j < 7; ++j) Xk[j] = st->X + (size_t)((st->head + j) % 7) * c->n2;
      const int nh = (st->head + 6) % 7;
      x_verlet((int)c->n2, Xk, st->Y, c->prm.kappa, c->prm.alpha, c->prm.c, st->X + (size_t)nh * c->n2, c->s);
      st->head = nh;
      baoab_pre(3 * c->N, st->R, st->V, st->A, c->prm.dt, c1, c2, xi + (size_t)3 * c->N * k, c->s);
      HIPCHK(c, hipGetLastError());
    } else if ((s = xlbomd_integrate(c, st))) {
      return stop(s);
    }
    double e[3];
    int rank = 0;
    double rel = 0, w0 = 0, S = 0.0;
    // energies (a host round trip) only for a report
    if ((s = evaluate_state(c, st, rep ? e : nullptr, &rank, &rel, &w0, rep ? &S : nullptr))) return stop(s);
    kick_drift(3 * c->N, st->R, st->V, st->A, c->prm.dt, 0, c->s);
    double ke = NAN;
    if (rep || t_guard) {
      // kinetic energy from V (host copy of a few KB)
      V.resize(3 * c->N);
      HIPCHK(c, hipMemcpyAsync(V.data(), st->V, sizeof(double) * 3 * c->N, hipMemcpyDeviceToHost, c->s));
      HIPCHK(c, hipStreamSynchronize(c->s));
      ke = 0.0;
      for (double v : V) ke += v * v;
      ke *= 0.5 * c->model.mass / ACC;
    }
    const double T_ion = 2.0 * ke / (dof * KB);
    xlbomd_status status = XLBOMD_OK;
    if (!std::isfinite(w0) || (rep && !(std::isfinite(e[0]) && std::isfinite(e[1]) && std::isfinite(e[2]) &&
                                        std::isfinite(ke))))
      status = fail(c, XLBOMD_E_NONFINITE, "non-finite residual or energies at step %d", k);
    else if (c->prm.w0_limit > 0.0 && w0 > c->prm.w0_limit)
      status = fail(c, XLBOMD_E_UNSTABLE, "||D0 - X|| = %.3e above its limit %.3e at step %d", w0,
                    c->prm.w0_limit, k);
    else if (t_guard && !(T_ion <= c->prm.T_ion_limit))
      status = fail(c, XLBOMD_E_UNSTABLE, "T_ion = %.4g K above its limit %.4g K at step %d", T_ion,
                    c->prm.T_ion_limit, k);
    if (rep) {
      xlbomd_report &r = rep[k];
      r.KE = ke;
      r.TS = 2.0 * S / c->beta;  // -2 T_e S with S in units of k_B: 2 k_B T_e S = 2 S / beta
      r.U = e[0] + e[1] + e[2] - r.TS;
      r.E_tot = r.KE + r.U;
      r.T_ion = T_ion;
      r.mu = st->mu;
      r.W0 = w0;
      r.relres = rel;
      r.rank = rank;
      r.status = status;
      r.levels = c->L;
      r.mu_passes = c->mu_passes;
    }
    if (status != XLBOMD_OK) return status;
  }
  HIPCHK(c, hipStreamSynchronize(c->s));
  return XLBOMD_OK;
}

xlbomd_status xlbomd_step(xlbomd_handle c, xlbomd_md_state *st, int n_steps, xlbomd_report *rep) {
  if (!c || !st || n_steps < 0) return XLBOMD_E_ARG;
  return md_steps(c, st, n_steps, rep, 1.0, 0.0, nullptr);
}

xlbomd_status xlbomd_ensemble_step(xlbomd_handle *h, xlbomd_md_state *st, int count, int n_steps,
                                   xlbomd_report *rep) {
  if (!h || !st || count < 0 || n_steps < 0) return XLBOMD_E_ARG;
  for (int i = 0; i < count; ++i) {
    if (!h[i]) return XLBOMD_E_ARG;
    for (int j = 0; j < i; ++j)
      if (h[j] == h[i]) return XLBOMD_E_ARG;  // a handle's workspace serves one member
  }
  // members are taken in index order by up to 16 host threads (the caller
  // chooses the order); each runs xlbomd_step on its own handle (and so its
  // own stream and workspace), so a member's result does not depend on it
  std::vector<xlbomd_status> status(count, XLBOMD_OK);
  std::atomic<int> next(0);
  auto worker = [&]() {
    for (int i = next++; i < count; i = next++) {
      if (hipSetDevice(h[i]->device) != hipSuccess) {
        status[i] = XLBOMD_E_HIP;
        continue;
      }
      status[i] = xlbomd_step(h[i], &st[i], n_steps, rep ? rep + (size_t)i * n_steps : nullptr);
    }
  };
  const int nt = std::min(count, 16);
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; ++t) pool.emplace_back(worker);
  if (nt > 0) worker();
  for (auto &t : pool) t.join();
  for (int i = 0; i < count; ++i)
    if (status[i] != XLBOMD_OK) return status[i];
  return XLBOMD_OK;
}

xlbomd_status xlbomd_step_langevin(xlbomd_handle c, xlbomd_md_state *st, int n_steps, double gamma,
                                   double T_ion, const double *xi, xlbomd_report *rep) {
  if (!c || !st || n_steps < 0 || !(gamma >= 0.0) || !(T_ion >= 0.0) || !std::isfinite(gamma) ||
      !std::isfinite(T_ion) || (n_steps > 0 && !xi))
    return XLBOMD_E_ARG;
  const double c1 = std::exp(-gamma * c->prm.dt);
  const double c2 = std::sqrt(KB * T_ion * ACC / c->model.mass * (1.0 - c1 * c1));
  return md_steps(c, st, n_steps, rep, c1, c2, xi);
}

xlbomd_status xlbomd_scf(xlbomd_handle c, double *X, const xlbomd_scf_params *p, double *history,
                         int history_len, xlbomd_scf_report *rep) {
  if (!c || !X || !p) return XLBOMD_E_ARG;
  const int m = p->m;
  if (m < 1 || m > MMAX - 2 || p->max_iter < 0 || p->max_mix < 0 || !(p->mix > 0.0 && p->mix <= 1.0) ||
      !(p->tol >= 0.0) || !(p->mix_tol >= 0.0) || history_len < 0)
    return fail(c, XLBOMD_E_ARG, "bad scf settings");
  if (!c->geom) return fail(c, XLBOMD_E_STATE, "positions not set");
  const int n2 = (int)c->n2;
  xlbomd_status s;
  xlbomd_scf_report r{};
  int nh = 0;
  auto record = [&](double v) {
    if (history && nh < history_len) history[nh++] = v;
  };
  // the Krylov kernel owns f64[0..4], Vk[0..m-1], Wk[0..m-1]; the SCF keeps its
  // own matrices in the two slots after them
  if ((s = ensure_krylov(c, m + 2))) return s;
  double *F = c->f64[5];
  double *Pm = c->Wk[m], *Ptrial = c->Wk[m + 1], *Ystep = c->Vk[m], *Xtrial = c->Vk[m + 1];
  double mu = NAN;
  auto resid = [&](const double *Xc, double *Pout, double &res) -> xlbomd_status {
    fock_t(c, Xc, F, 1);
    xlbomd_status q = fermi(c, F, &mu, Pout, true);
    if (q) return q;
    ++r.evaluations;
    axpby(n2, 1.0, Pout, -1.0, Xc, c->f64[0], 0, c->s);
    const void *a[1] = {c->f64[0]};
    dots(n2, 1, a, a, c->dscal + S_DOTS, 0, c->red, c->s);
    double r2;
    q = get_scalars(c, S_DOTS, 1, &r2);
    res = std::sqrt(r2);
    if (!std::isfinite(res)) return fail(c, XLBOMD_E_NONFINITE, "non-finite SCF residual");
    return q;
  };
  // linear mixing settles into a stable fixed point; Newton-Krylov then converges fast
  double res = 0.0;
  if ((s = resid(X, Pm, res))) return s;
  record(res);
  while (r.mix_steps < p->max_mix && res > p->mix_tol && res > p->tol) {
    axpby(n2, 1.0 - p->mix, X, p->mix, Pm, X, 0, c->s);
    ++r.mix_steps;
    if ((s = resid(X, Pm, res))) return s;
    record(res);
  }
  while (r.newton_steps < p->max_iter && res > p->tol) {
    int rank;
    double rel;
    // the chain cached by the last resid() call belongs to the current X
    if ((s = krylov(c, X, Pm, m, 0.0, Ystep, &rank, &rel, nullptr))) return s;
    r.responses += rank;
    double lam = 1.0, rt = 0.0;
    while (true) {
      axpby(n2, 1.0, X, -lam, Ystep, Xtrial, 0, c->s);
      if ((s = resid(Xtrial, Ptrial, rt))) return s;
      if (rt < res || lam < 1e-4) break;
      lam *= 0.5;
    }
    HIPCHK(c, hipMemcpyAsync(X, Xtrial, c->n2 * 8, hipMemcpyDeviceToDevice, c->s));
    HIPCHK(c, hipMemcpyAsync(Pm, Ptrial, c->n2 * 8, hipMemcpyDeviceToDevice, c->s));
    res = rt;
    ++r.newton_steps;
    record(res);
  }
  r.residual = res;
  if (rep) *rep = r;
  HIPCHK(c, hipStreamSynchronize(c->s));
  if (!(res <= p->tol)) return fail(c, XLBOMD_E_NOCONV, "SCF residual %.3e above tolerance", res);
  return XLBOMD_OK;
}

xlbomd_status xlbomd_matmul(xlbomd_handle c, const double *A, const double *B, double *Cout, int sym_out,
                            int reps) {
  if (!c || !A || !B || !Cout || reps < 1) return XLBOMD_E_ARG;
  const int n2 = (int)c->n2;
  const void *a = A, *b = B;
  void *o = Cout;
  if (c->rs32) {
    convert(n2, A, 0, c->w[0], 1, c->s);
    // the split kernels take their second operand by rows (op(B) = B^T), so
    // they get B^T: A (B^T)^T = A B for any B
    convert_t(c->n, B, (float *)c->w[1], c->s);
    a = c->w[0];
    b = c->w[1];
    o = c->w[2];
  }
  for (int r = 0; r < reps; ++r) mr(c, a, b, o, 1.0, sym_out ? 1 : 0);
  if (c->rs32) convert(n2, c->w[2], 1, Cout, 0, c->s);
  HIPCHK(c, hipGetLastError());
  return XLBOMD_OK;
}

xlbomd_status xlbomd_profile(xlbomd_handle c, int enable) {
  if (!c) return XLBOMD_E_ARG;
  HIPCHK(c, hipStreamSynchronize(c->s));
  c->recs.clear();
  c->prof = enable != 0;
  if (c->prof && c->evpool.empty()) {
    c->evpool.resize(2 * 65536);
    // timing-only events: profile_read synchronises the stream before reading
    // them, so the system-scope fence (a cache writeback and invalidate at every
    // record, ~10 us between back-to-back kernels) is not needed
    for (auto &e : c->evpool) HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  }
  return XLBOMD_OK;
}

xlbomd_status xlbomd_profile_read(xlbomd_handle c, double *out) {
  if (!c || !out) return XLBOMD_E_ARG;
  HIPCHK(c, hipStreamSynchronize(c->s));
  for (int i = 0; i < 3 * PC_N; ++i) out[i] = 0.0;
  for (const auto &r : c->recs) {
    float ms = 0.0f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->evpool[r.ev], c->evpool[r.ev + 1]));
    out[3 * r.cls + 0] += 1.0;
    out[3 * r.cls + 1] += ms;
    out[3 * r.cls + 2] += r.work;
  }
  return XLBOMD_OK;
}

}  // extern "C"
