// Elementwise, reduction and scalar kernels of the hot path (all memory-bound
// or latency-bound; FP64 accumulation everywhere).
//
// Reductions are deterministic: a fixed grid of RED_BLOCKS workgroups writes
// one partial per block, and a single workgroup sums the partials in a fixed
// order.  No floating-point atomics are used.
#include "common.h"

#include <cmath>

namespace xl {
namespace {

constexpr int RED_BLOCKS = 1024;
constexpr int MAXK = 16;
// largest chemical-potential move of one Newton pass, in units of 1/beta, and
// the bracket of the six-term series solve (the series in 1 - exp(-beta dmu)
// is accurate only well inside its radius of convergence)
constexpr double MU_STEP = 1.0;
constexpr double SERIES_STEP = 0.3;

template <typename T>
__device__ inline double ld(const void *p, size_t i) {
  return (double)((const T *)p)[i];
}

template <typename T>
__global__ void k_axpby(size_t n2, double a, const void *x, double b, const void *y, void *out) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n2;
       i += (size_t)gridDim.x * blockDim.x) {
    double v = a * ld<T>(x, i);
    if (y) v += b * ld<T>(y, i);
    ((T *)out)[i] = (T)v;
  }
}

template <typename T>
__global__ void k_axpbyI(int n, const double *a_dev, double a, const void *x, const double *b_dev,
                         double b, const void *y, const double *g_dev, double g, void *out) {
  const double av = a_dev ? *a_dev : a;
  const double bv = b_dev ? *b_dev : b;
  const double gv = g_dev ? *g_dev : g;
  const size_t n2 = (size_t)n * n;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n2;
       i += (size_t)gridDim.x * blockDim.x) {
    double v = 0.0;
    if (x) v += av * ld<T>(x, i);
    if (y) v += bv * ld<T>(y, i);
    if (i / n == i % n) v += gv;
    ((T *)out)[i] = (T)v;
  }
}

// out = 2 (H + s M) - sub in FP64 from H, M of element type T, s a device
// scalar, sub FP64 or null: the canonical response written to the caller in
// one pass (with the Krylov kernel's - V folded in)
template <typename T>
__global__ void k_canon_out(size_t n2, const void *H, const void *M, const double *s_dev, const double *sub,
                            double *out) {
  const double sv = *s_dev;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n2; i += (size_t)gridDim.x * blockDim.x) {
    const double r = 2.0 * (ld<T>(H, i) + sv * ld<T>(M, i));
    out[i] = sub ? r - sub[i] : r;
  }
}

// out = sum_j a_j X_j + g I over four matrices (null X_j skipped); out may
// alias any X_j (each element is read before it is written)
template <typename T>
__global__ void k_poly_comb(int n, const void *X0, const void *X1, const void *X2, const void *X3,
                            double a0, double a1, double a2, double a3, double g, void *out) {
  const size_t n2 = (size_t)n * n;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n2;
       i += (size_t)gridDim.x * blockDim.x) {
    double v = (i / n == i % n) ? g : 0.0;
    if (X0) v += a0 * ld<T>(X0, i);
    if (X1) v += a1 * ld<T>(X1, i);
    if (X2) v += a2 * ld<T>(X2, i);
    if (X3) v += a3 * ld<T>(X3, i);
    ((T *)out)[i] = (T)v;
  }
}

// out = in^T, FP64 -> FP32, by 32 x 32 tiles staged in LDS (coalesced both ways)
__global__ __launch_bounds__(256) void k_convert_t(int n, const double *in, float *out) {
  __shared__ float t[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int i = by + r, j = bx + tx;
    if (i < n && j < n) t[r][tx] = (float)in[(size_t)i * n + j];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int i = bx + r, j = by + tx;
    if (i < n && j < n) out[(size_t)i * n + j] = t[tx][r];
  }
}

template <typename TI, typename TO>
__global__ void k_convert(size_t n2, const void *in, void *out, double scale) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n2;
       i += (size_t)gridDim.x * blockDim.x)
    ((TO *)out)[i] = scale == 1.0 ? (TO)((const TI *)in)[i] : (TO)(scale * (double)((const TI *)in)[i]);
}

// out = a + (double) b, and its FP32 rounding (nullable)
__global__ void k_add_mixed(size_t n2, const double *a, const float *b, double *out, float *out32) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n2;
       i += (size_t)gridDim.x * blockDim.x) {
    const double v = a[i] + (double)b[i];
    out[i] = v;
    if (out32) out32[i] = (float)v;
  }
}

// M <- (M + M^T)/2 by 32x32 tiles of the upper triangle (tile pairs staged in LDS)
template <typename T>
__global__ void k_symmetrize(int n, T *M) {
  __shared__ double a[32][33], b[32][33];
  const int T32 = (n + 31) / 32;
  int bid = blockIdx.x, bi = 0, start = 0;
  while (start + (T32 - bi) <= bid) {
    start += T32 - bi;
    ++bi;
  }
  const int bj = bi + (bid - start);
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    int i = bi * 32 + r, j = bj * 32 + tx;
    a[r][tx] = (i < n && j < n) ? (double)M[(size_t)i * n + j] : 0.0;
    i = bj * 32 + r;
    j = bi * 32 + tx;
    b[r][tx] = (i < n && j < n) ? (double)M[(size_t)i * n + j] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    int i = bi * 32 + r, j = bj * 32 + tx;
    const double v = 0.5 * (a[r][tx] + b[tx][r]);
    if (i < n && j < n) M[(size_t)i * n + j] = (T)v;
    i = bj * 32 + r;
    j = bi * 32 + tx;
    const double w = 0.5 * (b[r][tx] + a[tx][r]);
    if (i < n && j < n && bi != bj) M[(size_t)i * n + j] = (T)w;
  }
}

__global__ void k_lincomb(size_t n2, int k, const double *const *M, const double *coef, double *out) {
  __shared__ double c[40];
  __shared__ const double *mp[40];
  if (threadIdx.x < k) {
    c[threadIdx.x] = coef[threadIdx.x];
    mp[threadIdx.x] = M[threadIdx.x];
  }
  __syncthreads();
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n2;
       i += (size_t)gridDim.x * blockDim.x) {
    double v = 0.0;
    for (int j = 0; j < k; ++j) v += c[j] * mp[j][i];
    out[i] = v;
  }
}

__device__ inline double block_sum(double v, double *sh) {
  // 256 threads
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return r;
}

struct PtrPack {
  const void *x[MAXK];
  const void *y[MAXK];
};

// All k dot products in one pass over the elements.  Pairs that repeat the
// previous pair's x (or y) matrix reuse the loaded values, so a matrix shared
// by consecutive pairs (the new direction in Gram-Schmidt, W_k in a row of
// the overlap matrix) is read once.  Each thread takes two consecutive
// elements per step (one 16-byte load per FP64 matrix) and issues the loads
// of all k pairs before the first product, so every stream has a load in
// flight at once; KB (4, 8 or 16) bounds k for the register arrays.  An odd
// last element goes to thread 0 of block 0.  The summation order is fixed.
template <typename T> struct Pair2;
template <> struct Pair2<double> { typedef double2 type; };
template <> struct Pair2<float> { typedef float2 type; };

template <typename T, int KB>
__global__ __launch_bounds__(256) void k_dots_partial(size_t n2, int k, PtrPack pp, double *part) {
  typedef typename Pair2<T>::type P2;
  __shared__ double sh[4];
  double v[KB];
#pragma unroll
  for (int a = 0; a < KB; ++a) v[a] = 0.0;
  const size_t h = n2 / 2, stride = (size_t)gridDim.x * blockDim.x;
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < h; q += stride) {
    P2 xs[KB], ys[KB];
#pragma unroll
    for (int a = 0; a < KB; ++a) {
      if (a < k) {
        if (a == 0 || pp.x[a] != pp.x[a - 1])
          xs[a] = ((const P2 *)pp.x[a])[q];
        else
          xs[a] = xs[a - 1];
        if (a == 0 || pp.y[a] != pp.y[a - 1])
          ys[a] = ((const P2 *)pp.y[a])[q];
        else
          ys[a] = ys[a - 1];
      }
    }
#pragma unroll
    for (int a = 0; a < KB; ++a) {
      if (a < k) {
        v[a] += (double)xs[a].x * (double)ys[a].x;
        v[a] += (double)xs[a].y * (double)ys[a].y;
      }
    }
  }
  if ((n2 & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    const size_t i = n2 - 1;
#pragma unroll
    for (int a = 0; a < KB; ++a)
      if (a < k) v[a] += (double)((const T *)pp.x[a])[i] * (double)((const T *)pp.y[a])[i];
  }
#pragma unroll
  for (int a = 0; a < KB; ++a) {
    if (a < k) {
      const double t = block_sum(v[a], sh);
      if (threadIdx.x == 0) part[(size_t)a * gridDim.x + blockIdx.x] = t;
    }
  }
}

// Gram-Schmidt update with the next reduction in the same pass:
// out = v - sum_{j<k} c_j V_j (subtractions in j order), and the block
// partials of <V_j, out> for j < k (SELF = false, the next sweep's
// coefficients) or of <out, out> (SELF = true, the norm).  The pointers V_j
// and the coefficients c_j are device arrays.  Each thread takes two
// consecutive elements per step; an odd last element goes to thread 0 of
// block 0.  Partials: part[a * gridDim.x + block].
constexpr int ORTH_KMAX = 32;
template <int KB, bool SELF>
__global__ __launch_bounds__(256) void k_orth_dots(size_t n2, int k, const double *v, const double *const *Vs,
                                                   const double *c, double *out, double *part) {
  __shared__ double cs[ORTH_KMAX];
  __shared__ const double *vp[ORTH_KMAX];
  __shared__ double sh[4];
  if (threadIdx.x < k) {
    cs[threadIdx.x] = c[threadIdx.x];
    vp[threadIdx.x] = Vs[threadIdx.x];
  }
  __syncthreads();
  constexpr int ND = SELF ? 1 : KB;
  double d[ND];
#pragma unroll
  for (int a = 0; a < ND; ++a) d[a] = 0.0;
  const size_t h = n2 / 2, stride = (size_t)gridDim.x * blockDim.x;
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < h; q += stride) {
    double2 x = ((const double2 *)v)[q], w[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j)
      if (j < k) w[j] = ((const double2 *)vp[j])[q];
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      if (j < k) {
        x.x -= cs[j] * w[j].x;
        x.y -= cs[j] * w[j].y;
      }
    }
    ((double2 *)out)[q] = x;
    if (SELF) {
      d[0] += x.x * x.x;
      d[0] += x.y * x.y;
    } else {
#pragma unroll
      for (int j = 0; j < ND; ++j) {
        if (j < k) {
          d[j] += w[j].x * x.x;
          d[j] += w[j].y * x.y;
        }
      }
    }
  }
  if ((n2 & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    const size_t i = n2 - 1;
    double x = v[i];
    for (int j = 0; j < k; ++j) x -= cs[j] * vp[j][i];
    out[i] = x;
    if (SELF) {
      d[0] += x * x;
    } else {
#pragma unroll
      for (int j = 0; j < ND; ++j)
        if (j < k) d[j] += vp[j][i] * x;
    }
  }
  const int nd = SELF ? 1 : k;
#pragma unroll
  for (int a = 0; a < ND; ++a) {
    if (a < nd) {
      const double t = block_sum(d[a], sh);
      if (threadIdx.x == 0) part[(size_t)a * gridDim.x + blockIdx.x] = t;
    }
  }
}

__global__ __launch_bounds__(256) void k_final(int k, int nb, const double *part, double *res) {
  __shared__ double sh[4];
  for (int a = 0; a < k; ++a) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) v += part[(size_t)a * nb + b];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) res[a] = v;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_trace_partial(int n, const void *M, double *part) {
  __shared__ double sh[4];
  double v = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    v += ld<T>(M, (size_t)i * n + i);
  v = block_sum(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// Lanczos recurrence for spectral bounds.  w = F q_j (one wavefront per row,
// F symmetric, row-major), then one workgroup finishes the step:
// alpha_j = w.q_j, w <- w - alpha_j q_j - beta_{j-1} q_{j-1}, beta_j = |w|,
// q_{j+1} = w / beta_j.  Q holds the Lanczos vectors row by row; ab[2j] and
// ab[2j+1] receive alpha_j and beta_j.
// The pair version reads rows as 16-byte pairs (n even, F and q 16-byte aligned).
__global__ __launch_bounds__(256) void k_symv(int n, const double *F, const double *q, double *w) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const double *f = F + (size_t)row * n;
  double acc = 0.0;
  for (int j = lane; j < n; j += 64) acc += f[j] * q[j];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if (lane == 0) w[row] = acc;
}
__global__ __launch_bounds__(256) void k_symv2(int n, const double *F, const double *q, double *w) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const double2 *f = (const double2 *)(F + (size_t)row * n);
  const double2 *q2 = (const double2 *)q;
  double acc = 0.0;
  for (int j = lane; j < n / 2; j += 64) {
    const double2 a = f[j], b = q2[j];
    acc += a.x * b.x;
    acc += a.y * b.y;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if (lane == 0) w[row] = acc;
}

// sum over a workgroup of LB threads (a multiple of 64); the result is returned to every thread
template <int LB>
__device__ inline double block_sum_all(double v, double *sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int i = 0; i < LB / 64; ++i) r += sh[i];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(1024) void k_lanczos_step(int n, int j, double *Q, const double *w,
                                                       double *ab) {
  __shared__ double sh[16];
  const double *qj = Q + (size_t)j * n;
  const double *qp = j > 0 ? Q + (size_t)(j - 1) * n : nullptr;
  double *qn = Q + (size_t)(j + 1) * n;
  const double bprev = j > 0 ? ab[2 * j - 1] : 0.0;
  double a = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) a += w[i] * qj[i];
  a = block_sum_all<1024>(a, sh);
  double b = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) {
    double v = w[i] - a * qj[i];
    if (qp) v -= bprev * qp[i];
    qn[i] = v;
    b += v * v;
  }
  b = block_sum_all<1024>(b, sh);
  const double bc = sqrt(b);
  if (threadIdx.x == 0) {
    ab[2 * j] = a;
    ab[2 * j + 1] = bc;
  }
  const double inv = bc > 0.0 ? 1.0 / bc : 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) qn[i] *= inv;
}

// Lanczos start vector: q_i = u_i - 1/2 with u_i the top 53 bits of the
// SplitMix64 output for index i (Steele, Lea and Flood, OOPSLA 2014), scaled to
// unit norm; one workgroup, integer arithmetic, so the same bits on every call.
__global__ __launch_bounds__(1024) void k_lanczos_start(int n, double *q) {
  __shared__ double sh[16];
  double ss = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) {
    unsigned long long z = (unsigned long long)(i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const double v = (double)(z >> 11) * 0x1.0p-53 - 0.5;
    q[i] = v;
    ss += v * v;
  }
  ss = block_sum_all<1024>(ss, sh);
  const double inv = 1.0 / sqrt(ss);
  for (int i = threadIdx.x; i < n; i += 1024) q[i] *= inv;
}

// Gershgorin: one wavefront per row
__global__ __launch_bounds__(256) void k_gersh_rows(int n, const double *F, double *lohi) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  double s = 0.0;
  for (int j = lane; j < n; j += 64)
    if (j != row) s += fabs(F[(size_t)row * n + j]);
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if (lane == 0) {
    const double d = F[(size_t)row * n + row];
    lohi[2 * row] = d - s;
    lohi[2 * row + 1] = d + s;
  }
}

__global__ __launch_bounds__(256) void k_gersh_final(int n, const double *lohi, double *res) {
  // fmin / fmax drop NaN operands, so a NaN row is counted apart and turns
  // the result into NaN (the caller reports a non-finite matrix)
  __shared__ double smin[256], smax[256];
  __shared__ int snan[256];
  double lo = INFINITY, hi = -INFINITY;
  int bad = 0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const double a = lohi[2 * i], b = lohi[2 * i + 1];
    bad |= !(a == a) || !(b == b);
    lo = fmin(lo, a);
    hi = fmax(hi, b);
  }
  smin[threadIdx.x] = lo;
  smax[threadIdx.x] = hi;
  snan[threadIdx.x] = bad;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + o]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + o]);
      snan[threadIdx.x] |= snan[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    res[0] = snan[0] ? NAN : smin[0];
    res[1] = snan[0] ? NAN : smax[0];
  }
}

// ---- chemical potential: solve sum_{k<6} (1-c)^k tau_k = n_occ for dmu, c = exp(-beta dmu),
// by bisection on dmu in [-0.3/beta, 0.3/beta] (the truncated series is accurate there for
// the warm starts of a trajectory).  out[0] = dmu, out[1] = c, out[2] = 2/(1+c) (Newton-Schulz
// start for (cI + (1-c)D)^-1), out[3] = flag (1: root outside the bracket, clamped).
__global__ void k_mu_series(const double *tau, double n_occ, double beta, double tol_n, double *out) {
  if (threadIdx.x != 0) return;
  auto g = [&](double dmu) {
    const double x = -expm1(-beta * dmu);  // 1 - c
    double s = 0.0, p = 1.0;
    for (int k = 0; k < 6; ++k) {
      s += p * tau[k];
      p *= x;
    }
    return s - n_occ;
  };
  double lo = -SERIES_STEP / beta, hi = SERIES_STEP / beta;
  double flag = 0.0;
  double dmu;
  if (fabs(tau[0] - n_occ) <= tol_n) {
    dmu = 0.0;  // the trace is already N_occ to the storage precision
  } else if (g(lo) > 0.0) {
    dmu = lo;
    flag = 1.0;
  } else if (g(hi) < 0.0) {
    dmu = hi;
    flag = 1.0;
  } else {
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      if (g(mid) < 0.0)
        lo = mid;
      else
        hi = mid;
    }
    dmu = 0.5 * (lo + hi);
  }
  const double c = exp(-beta * dmu);
  out[0] = dmu;
  out[1] = c;
  out[2] = 2.0 / (1.0 + c);
  out[3] = flag;
  out[4] = 1.0 - c;
}

// Newton step on mu from t01 = (Tr D, Tr D(I-D)): dmu = (n_occ - t0) / (beta t1).
// out layout as k_mu_series.
__global__ void k_mu_newton(const double *t01, double n_occ, double beta, double tol_n, double *out) {
  if (threadIdx.x != 0) return;
  const double t0 = t01[0], t1 = t01[1];
  double dmu = (t1 > 0.0 && fabs(n_occ - t0) > tol_n) ? (n_occ - t0) / (beta * t1) : 0.0;
  const double lim = MU_STEP / beta;
  double flag = 0.0;
  if (dmu > lim) {
    dmu = lim;
    flag = 1.0;
  }
  if (dmu < -lim) {
    dmu = -lim;
    flag = 1.0;
  }
  const double c = exp(-beta * dmu);
  out[0] = dmu;
  out[1] = c;
  out[2] = 2.0 / (1.0 + c);
  out[3] = flag;
  out[4] = 1.0 - c;
}

// Krylov: solve O coef = rhs (k x k, FP64, Gaussian elimination with partial
// pivoting) and resid2 = ||sum W_i c_i - W0||^2 = c^T O c - 2 c^T rhs + ||W0||^2
// (the last term is read from resid2[1] on entry).
// k_rank (device, may be null): a basis that broke down at rank r >= 0 solves
// only the leading r x r system (the remaining coefficients are zero).
// One wavefront; the augmented matrix lives in LDS (no per-lane scratch).
// Lane 0 picks each pivot and does the back substitution; in each
// elimination, lane r updates row r, so every entry sees the operations of a
// sequential elimination in the same order.
__global__ __launch_bounds__(64) void k_krylov_solve(int k, const double *O, const double *rhs, double *coef,
                                                     double *resid2, const double *k_rank) {
  __shared__ double a[32][33];
  __shared__ double x[32];
  __shared__ int piv_s, sing_s;
  const int t = threadIdx.x;
  const int kfull = k;
  if (k_rank && *k_rank >= 0.0 && (int)*k_rank < k) k = (int)*k_rank;
  for (int idx = t; idx < k * (k + 1); idx += 64) {
    const int i = idx / (k + 1), j = idx - i * (k + 1);
    a[i][j] = j < k ? O[i * 32 + j] : rhs[i];
  }
  if (t == 0) sing_s = 0;
  __syncthreads();
  for (int c = 0; c < k; ++c) {
    if (t == 0) {
      int piv = c;
      for (int r = c + 1; r < k; ++r)
        if (fabs(a[r][c]) > fabs(a[piv][c])) piv = r;
      piv_s = piv;
    }
    __syncthreads();
    const int piv = piv_s;
    if (piv != c)
      for (int j = t; j <= k; j += 64) {
        const double tmp = a[c][j];
        a[c][j] = a[piv][j];
        a[piv][j] = tmp;
      }
    __syncthreads();
    // every lane reads the same pivot, so the exit is uniform
    if (a[c][c] == 0.0) {
      if (t == 0) sing_s = 1;
      break;
    }
    if (t > c && t < k) {
      const double f = a[t][c] / a[c][c];
      for (int j = c; j <= k; ++j) a[t][j] -= f * a[c][j];
    }
    __syncthreads();
  }
  __syncthreads();
  if (t != 0) return;
  const int singular = sing_s;
  for (int i = k - 1; i >= 0; --i) {
    double s = singular ? 0.0 : a[i][k];
    if (!singular) {
      for (int j = i + 1; j < k; ++j) s -= a[i][j] * x[j];
      s /= a[i][i];
    }
    x[i] = s;
  }
  double q = 0.0, l = 0.0;
  for (int i = k; i < kfull; ++i) coef[i] = 0.0;
  for (int i = 0; i < k; ++i) {
    coef[i] = x[i];
    l += x[i] * rhs[i];
    for (int j = 0; j < k; ++j) q += x[i] * O[i * 32 + j] * x[j];
  }
  resid2[0] = q - 2.0 * l + resid2[1];
  resid2[2] = singular;
}

__global__ void k_xverlet(size_t n2, const double *X0, const double *X1, const double *X2,
                          const double *X3, const double *X4, const double *X5, const double *X6,
                          const double *Y, double kappa, double alpha, double c0, double c1,
                          double c2, double c3, double c4, double c5, double c6, double *out) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n2;
       i += (size_t)gridDim.x * blockDim.x) {
    const double x0 = X0[i], x1 = X1[i];
    const double damp = c0 * x0 + c1 * x1 + c2 * X2[i] + c3 * X3[i] + c4 * X4[i] + c5 * X5[i] +
                        c6 * X6[i];
    out[i] = 2.0 * x0 - x1 - kappa * Y[i] + alpha * damp;
  }
}

__global__ void k_kick_drift(int n3, double *R, double *V, const double *A, double dt, int drift) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n3) return;
  const double v = V[i] + 0.5 * dt * A[i];
  V[i] = v;
  if (drift) R[i] += dt * v;
}

__global__ void k_baoab_pre(int n3, double *R, double *V, const double *A, double dt, double c1, double c2,
                            const double *xi) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n3) return;
  double v = V[i] + 0.5 * dt * A[i];
  double r = R[i] + 0.5 * dt * v;
  v = c1 * v + c2 * xi[i];
  R[i] = r + 0.5 * dt * v;
  V[i] = v;
}

__global__ void k_accel(int n3, const double *f, double s, double *A) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n3) A[i] = f[i] * s;
}

inline int grid_for(size_t n) {
  size_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

int reduce_partials_capacity() { return RED_BLOCKS * MAXK + 2 * 65536; }

void axpby(int n2, double a, const void *x, double b, const void *y, void *out, int is32,
           hipStream_t s) {
  if (is32)
    hipLaunchKernelGGL(k_axpby<float>, dim3(grid_for(n2)), dim3(256), 0, s, (size_t)n2, a, x, b, y, out);
  else
    hipLaunchKernelGGL(k_axpby<double>, dim3(grid_for(n2)), dim3(256), 0, s, (size_t)n2, a, x, b, y, out);
}

void axpbyI_dev(int n, const double *a_dev, double a, const void *x, const double *b_dev, double b,
                const void *y, const double *g_dev, double g, void *out, int is32, hipStream_t s) {
  const size_t n2 = (size_t)n * n;
  if (is32)
    hipLaunchKernelGGL(k_axpbyI<float>, dim3(grid_for(n2)), dim3(256), 0, s, n, a_dev, a, x, b_dev, b, y,
                       g_dev, g, out);
  else
    hipLaunchKernelGGL(k_axpbyI<double>, dim3(grid_for(n2)), dim3(256), 0, s, n, a_dev, a, x, b_dev, b,
                       y, g_dev, g, out);
}

void convert(int n2, const void *in, int in32, void *out, int out32, hipStream_t s, double scale) {
  const dim3 g(grid_for(n2)), b(256);
  if (in32 && out32)
    hipLaunchKernelGGL((k_convert<float, float>), g, b, 0, s, (size_t)n2, in, out, scale);
  else if (in32)
    hipLaunchKernelGGL((k_convert<float, double>), g, b, 0, s, (size_t)n2, in, out, scale);
  else if (out32)
    hipLaunchKernelGGL((k_convert<double, float>), g, b, 0, s, (size_t)n2, in, out, scale);
  else
    hipLaunchKernelGGL((k_convert<double, double>), g, b, 0, s, (size_t)n2, in, out, scale);
}

void canon_out(int n2, const void *H, const void *M, const double *s_dev, const double *sub, double *out,
               int is32, hipStream_t s) {
  if (is32)
    hipLaunchKernelGGL(k_canon_out<float>, dim3(grid_for(n2)), dim3(256), 0, s, (size_t)n2, H, M, s_dev, sub,
                       out);
  else
    hipLaunchKernelGGL(k_canon_out<double>, dim3(grid_for(n2)), dim3(256), 0, s, (size_t)n2, H, M, s_dev, sub,
                       out);
}

void add_mixed(int n2, const double *a, const float *b, double *out, float *out32, hipStream_t s) {
  hipLaunchKernelGGL(k_add_mixed, dim3(grid_for(n2)), dim3(256), 0, s, (size_t)n2, a, b, out, out32);
}

void symmetrize(int n, void *M, int is32, hipStream_t s) {
  const int T = (n + 31) / 32;
  const int blocks = T * (T + 1) / 2;
  if (is32)
    hipLaunchKernelGGL(k_symmetrize<float>, dim3(blocks), dim3(256), 0, s, n, (float *)M);
  else
    hipLaunchKernelGGL(k_symmetrize<double>, dim3(blocks), dim3(256), 0, s, n, (double *)M);
}

void lincomb_dev(int n2, int k, const double *const *M, const double *coef, double *out,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_lincomb, dim3(grid_for(n2)), dim3(256), 0, s, (size_t)n2, k, M, coef, out);
}

void dots(int n2, int k, const void *const *X, const void *const *Y, double *res, int is32,
          double *partials, hipStream_t s) {
  PtrPack pp{};
  for (int i = 0; i < k; ++i) {
    pp.x[i] = X[i];
    pp.y[i] = Y[i];
  }
  int nb = grid_for(n2);
  if (nb > RED_BLOCKS) nb = RED_BLOCKS;
  if (is32) {
    if (k <= 4)
      hipLaunchKernelGGL((k_dots_partial<float, 4>), dim3(nb), dim3(256), 0, s, (size_t)n2, k, pp, partials);
    else if (k <= 8)
      hipLaunchKernelGGL((k_dots_partial<float, 8>), dim3(nb), dim3(256), 0, s, (size_t)n2, k, pp, partials);
    else
      hipLaunchKernelGGL((k_dots_partial<float, 16>), dim3(nb), dim3(256), 0, s, (size_t)n2, k, pp, partials);
  } else {
    if (k <= 4)
      hipLaunchKernelGGL((k_dots_partial<double, 4>), dim3(nb), dim3(256), 0, s, (size_t)n2, k, pp, partials);
    else if (k <= 8)
      hipLaunchKernelGGL((k_dots_partial<double, 8>), dim3(nb), dim3(256), 0, s, (size_t)n2, k, pp, partials);
    else
      hipLaunchKernelGGL((k_dots_partial<double, 16>), dim3(nb), dim3(256), 0, s, (size_t)n2, k, pp, partials);
  }
  hipLaunchKernelGGL(k_final, dim3(1), dim3(256), 0, s, k, nb, partials, res);
}

void orth_dots(int n2, int k, const double *v, const double *const *Vs, const double *c, double *out, int self,
               double *res, double *partials, hipStream_t s) {
  int nb = grid_for(n2);
  if (nb > RED_BLOCKS) nb = RED_BLOCKS;
#define XL_ORTH(KB)                                                                                       \
  if (self)                                                                                               \
    hipLaunchKernelGGL((k_orth_dots<KB, true>), dim3(nb), dim3(256), 0, s, (size_t)n2, k, v, Vs, c, out,  \
                       partials);                                                                         \
  else                                                                                                    \
    hipLaunchKernelGGL((k_orth_dots<KB, false>), dim3(nb), dim3(256), 0, s, (size_t)n2, k, v, Vs, c, out, \
                       partials);
  if (k <= 4) {
    XL_ORTH(4)
  } else if (k <= 8) {
    XL_ORTH(8)
  } else {
    XL_ORTH(ORTH_KMAX)
  }
#undef XL_ORTH
  hipLaunchKernelGGL(k_final, dim3(1), dim3(256), 0, s, self ? 1 : k, nb, partials, res);
}

void trace(int n, const void *M, double *res, int is32, double *partials, hipStream_t s) {
  int nb = (n + 255) / 256;
  if (nb > RED_BLOCKS) nb = RED_BLOCKS;
  if (is32)
    hipLaunchKernelGGL(k_trace_partial<float>, dim3(nb), dim3(256), 0, s, n, M, partials);
  else
    hipLaunchKernelGGL(k_trace_partial<double>, dim3(nb), dim3(256), 0, s, n, M, partials);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(256), 0, s, 1, nb, partials, res);
}

void gershgorin(int n, const double *F, double *res, double *partials, hipStream_t s) {
  hipLaunchKernelGGL(k_gersh_rows, dim3((n + 3) / 4), dim3(256), 0, s, n, F, partials);
  hipLaunchKernelGGL(k_gersh_final, dim3(1), dim3(256), 0, s, n, partials, res);
}

void poly_comb(int n, const void *const X[4], const double a[4], double g, void *out, int is32,
               hipStream_t s) {
  const size_t n2 = (size_t)n * n;
  if (is32)
    hipLaunchKernelGGL(k_poly_comb<float>, dim3(grid_for(n2)), dim3(256), 0, s, n, X[0], X[1], X[2], X[3],
                       a[0], a[1], a[2], a[3], g, out);
  else
    hipLaunchKernelGGL(k_poly_comb<double>, dim3(grid_for(n2)), dim3(256), 0, s, n, X[0], X[1], X[2], X[3],
                       a[0], a[1], a[2], a[3], g, out);
}

void convert_t(int n, const double *in, float *out, hipStream_t s) {
  const int g = (n + 31) / 32;
  hipLaunchKernelGGL(k_convert_t, dim3(g, g), dim3(256), 0, s, n, in, out);
}

void lanczos_start(int n, double *Q, hipStream_t s) {
  hipLaunchKernelGGL(k_lanczos_start, dim3(1), dim3(1024), 0, s, n, Q);
}

void lanczos(int n, int k, const double *F, double *Q, double *w, double *ab, hipStream_t s) {
  // Q is the library's (16-byte aligned, rows of even length); F may be the caller's
  const bool pairs = n % 2 == 0 && ((uintptr_t)F % 16) == 0 && ((uintptr_t)Q % 16) == 0;
  for (int j = 0; j < k; ++j) {
    const double *qj = Q + (size_t)j * n;
    if (pairs)
      hipLaunchKernelGGL(k_symv2, dim3((n + 3) / 4), dim3(256), 0, s, n, F, qj, w);
    else
      hipLaunchKernelGGL(k_symv, dim3((n + 3) / 4), dim3(256), 0, s, n, F, qj, w);
    hipLaunchKernelGGL(k_lanczos_step, dim3(1), dim3(1024), 0, s, n, j, Q, w, ab);
  }
}

void mu_series_solve(const double *tau, double n_occ, double beta, double tol_n, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_mu_series, dim3(1), dim3(64), 0, s, tau, n_occ, beta, tol_n, out);
}

void mu_newton(const double *t01, double n_occ, double beta, double tol_n, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_mu_newton, dim3(1), dim3(64), 0, s, t01, n_occ, beta, tol_n, out);
}

void krylov_solve(int k, const double *O, const double *rhs, double *coef, double *resid2,
                  const double *k_rank, hipStream_t s) {
  hipLaunchKernelGGL(k_krylov_solve, dim3(1), dim3(64), 0, s, k, O, rhs, coef, resid2, k_rank);
}

void x_verlet(int n2, const double *const *Xk, const double *Y, double kappa, double alpha,
              const double *c, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_xverlet, dim3(grid_for(n2)), dim3(256), 0, s, (size_t)n2, Xk[0], Xk[1], Xk[2],
                     Xk[3], Xk[4], Xk[5], Xk[6], Y, kappa, alpha, c[0], c[1], c[2], c[3], c[4],
                     c[5], c[6], out);
}

void kick_drift(int n3, double *R, double *V, const double *A, double dt, int drift,
                hipStream_t s) {
  hipLaunchKernelGGL(k_kick_drift, dim3((n3 + 255) / 256), dim3(256), 0, s, n3, R, V, A, dt, drift);
}

void baoab_pre(int n3, double *R, double *V, const double *A, double dt, double c1, double c2,
               const double *xi, hipStream_t s) {
  hipLaunchKernelGGL(k_baoab_pre, dim3((n3 + 255) / 256), dim3(256), 0, s, n3, R, V, A, dt, c1, c2, xi);
}

void accel(int n3, const double *frc, double sc, double *A, hipStream_t s) {
  hipLaunchKernelGGL(k_accel, dim3((n3 + 255) / 256), dim3(256), 0, s, n3, frc, sc, A);
}

}  // namespace xl
