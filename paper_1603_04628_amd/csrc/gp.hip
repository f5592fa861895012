// gp.hip -- Gaussian-process surrogate on the device, FP64 throughout
// (paper Sec. 2.2-2.3):
//   covariance   C = sigma_f^2 exp(-d^2 / 2 l^2) + sigma_n^2 I
//                (Eqs. quadraticKernelEq, d2Eq, covarianceEq)
//   factor       C = L L^T (blocked right-looking Cholesky, panels of 32)
//   weights      alpha = C^-1 y by two triangular solves
//   prediction   mean = K* alpha (Eq. predMeanEq),
//                var = sigma_f^2 - |L^-1 k*|^2 (diagonal of Eq. predVarEq), with
//                L^-1 formed once per factorisation so that a query is a
//                parallel product, not a sequential solve
//   evidence     -1/2 y^T alpha - sum log L_ii - n/2 log 2 pi (Eq. evidenceEq)
// Options: each point's own noise variance on the diagonal (heteroscedastic),
// the periodic kernel of App. B (Eq. periodicKernel) on a single input, and
// hyperparameters that maximise the evidence (gp_optimize).
// Database sizes here are hundreds of points: the triangular solves are
// latency bound, so one workgroup walks the columns with barriers; the
// factorisation spreads each panel's update over many workgroups, and
// prediction gives each query a workgroup of its own.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "engine.h"

struct hmd_gp {
  hmd_ctx* ctx = nullptr;
  hmd_gp_hyper hyp{};
  int d = 0;
  int n = 0, cap = 0;
  std::vector<double> X, y, se;  // database (host copy)
  double scale[4] = {1, 1, 1, 1};
  double s_q = 1.0, sigma_n = 0.0;
  double* dX = nullptr;      // cap x 4, row-major
  double* dy = nullptr;      // scaled outputs
  double* dL = nullptr;      // cap x cap, column-major (leading dimension cap)
  double* dLi = nullptr;     // L^-1, same layout (lower triangle)
  double* dalpha = nullptr;  // C^-1 y
  double* dtmp = nullptr;    // cap
  double* dnoise = nullptr;  // cap: per-point noise variances (heteroscedastic)
  double* dq = nullptr;      // query staging
  double* dout = nullptr;    // predictions / scalars
  int* dinfo = nullptr;
  size_t q_cap = 0;
};

namespace hmd {
namespace {

constexpr int GP_MAXD = 4;
constexpr int GP_MAXN = 6144;  // database points: k* and the substitution vectors fit one workgroup's LDS

struct KParams {
  double inv_scale[GP_MAXD];
  double sf2, inv_2l2, sn2;
  double pi_over_T;  // periodic kernel: pi / T
  int d;
  int kind;          // 0 squared exponential (Eq. quadraticKernelEq), 1 periodic (Eq. periodicKernel)
};

// K(a, b): sigma_f^2 exp(-d^2 / 2 l^2) on the normalised distance of Eq.
// d2Eq, or sigma_f^2 exp(-2 sin^2(pi |t - t'| / T) / l^2) on the first input
__device__ __forceinline__ double sqexp(const double* a, const double* b, const KParams& P) {
  if (P.kind == 1) {
    const double sn = sin(P.pi_over_T * fabs(a[0] - b[0]));
    return P.sf2 * exp(-4.0 * sn * sn * P.inv_2l2);
  }
  double d2 = 0.0;
  for (int k = 0; k < P.d; ++k) {
    const double t = (a[k] - b[k]) * P.inv_scale[k];
    d2 += t * t;
  }
  return P.sf2 * exp(-d2 * P.inv_2l2);
}

// Lower triangle (and diagonal) of C for rows/cols [0, n); the diagonal
// takes noise[i] when given (per-point variances), else sn2.
__global__ void k_gp_cov(int n, int ld, const double* __restrict__ X, KParams P, const double* __restrict__ noise,
                         double* __restrict__ L) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n || j >= n || i < j) return;
  double c = sqexp(X + GP_MAXD * i, X + GP_MAXD * j, P);
  if (i == j) c += noise ? noise[i] : P.sn2;
  L[i + size_t(j) * ld] = c;
}

// In-place blocked right-looking Cholesky of the lower triangle, panels of
// CB columns, three launches per panel: the diagonal block factored in LDS
// by one workgroup, the rows below it solved against it (one row per
// thread), and the trailing lower triangle updated in CB x CB tiles.
// info = 0 on success, k + 1 if the k-th pivot is not positive; once set,
// the remaining launches return at once.
constexpr int CB = 32;

__global__ __launch_bounds__(256) void k_chol_diag(int n, int ld, double* __restrict__ A, int* __restrict__ info,
                                                   int k0) {
  __shared__ double a[CB][CB + 1];
  __shared__ int bad;
  const int tid = threadIdx.x, kb = min(CB, n - k0);
  if (k0 > 0 && *info != 0) return;  // an earlier pivot failed (uniform)
  if (tid == 0) bad = 0;
  for (int e = tid; e < kb * kb; e += blockDim.x) {
    const int r = e / kb, c = e % kb;
    a[r][c] = r >= c ? A[(k0 + r) + size_t(k0 + c) * ld] : 0.0;
  }
  __syncthreads();
  for (int c = 0; c < kb; ++c) {
    if (tid == 0) {
      const double d = a[c][c];
      if (!(d > 0.0)) bad = k0 + c + 1;
      else a[c][c] = sqrt(d);
    }
    __syncthreads();
    if (bad) break;
    if (tid > c && tid < kb) a[tid][c] /= a[c][c];
    __syncthreads();
    for (int e = tid; e < kb * kb; e += blockDim.x) {
      const int r = e / kb, q = e % kb;
      if (q > c && r >= q) a[r][q] -= a[r][c] * a[q][c];
    }
    __syncthreads();
  }
  for (int e = tid; e < kb * kb; e += blockDim.x) {
    const int r = e / kb, c = e % kb;
    if (r >= c) A[(k0 + r) + size_t(k0 + c) * ld] = a[r][c];
  }
  if (tid == 0) *info = bad;
}

// Rows k0 + kb .. n - 1 of the panel: x L_kk^T = a, by forward substitution
// along the row.
__global__ __launch_bounds__(256) void k_chol_panel(int n, int ld, double* __restrict__ A,
                                                    const int* __restrict__ info, int k0) {
  __shared__ double l[CB][CB + 1];
  if (*info != 0) return;
  const int tid = threadIdx.x, kb = CB;  // a panel with rows below it is full width
  for (int e = tid; e < kb * kb; e += blockDim.x) {
    const int r = e / kb, c = e % kb;
    l[r][c] = r >= c ? A[(k0 + r) + size_t(k0 + c) * ld] : 0.0;
  }
  __syncthreads();
  const int i = k0 + kb + blockIdx.x * blockDim.x + tid;
  if (i >= n) return;
  double x[CB];
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    double t = A[i + size_t(k0 + c) * ld];
#pragma unroll
    for (int m = 0; m < c; ++m) t -= x[m] * l[c][m];
    x[c] = t / l[c][c];
    A[i + size_t(k0 + c) * ld] = x[c];
  }
}

// Trailing update A_ij -= sum_c P_ic P_jc over the lower triangle from row
// and column k0 + CB on, one CB x CB tile per workgroup (tiles numbered row
// by row over the lower triangle of tiles).
__global__ __launch_bounds__(256) void k_chol_update(int n, int ld, double* __restrict__ A,
                                                     const int* __restrict__ info, int k0) {
  __shared__ double pi[CB][CB + 1], pj[CB][CB + 1];
  if (*info != 0) return;
  const int t0 = k0 + CB, b = blockIdx.x;
  int ti = int((sqrt(8.0 * double(b) + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= b) ++ti;
  while (ti * (ti + 1) / 2 > b) --ti;
  const int tj = b - ti * (ti + 1) / 2;
  const int i0 = t0 + ti * CB, j0 = t0 + tj * CB;
  const int tid = threadIdx.x;
  for (int e = tid; e < CB * CB; e += blockDim.x) {
    const int r = e % CB, c = e / CB;
    pi[r][c] = i0 + r < n ? A[(i0 + r) + size_t(k0 + c) * ld] : 0.0;
    pj[r][c] = j0 + r < n ? A[(j0 + r) + size_t(k0 + c) * ld] : 0.0;
  }
  __syncthreads();
  const int r = tid % CB;
  for (int q = tid / CB; q < CB; q += blockDim.x / CB) {
    const int i = i0 + r, j = j0 + q;
    if (i < n && j <= i) {
      double t = 0.0;
#pragma unroll 8
      for (int c = 0; c < CB; ++c) t += pi[r][c] * pj[q][c];
      A[i + size_t(j) * ld] -= t;
    }
  }
}

// x = L^-1 b (lower) then, if `both`, x = L^-T x: column-oriented
// substitution in one workgroup; b is overwritten by the result.
__global__ __launch_bounds__(1024) void k_gp_solve(int n, int ld, const double* __restrict__ L, double* __restrict__ b,
                                                   int both) {
  __shared__ double xk;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int k = 0; k < n; ++k) {
    if (tid == 0) {
      xk = b[k] / L[k + size_t(k) * ld];
      b[k] = xk;
    }
    __syncthreads();
    for (int i = k + 1 + tid; i < n; i += nt) b[i] -= L[i + size_t(k) * ld] * xk;
    __syncthreads();
  }
  if (!both) return;
  for (int k = n - 1; k >= 0; --k) {
    if (tid == 0) {
      xk = b[k] / L[k + size_t(k) * ld];
      b[k] = xk;
    }
    __syncthreads();
    for (int i = tid; i < k; i += nt) b[i] -= L[k + size_t(i) * ld] * xk;
    __syncthreads();
  }
}

// Device-pointer interop: queries row-major with d columns -> the padded
// layout of the predict kernel; results (scaled back to output units) into
// separate mean and variance arrays.
__global__ void k_gp_pack(int m, int d, const double* __restrict__ src, double* __restrict__ dst) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  for (int k = 0; k < GP_MAXD; ++k) dst[size_t(q) * GP_MAXD + k] = k < d ? src[size_t(q) * d + k] : 0.0;
}

__global__ void k_gp_unpack(int m, int have_data, const double* __restrict__ res, double s_q, double sf2,
                            double* __restrict__ mean, double* __restrict__ var) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  mean[q] = have_data ? res[2 * q] * s_q : 0.0;
  var[q] = (have_data ? res[2 * q + 1] : sf2) * s_q * s_q;
}

// Column j of L^-1 per workgroup: forward substitution of L x = e_j, whose
// entries above j are zero. x lives in LDS (dynamic, n doubles); every
// thread derives the pivot value itself, so one barrier per step suffices.
__global__ __launch_bounds__(256) void k_gp_tri_inv(int n, int ld, const double* __restrict__ L,
                                                    double* __restrict__ Li) {
  extern __shared__ double x[];
  const int j = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  for (int i = j + tid; i < n; i += nt) x[i] = i == j ? 1.0 : 0.0;
  for (int k = j; k < n; ++k) {
    __syncthreads();
    const double xk = x[k] / L[k + size_t(k) * ld];
    // the pivot slot is not rewritten in this step, the others only by their owner
    for (int i = k + 1 + tid; i < n; i += nt) x[i] -= L[i + size_t(k) * ld] * xk;
    if (tid == 0) Li[k + size_t(j) * ld] = xk;
  }
}

// L grew by row r (its leading rows unchanged): row r of L^-1 is
// -(1 / L_rr) sum_{j<=k<r} L_rk (L^-1)_kj for j < r, and 1 / L_rr on the
// diagonal. One wavefront per column j; row r of L staged in LDS.
__global__ __launch_bounds__(256) void k_gp_inv_append_row(int r, int ld, const double* __restrict__ L,
                                                           double* __restrict__ Li) {
  extern __shared__ double lr[];
  const int tid = threadIdx.x, lane = tid & 63;
  for (int k = tid; k < r; k += blockDim.x) lr[k] = L[r + size_t(k) * ld];
  __syncthreads();
  const double inv_d = 1.0 / L[r + size_t(r) * ld];
  const int j = blockIdx.x * (blockDim.x / 64) + (tid >> 6);
  if (j > r) return;
  if (j == r) {
    if (lane == 0) Li[r + size_t(r) * ld] = inv_d;
    return;
  }
  const double* col = Li + size_t(j) * ld;
  double t = 0.0;
  for (int k = j + lane; k < r; k += 64) t += lr[k] * col[k];
  for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
  if (lane == 0) Li[r + size_t(j) * ld] = -t * inv_d;
}

// One query per workgroup: k* in LDS (dynamic, n doubles), mean = k* . alpha,
// variance = sigma_f^2 - |L^-1 k*|^2, both by block reduction.
__global__ __launch_bounds__(256) void k_gp_predict(int n, int ld, const double* __restrict__ X,
                                                    const double* __restrict__ Xq, const double* __restrict__ Li,
                                                    const double* __restrict__ alpha, KParams P,
                                                    double* __restrict__ out) {
  extern __shared__ double ks[];
  __shared__ double red[2][256];
  const int q = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  double sm = 0.0, sv = 0.0;
  for (int i = tid; i < n; i += nt) {
    const double k = sqexp(X + GP_MAXD * i, Xq + GP_MAXD * q, P);
    ks[i] = k;
    sm += k * alpha[i];
  }
  __syncthreads();
  for (int i = tid; i < n; i += nt) {  // row i of L^-1 k*: column-major reads are coalesced over i
    double w0 = 0.0, w1 = 0.0;
    int j = 0;
    for (; j + 1 <= i; j += 2) {
      w0 += Li[i + size_t(j) * ld] * ks[j];
      w1 += Li[i + size_t(j + 1) * ld] * ks[j + 1];
    }
    if (j == i) w0 += Li[i + size_t(j) * ld] * ks[j];
    const double w = w0 + w1;
    sv += w * w;
  }
  red[0][tid] = sm;
  red[1][tid] = sv;
  __syncthreads();
  for (int o = nt / 2; o > 0; o >>= 1) {
    if (tid < o) {
      red[0][tid] += red[0][tid + o];
      red[1][tid] += red[1][tid + o];
    }
    __syncthreads();
  }
  if (tid == 0) {
    out[2 * q] = red[0][0];
    out[2 * q + 1] = P.sf2 - red[1][0];
  }
}

// out[0] = y^T alpha, out[1] = sum log L_ii.
__global__ __launch_bounds__(256) void k_gp_lml(int n, int ld, const double* __restrict__ L,
                                                const double* __restrict__ y, const double* __restrict__ alpha,
                                                double* __restrict__ out) {
  __shared__ double r0[256], r1[256];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    a += y[i] * alpha[i];
    b += log(L[i + size_t(i) * ld]);
  }
  r0[threadIdx.x] = a;
  r1[threadIdx.x] = b;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      r0[threadIdx.x] += r0[threadIdx.x + o];
      r1[threadIdx.x] += r1[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = r0[0];
    out[1] = r1[0];
  }
}

// New last row of L for the point at index n: row = L^-1 c, then the pivot.
__global__ __launch_bounds__(1024) void k_gp_append_row(int n, int ld, const double* __restrict__ X, KParams P,
                                                        double* __restrict__ L, double* __restrict__ row,
                                                        int* __restrict__ info) {
  __shared__ double xk;
  __shared__ double red[1024];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < n; i += nt) row[i] = sqexp(X + GP_MAXD * i, X + GP_MAXD * n, P);
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (tid == 0) {
      xk = row[k] / L[k + size_t(k) * ld];
      row[k] = xk;
    }
    __syncthreads();
    for (int i = k + 1 + tid; i < n; i += nt) row[i] -= L[i + size_t(k) * ld] * xk;
    __syncthreads();
  }
  double s = 0.0;
  for (int i = tid; i < n; i += nt) {
    s += row[i] * row[i];
    L[n + size_t(i) * ld] = row[i];
  }
  red[tid] = s;
  __syncthreads();
  for (int o = nt / 2; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  if (tid == 0) {
    const double c = P.sf2 + P.sn2 - red[0];
    if (c > 0.0) {
      L[n + size_t(n) * ld] = sqrt(c);
      *info = 0;
    } else {
      *info = n + 1;
    }
  }
}

KParams kparams(const hmd_gp* g) {
  KParams P{};
  for (int k = 0; k < GP_MAXD; ++k) P.inv_scale[k] = k < g->d ? 1.0 / g->scale[k] : 0.0;
  P.sf2 = g->hyp.sigma_f * g->hyp.sigma_f;
  P.inv_2l2 = 1.0 / (2.0 * g->hyp.ell * g->hyp.ell);
  P.sn2 = g->sigma_n * g->sigma_n;
  P.d = g->d;
  P.kind = g->hyp.kernel;
  P.pi_over_T = g->hyp.kernel == 1 ? M_PI / g->hyp.period : 0.0;
  return P;
}

// Normalisation of Eq. d2Eq and the output scale (host, FP64).
void normalise(hmd_gp* g) {
  const int n = g->n, d = g->d;
  for (int k = 0; k < d; ++k) {
    const double fallback = 0.25 * g->hyp.range[k];
    double m = 0.0;
    if (g->hyp.scale_mode == 0 && n >= 2) {
      double s = 0.0;
      for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) s += std::fabs(g->X[size_t(i) * d + k] - g->X[size_t(j) * d + k]);
      m = s / (0.5 * double(n) * double(n - 1));
    }
    g->scale[k] = m > 0.0 ? m : fallback;
  }
  g->s_q = 1.0;
  if (g->hyp.out_scale && n > 0) {
    double s = 0.0;
    for (double v : g->y) s += v * v;
    s = std::sqrt(s / double(n));
    if (s > 0.0) g->s_q = s;
  }
  if (g->hyp.sigma_n >= 0.0) {
    g->sigma_n = g->hyp.sigma_n / g->s_q;
  } else {
    double s = 0.0;
    for (double v : g->se) s += v;
    g->sigma_n = n > 0 ? (s / double(n)) / g->s_q : 0.0;
  }
}

int reserve(hmd_gp* g, int need) {
  hmd_ctx* ctx = g->ctx;
  if (need <= g->cap) return HMD_OK;
  int cap = g->cap > 0 ? g->cap : 64;
  while (cap < need) cap *= 2;
  for (double* p : {g->dX, g->dy, g->dL, g->dLi, g->dalpha, g->dtmp, g->dnoise})
    if (p) (void)hipFree(p);
  HMD_HIP(ctx, hipMalloc(&g->dX, sizeof(double) * GP_MAXD * cap));
  HMD_HIP(ctx, hipMalloc(&g->dy, sizeof(double) * cap));
  HMD_HIP(ctx, hipMalloc(&g->dL, sizeof(double) * size_t(cap) * cap));
  HMD_HIP(ctx, hipMalloc(&g->dLi, sizeof(double) * size_t(cap) * cap));
  HMD_HIP(ctx, hipMalloc(&g->dalpha, sizeof(double) * cap));
  HMD_HIP(ctx, hipMalloc(&g->dtmp, sizeof(double) * (cap + 1)));
  HMD_HIP(ctx, hipMalloc(&g->dnoise, sizeof(double) * cap));
  g->cap = cap;
  return HMD_OK;
}

int upload_db(hmd_gp* g) {
  hmd_ctx* ctx = g->ctx;
  std::vector<double> xs(size_t(GP_MAXD) * g->n, 0.0), ys(g->n), nz(g->n);
  for (int i = 0; i < g->n; ++i) {
    for (int k = 0; k < g->d; ++k) xs[size_t(i) * GP_MAXD + k] = g->X[size_t(i) * g->d + k];
    ys[i] = g->y[i] / g->s_q;
    const double e = g->se[i] / g->s_q;
    nz[i] = e * e;
  }
  HMD_HIP(ctx, hipMemcpyAsync(g->dX, xs.data(), 8 * xs.size(), hipMemcpyHostToDevice, ctx->stream));
  HMD_HIP(ctx, hipMemcpyAsync(g->dy, ys.data(), 8 * ys.size(), hipMemcpyHostToDevice, ctx->stream));
  HMD_HIP(ctx, hipMemcpyAsync(g->dnoise, nz.data(), 8 * nz.size(), hipMemcpyHostToDevice, ctx->stream));
  // the host staging vectors end with this function
  HMD_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return HMD_OK;
}

int solve_alpha(hmd_gp* g, bool grown_by_row, bool inverse = true) {
  hmd_ctx* ctx = g->ctx;
  hipStream_t s = ctx->stream;
  HMD_HIP(ctx, hipMemcpyAsync(g->dalpha, g->dy, 8 * size_t(g->n), hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(k_gp_solve, dim3(1), dim3(1024), 0, s, g->n, g->cap, g->dL, g->dalpha, 1);
  HMD_HIP(ctx, hipGetLastError());
  if (!inverse) return HMD_OK;
  // L^-1 follows the factor: extended by its new row, or formed anew
  const size_t lds = sizeof(double) * size_t(g->n);
  if (grown_by_row)
    hipLaunchKernelGGL(k_gp_inv_append_row, dim3((g->n + 3) / 4), dim3(256), lds, s, g->n - 1, g->cap, g->dL,
                       g->dLi);
  else
    hipLaunchKernelGGL(k_gp_tri_inv, dim3(g->n), dim3(256), lds, s, g->n, g->cap, g->dL, g->dLi);
  HMD_HIP(ctx, hipGetLastError());
  return HMD_OK;
}

// Full refit: normalisation, covariance, factorisation, weights and L^-1.
// The evidence search refits at fixed data (upload false: the database and
// its scaling are already on the device) and needs no L^-1 (inverse false).
int refit(hmd_gp* g, bool upload = true, bool inverse = true) {
  hmd_ctx* ctx = g->ctx;
  normalise(g);
  if (g->n == 0) return HMD_OK;
  int rc = reserve(g, g->n);
  if (rc != HMD_OK) return rc;
  if (upload && (rc = upload_db(g)) != HMD_OK) return rc;
  hipStream_t s = ctx->stream;
  const KParams P = kparams(g);
  hipLaunchKernelGGL(k_gp_cov, dim3((g->n + 255) / 256, g->n), dim3(256), 0, s, g->n, g->cap, g->dX, P,
                     g->hyp.noise_mode == 1 ? g->dnoise : nullptr, g->dL);
  for (int k0 = 0; k0 < g->n; k0 += CB) {
    hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(256), 0, s, g->n, g->cap, g->dL, g->dinfo, k0);
    const int rest = g->n - k0 - CB;
    if (rest > 0) {
      const int nt = (rest + CB - 1) / CB;
      hipLaunchKernelGGL(k_chol_panel, dim3((rest + 255) / 256), dim3(256), 0, s, g->n, g->cap, g->dL, g->dinfo, k0);
      hipLaunchKernelGGL(k_chol_update, dim3(nt * (nt + 1) / 2), dim3(256), 0, s, g->n, g->cap, g->dL, g->dinfo,
                         k0);
    }
  }
  HMD_HIP(ctx, hipGetLastError());
  int info = 0;
  HMD_HIP(ctx, hipMemcpyAsync(&info, g->dinfo, sizeof(int), hipMemcpyDeviceToHost, s));
  HMD_HIP(ctx, hipStreamSynchronize(s));
  if (info != 0) {
    ctx->err = "gp: covariance not positive definite at pivot " + std::to_string(info - 1);
    return HMD_ENOTSPD;
  }
  return solve_alpha(g, false, inverse);
}

}  // namespace
}  // namespace hmd

using namespace hmd;

extern "C" {

void hmd_gp_hyper_default(hmd_gp_hyper* h) {
  if (!h) return;
  h->sigma_f = 1.0;
  h->ell = 1.0;
  h->sigma_n = -1.0;
  h->scale_mode = 0;
  h->range[0] = 16.0;   // channel heights 4..20
  h->range[1] = 0.049;  // body forces 0.001..0.05
  h->range[2] = 1.0;
  h->range[3] = 1.0;
  h->out_scale = 1;
  h->noise_mode = 0;
  h->kernel = 0;
  h->period = 1.0;
}

int gp_fit(hmd_ctx* ctx, const double* X, const double* y, const double* y_se, int n, int d,
           const hmd_gp_hyper* hyper, hmd_gp** out) {
  if (!ctx || !out || n < 0 || n > GP_MAXN || d < 1 || d > GP_MAXD || (n > 0 && (!X || !y))) {
    if (ctx) ctx->err = "gp_fit: bad arguments (1 <= d <= 4, 0 <= n <= 6144)";
    return HMD_EINVAL;
  }
  HMD_HIP(ctx, hipSetDevice(ctx->device));
  auto* g = new hmd_gp();
  g->ctx = ctx;
  if (hyper) g->hyp = *hyper;
  else hmd_gp_hyper_default(&g->hyp);
  if (!(g->hyp.sigma_f > 0.0) || !(g->hyp.ell > 0.0) || g->hyp.noise_mode < 0 || g->hyp.noise_mode > 1 ||
      g->hyp.kernel < 0 || g->hyp.kernel > 1 || (g->hyp.kernel == 1 && (d != 1 || !(g->hyp.period > 0.0)))) {
    delete g;
    ctx->err = "gp_fit: sigma_f, ell positive; noise_mode 0/1; kernel 0, or 1 (periodic) with d = 1 and period > 0";
    return HMD_EINVAL;
  }
  g->d = d;
  g->n = n;
  g->X.assign(X, X + size_t(n) * d);
  g->y.assign(y, y + n);
  g->se.assign(n, 0.0);
  if (y_se) g->se.assign(y_se, y_se + n);
  if (hipMalloc(&g->dinfo, sizeof(int)) != hipSuccess || hipMalloc(&g->dout, sizeof(double) * 4) != hipSuccess) {
    gp_free(g);
    ctx->err = "gp_fit: device allocation failed";
    return HMD_ENOMEM;
  }
  const int rc = refit(g);
  if (rc != HMD_OK) {
    gp_free(g);
    return rc;
  }
  HMD_HIP(ctx, hipStreamSynchronize(ctx->stream));
  *out = g;
  return HMD_OK;
}

int gp_append(hmd_gp* g, const double* x, double y, double y_se) {
  if (!g || !x) return HMD_EINVAL;
  hmd_ctx* ctx = g->ctx;
  if (g->n >= GP_MAXN) {
    ctx->err = "gp_append: the database holds at most 6144 points";
    return HMD_EINVAL;
  }
  HMD_HIP(ctx, hipSetDevice(ctx->device));
  g->X.insert(g->X.end(), x, x + g->d);
  g->y.push_back(y);
  g->se.push_back(y_se);
  g->n += 1;
  // fixed normalisation, fixed noise and no output scaling: extend L by one
  // row; otherwise the normalisation moved and the factor is rebuilt
  const bool rank1 = (g->hyp.scale_mode == 1 || g->hyp.kernel == 1) && g->hyp.out_scale == 0 &&
                     (g->hyp.sigma_n >= 0.0 || g->hyp.noise_mode == 1) && g->n >= 2 && g->n <= g->cap;
  // returns with the factor, weights and L^-1 complete, so that a following
  // prediction on any stream sees them
  auto full_refit = [&]() -> int {
    const int r = refit(g);
    if (r != HMD_OK) return r;
    HMD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return HMD_OK;
  };
  if (!rank1) return full_refit();
  normalise(g);
  int rc = upload_db(g);
  if (rc != HMD_OK) return rc;
  hipStream_t s = ctx->stream;
  KParams P1 = kparams(g);
  if (g->hyp.noise_mode == 1) {
    const double e = y_se / g->s_q;
    P1.sn2 = e * e;
  }
  hipLaunchKernelGGL(k_gp_append_row, dim3(1), dim3(1024), 0, s, g->n - 1, g->cap, g->dX, P1, g->dL, g->dtmp,
                     g->dinfo);
  int info = 0;
  HMD_HIP(ctx, hipMemcpyAsync(&info, g->dinfo, sizeof(int), hipMemcpyDeviceToHost, s));
  HMD_HIP(ctx, hipStreamSynchronize(s));
  if (info != 0) return full_refit();
  rc = solve_alpha(g, true);
  if (rc != HMD_OK) return rc;
  HMD_HIP(ctx, hipStreamSynchronize(s));
  return HMD_OK;
}

int gp_predict(hmd_gp* g, const double* Xs, int m, double* mean, double* var) {
  if (!g || m < 0 || (m > 0 && (!Xs || !mean || !var))) return HMD_EINVAL;
  hmd_ctx* ctx = g->ctx;
  if (m == 0) return HMD_OK;
  const double sf2 = g->hyp.sigma_f * g->hyp.sigma_f;
  if (g->n == 0) {  // prior: zero mean, signal variance
    for (int q = 0; q < m; ++q) {
      mean[q] = 0.0;
      var[q] = sf2 * g->s_q * g->s_q;
    }
    return HMD_OK;
  }
  HMD_HIP(ctx, hipSetDevice(ctx->device));
  const size_t need_q = size_t(GP_MAXD) * m;
  if (need_q + 2 * size_t(m) > g->q_cap) {
    if (g->dq) (void)hipFree(g->dq);
    g->q_cap = 2 * (need_q + 2 * size_t(m));
    HMD_HIP(ctx, hipMalloc(&g->dq, sizeof(double) * g->q_cap));
  }
  double* dXq = g->dq;
  double* dres = g->dq + need_q;
  std::vector<double> xs(need_q, 0.0), res(2 * size_t(m));
  for (int q = 0; q < m; ++q)
    for (int k = 0; k < g->d; ++k) xs[size_t(q) * GP_MAXD + k] = Xs[size_t(q) * g->d + k];
  hipStream_t s = ctx->stream;
  HMD_HIP(ctx, hipMemcpyAsync(dXq, xs.data(), 8 * xs.size(), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_gp_predict, dim3(m), dim3(256), sizeof(double) * size_t(g->n), s, g->n, g->cap, g->dX, dXq,
                     g->dLi, g->dalpha, kparams(g), dres);
  HMD_HIP(ctx, hipGetLastError());
  HMD_HIP(ctx, hipMemcpyAsync(res.data(), dres, 8 * res.size(), hipMemcpyDeviceToHost, s));
  HMD_HIP(ctx, hipStreamSynchronize(s));
  for (int q = 0; q < m; ++q) {
    mean[q] = res[2 * q] * g->s_q;
    var[q] = res[2 * q + 1] * g->s_q * g->s_q;
  }
  return HMD_OK;
}

int gp_predict_dev(hmd_gp* g, const double* dXs, int m, double* dmean, double* dvar, void* stream) {
  if (!g || m < 0 || (m > 0 && (!dXs || !dmean || !dvar))) return HMD_EINVAL;
  hmd_ctx* ctx = g->ctx;
  if (m == 0) return HMD_OK;
  HMD_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : ctx->stream;
  const double sf2 = g->hyp.sigma_f * g->hyp.sigma_f;
  const size_t need_q = size_t(GP_MAXD) * m;
  if (need_q + 2 * size_t(m) > g->q_cap) {
    HMD_HIP(ctx, hipStreamSynchronize(s));  // the old scratch may still be read
    if (g->dq) (void)hipFree(g->dq);
    g->q_cap = 2 * (need_q + 2 * size_t(m));
    HMD_HIP(ctx, hipMalloc(&g->dq, sizeof(double) * g->q_cap));
  }
  double* dXq = g->dq;
  double* dres = g->dq + need_q;
  hipLaunchKernelGGL(k_gp_pack, dim3((m + 255) / 256), dim3(256), 0, s, m, g->d, dXs, dXq);
  HMD_HIP(ctx, hipGetLastError());
  if (g->n > 0) {
    hipLaunchKernelGGL(k_gp_predict, dim3(m), dim3(256), sizeof(double) * size_t(g->n), s, g->n, g->cap, g->dX,
                       dXq, g->dLi, g->dalpha, kparams(g), dres);
    HMD_HIP(ctx, hipGetLastError());
  }
  hipLaunchKernelGGL(k_gp_unpack, dim3((m + 255) / 256), dim3(256), 0, s, m, g->n > 0 ? 1 : 0, dres, g->s_q, sf2,
                     dmean, dvar);
  HMD_HIP(ctx, hipGetLastError());
  return HMD_OK;
}

int gp_log_marginal(hmd_gp* g, double* lml) {
  if (!g || !lml) return HMD_EINVAL;
  hmd_ctx* ctx = g->ctx;
  if (g->n == 0) {
    *lml = 0.0;
    return HMD_OK;
  }
  HMD_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  hipLaunchKernelGGL(k_gp_lml, dim3(1), dim3(256), 0, s, g->n, g->cap, g->dL, g->dy, g->dalpha, g->dout);
  double h[2];
  HMD_HIP(ctx, hipMemcpyAsync(h, g->dout, sizeof(h), hipMemcpyDeviceToHost, s));
  HMD_HIP(ctx, hipStreamSynchronize(s));
  *lml = -0.5 * h[0] - h[1] - 0.5 * double(g->n) * std::log(2.0 * M_PI);
  return HMD_OK;
}

// Hyperparameters that maximise Eq. evidenceEq (Sec. 2.3; App. B).  The
// evidence can have several local maxima (the periodic kernel's has in ell),
// so the search first evaluates it on a grid of 17 points per chosen
// parameter, a quarter decade apart over two decades either side of the
// start, then refines from the best grid point by cyclic golden-section
// searches over the logarithm of each chosen parameter, bracketed by a factor
// 10 around the current value, each refit on the device, until a cycle gains
// less than 1e-12 relative (at most 30 cycles).
int gp_optimize(hmd_gp* g, int mask, double* lml) {
  if (!g || mask <= 0 || mask > 7) return HMD_EINVAL;
  hmd_ctx* ctx = g->ctx;
  if (g->n < 1 || ((mask & 4) && g->hyp.noise_mode == 1)) {
    ctx->err = "gp_optimize: needs data, and sigma_n only with uniform noise";
    return HMD_EINVAL;
  }
  if (mask & 4) g->hyp.sigma_n = g->sigma_n * g->s_q;  // held explicitly from here on
  // the database and its scaling stay on the device through the search
  // (they do not depend on sigma_f, ell or sigma_n); L^-1 is formed once
  // at the end
  HMD_TRY(reserve(g, g->n));
  normalise(g);
  HMD_TRY(upload_db(g));
  auto get = [&](int k) {
    return k == 0 ? g->hyp.sigma_f : (k == 1 ? g->hyp.ell : g->hyp.sigma_n / g->s_q);
  };
  auto set = [&](int k, double v) {
    if (k == 0) g->hyp.sigma_f = v;
    else if (k == 1) g->hyp.ell = v;
    else g->hyp.sigma_n = v * g->s_q;
  };
  auto eval = [&](int k, double logv, double* out) -> int {
    set(k, std::exp(logv));
    const int rc = refit(g, false, false);
    if (rc == HMD_ENOTSPD) {
      *out = -INFINITY;
      return HMD_OK;
    }
    if (rc != HMD_OK) return rc;
    return gp_log_marginal(g, out);
  };
  int idx[3], m = 0, total = 1;
  double c0[3], cbest[3];
  for (int k = 0; k < 3; ++k)
    if (mask & (1 << k)) {
      idx[m] = k;
      c0[m] = cbest[m] = std::log(get(k));
      ++m;
      total *= 17;
    }
  double gbest = -INFINITY;
  for (int p = 0; p < total; ++p) {
    int r = p;
    for (int j = 0; j < m; ++j, r /= 17) set(idx[j], std::exp(c0[j] + std::log(10.0) * (-2.0 + 0.25 * (r % 17))));
    const int rc = refit(g, false, false);
    if (rc == HMD_ENOTSPD) continue;
    if (rc != HMD_OK) return rc;
    double f;
    HMD_TRY(gp_log_marginal(g, &f));
    if (f > gbest) {
      gbest = f;
      for (int j = 0; j < m; ++j) cbest[j] = std::log(get(idx[j]));
    }
  }
  for (int j = 0; j < m; ++j) set(idx[j], std::exp(cbest[j]));
  const double gr = 0.5 * (std::sqrt(5.0) - 1.0);
  double best = -INFINITY;
  HMD_TRY(eval(0, std::log(get(0)), &best));
  for (int cycle = 0; cycle < 30; ++cycle) {
    const double start = best;
    for (int k = 0; k < 3; ++k) {
      if (!(mask & (1 << k))) continue;
      const double c0 = std::log(get(k));
      double a = c0 - std::log(10.0), b = c0 + std::log(10.0);
      double x1 = b - gr * (b - a), x2 = a + gr * (b - a), f1, f2;
      HMD_TRY(eval(k, x1, &f1));
      HMD_TRY(eval(k, x2, &f2));
      for (int it = 0; it < 60; ++it) {
        if (f1 >= f2) {
          b = x2; x2 = x1; f2 = f1; x1 = b - gr * (b - a);
          HMD_TRY(eval(k, x1, &f1));
        } else {
          a = x1; x1 = x2; f1 = f2; x2 = a + gr * (b - a);
          HMD_TRY(eval(k, x2, &f2));
        }
      }
      double fc;
      const double xc = 0.5 * (a + b);
      HMD_TRY(eval(k, xc, &fc));
      double fold;
      HMD_TRY(eval(k, c0, &fold));
      if (fc >= fold) {
        HMD_TRY(eval(k, xc, &best));
      } else {
        best = fold;  // the search did not beat the start: keep it (already refit)
      }
    }
    if (std::fabs(best - start) <= 1e-12 * std::fabs(best)) break;
  }
  HMD_TRY(refit(g, false, true));  // at the kept values, with L^-1 for predictions
  if (lml) *lml = best;
  HMD_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return HMD_OK;
}

int gp_hyper_get(const hmd_gp* g, hmd_gp_hyper* hyper) {
  if (!g || !hyper) return HMD_EINVAL;
  *hyper = g->hyp;
  return HMD_OK;
}

int gp_size(const hmd_gp* g) { return g ? g->n : 0; }

int gp_inputs(const hmd_gp* g, double* X, int* n, int* d) {
  if (!g) return HMD_EINVAL;
  if (n) *n = g->n;
  if (d) *d = g->d;
  if (X) std::copy(g->X.begin(), g->X.begin() + size_t(g->n) * g->d, X);
  return HMD_OK;
}

int gp_outputs(const hmd_gp* g, double* y, double* y_se) {
  if (!g) return HMD_EINVAL;
  if (y) std::copy(g->y.begin(), g->y.begin() + g->n, y);
  if (y_se) std::copy(g->se.begin(), g->se.begin() + g->n, y_se);
  return HMD_OK;
}

int gp_scales(const hmd_gp* g, double* scale, double* s_q, double* sigma_n) {
  if (!g) return HMD_EINVAL;
  if (scale)
    for (int k = 0; k < g->d; ++k) scale[k] = g->scale[k];
  if (s_q) *s_q = g->s_q;
  if (sigma_n) *sigma_n = g->sigma_n;
  return HMD_OK;
}

void gp_free(hmd_gp* g) {
  if (!g) return;
  for (void* p : {(void*)g->dX, (void*)g->dy, (void*)g->dL, (void*)g->dLi, (void*)g->dalpha, (void*)g->dtmp,
                  (void*)g->dnoise, (void*)g->dq,
                  (void*)g->dout, (void*)g->dinfo})
    if (p) (void)hipFree(p);
  delete g;
}

}  // extern "C"
