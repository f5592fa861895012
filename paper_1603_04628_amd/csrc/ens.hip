// ens.hip -- MLP deep ensemble on the device (a learned surrogate beside the
// paper's GP): members of 2 -> H -> H -> 1 tanh networks, FP32 weights and
// accumulation, trained full-batch on the mean squared error with Adam.
//
// Training runs every iteration of every member in one launch: one workgroup
// per member keeps its parameters in LDS, each thread owns a fixed slice of
// the parameters (their gradient sums and Adam moments stay in registers),
// and the batch streams through LDS in chunks of CHUNK samples (forward,
// back-propagation, per-parameter gradient sums).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "engine.h"

struct hmd_ens {
  hmd_ctx* ctx = nullptr;
  hmd_ens_cfg cfg{};
  int P = 0;                 // parameters per member
  double mu[2] = {0, 0}, sd[2] = {1, 1}, s_q = 1.0;
  float* dparams = nullptr;  // members x P
  std::vector<double> loss;  // final training loss per member
  std::vector<double> X, y;  // training set (host copy, for refits)
  // prediction buffers, grown on demand and kept for later calls
  double* dq = nullptr;      // queries, 2 per row
  float* dy = nullptr;       // members x queries outputs
  double* dout = nullptr;    // mean, std per query
  int qcap = 0;
};

namespace hmd {
namespace {

constexpr int ENS_TPB = 256;
constexpr int CHUNK = 32;
constexpr int MAXH = 64;

__host__ __device__ inline int nparams(int H) { return H * H + 5 * H + 1; }

// Which tensor a flat parameter index belongs to, and its (row, col).
struct Slot {
  int kind, o, i;  // kind: 0 W1, 1 b1, 2 W2, 3 b2, 4 W3, 5 b3, -1 none
};

__device__ __forceinline__ Slot decode(int p, int H) {
  Slot s{-1, 0, 0};
  if (p < 2 * H) s = Slot{0, p / 2, p % 2};
  else if (p < 3 * H) s = Slot{1, p - 2 * H, 0};
  else if (p < 3 * H + H * H) s = Slot{2, (p - 3 * H) / H, (p - 3 * H) % H};
  else if (p < 4 * H + H * H) s = Slot{3, p - 3 * H - H * H, 0};
  else if (p < 5 * H + H * H) s = Slot{4, p - 4 * H - H * H, 0};
  else if (p == 5 * H + H * H) s = Slot{5, 0, 0};
  return s;
}

// Training is split over (chunk of CHUNK points, member) workgroups so that
// every iteration runs on many CUs: k_ens_chunk computes one chunk's forward
// and backward pass and its share of the gradient and loss (MSE over all N
// points: the 2/N and 1/N factors are applied here; wts, when given, holds
// each member's bootstrap count per point); k_ens_adam sums the shares of
// each member and takes one Adam step.
__global__ __launch_bounds__(ENS_TPB) void k_ens_chunk(int N, int H, const float* __restrict__ Xs,
                                                       const float* __restrict__ ys,
                                                       const float* __restrict__ wts,
                                                       const float* __restrict__ params, float* __restrict__ gpart,
                                                       float* __restrict__ lpart) {
  extern __shared__ float lds[];
  const int P = H * H + 5 * H + 1;
  // activation rows are padded to H + 1 floats so that lanes walking
  // different rows at the same column hit different LDS banks
  const int HP = H + 1;
  float* th = lds;                   // P
  float* x = th + P;                 // CHUNK x 2
  float* h1 = x + 2 * CHUNK;         // CHUNK x HP
  float* h2 = h1 + CHUNK * HP;       // CHUNK x HP
  float* dz2 = h2 + CHUNK * HP;      // CHUNK x HP
  float* dz1 = dz2 + CHUNK * HP;     // CHUNK x HP
  float* dout = dz1 + CHUNK * HP;    // CHUNK
  float* red = dout + CHUNK;         // ENS_TPB
  float* W1 = th;
  float* b1 = W1 + 2 * H;
  float* W2 = b1 + H;
  float* b2 = W2 + H * H;
  float* W3 = b2 + H;
  float* b3 = W3 + H;

  const int tid = threadIdx.x, member = blockIdx.y, chunk = blockIdx.x, nchunk = gridDim.x;
  const float* my = params + size_t(member) * P;
  for (int p = tid; p < P; p += ENS_TPB) th[p] = my[p];
  const int c0 = chunk * CHUNK, nc = min(CHUNK, N - c0);
  for (int e = tid; e < 2 * nc; e += ENS_TPB) x[e] = Xs[2 * c0 + e];
  __syncthreads();
  const float invN = 1.0f / float(N);
  for (int e = tid; e < nc * H; e += ENS_TPB) {
    const int s = e / H, o = e % H;
    h1[s * HP + o] = tanhf(W1[2 * o] * x[2 * s] + W1[2 * o + 1] * x[2 * s + 1] + b1[o]);
  }
  __syncthreads();
  // lanes run over points (same output unit): the W2 row is a broadcast and
  // the padded activation rows spread over the banks
  for (int e = tid; e < nc * H; e += ENS_TPB) {
    const int s = e % nc, o = e / nc;
    float a = b2[o];
    const float* w = W2 + o * H;
    const float* hh = h1 + s * HP;
    for (int i = 0; i < H; ++i) a += w[i] * hh[i];
    h2[s * HP + o] = tanhf(a);
  }
  __syncthreads();
  float lsum = 0.f;
  if (tid < nc) {
    float a = b3[0];
    const float* hh = h2 + tid * HP;
    for (int o = 0; o < H; ++o) a += W3[o] * hh[o];
    // bootstrap: the point's count in this member's resample weights its
    // squared residual (the mean still over N)
    const float w = wts ? wts[size_t(member) * N + c0 + tid] : 1.0f;
    const float r = a - ys[c0 + tid];
    lsum = w * r * r;
    dout[tid] = 2.0f * w * r * invN;
  }
  __syncthreads();
  for (int e = tid; e < nc * H; e += ENS_TPB) {
    const int s = e / H, o = e % H;
    const float t = h2[s * HP + o];
    dz2[s * HP + o] = dout[s] * W3[o] * (1.0f - t * t);
  }
  __syncthreads();
  for (int e = tid; e < nc * H; e += ENS_TPB) {
    const int s = e / H, i = e % H;
    float a = 0.f;
    const float* dz = dz2 + s * HP;
    for (int o = 0; o < H; ++o) a += dz[o] * W2[o * H + i];
    const float t = h1[s * HP + i];
    dz1[s * HP + i] = a * (1.0f - t * t);
  }
  __syncthreads();
  float* gout = gpart + (size_t(member) * nchunk + chunk) * P;
  for (int p = tid; p < P; p += ENS_TPB) {
    const Slot q = decode(p, H);
    float a = 0.f;
    switch (q.kind) {
      case 0: for (int s = 0; s < nc; ++s) a += dz1[s * HP + q.o] * x[2 * s + q.i]; break;
      case 1: for (int s = 0; s < nc; ++s) a += dz1[s * HP + q.o]; break;
      case 2: for (int s = 0; s < nc; ++s) a += dz2[s * HP + q.o] * h1[s * HP + q.i]; break;
      case 3: for (int s = 0; s < nc; ++s) a += dz2[s * HP + q.o]; break;
      case 4: for (int s = 0; s < nc; ++s) a += dout[s] * h2[s * HP + q.o]; break;
      case 5: for (int s = 0; s < nc; ++s) a += dout[s]; break;
      default: break;
    }
    gout[p] = a;
  }
  red[tid] = lsum;
  __syncthreads();
  for (int o = ENS_TPB / 2; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  if (tid == 0) lpart[size_t(member) * nchunk + chunk] = red[0] * invN;
}

// Per member: the gradient summed over chunks, then (unless grad_out is set,
// which receives the gradient instead) one Adam step (Kingma & Ba 2015,
// beta = (0.9, 0.999), eps = 1e-8).  Grid: (parameter blocks, members); the
// step number is *tbase + k + 1.  loss_out receives the loss at the
// parameters before the step.
__global__ __launch_bounds__(ENS_TPB) void k_ens_adam(int P, int nchunk, const float* __restrict__ gpart,
                                                      const float* __restrict__ lpart, float* __restrict__ params,
                                                      float* __restrict__ mom, float* __restrict__ vel,
                                                      const int* __restrict__ tbase, int k, float lr,
                                                      float* __restrict__ loss_out, float* __restrict__ grad_out) {
  const int member = blockIdx.y, p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < P) {
    const float* gm = gpart + size_t(member) * nchunk * P;
    float g = 0.f;
    for (int c = 0; c < nchunk; ++c) g += gm[size_t(c) * P + p];
    if (grad_out) {
      grad_out[size_t(member) * P + p] = g;
    } else {
      const int t = *tbase + k + 1;
      const float c1 = float(1.0 / (1.0 - pow(0.9, double(t)))), c2 = float(1.0 / (1.0 - pow(0.999, double(t))));
      float* m = mom + size_t(member) * P;
      float* v = vel + size_t(member) * P;
      const float mk = 0.9f * m[p] + 0.1f * g, vk = 0.999f * v[p] + 0.001f * g * g;
      m[p] = mk;
      v[p] = vk;
      params[size_t(member) * P + p] -= lr * (mk * c1) / (sqrtf(vk * c2) + 1e-8f);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    float l = 0.f;
    for (int c = 0; c < nchunk; ++c) l += lpart[size_t(member) * nchunk + c];
    loss_out[member] = l;
  }
}

__global__ void k_ens_tick(int* tbase, int k) { *tbase += k; }

// Prediction, member by member: one wavefront per (block of PQB queries,
// member), lane o holding hidden unit o.  The member's W2 sits transposed in
// LDS so lane o reads its column with consecutive addresses; the layer-1
// activations of the PQB queries are shared through LDS; the output layer is
// a wavefront sum.
constexpr int PQB = 8;

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__global__ __launch_bounds__(64) void k_ens_member_out(int m, int H, const float* __restrict__ params,
                                                       const double* __restrict__ Xq, double mu0, double mu1,
                                                       double sd0, double sd1, float* __restrict__ yout) {
  __shared__ float w2t[MAXH * MAXH];
  __shared__ float h1[PQB][MAXH];
  const int k = blockIdx.y, o = threadIdx.x, q0 = blockIdx.x * PQB;
  const int P = nparams(H);
  const float* W1 = params + size_t(k) * P;
  const float* b1 = W1 + 2 * H;
  const float* W2 = b1 + H;
  const float* b2 = W2 + H * H;
  const float* W3 = b2 + H;
  const float b3 = W3[H];
  for (int t = o; t < H * H; t += 64) w2t[(t % H) * H + t / H] = W2[t];  // W2 row o' = output unit o'
  const bool unit = o < H;
  if (unit) {
    const float w10 = W1[2 * o], w11 = W1[2 * o + 1], c1 = b1[o];
#pragma unroll
    for (int q = 0; q < PQB; ++q) {
      const int qq = q0 + q < m ? q0 + q : m - 1;
      const float x0 = float((Xq[2 * qq] - mu0) / sd0), x1 = float((Xq[2 * qq + 1] - mu1) / sd1);
      h1[q][o] = tanhf(w10 * x0 + w11 * x1 + c1);
    }
  }
  __syncthreads();
  float a[PQB];
  const float c2 = unit ? b2[o] : 0.0f;
#pragma unroll
  for (int q = 0; q < PQB; ++q) a[q] = c2;
  if (unit)
    for (int i = 0; i < H; ++i) {
      const float w = w2t[i * H + o];
#pragma unroll
      for (int q = 0; q < PQB; ++q) a[q] += w * h1[q][i];
    }
  const float w3 = unit ? W3[o] : 0.0f;
#pragma unroll
  for (int q = 0; q < PQB; ++q) {
    const float v = wave_sum_f(unit ? w3 * tanhf(a[q]) : 0.0f);
    if (o == 0 && q0 + q < m) yout[size_t(k) * m + q0 + q] = b3 + v;
  }
}

// Ensemble mean and sample standard deviation (M - 1) per query, FP64.
__global__ __launch_bounds__(128) void k_ens_reduce(int m, int members, const float* __restrict__ yout,
                                                    double s_q, double* __restrict__ mean_out,
                                                    double* __restrict__ std_out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  double sum = 0.0, sum2 = 0.0;
  for (int k = 0; k < members; ++k) {
    const double yo = double(yout[size_t(k) * m + q]) * s_q;
    sum += yo;
    sum2 += yo * yo;
  }
  const double mean = sum / members;
  const double var = members > 1 ? (sum2 - members * mean * mean) / (members - 1) : 0.0;
  mean_out[q] = mean;
  std_out[q] = sqrt(var > 0.0 ? var : 0.0);
}

size_t train_lds_bytes(int H) {
  return sizeof(float) * (size_t(nparams(H)) + 2 * CHUNK + 4 * size_t(CHUNK) * (H + 1) + CHUNK + ENS_TPB);
}

// Glorot-uniform start of one member: Philox4x32-10 keyed by the seed, word
// p mod 4 of counter (p div 4, member, 2, 0); biases zero.
void glorot(int H, int member, uint64_t seed, float* out) {
  const int P = nparams(H);
  const uint32_t key[2] = {uint32_t(seed & 0xffffffffu), uint32_t(seed >> 32)};
  std::vector<double> u(P);
  for (int j = 0; 4 * j < P; ++j) {
    const uint32_t ctr[4] = {uint32_t(j), uint32_t(member), 2u, 0u};
    uint32_t r[4];
    philox4x32_10(ctr, key, r);
    for (int w = 0; w < 4 && 4 * j + w < P; ++w) u[4 * j + w] = (double(r[w]) + 0.5) / 4294967296.0;
  }
  for (int p = 0; p < P; ++p) out[p] = 0.f;
  const double l1 = std::sqrt(6.0 / (2.0 + H)), l2 = std::sqrt(6.0 / (2.0 * H)), l3 = std::sqrt(6.0 / (H + 1.0));
  for (int p = 0; p < 2 * H; ++p) out[p] = float(l1 * (2.0 * u[p] - 1.0));
  for (int p = 3 * H; p < 3 * H + H * H; ++p) out[p] = float(l2 * (2.0 * u[p] - 1.0));
  for (int p = 4 * H + H * H; p < 5 * H + H * H; ++p) out[p] = float(l3 * (2.0 * u[p] - 1.0));
}

// Bootstrap resample of member `member` (counts per point): draw j takes
// point (r n) >> 32 for the Philox word r of counter (j div 4, member, 3, 0),
// word j mod 4, keyed by the seed.
void bootstrap_counts(int n, int member, uint64_t seed, float* out) {
  const uint32_t key[2] = {uint32_t(seed & 0xffffffffu), uint32_t(seed >> 32)};
  for (int i = 0; i < n; ++i) out[i] = 0.f;
  for (int j = 0; 4 * j < n; ++j) {
    const uint32_t ctr[4] = {uint32_t(j), uint32_t(member), 3u, 0u};
    uint32_t r[4];
    philox4x32_10(ctr, key, r);
    for (int w = 0; w < 4 && 4 * j + w < n; ++w) out[(uint64_t(r[w]) * uint64_t(n)) >> 32] += 1.f;
  }
}

int check_cfg(hmd_ctx* ctx, const hmd_ens_cfg& c, int n) {
  if (c.members < 1 || c.members > 64 || c.hidden < 1 || c.hidden > MAXH || c.iters < 0 || !(c.lr > 0.0) || n < 1 ||
      c.bootstrap < 0 || c.bootstrap > 1) {
    ctx->err = "ens: 1..64 members, 1..64 hidden units, iters >= 0, lr > 0, n >= 1, bootstrap 0 or 1";
    return HMD_EINVAL;
  }
  return HMD_OK;
}

// Standardise inputs and scale outputs (host, FP64), upload as FP32; with
// the bootstrap option also each member's counts (*dw, members x n).
int stage_data(hmd_ens* e, const double* X, const double* y, int n, float** dX, float** dy, float** dw) {
  hmd_ctx* ctx = e->ctx;
  for (int k = 0; k < 2; ++k) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += X[2 * i + k];
    e->mu[k] = s / n;
    double v = 0.0;
    for (int i = 0; i < n; ++i) v += (X[2 * i + k] - e->mu[k]) * (X[2 * i + k] - e->mu[k]);
    e->sd[k] = std::sqrt(v / n);
    if (!(e->sd[k] > 0.0)) e->sd[k] = 1.0;
  }
  double s2 = 0.0;
  for (int i = 0; i < n; ++i) s2 += y[i] * y[i];
  e->s_q = std::sqrt(s2 / n);
  if (!(e->s_q > 0.0)) e->s_q = 1.0;
  std::vector<float> xs(2 * size_t(n)), ys(n);
  for (int i = 0; i < n; ++i) {
    for (int k = 0; k < 2; ++k) xs[2 * i + k] = float((X[2 * i + k] - e->mu[k]) / e->sd[k]);
    ys[i] = float(y[i] / e->s_q);
  }
  HMD_HIP(ctx, hipMalloc(dX, sizeof(float) * xs.size()));
  HMD_HIP(ctx, hipMalloc(dy, sizeof(float) * ys.size()));
  HMD_HIP(ctx, hipMemcpyAsync(*dX, xs.data(), sizeof(float) * xs.size(), hipMemcpyHostToDevice, ctx->stream));
  HMD_HIP(ctx, hipMemcpyAsync(*dy, ys.data(), sizeof(float) * ys.size(), hipMemcpyHostToDevice, ctx->stream));
  *dw = nullptr;
  if (e->cfg.bootstrap) {
    const int M = e->cfg.members;
    std::vector<float> w(size_t(M) * n);
    for (int k = 0; k < M; ++k) bootstrap_counts(n, k, e->cfg.seed, w.data() + size_t(k) * n);
    HMD_HIP(ctx, hipMalloc(dw, sizeof(float) * w.size()));
    HMD_HIP(ctx, hipMemcpy(*dw, w.data(), sizeof(float) * w.size(), hipMemcpyHostToDevice));
  }
  return HMD_OK;
}

int run_train(hmd_ens* e, int n, const float* dX, const float* dy, const float* dw, int mode, float* dgrad) {
  hmd_ctx* ctx = e->ctx;
  const hmd_ens_cfg& c = e->cfg;
  const size_t lds = train_lds_bytes(c.hidden);
  const int nchunk = (n + CHUNK - 1) / CHUNK, P = e->P, M = c.members;
  float *gpart = nullptr, *lpart = nullptr, *mom = nullptr, *vel = nullptr, *dloss = nullptr;
  int* tstep = nullptr;
  hipError_t err = hipMalloc(&gpart, sizeof(float) * size_t(M) * nchunk * P);
  if (err == hipSuccess) err = hipMalloc(&lpart, sizeof(float) * size_t(M) * nchunk);
  if (err == hipSuccess) err = hipMalloc(&mom, sizeof(float) * size_t(M) * P);
  if (err == hipSuccess) err = hipMalloc(&vel, sizeof(float) * size_t(M) * P);
  if (err == hipSuccess) err = hipMalloc(&dloss, sizeof(float) * M);
  if (err == hipSuccess) err = hipMalloc(&tstep, sizeof(int) * M);
  hipStream_t s = ctx->stream;
  if (err == hipSuccess) err = hipMemsetAsync(mom, 0, sizeof(float) * size_t(M) * P, s);
  if (err == hipSuccess) err = hipMemsetAsync(vel, 0, sizeof(float) * size_t(M) * P, s);
  if (err == hipSuccess) err = hipMemsetAsync(tstep, 0, sizeof(int) * M, s);
  const int iters = mode == 1 ? 1 : c.iters;
  const dim3 agrid((P + ENS_TPB - 1) / ENS_TPB, M);
  auto iteration = [&](int k) {
    hipLaunchKernelGGL(k_ens_chunk, dim3(nchunk, M), dim3(ENS_TPB), lds, s, n, c.hidden, dX, dy, dw, e->dparams,
                       gpart, lpart);
    hipLaunchKernelGGL(k_ens_adam, agrid, dim3(ENS_TPB), 0, s, P, nchunk, gpart, lpart, e->dparams, mom, vel,
                       tstep, k, float(c.lr), dloss, mode == 1 ? dgrad : nullptr);
  };
  // iterations in captured blocks of kBlock (a graph replay per block), the
  // remainder as direct launches; the step counter advances once per block
  constexpr int kBlock = 100;
  const int nblock = iters / kBlock;
  if (err == hipSuccess && nblock > 0) {
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    err = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (err == hipSuccess) {
      for (int k = 0; k < kBlock; ++k) iteration(k);
      hipLaunchKernelGGL(k_ens_tick, dim3(1), dim3(1), 0, s, tstep, kBlock);
      err = hipStreamEndCapture(s, &g);
    }
    if (err == hipSuccess) err = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    for (int r = 0; r < nblock && err == hipSuccess; ++r) err = hipGraphLaunch(ge, s);
    if (ge) (void)hipGraphExecDestroy(ge);
    if (g) (void)hipGraphDestroy(g);
  }
  for (int k = 0; k < iters - nblock * kBlock && err == hipSuccess; ++k) {
    iteration(k);
    err = hipGetLastError();
  }
  std::vector<float> loss(M, 0.f);
  if (err == hipSuccess && iters > 0)
    err = hipMemcpyAsync(loss.data(), dloss, sizeof(float) * M, hipMemcpyDeviceToHost, s);
  if (err == hipSuccess) err = hipStreamSynchronize(s);
  for (void* p : {(void*)gpart, (void*)lpart, (void*)mom, (void*)vel, (void*)dloss, (void*)tstep})
    if (p) (void)hipFree(p);
  if (err != hipSuccess) {
    ctx->err = std::string("ens training: ") + hipGetErrorString(err);
    return HMD_EDEVICE;
  }
  e->loss.assign(loss.begin(), loss.end());
  return HMD_OK;
}

int init_params(hmd_ens* e) {
  hmd_ctx* ctx = e->ctx;
  const hmd_ens_cfg& c = e->cfg;
  e->P = nparams(c.hidden);
  std::vector<float> h(size_t(c.members) * e->P);
  for (int k = 0; k < c.members; ++k) glorot(c.hidden, k, c.seed, h.data() + size_t(k) * e->P);
  HMD_HIP(ctx, hipMalloc(&e->dparams, sizeof(float) * h.size()));
  HMD_HIP(ctx, hipMemcpyAsync(e->dparams, h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice, ctx->stream));
  return HMD_OK;
}

}  // namespace
}  // namespace hmd

using namespace hmd;

extern "C" {

void hmd_ens_cfg_default(hmd_ens_cfg* c) {
  if (!c) return;
  c->members = 5;
  c->hidden = 64;
  c->iters = 5000;
  c->lr = 1e-3;
  c->seed = 0;
  c->bootstrap = 0;
}

int ens_fit(hmd_ctx* ctx, const double* X, const double* y, int n, const hmd_ens_cfg* cfg, hmd_ens** out) {
  if (!ctx || !X || !y || !out) return HMD_EINVAL;
  hmd_ens_cfg c;
  if (cfg) c = *cfg;
  else hmd_ens_cfg_default(&c);
  int rc = check_cfg(ctx, c, n);
  if (rc != HMD_OK) return rc;
  HMD_HIP(ctx, hipSetDevice(ctx->device));
  auto* e = new hmd_ens();
  e->ctx = ctx;
  e->cfg = c;
  e->X.assign(X, X + 2 * size_t(n));
  e->y.assign(y, y + n);
  rc = ens_refit(e);
  if (rc != HMD_OK) {
    ens_free(e);
    return rc;
  }
  *out = e;
  return HMD_OK;
}

int ens_append(hmd_ens* e, const double* x, double y) {
  if (!e || !x) return HMD_EINVAL;
  e->X.push_back(x[0]);
  e->X.push_back(x[1]);
  e->y.push_back(y);
  return HMD_OK;
}

int ens_refit(hmd_ens* e) {
  if (!e) return HMD_EINVAL;
  hmd_ctx* ctx = e->ctx;
  const int n = int(e->y.size());
  int rc = check_cfg(ctx, e->cfg, n);
  if (rc != HMD_OK) return rc;
  HMD_HIP(ctx, hipSetDevice(ctx->device));
  if (e->dparams) {
    (void)hipFree(e->dparams);
    e->dparams = nullptr;
  }
  float *dX = nullptr, *dy = nullptr, *dw = nullptr;
  if ((rc = init_params(e)) == HMD_OK && (rc = stage_data(e, e->X.data(), e->y.data(), n, &dX, &dy, &dw)) == HMD_OK)
    rc = run_train(e, n, dX, dy, dw, 0, nullptr);
  for (void* p : {(void*)dX, (void*)dy, (void*)dw})
    if (p) (void)hipFree(p);
  return rc;
}

int ens_size(const hmd_ens* e) { return e ? int(e->y.size()) : 0; }

int ens_predict(hmd_ens* e, const double* Xs, int m, double* mean, double* std) {
  if (!e || m < 0 || (m > 0 && (!Xs || !mean || !std))) return HMD_EINVAL;
  if (m == 0) return HMD_OK;
  hmd_ctx* ctx = e->ctx;
  HMD_HIP(ctx, hipSetDevice(ctx->device));
  if (m > e->qcap) {
    if (e->dq) (void)hipFree(e->dq);
    if (e->dy) (void)hipFree(e->dy);
    if (e->dout) (void)hipFree(e->dout);
    e->dq = nullptr; e->dy = nullptr; e->dout = nullptr; e->qcap = 0;
    const int cap = std::max(m, 256);
    HMD_HIP(ctx, hipMalloc(&e->dq, sizeof(double) * 2 * cap));
    HMD_HIP(ctx, hipMalloc(&e->dy, sizeof(float) * size_t(e->cfg.members) * cap));
    HMD_HIP(ctx, hipMalloc(&e->dout, sizeof(double) * 2 * cap));
    e->qcap = cap;
  }
  std::vector<double> res(2 * size_t(m));  // means, then standard deviations
  HMD_HIP(ctx, hipMemcpyAsync(e->dq, Xs, sizeof(double) * 2 * m, hipMemcpyHostToDevice, ctx->stream));
  hipLaunchKernelGGL(k_ens_member_out, dim3((m + PQB - 1) / PQB, e->cfg.members), dim3(64), 0, ctx->stream, m,
                     e->cfg.hidden, e->dparams, e->dq, e->mu[0], e->mu[1], e->sd[0], e->sd[1], e->dy);
  HMD_HIP(ctx, hipGetLastError());
  hipLaunchKernelGGL(k_ens_reduce, dim3((m + 127) / 128), dim3(128), 0, ctx->stream, m, e->cfg.members, e->dy,
                     e->s_q, e->dout, e->dout + m);
  HMD_HIP(ctx, hipGetLastError());
  HMD_HIP(ctx, hipMemcpyAsync(res.data(), e->dout, sizeof(double) * res.size(), hipMemcpyDeviceToHost,
                              ctx->stream));
  HMD_HIP(ctx, hipStreamSynchronize(ctx->stream));
  for (int q = 0; q < m; ++q) {
    mean[q] = res[q];
    std[q] = res[size_t(m) + q];
  }
  return HMD_OK;
}

int ens_predict_dev(hmd_ens* e, const double* dXs, int m, double* dmean, double* dstd, void* stream) {
  if (!e || m < 0 || (m > 0 && (!dXs || !dmean || !dstd))) return HMD_EINVAL;
  if (m == 0) return HMD_OK;
  hmd_ctx* ctx = e->ctx;
  HMD_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : ctx->stream;
  if (m > e->qcap) {
    HMD_HIP(ctx, hipStreamSynchronize(s));  // the old scratch may still be read
    if (e->dq) (void)hipFree(e->dq);
    if (e->dy) (void)hipFree(e->dy);
    if (e->dout) (void)hipFree(e->dout);
    e->dq = nullptr; e->dy = nullptr; e->dout = nullptr; e->qcap = 0;
    const int cap = std::max(m, 256);
    HMD_HIP(ctx, hipMalloc(&e->dq, sizeof(double) * 2 * cap));
    HMD_HIP(ctx, hipMalloc(&e->dy, sizeof(float) * size_t(e->cfg.members) * cap));
    HMD_HIP(ctx, hipMalloc(&e->dout, sizeof(double) * 2 * cap));
    e->qcap = cap;
  }
  hipLaunchKernelGGL(k_ens_member_out, dim3((m + PQB - 1) / PQB, e->cfg.members), dim3(64), 0, s, m,
                     e->cfg.hidden, e->dparams, dXs, e->mu[0], e->mu[1], e->sd[0], e->sd[1], e->dy);
  HMD_HIP(ctx, hipGetLastError());
  hipLaunchKernelGGL(k_ens_reduce, dim3((m + 127) / 128), dim3(128), 0, s, m, e->cfg.members, e->dy, e->s_q,
                     dmean, dstd);
  HMD_HIP(ctx, hipGetLastError());
  return HMD_OK;
}

int ens_loss(const hmd_ens* e, double* loss) {
  if (!e || !loss) return HMD_EINVAL;
  for (size_t k = 0; k < e->loss.size(); ++k) loss[k] = e->loss[k];
  return HMD_OK;
}

int ens_grad_init(hmd_ctx* ctx, const double* X, const double* y, int n, const hmd_ens_cfg* cfg, int member,
                  double* params, double* grad, int* n_params) {
  if (!ctx || !X || !y) return HMD_EINVAL;
  hmd_ens_cfg c;
  if (cfg) c = *cfg;
  else hmd_ens_cfg_default(&c);
  int rc = check_cfg(ctx, c, n);
  if (rc != HMD_OK) return rc;
  if (member < 0 || member >= c.members) return HMD_EINVAL;
  HMD_HIP(ctx, hipSetDevice(ctx->device));
  hmd_ens e;
  e.ctx = ctx;
  e.cfg = c;
  float *dX = nullptr, *dy = nullptr, *dg = nullptr, *dw = nullptr;
  if ((rc = init_params(&e)) == HMD_OK && (rc = stage_data(&e, X, y, n, &dX, &dy, &dw)) == HMD_OK) {
    if (hipMalloc(&dg, sizeof(float) * size_t(c.members) * e.P) != hipSuccess) rc = HMD_ENOMEM;
    else rc = run_train(&e, n, dX, dy, dw, 1, dg);
  }
  if (rc == HMD_OK) {
    std::vector<float> hp(e.P), hg(e.P);
    if (hipMemcpy(hp.data(), e.dparams + size_t(member) * e.P, sizeof(float) * e.P, hipMemcpyDeviceToHost) !=
            hipSuccess ||
        hipMemcpy(hg.data(), dg + size_t(member) * e.P, sizeof(float) * e.P, hipMemcpyDeviceToHost) != hipSuccess)
      rc = HMD_EDEVICE;
    for (int p = 0; p < e.P; ++p) {
      if (params) params[p] = hp[p];
      if (grad) grad[p] = hg[p];
    }
    if (n_params) *n_params = e.P;
  }
  for (void* p : {(void*)dX, (void*)dy, (void*)dg, (void*)dw, (void*)e.dparams})
    if (p) (void)hipFree(p);
  return rc;
}

int ens_members(const hmd_ens* e) { return e ? e->cfg.members : 0; }

void ens_free(hmd_ens* e) {
  if (!e) return;
  if (e->dparams) (void)hipFree(e->dparams);
  if (e->dq) (void)hipFree(e->dq);
  if (e->dy) (void)hipFree(e->dy);
  if (e->dout) (void)hipFree(e->dout);
  delete e;
}

}  // extern "C"
