// Path-count predictor: a 32 -> 128 -> 128 -> 65 multilayer perceptron with
// BF16 operands on the matrix cores and FP32 accumulation, trained with Adam
// on FP32 master weights.  Inputs are the 32 structural features of a CFG;
// outputs are log1p of the number of simple paths with L entries (L = 1..64,
// deeper levels pooled into 64) and log1p of the prime-path count.  The
// predictions size the path pool of the batched form; results never depend on
// them.
//
// Every matrix product is C = A * Bt^T with A (M x K) and Bt (N x K) stored
// row-major in bf16 (K contiguous), M and N multiples of 64, K a multiple of
// 32: one workgroup of 4 waves computes a 64 x 64 tile, each wave a 16 x 64
// strip as four 16x16x32 MFMA accumulators.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "internal.h"

namespace tpg {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kIn = 32, kHid = 128, kOut = 65, kOutPad = 128;

// fp32 -> bf16, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
static inline uint16_t f2bf_host(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

struct GemmArgs {
  const uint16_t* A;
  int lda;
  const uint16_t* Bt;
  int ldb;
  int M, N, K;
  const float* bias;       // [N] or null
  const float* gate;       // multiply by (gate[row * ld_gate + col] > 0) or null
  int ld_gate;
  int relu;                // apply max(0, .)
  float* C;                // fp32 out or null
  int ldc;
  uint16_t* Cb;            // bf16 out (row-major) or null
  int ldcb;
  uint16_t* Cbt;           // bf16 out transposed (N x M) or null
  int ldcbt;
  int valid_m, valid_n;    // outside: written as 0
};

__global__ __launch_bounds__(256) void k_gemm_nt(GemmArgs g) {
  const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  const int m0 = (int)blockIdx.y * 64 + wave * 16;
  const int n0 = (int)blockIdx.x * 64;
  const int r = lane & 15, kq = (lane >> 4) * 8;
  f32x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const uint16_t* arow = g.A + (size_t)(m0 + r) * g.lda + kq;
  for (int k0 = 0; k0 < g.K; k0 += 32) {
    const bf16x8 a = *reinterpret_cast<const bf16x8*>(arow + k0);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const bf16x8 b =
          *reinterpret_cast<const bf16x8*>(g.Bt + (size_t)(n0 + 16 * t + r) * g.ldb + kq + k0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
    }
  }
  // lane holds D[4 * (lane / 16) + j][lane % 16] of each 16x16 tile
#pragma unroll
  for (int t = 0; t < 4; ++t) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = m0 + 4 * (lane >> 4) + j;
      const int col = n0 + 16 * t + (lane & 15);
      float v = acc[t][j];
      if (g.bias) v += g.bias[col];
      if (g.relu) v = v > 0.f ? v : 0.f;
      if (g.gate && !(g.gate[(size_t)row * g.ld_gate + col] > 0.f)) v = 0.f;
      if (row >= g.valid_m || col >= g.valid_n) v = 0.f;
      if (g.C) g.C[(size_t)row * g.ldc + col] = v;
      const uint16_t h = f2bf(v);
      if (g.Cb) g.Cb[(size_t)row * g.ldcb + col] = h;
      if (g.Cbt) g.Cbt[(size_t)col * g.ldcbt + row] = h;
    }
  }
}

static hipError_t gemm(const GemmArgs& a, hipStream_t st) {
  if (a.M % 64 || a.N % 64 || a.K % 32) return hipErrorInvalidValue;
  dim3 grid((unsigned)(a.N / 64), (unsigned)(a.M / 64));
  k_gemm_nt<<<grid, 256, 0, st>>>(a);
  return hipGetLastError();
}

// features -> normalized bf16 rows (and the transposed copy, 64 rows)
__global__ void k_prep(const float* x, int n, int rows, const float* mean, const float* stdv,
                       uint16_t* xb, uint16_t* xbt) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= rows * kIn) return;
  const int b = i / kIn, f = i % kIn;
  const float v = b < n ? (x[(size_t)b * kIn + f] - mean[f]) / stdv[f] : 0.f;
  const uint16_t h = f2bf(v);
  xb[(size_t)b * kIn + f] = h;
  xbt[(size_t)f * rows + b] = h;
}

// d loss / d y for loss = mean over n x 65 of (y - t)^2; loss sum accumulated
__global__ void k_loss_grad(const float* y, const float* t, int n, int rows, float* dy,
                            uint16_t* dyb, uint16_t* dybt, float* loss_sum) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= rows * kOutPad) return;
  const int b = i / kOutPad, o = i % kOutPad;
  float g = 0.f, sq = 0.f;
  if (b < n && o < kOut) {
    const float e = y[(size_t)b * kOutPad + o] - t[(size_t)b * kOut + o];
    g = 2.f * e / (float)(n * kOut);
    sq = e * e;
  }
  dy[i] = g;
  const uint16_t h = f2bf(g);
  dyb[i] = h;
  dybt[(size_t)o * rows + b] = h;
  if (sq != 0.f) atomicAdd(loss_sum, sq);
}

__global__ void k_colsum(const float* g, int rows, int cols, int valid, float* out) {
  const int c = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (c >= valid) return;
  float s = 0.f;
  for (int r = 0; r < rows; ++r) s += g[(size_t)r * cols + c];
  out[c] = s;
}

struct AdamArgs {
  float* w;
  float* m;
  float* v;
  const float* g;
  int n;
  float lr, b1, b2, eps, c1, c2;  // c1 = 1 - b1^t, c2 = 1 - b2^t
};

__global__ void k_adam(AdamArgs a) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= a.n) return;
  const float g = a.g[i];
  const float m = a.b1 * a.m[i] + (1.f - a.b1) * g;
  const float v = a.b2 * a.v[i] + (1.f - a.b2) * g * g;
  a.m[i] = m;
  a.v[i] = v;
  a.w[i] -= a.lr * (m / a.c1) / (sqrtf(v / a.c2) + a.eps);
}

// fp32 master W (rows x cols, first valid_cols used) -> bf16 W and W^T
__global__ void k_refresh(const float* w, int rows, int cols, uint16_t* wb, uint16_t* wbt,
                          int ld_t) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= rows * cols) return;
  const int r = i / cols, c = i % cols;
  const uint16_t h = f2bf(w[i]);
  wb[i] = h;
  wbt[(size_t)c * ld_t + r] = h;
}

}  // namespace tpg

using namespace tpg;

// parameters, packed: W1 [32][128], b1 [128], W2 [128][128], b2 [128],
// W3 [128][65], b3 [65]
#define TPG_MLP_NPARAMS_ (kIn * kHid + kHid + kHid * kHid + kHid + kHid * kOut + kOut)

struct tpg_mlp {
  int device = 0;
  hipStream_t st = nullptr;
  // fp32 masters (W3 / b3 padded to 128 columns), Adam moments, gradients
  float* w1 = nullptr; float* w2 = nullptr; float* w3 = nullptr;
  float* b1 = nullptr; float* b2 = nullptr; float* b3 = nullptr;
  float* mom = nullptr;   // m then v for all of the above, same layout
  float* grad = nullptr;  // gradients, same layout
  float* master = nullptr;  // base of the fp32 block
  size_t n_master = 0;
  // bf16 copies: W (in x out) and W^T (out x in); W1^T is 128 x 32, W1 is 64 x 128
  uint16_t* w1b = nullptr; uint16_t* w1bt = nullptr;
  uint16_t* w2b = nullptr; uint16_t* w2bt = nullptr;
  uint16_t* w3b = nullptr; uint16_t* w3bt = nullptr;
  float* mean = nullptr; float* stdv = nullptr;
  float h_mean[kIn], h_std[kIn];
  int64_t step = 0;
  // activations for up to `rows` rows
  int rows = 0;
  void* act = nullptr;
  size_t act_bytes = 0;
  float *x = nullptr, *t = nullptr, *h1 = nullptr, *h2 = nullptr, *y = nullptr, *dy = nullptr,
        *dh2 = nullptr, *dh1 = nullptr, *loss = nullptr;
  uint16_t *xb = nullptr, *xbt = nullptr, *h1b = nullptr, *h1bt = nullptr, *h2b = nullptr,
           *h2bt = nullptr, *dyb = nullptr, *dybt = nullptr, *dh2b = nullptr, *dh2bt = nullptr,
           *dh1b = nullptr, *dh1bt = nullptr;
};

namespace {

// fp32 block layout (floats): w1 64x128 (rows 32..63 stay 0), b1 128, w2 128x128,
// b2 128, w3 128x128, b3 128
constexpr size_t oW1 = 0, oB1 = oW1 + 64 * kHid, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid,
                 oW3 = oB2 + kHid, oB3 = oW3 + kHid * kOutPad, oEnd = oB3 + kOutPad;

tpg_status mlp_alloc(tpg_mlp* m) {
  TPG_HIP(hipSetDevice(m->device));
  TPG_HIP(hipStreamCreateWithFlags(&m->st, hipStreamNonBlocking));
  m->n_master = oEnd;
  TPG_HIP(hipMalloc(&m->master, sizeof(float) * oEnd * 4));  // w, m, v, grad
  TPG_HIP(hipMemset(m->master, 0, sizeof(float) * oEnd * 4));
  m->w1 = m->master + oW1;
  m->b1 = m->master + oB1;
  m->w2 = m->master + oW2;
  m->b2 = m->master + oB2;
  m->w3 = m->master + oW3;
  m->b3 = m->master + oB3;
  m->mom = m->master + oEnd;
  m->grad = m->master + 3 * oEnd;
  uint16_t* bb = nullptr;
  const size_t nb = 2 * (64 * kHid + kHid * kHid + kHid * kOutPad);
  TPG_HIP(hipMalloc(&bb, sizeof(uint16_t) * nb));
  TPG_HIP(hipMemset(bb, 0, sizeof(uint16_t) * nb));
  m->w1b = bb;
  m->w1bt = m->w1b + 64 * kHid;
  m->w2b = m->w1bt + 64 * kHid;
  m->w2bt = m->w2b + kHid * kHid;
  m->w3b = m->w2bt + kHid * kHid;
  m->w3bt = m->w3b + kHid * kOutPad;
  TPG_HIP(hipMalloc(&m->mean, sizeof(float) * 2 * kIn));
  m->stdv = m->mean + kIn;
  for (int i = 0; i < kIn; ++i) m->h_mean[i] = 0.f, m->h_std[i] = 1.f;
  TPG_HIP(hipMemcpy(m->mean, m->h_mean, sizeof(float) * kIn, hipMemcpyHostToDevice));
  TPG_HIP(hipMemcpy(m->stdv, m->h_std, sizeof(float) * kIn, hipMemcpyHostToDevice));
  return TPG_OK;
}

tpg_status mlp_rows(tpg_mlp* m, int n) {
  const int rows = ((n + 63) / 64) * 64;
  if (rows <= m->rows) return TPG_OK;
  if (m->act) TPG_HIP(hipFree(m->act));
  m->act = nullptr;
  const size_t R = (size_t)rows;
  size_t floats = R * kIn + R * kOut + 2 * R * kHid + 2 * R * kOutPad + 2 * R * kHid + 64;
  size_t halves = R * kIn + 64 * R + 2 * (2 * R * kHid) + 2 * R * kOutPad + 2 * (2 * R * kHid);
  m->act_bytes = floats * 4 + halves * 2 + 1024;
  TPG_HIP(hipMalloc(&m->act, m->act_bytes));
  TPG_HIP(hipMemset(m->act, 0, m->act_bytes));
  float* f = (float*)m->act;
  m->x = f; f += R * kIn;
  m->t = f; f += R * kOut;
  m->h1 = f; f += R * kHid;
  m->h2 = f; f += R * kHid;
  m->y = f; f += R * kOutPad;
  m->dy = f; f += R * kOutPad;
  m->dh2 = f; f += R * kHid;
  m->dh1 = f; f += R * kHid;
  m->loss = f; f += 64;
  uint16_t* h = (uint16_t*)f;
  m->xb = h; h += R * kIn;
  m->xbt = h; h += 64 * R;
  m->h1b = h; h += R * kHid;
  m->h1bt = h; h += R * kHid;
  m->h2b = h; h += R * kHid;
  m->h2bt = h; h += R * kHid;
  m->dyb = h; h += R * kOutPad;
  m->dybt = h; h += R * kOutPad;
  m->dh2b = h; h += R * kHid;
  m->dh2bt = h; h += R * kHid;
  m->dh1b = h; h += R * kHid;
  m->dh1bt = h; h += R * kHid;
  m->rows = rows;
  return TPG_OK;
}

tpg_status refresh_bf16(tpg_mlp* m) {
  hipStream_t st = m->st;
  // W1 master is 64 x 128 (rows >= 32 zero): W1^T is 128 x 32 for the forward
  k_refresh<<<(64 * kHid + 255) / 256, 256, 0, st>>>(m->w1, 64, kHid, m->w1b, m->w1bt, 64);
  k_refresh<<<(kHid * kHid + 255) / 256, 256, 0, st>>>(m->w2, kHid, kHid, m->w2b, m->w2bt, kHid);
  k_refresh<<<(kHid * kOutPad + 255) / 256, 256, 0, st>>>(m->w3, kHid, kOutPad, m->w3b, m->w3bt, kHid);
  TPG_HIP(hipGetLastError());
  return TPG_OK;
}

GemmArgs ga(const uint16_t* A, int lda, const uint16_t* Bt, int ldb, int M, int N, int K) {
  GemmArgs g{};
  g.A = A;
  g.lda = lda;
  g.Bt = Bt;
  g.ldb = ldb;
  g.M = M;
  g.N = N;
  g.K = K;
  g.valid_m = M;
  g.valid_n = N;
  return g;
}

tpg_status forward(tpg_mlp* m, int n) {
  const int R = m->rows;
  hipStream_t st = m->st;
  k_prep<<<(R * kIn + 255) / 256, 256, 0, st>>>(m->x, n, R, m->mean, m->stdv, m->xb, m->xbt);
  // W1^T as stored is 128 x 64 with ld 64 (columns 32..63 zero): use K = 32
  GemmArgs g1 = ga(m->xb, kIn, m->w1bt, 64, R, kHid, kIn);
  g1.bias = m->b1;
  g1.relu = 1;
  g1.C = m->h1;
  g1.ldc = kHid;
  g1.Cb = m->h1b;
  g1.ldcb = kHid;
  g1.Cbt = m->h1bt;
  g1.ldcbt = R;
  g1.valid_m = n;
  TPG_HIP(gemm(g1, st));
  GemmArgs g2 = ga(m->h1b, kHid, m->w2bt, kHid, R, kHid, kHid);
  g2.bias = m->b2;
  g2.relu = 1;
  g2.C = m->h2;
  g2.ldc = kHid;
  g2.Cb = m->h2b;
  g2.ldcb = kHid;
  g2.Cbt = m->h2bt;
  g2.ldcbt = R;
  g2.valid_m = n;
  TPG_HIP(gemm(g2, st));
  GemmArgs g3 = ga(m->h2b, kHid, m->w3bt, kHid, R, kOutPad, kHid);
  g3.bias = m->b3;
  g3.C = m->y;
  g3.ldc = kOutPad;
  g3.valid_m = n;
  g3.valid_n = kOut;
  TPG_HIP(gemm(g3, st));
  return TPG_OK;
}

// gradients of the mean squared error into m->grad (fp32 block layout)
tpg_status backward(tpg_mlp* m, int n) {
  const int R = m->rows;
  hipStream_t st = m->st;
  TPG_HIP(hipMemsetAsync(m->loss, 0, sizeof(float), st));
  k_loss_grad<<<(R * kOutPad + 255) / 256, 256, 0, st>>>(m->y, m->t, n, R, m->dy, m->dyb, m->dybt,
                                                         m->loss);
  float* G = m->grad;
  // dW3 = H2^T dY  (128 x 128), db3
  GemmArgs w3 = ga(m->h2bt, R, m->dybt, R, kHid, kOutPad, R);
  w3.C = G + oW3;
  w3.ldc = kOutPad;
  w3.valid_n = kOut;
  TPG_HIP(gemm(w3, st));
  k_colsum<<<1, 128, 0, st>>>(m->dy, R, kOutPad, kOutPad, G + oB3);
  // dH2 = (dY W3^T) * (H2 > 0)
  GemmArgs h2 = ga(m->dyb, kOutPad, m->w3b, kOutPad, R, kHid, kOutPad);
  h2.gate = m->h2;
  h2.ld_gate = kHid;
  h2.C = m->dh2;
  h2.ldc = kHid;
  h2.Cb = m->dh2b;
  h2.ldcb = kHid;
  h2.Cbt = m->dh2bt;
  h2.ldcbt = R;
  h2.valid_m = n;
  TPG_HIP(gemm(h2, st));
  // dW2 = H1^T dH2, db2
  GemmArgs w2 = ga(m->h1bt, R, m->dh2bt, R, kHid, kHid, R);
  w2.C = G + oW2;
  w2.ldc = kHid;
  TPG_HIP(gemm(w2, st));
  k_colsum<<<1, 128, 0, st>>>(m->dh2, R, kHid, kHid, G + oB2);
  // dH1 = (dH2 W2^T) * (H1 > 0)
  GemmArgs h1 = ga(m->dh2b, kHid, m->w2b, kHid, R, kHid, kHid);
  h1.gate = m->h1;
  h1.ld_gate = kHid;
  h1.C = m->dh1;
  h1.ldc = kHid;
  h1.Cbt = m->dh1bt;
  h1.ldcbt = R;
  h1.valid_m = n;
  TPG_HIP(gemm(h1, st));
  // dW1 = X^T dH1 (64 x 128, rows 32..63 of X^T are zero), db1
  GemmArgs w1 = ga(m->xbt, R, m->dh1bt, R, 64, kHid, R);
  w1.C = G + oW1;
  w1.ldc = kHid;
  w1.valid_m = kIn;
  TPG_HIP(gemm(w1, st));
  k_colsum<<<1, 128, 0, st>>>(m->dh1, R, kHid, kHid, G + oB1);
  TPG_HIP(hipGetLastError());
  return TPG_OK;
}

tpg_status upload_rows(tpg_mlp* m, const float* x, const float* t, int n) {
  TPG_TRY(mlp_rows(m, n));
  TPG_HIP(hipMemcpyAsync(m->x, x, sizeof(float) * kIn * n, hipMemcpyHostToDevice, m->st));
  if (t) TPG_HIP(hipMemcpyAsync(m->t, t, sizeof(float) * kOut * n, hipMemcpyHostToDevice, m->st));
  return TPG_OK;
}

// packed <-> padded fp32 block
void pack_params(const std::vector<float>& blk, float* p) {
  size_t q = 0;
  for (int i = 0; i < kIn; ++i)
    for (int j = 0; j < kHid; ++j) p[q++] = blk[oW1 + i * kHid + j];
  for (int j = 0; j < kHid; ++j) p[q++] = blk[oB1 + j];
  for (int i = 0; i < kHid; ++i)
    for (int j = 0; j < kHid; ++j) p[q++] = blk[oW2 + i * kHid + j];
  for (int j = 0; j < kHid; ++j) p[q++] = blk[oB2 + j];
  for (int i = 0; i < kHid; ++i)
    for (int j = 0; j < kOut; ++j) p[q++] = blk[oW3 + i * kOutPad + j];
  for (int j = 0; j < kOut; ++j) p[q++] = blk[oB3 + j];
}

void unpack_params(const float* p, std::vector<float>& blk) {
  blk.assign(oEnd, 0.f);
  size_t q = 0;
  for (int i = 0; i < kIn; ++i)
    for (int j = 0; j < kHid; ++j) blk[oW1 + i * kHid + j] = p[q++];
  for (int j = 0; j < kHid; ++j) blk[oB1 + j] = p[q++];
  for (int i = 0; i < kHid; ++i)
    for (int j = 0; j < kHid; ++j) blk[oW2 + i * kHid + j] = p[q++];
  for (int j = 0; j < kHid; ++j) blk[oB2 + j] = p[q++];
  for (int i = 0; i < kHid; ++i)
    for (int j = 0; j < kOut; ++j) blk[oW3 + i * kOutPad + j] = p[q++];
  for (int j = 0; j < kOut; ++j) blk[oB3 + j] = p[q++];
}

uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

extern "C" {

int32_t tpg_mlp_num_params(void) { return TPG_MLP_NPARAMS_; }

tpg_status tpg_mlp_create(int32_t device, uint64_t seed, tpg_mlp** out) {
  if (!out) return fail(TPG_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
    (void)hipGetLastError();
    return fail(TPG_ERR_DEVICE, "no HIP device available");
  }
  if (device < 0) TPG_HIP(hipGetDevice(&device));
  tpg_mlp* m = new (std::nothrow) tpg_mlp;
  if (!m) return fail(TPG_ERR_OOM_HOST, "mlp");
  m->device = device;
  tpg_status s = mlp_alloc(m);
  if (s != TPG_OK) {
    tpg_mlp_free(m);
    return s;
  }
  // He-uniform initialization from a counter-based generator; biases zero
  std::vector<float> p(TPG_MLP_NPARAMS_, 0.f);
  uint64_t st = seed;
  auto uni = [&]() { return (double)(splitmix(st) >> 11) * (1.0 / 9007199254740992.0); };
  size_t q = 0;
  const int fan[3] = {kIn, kHid, kHid}, outs[3] = {kHid, kHid, kOut};
  for (int l = 0; l < 3; ++l) {
    const double lim = std::sqrt(6.0 / fan[l]);
    for (int i = 0; i < fan[l] * outs[l]; ++i) p[q++] = (float)((2.0 * uni() - 1.0) * lim);
    q += outs[l];
  }
  s = tpg_mlp_set_params(m, p.data());
  if (s != TPG_OK) {
    tpg_mlp_free(m);
    return s;
  }
  *out = m;
  return TPG_OK;
}

void tpg_mlp_free(tpg_mlp* m) {
  if (!m) return;
  (void)hipSetDevice(m->device);
  if (m->st) (void)hipStreamSynchronize(m->st);
  if (m->master) (void)hipFree(m->master);
  if (m->w1b) (void)hipFree(m->w1b);
  if (m->mean) (void)hipFree(m->mean);
  if (m->act) (void)hipFree(m->act);
  if (m->st) (void)hipStreamDestroy(m->st);
  delete m;
}

tpg_status tpg_mlp_set_params(tpg_mlp* m, const float* params) {
  if (!m || !params) return fail(TPG_ERR_INVALID_ARG, "NULL argument");
  std::vector<float> blk;
  unpack_params(params, blk);
  TPG_HIP(hipSetDevice(m->device));
  TPG_HIP(hipMemcpy(m->master, blk.data(), sizeof(float) * oEnd, hipMemcpyHostToDevice));
  TPG_HIP(hipMemset(m->mom, 0, sizeof(float) * 2 * oEnd));
  m->step = 0;
  TPG_TRY(refresh_bf16(m));
  TPG_HIP(hipStreamSynchronize(m->st));
  return TPG_OK;
}

tpg_status tpg_mlp_get_params(const tpg_mlp* m, float* params) {
  if (!m || !params) return fail(TPG_ERR_INVALID_ARG, "NULL argument");
  std::vector<float> blk(oEnd);
  TPG_HIP(hipStreamSynchronize(m->st));
  TPG_HIP(hipMemcpy(blk.data(), m->master, sizeof(float) * oEnd, hipMemcpyDeviceToHost));
  pack_params(blk, params);
  return TPG_OK;
}

tpg_status tpg_mlp_set_normalizer(tpg_mlp* m, const float* mean, const float* stdv) {
  if (!m || !mean || !stdv) return fail(TPG_ERR_INVALID_ARG, "NULL argument");
  for (int i = 0; i < kIn; ++i) {
    m->h_mean[i] = mean[i];
    m->h_std[i] = stdv[i] > 1e-12f ? stdv[i] : 1.f;
  }
  TPG_HIP(hipMemcpy(m->mean, m->h_mean, sizeof(float) * kIn, hipMemcpyHostToDevice));
  TPG_HIP(hipMemcpy(m->stdv, m->h_std, sizeof(float) * kIn, hipMemcpyHostToDevice));
  return TPG_OK;
}

tpg_status tpg_mlp_forward(tpg_mlp* m, const float* x, int32_t n, float* y) {
  if (!m || !x || !y || n < 1) return fail(TPG_ERR_INVALID_ARG, "bad argument");
  TPG_HIP(hipSetDevice(m->device));
  TPG_TRY(upload_rows(m, x, nullptr, n));
  TPG_TRY(forward(m, n));
  std::vector<float> yp((size_t)n * kOutPad);
  TPG_HIP(hipMemcpyAsync(yp.data(), m->y, sizeof(float) * yp.size(), hipMemcpyDeviceToHost, m->st));
  TPG_HIP(hipStreamSynchronize(m->st));
  for (int b = 0; b < n; ++b) memcpy(y + (size_t)b * kOut, yp.data() + (size_t)b * kOutPad, sizeof(float) * kOut);
  return TPG_OK;
}

tpg_status tpg_mlp_gradients(tpg_mlp* m, const float* x, const float* t, int32_t n, float* grad,
                             float* loss) {
  if (!m || !x || !t || n < 1) return fail(TPG_ERR_INVALID_ARG, "bad argument");
  TPG_HIP(hipSetDevice(m->device));
  TPG_TRY(upload_rows(m, x, t, n));
  TPG_TRY(forward(m, n));
  TPG_TRY(backward(m, n));
  TPG_HIP(hipStreamSynchronize(m->st));
  if (grad) {
    std::vector<float> blk(oEnd);
    TPG_HIP(hipMemcpy(blk.data(), m->grad, sizeof(float) * oEnd, hipMemcpyDeviceToHost));
    pack_params(blk, grad);
  }
  if (loss) {
    float s = 0;
    TPG_HIP(hipMemcpy(&s, m->loss, sizeof(float), hipMemcpyDeviceToHost));
    *loss = s / (float)(n * kOut);
  }
  return TPG_OK;
}

tpg_status tpg_mlp_train_step(tpg_mlp* m, const float* x, const float* t, int32_t n, float lr,
                              float* loss) {
  if (!m || !x || !t || n < 1) return fail(TPG_ERR_INVALID_ARG, "bad argument");
  TPG_HIP(hipSetDevice(m->device));
  TPG_TRY(upload_rows(m, x, t, n));
  TPG_TRY(forward(m, n));
  TPG_TRY(backward(m, n));
  m->step += 1;
  AdamArgs a{};
  a.w = m->master;
  a.m = m->mom;
  a.v = m->mom + oEnd;
  a.g = m->grad;
  a.n = (int)oEnd;
  a.lr = lr;
  a.b1 = 0.9f;
  a.b2 = 0.999f;
  a.eps = 1e-8f;
  a.c1 = (float)(1.0 - std::pow(0.9, (double)m->step));
  a.c2 = (float)(1.0 - std::pow(0.999, (double)m->step));
  k_adam<<<(unsigned)((oEnd + 255) / 256), 256, 0, m->st>>>(a);
  TPG_HIP(hipGetLastError());
  TPG_TRY(refresh_bf16(m));
  if (loss) {
    float s = 0;
    TPG_HIP(hipMemcpyAsync(&s, m->loss, sizeof(float), hipMemcpyDeviceToHost, m->st));
    TPG_HIP(hipStreamSynchronize(m->st));
    *loss = s / (float)(n * kOut);
  }
  return TPG_OK;
}

// File: "TPGMLP1\n", int32 n_params, 32 means, 32 stds, n_params fp32 values.
tpg_status tpg_mlp_save(const tpg_mlp* m, const char* path) {
  if (!m || !path) return fail(TPG_ERR_INVALID_ARG, "NULL argument");
  std::vector<float> p(TPG_MLP_NPARAMS_);
  TPG_TRY(tpg_mlp_get_params(m, p.data()));
  FILE* f = fopen(path, "wb");
  if (!f) return fail(TPG_ERR_INVALID_ARG, "cannot open %s", path);
  const int32_t np = TPG_MLP_NPARAMS_;
  bool ok = fwrite("TPGMLP1\n", 1, 8, f) == 8 && fwrite(&np, 4, 1, f) == 1 &&
            fwrite(m->h_mean, 4, kIn, f) == (size_t)kIn && fwrite(m->h_std, 4, kIn, f) == (size_t)kIn &&
            fwrite(p.data(), 4, p.size(), f) == p.size();
  ok = (fclose(f) == 0) && ok;
  return ok ? TPG_OK : fail(TPG_ERR_INVALID_ARG, "write failed: %s", path);
}

tpg_status tpg_mlp_load(int32_t device, const char* path, tpg_mlp** out) {
  if (!path || !out) return fail(TPG_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  FILE* f = fopen(path, "rb");
  if (!f) return fail(TPG_ERR_INVALID_ARG, "cannot open %s", path);
  char magic[8];
  int32_t np = 0;
  float mean[kIn], stdv[kIn];
  std::vector<float> p(TPG_MLP_NPARAMS_);
  bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "TPGMLP1\n", 8) == 0 &&
            fread(&np, 4, 1, f) == 1 && np == TPG_MLP_NPARAMS_ &&
            fread(mean, 4, kIn, f) == (size_t)kIn && fread(stdv, 4, kIn, f) == (size_t)kIn &&
            fread(p.data(), 4, p.size(), f) == p.size();
  fclose(f);
  if (!ok) return fail(TPG_ERR_INVALID_ARG, "%s is not a predictor file", path);
  tpg_mlp* m = nullptr;
  TPG_TRY(tpg_mlp_create(device, 0, &m));
  tpg_status s = tpg_mlp_set_params(m, p.data());
  if (s == TPG_OK) s = tpg_mlp_set_normalizer(m, mean, stdv);
  if (s != TPG_OK) {
    tpg_mlp_free(m);
    return s;
  }
  *out = m;
  return TPG_OK;
}

}  // extern "C"
