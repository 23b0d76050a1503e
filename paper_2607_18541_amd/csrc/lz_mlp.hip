// lz_mlp.hip -- gfx950 kernels of the per-block threshold selector.
//
// A 64 -> 128 -> 128 -> 16 perceptron (ReLU, softmax over 16 threshold
// tuples) scores encoder settings per LZ block from its match-length /
// distance-class histogram (the quantities Sec. 3.3 and Sec. 4.3 tie to
// throughput and to offset cost).  Shapes are tiny (batch 256, width 128), so
// the kernels are latency-bound: one fp32 GEMM kernel with 16x16 LDS tiles
// and fused bias / ReLU / ReLU-gradient epilogues, a softmax cross-entropy
// kernel, a column-sum kernel for bias gradients and an Adam kernel.  Matrix
// cores would not shorten a chain of dependent launches at these sizes.
//
// Parameter vector (fp32, row-major): W1 64x128, b1 128, W2 128x128, b2 128,
// W3 128x16, b3 16 = 26,896 values.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <mutex>
#include <vector>

#include "lz_internal.h"

namespace {

constexpr int IN = 64, H = 128, OUT = 16;
constexpr uint64_t OW1 = 0, OB1 = OW1 + IN * H, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H, OB3 = OW3 + H * OUT,
                   NP = OB3 + OUT;
constexpr int T = 16;

// C[M,N] (ldc) = op(A)[M,K] * op(B)[K,N] (+ bias[N]); epilogue: 0 none,
// 1 ReLU, 2 multiply by (R[M,N] > 0) (ReLU gradient; R has ldc).
// op(A) = A (lda, row-major) or A^T when TA; likewise B.
template <bool TA, bool TB>
__global__ __launch_bounds__(T * T) void k_gemm(int M, int N, int K, const float* __restrict__ A, int lda,
                                                 const float* __restrict__ B, int ldb, float* __restrict__ C, int ldc,
                                                 const float* __restrict__ bias, int epi, const float* __restrict__ R) {
  __shared__ float sa[T][T + 1], sb[T][T + 1];
  const int tx = threadIdx.x % T, ty = threadIdx.x / T;
  const int row = blockIdx.y * T + ty, col = blockIdx.x * T + tx;
  float acc = 0.f;
  for (int k0 = 0; k0 < K; k0 += T) {
    const int ka = k0 + tx, kb = k0 + ty;
    float a = 0.f, b = 0.f;
    if (row < M && ka < K) a = TA ? A[(size_t)ka * lda + row] : A[(size_t)row * lda + ka];
    if (kb < K && col < N) b = TB ? B[(size_t)col * ldb + kb] : B[(size_t)kb * ldb + col];
    sa[ty][tx] = a;
    sb[ty][tx] = b;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < T; ++k) acc = fmaf(sa[ty][k], sb[k][tx], acc);
    __syncthreads();
  }
  if (row < M && col < N) {
    if (bias) acc += bias[col];
    if (epi == 1) acc = fmaxf(acc, 0.f);
    if (epi == 2) acc = (R[(size_t)row * ldc + col] > 0.f) ? acc : 0.f;
    C[(size_t)row * ldc + col] = acc;
  }
}

// dlogits = (softmax(logits) - onehot(label)) / B; loss[0] += mean CE.
__global__ void k_softmax_ce(int Bn, const float* __restrict__ logits, const int32_t* __restrict__ labels,
                             float* __restrict__ dlogits, float* __restrict__ loss) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= Bn) return;
  const float* z = logits + (size_t)r * OUT;
  float mx = z[0];
  for (int j = 1; j < OUT; ++j) mx = fmaxf(mx, z[j]);
  float s = 0.f;
  for (int j = 0; j < OUT; ++j) s += expf(z[j] - mx);
  const int y = labels[r];
  for (int j = 0; j < OUT; ++j) {
    const float p = expf(z[j] - mx) / s;
    dlogits[(size_t)r * OUT + j] = (p - (j == y ? 1.f : 0.f)) / (float)Bn;
  }
  if (loss) atomicAdd(loss, (logf(s) - (z[y] - mx)) / (float)Bn);
}

// out[j] = sum_r X[r, j] (bias gradients)
__global__ void k_colsum(int Bn, int N, const float* __restrict__ X, float* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  float s = 0.f;
  for (int r = 0; r < Bn; ++r) s += X[(size_t)r * N + j];
  out[j] = s;
}

__global__ void k_adam(uint64_t n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

template <bool TA, bool TB>
void gemm(hipStream_t s, int M, int N, int K, const float* A, int lda, const float* B, int ldb, float* C, int ldc,
          const float* bias, int epi, const float* R) {
  dim3 grid((N + T - 1) / T, (M + T - 1) / T);
  hipLaunchKernelGGL((k_gemm<TA, TB>), grid, dim3(T * T), 0, s, M, N, K, A, lda, B, ldb, C, ldc, bias, epi, R);
}

// Backward pass with its per-row work buffer `work` (batch x 272 floats:
// dlogits, then the two hidden-layer gradients; every element is written
// before it is read, so the buffer needs no clearing).
int backward(const float* d_params, uint32_t batch, const float* d_x, const float* d_h1, const float* d_h2,
             const float* d_logits, const int32_t* d_labels, float* d_grads, float* work, float* d_loss,
             hipStream_t s) {
  const float* P = d_params;
  float* d3 = work;                          // batch x 16
  float* dh2 = d3 + (size_t)batch * OUT;     // batch x 128
  float* dh1 = dh2 + (size_t)batch * H;      // batch x 128
  hipLaunchKernelGGL(k_softmax_ce, dim3((batch + 255) / 256), dim3(256), 0, s, (int)batch, d_logits, d_labels, d3,
                     d_loss);
  // layer 3
  gemm<true, false>(s, H, OUT, batch, d_h2, H, d3, OUT, d_grads + OW3, OUT, nullptr, 0, nullptr);
  hipLaunchKernelGGL(k_colsum, dim3(1), dim3(64), 0, s, (int)batch, OUT, d3, d_grads + OB3);
  gemm<false, true>(s, batch, H, OUT, d3, OUT, P + OW3, OUT, dh2, H, nullptr, 2, d_h2);
  // layer 2
  gemm<true, false>(s, H, H, batch, d_h1, H, dh2, H, d_grads + OW2, H, nullptr, 0, nullptr);
  hipLaunchKernelGGL(k_colsum, dim3(1), dim3(128), 0, s, (int)batch, H, dh2, d_grads + OB2);
  gemm<false, true>(s, batch, H, H, dh2, H, P + OW2, H, dh1, H, nullptr, 2, d_h1);
  // layer 1
  gemm<true, false>(s, IN, H, batch, d_x, IN, dh1, H, d_grads + OW1, H, nullptr, 0, nullptr);
  hipLaunchKernelGGL(k_colsum, dim3(1), dim3(128), 0, s, (int)batch, H, dh1, d_grads + OB1);
  if (hipGetLastError() != hipSuccess) return lz::fail(LZ_E_HIP, "backward launch failed");
  return 0;
}

constexpr uint32_t kNoAllocMaxBatch = 4096;
constexpr uint64_t kWorkPerRow = OUT + 2 * H;  // 272 floats

}  // namespace

// Work buffer of the allocation-free backward pass: a file-scope device array
// (4096 x 272 floats = 4.25 MiB; one copy per GPU, alive until the process
// ends).  In host code its name is a host-side stand-in, not a device
// address; kernels get the address hipGetSymbolAddress returns for the
// current device.
static __device__ __align__(256) float scratch[(uint64_t)kNoAllocMaxBatch * kWorkPerRow];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of `scratch`, resolved once per device.
int scratch_for_current_device(float** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return lz::fail(LZ_E_HIP, "hipGetDevice failed");
  if (dev < 0 || dev >= kMaxDevices) return lz::fail(LZ_E_INVAL, "device %d beyond the %d supported", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return lz::fail(LZ_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = (float*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return 0;
}

}  // namespace

extern "C" {

uint64_t lz_mlp_param_count(void) { return NP; }

// Forward pass for `batch` rows of x [batch x 64]: h1, h2 [batch x 128] and
// logits [batch x 16] (device buffers, row-major).
int lz_mlp_forward(const float* d_params, uint32_t batch, const float* d_x, float* d_h1, float* d_h2, float* d_logits,
                   void* stream) {
  if (!d_params || !d_x || !d_h1 || !d_h2 || !d_logits) return lz::fail(LZ_E_INVAL, "null argument");
  if (batch == 0) return 0;
  hipStream_t s = (hipStream_t)stream;
  const float* P = d_params;
  gemm<false, false>(s, batch, H, IN, d_x, IN, P + OW1, H, d_h1, H, P + OB1, 1, nullptr);
  gemm<false, false>(s, batch, H, H, d_h1, H, P + OW2, H, d_h2, H, P + OB2, 1, nullptr);
  gemm<false, false>(s, batch, OUT, H, d_h2, H, P + OW3, OUT, d_logits, OUT, P + OB3, 0, nullptr);
  if (hipGetLastError() != hipSuccess) return lz::fail(LZ_E_HIP, "forward launch failed");
  return 0;
}

// Gradient of the mean softmax cross-entropy (labels int32 in [0,16)) into
// d_grads [26,896]; d_work needs batch x (16 + 128 + 128) floats; d_loss (may
// be null) receives += the mean loss.  Uses the activations of lz_mlp_forward.
int lz_mlp_backward(const float* d_params, uint32_t batch, const float* d_x, const float* d_h1, const float* d_h2,
                    const float* d_logits, const int32_t* d_labels, float* d_grads, float* d_work, float* d_loss,
                    void* stream) {
  if (!d_params || !d_x || !d_h1 || !d_h2 || !d_logits || !d_labels || !d_grads || !d_work)
    return lz::fail(LZ_E_INVAL, "null argument");
  if (batch == 0) return 0;
  return backward(d_params, batch, d_x, d_h1, d_h2, d_logits, d_labels, d_grads, d_work, d_loss, (hipStream_t)stream);
}

// lz_mlp_backward with its work buffer in the library's per-device `scratch`
// array: no allocation of any kind.  Calls on one GPU share that array, so
// calls that overlap on one GPU (e.g. on two streams) race.
int lz_mlp_backward_noalloc(const float* d_params, uint32_t batch, const float* d_x, const float* d_h1,
                            const float* d_h2, const float* d_logits, const int32_t* d_labels, float* d_grads,
                            float* d_loss, void* stream) {
  if (!d_params || !d_x || !d_h1 || !d_h2 || !d_logits || !d_labels || !d_grads)
    return lz::fail(LZ_E_INVAL, "null argument");
  if (batch > kNoAllocMaxBatch)
    return lz::fail(LZ_E_INVAL, "batch %u exceeds the allocation-free maximum of %u rows", batch, kNoAllocMaxBatch);
  float* work = nullptr;
  const int rc = scratch_for_current_device(&work);
  if (rc) return rc;
  if (batch == 0) return 0;
  return backward(d_params, batch, d_x, d_h1, d_h2, d_logits, d_labels, d_grads, work, d_loss, (hipStream_t)stream);
}

// Device workspace of lz_selector_train: parameters, gradients and the two
// Adam moments, the (shuffled, normalised) training rows and labels, and one
// batch of activations, work buffer and loss; regions 256-byte aligned.
static uint64_t train_layout(uint64_t n_rows, uint32_t batch, uint64_t off[11]) {
  auto a256 = [](uint64_t x) { return (x + 255) & ~uint64_t(255); };
  const uint64_t sizes[11] = {4 * NP, 4 * NP, 4 * NP, 4 * NP, 4 * n_rows * IN, 4 * n_rows, 4ull * batch * H,
                              4ull * batch * H, 4ull * batch * OUT, 4ull * batch * (OUT + 2 * H), 4};
  uint64_t o = 0;
  for (int i = 0; i < 11; ++i) {
    off[i] = o;
    o += a256(sizes[i]);
  }
  return o;
}

int lz_selector_train_bytes(uint64_t n_rows, uint32_t batch, uint64_t* bytes) {
  if (!bytes || batch == 0) return lz::fail(LZ_E_INVAL, "bad argument");
  uint64_t off[11];
  *bytes = train_layout(n_rows, batch, off);
  return 0;
}

// Mini-batch training of the selector's network with the kernels above:
// per epoch a seeded permutation of the rows (features normalised with the
// selector's mu / sd), then per batch forward, backward and one Adam step.
// loss_hist[e] (may be null) receives epoch e's mean loss.  Synchronises
// `stream` once per epoch (to read the loss) and at the end.
int lz_selector_train(lz_selector* sel, const float* feats, const int32_t* labels, uint64_t n_rows, uint32_t epochs,
                      uint32_t batch, float lr, uint64_t seed, void* d_work, uint64_t work_bytes, float* loss_hist,
                      void* stream) {
  if (!sel || (n_rows && (!feats || !labels)) || !d_work || batch == 0) return lz::fail(LZ_E_INVAL, "bad argument");
  if ((uintptr_t)d_work & 255u) return lz::fail(LZ_E_INVAL, "d_work must be 256-byte aligned");
  for (uint64_t r = 0; r < n_rows; ++r)
    if (labels[r] < 0 || labels[r] >= OUT) return lz::fail(LZ_E_INVAL, "label %d of row %llu out of range",
                                                           labels[r], (unsigned long long)r);
  uint64_t off[11];
  if (work_bytes < train_layout(n_rows, batch, off)) return lz::fail(LZ_E_NOMEM, "training workspace too small");
  if (n_rows == 0) return 0;
  hipStream_t s = (hipStream_t)stream;
  uint8_t* W = (uint8_t*)d_work;
  float* P = (float*)(W + off[0]);
  float* G = (float*)(W + off[1]);
  float* M = (float*)(W + off[2]);
  float* V = (float*)(W + off[3]);
  float* X = (float*)(W + off[4]);
  int32_t* Y = (int32_t*)(W + off[5]);
  float* h1 = (float*)(W + off[6]);
  float* h2 = (float*)(W + off[7]);
  float* lg = (float*)(W + off[8]);
  float* work = (float*)(W + off[9]);
  float* loss = (float*)(W + off[10]);
  std::vector<float> zeros(NP, 0.f), hx(n_rows * IN);
  std::vector<int32_t> hy(n_rows);
  std::vector<uint64_t> perm(n_rows);
  if (hipMemcpyAsync(P, sel->params.data(), 4 * NP, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(M, zeros.data(), 4 * NP, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(V, zeros.data(), 4 * NP, hipMemcpyHostToDevice, s) != hipSuccess)
    return lz::fail(LZ_E_HIP, "parameter upload failed");
  uint64_t st = seed;
  uint32_t step = 0;
  for (uint32_t ep = 0; ep < epochs; ++ep) {
    // Fisher-Yates over SplitMix64 draws
    for (uint64_t r = 0; r < n_rows; ++r) perm[r] = r;
    for (uint64_t r = n_rows - 1; r > 0; --r) {
      st += 0x9E3779B97F4A7C15ull;
      uint64_t z = st;
      z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
      z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
      z ^= z >> 31;
      std::swap(perm[r], perm[z % (r + 1)]);
    }
    for (uint64_t r = 0; r < n_rows; ++r) {
      const float* f = feats + perm[r] * IN;
      for (int i = 0; i < IN; ++i) hx[r * IN + i] = (f[i] - sel->mu[i]) / sel->sd[i];
      hy[r] = labels[perm[r]];
    }
    const float zero = 0.f;
    float ep_loss = 0.f;
    if (hipMemcpyAsync(X, hx.data(), 4 * n_rows * IN, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(Y, hy.data(), 4 * n_rows, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(loss, &zero, 4, hipMemcpyHostToDevice, s) != hipSuccess)
      return lz::fail(LZ_E_HIP, "training rows upload failed");
    uint64_t nb = 0;
    for (uint64_t r0 = 0; r0 < n_rows; r0 += batch, ++nb) {
      const uint32_t B = (uint32_t)std::min<uint64_t>(batch, n_rows - r0);
      int rc = lz_mlp_forward(P, B, X + r0 * IN, h1, h2, lg, stream);
      if (!rc) rc = backward(P, B, X + r0 * IN, h1, h2, lg, Y + r0, G, work, loss, s);
      if (!rc) rc = lz_mlp_adam(P, G, M, V, NP, lr, 0.9f, 0.999f, 1e-8f, ++step, stream);
      if (rc) return rc;
    }
    if (hipMemcpyAsync(&ep_loss, loss, 4, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
      return lz::fail(LZ_E_HIP, "training epoch %u failed", ep);
    if (loss_hist) loss_hist[ep] = ep_loss / (float)nb;
  }
  if (hipMemcpyAsync(sel->params.data(), P, 4 * NP, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return lz::fail(LZ_E_HIP, "parameter download failed");
  return 0;
}

// One Adam step (Kingma & Ba), bias-corrected; `step` counts from 1.
int lz_mlp_adam(float* d_params, const float* d_grads, float* d_m, float* d_v, uint64_t n, float lr, float beta1,
                float beta2, float eps, uint32_t step, void* stream) {
  if (!d_params || !d_grads || !d_m || !d_v || step == 0) return lz::fail(LZ_E_INVAL, "bad argument");
  const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, n, d_params,
                     d_grads, d_m, d_v, lr, beta1, beta2, eps, c1, c2);
  if (hipGetLastError() != hipSuccess) return lz::fail(LZ_E_HIP, "adam launch failed");
  return 0;
}

}  // extern "C"
