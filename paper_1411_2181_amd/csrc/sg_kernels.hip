// Surrogate network kernels (forward, backward, Adam) and their C ABI.
//
// The network (6 -> 128 -> 128 -> 3, tanh) runs with bfloat16 parameters and
// float32 accumulation.  Every reduction (over hidden units in the forward
// pass, over rows in the parameter gradient and the loss) is a fixed-order
// loop, so results are bit-reproducible.  Sizes are tiny next to a lattice
// step (a few thousand rows), so the kernels favour simplicity: one thread
// per hidden unit and row tile in the forward pass, one thread per parameter
// for the gradient.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/lbmve.h"
#include "../../include/lbmve_surrogate.h"

namespace {

constexpr int NI = 6, NH = 128, NO = 3;
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + NI * NH;
constexpr int OFF_W2 = OFF_B1 + NH;
constexpr int OFF_B2 = OFF_W2 + NH * NH;
constexpr int OFF_W3 = OFF_B2 + NH;
constexpr int OFF_B3 = OFF_W3 + NH * NO;
constexpr int NP = OFF_B3 + NO;
constexpr int ROWS = 16;   // rows per forward workgroup

// float -> bfloat16 bits, round to nearest even (NaN kept quiet)
__host__ __device__ inline uint16_t f2bf(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf2f(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

__global__ void k_refresh(const float* __restrict__ P, uint16_t* __restrict__ Wb, int np) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < np) Wb[i] = f2bf(P[i]);
}

// Forward pass of ROWS rows per workgroup of NH threads (thread j = unit j).
__global__ void __launch_bounds__(NH) k_forward(const float* __restrict__ x, int n,
                                                const uint16_t* __restrict__ Wb,
                                                float* __restrict__ z, float* __restrict__ h1g,
                                                float* __restrict__ h2g) {
  __shared__ float xs[ROWS][NI];
  __shared__ float h1s[ROWS][NH];
  __shared__ float h2s[ROWS][NH];
  const int j = threadIdx.x;
  const int r0 = blockIdx.x * ROWS;
  for (int k = j; k < ROWS * NI; k += NH) {
    const int r = r0 + k / NI;
    xs[k / NI][k % NI] = r < n ? x[(size_t)r * NI + k % NI] : 0.f;
  }
  __syncthreads();
  {
    const float b = bf2f(Wb[OFF_B1 + j]);
    float w[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) w[k] = bf2f(Wb[OFF_W1 + k * NH + j]);
    for (int r = 0; r < ROWS; ++r) {
      float acc = b;
#pragma unroll
      for (int k = 0; k < NI; ++k) acc += xs[r][k] * w[k];
      const float h = tanhf(acc);
      h1s[r][j] = h;
      if (h1g && r0 + r < n) h1g[(size_t)(r0 + r) * NH + j] = h;
    }
  }
  __syncthreads();
  {
    float acc[ROWS];
    const float b = bf2f(Wb[OFF_B2 + j]);
#pragma unroll
    for (int r = 0; r < ROWS; ++r) acc[r] = b;
    for (int k = 0; k < NH; ++k) {
      const float w = bf2f(Wb[OFF_W2 + k * NH + j]);
#pragma unroll
      for (int r = 0; r < ROWS; ++r) acc[r] += h1s[r][k] * w;
    }
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      const float h = tanhf(acc[r]);
      h2s[r][j] = h;
      if (h2g && r0 + r < n) h2g[(size_t)(r0 + r) * NH + j] = h;
    }
  }
  __syncthreads();
  if (j < ROWS * NO) {
    const int r = j / NO, o = j % NO;
    if (r0 + r < n) {
      float acc = bf2f(Wb[OFF_B3 + o]);
      for (int k = 0; k < NH; ++k) acc += h2s[r][k] * bf2f(Wb[OFF_W3 + k * NO + o]);
      z[(size_t)(r0 + r) * NO + o] = acc;
    }
  }
}

// Output deltas d = dL/dz (scaled by 1/n) and the per-row loss.
__global__ void k_delta(const float* __restrict__ z, const float* __restrict__ t,
                        const float* __restrict__ m, int n, float* __restrict__ d,
                        float* __restrict__ rowloss) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const float inv = 1.0f / (float)n;
  const float mk = m[r];
  const float e0 = z[r * NO] - t[r * NO], e1 = z[r * NO + 1] - t[r * NO + 1];
  const float z2 = z[r * NO + 2], t2 = t[r * NO + 2];
  d[r * NO] = mk * e0 * inv;
  d[r * NO + 1] = mk * e1 * inv;
  d[r * NO + 2] = (1.0f / (1.0f + expf(-z2)) - t2) * inv;
  const float sp = fmaxf(z2, 0.f) + log1pf(expf(-fabsf(z2)));
  rowloss[r] = 0.5f * mk * (e0 * e0 + e1 * e1) + sp - t2 * z2;
}

// dz2[r][j] = (sum_o d[r][o] W3[j][o]) (1 - h2[r][j]^2)
__global__ void k_back2(const float* __restrict__ d, const float* __restrict__ h2,
                        const uint16_t* __restrict__ Wb, int n, float* __restrict__ dz2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n * NH) return;
  const int r = (int)(i / NH), j = (int)(i % NH);
  float acc = 0.f;
#pragma unroll
  for (int o = 0; o < NO; ++o) acc += d[r * NO + o] * bf2f(Wb[OFF_W3 + j * NO + o]);
  const float h = h2[i];
  dz2[i] = acc * (1.f - h * h);
}

// dz1[r][k] = (sum_j dz2[r][j] W2[k][j]) (1 - h1[r][k]^2)
__global__ void k_back1(const float* __restrict__ dz2, const float* __restrict__ h1,
                        const uint16_t* __restrict__ Wb, int n, float* __restrict__ dz1) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n * NH) return;
  const int r = (int)(i / NH), k = (int)(i % NH);
  float acc = 0.f;
  for (int j = 0; j < NH; ++j) acc += dz2[(size_t)r * NH + j] * bf2f(Wb[OFF_W2 + k * NH + j]);
  const float h = h1[i];
  dz1[i] = acc * (1.f - h * h);
}

// One thread per parameter: sum over rows of (layer input) x (unit delta).
__global__ void k_wgrad(const float* __restrict__ x, const float* __restrict__ h1,
                        const float* __restrict__ h2, const float* __restrict__ d,
                        const float* __restrict__ dz1, const float* __restrict__ dz2, int n,
                        float* __restrict__ G) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NP) return;
  float acc = 0.f;
  if (p < OFF_B1) {
    const int k = p / NH, j = p % NH;
    for (int r = 0; r < n; ++r) acc += x[(size_t)r * NI + k] * dz1[(size_t)r * NH + j];
  } else if (p < OFF_W2) {
    const int j = p - OFF_B1;
    for (int r = 0; r < n; ++r) acc += dz1[(size_t)r * NH + j];
  } else if (p < OFF_B2) {
    const int k = (p - OFF_W2) / NH, j = (p - OFF_W2) % NH;
    for (int r = 0; r < n; ++r) acc += h1[(size_t)r * NH + k] * dz2[(size_t)r * NH + j];
  } else if (p < OFF_W3) {
    const int j = p - OFF_B2;
    for (int r = 0; r < n; ++r) acc += dz2[(size_t)r * NH + j];
  } else if (p < OFF_B3) {
    const int k = (p - OFF_W3) / NO, o = (p - OFF_W3) % NO;
    for (int r = 0; r < n; ++r) acc += h2[(size_t)r * NH + k] * d[(size_t)r * NO + o];
  } else {
    const int o = p - OFF_B3;
    for (int r = 0; r < n; ++r) acc += d[(size_t)r * NO + o];
  }
  G[p] = acc;
}

// Sum of the per-row losses in a fixed order (one workgroup).
__global__ void k_loss(const float* __restrict__ rowloss, int n, float* __restrict__ out) {
  __shared__ float part[256];
  float acc = 0.f;
  for (int r = threadIdx.x; r < n; r += blockDim.x) acc += rowloss[r];
  part[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int i = 0; i < (int)blockDim.x; ++i) s += part[i];
    out[0] = s / (float)n;
  }
}

__global__ void k_adam(float* __restrict__ P, const float* __restrict__ G, float* __restrict__ M,
                       float* __restrict__ V, uint16_t* __restrict__ Wb, int np, float lr,
                       float bc1, float bc2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const float g = G[i];
  const float m = 0.9f * M[i] + 0.1f * g;
  const float v = 0.999f * V[i] + 0.001f * g * g;
  M[i] = m;
  V[i] = v;
  const float p = P[i] - lr * (m / bc1) / (sqrtf(v / bc2) + 1e-8f);
  P[i] = p;
  Wb[i] = f2bf(p);
}

size_t al(size_t v) { return (v + 255) / 256 * 256; }

struct Lay {
  size_t P, Wb, M, V, G, h1, h2, z, d, dz1, dz2, rowloss, loss, total;
};

Lay layout(int bmax) {
  Lay L{};
  size_t o = 0;
  auto take = [&](size_t b) { const size_t r = o; o = al(o + b); return r; };
  L.P = take(NP * 4);
  L.Wb = take(NP * 2);
  L.M = take(NP * 4);
  L.V = take(NP * 4);
  L.G = take(NP * 4);
  L.h1 = take((size_t)bmax * NH * 4);
  L.h2 = take((size_t)bmax * NH * 4);
  L.z = take((size_t)bmax * NO * 4);
  L.d = take((size_t)bmax * NO * 4);
  L.dz1 = take((size_t)bmax * NH * 4);
  L.dz2 = take((size_t)bmax * NH * 4);
  L.rowloss = take((size_t)bmax * 4);
  L.loss = take(4);
  L.total = o;
  return L;
}

// ---- scratch of the allocation-free gradient --------------------------------------
// Per-row activations, deltas and losses of up to SG_NOALLOC_MAX_ROWS rows in
// one file-scope device array: every GPU the library runs on holds its own
// copy until the process ends.  In host code the array's name is only a
// host-side stand-in: the device address is what hipGetSymbolAddress returns
// with that device current, resolved once per device and kept below.
constexpr size_t SC_H = (size_t)SG_NOALLOC_MAX_ROWS * NH;   // h1, h2, dz1, dz2
constexpr size_t SC_O = (size_t)SG_NOALLOC_MAX_ROWS * NO;   // z, d
constexpr size_t SC_FLOATS = 4 * SC_H + 2 * SC_O + SG_NOALLOC_MAX_ROWS;
static __device__ __align__(256) float scratch[SC_FLOATS];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
float* scratch_dev[MAX_DEVICES] = {};

// Device address of the scratch array on the current device (nullptr if it
// cannot be resolved).
float* scratch_of_current_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    scratch_dev[dev] = static_cast<float*>(p);
  }
  return scratch_dev[dev];
}

// Buffers of one backward pass.
struct Bufs {
  float *h1, *h2, *z, *d, *dz1, *dz2, *rowloss, *G, *loss;
};

}  // namespace

struct sg_ctx {
  int bmax = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  float* scratch = nullptr;   // this device's scratch array (allocation-free gradient)
  Lay L{};
  int step = 0;
  template <typename P>
  P* at(size_t o) const { return reinterpret_cast<P*>(ws + o); }
};

namespace {

Bufs workspace_bufs(const sg_ctx* s) {
  return Bufs{s->at<float>(s->L.h1), s->at<float>(s->L.h2), s->at<float>(s->L.z),
              s->at<float>(s->L.d), s->at<float>(s->L.dz1), s->at<float>(s->L.dz2),
              s->at<float>(s->L.rowloss), s->at<float>(s->L.G), s->at<float>(s->L.loss)};
}

int backward(sg_ctx* s, const float* x, const float* t, const float* m, int n, const Bufs& b) {
  hipStream_t st = s->stream;
  const uint16_t* Wb = s->at<uint16_t>(s->L.Wb);
  k_forward<<<(n + ROWS - 1) / ROWS, NH, 0, st>>>(x, n, Wb, b.z, b.h1, b.h2);
  k_delta<<<(n + 255) / 256, 256, 0, st>>>(b.z, t, m, n, b.d, b.rowloss);
  const int64_t nh = (int64_t)n * NH;
  k_back2<<<(unsigned)((nh + 255) / 256), 256, 0, st>>>(b.d, b.h2, Wb, n, b.dz2);
  k_back1<<<(unsigned)((nh + 255) / 256), 256, 0, st>>>(b.dz2, b.h1, Wb, n, b.dz1);
  k_wgrad<<<(NP + 255) / 256, 256, 0, st>>>(x, b.h1, b.h2, b.d, b.dz1, b.dz2, n, b.G);
  k_loss<<<1, 256, 0, st>>>(b.rowloss, n, b.loss);
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EHIP;
}

}  // namespace

extern "C" {

int32_t sg_param_count(void) { return NP; }

int sg_workspace_bytes(int32_t bmax, size_t* bytes) {
  if (!bytes || bmax < 1 || bmax > (1 << 24)) return LBM_EINVAL;
  *bytes = layout(bmax).total;
  return LBM_OK;
}

int sg_init(int32_t bmax, void* ws, size_t bytes, void* stream, sg_ctx** out) {
  if (!out || !ws || bmax < 1 || bmax > (1 << 24)) return LBM_EINVAL;
  *out = nullptr;
  const Lay L = layout(bmax);
  if (bytes < L.total) return LBM_ENOMEM;
  sg_ctx* s = new (std::nothrow) sg_ctx();
  if (!s) return LBM_EINVAL;
  s->bmax = bmax;
  s->stream = (hipStream_t)stream;
  s->ws = (char*)ws;
  s->L = L;
  // the scratch array of the device this context runs on (current now)
  s->scratch = scratch_of_current_device();
  if (!s->scratch) {
    delete s;
    return LBM_EHIP;
  }
  *out = s;
  return LBM_OK;
}

int sg_set_params(sg_ctx* s, const float* host, size_t n) {
  if (!s || !host || n != (size_t)NP) return LBM_EINVAL;
  if (hipStreamSynchronize(s->stream) != hipSuccess) return LBM_EHIP;
  std::vector<float> zero(NP, 0.f);
  if (hipMemcpy(s->at<float>(s->L.P), host, NP * 4, hipMemcpyHostToDevice) ||
      hipMemcpy(s->at<float>(s->L.M), zero.data(), NP * 4, hipMemcpyHostToDevice) ||
      hipMemcpy(s->at<float>(s->L.V), zero.data(), NP * 4, hipMemcpyHostToDevice))
    return LBM_EHIP;
  k_refresh<<<(NP + 255) / 256, 256, 0, s->stream>>>(s->at<float>(s->L.P), s->at<uint16_t>(s->L.Wb), NP);
  s->step = 0;
  return hipStreamSynchronize(s->stream) == hipSuccess ? LBM_OK : LBM_EHIP;
}

int sg_get_params(sg_ctx* s, float* host, size_t n) {
  if (!s || !host || n != (size_t)NP) return LBM_EINVAL;
  if (hipStreamSynchronize(s->stream) != hipSuccess) return LBM_EHIP;
  return hipMemcpy(host, s->at<float>(s->L.P), NP * 4, hipMemcpyDeviceToHost) == hipSuccess ? LBM_OK
                                                                                              : LBM_EHIP;
}

int sg_get_working_params(sg_ctx* s, float* host, size_t n) {
  if (!s || !host || n != (size_t)NP) return LBM_EINVAL;
  if (hipStreamSynchronize(s->stream) != hipSuccess) return LBM_EHIP;
  std::vector<uint16_t> b(NP);
  if (hipMemcpy(b.data(), s->at<uint16_t>(s->L.Wb), NP * 2, hipMemcpyDeviceToHost) != hipSuccess)
    return LBM_EHIP;
  for (int i = 0; i < NP; ++i) host[i] = bf2f(b[i]);
  return LBM_OK;
}

int sg_forward(sg_ctx* s, const float* x, int32_t n, float* z) {
  if (!s || !x || !z || n < 1 || n > s->bmax) return LBM_EINVAL;
  k_forward<<<(n + ROWS - 1) / ROWS, NH, 0, s->stream>>>(x, n, s->at<uint16_t>(s->L.Wb), z, nullptr, nullptr);
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EHIP;
}

int sg_gradient(sg_ctx* s, const float* x, const float* t, const float* m, int32_t n, float* grad,
                float* loss) {
  if (!s || !x || !t || !m || !grad || !loss || n < 1 || n > s->bmax) return LBM_EINVAL;
  const int e = backward(s, x, t, m, n, workspace_bufs(s));
  if (e) return e;
  if (hipMemcpyAsync(grad, s->at<float>(s->L.G), NP * 4, hipMemcpyDeviceToHost, s->stream) ||
      hipMemcpyAsync(loss, s->at<float>(s->L.loss), 4, hipMemcpyDeviceToHost, s->stream) ||
      hipStreamSynchronize(s->stream))
    return LBM_EHIP;
  return LBM_OK;
}

int sg_train_step(sg_ctx* s, const float* x, const float* t, const float* m, int32_t n, float lr,
                  float* loss) {
  if (!s || !x || !t || !m || !loss || n < 1 || n > s->bmax || !(lr > 0.f)) return LBM_EINVAL;
  int e = backward(s, x, t, m, n, workspace_bufs(s));
  if (e) return e;
  s->step += 1;
  const float bc1 = 1.f - powf(0.9f, (float)s->step);
  const float bc2 = 1.f - powf(0.999f, (float)s->step);
  k_adam<<<(NP + 255) / 256, 256, 0, s->stream>>>(s->at<float>(s->L.P), s->at<float>(s->L.G),
                                                  s->at<float>(s->L.M), s->at<float>(s->L.V),
                                                  s->at<uint16_t>(s->L.Wb), NP, lr, bc1, bc2);
  if (hipGetLastError() != hipSuccess) return LBM_EHIP;
  if (hipMemcpyAsync(loss, s->at<float>(s->L.loss), 4, hipMemcpyDeviceToHost, s->stream) ||
      hipStreamSynchronize(s->stream))
    return LBM_EHIP;
  return LBM_OK;
}

int sg_gradient_noalloc(sg_ctx* s, const float* x, const float* t, const float* m, int32_t n,
                        float* grad_dev, float* loss_dev) {
  if (!s || !x || !t || !m || !grad_dev || !loss_dev || n < 1) return LBM_EINVAL;
  if (n > SG_NOALLOC_MAX_ROWS) return LBM_EINVAL;
  if (!s->scratch) return LBM_EHIP;
  float* p = s->scratch;
  const Bufs b{p, p + SC_H, p + 4 * SC_H, p + 4 * SC_H + SC_O, p + 2 * SC_H, p + 3 * SC_H,
               p + 4 * SC_H + 2 * SC_O, grad_dev, loss_dev};
  return backward(s, x, t, m, n, b);
}

void sg_destroy(sg_ctx* s) {
  if (!s) return;
  hipStreamSynchronize(s->stream);
  delete s;
}

}  // extern "C"
