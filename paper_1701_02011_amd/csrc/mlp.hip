// The learned part: a small network that predicts the core-pair parts of E(3) from pair
// quantities of first order, trained and evaluated by the kernels below (no library).
//
// Network: 16 -> 128 -> 128 -> 128 -> 1, exact-erf GELU after each hidden layer, linear
// output.  The products use BF16-rounded weights (round to nearest even) with FP32
// activations and FP32 sums; training keeps an FP32 master copy of the weights and updates
// it by Adam on the mean squared error of standardised targets (full batch, so every run
// with the same inputs and seed gives the same weights).  Features and targets are
// standardised with the training set's mean and standard deviation, which travel in the
// weights blob.
#include "../../include/dsrg.h"
#include "../../include/dsrg_testing.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

namespace dsrg {
void set_last_error(const char* m);   // the library's message of the last failing call
}

namespace dsrg_mlp {

constexpr int kIn = DSRG_MLP_FEATURES, kHid = 128, kLayers = 4;
constexpr int kDin[kLayers] = {kIn, kHid, kHid, kHid};
constexpr int kDout[kLayers] = {kHid, kHid, kHid, 1};
constexpr int kHeader = 64;   // floats before the parameters
// parameter offsets (floats, from the start of the parameters): W_l [dout][din], then b_l
constexpr int woff(int l) {
  int o = 0;
  for (int k = 0; k < l; ++k) o += kDout[k] * kDin[k] + kDout[k];
  return o;
}
constexpr int boff(int l) { return woff(l) + kDout[l] * kDin[l]; }
constexpr int kParams = woff(kLayers);
static_assert((kHeader + kParams) * 4 == DSRG_MLP_WEIGHTS_BYTES, "weights blob size");
constexpr uint32_t kMagic = 0x4d4c5031u;   // "MLP1"

struct Err : std::runtime_error {
  int code;
  Err(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};
#define MCHECK(x)                                                                            \
  do {                                                                                       \
    hipError_t e_ = (x);                                                                     \
    if (e_ != hipSuccess) {                                                                  \
      (void)hipGetLastError();                                                               \
      throw Err(e_ == hipErrorOutOfMemory ? DSRG_E_OOM : DSRG_E_HIP,                         \
                std::string(#x) + ": " + hipGetErrorString(e_));                            \
    }                                                                                        \
  } while (0)

__host__ __device__ inline float bf16_round(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  u = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
  float r;
  memcpy(&r, &u, 4);
  return r;
}

__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// z[r][o] = b[o] + sum_i bf16(W[o][i]) x[r][i]; a = gelu(z) (hidden) or z (output).  The
// first layer standardises its inputs on the fly (x - mean) / std.
__global__ __launch_bounds__(256) void dense_fwd_kernel(const float* __restrict__ in, int din, int dout, long long n,
                                                        const float* __restrict__ W, const float* __restrict__ b,
                                                        const float* __restrict__ mean, const float* __restrict__ sd,
                                                        float* __restrict__ z, float* __restrict__ a, int act) {
  const long long t = blockIdx.x * 256LL + threadIdx.x;
  if (t >= n * dout) return;
  const long long r = t / dout;
  const int o = (int)(t - r * dout);
  const float* x = in + r * din;
  const float* w = W + (long long)o * din;
  float acc = b[o];
  for (int i = 0; i < din; ++i) {
    float xi = x[i];
    if (mean) xi = (xi - mean[i]) / sd[i];
    acc += bf16_round(w[i]) * xi;
  }
  z[t] = acc;
  a[t] = act ? gelu(acc) : acc;
}

// MSE of standardised targets: d[r] = 2 (out[r] - ys[r]) / n, partial sums of squares per
// workgroup (summed in a fixed order on the host)
__global__ __launch_bounds__(256) void loss_kernel(const float* __restrict__ out, const float* __restrict__ ys,
                                                   long long n, float* __restrict__ d, double* __restrict__ part) {
  __shared__ double sh[256];
  const long long r = blockIdx.x * 256LL + threadIdx.x;
  double e2 = 0.0;
  if (r < n) {
    const float e = out[r] - ys[r];
    d[r] = 2.0f * e / (float)n;
    e2 = (double)e * e;
  }
  sh[threadIdx.x] = e2;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// dz = da * gelu'(z) (hidden layers)
__global__ __launch_bounds__(256) void gelu_bwd_kernel(const float* __restrict__ z, float* __restrict__ da, long long m) {
  const long long t = blockIdx.x * 256LL + threadIdx.x;
  if (t < m) da[t] *= gelu_grad(z[t]);
}

// da_in[r][i] = sum_o dz[r][o] bf16(W[o][i])
__global__ __launch_bounds__(256) void dense_bwd_input_kernel(const float* __restrict__ dz, int din, int dout, long long n,
                                                              const float* __restrict__ W, float* __restrict__ da_in) {
  const long long t = blockIdx.x * 256LL + threadIdx.x;
  if (t >= n * din) return;
  const long long r = t / din;
  const int i = (int)(t - r * din);
  float acc = 0.f;
  for (int o = 0; o < dout; ++o) acc += dz[r * dout + o] * bf16_round(W[(long long)o * din + i]);
  da_in[t] = acc;
}

// gW[o][i] = sum_r dz[r][o] x[r][i] (x standardised for the first layer), gb[o] = sum_r dz[r][o];
// thread (o, i) with i == din for the bias; rows summed in order
__global__ __launch_bounds__(256) void dense_bwd_weight_kernel(const float* __restrict__ dz, const float* __restrict__ in,
                                                               int din, int dout, long long n,
                                                               const float* __restrict__ mean, const float* __restrict__ sd,
                                                               float* __restrict__ gW, float* __restrict__ gb) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= dout * (din + 1)) return;
  const int o = t / (din + 1), i = t - o * (din + 1);
  float acc = 0.f;
  if (i == din) {
    for (long long r = 0; r < n; ++r) acc += dz[r * dout + o];
    gb[o] = acc;
    return;
  }
  for (long long r = 0; r < n; ++r) {
    float xi = in[r * din + i];
    if (mean) xi = (xi - mean[i]) / sd[i];
    acc += dz[r * dout + o] * xi;
  }
  gW[(long long)o * din + i] = acc;
}

// Adam on the FP32 master parameters (bias-corrected moments)
__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ w, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v, int np, float lr,
                                                   float b1, float b2, float eps, float c1, float c2) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= np) return;
  const float gt = g[t];
  const float mt = b1 * m[t] + (1.f - b1) * gt;
  const float vt = b2 * v[t] + (1.f - b2) * gt * gt;
  m[t] = mt;
  v[t] = vt;
  w[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + eps);
}

static unsigned blocks(long long n) { return (unsigned)((n + 255) / 256); }

// Device buffers of one network evaluation over n rows.
struct Net {
  long long n = 0;
  float *x = nullptr, *ys = nullptr, *p = nullptr, *g = nullptr, *mean = nullptr, *sd = nullptr;
  float *z[kLayers] = {}, *a[kLayers] = {}, *d = nullptr, *d2 = nullptr;
  double* part = nullptr;
  std::vector<void*> owned;
  template <class T>
  T* alloc(size_t count) {
    void* q = nullptr;
    MCHECK(hipMalloc(&q, count * sizeof(T) + 16));
    owned.push_back(q);
    return (T*)q;
  }
  explicit Net(long long n_) : n(n_) {
    x = alloc<float>((size_t)n * kIn);
    ys = alloc<float>((size_t)n);
    p = alloc<float>(kParams);
    g = alloc<float>(kParams);
    mean = alloc<float>(kIn);
    sd = alloc<float>(kIn);
    for (int l = 0; l < kLayers; ++l) {
      z[l] = alloc<float>((size_t)n * kDout[l]);
      a[l] = alloc<float>((size_t)n * kDout[l]);
    }
    d = alloc<float>((size_t)n * kHid);
    d2 = alloc<float>((size_t)n * kHid);
    part = alloc<double>((size_t)blocks(n));
  }
  ~Net() {
    for (void* q : owned) (void)hipFree(q);
  }
  void forward(hipStream_t st) {
    const float* in = x;
    for (int l = 0; l < kLayers; ++l) {
      const bool first = l == 0;
      hipLaunchKernelGGL(dense_fwd_kernel, dim3(blocks(n * kDout[l])), dim3(256), 0, st, in, kDin[l], kDout[l], n,
                         p + woff(l), p + boff(l), first ? mean : nullptr, first ? sd : nullptr, z[l], a[l],
                         l + 1 < kLayers ? 1 : 0);
      in = a[l];
    }
  }
  // loss (mean square over rows) and the gradient of every parameter into g
  double backward(hipStream_t st) {
    const long long nb = blocks(n);
    hipLaunchKernelGGL(loss_kernel, dim3((unsigned)nb), dim3(256), 0, st, a[kLayers - 1], ys, n, d, part);
    float* dz = d;   // [n][dout] of the current layer
    float* spare = d2;
    for (int l = kLayers - 1; l >= 0; --l) {
      const float* in = l ? a[l - 1] : x;
      const bool first = l == 0;
      const int nt = kDout[l] * (kDin[l] + 1);
      hipLaunchKernelGGL(dense_bwd_weight_kernel, dim3(blocks(nt)), dim3(256), 0, st, dz, in, kDin[l], kDout[l], n,
                         first ? mean : nullptr, first ? sd : nullptr, g + woff(l), g + boff(l));
      if (l == 0) break;
      hipLaunchKernelGGL(dense_bwd_input_kernel, dim3(blocks(n * kDin[l])), dim3(256), 0, st, dz, kDin[l], kDout[l], n,
                         p + woff(l), spare);
      hipLaunchKernelGGL(gelu_bwd_kernel, dim3(blocks(n * kDin[l])), dim3(256), 0, st, z[l - 1], spare, n * kDin[l]);
      std::swap(dz, spare);
    }
    MCHECK(hipGetLastError());
    std::vector<double> h((size_t)nb);
    MCHECK(hipMemcpyAsync(h.data(), part, nb * sizeof(double), hipMemcpyDeviceToHost, st));
    MCHECK(hipStreamSynchronize(st));
    double s = 0.0;
    for (double v : h) s += v;
    return s / (double)n;
  }
};

// standardisation of the columns of X (n x kIn) and of y: mean and population standard
// deviation (1 where a column is constant)
static void fit_scaling(const float* X, const double* y, long long n, float* mean, float* sd, double& ym, double& ys) {
  for (int i = 0; i < kIn; ++i) {
    double s = 0, s2 = 0;
    for (long long r = 0; r < n; ++r) s += X[r * kIn + i];
    const double m = s / n;
    for (long long r = 0; r < n; ++r) s2 += (X[r * kIn + i] - m) * (X[r * kIn + i] - m);
    const double v = std::sqrt(s2 / n);
    mean[i] = (float)m;
    sd[i] = v > 0 ? (float)v : 1.0f;
  }
  double s = 0, s2 = 0;
  for (long long r = 0; r < n; ++r) s += y[r];
  ym = s / n;
  for (long long r = 0; r < n; ++r) s2 += (y[r] - ym) * (y[r] - ym);
  ys = std::sqrt(s2 / n);
  if (!(ys > 0)) ys = 1.0;
}

// counter-based uniform numbers in [-1, 1): splitmix64 of (seed, index)
static double uniform_pm1(uint64_t seed, uint64_t k) {
  uint64_t z = seed + 0x9e3779b97f4a7c15ull * (k + 1);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

static void check_blob(const float* w) {
  uint32_t magic;
  memcpy(&magic, w, 4);
  if (magic != kMagic) throw Err(DSRG_E_ARG, "not a weights blob of this network");
  for (int k = 0; k < kHeader + kParams; ++k)
    if (!std::isfinite(w[k])) throw Err(DSRG_E_NONFINITE, "non-finite value in the weights");
}

static void upload(Net& net, const float* blob, const float* X, const double* y, hipStream_t st) {
  const float* head = blob;
  MCHECK(hipMemcpyAsync(net.p, blob + kHeader, kParams * sizeof(float), hipMemcpyHostToDevice, st));
  MCHECK(hipMemcpyAsync(net.mean, head + 8, kIn * sizeof(float), hipMemcpyHostToDevice, st));
  MCHECK(hipMemcpyAsync(net.sd, head + 24, kIn * sizeof(float), hipMemcpyHostToDevice, st));
  MCHECK(hipMemcpyAsync(net.x, X, (size_t)net.n * kIn * sizeof(float), hipMemcpyHostToDevice, st));
  if (y) {
    std::vector<float> ys((size_t)net.n);
    for (long long r = 0; r < net.n; ++r) ys[r] = (float)((y[r] - head[40]) / head[41]);
    MCHECK(hipMemcpyAsync(net.ys, ys.data(), net.n * sizeof(float), hipMemcpyHostToDevice, st));
    MCHECK(hipStreamSynchronize(st));   // ys is a host temporary
  }
}

static void check_rows(const float* X, long long n) {
  for (long long k = 0; k < n * kIn; ++k)
    if (!std::isfinite(X[k])) throw Err(DSRG_E_NONFINITE, "non-finite feature");
}

template <class F>
static int guarded(F&& f) {
  try {
    const int rc = f();
    dsrg::set_last_error("");
    return rc;
  } catch (const Err& e) {
    dsrg::set_last_error(e.what());
    return e.code;
  } catch (const std::exception& e) {
    dsrg::set_last_error(e.what());
    return DSRG_E_HIP;
  }
}

}  // namespace dsrg_mlp

using namespace dsrg_mlp;

extern "C" int dsrg_mlp_train(const float* X, const double* y, int64_t n, int32_t epochs, uint64_t seed,
                              void* weights_out) {
  return guarded([&] {
    if (!X || !y || !weights_out || n < 2 || epochs < 0) throw Err(DSRG_E_ARG, "null array, n < 2 or epochs < 0");
    check_rows(X, n);
    for (long long r = 0; r < n; ++r)
      if (!std::isfinite(y[r])) throw Err(DSRG_E_NONFINITE, "non-finite target");
    std::vector<float> blob((size_t)(kHeader + kParams), 0.f);
    const uint32_t head[8] = {kMagic, 1u, (uint32_t)kIn, (uint32_t)kHid, (uint32_t)(kLayers - 1), (uint32_t)epochs, 0, 0};
    memcpy(blob.data(), head, sizeof(head));
    double ym, ys;
    fit_scaling(X, y, n, blob.data() + 8, blob.data() + 24, ym, ys);
    blob[40] = (float)ym;
    blob[41] = (float)ys;
    // uniform initialisation in +-1/sqrt(fan_in), biases zero
    for (int l = 0; l < kLayers; ++l) {
      const double lim = 1.0 / std::sqrt((double)kDin[l]);
      for (int k = 0; k < kDout[l] * kDin[l]; ++k)
        blob[kHeader + woff(l) + k] = (float)(lim * uniform_pm1(seed, (uint64_t)(woff(l) + k)));
    }
    hipStream_t st = nullptr;
    Net net(n);
    upload(net, blob.data(), X, y, st);
    float *m = net.alloc<float>(kParams), *v = net.alloc<float>(kParams);
    MCHECK(hipMemsetAsync(m, 0, kParams * sizeof(float), st));
    MCHECK(hipMemsetAsync(v, 0, kParams * sizeof(float), st));
    const float lr = 1e-3f, b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    double c1 = 1, c2 = 1;
    for (int e = 0; e < epochs; ++e) {
      net.forward(st);
      net.backward(st);
      c1 *= b1;
      c2 *= b2;
      hipLaunchKernelGGL(adam_kernel, dim3(blocks(kParams)), dim3(256), 0, st, net.p, net.g, m, v, kParams, lr, b1,
                         b2, eps, (float)(1.0 - c1), (float)(1.0 - c2));
    }
    MCHECK(hipMemcpyAsync(blob.data() + kHeader, net.p, kParams * sizeof(float), hipMemcpyDeviceToHost, st));
    MCHECK(hipStreamSynchronize(st));
    MCHECK(hipGetLastError());
    memcpy(weights_out, blob.data(), blob.size() * sizeof(float));
    return DSRG_OK;
  });
}

extern "C" int dsrg_mlp_predict(const void* weights, const float* X, int64_t n, double* y_out) {
  return guarded([&] {
    if (!weights || !X || !y_out || n < 0) throw Err(DSRG_E_ARG, "null array or n < 0");
    if (n == 0) return DSRG_OK;
    const float* blob = (const float*)weights;
    check_blob(blob);
    check_rows(X, n);
    hipStream_t st = nullptr;
    Net net(n);
    upload(net, blob, X, nullptr, st);
    net.forward(st);
    std::vector<float> out((size_t)n);
    MCHECK(hipMemcpyAsync(out.data(), net.a[kLayers - 1], n * sizeof(float), hipMemcpyDeviceToHost, st));
    MCHECK(hipStreamSynchronize(st));
    MCHECK(hipGetLastError());
    for (long long r = 0; r < n; ++r) y_out[r] = (double)out[r] * blob[41] + blob[40];
    return DSRG_OK;
  });
}

extern "C" int dsrg_test_mlp_grad(const void* weights, const float* X, const double* y, int64_t n, double* loss,
                                  float* grad) {
  return guarded([&] {
    if (!weights || !X || !y || !loss || !grad || n < 1) throw Err(DSRG_E_ARG, "null array or n < 1");
    const float* blob = (const float*)weights;
    check_blob(blob);
    check_rows(X, n);
    hipStream_t st = nullptr;
    Net net(n);
    upload(net, blob, X, y, st);
    net.forward(st);
    *loss = net.backward(st);
    MCHECK(hipMemcpyAsync(grad, net.g, kParams * sizeof(float), hipMemcpyDeviceToHost, st));
    MCHECK(hipStreamSynchronize(st));
    return DSRG_OK;
  });
}
