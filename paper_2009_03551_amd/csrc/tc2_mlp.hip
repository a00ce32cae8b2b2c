// Block-skip network of the TC2 solver: a multilayer perceptron 8 -> 64 -> 64 -> 1
// (ReLU) giving the logit that a candidate output block falls under the drop
// threshold.  Forward, gradient (mean binary cross-entropy on logits) and Adam
// kernels written for gfx950, and the C-ABI entry points that train and
// evaluate it on the device.
//
// Parameter layout (MLP_NP = 4801 floats): W1 (64 x 8 row-major), b1 (64),
// W2 (64 x 64 row-major, W2[j][k] maps input k to output j), b2 (64), w3 (64), b3.
#include "tc2_device.h"
#include "../../include/tc2.h"

#include <cmath>
#include <mutex>
#include <vector>

namespace tc2 {

constexpr int OFF_W1 = 0, OFF_B1 = 512, OFF_W2 = 576, OFF_B2 = 4672, OFF_W3 = 4736, OFF_B3 = 4800;
static_assert(MLP_NP == OFF_B3 + 1, "parameter layout");

// One thread per sample: logits of rows of x (n x 8).
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ th,
                                                     const float* __restrict__ x, long long n,
                                                     float* __restrict__ out) {
  __shared__ float s[MLP_NP];
  for (int p = threadIdx.x; p < MLP_NP; p += blockDim.x) s[p] = th[p];
  __syncthreads();
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float xi[MLP_NF];
#pragma unroll
  for (int f = 0; f < MLP_NF; ++f) xi[f] = x[i * MLP_NF + f];
  float h1[MLP_NH];
#pragma unroll
  for (int j = 0; j < MLP_NH; ++j) {
    float a = s[OFF_B1 + j];
#pragma unroll
    for (int f = 0; f < MLP_NF; ++f) a += s[OFF_W1 + j * MLP_NF + f] * xi[f];
    h1[j] = fmaxf(a, 0.f);
  }
  float z = s[OFF_B3];
  for (int j = 0; j < MLP_NH; ++j) {
    float a = s[OFF_B2 + j];
#pragma unroll
    for (int k = 0; k < MLP_NH; ++k) a += s[OFF_W2 + j * MLP_NH + k] * h1[k];
    z += s[OFF_W3 + j] * fmaxf(a, 0.f);
  }
  out[i] = z;
}

// Gradient of the mean loss softplus(z) - y z over samples [0, n) with weight
// 1/n_total, accumulated per block in LDS; gpart (gridDim x MLP_NP) and
// lpart (gridDim) receive the block sums.
__global__ __launch_bounds__(256) void k_mlp_grad(const float* __restrict__ th,
                                                  const float* __restrict__ x,
                                                  const float* __restrict__ y, long long n,
                                                  double inv_n, float* __restrict__ gpart,
                                                  double* __restrict__ lpart) {
  __shared__ float s[MLP_NP];
  __shared__ float g[MLP_NP];
  __shared__ double sl[256];
  for (int p = threadIdx.x; p < MLP_NP; p += blockDim.x) {
    s[p] = th[p];
    g[p] = 0.f;
  }
  __syncthreads();
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double loss = 0.0;
  if (i < n) {
    float xi[MLP_NF];
#pragma unroll
    for (int f = 0; f < MLP_NF; ++f) xi[f] = x[i * MLP_NF + f];
    float h1[MLP_NH], h2[MLP_NH];
#pragma unroll
    for (int j = 0; j < MLP_NH; ++j) {
      float a = s[OFF_B1 + j];
#pragma unroll
      for (int f = 0; f < MLP_NF; ++f) a += s[OFF_W1 + j * MLP_NF + f] * xi[f];
      h1[j] = fmaxf(a, 0.f);
    }
    float z = s[OFF_B3];
    for (int j = 0; j < MLP_NH; ++j) {
      float a = s[OFF_B2 + j];
#pragma unroll
      for (int k = 0; k < MLP_NH; ++k) a += s[OFF_W2 + j * MLP_NH + k] * h1[k];
      h2[j] = fmaxf(a, 0.f);
      z += s[OFF_W3 + j] * h2[j];
    }
    const float yi = y[i];
    // softplus(z) - y z, evaluated without overflow
    loss = (double)(fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))) - yi * z) * inv_n;
    const float dz = (float)((1.0 / (1.0 + exp(-(double)z)) - yi) * inv_n);
    atomicAdd(&g[OFF_B3], dz);
    float dh1[MLP_NH];
#pragma unroll
    for (int k = 0; k < MLP_NH; ++k) dh1[k] = 0.f;
    for (int j = 0; j < MLP_NH; ++j) {
      atomicAdd(&g[OFF_W3 + j], dz * h2[j]);
      const float da2 = h2[j] > 0.f ? dz * s[OFF_W3 + j] : 0.f;
      if (da2 != 0.f) {
        atomicAdd(&g[OFF_B2 + j], da2);
#pragma unroll
        for (int k = 0; k < MLP_NH; ++k) {
          if (h1[k] > 0.f) atomicAdd(&g[OFF_W2 + j * MLP_NH + k], da2 * h1[k]);
          dh1[k] += s[OFF_W2 + j * MLP_NH + k] * da2;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < MLP_NH; ++k) {
      const float da1 = h1[k] > 0.f ? dh1[k] : 0.f;
      if (da1 != 0.f) {
        atomicAdd(&g[OFF_B1 + k], da1);
#pragma unroll
        for (int f = 0; f < MLP_NF; ++f) atomicAdd(&g[OFF_W1 + k * MLP_NF + f], da1 * xi[f]);
      }
    }
  }
  sl[threadIdx.x] = loss;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sl[threadIdx.x] += sl[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) lpart[blockIdx.x] = sl[0];
  for (int p = threadIdx.x; p < MLP_NP; p += blockDim.x)
    gpart[(size_t)blockIdx.x * MLP_NP + p] = g[p];
}

// Sum of the block partials in block order.
__global__ void k_mlp_sum(const float* gpart, const double* lpart, int nblk, float* grad,
                          double* loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < MLP_NP) {
    double acc = 0.0;
    for (int b = 0; b < nblk; ++b) acc += gpart[(size_t)b * MLP_NP + p];
    grad[p] = (float)acc;
  }
  if (p == 0) {
    double l = 0.0;
    for (int b = 0; b < nblk; ++b) l += lpart[b];
    *loss = l;
  }
}

// Adam (Kingma & Ba) with bias correction, step t >= 1.
__global__ void k_adam(float* th, float* m, float* v, const float* g, float lr, float b1,
                       float b2, float eps, int t) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= MLP_NP) return;
  const float gp = g[p];
  const float mp = b1 * m[p] + (1.f - b1) * gp;
  const float vp = b2 * v[p] + (1.f - b2) * gp * gp;
  m[p] = mp;
  v[p] = vp;
  const float mh = mp / (1.f - powf(b1, (float)t));
  const float vh = vp / (1.f - powf(b2, (float)t));
  th[p] -= lr * mh / (sqrtf(vh) + eps);
}

// Scratch of tc2_mlp_grad_noalloc: the per-block gradient partials (float,
// TC2_MLP_NOALLOC_MAX_N / 256 blocks of MLP_NP) followed by the per-block loss
// partials (double).  Every device the library runs on holds its own copy
// until the process ends.
constexpr int NA_BLOCKS = TC2_MLP_NOALLOC_MAX_N / 256;
constexpr size_t NA_GPART = (size_t)NA_BLOCKS * MLP_NP * sizeof(float);
constexpr size_t NA_LPART_OFF = (NA_GPART + 255) / 256 * 256;
constexpr size_t NA_BYTES = NA_LPART_OFF + (size_t)NA_BLOCKS * sizeof(double);
static __device__ __align__(256) unsigned char scratch[NA_BYTES];

}  // namespace tc2

using namespace tc2;

namespace {

struct DevMem {
  void* p = nullptr;
  ~DevMem() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t n) { return tc2::dev_malloc(&p, n < 256 ? 256 : n); }
  template <typename T> T* as() const { return (T*)p; }
};

#define MLPCHK(x)                                                        \
  do {                                                                   \
    hipError_t e_ = (x);                                                 \
    if (e_ != hipSuccess) return e_ == hipErrorOutOfMemory ? TC2_ENOMEM : TC2_EDEVICE; \
  } while (0)

tc2_status use_device(int device) {
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return TC2_EDEVICE;
  if (device < 0 || device >= ndev) return TC2_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return TC2_EDEVICE;
  return TC2_OK;
}

bool finite_all(const float* p, long long n) {
  for (long long i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// gradient and loss of the mean loss over rows [0, n) of the device data
tc2_status grad_dev(hipStream_t st, const float* th, const float* x, const float* y, long long n,
                    long long n_total, DevMem& gpart, DevMem& lpart, float* grad, double* loss) {
  const int nblk = (int)((n + 255) / 256);
  hipLaunchKernelGGL(k_mlp_grad, dim3(nblk), dim3(256), 0, st, th, x, y, n, 1.0 / (double)n_total,
                     gpart.as<float>(), lpart.as<double>());
  hipLaunchKernelGGL(k_mlp_sum, dim3((MLP_NP + 255) / 256), dim3(256), 0, st, gpart.as<float>(),
                     lpart.as<double>(), nblk, grad, loss);
  MLPCHK(hipGetLastError());
  return TC2_OK;
}

// Device address of `scratch` on each device, looked up once per device with
// that device current (the array's host-side name is not a device address).
constexpr int NA_MAX_DEVICES = 64;
std::mutex na_lock;
void* na_ptr[NA_MAX_DEVICES] = {};

tc2_status scratch_of(int device, void** out) {
  if (device < 0 || device >= NA_MAX_DEVICES) return TC2_EDEVICE;
  std::lock_guard<std::mutex> g(na_lock);
  if (!na_ptr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return TC2_EDEVICE;
    na_ptr[device] = p;
  }
  *out = na_ptr[device];
  return TC2_OK;
}

}  // namespace

extern "C" {

tc2_status tc2_mlp_grad_noalloc(const float* theta, const float* x, const float* y, int64_t n,
                                void* hip_stream, float* grad, double* loss) {
  if (!theta || !x || !y || !grad || !loss || n <= 0) return TC2_EINVAL;
  if (n > TC2_MLP_NOALLOC_MAX_N) return TC2_EINVAL;
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return TC2_EDEVICE;
  void* base = nullptr;
  if (tc2_status s = scratch_of(device, &base); s != TC2_OK) return s;
  float* gpart = (float*)base;
  double* lpart = (double*)((unsigned char*)base + NA_LPART_OFF);
  hipStream_t st = (hipStream_t)hip_stream;
  const int nblk = (int)((n + 255) / 256);
  // every partial the sum reads is written by the gradient kernel first: no
  // clearing is needed
  hipLaunchKernelGGL(k_mlp_grad, dim3(nblk), dim3(256), 0, st, theta, x, y, (long long)n,
                     1.0 / (double)n, gpart, lpart);
  hipLaunchKernelGGL(k_mlp_sum, dim3((MLP_NP + 255) / 256), dim3(256), 0, st, gpart, lpart, nblk,
                     grad, loss);
  MLPCHK(hipGetLastError());
  return TC2_OK;
}

tc2_status tc2_mlp_forward(const float* theta, const float* x, int64_t n, int32_t device,
                           float* logits) {
  if (!theta || (n > 0 && (!x || !logits)) || n < 0) return TC2_EINVAL;
  if (!finite_all(theta, MLP_NP) || !finite_all(x, n * MLP_NF)) return TC2_ENAN;
  tc2_status s = use_device(device);
  if (s != TC2_OK) return s;
  if (n == 0) return TC2_OK;
  DevMem dth, dx, dout;
  MLPCHK(dth.alloc(MLP_NP * 4));
  MLPCHK(dx.alloc((size_t)n * MLP_NF * 4));
  MLPCHK(dout.alloc((size_t)n * 4));
  MLPCHK(hipMemcpy(dth.p, theta, MLP_NP * 4, hipMemcpyHostToDevice));
  MLPCHK(hipMemcpy(dx.p, x, (size_t)n * MLP_NF * 4, hipMemcpyHostToDevice));
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, 0,
                     dth.as<float>(), dx.as<float>(), (long long)n, dout.as<float>());
  MLPCHK(hipGetLastError());
  MLPCHK(hipMemcpy(logits, dout.p, (size_t)n * 4, hipMemcpyDeviceToHost));
  return TC2_OK;
}

tc2_status tc2_mlp_grad(const float* theta, const float* x, const float* y, int64_t n,
                        int32_t device, float* grad, double* loss) {
  if (!theta || !x || !y || !grad || !loss || n <= 0) return TC2_EINVAL;
  if (!finite_all(theta, MLP_NP) || !finite_all(x, n * MLP_NF) || !finite_all(y, n)) return TC2_ENAN;
  tc2_status s = use_device(device);
  if (s != TC2_OK) return s;
  DevMem dth, dx, dy, gpart, lpart, dg, dl;
  const int nblk = (int)((n + 255) / 256);
  MLPCHK(dth.alloc(MLP_NP * 4));
  MLPCHK(dx.alloc((size_t)n * MLP_NF * 4));
  MLPCHK(dy.alloc((size_t)n * 4));
  MLPCHK(gpart.alloc((size_t)nblk * MLP_NP * 4));
  MLPCHK(lpart.alloc((size_t)nblk * 8));
  MLPCHK(dg.alloc(MLP_NP * 4));
  MLPCHK(dl.alloc(8));
  MLPCHK(hipMemcpy(dth.p, theta, MLP_NP * 4, hipMemcpyHostToDevice));
  MLPCHK(hipMemcpy(dx.p, x, (size_t)n * MLP_NF * 4, hipMemcpyHostToDevice));
  MLPCHK(hipMemcpy(dy.p, y, (size_t)n * 4, hipMemcpyHostToDevice));
  s = grad_dev(0, dth.as<float>(), dx.as<float>(), dy.as<float>(), n, n, gpart, lpart,
               dg.as<float>(), dl.as<double>());
  if (s != TC2_OK) return s;
  MLPCHK(hipMemcpy(grad, dg.p, MLP_NP * 4, hipMemcpyDeviceToHost));
  MLPCHK(hipMemcpy(loss, dl.p, 8, hipMemcpyDeviceToHost));
  return TC2_OK;
}

tc2_status tc2_mlp_train(const float* x, const float* y, int64_t n, const tc2_mlp_train_opts* o,
                         float* theta, double* loss_per_epoch) {
  if (!x || !y || !o || !theta || n <= 0) return TC2_EINVAL;
  if (o->epochs < 1 || o->batch < 1 || !(o->lr > 0.f) || !(o->beta1 >= 0.f && o->beta1 < 1.f) ||
      !(o->beta2 >= 0.f && o->beta2 < 1.f) || !(o->adam_eps > 0.f))
    return TC2_EINVAL;
  if (!finite_all(theta, MLP_NP) || !finite_all(x, n * MLP_NF) || !finite_all(y, n)) return TC2_ENAN;
  tc2_status s = use_device(o->device);
  if (s != TC2_OK) return s;
  const long long B = std::min<long long>(o->batch, n);
  const int nblk = (int)((B + 255) / 256);
  DevMem dth, dm, dv, dx, dy, gpart, lpart, dg, dl;
  MLPCHK(dth.alloc(MLP_NP * 4));
  MLPCHK(dm.alloc(MLP_NP * 4));
  MLPCHK(dv.alloc(MLP_NP * 4));
  MLPCHK(dx.alloc((size_t)n * MLP_NF * 4));
  MLPCHK(dy.alloc((size_t)n * 4));
  MLPCHK(gpart.alloc((size_t)nblk * MLP_NP * 4));
  MLPCHK(lpart.alloc((size_t)nblk * 8));
  MLPCHK(dg.alloc(MLP_NP * 4));
  MLPCHK(dl.alloc(8));
  MLPCHK(hipMemcpy(dth.p, theta, MLP_NP * 4, hipMemcpyHostToDevice));
  MLPCHK(hipMemset(dm.p, 0, MLP_NP * 4));
  MLPCHK(hipMemset(dv.p, 0, MLP_NP * 4));
  MLPCHK(hipMemcpy(dx.p, x, (size_t)n * MLP_NF * 4, hipMemcpyHostToDevice));
  MLPCHK(hipMemcpy(dy.p, y, (size_t)n * 4, hipMemcpyHostToDevice));
  int t = 0;
  for (int ep = 0; ep < o->epochs; ++ep) {
    double ep_loss = 0.0;
    for (long long b0 = 0; b0 < n; b0 += B) {
      const long long nb = std::min<long long>(B, n - b0);
      s = grad_dev(0, dth.as<float>(), dx.as<float>() + b0 * MLP_NF, dy.as<float>() + b0, nb, nb,
                   gpart, lpart, dg.as<float>(), dl.as<double>());
      if (s != TC2_OK) return s;
      ++t;
      hipLaunchKernelGGL(k_adam, dim3((MLP_NP + 255) / 256), dim3(256), 0, 0, dth.as<float>(),
                         dm.as<float>(), dv.as<float>(), dg.as<float>(), o->lr, o->beta1, o->beta2,
                         o->adam_eps, t);
      MLPCHK(hipGetLastError());
      double bl = 0.0;
      MLPCHK(hipMemcpy(&bl, dl.p, 8, hipMemcpyDeviceToHost));
      ep_loss += bl * (double)nb / (double)n;
    }
    if (loss_per_epoch) loss_per_epoch[ep] = ep_loss;
  }
  MLPCHK(hipMemcpy(theta, dth.p, MLP_NP * 4, hipMemcpyDeviceToHost));
  return TC2_OK;
}

}  // extern "C"
