// surrogate.hip -- training and use of the learned eccentric-phase surrogate.
//
// Training (on the device, by the kernels of mlp.hip): samples (f, Mc, e0)
// uniform over f in [10, 100] mHz, Mc in [10, 50] Msun, e0 in [0, 0.15];
// targets from the plain template code (Psi_e in units of e0^2 Psi_N);
// Adam with a cosine-decayed step size; the last 1/16 of the samples is held
// out.  Use (in the semi-coherent stages, Np >= 16): the network is evaluated
// at four knots per partition, its values are interpolated to every bin, and
// a particle keeps the surrogate only if, in every partition, the phase
// residual against the analytic term at the knots and mid-points (after its
// mean is removed) implies a mismatch <= 1e-3; otherwise it falls back to the
// analytic template.  The final coherent stage (Np = 1) never uses it.
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/fstat.h"
#include "fstat_api_internal.h"
#include "mlp.h"

namespace fstat {

constexpr double kSurMismatch = 1e-3;

__global__ void k_zero_ull(unsigned long long* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// mean of the per-sample squared errors of one batch -> out[0] (one block)
__global__ void k_batch_mean(const float* __restrict__ sq, int B, double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < B; i += blockDim.x) s += (double)sq[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0] / (double)B;
}

// running (sum of squares, max |error|) over validation batches (one block)
__global__ void k_val_acc(const float* __restrict__ y, const float* __restrict__ t, int B,
                          double* __restrict__ acc) {
  __shared__ double s2[256], mx[256];
  double a = 0.0, m = 0.0;
  for (int i = threadIdx.x; i < B; i += blockDim.x) {
    double e = (double)y[i] - (double)t[i];
    a += e * e;
    m = fmax(m, fabs(e));
  }
  s2[threadIdx.x] = a;
  mx[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s2[threadIdx.x] += s2[threadIdx.x + o];
      mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    acc[0] += s2[0];
    acc[1] = fmax(acc[1], mx[0]);
  }
}

static uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// uniform(-sqrt(3/fan_in), +sqrt(3/fan_in)) weights, zero biases
static void init_params(std::vector<float>& p, uint64_t seed) {
  p.assign(kNParams, 0.0f);
  uint64_t s = seed;
  auto fill = [&](int64_t off, int64_t count, int fan_in) {
    double lim = std::sqrt(3.0 / fan_in);
    for (int64_t i = 0; i < count; ++i) {
      double u = (double)(splitmix64(s) >> 11) * 0x1.0p-53;
      p[off + i] = (float)((2.0 * u - 1.0) * lim);
    }
  };
  fill(mlp_off_w(0), (int64_t)kHid * 3, 3);
  for (int l = 1; l < 4; ++l) fill(mlp_off_w(l), (int64_t)kHid * kHid, kHid);
  fill(mlp_off_w(4), kHid, kHid);
}

template <typename T>
static int grow(T** p, size_t* cap, size_t need, const char* what) {
  if (*p && *cap >= need) return FSTAT_OK;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *cap = 0;
  int rc = hip_check(hipMalloc((void**)p, (need ? need : 1) * sizeof(T)), what);
  if (!rc) *cap = need;
  return rc;
}

static int64_t knot_rows(int64_t n, int32_t stride) { return ((n * stride * 4 + 63) / 64) * 64; }

int sur_ensure(fstat_plan_s* P, int64_t n, int32_t stride) {
  if (!P->sur || !P->sur_trained)
    return set_error(FSTAT_EINVAL, "surrogate requested but not trained (fstat_surrogate_train)");
  int64_t rows = knot_rows(n, stride);
  if (rows > (int64_t)INT32_MAX) return set_error(FSTAT_EINVAL, "too many surrogate knots");
  int rc = P->sur->infer_alloc(rows);
  if (!rc) rc = grow(&P->sur_X, &P->cap_sur_X, (size_t)rows * 3, "alloc knots");
  if (!rc) rc = grow(&P->sur_ek, &P->cap_sur_ek, (size_t)n * stride * 8, "alloc knot coeffs");
  if (!rc) rc = grow(&P->sur_mm, &P->cap_sur_mm, (size_t)n * stride, "alloc mismatch");
  if (!rc) rc = grow(&P->sur_counters, &P->cap_sur_counters, 2, "alloc counters");
  return rc;
}

// after k_setup: knots -> network -> spot check -> per-particle decision
int sur_prepare(fstat_plan_s* P, int64_t n, int32_t stride, hipStream_t s) {
  int64_t rows = knot_rows(n, stride);
  hipLaunchKernelGGL(k_zero_ull, dim3(1), dim3(64), 0, s, P->sur_counters, 2);
  launch_sur_knots(P->grid, stride, n, rows, P->ws, P->sur_X, s);
  P->sur->infer(P->sur_X, rows, s);
  launch_sur_check(P->grid, stride, n, P->ws, P->sur->yinf, P->sur_ek, P->sur_mm, kSurMismatch,
                   P->sur_counters, s);
  return hip_check(hipGetLastError(), "surrogate launch");
}

void sur_release(fstat_plan_s* P) {
  if (P->sur) {
    P->sur->release();
    delete P->sur;
    P->sur = nullptr;
  }
  for (void* p : {(void*)P->sur_X, (void*)P->sur_ek, (void*)P->sur_mm, (void*)P->sur_counters})
    if (p) (void)hipFree(p);
  P->sur_X = nullptr; P->sur_ek = nullptr; P->sur_mm = nullptr; P->sur_counters = nullptr;
  P->sur_trained = false;
}

}  // namespace fstat

using namespace fstat;

extern "C" int fstat_surrogate_train(fstat_plan_t P, fstat_surrogate_desc* d, void* hip_stream) {
  if (!P || !d) return set_error(FSTAT_EINVAL, "null plan or descriptor");
  const int B = d->batch;
  if (B < 64 || B % 64 || B > (1 << 20)) return set_error(FSTAT_EINVAL, "batch must be a multiple of 64");
  if (d->n_samples < 17 * (int64_t)B || d->n_samples > ((int64_t)1 << 31))
    return set_error(FSTAT_EINVAL, "n_samples must be >= 17 batches");
  if (d->steps < 1 || !(d->lr > 0.0)) return set_error(FSTAT_EINVAL, "steps >= 1 and lr > 0 required");
  hipStream_t s = (hipStream_t)hip_stream;
  if (!P->sur) P->sur = new Mlp();
  Mlp& net = *P->sur;
  int rc = net.alloc(B);
  if (rc) return rc;
  const int64_t n = d->n_samples;
  const int64_t nval = ((n / 16) / B) * B;
  const int64_t ntrain = ((n - nval) / B) * B;
  float *X = nullptr, *T = nullptr;
  double *loss = nullptr, *vacc = nullptr;
  rc = hip_check(hipMalloc(&X, sizeof(float) * 3 * n), "alloc X");
  if (!rc) rc = hip_check(hipMalloc(&T, sizeof(float) * n), "alloc T");
  if (!rc) rc = hip_check(hipMalloc(&loss, sizeof(double) * d->steps), "alloc loss");
  if (!rc) rc = hip_check(hipMalloc(&vacc, sizeof(double) * 2), "alloc val");
  std::vector<float> p0;
  init_params(p0, d->seed);
  if (!rc) rc = hip_check(hipMemcpyAsync(net.params, p0.data(), sizeof(float) * kNParams,
                                         hipMemcpyHostToDevice, s), "copy params");
  if (!rc) rc = hip_check(hipMemsetAsync(net.m1, 0, sizeof(float) * kNParams, s), "zero m1");
  if (!rc) rc = hip_check(hipMemsetAsync(net.m2, 0, sizeof(float) * kNParams, s), "zero m2");
  if (!rc) rc = hip_check(hipMemsetAsync(vacc, 0, sizeof(double) * 2, s), "zero val");
  if (!rc) {
    launch_sur_data(d->seed, n, X, T, s);
    net.refresh_bf16(s);
    for (int st = 0; st < d->steps; ++st) {
      int64_t off = ((int64_t)st * B) % ntrain;
      float lr = (float)(d->lr * 0.5 * (1.0 + std::cos(M_PI * st / (double)d->steps)));
      net.forward(X + 3 * off, T + off, B, s);
      hipLaunchKernelGGL(k_batch_mean, dim3(1), dim3(256), 0, s, net.sq, B, loss + st);
      net.backward(X + 3 * off, B, s);
      net.adam(st + 1, lr, s);
    }
    for (int64_t off = ntrain; off + B <= ntrain + nval; off += B) {
      net.forward(X + 3 * off, nullptr, B, s);
      hipLaunchKernelGGL(k_val_acc, dim3(1), dim3(256), 0, s, net.y, T + off, B, vacc);
    }
    rc = hip_check(hipGetLastError(), "training launch");
  }
  double hv[2] = {0.0, 0.0};
  if (!rc) rc = hip_check(hipMemcpyAsync(hv, vacc, sizeof(hv), hipMemcpyDeviceToHost, s), "copy val");
  if (!rc && d->loss_trace)
    rc = hip_check(hipMemcpyAsync(d->loss_trace, loss, sizeof(double) * d->steps,
                                  hipMemcpyDeviceToHost, s), "copy loss");
  if (!rc) rc = hip_check(hipStreamSynchronize(s), "training");
  if (X) (void)hipFree(X);
  if (T) (void)hipFree(T);
  if (loss) (void)hipFree(loss);
  if (vacc) (void)hipFree(vacc);
  if (rc) return rc;
  d->val_rmse = nval > 0 ? std::sqrt(hv[0] / (double)nval) : 0.0;
  d->val_max = hv[1];
  P->sur_trained = true;
  return FSTAT_OK;
}

extern "C" int fstat_surrogate_stats(fstat_plan_t P, int64_t* used, int64_t* fallback,
                                     int32_t* flags, int64_t n) {
  if (!P || !P->sur_counters) return set_error(FSTAT_EINVAL, "no surrogate evaluation yet");
  if (flags && (n < 0 || n > P->last.n))
    return set_error(FSTAT_EINVAL, "flags for %lld particles, the last evaluation had %lld",
                     (long long)n, (long long)P->last.n);
  unsigned long long c[2] = {0, 0};
  int rc = hip_check(hipMemcpy(c, P->sur_counters, sizeof(c), hipMemcpyDeviceToHost), "read counters");
  // the per-particle decision is the `sur` field of each particle's constants
  if (!rc && flags && n > 0)
    rc = hip_check(hipMemcpy2D(flags, sizeof(int32_t), &P->ws.pc[0].sur, sizeof(PartConst),
                               sizeof(int32_t), (size_t)n, hipMemcpyDeviceToHost), "read flags");
  if (rc) return rc;
  if (used) *used = (int64_t)c[0];
  if (fallback) *fallback = (int64_t)c[1];
  return FSTAT_OK;
}

extern "C" int fstat_surrogate_params(fstat_plan_t P, const float* in, float* out, void* hip_stream) {
  if (!P) return set_error(FSTAT_EINVAL, "null plan");
  hipStream_t s = (hipStream_t)hip_stream;
  int rc = FSTAT_OK;
  if (out) {
    if (!P->sur || !P->sur_trained) return set_error(FSTAT_EINVAL, "no trained surrogate to read");
    rc = hip_check(hipMemcpyAsync(out, P->sur->params, sizeof(float) * kNParams,
                                  hipMemcpyDeviceToHost, s), "read surrogate weights");
    if (!rc) rc = hip_check(hipStreamSynchronize(s), "read surrogate weights");
    if (rc) return rc;
  }
  if (in) {
    for (int64_t i = 0; i < kNParams; ++i)
      if (!std::isfinite(in[i])) return set_error(FSTAT_EINVAL, "weight %lld is not finite", (long long)i);
    if (!P->sur) P->sur = new Mlp();
    rc = P->sur->alloc(64);
    if (!rc) rc = hip_check(hipMemcpyAsync(P->sur->params, in, sizeof(float) * kNParams,
                                           hipMemcpyHostToDevice, s), "copy surrogate weights");
    if (!rc) {
      P->sur->refresh_bf16(s);
      rc = hip_check(hipGetLastError(), "surrogate weights");
    }
    if (!rc) rc = hip_check(hipStreamSynchronize(s), "copy surrogate weights");
    if (rc) return rc;
    P->sur_trained = true;
  }
  return FSTAT_OK;
}
