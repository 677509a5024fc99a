// mlp.h -- the surrogate network's sizes, parameter layout and host object.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fstat {

constexpr int kHid = 256;
// flat layout: W1[256][3] b1[256] | W2 b2 | W3 b3 | W4 b4 | w5[256] b5
__host__ __device__ constexpr int64_t mlp_off_w(int l) {
  return l == 0 ? 0 : (l == 4 ? 198400 : 1024 + (int64_t)(l - 1) * (kHid * kHid + kHid));
}
__host__ __device__ constexpr int64_t mlp_off_b(int l) {
  return l == 0 ? 768 : (l == 4 ? 198656 : mlp_off_w(l) + (int64_t)kHid * kHid);
}
constexpr int64_t kNParams = 198657;
static_assert(mlp_off_b(3) + kHid == mlp_off_w(4), "layout");

// device buffers of one network (parameters, Adam moments, activations)
struct Mlp {
  float* params = nullptr;   // FP32 master weights
  float* grad = nullptr;
  float* m1 = nullptr;
  float* m2 = nullptr;
  uint16_t* wbf = nullptr;   // BF16 copies of W2..W4
  float* red = nullptr;      // partial column sums of the backward pass
  float* splitk = nullptr;   // split-K partial weight gradients [16][256][256]
  float* yinf = nullptr;     // outputs of infer()
  int64_t cap_inf = 0;
  float* z[4] = {nullptr, nullptr, nullptr, nullptr};        // pre-activations [B][256]
  uint16_t* h[4] = {nullptr, nullptr, nullptr, nullptr};     // BF16 activations
  float* dz = nullptr;
  uint16_t* dzb = nullptr;
  float* dh = nullptr;
  float* y = nullptr;
  float* dy = nullptr;
  float* sq = nullptr;
  int cap_batch = 0;

  int alloc(int batch);
  void release_acts();
  void release();
  void refresh_bf16(hipStream_t s);
  void forward(const float* x, const float* tgt, int B, hipStream_t s);
  void backward(const float* x, int B, hipStream_t s);
  void adam(int t, float lr, hipStream_t s);
  int infer_alloc(int64_t rows);
  void infer(const float* x, int64_t rows, hipStream_t s);   // -> yinf[rows]
};

}  // namespace fstat
