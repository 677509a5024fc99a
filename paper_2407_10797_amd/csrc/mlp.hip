// mlp.hip -- learned surrogate for the eccentric phase correction Psi_e (App. A):
// a 3 -> 256 -> 256 -> 256 -> 256 -> 1 SiLU network, BF16 operands on MFMA with
// FP32 accumulation, FP32 master weights and Adam, trained on the GPU by the
// kernels below on samples produced by the plain template code.
//
// Parameter layout (flat FP32, 198,657 values):
//   W1[256][3] b1[256] | W2[256][256] b2[256] | W3 b3 | W4 b4 | w5[256] b5
// Inputs: (f, Mc, e0) mapped linearly to [-1, 1] over f in [10, 100] mHz,
// Mc in [10, 50] Msun, e0 in [0, 0.15].  Output: Psi_e / ((2355/1462) e0^2 Psi_N),
// the eccentric term in units of the factors the plain path computes anyway
// (e0^2 and the Newtonian phase), so that Psi_e = -(2355/1462) e0^2 Psi_N y.
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/fstat.h"
#include "fstat_api_internal.h"
#include "mlp.h"

namespace fstat {

typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

// gfx950's 16x16x32 BF16 MFMA: lane l supplies A[l % 16][k] and B[k][l % 16]
// for its eight k of group l / 16 (the same k for A and B, so the order of k
// within a group does not matter), and receives D[4 (l / 16) + r][l % 16].
__device__ __forceinline__ v4f mfma32(v8s a, v8s b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a),
                                                 __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
}

__device__ __forceinline__ uint16_t f2bf(float f) {   // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ float sigm(float z) { return 1.0f / (1.0f + __expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigm(z); }
__device__ __forceinline__ float dsilu(float z) {
  float s = sigm(z);
  return s * (1.0f + z * (1.0f - s));
}

// ---------------------------------------------------------------------------
// C[m][n] = sum_k A(m,k) B(k,n), A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn]
// (BF16), FP32 accumulate.  Block = 4 wavefronts = 64x64 outputs, each wave a
// 32x32 quadrant of 2x2 MFMA 16x16x32 tiles; K advances 32 at a time through
// LDS.  M, N multiples of 64, K a multiple of 32 (checked by the host).
// Split K: block z covers k in [z * kper, (z + 1) * kper) and writes C + z * cz.
// Epilogue FWD: z = acc + bias[n] -> Z[m][n] (FP32), H[m][n] = bf16(SiLU(z)).
// Epilogue STORE: C[m][n] = acc.
// ---------------------------------------------------------------------------
enum { kEpiFwd = 0, kEpiStore = 1 };
constexpr int kGemmK = 32;

template <int EPI>
__global__ __launch_bounds__(256) void k_gemm_bf16(const uint16_t* __restrict__ A, int64_t sam,
                                                   int64_t sak, const uint16_t* __restrict__ B,
                                                   int64_t sbk, int64_t sbn, int M, int N, int K,
                                                   float* __restrict__ C, int64_t ldc,
                                                   const float* __restrict__ bias,
                                                   uint16_t* __restrict__ H, int64_t ldh,
                                                   int kper, int64_t cz) {
  __shared__ __align__(16) uint16_t As[64][kGemmK + 8];   // rows of 80 B (16-byte multiple)
  __shared__ uint16_t Bs[kGemmK][64 + 4];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int wr = w >> 1, wc = w & 1;
  const int kbeg = blockIdx.z * kper, kend = min(K, kbeg + kper);
  C += (int64_t)blockIdx.z * cz;
  v4f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kbeg; k0 < kend; k0 += kGemmK) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {       // 64x32 A tile and 32x64 B tile, 8 elements per thread
      int idx = t * 8 + e;
      int ar = idx >> 5, ak = idx & 31;
      As[ar][ak] = A[(int64_t)(m0 + ar) * sam + (int64_t)(k0 + ak) * sak];
      int bk = idx >> 6, bn = idx & 63;
      Bs[bk][bn] = B[(int64_t)(k0 + bk) * sbk + (int64_t)(n0 + bn) * sbn];
    }
    __syncthreads();
    const int kb = 8 * (lane >> 4), rr = lane & 15;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int row = 32 * wr + 16 * i + rr;
      const v8s a = *reinterpret_cast<const v8s*>(&As[row][kb]);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        v8s b;
        const int col = 32 * wc + 16 * j + rr;
#pragma unroll
        for (int q = 0; q < 8; ++q) b[q] = (short)Bs[kb + q][col];
        acc[i][j] = mfma32(a, b, acc[i][j]);
      }
    }
    __syncthreads();
  }
  // lane holds D[4 (lane/16) + r][lane % 16] of each 16x16 tile
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int m = m0 + 32 * wr + 16 * i + 4 * (lane >> 4) + r;
        int n = n0 + 32 * wc + 16 * j + (lane & 15);
        float v = acc[i][j][r];
        if (EPI == kEpiFwd) {
          float z = v + bias[n];
          C[(int64_t)m * ldc + n] = z;
          H[(int64_t)m * ldh + n] = f2bf(silu(z));
        } else {
          C[(int64_t)m * ldc + n] = v;
        }
      }
}

// first layer 3 -> 256 (VALU): z1 = W1 x + b1, h1 = bf16(SiLU(z1))
__global__ void k_layer_in(const float* __restrict__ x, int B, const float* __restrict__ W1,
                           const float* __restrict__ b1, float* __restrict__ z1,
                           uint16_t* __restrict__ h1) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)B * kHid) return;
  int m = (int)(g / kHid), n = (int)(g % kHid);
  float z = b1[n] + W1[n * 3 + 0] * x[m * 3 + 0] + W1[n * 3 + 1] * x[m * 3 + 1] +
            W1[n * 3 + 2] * x[m * 3 + 2];
  z1[g] = z;
  h1[g] = f2bf(silu(z));
}

// output layer 256 -> 1 (FP32 from the FP32 pre-activations), squared error,
// dy = 2 (y - t) / B.  One wavefront per sample.
__global__ void k_layer_out(const float* __restrict__ z4, int B, const float* __restrict__ w5,
                            const float* __restrict__ b5, const float* __restrict__ tgt,
                            float* __restrict__ y, float* __restrict__ dy,
                            float* __restrict__ sqerr) {
  int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, lane = threadIdx.x & 63;
  if (wave >= B) return;
  float s = 0.f;
  for (int k = lane; k < kHid; k += 64) s += w5[k] * silu(z4[(int64_t)wave * kHid + k]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) {
    float yy = s + b5[0];
    y[wave] = yy;
    if (tgt) {
      float e = yy - tgt[wave];
      dy[wave] = 2.0f * e / (float)B;
      sqerr[wave] = e * e;
    }
  }
}

// dz4 = dy w5 * SiLU'(z4) (bf16 and FP32 copies); also dW5, db5 (one block
// per output unit, ordered reductions over the batch)
__global__ void k_out_back(const float* __restrict__ z4, int B, const float* __restrict__ w5,
                           const float* __restrict__ dy, float* __restrict__ dz,
                           uint16_t* __restrict__ dzb) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)B * kHid) return;
  int m = (int)(g / kHid), n = (int)(g % kHid);
  float d = dy[m] * w5[n] * dsilu(z4[g]);
  dz[g] = d;
  dzb[g] = f2bf(d);
}

// Column reductions over the batch, in two fixed-order passes (no atomics):
// part[s][q][n] = sum over the rows m of slice s of v(m, n) * wq(m), where
// v = a[m][n] (or SiLU(a[m][n])) and wq(m) = wv[m * wstride + q] for q < NW,
// 1 otherwise; then out_q[n * ostr_q] = sum_s part[s][q][n].  Block = 64 columns x 4
// row groups; grid = (256 / 64, slices).
constexpr int kRedSlices = 64;

template <int Q, int NW, bool SILU>
__global__ __launch_bounds__(256) void k_colred(const float* __restrict__ a, int B,
                                                const float* __restrict__ wv, int wstride,
                                                float* __restrict__ part) {
  __shared__ float red[4][Q][64];
  const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + c;
  const int rows = (B + gridDim.y - 1) / gridDim.y;
  const int m0 = blockIdx.y * rows, m1 = min(B, m0 + rows);
  float acc[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) acc[q] = 0.f;
  for (int m = m0 + g; m < m1; m += 4) {
    float v = a[(int64_t)m * kHid + n];
    if (SILU) v = silu(v);
#pragma unroll
    for (int q = 0; q < Q; ++q) acc[q] += q < NW ? v * wv[(int64_t)m * wstride + q] : v;
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) red[g][q][c] = acc[q];
  __syncthreads();
  if (g == 0) {
#pragma unroll
    for (int q = 0; q < Q; ++q)
      part[((int64_t)blockIdx.y * Q + q) * kHid + n] =
          red[0][q][c] + red[1][q][c] + red[2][q][c] + red[3][q][c];
  }
}

struct RedOut {
  float* p[4];
  int stride[4];
};

template <int Q>
__global__ void k_colfin(const float* __restrict__ part, int slices, RedOut o) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= kHid) return;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    float s = 0.f;
    for (int k = 0; k < slices; ++k) s += part[((int64_t)k * Q + q) * kHid + n];
    o.p[q][(int64_t)n * o.stride[q]] = s;
  }
}

// dz_prev = dh * SiLU'(z_prev)  (dh FP32 from the GEMM)
__global__ void k_act_back(const float* __restrict__ dh, const float* __restrict__ zprev, int64_t n,
                           float* __restrict__ dz, uint16_t* __restrict__ dzb) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  float d = dh[g] * dsilu(zprev[g]);
  dz[g] = d;
  if (dzb) dzb[g] = f2bf(d);
}

// out[i] = sum_s part[s][i], i < 256 * 256 (split-K partial products, fixed order)
constexpr int kSplitK = 16;
__global__ void k_splitsum(const float* __restrict__ part, int ks, float* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)kHid * kHid) return;
  float s = 0.f;
  for (int k = 0; k < ks; ++k) s += part[(int64_t)k * kHid * kHid + i];
  out[i] = s;
}

// sum of dy over the batch -> db5 (one block, fixed order)
__global__ void k_sum_dy(const float* __restrict__ dy, int B, float* __restrict__ out) {
  __shared__ float red[256];
  float s = 0.f;
  for (int i = threadIdx.x; i < B; i += blockDim.x) s += dy[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// Inference-only forward of the whole network on R rows, keeping no
// activations (knot evaluation).  One wavefront per 16 rows, four per block;
// the weights pass through LDS in 16 KB k-slabs of 32 shared by the four
// waves.  Layer 1 runs on the VALU straight into the MFMA A-operand layout
// (lane l: row l % 16, k = 32 kb + 8 (l / 16) + j); layers 2-4 are 16x16x32
// BF16 MFMA tiles over all 256 outputs with the weights' BF16 copies read from
// the LDS slabs in the B-operand layout (col l % 16, same k); between layers
// the 16x256 tile goes through the wave's own LDS rows to turn the D layout
// (row 4 (l / 16) + r, col l % 16) back into the A layout.  The output unit
// is a lane reduction.  Same operand rounding as the training forward: BF16
// hidden activations, FP32 last pre-activation, FP32 output layer.
__global__ __launch_bounds__(256, 2) void k_mlp_infer(const float* __restrict__ x, int64_t R,
                                                   const float* __restrict__ P,
                                                   const uint16_t* __restrict__ wbf,
                                                   float* __restrict__ y) {
  __shared__ __align__(16) uint16_t T[4][16][kHid + 8];
  __shared__ __align__(16) uint16_t Ws[2][kHid][kGemmK + 8];   // two k-slabs of W (rows n, 32 k)
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c16 = lane & 15, g4 = lane >> 4;
  const int64_t r0 = ((int64_t)blockIdx.x * 4 + w) * 16;
  const int64_t row = r0 + c16 < R ? r0 + c16 : R - 1;
  const float x0 = x[row * 3 + 0], x1 = x[row * 3 + 1], x2 = x[row * 3 + 2];
  constexpr int NK = kHid / kGemmK;
  v8s a[NK];
  {
    const float* W1 = P + mlp_off_w(0);
    const float* b1 = P + mlp_off_b(0);
#pragma unroll
    for (int kb = 0; kb < NK; ++kb)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = kGemmK * kb + 8 * g4 + j;
        float z = b1[k] + W1[3 * k] * x0 + W1[3 * k + 1] * x1 + W1[3 * k + 2] * x2;
        a[kb][j] = (short)f2bf(silu(z));
      }
  }
  v4f acc[16];
  // W_l[n][k] in k-slabs of 32 (16 KB), staged in LDS once for the block's four
  // waves and double-buffered: slab kb + 1 is fetched while slab kb is used
  const int tid = threadIdx.x;                      // row n of W that this thread stages
  for (int L = 0; L < 3; ++L) {
    const uint16_t* W = wbf + (size_t)L * kHid * kHid;
    const float* bias = P + mlp_off_b(L + 1);
#pragma unroll
    for (int nt = 0; nt < 16; ++nt) acc[nt] = v4f{0.f, 0.f, 0.f, 0.f};
    {
      const uint4* src = reinterpret_cast<const uint4*>(W + (size_t)tid * kHid);
#pragma unroll
      for (int q = 0; q < 4; ++q) *reinterpret_cast<uint4*>(&Ws[0][tid][8 * q]) = src[q];
    }
    __syncthreads();
#pragma unroll
    for (int kb = 0; kb < NK; ++kb) {
      uint4 nxt[4];
      if (kb + 1 < NK) {
        const uint4* src =
            reinterpret_cast<const uint4*>(W + (size_t)tid * kHid + kGemmK * (kb + 1));
#pragma unroll
        for (int q = 0; q < 4; ++q) nxt[q] = src[q];
      }
#pragma unroll
      for (int nt = 0; nt < 16; ++nt) {
        const v8s b = *reinterpret_cast<const v8s*>(&Ws[kb & 1][16 * nt + c16][8 * g4]);
        acc[nt] = mfma32(a[kb], b, acc[nt]);
      }
      if (kb + 1 < NK) {
#pragma unroll
        for (int q = 0; q < 4; ++q) *reinterpret_cast<uint4*>(&Ws[(kb + 1) & 1][tid][8 * q]) = nxt[q];
      }
      __syncthreads();
    }
    if (L < 2) {
#pragma unroll
      for (int nt = 0; nt < 16; ++nt) {
        const float bn = bias[16 * nt + c16];
#pragma unroll
        for (int r = 0; r < 4; ++r) T[w][4 * g4 + r][16 * nt + c16] = f2bf(silu(acc[nt][r] + bn));
      }
      __syncthreads();
#pragma unroll
      for (int kb = 0; kb < NK; ++kb)
        a[kb] = *reinterpret_cast<const v8s*>(&T[w][c16][kGemmK * kb + 8 * g4]);
      __syncthreads();
    }
  }
  const float* w5 = P + mlp_off_w(4);
  const float* b4 = P + mlp_off_b(3);
  float s[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int nt = 0; nt < 16; ++nt) {
    const int n = 16 * nt + c16;
    const float wn = w5[n], bn = b4[n];
#pragma unroll
    for (int r = 0; r < 4; ++r) s[r] += wn * silu(acc[nt][r] + bn);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) s[r] += __shfl_xor(s[r], o, 64);
  if (c16 == 0) {
    const float b5 = P[mlp_off_b(4)];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t m = r0 + 4 * g4 + r;
      if (m < R) y[m] = s[r] + b5;
    }
  }
}

// Adam on the flat parameter vector; refreshes the BF16 copies of W2..W4
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2, uint16_t* __restrict__ wbf) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float gi = g[i];
  float mi = b1 * m[i] + (1.f - b1) * gi;
  float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pi;
  for (int l = 0; l < 3; ++l) {
    int64_t o = mlp_off_w(l + 1);
    if (i >= o && i < o + (int64_t)kHid * kHid) wbf[(int64_t)l * kHid * kHid + (i - o)] = f2bf(pi);
  }
}

__global__ void k_to_bf16(const float* __restrict__ p, uint16_t* __restrict__ wbf) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3ll * kHid * kHid) return;
  int l = (int)(i / ((int64_t)kHid * kHid));
  wbf[i] = f2bf(p[mlp_off_w(l + 1) + (i - (int64_t)l * kHid * kHid)]);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static inline unsigned nb(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

int Mlp::alloc(int batch) {
  if (batch <= cap_batch && params) return FSTAT_OK;
  release_acts();
  int rc;
  auto A = [&](void** p, size_t bytes) { return hip_check(hipMalloc(p, bytes ? bytes : 1), "mlp alloc"); };
  if (!params) {
    if ((rc = A((void**)&params, sizeof(float) * kNParams))) return rc;
    if ((rc = A((void**)&grad, sizeof(float) * kNParams))) return rc;
    if ((rc = A((void**)&m1, sizeof(float) * kNParams))) return rc;
    if ((rc = A((void**)&m2, sizeof(float) * kNParams))) return rc;
    if ((rc = A((void**)&wbf, sizeof(uint16_t) * 3 * kHid * kHid))) return rc;
    if ((rc = A((void**)&red, sizeof(float) * kRedSlices * 4 * kHid))) return rc;
    if ((rc = A((void**)&splitk, sizeof(float) * kSplitK * kHid * kHid))) return rc;
  }
  size_t BH = (size_t)batch * kHid;
  for (int l = 0; l < 4; ++l) {
    if ((rc = A((void**)&z[l], sizeof(float) * BH))) return rc;
    if ((rc = A((void**)&h[l], sizeof(uint16_t) * BH))) return rc;
  }
  if ((rc = A((void**)&dz, sizeof(float) * BH))) return rc;
  if ((rc = A((void**)&dzb, sizeof(uint16_t) * BH))) return rc;
  if ((rc = A((void**)&dh, sizeof(float) * BH))) return rc;
  if ((rc = A((void**)&y, sizeof(float) * batch))) return rc;
  if ((rc = A((void**)&dy, sizeof(float) * batch))) return rc;
  if ((rc = A((void**)&sq, sizeof(float) * batch))) return rc;
  cap_batch = batch;
  return FSTAT_OK;
}

void Mlp::release_acts() {
  for (int l = 0; l < 4; ++l) {
    if (z[l]) (void)hipFree(z[l]);
    if (h[l]) (void)hipFree(h[l]);
    z[l] = nullptr; h[l] = nullptr;
  }
  for (void* p : {(void*)dz, (void*)dzb, (void*)dh, (void*)y, (void*)dy, (void*)sq})
    if (p) (void)hipFree(p);
  dz = nullptr; dzb = nullptr; dh = nullptr; y = nullptr; dy = nullptr; sq = nullptr;
  cap_batch = 0;
}

void Mlp::release() {
  release_acts();
  for (void* p : {(void*)params, (void*)grad, (void*)m1, (void*)m2, (void*)wbf, (void*)red,
                  (void*)splitk, (void*)yinf})
    if (p) (void)hipFree(p);
  params = grad = m1 = m2 = red = splitk = yinf = nullptr;
  cap_inf = 0;
  wbf = nullptr;
}

int Mlp::infer_alloc(int64_t rows) {
  if (yinf && rows <= cap_inf) return FSTAT_OK;
  if (yinf) (void)hipFree(yinf);
  yinf = nullptr;
  cap_inf = 0;
  int rc = hip_check(hipMalloc((void**)&yinf, sizeof(float) * (rows > 0 ? rows : 1)), "mlp alloc");
  if (!rc) cap_inf = rows;
  return rc;
}

void Mlp::infer(const float* x, int64_t rows, hipStream_t s) {
  if (rows <= 0) return;
  hipLaunchKernelGGL(k_mlp_infer, dim3(nb(rows, 64)), dim3(256), 0, s, x, rows, params, wbf, yinf);
}

void Mlp::refresh_bf16(hipStream_t s) {
  hipLaunchKernelGGL(k_to_bf16, dim3(nb(3ll * kHid * kHid, 256)), dim3(256), 0, s, params, wbf);
}

// forward on B rows of x (B multiple of 64); tgt may be NULL
void Mlp::forward(const float* x, const float* tgt, int B, hipStream_t s) {
  const float* P = params;
  hipLaunchKernelGGL(k_layer_in, dim3(nb((int64_t)B * kHid, 256)), dim3(256), 0, s, x, B,
                     P + mlp_off_w(0), P + mlp_off_b(0), z[0], h[0]);
  for (int l = 1; l < 4; ++l) {
    // Z_l = H_{l-1} W_l^T + b_l:  A = H (row-major, ld kHid), B(k,n) = W_l[n][k]
    hipLaunchKernelGGL((k_gemm_bf16<kEpiFwd>), dim3(kHid / 64, B / 64), dim3(256), 0, s, h[l - 1],
                       (int64_t)kHid, (int64_t)1, wbf + (size_t)(l - 1) * kHid * kHid, (int64_t)1,
                       (int64_t)kHid, B, kHid, kHid, z[l], (int64_t)kHid, P + mlp_off_b(l), h[l],
                       (int64_t)kHid, kHid, (int64_t)0);
  }
  hipLaunchKernelGGL(k_layer_out, dim3(nb((int64_t)B * 64, 256)), dim3(256), 0, s, z[3], B,
                     P + mlp_off_w(4), P + mlp_off_b(4), tgt, y, dy, sq);
}

// backward after forward(x, tgt): fills grad (flat layout)
void Mlp::backward(const float* x, int B, hipStream_t s) {
  float* G = grad;
  const int sl = B / 64 < kRedSlices ? B / 64 : kRedSlices;
  int ks = kSplitK;
  while (ks > 1 && (B % (kGemmK * ks))) ks >>= 1;
  // dW5[k] = sum_m dy[m] SiLU(z4[m][k]); db5 = sum_m dy[m]
  hipLaunchKernelGGL((k_colred<1, 1, true>), dim3(kHid / 64, sl), dim3(256), 0, s, z[3], B, dy, 1, red);
  hipLaunchKernelGGL(k_colfin<1>, dim3(1), dim3(kHid), 0, s, red, sl,
                     RedOut{{G + mlp_off_w(4), nullptr, nullptr, nullptr}, {1, 0, 0, 0}});
  hipLaunchKernelGGL(k_sum_dy, dim3(1), dim3(256), 0, s, dy, B, G + mlp_off_b(4));
  hipLaunchKernelGGL(k_out_back, dim3(nb((int64_t)B * kHid, 256)), dim3(256), 0, s, z[3], B,
                     params + mlp_off_w(4), dy, dz, dzb);
  for (int l = 3; l >= 1; --l) {
    // dW_l = dZ_l^T H_{l-1}: A(m,k) = dZ[k][m], B(k,n) = H_{l-1}[k][n]; K = B split
    // into kSplitK slices (16 blocks would not fill the chip), then summed in order
    hipLaunchKernelGGL((k_gemm_bf16<kEpiStore>), dim3(kHid / 64, kHid / 64, ks), dim3(256), 0, s,
                       dzb, (int64_t)1, (int64_t)kHid, h[l - 1], (int64_t)kHid, (int64_t)1, kHid,
                       kHid, B, splitk, (int64_t)kHid, nullptr, nullptr, (int64_t)0, B / ks,
                       (int64_t)kHid * kHid);
    hipLaunchKernelGGL(k_splitsum, dim3(nb((int64_t)kHid * kHid, 256)), dim3(256), 0, s, splitk,
                       ks, G + mlp_off_w(l));
    hipLaunchKernelGGL((k_colred<1, 0, false>), dim3(kHid / 64, sl), dim3(256), 0, s, dz, B,
                       (const float*)nullptr, 0, red);
    hipLaunchKernelGGL(k_colfin<1>, dim3(1), dim3(kHid), 0, s, red, sl,
                       RedOut{{G + mlp_off_b(l), nullptr, nullptr, nullptr}, {1, 0, 0, 0}});
    // dH_{l-1} = dZ_l W_l: A = dZ (ld kHid), B(k,n) = W_l[k][n]
    hipLaunchKernelGGL((k_gemm_bf16<kEpiStore>), dim3(kHid / 64, B / 64), dim3(256), 0, s, dzb,
                       (int64_t)kHid, (int64_t)1, wbf + (size_t)(l - 1) * kHid * kHid,
                       (int64_t)kHid, (int64_t)1, B, kHid, kHid, dh, (int64_t)kHid, nullptr,
                       nullptr, (int64_t)0, kHid, (int64_t)0);
    hipLaunchKernelGGL(k_act_back, dim3(nb((int64_t)B * kHid, 256)), dim3(256), 0, s, dh,
                       z[l - 1], (int64_t)B * kHid, dz, dzb);
  }
  // dW1[n][k] = sum_m dz1[m][n] x[m][k]; db1[n] = sum_m dz1[m][n]
  hipLaunchKernelGGL((k_colred<4, 3, false>), dim3(kHid / 64, sl), dim3(256), 0, s, dz, B, x, 3, red);
  hipLaunchKernelGGL(k_colfin<4>, dim3(1), dim3(kHid), 0, s, red, sl,
                     RedOut{{G + mlp_off_w(0), G + mlp_off_w(0) + 1, G + mlp_off_w(0) + 2,
                             G + mlp_off_b(0)}, {3, 3, 3, 1}});
}

void Mlp::adam(int t, float lr, hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3(nb(kNParams, 256)), dim3(256), 0, s, params, grad, m1, m2,
                     (int64_t)kNParams, lr, b1, b2, eps, c1, c2, wbf);
}

}  // namespace fstat

using namespace fstat;

extern "C" int fstat_mlp_grad(const float* params, const float* x, const float* t, int32_t B,
                              double* loss, float* grad, float* y_out) {
  if (!params || !x || !t || B < 64 || (B % 64) || !loss || !grad)
    return set_error(FSTAT_EINVAL, "fstat_mlp_grad: bad arguments (B must be a multiple of 64)");
  Mlp net;
  int rc = net.alloc(B);
  float *dx = nullptr, *dt = nullptr;
  if (!rc) rc = hip_check(hipMalloc(&dx, sizeof(float) * 3 * B), "alloc x");
  if (!rc) rc = hip_check(hipMalloc(&dt, sizeof(float) * B), "alloc t");
  hipStream_t s = nullptr;
  if (!rc) rc = hip_check(hipMemcpy(net.params, params, sizeof(float) * kNParams, hipMemcpyHostToDevice), "copy");
  if (!rc) rc = hip_check(hipMemcpy(dx, x, sizeof(float) * 3 * B, hipMemcpyHostToDevice), "copy");
  if (!rc) rc = hip_check(hipMemcpy(dt, t, sizeof(float) * B, hipMemcpyHostToDevice), "copy");
  if (!rc) {
    net.refresh_bf16(s);
    net.forward(dx, dt, B, s);
    net.backward(dx, B, s);
    rc = hip_check(hipGetLastError(), "mlp launch");
  }
  std::vector<float> sq(B);
  if (!rc) rc = hip_check(hipMemcpy(grad, net.grad, sizeof(float) * kNParams, hipMemcpyDeviceToHost), "copy grad");
  if (!rc) rc = hip_check(hipMemcpy(sq.data(), net.sq, sizeof(float) * B, hipMemcpyDeviceToHost), "copy loss");
  if (!rc && y_out) rc = hip_check(hipMemcpy(y_out, net.y, sizeof(float) * B, hipMemcpyDeviceToHost), "copy y");
  if (!rc) {
    double l = 0.0;
    for (int i = 0; i < B; ++i) l += sq[i];
    *loss = l / B;
  }
  if (dx) (void)hipFree(dx);
  if (dt) (void)hipFree(dt);
  net.release();
  return rc;
}

extern "C" int fstat_mlp_forward(const float* params, const float* x, int64_t R, float* y) {
  if (!params || !x || !y || R < 1 || R > ((int64_t)1 << 31))
    return set_error(FSTAT_EINVAL, "fstat_mlp_forward: bad arguments");
  Mlp net;
  int rc = hip_check(hipMalloc((void**)&net.params, sizeof(float) * kNParams), "alloc params");
  if (!rc) rc = hip_check(hipMalloc((void**)&net.wbf, sizeof(uint16_t) * 3 * kHid * kHid), "alloc wbf");
  if (!rc) rc = net.infer_alloc(R);
  float* dx = nullptr;
  if (!rc) rc = hip_check(hipMalloc(&dx, sizeof(float) * 3 * R), "alloc x");
  hipStream_t s = nullptr;
  if (!rc) rc = hip_check(hipMemcpy(net.params, params, sizeof(float) * kNParams, hipMemcpyHostToDevice), "copy");
  if (!rc) rc = hip_check(hipMemcpy(dx, x, sizeof(float) * 3 * R, hipMemcpyHostToDevice), "copy");
  if (!rc) {
    net.refresh_bf16(s);
    net.infer(dx, R, s);
    rc = hip_check(hipGetLastError(), "mlp launch");
  }
  if (!rc) rc = hip_check(hipMemcpy(y, net.yinf, sizeof(float) * R, hipMemcpyDeviceToHost), "copy y");
  if (dx) (void)hipFree(dx);
  net.release();
  return rc;
}
