// fstat_kernels.hip -- gfx950 kernels of the batched semi-coherent F-statistic.
//
// One evaluation (Sec. II.B, Eq. semi-cohF of arXiv:2407.10797) is a chain of
// small kernels around one heavy one:
//   k_setup         one wavefront per particle: intrinsic parameters -> PN
//                   constants, sky frame, support [f_lo, f_hi] (t_f inverted by
//                   a 64-point search), Np partition edges (bin indices) and the
//                   work-item counts: a work item is the part of a partition
//                   inside one tile of the global tiling of the band
//   k_scan_*        exclusive scan of the work-item counts (three passes)
//   k_fill          work list: item -> (particle*stride + partition, tile index)
//   k_interp_nodes  exact template at 10 Chebyshev nodes and both ends of every
//                   item -> interpolation record, or hand-over to the exact loop
//   k_tile_*        items grouped by tile; scheduling units of <= 32 items
//   k_eval_interp   persistent blocks take units dynamically, stage the tile's
//                   data in LDS, and evaluate the interpolated template at every
//                   bin of each item (FP64: advanced by a difference recurrence
//                   along each lane's run of bins): the N-term sums per item
//                   (deterministic, no float atomics); the M-terms come from the
//                   node kernel's quadrature
//   k_eval_exact    the exact template at every bin, for handed-over items, for
//                   refinement and under FSTAT_EVAL_EXACT (FP64 and mixed)
//   k_mark          partitions whose interpolation error could matter -> exact
//   k_solve         one thread per (particle, partition): ordered sum of the
//                   item partials and the 2x2 Hermitian closed form of F_l
//   k_mean          one wavefront per particle: F_hat = mean_l F_l, or -inf / NaN
#include "fstat_internal.h"
#include <type_traits>

#include "fstat_kernels.h"
#include "philox.h"

namespace fstat {

// ---------------------------------------------------------------------------
// plan-time per-bin preparation
// ---------------------------------------------------------------------------
// C(f) = (1 - z^2)(-i pi f L) exp(-i pi f L), z = exp(-2 i pi f L): the part of
// the TDI-X transfer shared by every template.  With g = f^{-7/6} e^{-i Psi}
// (App. A) and <a,b> = 4 df Re sum a conj(b) / S (Sec. II.A):
//   w_j = 4 df s_j conj(C_j) f_j^{-7/6} / S_j,   u_j = 4 df |C_j|^2 f_j^{-7/3} / S_j.
__global__ void k_prep(Grid g, const double* __restrict__ data, const double* __restrict__ psd,
                       double* __restrict__ wr, double* __restrict__ wi, double* __restrict__ u,
                       double* __restrict__ s0, double* __restrict__ c0) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= g.nbins) return;
  const int64_t jc = (int64_t)blockIdx.y * g.nbins + j;   // channel blockIdx.y
  double f = (double)(g.k_lo + j) * g.df;
  double s, c;
  sincospi(kLs * f, &s, &c);
  double x0 = kPi * kLs * f;
  double zr = c * c - s * s, zi = -2.0 * s * c;
  double omr = 1.0 - (zr * zr - zi * zi), omi = -2.0 * zr * zi;  // 1 - z^2
  double er = -x0 * s, ei = -x0 * c;                               // -i x0 e^{-i x0}
  double Cr = omr * er - omi * ei, Ci = omr * ei + omi * er;
  double amp = pow(f, -7.0 / 6.0);
  double wgt = 4.0 * g.df / psd[jc];
  double dr = data[2 * jc], di = data[2 * jc + 1];
  // s conj(C)
  double pr = dr * Cr + di * Ci, pi = di * Cr - dr * Ci;
  wr[jc] = wgt * amp * pr;
  wi[jc] = wgt * amp * pi;
  u[jc] = wgt * amp * amp * (Cr * Cr + Ci * Ci);
  if (blockIdx.y == 0) {
    s0[j] = s;
    c0[j] = c;
  }
}

// max of u over the band (one block, grid-stride) -> *out
__global__ void k_max(const double* __restrict__ u, int64_t n, double* __restrict__ out) {
  __shared__ double red[1024];
  double m = 0.0;
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) m = fmax(m, u[j]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// Normalise so that max u = 1: F is invariant under (w, u) -> (g w, g^2 u)
// (a rescaling of the template), and FP32 copies stay in range.
__global__ void k_scale(Grid g, const double* __restrict__ umax, double* __restrict__ wr,
                        double* __restrict__ wi, double* __restrict__ u,
                        const double* __restrict__ s0, const double* __restrict__ c0,
                        float* __restrict__ wr32, float* __restrict__ wi32,
                        float* __restrict__ u32, float* __restrict__ s032,
                        float* __restrict__ c032) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= g.nbins) return;
  const int64_t jc = (int64_t)blockIdx.y * g.nbins + j;   // channel blockIdx.y
  double m = umax[0];
  double gam2 = (m > 0.0) ? 1.0 / m : 1.0;
  double gam = sqrt(gam2);
  double a = wr[jc] * gam, b = wi[jc] * gam, c = u[jc] * gam2;
  wr[jc] = a; wi[jc] = b; u[jc] = c;
  if (wr32) {
    wr32[jc] = (float)a; wi32[jc] = (float)b; u32[jc] = (float)c;
    if (blockIdx.y == 0) { s032[j] = (float)s0[j]; c032[j] = (float)c0[j]; }
  }
}

// ---------------------------------------------------------------------------
// particle setup: constants, support, partition boundaries, work counts
// ---------------------------------------------------------------------------
__device__ __forceinline__ double bin_freq(const Grid& g, int64_t j) {
  return (double)(g.k_lo + j) * g.df;
}

// Work item c of a partition with bins [a, b): its part inside bin tile
// a / T + c of the global tiling of the band into tiles of T bins.
__device__ __forceinline__ int item_tile(int a, int c, int T) { return a / T + c; }
// With several channels a partition has (tiles met) x (channels) items:
// item c covers tile offset c / nch of channel c % nch.
__device__ __forceinline__ void item_split(int c, int nch, int& ct, int& ch) {
  ct = c / nch;
  ch = c - ct * nch;
}
// The item's tile in the numbering of all channels' tiles, channel by
// channel (ntiles = nch x tiles per channel).
__device__ __forceinline__ int item_xtile(int a, int c, int T, int nch, int ntiles) {
  int ct, ch;
  item_split(c, nch, ct, ch);
  return ch * (ntiles / nch) + item_tile(a, ct, T);
}
__device__ __forceinline__ void item_bins(int a, int b, int c, int T, int& b0, int& b1) {
  const int t = a / T + c;
  b0 = max(a, t * T);
  b1 = min(b, (t + 1) * T);
}

// smallest j in [lo, hi+1] with f_j >= e
__device__ int first_bin_at_or_above(const Grid& g, double e, int lo, int hi) {
  double jd = ceil(e / g.df) - (double)g.k_lo;
  int j = (jd < (double)lo) ? lo : (jd > (double)(hi + 1) ? hi + 1 : (int)jd);
  while (j > lo && bin_freq(g, j - 1) >= e) --j;
  while (j <= hi && bin_freq(g, j) < e) ++j;
  return j;
}

__device__ double tf_only(const PartConst& P, double f) {
  double fr, tf;
  phase_and_tf(P, f, fr, tf);
  return tf;
}

// Frequency where t_f (increasing in f) reaches t on [fa, fb], by one
// wavefront: rounds of a 64-point search (each lane evaluates one interior
// point, the ballot of points below t brackets the root; 65x narrower per
// round) down to a few ulps, then bisection to the double resolution.
__device__ double invert_tf(const PartConst& P, double t, double fa, double fb, int lane) {
  for (int it = 0; it < 12; ++it) {
    const double h = (fb - fa) * (1.0 / 65.0);
    if (!(h > 64.0 * 2.3e-16 * fb)) break;
    const double f = fa + h * (double)(lane + 1);
    const uint64_t below = __ballot(tf_only(P, f) < t);
    const int k = __popcll(below);                 // points below t (a prefix: t_f increases)
    const double nfa = k > 0 ? fa + h * (double)k : fa;
    const double nfb = k < 64 ? fa + h * (double)(k + 1) : fb;
    fa = nfa;
    fb = fmin(nfb, fb);
  }
  for (int it = 0; it < 200; ++it) {
    const double fm = 0.5 * (fa + fb);
    if (fm <= fa || fm >= fb) break;
    if (tf_only(P, fm) < t) fa = fm; else fb = fm;
  }
  return fb;
}

// One wavefront per particle: constants, support, partition edges (one per
// lane), work-item counts.
__global__ __launch_bounds__(256) void k_setup(Grid g, const double* __restrict__ params,
                                               int64_t n, const int32_t* __restrict__ np,
                                               int32_t np_uniform, int32_t stride, int32_t chunk,
                                               const uint8_t* __restrict__ skip,
                                               PartConst* __restrict__ pc,
                                               int32_t* __restrict__ bounds,
                                               int32_t* __restrict__ cnt) {
  const int lane = threadIdx.x & 63;
  const int64_t p = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (p >= n) return;                      // whole wavefronts
  const double* th = params + 6 * p;
  int npi = np ? np[p] : np_uniform;
  PartConst P;
  bool ok = true;
  for (int i = 0; i < 6; ++i) ok = ok && isfinite(th[i]);
  ok = ok && th[1] > 0.0 && fabs(th[2]) < 1.0 && th[5] >= 0.0 && npi >= 1 && npi <= stride;
  int32_t* bp = bounds + p * (int64_t)(stride + 1);
  int32_t* cp = cnt + p * (int64_t)stride;
  for (int l = lane; l < stride; l += 64) cp[l] = 0;
  P.np = npi;
  P.j_lo = 0; P.j_hi = -1;
  if (!ok) {
    P.status = kStatusInvalid;
    if (lane == 0) pc[p] = P;
    return;
  }
  if (skip && skip[p]) {  // outside the search box: not evaluated (let-them-fly)
    P.status = kStatusEmpty;
    if (lane == 0) pc[p] = P;
    return;
  }
  fill_constants(P, th);
  int last = (int)g.nbins - 1;
  double f_first = bin_freq(g, 0), f_last = bin_freq(g, last);
  double t_first = tf_only(P, f_first), t_last = tf_only(P, f_last);
  bool empty = (t_last < 0.0) || (t_first > g.T_obs);
  double flo = 0.0, fhi = 0.0;
  if (!empty) {
    flo = (t_first >= 0.0) ? f_first : invert_tf(P, 0.0, f_first, f_last, lane);
    fhi = (t_last <= g.T_obs) ? f_last : invert_tf(P, g.T_obs, f_first, f_last, lane);
    empty = !(flo <= fhi);
  }
  int jlo = 0, jhi = -1;
  if (!empty) {
    jlo = first_bin_at_or_above(g, flo, 0, last);
    // largest j with f_j <= fhi
    int j = first_bin_at_or_above(g, fhi, 0, last);
    if (j > last || bin_freq(g, j) > fhi) --j;
    jhi = j;
    empty = jlo > jhi;
  }
  P.flo = flo; P.fhi = fhi;
  if (empty) {
    P.status = kStatusEmpty;
    if (lane == 0) pc[p] = P;
    return;
  }
  P.status = kStatusOk;
  P.j_lo = jlo; P.j_hi = jhi;
  if (lane == 0) pc[p] = P;
  // edges e_l = flo + span l / Np: bin bp[l] is the first at or above e_l; each
  // lane computes both edges of its partitions (no exchange between lanes)
  const double span = fhi - flo;
  auto edge = [&](int l) -> int {
    if (l == 0) return jlo;
    if (l == npi) return jhi + 1;
    return first_bin_at_or_above(g, flo + (span * (double)l) / (double)npi, jlo, jhi);
  };
  for (int l = lane; l < npi; l += 64) {
    const int a = edge(l), b = edge(l + 1);
    bp[l] = a;
    if (l == npi - 1) bp[npi] = b;
    cp[l] = b > a ? ((b - 1) / chunk - a / chunk + 1) * g.chan.n : 0;   // tiles met x channels
  }
}

// Exclusive scan of cnt[m] into off[m] in three passes over blocks of
// kScanBlock counts: block sums, a one-block scan of the sums (which also
// writes *total and clears the exact-path counters), then each block's local
// scan plus its offset.
constexpr int kScanBlock = 4096;   // counts per block (1024 threads x 4)

template <typename T>
__device__ __forceinline__ T block_excl_scan(T x, T* sh, T& total) {
  // inclusive scan across the 1024 threads of the block (Hillis-Steele in LDS)
  const int t = threadIdx.x;
  sh[t] = x;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    T y = t >= o ? sh[t - o] : T(0);
    __syncthreads();
    sh[t] += y;
    __syncthreads();
  }
  total = sh[1023];
  T r = sh[t] - x;
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(1024) void k_scan_sums(const int32_t* __restrict__ cnt, int64_t m,
                                                    int32_t* __restrict__ bsum) {
  __shared__ int32_t red[1024];
  const int64_t i0 = (int64_t)blockIdx.x * kScanBlock + 4 * threadIdx.x;
  int32_t v = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) v += (i0 + e < m) ? cnt[i0 + e] : 0;
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = red[0];
}

// nb <= 1024 * 4 block sums (m <= 16.7M counts), one block
__global__ __launch_bounds__(1024) void k_scan_top(int32_t* __restrict__ bsum, int32_t nb,
                                                   int32_t* __restrict__ total,
                                                   int32_t* __restrict__ ndirect,
                                                   int32_t* __restrict__ nrefine) {
  __shared__ int32_t sh[1024];
  const int i0 = 4 * threadIdx.x;
  int32_t v[4], x = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) { v[e] = (i0 + e < nb) ? bsum[i0 + e] : 0; x += v[e]; }
  int32_t tot;
  int32_t run = block_excl_scan(x, sh, tot);
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (i0 + e < nb) { bsum[i0 + e] = run; run += v[e]; }
  if (threadIdx.x == 0) {
    total[0] = tot;
    ndirect[0] = 0;
    nrefine[0] = 0;
  }
}

__global__ __launch_bounds__(1024) void k_scan_apply(const int32_t* __restrict__ cnt, int64_t m,
                                                     const int32_t* __restrict__ bsum,
                                                     int32_t* __restrict__ off) {
  __shared__ int32_t sh[1024];
  const int64_t i0 = (int64_t)blockIdx.x * kScanBlock + 4 * threadIdx.x;
  int32_t v[4], x = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) { v[e] = (i0 + e < m) ? cnt[i0 + e] : 0; x += v[e]; }
  int32_t tot;
  int32_t run = block_excl_scan(x, sh, tot) + bsum[blockIdx.x];
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (i0 + e < m) { off[i0 + e] = run; run += v[e]; }
}

__global__ void k_fill(const int32_t* __restrict__ cnt, const int32_t* __restrict__ off, int64_t m,
                       int2* __restrict__ items) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  int c = cnt[q], o = off[q];
  for (int i = 0; i < c; ++i) items[o + i] = make_int2((int)q, i);
}

// Prefix sums of the per-bin weight u (one channel): out[0] = 0,
// out[j + 1] = u_0 + ... + u_j.  The refinement estimate takes an item's
// sum of u from two entries.  Same three passes as the count scan.
__global__ __launch_bounds__(1024) void k_uscan_sums(const double* __restrict__ u, int64_t n,
                                                     double* __restrict__ bsum) {
  __shared__ double red[1024];
  const int64_t i0 = (int64_t)blockIdx.x * kScanBlock + 4 * threadIdx.x;
  double v = 0.0;
#pragma unroll
  for (int e = 0; e < 4; ++e) v += (i0 + e < n) ? u[i0 + e] : 0.0;
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(1024) void k_uscan_top(double* __restrict__ bsum, int32_t nb) {
  __shared__ double sh[1024];
  const int i0 = 4 * threadIdx.x;
  double v[4], x = 0.0;
#pragma unroll
  for (int e = 0; e < 4; ++e) { v[e] = (i0 + e < nb) ? bsum[i0 + e] : 0.0; x += v[e]; }
  double tot;
  double run = block_excl_scan(x, sh, tot);
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (i0 + e < nb) { bsum[i0 + e] = run; run += v[e]; }
}

__global__ __launch_bounds__(1024) void k_uscan_apply(const double* __restrict__ u, int64_t n,
                                                      const double* __restrict__ bsum,
                                                      double* __restrict__ out) {
  __shared__ double sh[1024];
  const int64_t i0 = (int64_t)blockIdx.x * kScanBlock + 4 * threadIdx.x;
  double v[4], x = 0.0;
#pragma unroll
  for (int e = 0; e < 4; ++e) { v[e] = (i0 + e < n) ? u[i0 + e] : 0.0; x += v[e]; }
  double tot;
  double run = block_excl_scan(x, sh, tot) + bsum[blockIdx.x];
  if (blockIdx.x == 0 && threadIdx.x == 0) out[0] = 0.0;
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (i0 + e < n) { run += v[e]; out[i0 + e + 1] = run; }
}

// ---------------------------------------------------------------------------
// the hot loop, FP64
// ---------------------------------------------------------------------------
__device__ __forceinline__ void kahan_add(double& s, double& c, double x) {
  double y = x - c;
  double t = s + y;
  c = (t - s) - y;
  s = t;
}
__device__ __forceinline__ void kahan_addf(float& s, float& c, float x) {
  float y = x - c;
  float t = s + y;
  c = (t - s) - y;
  s = t;
}

// Sums of eight per-lane values over the wavefront in 10 exchanges instead of
// 8 x 6: each step hands half of the remaining values to the partner lane
// (xor 32, 16, 8), then the last value is summed over lanes xor 4, 2, 1.
// Returns the total of value number idx = 4 b5 + 2 b4 + b3 (b = lane bits);
// lanes with (lane & 7) == 0 hold the eight distinct totals.  Fixed order.
__device__ __forceinline__ double wave_sum8(const double* a, int lane, int& idx) {
  const bool h5 = (lane & 32) != 0, h4 = (lane & 16) != 0, h3 = (lane & 8) != 0;
  double b[4], c[2];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double keep = h5 ? a[4 + i] : a[i], give = h5 ? a[i] : a[4 + i];
    b[i] = keep + __shfl_xor(give, 32, 64);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double keep = h4 ? b[2 + i] : b[i], give = h4 ? b[i] : b[2 + i];
    c[i] = keep + __shfl_xor(give, 16, 64);
  }
  double d = (h3 ? c[1] : c[0]) + __shfl_xor(h3 ? c[0] : c[1], 8, 64);
#pragma unroll
  for (int o = 4; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
  idx = (h5 ? 4 : 0) + (h4 ? 2 : 0) + (h3 ? 1 : 0);
  return d;
}

// The same for four values: idx = 2 b5 + b4; lanes with (lane & 15) == 0
// hold the four totals.
__device__ __forceinline__ double wave_sum4(const double* a, int lane, int& idx) {
  const bool h5 = (lane & 32) != 0, h4 = (lane & 16) != 0;
  double b[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double keep = h5 ? a[2 + i] : a[i], give = h5 ? a[i] : a[2 + i];
    b[i] = keep + __shfl_xor(give, 32, 64);
  }
  double d = (h4 ? b[1] : b[0]) + __shfl_xor(h4 ? b[0] : b[1], 16, 64);
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
  idx = (h5 ? 2 : 0) + (h4 ? 1 : 0);
  return d;
}

constexpr int kSmallItem = 8;   // exact kernel: items this short share a wavefront
constexpr int kBigItem = 256;   // exact kernel: items longer than this take a whole block

// Exact per-bin template loop.  FP64 (MIXED = false): everything in FP64,
// Kahan-compensated per-lane sums.  Mixed (MIXED = true): the phase, the orbit
// and the TDI response are evaluated in FP64 exactly as on the FP64 path and
// rounded once to FP32; the products with the FP32 data and the N-term sums
// (Z+, Zx) are FP32 with Kahan compensation, the M-terms (P, Q, R) are FP64
// sums of the rounded response.  The response is not computed in FP32: its
// sinc factors are formed from sin(x0 (1 +- k.n)) by angle addition and the
// two arms' contributions are subtracted, and in FP32 both cancel (relative
// errors of 1e-6..1e-5 for sources near an arm direction), which tilts the
// (T+, Tx) direction; the statistic amplifies such a tilt by ~sqrt(cond M) in
// the weak eigen-direction of the short, ill-conditioned partitions this
// kernel serves.  Rounding a correct response to FP32 tilts it by ~6e-8 only.
template <bool MIXED>
__global__ __launch_bounds__(256) void k_eval_exact(Grid g,
                                                    const PartConst* __restrict__ pc,
                                                    const int32_t* __restrict__ bounds, int32_t stride,
                                                    const int2* __restrict__ items,
                                                    const int32_t* __restrict__ total, int32_t chunk,
                                                    const double* __restrict__ wr,
                                                    const double* __restrict__ wi,
                                                    const double* __restrict__ u,
                                                    const float* __restrict__ wr32,
                                                    const float* __restrict__ wi32,
                                                    const float* __restrict__ u32,
                                                    const double* __restrict__ s0a,
                                                    const double* __restrict__ c0a,
                                                    const double* __restrict__ ek,
                                                    double* __restrict__ partials,
                                                    const int32_t* __restrict__ sel,
                                                    const int32_t* __restrict__ nsel) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int nwaves = (gridDim.x * blockDim.x) >> 6;
  __shared__ double2 s_tab[kSinTab];              // coarse angles of the template's sin/cos
  __shared__ double s_red[4][8];                  // per-wave sums of a block-wide item
  fill_sincos_table(s_tab);
  // The eight partition terms of bin j for the item (q, c) of a particle;
  // on the mixed path t[0..3] are FP32 products (widened).
  auto terms = [&](int q, int c, int j, double t[8]) {
    const int p = q / stride;
    const PartConst& P = pc[p];
    int ct, ch;
    item_split(c, g.chan.n, ct, ch);
    const int64_t co = (int64_t)ch * g.nbins;   // the channel's data
    const double* ekq = (ek && P.sur) ? ek + 8 * (int64_t)q : nullptr;
    double f = bin_freq(g, j);
    double cps, sps, tpr, tpi, txr, txi;
    template_fp64(P, f, s0a[j], c0a[j], cps, sps, tpr, tpi, txr, txi, ekq, g.chan.code[ch],
                  &g.orb, s_tab);
    if constexpr (MIXED) {
      const float cf = (float)cps, sf = (float)sps;
      const float pr = (float)tpr, pi = (float)tpi, xr = (float)txr, xi = (float)txi;
      const float a = wr32[co + j], b = wi32[co + j];
      const float Wr = a * cf - b * sf, Wi = a * sf + b * cf;   // w e^{i Phi}
      t[0] = (double)(Wr * pr + Wi * pi);
      t[1] = (double)(Wi * pr - Wr * pi);
      t[2] = (double)(Wr * xr + Wi * xi);
      t[3] = (double)(Wi * xr - Wr * xi);
      tpr = pr; tpi = pi; txr = xr; txi = xi;     // M-terms from the same rounded response
      const double uu = (double)u32[co + j];
      t[4] = uu * (tpr * tpr + tpi * tpi);
      t[5] = uu * (txr * txr + txi * txi);
      t[6] = uu * (tpr * txr + tpi * txi);
      t[7] = uu * (tpi * txr - tpr * txi);
    } else {
      double a = wr[co + j], b = wi[co + j], uu = u[co + j];
      double Wr = a * cps - b * sps, Wi = a * sps + b * cps;   // w e^{i Phi}
      t[0] = Wr * tpr + Wi * tpi;     // Z+ = sum W conj(T'+)
      t[1] = Wi * tpr - Wr * tpi;
      t[2] = Wr * txr + Wi * txi;     // Zx
      t[3] = Wi * txr - Wr * txi;
      t[4] = uu * (tpr * tpr + tpi * tpi);
      t[5] = uu * (txr * txr + txi * txi);
      t[6] = uu * (tpr * txr + tpi * txi);   // R = sum u T'+ conj(T'x)
      t[7] = uu * (tpi * txr - tpr * txi);
    }
  };
  auto bins_of = [&](int w, int& q, int& c, int& b0, int& b1) {
    const int2 it = items[w];
    q = it.x;
    c = it.y;
    const int p = q / stride, l = q - p * stride;
    const int32_t* bp = bounds + (int64_t)p * (stride + 1);
    int ct, ch;
    item_split(c, g.chan.n, ct, ch);
    item_bins(bp[l], bp[l + 1], ct, chunk, b0, b1);
  };
  // All items, or only those listed in sel (the interpolating kernel's
  // rejects and refinements).  Items of at most kSmallItem bins go in groups
  // of eight list entries per wavefront, eight lanes each (one bin per lane,
  // then a fixed three-step butterfly); larger ones one per wavefront in a
  // second sweep over the list, so that a list of long items (the refinement
  // pass) spreads over the whole grid, and on a short list those above
  // kBigItem bins one per block in a third.  Which path an item takes depends
  // on the item and the list's length alone, so its sums do not depend on the
  // order of the list.
  const int W = sel ? nsel[0] : total[0];
  const int G = (W + 7) >> 3;
  for (int gi = wave; gi < G; gi += nwaves) {
    const int slot = gi * 8 + (lane >> 3);
    const bool have = slot < W;
    int w = 0, q = 0, c = 0, b0 = 0, b1 = 0;
    if (have) {
      w = sel ? sel[slot] : slot;
      bins_of(w, q, c, b0, b1);
    }
    const bool small = have && b1 - b0 <= kSmallItem;
    if (!__any(small)) continue;
    double t[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) t[i] = 0.0;
    const int j = b0 + (lane & 7);
    if (small && j < b1) terms(q, c, j, t);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      t[i] += __shfl_xor(t[i], 4, 64);
      t[i] += __shfl_xor(t[i], 2, 64);
      t[i] += __shfl_xor(t[i], 1, 64);
    }
    if (small && (lane & 7) == 0) {
#pragma unroll
      for (int i = 0; i < 8; ++i) partials[(int64_t)w * 8 + i] = t[i];
    }
  }
  // Kahan-compensated sums of this thread's bins j0, j0 + step, ... < j1 of
  // one item (true sum ~ acc - cmp, returned compensated): the partition
  // matrix can have cond ~ 1e5..1e8, which amplifies summation error.
  auto thread_sums = [&](int qb, int cb, int j0, int j1, int step, double* acc) {
    double cmp[8];
    float accf[4], cmpf[4];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = cmp[i] = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) accf[i] = cmpf[i] = 0.0f;
    for (int j = j0; j < j1; j += step) {
      double tt[8];
      terms(qb, cb, j, tt);
      if constexpr (MIXED) {
#pragma unroll
        for (int i = 0; i < 4; ++i) kahan_addf(accf[i], cmpf[i], (float)tt[i]);
#pragma unroll
        for (int i = 4; i < 8; ++i) kahan_add(acc[i], cmp[i], tt[i]);
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) kahan_add(acc[i], cmp[i], tt[i]);
      }
    }
    if constexpr (MIXED) {
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[i] = (double)accf[i] - (double)cmpf[i];
#pragma unroll
      for (int i = 4; i < 8; ++i) acc[i] -= cmp[i];
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) acc[i] -= cmp[i];
    }
  };
  // A short list (rejects, refinement) leaves most wavefronts idle while a few
  // take its long items: there items above kBigItem bins take a whole block.
  // A long list (every item, FSTAT_EVAL_EXACT) fills the grid one item per
  // wavefront.
  const bool by_block = W < 4 * nwaves;
  // items of kSmallItem + 1 bins and more (up to kBigItem for a short list):
  // one per wavefront
  for (int slot = wave; slot < W; slot += nwaves) {
    // the slot is the same on every lane: keep the item's indices scalar
    const int wb = __builtin_amdgcn_readfirstlane(sel ? sel[slot] : slot);
    int qb, cb, bb0, bb1;
    bins_of(wb, qb, cb, bb0, bb1);
    qb = __builtin_amdgcn_readfirstlane(qb);
    cb = __builtin_amdgcn_readfirstlane(cb);
    bb0 = __builtin_amdgcn_readfirstlane(bb0);
    bb1 = __builtin_amdgcn_readfirstlane(bb1);
    if (bb1 - bb0 <= kSmallItem || (by_block && bb1 - bb0 > kBigItem)) continue;
    double acc[8];
    thread_sums(qb, cb, bb0 + lane, bb1, 64, acc);
    int idx;
    const double tot = wave_sum8(acc, lane, idx);
    if ((lane & 7) == 0) partials[(int64_t)wb * 8 + idx] = tot;
  }
  // longer items: one per block (a few long rejects or refined items would
  // otherwise each hold one wavefront for the whole pass); the four waves'
  // sums are added in a fixed order
  for (int slot = blockIdx.x; by_block && slot < W; slot += gridDim.x) {
    const int wb = __builtin_amdgcn_readfirstlane(sel ? sel[slot] : slot);
    int qb, cb, bb0, bb1;
    bins_of(wb, qb, cb, bb0, bb1);
    qb = __builtin_amdgcn_readfirstlane(qb);
    cb = __builtin_amdgcn_readfirstlane(cb);
    bb0 = __builtin_amdgcn_readfirstlane(bb0);
    bb1 = __builtin_amdgcn_readfirstlane(bb1);
    if (bb1 - bb0 <= kBigItem) continue;         // the same for every thread of the block
    double acc[8];
    thread_sums(qb, cb, bb0 + (int)threadIdx.x, bb1, (int)blockDim.x, acc);
    int idx;
    const double tot = wave_sum8(acc, lane, idx);
    if ((lane & 7) == 0) s_red[threadIdx.x >> 6][idx] = tot;
    __syncthreads();
    if (threadIdx.x < 8)
      partials[(int64_t)wb * 8 + threadIdx.x] =
          ((s_red[0][threadIdx.x] + s_red[1][threadIdx.x]) + s_red[2][threadIdx.x]) +
          s_red[3][threadIdx.x];
    __syncthreads();                              // s_red is rewritten by the next item
  }
}

// ---------------------------------------------------------------------------
// the hot loop, interpolating form (default)
// ---------------------------------------------------------------------------
// Within one work item (at most `chunk` consecutive bins of one partition)
// every factor of the template except the fast phase is smooth in f, and the
// phase is smooth once a linear term is taken out.  Per item, with m = j - b0
// and s = 2 m / (nb - 1) - 1 in [-1, 1]:
//   Phi(m) / (2 pi) = Phi_0 + B m + R(s),   R(-1) = R(+1) = 0 up to rounding,
// where Phi_0 is the whole phase (cycles, double-double) at the first bin and
// B the secant slope to the last bin; R and the four real components of the
// transfer (T''_+, T''_x) are replaced by their degree-9 interpolants through
// the 10 Chebyshev points of the first kind, written as monomials in s.  The
// node values and the two end-point values are evaluated exactly
// (template_node); an item whose interpolants miss either end point by more
// than 1e-12 cycles (phase; the exact phase itself carries ~1e-13) or 2e-13 of
// the largest transfer component, or that has fewer than kMinInterp bins,
// goes to the exact per-bin kernels (sel list).
// Items whose interpolation error could move their partition's F by more
// than the plan's refinement budget (default 5e-10, relative; the first-order
// estimate of k_mark) are evaluated again exactly.
// Node evaluation packs 5 items x 12 points onto one wavefront's lanes.
constexpr int kCheb = 10;
constexpr int kLanesItem = kCheb + 2;
constexpr int kItemsWave = 5;
constexpr int kMinInterp = 32;
constexpr double kInterpTolPhase = 1e-12;
constexpr double kInterpTolT = 2e-13;
constexpr int kUnitItems = 64;      // items per scheduling unit of the bin loop
constexpr double kTruncFloor = 6e-14;  // FP64 transfer truncation allowance
// Difference recurrence of the FP64 bin loop: shortest lane run that takes
// it (below, the set-up of about 160 operations per lane costs more than the
// ~15 it saves per bin), the largest |phi| of its series, and the largest
// phase error allowed from the neglected fifth difference [rad].
constexpr int kRecMinRun = 9;
constexpr double kRecPhiMax = 4e-3;
constexpr double kRecTrunc = 1e-13;
constexpr double kTwoPi = 6.283185307179586477;
// kStirF[k][j] = j! S(k, j) (S: Stirling numbers of the second kind), the
// j-th forward difference of t^k at t = 0; equivalently
// t^k = sum_j kStirF[k][j] C(t, j)
constexpr double kStirF[kCheb][kCheb] = {
    {1, 0, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 1, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 1, 2, 0, 0, 0, 0, 0, 0, 0},
    {0, 1, 6, 6, 0, 0, 0, 0, 0, 0},
    {0, 1, 14, 36, 24, 0, 0, 0, 0, 0},
    {0, 1, 30, 150, 240, 120, 0, 0, 0, 0},
    {0, 1, 62, 540, 1560, 1800, 720, 0, 0, 0},
    {0, 1, 126, 1806, 8400, 16800, 15120, 5040, 0, 0},
    {0, 1, 254, 5796, 40824, 126000, 191520, 141120, 40320, 0},
    {0, 1, 510, 18150, 186480, 834120, 1905120, 2328480, 1451520, 362880}};

__constant__ double c_cheb_s[kCheb];          // nodes cos(pi (k + 1/2) / 10)
// (sin, cos)(2 pi k / kSinTab) for the FP64 bin loop, which needs it only in
// the per-lane set-up of the difference recurrence and in the direct form
// (its LDS holds the tile instead)
__constant__ double2 c_sincos[kSinTab];
// Row tables of the node kernel, indexed [node kn][lane k of the item]: on a
// node lane (k < kCheb) the map node value kn -> monomial coefficient of s^k
// of the interpolant, on the end lanes k = kCheb, kCheb + 1 the map node
// value kn -> interpolant at s = -1, +1.
__constant__ double c_row9[kCheb][kLanesItem];      // degree-9 interpolant
// The mixed path's transfer interpolants: the Chebyshev series truncated
// after degree kDegT (its error, ~1e-10 on paper-scale items, is far below FP32
// rounding); node rows above kDegT are zero.  Items whose series truncated
// after degree kDegTLow stays within kInterpTolTMixed at both ends take that
// one (4 FP32 additions per bin fewer); degree 4 for every item would
// send enough items to the exact loop to cost more than it saves.
constexpr int kDegT = 6;
constexpr int kDegTLow = 4;
__constant__ double c_row6[kCheb][kLanesItem];
__constant__ double c_row4[kCheb][kLanesItem];
// Mixed loop: forward differences of the phase carried per bin where the
// rest may be dropped, and the largest phase error [turns] that dropping them
// may cause (the FP32 sine's own error is ~1e-7 turns).
constexpr int kMixDiff = 4;
constexpr double kMixTrunc = 1e-9;
// The FP64 loop's transfer interpolants may be truncated after degree 5 or 7
// per item when that keeps them within the item's own error (most paper-scale
// items need 5-7 of the 10 Chebyshev terms at the 2e-13 bar).
__constant__ double c_rowt[2][kCheb][kLanesItem];   // [0]: degree 5, [1]: degree 7
// Quadrature of an item's interpolant: sum over its bins of the degree-9
// interpolant through the nodes = sum_k W_k g(s_k), W_k = sum_j c_jk S_j(nb)
// with c_jk the node-to-Chebyshev-coefficient map and S_j(nb) = sum_m T_j(s_m)
// (zero for odd j: the bins are symmetric in s).  c_cheb_D[i][k] = c_{2i,k}.
__constant__ double c_cheb_D[5][kCheb];
// Least-squares fit of u on a u-tile: inverse Gram matrix of T_0..T_9 on the
// kUTile equispaced points s_m = 2m/(kUTile-1) - 1.
__constant__ double c_ufit_Ginv[kUCoef][kUCoef];

__device__ __forceinline__ double readlane_d(double x, int l) {
  int2 v = *reinterpret_cast<int2*>(&x);
  v.x = __builtin_amdgcn_readlane(v.x, l);
  v.y = __builtin_amdgcn_readlane(v.y, l);
  return *reinterpret_cast<double*>(&v);
}

template <typename T>
__device__ __forceinline__ T horner(const T* c, T s) {
  T r = c[kCheb - 1];
#pragma unroll
  for (int n = kCheb - 2; n >= 0; --n) r = r * s + c[n];
  return r;
}

template <int D, typename T>
__device__ __forceinline__ T horner_n(const T* c, T s) {
  T r = c[D];
#pragma unroll
  for (int n = D - 1; n >= 0; --n) r = r * s + c[n];
  return r;
}

// The same degree-9 polynomial by Estrin's scheme, with the powers s^2, s^4,
// s^8 shared by the five polynomials of a bin: 9 FMAs as in Horner's rule,
// but a dependency depth of 4 instead of 9.
static_assert(kCheb == 10, "estrin9 is written for degree 9");
__device__ __forceinline__ double estrin9(const double* c, double s, double s2, double s4,
                                          double s8) {
  const double q01 = fma(c[1], s, c[0]), q23 = fma(c[3], s, c[2]);
  const double q45 = fma(c[5], s, c[4]), q67 = fma(c[7], s, c[6]);
  const double q89 = fma(c[9], s, c[8]);
  const double a = fma(q23, s2, q01), b = fma(q67, s2, q45);
  return fma(q89, s8, fma(b, s4, a));
}

// Degree-D Estrin forms of the same monomial series (D = 5, 7) for the FP64
// loop's transfer interpolants truncated by the node kernel.
template <int D>
__device__ __forceinline__ double estrin_d(const double* c, double s, double s2, double s4,
                                           double s8) {
  static_assert(D == 5 || D == 7 || D == 9, "degree 5, 7 or 9");
  if constexpr (D == 9) {
    return estrin9(c, s, s2, s4, s8);
  } else if constexpr (D == 7) {
    const double q01 = fma(c[1], s, c[0]), q23 = fma(c[3], s, c[2]);
    const double q45 = fma(c[5], s, c[4]), q67 = fma(c[7], s, c[6]);
    return fma(fma(q67, s2, q45), s4, fma(q23, s2, q01));
  } else {
    const double q01 = fma(c[1], s, c[0]), q23 = fma(c[3], s, c[2]);
    const double q45 = fma(c[5], s, c[4]);
    return fma(q45, s4, fma(q23, s2, q01));
  }
}

// Per-item interpolation record: monomial coefficients of R (kCheb), then of
// Re T''_+, Im T''_+, Re T''_x, Im T''_x (nT each: kCheb, or kDegT + 1 on the
// mixed path), then A = frac(Phi_0), B' = B - rint(B), B, the item's state
// (0: the exact loop takes it; 1: interpolated; the FP64 bin loop sets 2 when
// it took the difference recurrence), the degree the FP64 loop evaluates the
// transfer interpolants at (5, 7 or 9), the item's first bin within its tile
// and its bin count, the step alpha = 2 / (bins - 1) of s per bin and -B / df
// (so that the bin loop needs nothing else per item, and no division).
constexpr int kRec = 5 * kCheb + 9;
static_assert(kRec == kInterpRec && kRec <= 64, "record layout");
template <bool MIXED> struct RecLayout {
  static constexpr int nT = MIXED ? kDegT + 1 : kCheb;
  static constexpr int tail = kCheb + 4 * nT;   // A, B', B, state, degree, first bin, bins, alpha, -B/df
};

// Chebyshev series sum_k c_k T_k(x) (Clenshaw).
__device__ __forceinline__ double cheb_eval10(const double* __restrict__ c, double x) {
  double b1 = 0.0, b2 = 0.0;
  const double x2 = 2.0 * x;
#pragma unroll
  for (int k = kUCoef - 1; k >= 1; --k) {
    const double b0 = fma(x2, b1, c[k] - b2);
    b2 = b1;
    b1 = b0;
  }
  return fma(x, b1, c[0] - b2);
}

// S_j(nb) = sum_{m < nb} T_j(2m/(nb-1) - 1) for j = 0, 2, .., 8, one nb per
// thread (Neumaier sums); S_j(1) = T_j(0) stands for the single bin at s = 0
// and S_j(0) = 0.
__global__ void k_cheb_sums(double* __restrict__ out) {
  const int nb = blockIdx.x * blockDim.x + threadIdx.x;
  if (nb > kSsumMax) return;
  double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, e[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int m = 0; m < nb; ++m) {
    const double s = nb > 1 ? 2.0 * (double)m / (double)(nb - 1) - 1.0 : 0.0;
    double tv[9];
    tv[0] = 1.0;
    tv[1] = s;
#pragma unroll
    for (int j = 2; j <= 8; ++j) tv[j] = fma(2.0 * s, tv[j - 1], -tv[j - 2]);
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      const double x = tv[2 * i], tt = a[i] + x;
      e[i] += (fabs(a[i]) >= fabs(x)) ? (a[i] - tt) + x : (x - tt) + a[i];
      a[i] = tt;
    }
  }
#pragma unroll
  for (int i = 0; i < 5; ++i) out[i * (kSsumMax + 1) + nb] = a[i] + e[i];
}

// Fit of u on each u-tile (one block of kUTile threads per tile): Chebyshev
// coefficients by least squares and the largest residual relative to the
// tile's largest |u|; a partial last tile is left unfit (residual inf).
__global__ __launch_bounds__(kUTile) void k_ufit(const double* __restrict__ u, int64_t nbins,
                                                 int32_t ntiles, double* __restrict__ coef,
                                                 double* __restrict__ resid) {
  __shared__ double red[kUCoef][kUTile / 64];
  __shared__ double c_s[kUCoef];
  __shared__ double mx[2][kUTile / 64];
  const int tile = blockIdx.x;
  const int m = threadIdx.x, lane = m & 63, wv = m >> 6;
  if (tile >= ntiles) return;
  const int64_t j = (int64_t)tile * kUTile + m;
  const bool full = (int64_t)(tile + 1) * kUTile <= nbins;
  const double um = (j < nbins) ? u[j] : 0.0;
  const double s = 2.0 * (double)m / (double)(kUTile - 1) - 1.0;
  double tk[kUCoef];
  tk[0] = 1.0;
  tk[1] = s;
#pragma unroll
  for (int k = 2; k < kUCoef; ++k) tk[k] = fma(2.0 * s, tk[k - 1], -tk[k - 2]);
#pragma unroll
  for (int k = 0; k < kUCoef; ++k) {
    double v = um * tk[k];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) red[k][wv] = v;
  }
  __syncthreads();
  if (m < kUCoef) {
    double c = 0.0;
#pragma unroll
    for (int k = 0; k < kUCoef; ++k) {
      double b = 0.0;
#pragma unroll
      for (int w = 0; w < kUTile / 64; ++w) b += red[k][w];
      c = fma(c_ufit_Ginv[m][k], b, c);
    }
    c_s[m] = c;
    if (full) coef[(int64_t)tile * kUCoef + m] = c;
    else coef[(int64_t)tile * kUCoef + m] = 0.0;
  }
  __syncthreads();
  double r = (j < nbins) ? fabs(um - cheb_eval10(c_s, s)) : 0.0, a = fabs(um);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    r = fmax(r, __shfl_xor(r, o, 64));
    a = fmax(a, __shfl_xor(a, o, 64));
  }
  if (lane == 0) { mx[0][wv] = r; mx[1][wv] = a; }
  __syncthreads();
  if (m == 0) {
    double rr = 0.0, aa = 0.0;
    for (int w = 0; w < kUTile / 64; ++w) { rr = fmax(rr, mx[0][w]); aa = fmax(aa, mx[1][w]); }
    resid[tile] = !full ? __builtin_inf() : (aa > 0.0 ? rr / aa : 0.0);
  }
}
// tolerances of the end-point check on the mixed path (FP32 products; its
// node phases are plain FP64, ~2e-9 cycles of rounding at 1e7 cycles, which
// the interpolant carries to its end points a few times over; the FP32 sine
// resolves ~6e-8 turns)
constexpr double kInterpTolPhaseMixed = 1e-7;
constexpr double kInterpTolTMixed = 3e-8;

// Node values, coefficients and end-point check of every work item (all
// lanes active: lanes 60..63 repeat the last point of the last item).  TAB:
// the plan has a numerical orbit (a separate instance keeps the table code
// out of the analytic kernel's registers).
template <bool MIXED, bool TAB>
__global__ __launch_bounds__(256, 2) void k_interp_nodes(Grid g,
                                                      const PartConst* __restrict__ pc,
                                                      const int32_t* __restrict__ bounds,
                                                      int32_t stride,
                                                      const int2* __restrict__ items,
                                                      const int32_t* __restrict__ total,
                                                      int32_t T,
                                                      const double* __restrict__ ek,
                                                      double* __restrict__ rec,
                                                      uint8_t* __restrict__ xflag,
                                                      float2* __restrict__ xerr,
                                                      int32_t* __restrict__ direct,
                                                      int32_t* __restrict__ ndirect,
                                                      UModel um,
                                                      double* __restrict__ partials) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int nwaves = (gridDim.x * blockDim.x) >> 6;
  __shared__ double2 s_tab[kSinTab];              // coarse angles of the template's sin/cos
  // the row tables in LDS (the coefficient loop reads one entry of each per
  // node and lane; from the constant tables each read is a vector memory load)
  __shared__ double s_r9[kCheb][kLanesItem], s_rT[kCheb][kLanesItem];
  __shared__ double s_rt[MIXED ? 1 : 2][kCheb][kLanesItem];
  // each lane's node values, read back by the lanes of its item (one write,
  // broadcast reads: LDS operations of one wave complete in order)
  constexpr int kNd = 14;
  __shared__ __align__(16) double s_nd[4][64][kNd];
  double* my_nd = s_nd[threadIdx.x >> 6][lane];
  for (int i = threadIdx.x; i < kCheb * kLanesItem; i += blockDim.x) {
    const int kn = i / kLanesItem, kk = i - kn * kLanesItem;
    s_r9[kn][kk] = c_row9[kn][kk];
    s_rT[kn][kk] = MIXED ? c_row6[kn][kk] : c_row9[kn][kk];
    if constexpr (!MIXED) {
      s_rt[0][kn][kk] = c_rowt[0][kn][kk];
      s_rt[1][kn][kk] = c_rowt[1][kn][kk];
    } else {
      s_rt[0][kn][kk] = c_row4[kn][kk];
    }
  }
  fill_sincos_table(s_tab);                       // ends with a block barrier
  const int W = total[0];
  const int G = (W + kItemsWave - 1) / kItemsWave;
  const int q = min(lane / kLanesItem, kItemsWave - 1);
  const int k = min(lane - q * kLanesItem, kLanesItem - 1);
  const int base = q * kLanesItem;
  for (int grp = wave; grp < G; grp += nwaves) {
    const int w = min(grp * kItemsWave + q, W - 1);
    const int2 it = items[w];
    const int p = it.x / stride, l = it.x - p * stride;
    const PartConst& P = pc[p];
    const int32_t* bp = bounds + (int64_t)p * (stride + 1);
    int ct, ch;
    item_split(it.y, g.chan.n, ct, ch);
    int b0, b1;
    item_bins(bp[l], bp[l + 1], ct, T, b0, b1);
    const int nb = b1 - b0;
    if (!__any(nb >= kMinInterp)) {
      // no item of this group is long enough to interpolate: all of them go
      // to the exact loop without evaluating their nodes
      if (k == kCheb && lane - base < kLanesItem && grp * kItemsWave + q < W) {
        xflag[w] = 1;
        rec[(int64_t)w * kRec + RecLayout<MIXED>::tail + 3] = 0.0;
        direct[atomicAdd(ndirect, 1)] = w;
      }
      continue;
    }
    const double* ekq = (ek && P.sur) ? ek + 8 * (int64_t)it.x : nullptr;
    const double sk = k < kCheb ? c_cheb_s[k] : (k == kCheb ? -1.0 : 1.0);
    const double mk = (sk + 1.0) * 0.5 * (double)(nb > 1 ? nb - 1 : 0);
    // exact frequency (k_lo + b0 + mk) df of the node, as double-double
    const dd f = dd_add(two_prod((double)(g.k_lo + b0), g.df), two_prod(mk, g.df));
    double v[5], v0lo;
    dd ph;
    if constexpr (MIXED)
      ph = dd{template_node_fp64(P, f.hi, ekq, v[1], v[2], v[3], v[4], g.chan.code[ch],
                                 TAB ? &g.orb : nullptr, s_tab), 0.0};
    else
      ph = template_node(P, f, ekq, v[1], v[2], v[3], v[4], g.chan.code[ch],
                         TAB ? &g.orb : nullptr, s_tab);
    const double p0h = __shfl(ph.hi, base + kCheb, 64);
    const double p0l = __shfl(ph.lo, base + kCheb, 64);
    const double peh = __shfl(ph.hi, base + kCheb + 1, 64);
    const double pel = __shfl(ph.lo, base + kCheb + 1, 64);
    const dd span = dd_add(dd{peh, pel}, dd{-p0h, -p0l});
    const double B = nb > 1 ? (span.hi + span.lo) / (double)(nb - 1) : 0.0;
    {
      const dd bm = two_prod(B, mk);
      const dd r = dd_add(dd_add(ph, dd{-p0h, -p0l}), dd{-bm.hi, -bm.lo});
      v[0] = r.hi;        // R at the node as a normalised double-double
      v0lo = r.lo;
    }
    // M-term integrands u |T+|^2, u |Tx|^2, u Re(T+ conj Tx), u Im(T+ conj Tx)
    // at this point, u from the smooth fit of its u-tile; usable when every
    // u-tile the item touches is fitted to within kUFitTol
    bool ufit = um.coef != nullptr && nb >= kMinInterp && nb <= kSsumMax;
    double gq[4], wq = 0.0, ures = 0.0;
    {
      // the channel's u-tiles follow those of the channels before it
      const int ub = ch * um.ntiles;
      const int ut0 = b0 / kUTile, ut1 = (b1 - 1) / kUTile;
      ufit = ufit && ut1 < um.ntiles &&
             (um.bad_prefix[ub + ut1 + 1] - um.bad_prefix[ub + ut0]) == 0;
      if (ufit)   // largest fit residual over the item's u-tiles (12 lanes share the scan)
        for (int ut = ut0 + k; ut <= ut1; ut += kLanesItem) ures = fmax(ures, um.resid[ub + ut]);
      const double x = (double)b0 + mk;
      const int ut = min(max((int)(x * (1.0 / kUTile)), 0), max(um.ntiles - 1, 0));
      const double loc = 2.0 * (x - (double)ut * kUTile) / (double)(kUTile - 1) - 1.0;
      const double uu = um.coef ? cheb_eval10(um.coef + (int64_t)(ub + ut) * kUCoef, loc) : 0.0;
      gq[0] = uu * fma(v[1], v[1], v[2] * v[2]);
      gq[1] = uu * fma(v[3], v[3], v[4] * v[4]);
      gq[2] = uu * fma(v[1], v[3], v[2] * v[4]);
      gq[3] = uu * fma(v[2], v[3], -v[1] * v[4]);
      if (k < kCheb && um.ssum) {
        const int nq = min(nb, kSsumMax);
#pragma unroll
        for (int i = 0; i < 5; ++i) wq = fma(c_cheb_D[i][k], um.ssum[i * (kSsumMax + 1) + nq], wq);
      }
    }
    typedef RecLayout<MIXED> L;
    // Lane k forms sum_kn row[kn][k] v_kn: on node lanes (k < kCheb) the
    // interpolant's monomial coefficient k, on the end lanes its value at the
    // lane's own end point, which the lane has evaluated exactly.
    // FP64 path: R compensated (a twice-the-working-precision dot product:
    // error-free products and sums, their errors summed apart): R reaches a
    // few cycles, the node-to-monomial map has entries of a few hundred, and a
    // plain double sum would leave ~1e-13 cycles of cancellation error in the
    // coefficients.  Mixed path: a plain sum (its tolerance is 1e-9 cycles).
    double aRs = 0.0, aRx = 0.0, tmax = 0.0, gmax = 0.0;
    double aT[4], aTt[2][4], aG[4];
#pragma unroll
    for (int fn = 0; fn < 4; ++fn) {
      aT[fn] = 0.0; aG[fn] = 0.0; aTt[0][fn] = 0.0; aTt[1][fn] = 0.0;
    }
    my_nd[0] = v[0]; my_nd[1] = v0lo;
    my_nd[2] = v[1]; my_nd[3] = v[2]; my_nd[4] = v[3]; my_nd[5] = v[4];
    my_nd[6] = gq[0]; my_nd[7] = gq[1]; my_nd[8] = gq[2]; my_nd[9] = gq[3];
    my_nd[10] = wq;
    // the node's largest transfer component and |M-term integrand|
    my_nd[12] = fmax(fmax(fabs(v[1]), fabs(v[2])), fmax(fabs(v[3]), fabs(v[4])));
    my_nd[13] = fmax(fabs(gq[0]), fabs(gq[1]));
    __builtin_amdgcn_wave_barrier();
    const double* item_nd = s_nd[threadIdx.x >> 6][base];
    // two nodes per pass (their LDS reads overlap); unrolled fully, the loop
    // hoists every node's table loads and needs more registers than the kernel
    // can hold at a useful occupancy
    // M-term integrands: lane 0 sums the quadrature, the end lanes interpolate
    const double sel0 = k == 0 ? 1.0 : 0.0, selE = k >= kCheb ? 1.0 : 0.0;
#pragma unroll 2
    for (int kn = 0; kn < kCheb; ++kn) {
      const double r9 = s_r9[kn][k];
      const double rT = MIXED ? s_rT[kn][k] : r9;
      const double2* nd = reinterpret_cast<const double2*>(item_nd + kNd * kn);
      const double2 n01 = nd[0], n23 = nd[1], n45 = nd[2], n67 = nd[3], n89 = nd[4], nab = nd[5],
                    ncd = nd[6];
      if constexpr (MIXED) {
        aRx = fma(n01.x, r9, aRx);
      } else {
        FSTAT_NO_CONTRACT
        const dd pr = two_prod(n01.x, r9);
        const dd sm = two_sum(aRs, pr.hi);
        aRs = sm.hi;
        aRx = fma(n01.y, r9, aRx + (sm.lo + pr.lo));
      }
      const double vt[4] = {n23.x, n23.y, n45.x, n45.y};
#pragma unroll
      for (int fn = 0; fn < 4; ++fn) {
        aT[fn] = fma(vt[fn], rT, aT[fn]);
#pragma unroll
        for (int v2 = 0; v2 < (MIXED ? 1 : 2); ++v2)
          aTt[v2][fn] = fma(vt[fn], s_rt[v2][kn][k], aTt[v2][fn]);
      }
      tmax = fmax(tmax, ncd.x);
      gmax = fmax(gmax, ncd.y);
      const double rg = fma(sel0, nab.x, selE * r9);
      const double gt[4] = {n67.x, n67.y, n89.x, n89.y};
#pragma unroll
      for (int fn = 0; fn < 4; ++fn) aG[fn] = fma(gt[fn], rg, aG[fn]);
    }
    __builtin_amdgcn_wave_barrier();   // the slots are rewritten by the next group
    const double tolP = MIXED ? kInterpTolPhaseMixed : kInterpTolPhase;
    const double tolT = MIXED ? kInterpTolTMixed : kInterpTolT;
    const double cR = aRs + aRx;
    bool bad = false;
    double err = 0.0;           // relative template error at this end point
    double errt[2] = {0.0, 0.0};   // transfer error of the degree-5 and -7 (mixed: 4) truncations
    double gerr = 0.0;          // M-term integrands' error (relative to max u |T|^2)
    if (k >= kCheb) {
      const double itmax = 1.0 / tmax;      // the estimates below need no correct rounding
      // (aRs - v0 is exact wherever the interpolant is close enough to pass)
      const double dph = fabs(((aRs - v[0]) + aRx) - v0lo);
      bad = !(dph <= tolP);
      err = 2.0 * kPi * dph;
#pragma unroll
      for (int fn = 1; fn < 5; ++fn) {
        const double d = fabs(aT[fn - 1] - v[fn]);
        bad = bad || !(d <= tolT * tmax);
        err = fmax(err, d * itmax);
#pragma unroll
        for (int v2 = 0; v2 < (MIXED ? 1 : 2); ++v2)
          errt[v2] = fmax(errt[v2], fabs(aTt[v2][fn - 1] - v[fn]) * itmax);
      }
#pragma unroll
      for (int fn = 0; fn < 4; ++fn) gerr = fmax(gerr, fabs(aG[fn] - gq[fn]));
      gerr = gmax > 0.0 ? gerr / gmax : (gerr > 0.0 ? 1.0 : 0.0);
    }
    const double tolG = MIXED ? kInterpTolTMixed : 4.0 * kInterpTolT;
    const uint64_t gbadmask = __ballot(k >= kCheb && !(gerr <= tolG));
    gerr = fmax(gerr, __shfl(gerr, base + kCheb + 1, 64));
#pragma unroll
    for (int kk = 0; kk < kLanesItem; ++kk) gerr = fmax(gerr, __shfl(ures, base + kk, 64));
    const uint64_t badmask = __ballot(bad);
    err = fmax(__shfl(err, base + kCheb, 64), __shfl(err, base + kCheb + 1, 64));
    double gsum[4];
#pragma unroll
    for (int fn = 0; fn < 4; ++fn) gsum[fn] = __shfl(aG[fn], base, 64);
    // FP64: lowest transfer degree whose truncation error stays within the
    // item's own interpolation error, or kTruncFloor of the largest component
    // (a larger allowance sends more items of ill-conditioned partitions to
    // the exact re-evaluation than the lower degree saves)
    int degT = MIXED ? kDegT : kCheb - 1;
    if constexpr (!MIXED) {
      const double allow = fmin(fmax(err, kTruncFloor), tolT);
      const double e7 = fmax(__shfl(errt[1], base + kCheb, 64), __shfl(errt[1], base + kCheb + 1, 64));
      const double e5 = fmax(__shfl(errt[0], base + kCheb, 64), __shfl(errt[0], base + kCheb + 1, 64));
      if (e5 <= allow) { degT = 5; err = fmax(err, e5); }
      else if (e7 <= allow) { degT = 7; err = fmax(err, e7); }
    } else {
      const double e4 = fmax(__shfl(errt[0], base + kCheb, 64), __shfl(errt[0], base + kCheb + 1, 64));
      if (e4 <= tolT) { degT = kDegTLow; err = fmax(err, e4); }
    }
    const bool mine = lane - base < kLanesItem && grp * kItemsWave + q < W;   // not a repeat lane
    if (!mine) continue;
    const bool mq = ufit && ((gbadmask >> base) & ((1ull << kLanesItem) - 1ull)) == 0ull;
    // items without quadrature M-terms (u not fitted on one of their u-tiles,
    // or M-term interpolants that miss an end point) go to the exact loop too
    const bool rej = nb < kMinInterp || !mq ||
                     ((badmask >> base) & ((1ull << kLanesItem) - 1ull)) != 0ull;
    if (mq && k < 4)
      partials[(int64_t)w * 8 + 4 + k] = k == 0 ? gsum[0] : (k == 1 ? gsum[1] : (k == 2 ? gsum[2] : gsum[3]));
    double* r = rec + (int64_t)w * kRec;
    if (k < kCheb) {
      r[k] = cR;
      if (k < L::nT) {
#pragma unroll
        for (int fn = 1; fn < 5; ++fn)
          r[kCheb + (fn - 1) * L::nT + k] =
              MIXED ? (degT == kDegTLow ? aTt[0][fn - 1] : aT[fn - 1])
                    : (degT == 5 ? aTt[0][fn - 1] : (degT == 7 ? aTt[1][fn - 1] : aT[fn - 1]));
      }
    } else if (k == kCheb) {
      FSTAT_NO_CONTRACT
      r[L::tail + 4] = (double)degT;
      r[L::tail] = (p0h - floor(p0h)) + p0l;     // fractional cycle at the first bin
      r[L::tail + 1] = B - rint(B);              // whole cycles per bin drop out (m is an integer)
      r[L::tail + 2] = B;
      r[L::tail + 3] = rej ? 0.0 : 1.0;
      r[L::tail + 5] = (double)(b0 % T);          // first bin within its tile
      r[L::tail + 6] = (double)nb;
      r[L::tail + 7] = nb > 1 ? 2.0 / (double)(nb - 1) : 0.0;
      r[L::tail + 8] = -B / g.df;
      xflag[w] = rej ? 1 : 0;
      // the template error times the norm sqrt(sum u) max|T| of the item's
      // templates, and the M-term quadrature's error bound: its relative error
      // at the end points times max u |T|^2 times the bin count (see k_mark)
      const int64_t uo = (int64_t)ch * (g.nbins + 1);
      const double U = um.upre ? fmax(um.upre[uo + b1] - um.upre[uo + b0], 0.0) : (double)nb;
      xerr[w] = make_float2((float)(err * tmax * sqrt(U)), mq ? (float)(gerr * gmax * nb) : 0.0f);
      if (rej) direct[atomicAdd(ndirect, 1)] = w;
    }
  }
}

// The bins of the interpolated items, tile by tile: the tile's w is staged
// once in LDS; each wave takes one item at a time, broadcasts its record into
// registers and runs the per-bin loop from LDS.
template <bool MIXED>
__global__ __launch_bounds__(256) void k_eval_interp(Grid g,
                                                     int32_t T,
                                                     const int32_t* __restrict__ tile_items,
                                                     const int32_t* __restrict__ tile_off,
                                                     const int32_t* __restrict__ unit_off,
                                                     int32_t ntiles,
                                                     int32_t* __restrict__ tile_ctr,
                                                     const double* __restrict__ wr64,
                                                     const double* __restrict__ wi64,
                                                     const float* __restrict__ wr32,
                                                     const float* __restrict__ wi32,
                                                     double* __restrict__ rec,
                                                     double* __restrict__ partials) {
  typedef typename std::conditional<MIXED, float, double>::type DT;
  extern __shared__ unsigned char smem[];
  // The tile's w (and on the FP64 path e_j) at a fixed stride of the largest
  // tile, so that every per-bin read shares one address register (constant
  // offsets) whatever the tile size.  Every item here has its M-terms from the
  // node kernel's quadrature (the others go to the exact loop), so u is not
  // staged; e_j is kept in FP32 (|e_j| <= half an ulp of f_j; its product with
  // t_f <~ 1e8 s enters the phase at <~ 1e-10 cycles, and FP32 rounding of it
  // at ~1e-17 cycles).  FP64: 20 B per bin, three blocks of 2560-bin tiles per
  // CU.
  constexpr int TS = MIXED ? kMaxTileMixed : kMaxTileFp64;
  const double2* s_tab = c_sincos;                       // FP64 loop: sin, cos table
  DT* s_wr = reinterpret_cast<DT*>(smem);
  DT* s_wi = s_wr + TS;
  float* s_e = reinterpret_cast<float*>(s_wi + TS);      // FP64 loop: grid rounding e_j
  __shared__ int s_unit[3];                       // tile, first item, item count
  __shared__ double s_rec[4][64];                // each wave's current item record
  const DT* gwr;
  const DT* gwi;
  if constexpr (MIXED) { gwr = wr32; gwi = wi32; }
  else { gwr = wr64; gwi = wi64; }
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int nwv = blockDim.x >> 6;
  const int nunits = unit_off[ntiles];
  for (;;) {
    // next unit (dynamic): up to kUnitItems items of one tile
    if (threadIdx.x == 0) {
      const int u = atomicAdd(tile_ctr, 1);
      int t = -1, first = 0, count = 0;
      if (u < nunits) {
        int lo = 0, hi = ntiles;                     // last tile with unit_off[t] <= u
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (unit_off[mid] <= u) lo = mid; else hi = mid;
        }
        t = lo;
        first = tile_off[t] + (u - unit_off[t]) * kUnitItems;
        count = min(kUnitItems, tile_off[t + 1] - first);
      }
      s_unit[0] = t; s_unit[1] = first; s_unit[2] = count;
    }
    __syncthreads();
    const int tx = s_unit[0];
    if (tx < 0) break;
    // tiles of all channels are numbered channel by channel
    const int ntpc = (int)((g.nbins + T - 1) / T);
    const int tch = tx / ntpc, t = tx - tch * ntpc;
    const int64_t co = (int64_t)tch * g.nbins;
    const int j0 = t * T;
    const int nt = min((int64_t)T, g.nbins - j0);
    for (int i = threadIdx.x; i < nt; i += blockDim.x) {
      s_wr[i] = gwr[co + j0 + i];
      s_wi[i] = gwi[co + j0 + i];
      if constexpr (!MIXED) {
        // f_j = (k_lo + j) df rounds to a double; e_j is the rounding error of
        // that product (one FMA), formed once per bin of the tile
        const double jd = (double)(g.k_lo + j0 + i);
        s_e[i] = (float)fma(jd, g.df, -(jd * g.df));
      }
    }
    __syncthreads();
    const int i0 = s_unit[1];
    const int cnt = s_unit[2];
    typedef RecLayout<MIXED> L;
    double* R = s_rec[wv];
    // Each item's record holds all the loop needs of it; a wave loads the next
    // item's record while it runs the current one, so that only the first
    // load of a unit is waited for.
    int wn = wv < cnt ? tile_items[i0 + wv] : 0;
    double rv = (wv < cnt && lane < kRec) ? rec[(int64_t)wn * kRec + lane] : 0.0;
    for (int idx = wv; idx < cnt; idx += nwv) {
      const int w = wn;
      // the record through the wave's LDS slot: one write, then broadcast reads
      // (LDS operations of one wave complete in order)
      if (lane < kRec) R[lane] = rv;
      __builtin_amdgcn_wave_barrier();
      const int idn = idx + nwv;
      wn = idn < cnt ? tile_items[i0 + idn] : 0;
      rv = (idn < cnt && lane < kRec) ? rec[(int64_t)wn * kRec + lane] : 0.0;
      if (R[L::tail + 3] == 0.0) {                 // evaluated by the exact kernel
        __builtin_amdgcn_wave_barrier();
        continue;
      }
      const int e0 = (int)R[L::tail + 5];         // LDS offset of the item's first bin
      const int nb = (int)R[L::tail + 6];
      double cR[kCheb];
#pragma unroll
      for (int n = 0; n < kCheb; ++n) cR[n] = R[n];
      const double A = R[L::tail];
      const double Bp = R[L::tail + 1];
      const int degT = (int)R[L::tail + 4];      // transfer degree (FP64 loop)
      const double alpha = R[L::tail + 7];        // 2 / (nb - 1)
      if constexpr (!MIXED) {
        // The grid is f_j = (k_lo + j) df rounded to a double; the interpolants
        // are exact in f, so the phase moves by (dPhi/df)(f_j - exact) =
        // -(B / df) e_j, with e_j the rounding error of the product (staged
        // with the tile): up to ~1e-9 cycles at t_f ~ 1e8 s.
        const double kB = R[L::tail + 8];           // -B / df
        // Difference recurrence for items whose lanes get runs of at least
        // kRecMinRun bins.  Lane l takes the contiguous bins m0 = l Lr ..
        // m0 + Lr - 1 (Lr odd, so that the lanes' LDS addresses fall in
        // distinct banks).  With a_k = alpha^k R^(k)(s0) / k! the phase is
        // Phi(m0 + t) = Phi(m0) + Bp t + sum_k a_k t^k; its forward differences
        // D_j (D_j(t + 1) = D_j(t) + D_{j+1}(t)) start at D_1 = Bp + sum_k a_k
        // and D_j = sum_k j! S(k, j) a_k (S: Stirling numbers of the second
        // kind).  Per bin the template factor advances as E0 <- E0 E1(t), with
        // E1(t) = E1(0) e^{i phi(t)} and phi(t) = 2 pi sum_{i<t} D_2(i) (D_2, D_3
        // advanced by their differences, D_4 held): no phase polynomial and no
        // sine per bin.  Over <= 33 bins the rounding of the products stays
        // near 1e-14, below the direct evaluation's own ~1e-13 cycles; an item
        // takes the direct loop when phi can leave the range of its series or
        // the neglected D_5 could move the phase by more than kRecTrunc.
        const int Lr = ((nb + 63) >> 6) | 1;
        const int m0 = lane * Lr;
        const int cnt = min(max(nb - m0, 0), Lr);
        double E0r = 0.0, E0i = 0.0, E1r = 0.0, E1i = 0.0, th2 = 0.0, th3 = 0.0, th4 = 0.0;
        bool use_rec = Lr >= kRecMinRun;
        if (use_rec) {
          const double s0 = fma(alpha, (double)m0, -1.0);
          // Taylor coefficients of R at s0 (repeated synthetic division)
          double p[kCheb];
#pragma unroll
          for (int n = 0; n < kCheb; ++n) p[n] = cR[n];
#pragma unroll
          for (int k = 0; k < kCheb - 1; ++k)
#pragma unroll
            for (int j = kCheb - 2; j >= k; --j) p[j] = fma(p[j + 1], s0, p[j]);
          double ap[kCheb];
          ap[0] = 1.0;
#pragma unroll
          for (int k = 1; k < kCheb; ++k) ap[k] = ap[k - 1] * alpha;
          double d1 = 0.0, d2 = 0.0, d3 = 0.0, d4 = 0.0, d5 = 0.0;
#pragma unroll
          for (int k = kCheb - 1; k >= 1; --k) {    // smallest terms first
            const double ak = p[k] * ap[k];
            d1 += ak;
            if (k >= 2) d2 = fma(kStirF[k][2], ak, d2);
            if (k >= 3) d3 = fma(kStirF[k][3], ak, d3);
            if (k >= 4) d4 = fma(kStirF[k][4], ak, d4);
            if (k >= 5) d5 = fma(kStirF[k][5], ak, d5);
          }
          d1 += Bp;
          sincos_tab(fma(Bp, (double)m0, p[0]) + A, s_tab, E0i, E0r);
          sincos_tab(d1, s_tab, E1i, E1r);
          th2 = kTwoPi * d2;
          th3 = kTwoPi * d3;
          th4 = kTwoPi * d4;
          const double x = (double)Lr;
          const double phimax = x * (fabs(th2) + x * (fabs(th3) + x * fabs(th4)));
          const double c5 = x * (x - 1.0) * (x - 2.0) * (x - 3.0) * (x - 4.0) * (1.0 / 120.0);
          const bool ok = cnt == 0 || (phimax <= kRecPhiMax && c5 * kTwoPi * fabs(d5) <= kRecTrunc);
          use_rec = __all(ok);
        }
        if (lane == 0 && use_rec) rec[(int64_t)w * kRec + L::tail + 3] = 2.0;   // for fstat_interp_stats
        // DT: degree of the transfer interpolants (5, 7 or 9)
        auto loop = [&](auto dt) {
          constexpr int DT = decltype(dt)::value;
          int idx;
          {
            // N-terms only.  They are linear in the transfer interpolants
            // T(s) = sum_k c_k s^k, so the loop sums the moments
            // sum_j w_j e^{i Phi_j} s_j^k (k <= DT) and the coefficients are
            // applied once per lane afterwards: no transfer polynomial per bin.
            double mr[DT + 1], mm[DT + 1];
            using First = std::true_type;
            using Next = std::false_type;
            if (use_rec) {
              // The run's bins are equally spaced in s, so the loop sums
              // binomial moments instead: per bin A_m += A_{m-1} (m = DT..1),
              // then A_0 += X_t, which leaves A_m = sum_t X_t C(cnt - 1 - t, m)
              // (X_t = w e^{i Phi} at the run's bin t); no power of s per bin.
              // They become power moments once per lane below.
              const double kBe = kTwoPi * kB;
              double phi = 0.0, t2 = th2, t3 = th3;
              double er = E0r, ei = E0i;
              auto rec_bin = [&](auto first, double a, double b, float ef) {
                constexpr bool F = decltype(first)::value;
                // the grid rounding as the factor 1 + i eps (|eps| <~ 1e-8)
                const double eps = kBe * (double)ef;
                const double xr = fma(-eps, ei, er), xi = fma(eps, er, ei);
                if constexpr (F) {
                  mr[0] = fma(-b, xi, a * xr);
                  mm[0] = fma(b, xr, a * xi);
#pragma unroll
                  for (int m = 1; m <= DT; ++m) mr[m] = mm[m] = 0.0;
                } else {
#pragma unroll
                  for (int m = DT; m >= 1; --m) {
                    mr[m] += mr[m - 1];
                    mm[m] += mm[m - 1];
                  }
                  mr[0] = fma(a, xr, fma(-b, xi, mr[0]));
                  mm[0] = fma(a, xi, fma(b, xr, mm[0]));
                }
                // E1(t) = E1(0) e^{i phi}: |phi| <= kRecPhiMax, series to phi^6
                // (cos) and phi^5 (sin), remainders below 1e-17
                const double z = phi * phi;
                const double cph = fma(fma3(1.0 / 24.0, z, -0.5), z, 1.0);
                const double sph = phi * fma(fma3(1.0 / 120.0, z, -1.0 / 6.0), z, 1.0);
                const double e1r = E1r * cph - E1i * sph, e1i = E1r * sph + E1i * cph;
                const double nr = er * e1r - ei * e1i;
                ei = er * e1i + ei * e1r;
                er = nr;
                phi += t2;
                t2 += t3;
                t3 += th4;
              };
              // the first bin sets the moments (lanes without bins take w = 0);
              // the rest of an odd run goes two bins per pass
              const int ib = e0 + m0;
              const bool any = cnt > 0;
              rec_bin(First{}, any ? s_wr[ib] : 0.0, any ? s_wi[ib] : 0.0, any ? s_e[ib] : 0.0f);
              int t = 1;
              for (; t + 1 < cnt; t += 2) {
                const double a1 = s_wr[ib + t], a2 = s_wr[ib + t + 1];
                const double b1 = s_wi[ib + t], b2 = s_wi[ib + t + 1];
                const float f1 = s_e[ib + t], f2 = s_e[ib + t + 1];
                rec_bin(Next{}, a1, b1, f1);
                rec_bin(Next{}, a2, b2, f2);
              }
              if (t < cnt) rec_bin(Next{}, s_wr[ib + t], s_wi[ib + t], s_e[ib + t]);
              // To power moments M_k = sum_t X_t s_t^k.  With u = cnt - 1 - t,
              // s_t = s_e - alpha u (s_e: the run's last bin): sum_t X_t u^j =
              // sum_m m! S(j, m) A_m, scaled by (-alpha)^j, then shifted to the
              // origin by M_k = sum_j C(k, j) s_e^(k - j) (...)_j.  Over a run
              // of <~ 0.03 in s every step keeps its terms near the result's
              // own size.
#pragma unroll
              for (int j = DT; j >= 2; --j) {
                double pr = kStirF[j][j] * mr[j], pi = kStirF[j][j] * mm[j];
#pragma unroll
                for (int m = j - 1; m >= 2; --m) {
                  pr = fma(kStirF[j][m], mr[m], pr);
                  pi = fma(kStirF[j][m], mm[m], pi);
                }
                mr[j] = pr + mr[1];
                mm[j] = pi + mm[1];
              }
              const double na = -alpha;
              double pw = na;
#pragma unroll
              for (int j = 1; j <= DT; ++j) {
                mr[j] *= pw;
                mm[j] *= pw;
                pw *= na;
              }
              const double se = fma(alpha, (double)(m0 + cnt - 1), -1.0);
#pragma unroll
              for (int k = 0; k < DT; ++k)
#pragma unroll
                for (int j = DT; j > k; --j) {
                  mr[j] = fma(se, mr[j - 1], mr[j]);
                  mm[j] = fma(se, mm[j - 1], mm[j]);
                }
            } else {
              // direct form: even moments from W = w e^{i Phi}, odd ones from
              // W s, both against even powers of s
              auto moments = [&](double Wr, double Wi, double s, double s2, double s4, double s8) {
                const double Vr = Wr * s, Vi = Wi * s;
                const double pe[5] = {1.0, s2, s4, s4 * s2, s8};
                mr[0] += Wr;
                mm[0] += Wi;
                mr[1] += Vr;
                mm[1] += Vi;
#pragma unroll
                for (int k = 2; k <= DT; ++k) {
                  const double xr = (k & 1) ? Vr : Wr, xi = (k & 1) ? Vi : Wi;
                  mr[k] = fma(xr, pe[k >> 1], mr[k]);
                  mm[k] = fma(xi, pe[k >> 1], mm[k]);
                }
              };
              auto one_bin = [&](int mi, double a, double b, double ej) {
                const double m = (double)mi;
                const double s = fma(alpha, m, -1.0);
                const double s2 = s * s, s4 = s2 * s2, s8 = s4 * s4;
                const double ph = fma(Bp, m, estrin9(cR, s, s2, s4, s8)) + fma(kB, ej, A);
                double sps, cps;
                sincos_tab(ph, s_tab, sps, cps);
                moments(a * cps - b * sps, a * sps + b * cps, s, s2, s4, s8);
              };
#pragma unroll
              for (int k = 0; k <= DT; ++k) mr[k] = mm[k] = 0.0;
              // lanes interleaved; two bins per pass (half the loop control per
              // bin), then at most one left over per lane
              int mi = lane;
              for (; mi + 64 < nb; mi += 128) {
                const int i1 = e0 + mi, i2 = i1 + 64;
                const double a1 = s_wr[i1], b1 = s_wi[i1], e1 = s_e[i1];
                const double a2 = s_wr[i2], b2 = s_wi[i2], e2 = s_e[i2];
                one_bin(mi, a1, b1, e1);
                one_bin(mi + 64, a2, b2, e2);
              }
              if (mi < nb) {
                const int i1 = e0 + mi;
                one_bin(mi, s_wr[i1], s_wi[i1], s_e[i1]);
              }
            }
            // sum Wr T+r + Wi T+i, sum Wi T+r - Wr T+i, and the same for x: FMA
            // chains, one transfer component pair at a time (fewer live registers)
            double acc[4];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
#pragma unroll
              for (int k = 0; k <= DT; ++k) {
                const double tr = R[kCheb + 2 * h * L::nT + k], ti = R[kCheb + (2 * h + 1) * L::nT + k];
                acc[2 * h] = fma(tr, mr[k], k ? fma(ti, mm[k], acc[2 * h]) : ti * mm[k]);
                acc[2 * h + 1] = fma(tr, mm[k], k ? fma(-ti, mr[k], acc[2 * h + 1]) : -ti * mr[k]);
              }
            }
            __builtin_amdgcn_wave_barrier();   // the slot is rewritten for the next item
            const double tot = wave_sum4(acc, lane, idx);
            if ((lane & 15) == 0) partials[(int64_t)w * 8 + idx] = tot;
          }
        };
        using D5 = std::integral_constant<int, 5>;
        using D7 = std::integral_constant<int, 7>;
        using D9 = std::integral_constant<int, 9>;
        if (degT == 5) loop(D5{});
        else if (degT == 7) loop(D7{});
        else loop(D9{});
      } else {
        // Lane l takes the contiguous bins m0 = l Lr .. m0 + Lr - 1 (Lr odd:
        // distinct LDS banks).  The phase R(s) + Bp m + A [turns] advances by
        // its forward differences in FP64: R has degree 9, so the ninth
        // difference is constant and every phase of the run is exact up to
        // rounding (~1e-13 turns over a run), no polynomial per bin; where a
        // bound on what the fifth to ninth differences add stays below
        // kMixTrunc on every lane's run, the wave holds the fourth constant
        // and forms only the first four.  The
        // N-terms are summed in FP32 as binomial moments (A_m += A_{m-1}, then
        // A_0 += w e^{i Phi}: A_m = sum_t w_t e^{i Phi_t} C(cnt - 1 - t, m)),
        // changed once per lane to power moments sum w e^{i Phi} s^k (k <= D)
        // over the run's <~ 0.03 in s, where each step keeps its terms near the
        // result's size; their FP32 rounding, ~1e-7 relative, is far inside the
        // mixed path's bar.  The transfer degree is kDegT, or kDegTLow where the
        // node kernel found it enough; the coefficients are applied in FP64.
        const int Lr = ((nb + 63) >> 6) | 1;
        const int m0 = lane * Lr;
        const int cnt = min(max(nb - m0, 0), Lr);
        double dd[kCheb];                 // dd[j]: j-th forward difference (j >= 1)
        double ph;
        bool trunc;
        {
          // Taylor coefficients of R at the run's start (repeated synthetic
          // division), a_k = alpha^k R^(k)(s0) / k!, D_j = sum_k j! S(k, j) a_k
          const double s0 = fma(alpha, (double)m0, -1.0);
          double p[kCheb];
#pragma unroll
          for (int n = 0; n < kCheb; ++n) p[n] = cR[n];
#pragma unroll
          for (int k = 0; k < kCheb - 1; ++k)
#pragma unroll
            for (int j = kCheb - 2; j >= k; --j) p[j] = fma(p[j + 1], s0, p[j]);
          // What the fifth to ninth differences add to the phase t bins in:
          // sum_{k>=5} a_k sum_{j>=5} C(t, j) j! S(k, j), whose inner sums are
          // at most sum_j C(t, j) j! S(k, j) = t^k; so with t < Lr it is below
          // sum_{k>=5} |R^(k)(s0) / k!| (alpha Lr)^k.
          const double x = alpha * (double)Lr;
          double xk = (x * x) * (x * x), bound = 0.0;
#pragma unroll
          for (int k = kMixDiff + 1; k < kCheb; ++k) {
            xk *= x;
            bound = fma(fabs(p[k]), xk, bound);
          }
          trunc = __all(cnt == 0 || bound <= kMixTrunc);
          double ap[kCheb];
          ap[1] = alpha;
#pragma unroll
          for (int k = 2; k < kCheb; ++k) ap[k] = ap[k - 1] * alpha;
#pragma unroll
          for (int j = 1; j < kCheb; ++j) dd[j] = 0.0;
#pragma unroll
          for (int k = kCheb - 1; k >= 1; --k) {    // smallest terms first
            const double ak = p[k] * ap[k];
#pragma unroll
            for (int j = 1; j <= k && j <= kMixDiff; ++j) dd[j] = fma(kStirF[k][j], ak, dd[j]);
          }
          if (!trunc) {                               // the wave carries all nine
#pragma unroll
            for (int k = kCheb - 1; k > kMixDiff; --k) {
              const double ak = p[k] * ap[k];
#pragma unroll
              for (int j = kMixDiff + 1; j <= k; ++j) dd[j] = fma(kStirF[k][j], ak, dd[j]);
            }
          }
          dd[1] += Bp;
          ph = fma(Bp, (double)m0, p[0]) + A;
          ph -= rint(ph);
        }
        if (lane == 0 && trunc) rec[(int64_t)w * kRec + L::tail + 3] = 2.0;   // for fstat_interp_stats
        // D: transfer degree; ND: forward differences carried (the last held)
        auto loop = [&](auto dt, auto ndt) {
          constexpr int D = decltype(dt)::value;
          constexpr int ND = decltype(ndt)::value;
          int idx;
          float mr[D + 1], mm[D + 1];
          auto bin = [&](auto first, float a, float b) {
            constexpr bool F = decltype(first)::value;
            const float rf = (float)(ph - rint(ph));
            const float sps = __builtin_amdgcn_sinf(rf), cps = __builtin_amdgcn_cosf(rf);
            if constexpr (F) {
              mr[0] = fmaf(-b, sps, a * cps);
              mm[0] = fmaf(b, cps, a * sps);
#pragma unroll
              for (int m = 1; m <= D; ++m) mr[m] = mm[m] = 0.0f;
            } else {
#pragma unroll
              for (int m = D; m >= 1; --m) {
                mr[m] += mr[m - 1];
                mm[m] += mm[m - 1];
              }
              mr[0] = fmaf(a, cps, fmaf(-b, sps, mr[0]));
              mm[0] = fmaf(a, sps, fmaf(b, cps, mm[0]));
            }
            ph += dd[1];
#pragma unroll
            for (int j = 1; j < ND; ++j) dd[j] += dd[j + 1];
          };
          using First = std::true_type;
          using Next = std::false_type;
          // the first bin sets the moments (lanes without bins take w = 0);
          // the rest of an odd run goes two bins per pass
          const int ib = e0 + m0;
          const bool any = cnt > 0;
          bin(First{}, any ? s_wr[ib] : 0.0f, any ? s_wi[ib] : 0.0f);
          int t = 1;
          for (; t + 1 < cnt; t += 2) {
            const float a1 = s_wr[ib + t], a2 = s_wr[ib + t + 1];
            const float b1 = s_wi[ib + t], b2 = s_wi[ib + t + 1];
            bin(Next{}, a1, b1);
            bin(Next{}, a2, b2);
          }
          if (t < cnt) bin(Next{}, s_wr[ib + t], s_wi[ib + t]);
          // to power moments: with u = cnt - 1 - t and s_t = s_e - alpha u,
          // sum_t X_t u^j = sum_m m! S(j, m) A_m, scaled by (-alpha)^j, then
          // shifted to the origin by M_k = sum_j C(k, j) s_e^(k - j) (...)_j
#pragma unroll
          for (int j = D; j >= 2; --j) {
            float pr = (float)kStirF[j][j] * mr[j], pi = (float)kStirF[j][j] * mm[j];
#pragma unroll
            for (int m = j - 1; m >= 2; --m) {
              pr = fmaf((float)kStirF[j][m], mr[m], pr);
              pi = fmaf((float)kStirF[j][m], mm[m], pi);
            }
            mr[j] = pr + mr[1];
            mm[j] = pi + mm[1];
          }
          const float na = (float)(-alpha);
          float pw = na;
#pragma unroll
          for (int j = 1; j <= D; ++j) {
            mr[j] *= pw;
            mm[j] *= pw;
            pw *= na;
          }
          const float se = (float)fma(alpha, (double)(m0 + cnt - 1), -1.0);
#pragma unroll
          for (int k = 0; k < D; ++k)
#pragma unroll
            for (int j = D; j > k; --j) {
              mr[j] = fmaf(se, mr[j - 1], mr[j]);
              mm[j] = fmaf(se, mm[j - 1], mm[j]);
            }
          double red[4];
#pragma unroll
          for (int k = 0; k <= D; ++k) {
            const double t0 = R[kCheb + k], t1 = R[kCheb + L::nT + k];
            const double t2 = R[kCheb + 2 * L::nT + k], t3 = R[kCheb + 3 * L::nT + k];
            const double r = mr[k], q = mm[k];
            red[0] = fma(t0, r, k ? fma(t1, q, red[0]) : t1 * q);
            red[1] = fma(t0, q, k ? fma(-t1, r, red[1]) : -t1 * r);
            red[2] = fma(t2, r, k ? fma(t3, q, red[2]) : t3 * q);
            red[3] = fma(t2, q, k ? fma(-t3, r, red[3]) : -t3 * r);
          }
          __builtin_amdgcn_wave_barrier();   // the slot is rewritten for the next item
          const double tot = wave_sum4(red, lane, idx);
          if ((lane & 15) == 0) partials[(int64_t)w * 8 + idx] = tot;
        };
        using DLow = std::integral_constant<int, kDegTLow>;
        using DHigh = std::integral_constant<int, kDegT>;
        using NShort = std::integral_constant<int, kMixDiff>;
        using NFull = std::integral_constant<int, kCheb - 1>;
        if (degT == kDegTLow) {
          if (trunc) loop(DLow{}, NShort{});
          else loop(DLow{}, NFull{});
        } else {
          if (trunc) loop(DHigh{}, NShort{});
          else loop(DHigh{}, NFull{});
        }
      }
    }
    __syncthreads();   // every wave is done with this unit's LDS and s_unit
  }
}

// Refinement of the FP64 interpolating loop's partitions.  With beta =
// H^{-1} z the maximiser and r the data minus its projection on the template
// span, a template error dA and an error dH_q of the quadrature M-terms move
// F = 1/2 z^H H^{-1} z (Sec. II.A, Eq. coherent_F_stat) to first order by
//     dF = Re <r, dA beta> + Re <A beta, dA beta> - 1/2 beta^H dH_q beta
// (the last two vanish where the M-terms are summed from the same
// interpolated templates).  |A beta|^2 = 2F; for Gaussian noise <r, v> is a
// normal variable of variance at most |v|^2; an item whose transfer and phase
// interpolants are off by at most e relative to its largest transfer
// component m contributes at most 2 e^2 m^2 sum(u) to |dA_k|^2 (k = +, x),
// and each entry of its quadrature M-terms is off by at most g (the
// quadrature's end-point error times max u|T|^2 times its bin count).  So
//   |dF| <~ sqrt 2 (kappa + sqrt(2F)) b sqrt(sum (e m)^2 sum u) + b^2 sum g / 2
// with b = |beta_+| + |beta_x| and kappa = kRefineKappa covering six standard
// deviations of the noise and an unmatched signal of SNR 10 in the
// partition.  Where this exceeds budget * max(|F|, 1), the items whose share
// of either term is above half the budget's share are evaluated again
// exactly, which brings the remainder under the budget.  Partitions within a
// factor kFragile of the pseudo-inverse cut are refined whole (a small error
// could flip the rank decision).
constexpr double kRefineKappa = 16.0;
constexpr double kFragile = 1e3;
__global__ void k_mark(const PartConst* __restrict__ pc, int64_t n, int32_t stride,
                       const int32_t* __restrict__ cnt, const int32_t* __restrict__ off,
                       const double* __restrict__ partials, const uint8_t* __restrict__ xflag,
                       const float2* __restrict__ xerr, double budget,
                       int32_t* __restrict__ refine, int32_t* __restrict__ nrefine) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n * stride) return;
  int64_t p = q / stride;
  int l = (int)(q - p * stride);
  const PartConst& P = pc[p];
  if (l >= P.np || P.status != kStatusOk) return;
  const int o = off[q], c = cnt[q];
  int ninterp = 0;
  double s2 = 0.0, mt = 0.0;
  for (int i = 0; i < c; ++i)
    if (xflag[o + i] == 0) {
      ++ninterp;
      const float2 x = xerr[o + i];
      s2 = fma((double)x.x, (double)x.x, s2);
      mt += (double)x.y;
    }
  if (ninterp == 0) return;
  double a[8], e[8];
  for (int k = 0; k < 8; ++k) a[k] = e[k] = 0.0;
  for (int i = 0; i < c; ++i)
    for (int k = 0; k < 8; ++k) {
      double x = partials[(int64_t)(o + i) * 8 + k];
      double t = a[k] + x;
      e[k] += (fabs(a[k]) >= fabs(x)) ? (a[k] - t) + x : (x - t) + a[k];
      a[k] = t;
    }
  for (int k = 0; k < 8; ++k) a[k] += e[k];
  const double Pm = a[4], Qm = a[5], rr = a[6], ri = a[7];
  const double hs = 0.5 * (Pm + Qm), hd = 0.5 * (Pm - Qm);
  const double lp = hs + sqrt(hd * hd + rr * rr + ri * ri);
  const double lm = (Pm * Qm - (rr * rr + ri * ri)) / lp;
  const bool all = !(lp > 0.0) || !(lm > kFragile * kRankCut * lp);
  double thr_t = 0.0, thr_m = 0.0;
  if (!all) {
    double beta[4];
    solve_beta(a, beta);
    const double F = solve_partition(a);
    const double b = hypot(beta[0], beta[1]) + hypot(beta[2], beta[3]);
    const double kt = 1.4142135623730951 * (kRefineKappa + sqrt(2.0 * fmax(F, 0.0))) * b;
    const double km = 0.5 * b * b;
    const double tol = budget * fmax(fabs(F), 1.0);
    if (kt * sqrt(s2) + km * mt <= tol) return;
    // refining every item above these leaves at most tol / 2 in each term
    thr_t = 0.5 * tol / (kt * sqrt((double)ninterp));
    thr_m = 0.5 * tol / (km * (double)ninterp);
  }
  auto sel = [&](int i) {
    if (xflag[o + i] != 0) return false;
    const float2 x = xerr[o + i];
    return all || (double)x.x > thr_t || (double)x.y > thr_m;
  };
  int nsel = 0;
  for (int i = 0; i < c; ++i)
    if (sel(i)) ++nsel;
  int at = atomicAdd(nrefine, nsel);
  for (int i = 0; i < c; ++i)
    if (sel(i)) refine[at++] = o + i;
}

// Bins of the last evaluation's items by the kind of per-bin work the
// interpolating loop did on them: out[0..2] direct phase and sine per bin at
// transfer degree 5, 7, 9, out[3..5] the difference recurrence at degree 5, 7,
// 9 (mixed path: [0] degree 4 and [2] degree 6 with all nine phase
// differences, [3] and [5] the same with four), out[6] evaluated exactly
// (rejects; refined items count where the interpolating loop ran them).
// out[7 + k] (k < 6): the lanes with bins (runs) of the items of kind k, each
// of which does its kind's per-lane work once (recurrence set-up, moments to
// power form, coefficients); out[13]: items evaluated exactly.
template <bool MIXED>
__global__ __launch_bounds__(256) void k_bin_mix(const int2* __restrict__ items,
                                                 const int32_t* __restrict__ total,
                                                 const int32_t* __restrict__ bounds,
                                                 int32_t stride, int32_t T, int32_t nch,
                                                 const double* __restrict__ rec,
                                                 const uint8_t* __restrict__ xflag,
                                                 unsigned long long* __restrict__ out) {
  typedef RecLayout<MIXED> L;
  __shared__ unsigned long long acc[kBinMix];
  if (threadIdx.x < kBinMix) acc[threadIdx.x] = 0ull;
  __syncthreads();
  const int W = total[0];
  for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < W; w += gridDim.x * blockDim.x) {
    const int2 it = items[w];
    const int p = it.x / stride, l = it.x - p * stride;
    const int32_t* bp = bounds + (int64_t)p * (stride + 1);
    int ct, ch, b0, b1;
    item_split(it.y, nch, ct, ch);
    item_bins(bp[l], bp[l + 1], ct, T, b0, b1);
    const int nb = b1 - b0;
    int kind = 6, runs = 1;
    if (!xflag[w]) {
      const double* r = rec + (int64_t)w * kRec;
      const int deg = (int)r[L::tail + 4];
      const bool dr = r[L::tail + 3] == 2.0;
      kind = (MIXED ? (deg == kDegTLow ? 0 : 2) : (deg == 5 ? 0 : (deg == 7 ? 1 : 2))) + (dr ? 3 : 0);
      // the recurrence's and the mixed loop's lanes take runs of Lr
      // contiguous bins, the FP64 direct form's lanes every 64th bin
      const int Lr = ((nb + 63) >> 6) | 1;
      runs = (MIXED || dr) ? (nb + Lr - 1) / Lr : min(nb, 64);
    }
    atomicAdd(&acc[kind], (unsigned long long)nb);
    atomicAdd(&acc[7 + kind], (unsigned long long)runs);
  }
  __syncthreads();
  if (threadIdx.x < kBinMix && acc[threadIdx.x]) atomicAdd(&out[threadIdx.x], acc[threadIdx.x]);
}

void launch_bin_mix(bool mixed, int32_t stride, int32_t chunk, int32_t nch, const WorkSpace& ws,
                    unsigned long long* out, hipStream_t s) {
  hipLaunchKernelGGL(mixed ? k_bin_mix<true> : k_bin_mix<false>, dim3(1024), dim3(256), 0, s,
                     ws.items, ws.total, ws.bounds, stride, chunk, nch, ws.rec, ws.xflag, out);
}

// ---- grouping of the work items by bin tile ---------------------------------
__global__ void k_tile_zero(int32_t* __restrict__ tcnt, int32_t* __restrict__ tcur, int32_t ntiles,
                            int32_t* __restrict__ tile_ctr) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ntiles) { tcnt[i] = 0; tcur[i] = 0; }
  if (i == 0) tile_ctr[0] = 0;
}

// Items per tile.  When the tiles fit in LDS the block first counts its own
// items there and then adds its non-zero counts to the global ones: with few
// tiles (a narrow band) every item would otherwise hit the same few counters.
constexpr int kTileHist = 8192;

__global__ __launch_bounds__(256) void k_tile_count(const int2* __restrict__ items,
                                                    const int32_t* __restrict__ total,
                                                    const int32_t* __restrict__ bounds,
                                                    int32_t stride, int32_t T, int32_t ntiles,
                                                    int32_t nch, int32_t* __restrict__ tcnt) {
  __shared__ int32_t h[kTileHist];
  const bool local = ntiles <= kTileHist;
  const int W = total[0];
  if (local) {
    for (int i = threadIdx.x; i < ntiles; i += blockDim.x) h[i] = 0;
    __syncthreads();
  }
  for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < W; w += gridDim.x * blockDim.x) {
    const int2 it = items[w];
    const int p = it.x / stride, l = it.x - p * stride;
    const int t = item_xtile(bounds[(int64_t)p * (stride + 1) + l], it.y, T, nch, ntiles);
    if (local) atomicAdd(&h[t], 1);
    else atomicAdd(&tcnt[t], 1);
  }
  if (local) {
    __syncthreads();
    for (int i = threadIdx.x; i < ntiles; i += blockDim.x)
      if (h[i]) atomicAdd(&tcnt[i], h[i]);
  }
}

// Exclusive scans of the per-tile item counts into off[0..n] and of the
// per-tile unit counts ceil(cnt / kUnitItems) into uoff[0..n] (a unit is the
// bin loop's scheduling step: one tile, up to kUnitItems of its items).  One
// block.

__global__ void k_tile_scan(const int32_t* __restrict__ tcnt, int32_t n, int32_t* __restrict__ off,
                            int32_t* __restrict__ uoff) {
  __shared__ int32_t part[1024], upart[1024];
  const int t = threadIdx.x, TB = blockDim.x;
  const int per = (n + TB - 1) / TB;
  const int a = t * per, b = min(n, a + per);
  int32_t sum = 0, usum = 0;
  for (int i = a; i < b; ++i) {
    sum += tcnt[i];
    usum += (tcnt[i] + kUnitItems - 1) / kUnitItems;
  }
  part[t] = sum;
  upart[t] = usum;
  __syncthreads();
  if (t == 0) {
    int32_t run = 0, urun = 0;
    for (int i = 0; i < TB; ++i) {
      int32_t x = part[i], y = upart[i];
      part[i] = run; upart[i] = urun;
      run += x; urun += y;
    }
    off[n] = run;
    uoff[n] = urun;
  }
  __syncthreads();
  int32_t run = part[t], urun = upart[t];
  for (int i = a; i < b; ++i) {
    off[i] = run; uoff[i] = urun;
    run += tcnt[i];
    urun += (tcnt[i] + kUnitItems - 1) / kUnitItems;
  }
}

// Items into tile order.  With the tiles in LDS, the block ranks its items per
// tile locally and reserves one range per tile with a single global atomic.
__global__ __launch_bounds__(256) void k_tile_scatter(const int2* __restrict__ items,
                                                      const int32_t* __restrict__ total,
                                                      const int32_t* __restrict__ bounds,
                                                      int32_t stride, int32_t T, int32_t ntiles,
                                                      int32_t nch,
                                                      const int32_t* __restrict__ off,
                                                      int32_t* __restrict__ tcur,
                                                      int32_t* __restrict__ tile_items) {
  __shared__ int32_t h[kTileHist];
  const bool local = ntiles <= kTileHist;
  const int W = total[0];
  if (!local) {
    for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < W; w += gridDim.x * blockDim.x) {
      const int2 it = items[w];
      const int p = it.x / stride, l = it.x - p * stride;
      const int t = item_xtile(bounds[(int64_t)p * (stride + 1) + l], it.y, T, nch, ntiles);
      tile_items[off[t] + atomicAdd(&tcur[t], 1)] = w;
    }
    return;
  }
  for (int i = threadIdx.x; i < ntiles; i += blockDim.x) h[i] = 0;
  __syncthreads();
  for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < W; w += gridDim.x * blockDim.x) {
    const int2 it = items[w];
    const int p = it.x / stride, l = it.x - p * stride;
    atomicAdd(&h[item_xtile(bounds[(int64_t)p * (stride + 1) + l], it.y, T, nch, ntiles)], 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < ntiles; i += blockDim.x)    // counts -> reserved bases
    if (h[i]) h[i] = off[i] + atomicAdd(&tcur[i], h[i]);
  __syncthreads();
  for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < W; w += gridDim.x * blockDim.x) {
    const int2 it = items[w];
    const int p = it.x / stride, l = it.x - p * stride;
    const int t = item_xtile(bounds[(int64_t)p * (stride + 1) + l], it.y, T, nch, ntiles);
    tile_items[atomicAdd(&h[t], 1)] = w;
  }
}

// every item is evaluated exactly: the reject count equals the item count
__global__ void k_copy_count(const int32_t* __restrict__ total, int32_t* __restrict__ ndirect) {
  if (threadIdx.x == 0) ndirect[0] = total[0];
}

// Chebyshev tables (long double on the host): node s_k = cos(pi (k + 1/2) / K);
// interpolant coefficients c_j = (2 / K) sum_k v_k cos(pi j (k + 1/2) / K)
// (c_0 halved) of p = sum_j c_j T_j(s); T_j expanded in monomials by
// T_{j+1} = 2 s T_j - T_{j-1}.
static double* g_ssum[64] = {};   // per device: S_j(nb) table (lives until the process ends)

int interp_tables_init() {
  static bool done[64] = {false};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  if (dev >= 0 && dev < 64 && done[dev]) return 0;
  const int K = kCheb;
  const long double pi = 3.141592653589793238462643383279502884L;
  long double M[kCheb][kCheb] = {};
  M[0][0] = 1.0L;
  M[1][1] = 1.0L;
  for (int j = 1; j + 1 < K; ++j)
    for (int n = 0; n < K; ++n)
      M[j + 1][n] = (n > 0 ? 2.0L * M[j][n - 1] : 0.0L) - M[j - 1][n];
  double S[kCheb], G[kCheb][kCheb], E[2][kCheb], G6[kCheb][kDegT + 1], E6[2][kCheb];
  for (int kk = 0; kk < K; ++kk) {
    S[kk] = (double)cosl(pi * (kk + 0.5L) / K);
    long double lm = 0.0L, lp = 0.0L, lm6 = 0.0L, lp6 = 0.0L;
    for (int n = 0; n < K; ++n) {
      long double gsum = 0.0L, g6 = 0.0L;
      for (int j = 0; j < K; ++j) {
        long double cj = (2.0L / K) * cosl(pi * j * (kk + 0.5L) / K) * (j == 0 ? 0.5L : 1.0L);
        gsum += cj * M[j][n];
        if (j <= kDegT) g6 += cj * M[j][n];
      }
      G[kk][n] = (double)gsum;
      lp += gsum;
      lm += (n & 1) ? -gsum : gsum;
      if (n <= kDegT) {
        G6[kk][n] = (double)g6;
        lp6 += g6;
        lm6 += (n & 1) ? -g6 : g6;
      }
    }
    E[0][kk] = (double)lm;
    E[1][kk] = (double)lp;
    E6[0][kk] = (double)lm6;
    E6[1][kk] = (double)lp6;
  }
  if (hipMemcpyToSymbol(HIP_SYMBOL(c_cheb_s), S, sizeof(S)) != hipSuccess) return -1;
  double R9[kCheb][kLanesItem], R6[kCheb][kLanesItem];
  for (int kk = 0; kk < K; ++kk) {
    for (int n = 0; n < K; ++n) {
      R9[kk][n] = G[kk][n];
      R6[kk][n] = n <= kDegT ? G6[kk][n] : 0.0;
    }
    for (int e = 0; e < 2; ++e) {
      R9[kk][kCheb + e] = E[e][kk];
      R6[kk][kCheb + e] = E6[e][kk];
    }
  }
  if (hipMemcpyToSymbol(HIP_SYMBOL(c_row9), R9, sizeof(R9)) != hipSuccess) return -1;
  {
    double2 tab[kSinTab];
    for (int i = 0; i < kSinTab; ++i) {
      const long double a = 2.0L * pi * (long double)i / (long double)kSinTab;
      tab[i] = make_double2((double)sinl(a), (double)cosl(a));
    }
    if (hipMemcpyToSymbol(HIP_SYMBOL(c_sincos), tab, sizeof(tab)) != hipSuccess) return -1;
  }
  if (hipMemcpyToSymbol(HIP_SYMBOL(c_row6), R6, sizeof(R6)) != hipSuccess) return -1;
  // truncations after degree 5 and 7 (FP64 loop)
  double Gt[2][kCheb][kCheb], Et[2][2][kCheb];
  for (int v = 0; v < 2; ++v) {
    const int dmax = v == 0 ? 5 : 7;
    for (int kk = 0; kk < K; ++kk) {
      long double lm = 0.0L, lp = 0.0L;
      for (int n = 0; n < K; ++n) {
        long double gsum = 0.0L;
        for (int j = 0; j <= dmax; ++j)
          gsum += (2.0L / K) * cosl(pi * j * (kk + 0.5L) / K) * (j == 0 ? 0.5L : 1.0L) * M[j][n];
        Gt[v][kk][n] = (double)gsum;
        lp += gsum;
        lm += (n & 1) ? -gsum : gsum;
      }
      Et[v][0][kk] = (double)lm;
      Et[v][1][kk] = (double)lp;
    }
  }
  double Rt[2][kCheb][kLanesItem];
  for (int v = 0; v < 2; ++v)
    for (int kk = 0; kk < K; ++kk) {
      for (int n = 0; n < K; ++n) Rt[v][kk][n] = Gt[v][kk][n];
      for (int e = 0; e < 2; ++e) Rt[v][kk][kCheb + e] = Et[v][e][kk];
    }
  if (hipMemcpyToSymbol(HIP_SYMBOL(c_rowt), Rt, sizeof(Rt)) != hipSuccess) return -1;
  {
    // truncation after degree kDegTLow (mixed loop)
    double R4[kCheb][kLanesItem];
    for (int kk = 0; kk < K; ++kk) {
      long double lm = 0.0L, lp = 0.0L;
      for (int n = 0; n < K; ++n) {
        long double gsum = 0.0L;
        for (int j = 0; j <= kDegTLow; ++j)
          gsum += (2.0L / K) * cosl(pi * j * (kk + 0.5L) / K) * (j == 0 ? 0.5L : 1.0L) * M[j][n];
        R4[kk][n] = (double)gsum;
        lp += gsum;
        lm += (n & 1) ? -gsum : gsum;
      }
      R4[kk][kCheb] = (double)lm;
      R4[kk][kCheb + 1] = (double)lp;
    }
    if (hipMemcpyToSymbol(HIP_SYMBOL(c_row4), R4, sizeof(R4)) != hipSuccess) return -1;
  }
  // quadrature weights' Chebyshev part (even degrees only)
  double D[5][kCheb];
  for (int i = 0; i < 5; ++i)
    for (int kk = 0; kk < K; ++kk)
      D[i][kk] = (double)((2.0L / K) * cosl(pi * (2 * i) * (kk + 0.5L) / K) * (i == 0 ? 0.5L : 1.0L));
  if (hipMemcpyToSymbol(HIP_SYMBOL(c_cheb_D), D, sizeof(D)) != hipSuccess) return -1;
  // inverse Gram matrix of the u-tile least-squares fit (Gauss-Jordan)
  long double Gm[kUCoef][2 * kUCoef] = {};
  for (int m = 0; m < kUTile; ++m) {
    const long double s = 2.0L * m / (kUTile - 1) - 1.0L;
    long double tv[kUCoef];
    tv[0] = 1.0L;
    tv[1] = s;
    for (int k = 2; k < kUCoef; ++k) tv[k] = 2.0L * s * tv[k - 1] - tv[k - 2];
    for (int a = 0; a < kUCoef; ++a)
      for (int b = 0; b < kUCoef; ++b) Gm[a][b] += tv[a] * tv[b];
  }
  for (int a = 0; a < kUCoef; ++a) Gm[a][kUCoef + a] = 1.0L;
  for (int c = 0; c < kUCoef; ++c) {
    int piv = c;
    for (int r = c + 1; r < kUCoef; ++r)
      if (fabsl(Gm[r][c]) > fabsl(Gm[piv][c])) piv = r;
    for (int b = 0; b < 2 * kUCoef; ++b) { long double x = Gm[c][b]; Gm[c][b] = Gm[piv][b]; Gm[piv][b] = x; }
    const long double d = Gm[c][c];
    for (int b = 0; b < 2 * kUCoef; ++b) Gm[c][b] /= d;
    for (int r = 0; r < kUCoef; ++r)
      if (r != c) {
        const long double f = Gm[r][c];
        for (int b = 0; b < 2 * kUCoef; ++b) Gm[r][b] -= f * Gm[c][b];
      }
  }
  double Gi[kUCoef][kUCoef];
  for (int a = 0; a < kUCoef; ++a)
    for (int b = 0; b < kUCoef; ++b) Gi[a][b] = (double)Gm[a][kUCoef + b];
  if (hipMemcpyToSymbol(HIP_SYMBOL(c_ufit_Ginv), Gi, sizeof(Gi)) != hipSuccess) return -1;
  // quadrature table S_j(nb), one per device
  double* tab = nullptr;
  if (hipMalloc((void**)&tab, sizeof(double) * 5 * (kSsumMax + 1)) != hipSuccess) return -1;
  hipLaunchKernelGGL(k_cheb_sums, dim3((kSsumMax + 256) / 256), dim3(256), 0, 0, tab);
  if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) return -1;
  if (dev >= 0 && dev < 64) {
    g_ssum[dev] = tab;
    done[dev] = true;
  }
  return 0;
}

const double* cheb_sums_table() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  return g_ssum[dev];
}

// ---------------------------------------------------------------------------
// surrogate for the eccentric phase term (App. A): training data, knots,
// spot check against the analytic term, per-particle decision
// ---------------------------------------------------------------------------
// network inputs (f, Mc, e0) mapped to [-1, 1] over f in [10, 100] mHz,
// Mc in [10, 50] Msun, e0 in [0, 0.15]
__device__ __forceinline__ float nn_f(double f) { return (float)(2.0 * (f - 0.01) / 0.09 - 1.0); }

// Training samples from the plain template code: target y = te / (ecc_k tN),
// the eccentric term in units of e0^2 and the Newtonian phase.
__global__ void k_sur_data(uint64_t seed, int64_t n, float* __restrict__ X, float* __restrict__ T) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t ctr[4] = {(uint64_t)i, 0ull, 0ull, 0ull}, o[4];
  philox4x64_10(ctr, seed, 0x5u, o);
  double u0 = (double)(o[0] >> 11) * 0x1.0p-53, u1 = (double)(o[1] >> 11) * 0x1.0p-53,
         u2 = (double)(o[2] >> 11) * 0x1.0p-53;
  double f = 0.01 + 0.09 * u0, mc = 10.0 + 40.0 * u1, e0 = 1e-4 + (0.15 - 1e-4) * u2;
  double th[6] = {0.0, mc, 0.0, 0.0, 0.0, e0};
  PartConst P;
  fill_constants(P, th);
  double tN, te;
  newton_and_ecc(P, f, tN, te);
  T[i] = (float)(te / (P.ecc_k * tN));
  X[3 * i + 0] = nn_f(f);
  X[3 * i + 1] = (float)P.nn_mc;
  X[3 * i + 2] = (float)P.nn_e0;
}

// four knots per partition (bins spread evenly over the partition), for
// particles with Np >= kSurMinNp; one thread per (partition, knot)
__device__ __forceinline__ bool sur_candidate(const PartConst& P, int l, const int32_t* bp) {
  return P.status == kStatusOk && P.np >= kSurMinNp && l < P.np && (bp[l + 1] - bp[l]) >= 4;
}
__device__ __forceinline__ int knot_bin(const int32_t* bp, int l, int a) {
  int nb = bp[l + 1] - bp[l];
  return bp[l] + (a * (nb - 1)) / 3;
}

__global__ void k_sur_knots(Grid g, const PartConst* __restrict__ pc,
                            const int32_t* __restrict__ bounds, int32_t stride, int64_t n,
                            int64_t rows, float* __restrict__ X) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows) return;
  if (t >= n * stride * 4) {   // padding rows of the network batch
    X[3 * t + 0] = 0.f; X[3 * t + 1] = 0.f; X[3 * t + 2] = 0.f;
    return;
  }
  int64_t q = t >> 2;
  int a = (int)(t & 3);
  int64_t p = q / stride;
  int l = (int)(q - p * stride);
  const PartConst& P = pc[p];
  const int32_t* bp = bounds + p * (stride + 1);
  float x0 = 0.f, x1 = 0.f, x2 = 0.f;
  if (sur_candidate(P, l, bp)) {
    x0 = nn_f(bin_freq(g, knot_bin(bp, l, a)));
    x1 = (float)P.nn_mc;
    x2 = (float)P.nn_e0;
  }
  X[3 * t + 0] = x0; X[3 * t + 1] = x1; X[3 * t + 2] = x2;
}

// knot values -> Lagrange coefficients; mismatch estimate from the residual of
// the interpolated surrogate against the analytic term at the four knots and
// the three mid-points, after removing its mean (a constant phase per
// partition is absorbed by the statistic): mm = (2 pi)^2 var(residual)
__global__ void k_sur_check(Grid g, const PartConst* __restrict__ pc,
                            const int32_t* __restrict__ bounds, int32_t stride, int64_t n,
                            const float* __restrict__ ynn, double* __restrict__ ek,
                            double* __restrict__ mm) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n * stride) return;
  int64_t p = q / stride;
  int l = (int)(q - p * stride);
  const PartConst& P = pc[p];
  const int32_t* bp = bounds + p * (stride + 1);
  if (!sur_candidate(P, l, bp)) {
    mm[q] = (P.status == kStatusOk && P.np >= kSurMinNp && l < P.np) ? 1e300 : 0.0;
    return;
  }
  double xa[4], va[4];
  for (int a = 0; a < 4; ++a) {
    xa[a] = bin_freq(g, knot_bin(bp, l, a));
    double tN, te;
    newton_and_ecc(P, xa[a], tN, te);
    va[a] = P.ecc_k * tN * (double)ynn[4 * q + a];
  }
  double* e = ek + 8 * q;
  for (int a = 0; a < 4; ++a) {
    double den = 1.0;
    for (int b = 0; b < 4; ++b)
      if (b != a) den *= xa[a] - xa[b];
    e[a] = xa[a];
    e[4 + a] = va[a] / den;
  }
  double r[7], mean = 0.0;
  for (int i = 0; i < 7; ++i) {
    int j = (i < 4) ? knot_bin(bp, l, i)
                    : (knot_bin(bp, l, i - 4) + knot_bin(bp, l, i - 3)) / 2;
    double f = bin_freq(g, j);
    double tN, te;
    newton_and_ecc(P, f, tN, te);
    r[i] = knot_interp(e, f) - te;
    mean += r[i];
  }
  mean /= 7.0;
  double var = 0.0;
  for (int i = 0; i < 7; ++i) var += (r[i] - mean) * (r[i] - mean);
  mm[q] = 4.0 * kPi * kPi * var / 7.0;
}

// particle uses the surrogate when every partition's estimate is <= thr
__global__ void k_sur_decide(PartConst* __restrict__ pc, int64_t n, int32_t stride,
                             const double* __restrict__ mm, double thr,
                             unsigned long long* __restrict__ counters) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  PartConst& P = pc[p];
  if (P.status != kStatusOk || P.np < kSurMinNp) return;
  double worst = 0.0;
  for (int l = 0; l < P.np; ++l) worst = fmax(worst, mm[p * stride + l]);
  int use = worst <= thr ? 1 : 0;
  P.sur = use;
  atomicAdd(counters + (use ? 0 : 1), 1ull);
}

// ---------------------------------------------------------------------------
// solve and mean
// ---------------------------------------------------------------------------
// Constant phase (turns) the statistic's template drops and the App. A
// waveform carries: -1/8 and the f-independent part of the alpha_5 term,
// c5' cN vfac^5 (1 + 3 ln sqrt 6).
__device__ __forceinline__ double dropped_phase(const PartConst& P) {
  double ph0 = -0.125 + P.c5v5 * (1.0 + 1.5 * log(6.0));
  return ph0 - rint(ph0);
}

// a_1..a_4 of the App. B basis from the pair beta solved against the scaled
// bin data (w, u) -> (gam w, gam^2 u): the template's beta is gam beta, the
// dropped phase turns it by e^{2 pi i ph0}, and s = (a1 - i a3) T+ g +
// (-a2 + i a4) Tx g.
__device__ __forceinline__ void amps_from_beta(const PartConst& P, const double* b, double gam,
                                               double* a) {
  double sc, cc;
  sincospi(2.0 * dropped_phase(P), &sc, &cc);
  const double pr = gam * (b[0] * cc - b[1] * sc), pi = gam * (b[1] * cc + b[0] * sc);
  const double xr = gam * (b[2] * cc - b[3] * sc), xi = gam * (b[3] * cc + b[2] * sc);
  a[0] = pr;
  a[1] = -xr;
  a[2] = -pi;
  a[3] = xi;
}

__global__ void k_solve(const PartConst* __restrict__ pc, int64_t n, int32_t stride,
                        const int32_t* __restrict__ cnt, const int32_t* __restrict__ off,
                        const double* __restrict__ partials, double* __restrict__ Fl,
                        double* __restrict__ F_part, int64_t part_stride,
                        double* __restrict__ amps, const double* __restrict__ umax) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n * stride) return;
  int64_t p = q / stride;
  int l = (int)(q - p * stride);
  const PartConst& P = pc[p];
  if (l >= P.np || P.status == kStatusInvalid) return;
  double F = 0.0;
  double am[4] = {0.0, 0.0, 0.0, 0.0};
  if (P.status == kStatusOk) {
    double a[8], e[8];
    for (int k = 0; k < 8; ++k) a[k] = e[k] = 0.0;
    int o = off[q], c = cnt[q];
    for (int i = 0; i < c; ++i)
      for (int k = 0; k < 8; ++k) {  // Neumaier sum over the chunks, in order
        double x = partials[(int64_t)(o + i) * 8 + k];
        double t = a[k] + x;
        e[k] += (fabs(a[k]) >= fabs(x)) ? (a[k] - t) + x : (x - t) + a[k];
        a[k] = t;
      }
    for (int k = 0; k < 8; ++k) a[k] += e[k];
    F = solve_partition(a);
    if (amps) {
      double beta[4];
      solve_beta(a, beta);
      const double m = umax[0];
      amps_from_beta(P, beta, m > 0.0 ? sqrt(1.0 / m) : 1.0, am);
    }
  }
  Fl[q] = F;
  if (F_part) F_part[p * part_stride + l] = F;
  if (amps)
    for (int k = 0; k < 4; ++k) amps[(p * part_stride + l) * 4 + k] = am[k];
}

// One wavefront per particle: lanes take every 64th partition, then a fixed
// butterfly (the result does not depend on the launch).
__global__ void k_mean(const PartConst* __restrict__ pc, int64_t n, int32_t stride,
                       const double* __restrict__ Fl, double* __restrict__ F_hat,
                       double* __restrict__ F_part, int64_t part_stride,
                       double* __restrict__ amps, unsigned long long* __restrict__ bin_counter) {
  const int lane = threadIdx.x & 63;
  const int64_t p = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (p >= n) return;
  const PartConst& P = pc[p];
  if (P.status == kStatusInvalid) {
    if (lane == 0) F_hat[p] = __builtin_nan("");
    for (int l = lane; l < P.np && l < part_stride; l += 64) {
      if (F_part) F_part[p * part_stride + l] = __builtin_nan("");
      if (amps)
        for (int k = 0; k < 4; ++k) amps[(p * part_stride + l) * 4 + k] = __builtin_nan("");
    }
    return;
  }
  if (P.status == kStatusEmpty) {
    if (lane == 0) F_hat[p] = -__builtin_inf();
    return;
  }
  double s = 0.0;
  for (int l = lane; l < P.np; l += 64) s += Fl[p * stride + l];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) {
    F_hat[p] = s / (double)P.np;
    if (bin_counter) atomicAdd(bin_counter, (unsigned long long)(P.j_hi - P.j_lo + 1));
  }
}

// ---------------------------------------------------------------------------
// template signal (for injections): sum_i a_i A^i with the full transfer
// ---------------------------------------------------------------------------
__global__ void k_waveform(Grid g, const PartConst* __restrict__ pc,
                           const double* __restrict__ amps, double* __restrict__ out) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= g.nbins) return;
  const PartConst& P = pc[0];
  if (P.status != kStatusOk || j < P.j_lo || j > P.j_hi) {
    out[2 * j] = 0.0;
    out[2 * j + 1] = 0.0;
    return;
  }
  double f = bin_freq(g, j);
  double s0, c0;
  sincospi(kLs * f, &s0, &c0);
  double cph, sph, tpr, tpi, txr, txi;
  template_fp64(P, f, s0, c0, cph, sph, tpr, tpi, txr, txi, nullptr, g.chan.code[0], &g.orb);
  // restore the constant phase the statistic drops
  double sc, cc;
  sincospi(2.0 * dropped_phase(P), &sc, &cc);
  double cps = cph * cc - sph * sc, sps = sph * cc + cph * sc;   // e^{i Phi_full}
  // full transfer: C(f) times the particle part T''
  double x0 = kPi * kLs * f;
  double zr = c0 * c0 - s0 * s0, zi = -2.0 * s0 * c0;
  double omr = 1.0 - (zr * zr - zi * zi), omi = -2.0 * zr * zi;
  double er = -x0 * s0, ei = -x0 * c0;
  double Cr = omr * er - omi * ei, Ci = omr * ei + omi * er;
  double Tpr = Cr * tpr - Ci * tpi, Tpi = Cr * tpi + Ci * tpr;
  double Txr = Cr * txr - Ci * txi, Txi = Cr * txi + Ci * txr;
  // h = f^{-7/6} e^{-i Phi} [(a1 - i a3) T+ + (-a2 + i a4) Tx]  (App. B basis)
  double a1 = amps[0], a2 = amps[1], a3 = amps[2], a4 = amps[3];
  double hr = (a1 * Tpr + a3 * Tpi) + (-a2 * Txr - a4 * Txi);
  double hi = (a1 * Tpi - a3 * Tpr) + (-a2 * Txi + a4 * Txr);
  double amp = pow(f, -7.0 / 6.0);
  // multiply by e^{-i Phi} = cps - i sps
  out[2 * j] = amp * (hr * cps + hi * sps);
  out[2 * j + 1] = amp * (hi * cps - hr * sps);
}

// ---------------------------------------------------------------------------
// extrinsic parameters from a_1..a_4 (App. B, Eq. extrinPara), one row per
// thread.  D_L = 2 / A and iota = arccos(-Ax / A) as printed.  For psi and
// phi_c the kernel uses the phases of the two circular parts of a,
//   (a1 + a4) + i (a2 - a3) = r1 e^{i (phi_c - 2 psi)},
//   (a1 - a4) - i (a2 + a3) = r2 e^{i (phi_c + 2 psi)},
// which give the same (psi, phi_c) as the printed arctangent ratios (whose
// arguments are 2 r1 r2 sin 2psi sin phi_c, 2 r1 r2 cos 2psi sin phi_c and
// 2 r1 r2 sin 2psi cos phi_c, read with the sign c = sgn(sin 2 psi)) and the
// same representative, phi_c in (0, pi] and psi in (-pi/2, pi/2], but stay
// accurate where those ratios approach 0/0.  At iota = 0 or pi one circular
// part vanishes (modulus below 64 ulp of the other) and only the other's
// phase is defined: psi = 0, phi_c = that phase.  All-zero a gives
// (inf, nan, nan, nan).  With the chirp mass (params != null) D_L is
// converted to metres with the App. A constant |A| D_L = sqrt(5/24)
// Mc^{5/6} / pi^{2/3} (geometric units), whose negative sign turns phi_c by pi.
// ---------------------------------------------------------------------------
__global__ void k_extrinsic(const double* __restrict__ amps, const double* __restrict__ params,
                            int64_t n, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a1 = amps[4 * i], a2 = amps[4 * i + 1], a3 = amps[4 * i + 2], a4 = amps[4 * i + 3];
  const double p1 = a1 + a4, p2 = a2 - a3, m1 = a1 - a4, m2 = -(a2 + a3);
  const double r1 = sqrt(p1 * p1 + p2 * p2), r2 = sqrt(m1 * m1 + m2 * m2);
  const double Ap = r1 + r2, Ax = r1 - r2;
  const double A = Ap + sqrt(fmax((Ap - Ax) * (Ap + Ax), 0.0));   // no cancellation at iota ~ 0
  double D, iota, psi, phic;
  if (!(A > 0.0)) {
    const double nan = __builtin_nan("");
    D = (A == 0.0) ? __builtin_inf() : nan;
    iota = psi = phic = nan;
  } else {
    D = 2.0 / A;
    iota = acos(fmin(fmax(-Ax / A, -1.0), 1.0));
    const double th1 = atan2(p2, p1);    // phi_c - 2 psi
    const double th2 = atan2(m2, m1);    // phi_c + 2 psi
    if (fmin(r1, r2) <= 64.0 * 2.220446049250313e-16 * fmax(r1, r2)) {
      psi = 0.0;
      phic = (r1 < r2) ? th2 : th1;
    } else {
      phic = 0.5 * (th1 + th2);          // (-pi, pi], defined modulo pi
      if (phic <= 0.0) phic += kPi;
      double d = th2 - phic;             // 2 psi, in (-2 pi, pi]
      if (d <= -kPi) d += 2.0 * kPi;
      psi = 0.5 * d;
    }
    if (params) {
      const double mc = params[6 * i + 1] * kMsunS;
      D *= kC * sqrt(5.0 / 24.0) * pow(mc, 5.0 / 6.0) / pow(kPi, 2.0 / 3.0);
      phic += (phic > 0.0) ? -kPi : kPi;
    }
  }
  out[4 * i] = D;
  out[4 * i + 1] = iota;
  out[4 * i + 2] = psi;
  out[4 * i + 3] = phic;
}

}  // namespace fstat

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
namespace fstat {

static inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

void launch_prep(const Grid& g, const double* data, const double* psd, BinData<double> b,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_prep, dim3(nblk(g.nbins, 256), g.chan.n), dim3(256), 0, s, g, data, psd, b.wr, b.wi,
                     b.u, b.s0, b.c0);
}

void launch_max(const double* u, int64_t n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_max, dim3(1), dim3(1024), 0, s, u, n, out);
}

void launch_scale(const Grid& g, const double* umax, BinData<double> b, BinData<float> b32,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(nblk(g.nbins, 256), g.chan.n), dim3(256), 0, s, g, umax, b.wr, b.wi, b.u,
                     b.s0, b.c0, b32.wr, b32.wi, b32.u, b32.s0, b32.c0);
}

void launch_setup(const Grid& g, const double* params, int64_t n,
                  const int32_t* np, int32_t np_uniform, int32_t stride, int32_t chunk,
                  const uint8_t* skip, const WorkSpace& ws, hipStream_t s) {
  hipLaunchKernelGGL(k_setup, dim3(nblk(n * 64, 256)), dim3(256), 0, s, g, params, n, np, np_uniform,
                     stride, chunk, skip, ws.pc, ws.bounds, ws.cnt);
}

void launch_worklist(int64_t m, const WorkSpace& ws, hipStream_t s) {
  const int32_t nb = (int32_t)((m + kScanBlock - 1) / kScanBlock);
  hipLaunchKernelGGL(k_scan_sums, dim3(nb), dim3(1024), 0, s, ws.cnt, m, ws.bsum);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, ws.bsum, nb, ws.total, ws.ndirect,
                     ws.nrefine);
  hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(1024), 0, s, ws.cnt, m, ws.bsum, ws.off);
  hipLaunchKernelGGL(k_fill, dim3(nblk(m, 256)), dim3(256), 0, s, ws.cnt, ws.off, m, ws.items);
}

int interp_max_tile(bool mixed) { return mixed ? kMaxTileMixed : kMaxTileFp64; }

void launch_eval(bool mixed, bool interp, double refine_budget, const Grid& g,
                 int64_t n_particles, int32_t stride, int32_t chunk, const WorkSpace& ws,
                 BinData<double> b, BinData<float> b32, const double* ek, int blocks,
                 hipStream_t s, hipEvent_t* ev_main, const UModel& um) {
  const int32_t* sel = nullptr;
  const int32_t* nsel = nullptr;
  if (!interp) hipLaunchKernelGGL(k_copy_count, dim3(1), dim3(64), 0, s, ws.total, ws.ndirect);
  if (interp) {
    const int32_t ntiles = (int32_t)((g.nbins + chunk - 1) / chunk) * g.chan.n;   // all channels
    hipLaunchKernelGGL(k_tile_zero, dim3(nblk(ntiles, 256)), dim3(256), 0, s, ws.tcnt, ws.tcur,
                       ntiles, ws.tile_ctr);
    hipLaunchKernelGGL(k_tile_count, dim3(1024), dim3(256), 0, s, ws.items, ws.total, ws.bounds,
                       stride, chunk, ntiles, g.chan.n, ws.tcnt);
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, s, ws.tcnt, ntiles, ws.toff, ws.uoff);
    hipLaunchKernelGGL(k_tile_scatter, dim3(1024), dim3(256), 0, s, ws.items, ws.total, ws.bounds,
                       stride, chunk, ntiles, g.chan.n, ws.toff, ws.tcur, ws.tile_items);
    {
      const bool tab = g.orb.coef != nullptr;
      auto nodes = mixed ? (tab ? k_interp_nodes<true, true> : k_interp_nodes<true, false>)
                         : (tab ? k_interp_nodes<false, true> : k_interp_nodes<false, false>);
      hipLaunchKernelGGL(nodes, dim3(blocks), dim3(256), 0, s, g, ws.pc, ws.bounds, stride,
                         ws.items, ws.total, chunk, ek, ws.rec, ws.xflag, ws.xerr, ws.direct,
                         ws.ndirect, um, ws.partials);
    }
    // w (and e_j on the FP64 path) at the largest tile's stride
    const size_t lds = mixed ? (size_t)kMaxTileMixed * 2 * sizeof(float)
                             : (size_t)kMaxTileFp64 * (2 * sizeof(double) + sizeof(float));
    if (ev_main) (void)hipEventRecord(ev_main[0], s);
    if (mixed)
      hipLaunchKernelGGL(k_eval_interp<true>, dim3(blocks), dim3(256), lds, s, g, chunk,
                         ws.tile_items, ws.toff, ws.uoff, ntiles, ws.tile_ctr, b.wr, b.wi,
                         b32.wr, b32.wi, ws.rec, ws.partials);
    else
      hipLaunchKernelGGL(k_eval_interp<false>, dim3(blocks), dim3(256), lds, s, g, chunk,
                         ws.tile_items, ws.toff, ws.uoff, ntiles, ws.tile_ctr, b.wr, b.wi,
                         b32.wr, b32.wi, ws.rec, ws.partials);
    if (ev_main) (void)hipEventRecord(ev_main[1], s);
    sel = ws.direct;
    nsel = ws.ndirect;
  }
  auto exact_pass = [&](const int32_t* list, const int32_t* count) {
    hipLaunchKernelGGL(mixed ? k_eval_exact<true> : k_eval_exact<false>, dim3(blocks), dim3(256),
                       0, s, g, ws.pc, ws.bounds, stride, ws.items, ws.total, chunk, b.wr, b.wi,
                       b.u, b32.wr, b32.wi, b32.u, b.s0, b.c0, ek, ws.partials, list, count);
  };
  if (!interp && ev_main) (void)hipEventRecord(ev_main[0], s);
  exact_pass(sel, nsel);
  if (!interp && ev_main) (void)hipEventRecord(ev_main[1], s);
  if (interp && !mixed && refine_budget > 0.0) {
    // the mixed path's bar (1e-4 + 1e-6 cond) already covers the interpolation error
    const int64_t m = (int64_t)n_particles * stride;
    hipLaunchKernelGGL(k_mark, dim3(nblk(m, 256)), dim3(256), 0, s, ws.pc, n_particles, stride,
                       ws.cnt, ws.off, ws.partials, ws.xflag, ws.xerr, refine_budget, ws.refine,
                       ws.nrefine);
    exact_pass(ws.refine, ws.nrefine);
  }
}

void launch_solve_mean(int64_t n, int32_t stride, const WorkSpace& ws, double* F_hat,
                       double* F_part, double* amps, int64_t part_stride, const double* umax,
                       unsigned long long* bin_counter, hipStream_t s) {
  int64_t m = n * stride;
  hipLaunchKernelGGL(k_solve, dim3(nblk(m, 256)), dim3(256), 0, s, ws.pc, n, stride, ws.cnt,
                     ws.off, ws.partials, ws.Fl, F_part, part_stride, amps, umax);
  hipLaunchKernelGGL(k_mean, dim3(nblk(n * 64, 256)), dim3(256), 0, s, ws.pc, n, stride, ws.Fl, F_hat,
                     F_part, part_stride, amps, bin_counter);
}

void launch_sur_data(uint64_t seed, int64_t n, float* X, float* T, hipStream_t s) {
  hipLaunchKernelGGL(k_sur_data, dim3(nblk(n, 128)), dim3(128), 0, s, seed, n, X, T);
}

void launch_sur_knots(const Grid& g, int32_t stride, int64_t n, int64_t rows, const WorkSpace& ws,
                      float* X, hipStream_t s) {
  hipLaunchKernelGGL(k_sur_knots, dim3(nblk(rows, 256)), dim3(256), 0, s, g, ws.pc, ws.bounds,
                     stride, n, rows, X);
}

void launch_sur_check(const Grid& g, int32_t stride, int64_t n, const WorkSpace& ws,
                      const float* ynn, double* ek, double* mm, double thr,
                      unsigned long long* counters, hipStream_t s) {
  hipLaunchKernelGGL(k_sur_check, dim3(nblk(n * stride, 128)), dim3(128), 0, s, g, ws.pc,
                     ws.bounds, stride, n, ynn, ek, mm);
  hipLaunchKernelGGL(k_sur_decide, dim3(nblk(n, 128)), dim3(128), 0, s, ws.pc, n, stride, mm, thr,
                     counters);
}

int uprefix_block_sums(int64_t n) { return (int)((n + kScanBlock - 1) / kScanBlock); }

void launch_uprefix(const double* u, int64_t n, double* bsum, double* out, hipStream_t s) {
  const int32_t nb = uprefix_block_sums(n);
  hipLaunchKernelGGL(k_uscan_sums, dim3(nb), dim3(1024), 0, s, u, n, bsum);
  hipLaunchKernelGGL(k_uscan_top, dim3(1), dim3(1024), 0, s, bsum, nb);
  hipLaunchKernelGGL(k_uscan_apply, dim3(nb), dim3(1024), 0, s, u, n, bsum, out);
}

void launch_ufit(const double* u, int64_t nbins, int32_t ntiles, double* coef, double* resid,
                 hipStream_t s) {
  if (ntiles > 0)
    hipLaunchKernelGGL(k_ufit, dim3(ntiles), dim3(kUTile), 0, s, u, nbins, ntiles, coef, resid);
}

void launch_extrinsic(const double* amps, const double* params, int64_t n, double* out,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_extrinsic, dim3(nblk(n, 256)), dim3(256), 0, s, amps, params, n, out);
}

void launch_waveform(const Grid& g, const PartConst* pc, const double* amps,
                     double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_waveform, dim3(nblk(g.nbins, 256)), dim3(256), 0, s, g, pc, amps, out);
}

}  // namespace fstat

namespace fstat {
hipError_t occupancy_fp64(int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_eval_exact<false>, 256, 0);
}
hipError_t occupancy_mixed(int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_eval_exact<true>, 256, 0);
}
}  // namespace fstat
