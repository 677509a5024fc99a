// fstat_kernels.h -- host-side launchers of the libfstat kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fstat_internal.h"

namespace fstat {

// frequency grid f_j = (k_lo + j) df, j < nbins; support window [0, T_obs]
// TDI channels: 0 X, 1 Y, 2 Z (first-generation Michelson at spacecraft 1, 2,
// 3), 3 A = (Z - X)/sqrt 2, 4 E = (X - 2Y + Z)/sqrt 6, 5 T = (X + Y + Z)/sqrt 3.
constexpr int kMaxChannels = 6;
struct Channels {
  int32_t n = 1;                                  // channels summed by the statistic
  int32_t code[kMaxChannels] = {0, 0, 0, 0, 0, 0};   // channel codes in data order
};

struct Grid {
  double df;
  double T_obs;
  int64_t k_lo;
  int64_t nbins;       // bins per channel
  Channels chan{};     // per-channel arrays are stacked channel-major
  OrbitTable orb{};    // spacecraft orbit (analytic unless a table is set)
};

// per-bin prepared data of one precision (structure of arrays)
template <typename T>
struct BinData {
  T* wr;   // Re w_j
  T* wi;   // Im w_j
  T* u;    // u_j
  T* s0;   // sin(pi f_j L)
  T* c0;   // cos(pi f_j L)
};

struct WorkSpace {
  PartConst* pc;      // [n]
  int32_t* bounds;    // [n][stride + 1]
  int32_t* cnt;       // [n][stride]
  int32_t* off;       // [n][stride]
  int32_t* total;     // [1]
  int32_t* bsum;      // [ceil(n stride / 4096)] block sums of the count scan
  int2* items;        // [capacity]
  double* partials;   // [capacity][8]
  double* Fl;         // [n][stride]
  int32_t* direct;    // [capacity] items the interpolating kernel hands to the exact kernel
  int32_t* ndirect;   // [1]
  int32_t* tcnt;      // [tiles] items per bin tile
  int32_t* tcur;      // [tiles] scatter cursors
  int32_t* toff;      // [tiles + 1] first item of each tile in tile_items
  int32_t* uoff;      // [tiles + 1] first scheduling unit of each tile
  int32_t* tile_items;  // [capacity] item indices grouped by bin tile
  int32_t* tile_ctr;  // [1] next unit to take (dynamic schedule)
  uint8_t* xflag;     // [capacity] 1: item evaluated by the exact kernel
  double* rec;        // [capacity][53] per-item interpolation records
  float2* xerr;       // [capacity] interpolation error of each interpolated item:
                      // x template (norm-weighted), y M-term quadrature (absolute)
  int32_t* refine;    // [capacity] interpolated items of ill-conditioned partitions
  int32_t* nrefine;   // [1]
};

void launch_prep(const Grid& g, const double* data, const double* psd, BinData<double> b,
                 hipStream_t s);
void launch_max(const double* u, int64_t n, double* out, hipStream_t s);
void launch_scale(const Grid& g, const double* umax, BinData<double> b, BinData<float> b32,
                  hipStream_t s);
void launch_setup(const Grid& g, const double* params, int64_t n,
                  const int32_t* np, int32_t np_uniform, int32_t stride, int32_t chunk,
                  const uint8_t* skip, const WorkSpace& ws, hipStream_t s);
void launch_worklist(int64_t m, const WorkSpace& ws, hipStream_t s);
int interp_tables_init();
constexpr int kMaxTileFp64 = 2560;   // largest tile (bins) of the LDS-staged loops
constexpr int kMaxTileMixed = 4608;   // FP32 w: 36 KB + 2 KB per block, four blocks per CU
int interp_max_tile(bool mixed);   // largest tile (bins) the LDS-staged loop accepts
constexpr int kInterpRec = 59;     // doubles per interpolation record

// Smooth model of the template-independent weight u = 4 df f^{-7/3} |C|^2 / S
// (scaled): a degree-9 Chebyshev least-squares fit per u-tile of kUTile bins,
// with its largest relative residual on the tile's bins.  Items whose bins
// lie in tiles fitted to within kUFitTol get their M-terms (P, Q, R) by
// quadrature of the interpolated u |T|^2 products instead of a per-bin sum.
constexpr int kUTile = 256;
constexpr int kUCoef = 10;
constexpr double kUFitTol = 1e-13;
constexpr int kSsumMax = 8192;     // largest item length of the quadrature table
struct UModel {
  const double* coef = nullptr;        // [ntiles][kUCoef] Chebyshev coefficients
  const int32_t* bad_prefix = nullptr; // [ntiles + 1] count of unfit tiles before each
  const double* resid = nullptr;       // [ntiles] largest relative residual of each fit
  int32_t ntiles = 0;
  const double* ssum = nullptr;        // [5][kSsumMax + 1]: sum_m T_2i(s_m), s_m = 2m/(nb-1) - 1
  const double* upre = nullptr;        // [channels][nbins + 1] prefix sums of u
};
const double* cheb_sums_table();       // the current device's quadrature table (after init)
void launch_ufit(const double* u, int64_t nbins, int32_t ntiles, double* coef, double* resid,
                 hipStream_t s);
// prefix sums out[0..n] of u[0..n) (bsum: uprefix_block_sums(n) doubles of scratch)
int uprefix_block_sums(int64_t n);
void launch_uprefix(const double* u, int64_t n, double* bsum, double* out, hipStream_t s);
void launch_eval(bool mixed, bool interp, double refine_budget, const Grid& g,
                 int64_t n_particles, int32_t stride, int32_t chunk,
                 const WorkSpace& ws, BinData<double> b, BinData<float> b32, const double* ek,
                 int blocks, hipStream_t s, hipEvent_t* ev_main = nullptr,
                 const UModel& um = UModel{});
void launch_sur_data(uint64_t seed, int64_t n, float* X, float* T, hipStream_t s);
void launch_sur_knots(const Grid& g, int32_t stride, int64_t n, int64_t rows, const WorkSpace& ws,
                      float* X, hipStream_t s);
void launch_sur_check(const Grid& g, int32_t stride, int64_t n, const WorkSpace& ws,
                      const float* ynn, double* ek, double* mm, double thr,
                      unsigned long long* counters, hipStream_t s);
// bins of the last evaluation by kind of interpolating-loop work, then the
// lane runs of those items by kind (out[kBinMix] accumulated)
constexpr int kBinMix = 14;
void launch_bin_mix(bool mixed, int32_t stride, int32_t chunk, int32_t nch, const WorkSpace& ws,
                    unsigned long long* out, hipStream_t s);
void launch_solve_mean(int64_t n, int32_t stride, const WorkSpace& ws, double* F_hat,
                       double* F_part, double* amps, int64_t part_stride, const double* umax,
                       unsigned long long* bin_counter, hipStream_t s);
void launch_extrinsic(const double* amps, const double* params, int64_t n, double* out,
                      hipStream_t s);
void launch_waveform(const Grid& g, const PartConst* pc, const double* amps,
                     double* out, hipStream_t s);

}  // namespace fstat
