// fstat_api_internal.h -- plan object and helpers shared by the host-side
// translation units of libfstat.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>
#include <array>
#include <vector>

#include "fstat_kernels.h"

struct PsoState;  // defined in pso.hip
namespace fstat {
struct Mlp;       // defined in mlp.h
}

struct fstat_plan_s {
  int device = 0;
  int num_cu = 0;
  int prec = 0;
  int chunk = 2048;                 // bins per work item (both precisions unless tuned)
  int chunk_mixed = 0;              // tuned value for the mixed path (0: use chunk)
  double refine_budget = 5e-10;    // see fstat_opts.refine_budget
  int grid_mult_fp64 = 1, grid_mult_mixed = 1;   // persistent-grid multiplier
  bool prefer_exact_fp64 = false, prefer_exact_mixed = false;   // autotuned bin-loop choice
  int blocks_fp64 = 0, blocks_mixed = 0;
  fstat::Grid grid{};
  fstat::BinData<double> b64{};
  fstat::BinData<float> b32{};
  fstat::WorkSpace ws{};
  double* umax = nullptr;           // max of u before scaling (the scale of the amplitudes)
  double* ucoef = nullptr;          // smooth model of u per u-tile (M-term quadrature)
  int32_t* ubad = nullptr;          // prefix count of u-tiles the model does not fit
  double* ures = nullptr;           // relative residual of the model per u-tile
  double* upre = nullptr;           // [channels][nbins + 1] prefix sums of u
  double* orb_coef = nullptr;       // numerical orbit (fstat_plan_set_orbit)
  int32_t n_utiles = 0;
  int32_t n_ufit = 0;               // u-tiles fitted to within tolerance
  struct {
    size_t pc = 0, bounds = 0, cnt = 0, off = 0, total = 0, items = 0, partials = 0, Fl = 0;
    size_t direct = 0, ndirect = 0, tcnt = 0, tcur = 0, toff = 0, uoff = 0, tile_items = 0,
           tile_ctr = 0;
    size_t xflag = 0, refine = 0, nrefine = 0, rec = 0, xerr = 0, bsum = 0;
    size_t params = 0, np = 0, F_hat = 0, F_part = 0, amps = 0;
  } cap;
  struct {
    double* params = nullptr;
    int32_t* np = nullptr;
    double* F_hat = nullptr;
    double* F_part = nullptr;
    double* amps = nullptr;
  } io;
  struct {                          // shape of the last fstat_eval (fstat_interp_stats)
    int64_t n = 0;
    int32_t stride = 0, chunk = 0;
    bool mixed = false, exact = false;
  } last;
  PsoState* pso = nullptr;
  // profiling (FSTAT_PROFILE)
  bool profile = false;
  std::vector<std::array<hipEvent_t, 4>> events;   // stage start, main start, main end, stage end
  unsigned long long* bin_counter = nullptr;
  // learned surrogate (surrogate.hip)
  fstat::Mlp* sur = nullptr;
  bool sur_trained = false;
  float* sur_X = nullptr;
  double* sur_ek = nullptr;
  double* sur_mm = nullptr;
  unsigned long long* sur_counters = nullptr;
  size_t cap_sur_X = 0, cap_sur_ek = 0, cap_sur_mm = 0, cap_sur_counters = 0;
};

namespace fstat {
inline int chunk_for(const fstat_plan_s* P, bool mixed) {
  return (mixed && P->chunk_mixed > 0) ? P->chunk_mixed : P->chunk;
}
int set_error(int code, const char* fmt, ...);
int hip_check(hipError_t e, const char* what);
int ensure_workspace(fstat_plan_s* P, int64_t n, int32_t stride, int chunk = 0);
int eval_device(fstat_plan_s* P, const double* params, int64_t n, const int32_t* np,
                int32_t np_uniform, int32_t stride, double* F_hat, double* F_part,
                int64_t part_stride, bool mixed, hipStream_t s, const uint8_t* skip = nullptr,
                bool allow_profile = true, bool surrogate = false, bool exact = false,
                double* amps = nullptr);
int sur_ensure(fstat_plan_s* P, int64_t n, int32_t stride);
int sur_prepare(fstat_plan_s* P, int64_t n, int32_t stride, hipStream_t s);
void sur_release(fstat_plan_s* P);
int eval_blocks(fstat_plan_s* P, bool mixed);
hipError_t occupancy_fp64(int* blocks_per_cu);
hipError_t occupancy_mixed(int* blocks_per_cu);
}  // namespace fstat

void pso_release(fstat_plan_s* P);
