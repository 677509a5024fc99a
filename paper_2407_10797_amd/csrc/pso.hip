// pso.hip -- particle swarm stage on the device (Sec. III.A of arXiv:2407.10797),
// many independent runs per launch (Sec. III.B: several runs per search box).
//
// One iteration = decode positions -> batched F_hat evaluation of every
// particle of every run (one persistent bin-loop launch) -> personal / ring-local
// / run best updates and the velocity-position step.  All state stays on the
// device; an iteration reads its index from a device counter, so it can be
// captured once as a hipGraph and replayed.
//
// Random numbers: Philox4x64-10 (Salmon et al., SC'11).  Key = (seed, run);
// counter = (t, particle, block, 0) with t = 0 for initialisation and t = k + 1
// for iteration k; three blocks give 12 uniforms u = (bits >> 11) 2^-53:
// u[0..5] and u[6..11] are (x0, v0 draw) at t = 0 and (r1, r2) afterwards.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/fstat.h"
#include "fstat_api_internal.h"
#include "philox.h"

namespace fstat {

struct PsoArgs {
  int32_t n_runs, n_part, iters, ring_k;
  double w_start, w_end, c1, c2, vmax;
  uint64_t seed;
};

__global__ void k_pso_init(PsoArgs a, double* __restrict__ x, double* __restrict__ v,
                           double* __restrict__ pbx, double* __restrict__ pbf,
                           double* __restrict__ gbf, int32_t* __restrict__ iter) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)a.n_runs * a.n_part) return;
  int r = (int)(g / a.n_part), i = (int)(g % a.n_part);
  double u[12];
  draw12(a.seed, (uint64_t)r, 0ull, (uint64_t)i, u);
  for (int j = 0; j < 6; ++j) {
    double xj = u[j];
    x[g * 6 + j] = xj;
    pbx[g * 6 + j] = xj;
    v[g * 6 + j] = u[6 + j] - xj;   // U[0 - x, 1 - x] in the normalised box
  }
  pbf[g] = -__builtin_inf();
  if (i == 0) gbf[r] = -__builtin_inf();
  if (g == 0) iter[0] = 0;
}

// normalised x -> physical parameters; particles outside [0,1]^6 are skipped
__global__ void k_pso_decode(PsoArgs a, const double* __restrict__ x,
                             const double* __restrict__ box, const int32_t* __restrict__ np_run,
                             double* __restrict__ params, int32_t* __restrict__ np,
                             uint8_t* __restrict__ skip) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)a.n_runs * a.n_part) return;
  int r = (int)(g / a.n_part);
  bool out = false;
  for (int j = 0; j < 6; ++j) {
    double xj = x[g * 6 + j];
    out = out || !(xj >= 0.0 && xj <= 1.0);
    double lo = box[r * 12 + 2 * j], hi = box[r * 12 + 2 * j + 1];
    params[g * 6 + j] = lo + xj * (hi - lo);
  }
  np[g] = np_run[r];
  skip[g] = out ? 1 : 0;
}

// one block per run, one thread per particle
__global__ void k_pso_update(PsoArgs a, const double* __restrict__ F, double* __restrict__ x,
                             double* __restrict__ v, double* __restrict__ pbx,
                             double* __restrict__ pbf, double* __restrict__ gbx,
                             double* __restrict__ gbf, double* __restrict__ trace,
                             const int32_t* __restrict__ iter) {
  extern __shared__ double sh[];
  double* spb = sh;                               // [n_part] personal bests
  int* sbest = (int*)(sh + a.n_part);             // [1] run best index
  const int r = blockIdx.x, i = threadIdx.x, Pn = a.n_part;
  const int k = iter[0];
  const int64_t g = (int64_t)r * Pn + i;
  if (i < Pn) {
    double f = F[g];
    if (f > pbf[g]) {   // strict improvement; -inf (outside the box) never wins
      pbf[g] = f;
      for (int j = 0; j < 6; ++j) pbx[g * 6 + j] = x[g * 6 + j];
    }
    spb[i] = pbf[g];
  }
  __syncthreads();
  if (i == 0) {
    int b = 0;
    for (int q = 1; q < Pn; ++q)
      if (spb[q] > spb[b]) b = q;   // lowest index wins ties
    sbest[0] = b;
    gbf[r] = spb[b];
    for (int j = 0; j < 6; ++j) gbx[r * 6 + j] = pbx[((int64_t)r * Pn + b) * 6 + j];
    if (trace) trace[(int64_t)k * a.n_runs + r] = spb[b];
  }
  __syncthreads();
  if (i >= Pn) return;
  // local best in the ring {i-K..i+K}; global best when the ring covers the swarm
  int lb;
  const int K = a.ring_k;
  if (K <= 0 || 2 * K + 1 >= Pn) {
    lb = sbest[0];
  } else {
    lb = -1;
    for (int d = -K; d <= K; ++d) {
      int q = ((i + d) % Pn + Pn) % Pn;
      if (lb < 0 || spb[q] > spb[lb] || (spb[q] == spb[lb] && q < lb)) lb = q;
    }
  }
  double w = (a.iters > 1) ? a.w_start + (a.w_end - a.w_start) * (double)k / (double)(a.iters - 1)
                           : a.w_start;
  double u[12];
  draw12(a.seed, (uint64_t)r, (uint64_t)k + 1ull, (uint64_t)i, u);
  const int64_t gl = (int64_t)r * Pn + lb;
  for (int j = 0; j < 6; ++j) {
    double xj = x[g * 6 + j];
    double vj = w * v[g * 6 + j] + a.c1 * u[j] * (pbx[g * 6 + j] - xj) +
                a.c2 * u[6 + j] * (pbx[gl * 6 + j] - xj);
    vj = fmin(fmax(vj, -a.vmax), a.vmax);
    v[g * 6 + j] = vj;
    x[g * 6 + j] = xj + vj;
  }
}

__global__ void k_pso_tick(int32_t* iter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) iter[0] += 1;
}

}  // namespace fstat

using namespace fstat;

struct PsoState {
  hipStream_t stream = nullptr;
};

void pso_release(fstat_plan_s* P) {
  if (P->pso) {
    if (P->pso->stream) (void)hipStreamDestroy(P->pso->stream);
    delete P->pso;
  }
  P->pso = nullptr;
}

namespace {

struct DevBufs {
  std::vector<void*> ptrs;
  ~DevBufs() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <typename T>
  int alloc(T** p, size_t n) {
    *p = nullptr;
    hipError_t e = hipMalloc((void**)p, (n ? n : 1) * sizeof(T));
    if (e != hipSuccess) return hip_check(e, "pso alloc");
    ptrs.push_back(*p);
    return FSTAT_OK;
  }
};

// $FSTAT_PROGRESS = N > 0: every N iterations wait for the stream and print
// one line to stderr (long stages report while they run).
// a progress line each time `done` (advanced by `step`) passes a multiple of
// $FSTAT_PROGRESS iterations
int report_progress(int done, int total, hipStream_t s, int step = 1) {
  static const long every = [] {
    const char* e = getenv("FSTAT_PROGRESS");
    return e ? strtol(e, nullptr, 10) : 0L;
  }();
  if (every <= 0 || done / every == (done - step) / every || done == total) return FSTAT_OK;
  int rc = hip_check(hipStreamSynchronize(s), "pso progress");
  if (!rc) {
    fprintf(stderr, "[pso] %d / %d iterations\n", done, total);
    fflush(stderr);
  }
  return rc;
}

}  // namespace

constexpr int kGraphIters = 16;   // PSO iterations per captured graph

extern "C" int pso_stage(fstat_plan_t P, const pso_stage_desc* d, pso_result* res,
                         void* hip_stream) {
  if (!P || !d || !res) return set_error(FSTAT_EINVAL, "null plan, descriptor or result");
  const int R = d->n_runs, Pn = d->n_part, I = d->iters;
  if (R < 1 || Pn < 1 || Pn > 1024 || I < 0) return set_error(FSTAT_EINVAL, "bad n_runs/n_part/iters");
  if (!d->box || !d->np) return set_error(FSTAT_EINVAL, "null box or np");
  if (!res->best_x || !res->best_F) return set_error(FSTAT_EINVAL, "null best_x or best_F");
  if (!(d->vmax > 0.0) || !std::isfinite(d->w_start) || !std::isfinite(d->w_end) ||
      !std::isfinite(d->c1) || !std::isfinite(d->c2))
    return set_error(FSTAT_EINVAL, "bad PSO coefficients");
  const bool mixed = (d->flags & FSTAT_EVAL_MIXED) != 0;
  const bool sur = (d->flags & FSTAT_EVAL_SURROGATE) != 0;
  const bool exact = (d->flags & FSTAT_EVAL_EXACT) != 0;
  if (sur && !P->sur_trained) return set_error(FSTAT_EINVAL, "surrogate requested but not trained");
  if (mixed && !(P->prec & FSTAT_MIXED)) return set_error(FSTAT_EINVAL, "plan has no mixed data");
  if (!mixed && !(P->prec & FSTAT_FP64)) return set_error(FSTAT_EINVAL, "plan has no FP64 data");
  int32_t stride = 1;
  for (int r = 0; r < R; ++r) {
    if (d->np[r] < 1 || d->np[r] > 65536) return set_error(FSTAT_EINVAL, "np[%d] out of range", r);
    stride = d->np[r] > stride ? d->np[r] : stride;
    for (int j = 0; j < 6; ++j) {
      double lo = d->box[r * 12 + 2 * j], hi = d->box[r * 12 + 2 * j + 1];
      if (!std::isfinite(lo) || !std::isfinite(hi) || hi < lo)
        return set_error(FSTAT_EINVAL, "box[%d][%d] is not a finite interval", r, j);
    }
  }
  int rc;
  if (!P->pso) P->pso = new PsoState();
  if (!P->pso->stream &&
      (rc = hip_check(hipStreamCreateWithFlags(&P->pso->stream, hipStreamNonBlocking), "stream")))
    return rc;
  hipStream_t s = P->pso->stream;
  // the caller's stream may still be writing the plan's data: order after it
  if ((rc = hip_check(hipStreamSynchronize((hipStream_t)hip_stream), "caller stream"))) return rc;

  const int64_t n = (int64_t)R * Pn;
  DevBufs B;
  double *x, *v, *pbx, *pbf, *gbx, *gbf, *box, *params, *F, *trace = nullptr;
  int32_t *np_run, *np, *iter;
  uint8_t* skip;
  if ((rc = B.alloc(&x, n * 6)) || (rc = B.alloc(&v, n * 6)) || (rc = B.alloc(&pbx, n * 6)) ||
      (rc = B.alloc(&pbf, n)) || (rc = B.alloc(&gbx, (size_t)R * 6)) || (rc = B.alloc(&gbf, R)) ||
      (rc = B.alloc(&box, (size_t)R * 12)) || (rc = B.alloc(&params, n * 6)) ||
      (rc = B.alloc(&F, n)) || (rc = B.alloc(&np_run, R)) || (rc = B.alloc(&np, n)) ||
      (rc = B.alloc(&iter, 1)) || (rc = B.alloc(&skip, n)))
    return rc;
  if (res->trace && I > 0 && (rc = B.alloc(&trace, (size_t)I * R))) return rc;
  if ((rc = hip_check(hipMemcpyAsync(box, d->box, sizeof(double) * R * 12, hipMemcpyHostToDevice, s), "copy box")) ||
      (rc = hip_check(hipMemcpyAsync(np_run, d->np, sizeof(int32_t) * R, hipMemcpyHostToDevice, s), "copy np")))
    return rc;
  if ((rc = ensure_workspace(P, n, stride, chunk_for(P, mixed)))) return rc;
  if (sur && (rc = sur_ensure(P, n, stride))) return rc;   // no allocation inside the capture
  (void)eval_blocks(P, mixed);   // occupancy query outside any capture
  PsoArgs a{R, Pn, I, d->ring_k, d->w_start, d->w_end, d->c1, d->c2, d->vmax, d->seed};
  const unsigned nb = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_pso_init, dim3(nb), dim3(256), 0, s, a, x, v, pbx, pbf, gbf, iter);
  const int tpb = ((Pn + 63) / 64) * 64;
  const size_t shmem = sizeof(double) * Pn + sizeof(int) * 2;
  auto iteration = [&]() -> int {
    hipLaunchKernelGGL(k_pso_decode, dim3(nb), dim3(256), 0, s, a, x, box, np_run, params, np, skip);
    int r2 = eval_device(P, params, n, np, 0, stride, F, nullptr, 0, mixed, s, skip, false, sur,
                         exact);
    if (r2) return r2;
    hipLaunchKernelGGL(k_pso_update, dim3(R), dim3(tpb), shmem, s, a, F, x, v, pbx, pbf, gbx, gbf,
                       trace, iter);
    hipLaunchKernelGGL(k_pso_tick, dim3(1), dim3(64), 0, s, iter);
    return hip_check(hipGetLastError(), "pso launch");
  };
  if (d->use_graph && I > 0) {
    // kGraphIters iterations per graph (the iteration counter lives on the
    // device, so consecutive iterations are identical launches): one graph
    // launch per kGraphIters iterations, and a second graph for the remainder
    auto capture = [&](int iters, hipGraphExec_t* exec) -> int {
      hipGraph_t graph = nullptr;
      int r2 = hip_check(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture");
      if (r2) return r2;
      int rci = 0;
      for (int k = 0; k < iters && !rci; ++k) rci = iteration();
      hipError_t ec = hipStreamEndCapture(s, &graph);
      if (!rci) rci = hip_check(ec, "end capture");
      if (!rci) rci = hip_check(hipGraphInstantiate(exec, graph, nullptr, nullptr, 0), "instantiate");
      if (graph) (void)hipGraphDestroy(graph);
      return rci;
    };
    const int G = I < kGraphIters ? I : kGraphIters;
    const int full = I / G, rest = I - full * G;
    hipGraphExec_t exec = nullptr, exec_rest = nullptr;
    rc = capture(G, &exec);
    if (!rc && rest) rc = capture(rest, &exec_rest);
    for (int k = 0; k < full && !rc; ++k) {
      rc = hip_check(hipGraphLaunch(exec, s), "graph launch");
      if (!rc) rc = report_progress((k + 1) * G, I, s, G);
    }
    if (!rc && rest) {
      rc = hip_check(hipGraphLaunch(exec_rest, s), "graph launch");
      if (!rc) rc = report_progress(I, I, s, rest);
    }
    if (!rc) rc = hip_check(hipStreamSynchronize(s), "pso graph");
    if (exec) (void)hipGraphExecDestroy(exec);
    if (exec_rest) (void)hipGraphExecDestroy(exec_rest);
    if (rc) return rc;
  } else {
    for (int k = 0; k < I; ++k)
      if ((rc = iteration()) || (rc = report_progress(k + 1, I, s))) return rc;
  }
  // results: run bests in physical units
  std::vector<double> hx((size_t)R * 6), hb((size_t)R * 12);
  memcpy(hb.data(), d->box, sizeof(double) * R * 12);
  if ((rc = hip_check(hipMemcpyAsync(hx.data(), gbx, sizeof(double) * R * 6, hipMemcpyDeviceToHost, s), "copy gbx")) ||
      (rc = hip_check(hipMemcpyAsync(res->best_F, gbf, sizeof(double) * R, hipMemcpyDeviceToHost, s), "copy gbf")))
    return rc;
  if (res->trace && trace &&
      (rc = hip_check(hipMemcpyAsync(res->trace, trace, sizeof(double) * I * R, hipMemcpyDeviceToHost, s), "copy trace")))
    return rc;
  if (res->final_x &&
      (rc = hip_check(hipMemcpyAsync(res->final_x, x, sizeof(double) * n * 6, hipMemcpyDeviceToHost, s), "copy x")))
    return rc;
  if ((rc = hip_check(hipStreamSynchronize(s), "pso results"))) return rc;
  for (int r = 0; r < R; ++r)
    for (int j = 0; j < 6; ++j) {
      double lo = hb[r * 12 + 2 * j], hi = hb[r * 12 + 2 * j + 1];
      res->best_x[r * 6 + j] = lo + hx[r * 6 + j] * (hi - lo);
    }
  return FSTAT_OK;
}
