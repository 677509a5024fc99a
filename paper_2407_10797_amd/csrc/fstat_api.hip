// fstat_api.hip -- C ABI of libfstat (see include/fstat.h): plans, batched
// evaluation and template generation.
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/fstat.h"
#include "fstat_api_internal.h"

using namespace fstat;

static_assert(sizeof(fstat_data_desc) == 64, "fstat_data_desc layout");

// ---- scratch memory of the allocation-free entry point ----------------------
// One fixed array per device, part of the library's device code: each GPU the
// library runs on holds its own copy, at its own address, until the process
// ends.  In host code the name `scratch` is a host-side stand-in, never a
// device address: fstat_plan_create takes the device address once per device
// (with that device current) and fstat_eval_noalloc passes only that address
// to the kernels.
static constexpr size_t kScratchBytes = FSTAT_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static char* g_scratch_dev[64] = {};   // per device: device address of `scratch`

namespace fstat {

static thread_local std::string g_err;

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return FSTAT_OK;
  return set_error(e == hipErrorOutOfMemory ? FSTAT_ENOMEM : FSTAT_EDEVICE, "%s: %s", what,
                   hipGetErrorString(e));
}

template <typename T>
static int dev_alloc(T** p, size_t count, const char* what) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hip_check(hipMalloc((void**)p, count * sizeof(T)), what);
}

template <typename T>
static void dev_free(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

// grow-only device buffer
template <typename T>
static int ensure(T** p, size_t* cap, size_t need, const char* what) {
  if (need <= *cap && *p) return FSTAT_OK;
  dev_free(*p);
  *cap = 0;
  int rc = dev_alloc(p, need, what);
  if (rc == FSTAT_OK) *cap = need;
  return rc;
}

int ensure_workspace(fstat_plan_s* P, int64_t n, int32_t stride, int chunk) {
  int rc;
  if (chunk <= 0) chunk = P->chunk;
  size_t m = (size_t)n * (size_t)stride;
  const size_t nch = (size_t)P->grid.chan.n;
  size_t cap_items = (size_t)n * ((size_t)((P->grid.nbins + chunk - 1) / chunk) + stride) * nch;
  if (cap_items > (size_t)INT32_MAX)
    return set_error(FSTAT_EINVAL, "work list too large (%zu items)", cap_items);
  if ((rc = ensure(&P->ws.pc, &P->cap.pc, (size_t)n, "alloc pc"))) return rc;
  if ((rc = ensure(&P->ws.bounds, &P->cap.bounds, (size_t)n * (stride + 1), "alloc bounds"))) return rc;
  if ((rc = ensure(&P->ws.cnt, &P->cap.cnt, m, "alloc cnt"))) return rc;
  if ((rc = ensure(&P->ws.off, &P->cap.off, m, "alloc off"))) return rc;
  if ((rc = ensure(&P->ws.Fl, &P->cap.Fl, m, "alloc Fl"))) return rc;
  if ((rc = ensure(&P->ws.total, &P->cap.total, 1, "alloc total"))) return rc;
  if (m > (size_t)4096 * 4096) return set_error(FSTAT_EINVAL, "n * stride above 16.7M partitions");
  if ((rc = ensure(&P->ws.bsum, &P->cap.bsum, (m + 4095) / 4096, "alloc scan sums"))) return rc;
  if ((rc = ensure(&P->ws.items, &P->cap.items, cap_items, "alloc items"))) return rc;
  if ((rc = ensure(&P->ws.partials, &P->cap.partials, cap_items * 8, "alloc partials"))) return rc;
  if ((rc = ensure(&P->ws.direct, &P->cap.direct, cap_items, "alloc direct"))) return rc;
  if ((rc = ensure(&P->ws.ndirect, &P->cap.ndirect, 1, "alloc ndirect"))) return rc;
  const size_t ntiles = (size_t)((P->grid.nbins + chunk - 1) / chunk) * nch;   // all channels
  if ((rc = ensure(&P->ws.tcnt, &P->cap.tcnt, ntiles, "alloc tcnt"))) return rc;
  if ((rc = ensure(&P->ws.tcur, &P->cap.tcur, ntiles, "alloc tcur"))) return rc;
  if ((rc = ensure(&P->ws.toff, &P->cap.toff, ntiles + 1, "alloc toff"))) return rc;
  if ((rc = ensure(&P->ws.uoff, &P->cap.uoff, ntiles + 1, "alloc uoff"))) return rc;
  if ((rc = ensure(&P->ws.tile_items, &P->cap.tile_items, cap_items, "alloc tile items"))) return rc;
  if ((rc = ensure(&P->ws.tile_ctr, &P->cap.tile_ctr, 1, "alloc tile counter"))) return rc;
  if ((rc = ensure(&P->ws.xflag, &P->cap.xflag, cap_items, "alloc item flags"))) return rc;
  if ((rc = ensure(&P->ws.rec, &P->cap.rec, cap_items * kInterpRec, "alloc interpolation records")))
    return rc;
  if ((rc = ensure(&P->ws.xerr, &P->cap.xerr, cap_items, "alloc item errors"))) return rc;
  if ((rc = ensure(&P->ws.refine, &P->cap.refine, cap_items, "alloc refine list"))) return rc;
  if ((rc = ensure(&P->ws.nrefine, &P->cap.nrefine, 1, "alloc refine count"))) return rc;
  return FSTAT_OK;
}

// Workspace for (n, stride, chunk) carved out of one buffer in 256-byte
// aligned pieces, in the order and sizes ensure_workspace allocates them.
// With base == nullptr only the byte count is computed.
static size_t carve_workspace(const fstat_plan_s* P, int64_t n, int32_t stride, int chunk,
                              char* base, WorkSpace* ws) {
  const size_t m = (size_t)n * (size_t)stride;
  const size_t nch = (size_t)P->grid.chan.n;
  const size_t ntiles = (size_t)((P->grid.nbins + chunk - 1) / chunk) * nch;
  const size_t cap_items = (size_t)n * ((size_t)((P->grid.nbins + chunk - 1) / chunk) + stride) * nch;
  size_t at = 0;
  WorkSpace w{};
  auto take = [&](auto** p, size_t count) {
    at = (at + 255) & ~(size_t)255;
    *p = base ? reinterpret_cast<std::remove_reference_t<decltype(*p)>>(base + at) : nullptr;
    at += (count ? count : 1) * sizeof(**p);
  };
  take(&w.pc, (size_t)n);
  take(&w.bounds, (size_t)n * (stride + 1));
  take(&w.cnt, m);
  take(&w.off, m);
  take(&w.Fl, m);
  take(&w.total, 1);
  take(&w.bsum, (m + 4095) / 4096);
  take(&w.items, cap_items);
  take(&w.partials, cap_items * 8);
  take(&w.direct, cap_items);
  take(&w.ndirect, 1);
  take(&w.tcnt, ntiles);
  take(&w.tcur, ntiles);
  take(&w.toff, ntiles + 1);
  take(&w.uoff, ntiles + 1);
  take(&w.tile_items, cap_items);
  take(&w.tile_ctr, 1);
  take(&w.xflag, cap_items);
  take(&w.rec, cap_items * kInterpRec);
  take(&w.xerr, cap_items);
  take(&w.refine, cap_items);
  take(&w.nrefine, 1);
  if (ws) *ws = w;
  return at;
}

// Device address of this device's scratch array, taken once per device.
static int scratch_init(int dev) {
  if (dev < 0 || dev >= 64) return set_error(FSTAT_EDEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[dev]) return FSTAT_OK;
  void* p = nullptr;
  int rc = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch address");
  if (rc) return rc;
  if (!p) return set_error(FSTAT_EDEVICE, "scratch address is null");
  g_scratch_dev[dev] = static_cast<char*>(p);
  return FSTAT_OK;
}

int eval_blocks(fstat_plan_s* P, bool mixed) {
  int& cached = mixed ? P->blocks_mixed : P->blocks_fp64;
  if (cached <= 0) {
    int per_cu = 0;
    hipError_t e = mixed ? occupancy_mixed(&per_cu) : occupancy_fp64(&per_cu);
    if (e != hipSuccess || per_cu < 1) per_cu = 2;
    cached = P->num_cu * per_cu;
  }
  return cached * (mixed ? P->grid_mult_mixed : P->grid_mult_fp64);
}


static int check_chunk(const fstat_plan_s* P, bool mixed, bool exact) {
  const int chunk = chunk_for(P, mixed);
  if (!exact && chunk > interp_max_tile(mixed))
    return set_error(FSTAT_EINVAL, "work-item size %d exceeds the LDS tile limit %d (use a smaller "
                     "chunk or FSTAT_EVAL_EXACT)", chunk, interp_max_tile(mixed));
  return FSTAT_OK;
}

// Enqueue the kernels of one evaluation on workspace `ws` (device pointers).
static int eval_enqueue(fstat_plan_s* P, const WorkSpace& ws, const double* params, int64_t n,
                        const int32_t* np, int32_t np_uniform, int32_t stride, double* F_hat,
                        double* F_part, int64_t part_stride, bool mixed, hipStream_t s,
                        const uint8_t* skip, bool allow_profile, bool surrogate, bool exact,
                        double* amps) {
  const int chunk = chunk_for(P, mixed);
  int rc;
  launch_setup(P->grid, params, n, np, np_uniform, stride, chunk, skip, ws, s);
  if (surrogate && (rc = sur_prepare(P, n, stride, s))) return rc;
  launch_worklist(n * (int64_t)stride, ws, s);
  // profiling: the whole bin-loop stage (e[0], e[3]) and its main kernel (e[1], e[2])
  std::array<hipEvent_t, 4> ev = {nullptr, nullptr, nullptr, nullptr};
  const bool prof = P->profile && allow_profile;
  if (prof) {
    for (auto& e : ev)
      if ((rc = hip_check(hipEventCreate(&e), "event"))) return rc;
    (void)hipEventRecord(ev[0], s);
  }
  UModel um;
  um.coef = P->ucoef;
  um.bad_prefix = P->ubad;
  um.resid = P->ures;
  um.ntiles = P->n_utiles;
  um.ssum = cheb_sums_table();
  if (!um.ssum) um.coef = nullptr;
  um.upre = P->upre;
  launch_eval(mixed, !exact, P->refine_budget, P->grid, n, stride, chunk, ws, P->b64, P->b32,
              surrogate ? P->sur_ek : nullptr, eval_blocks(P, mixed), s,
              prof ? &ev[1] : nullptr, um);
  if (prof) {
    (void)hipEventRecord(ev[3], s);
    P->events.push_back(ev);
  }
  launch_solve_mean(n, stride, ws, F_hat, F_part, amps, part_stride, P->umax,
                    prof ? P->bin_counter : nullptr, s);
  return hip_check(hipGetLastError(), "kernel launch");
}

// Enqueue one evaluation with device pointers on the plan's own (grow-only)
// workspace.
int eval_device(fstat_plan_s* P, const double* params, int64_t n, const int32_t* np,
                int32_t np_uniform, int32_t stride, double* F_hat, double* F_part,
                int64_t part_stride, bool mixed, hipStream_t s, const uint8_t* skip,
                bool allow_profile, bool surrogate, bool exact, double* amps) {
  // the autotuner may have found the exact loop faster for this plan's batches
  exact = exact || (mixed ? P->prefer_exact_mixed : P->prefer_exact_fp64);
  int rc = check_chunk(P, mixed, exact);
  if (rc) return rc;
  if ((rc = ensure_workspace(P, n, stride, chunk_for(P, mixed)))) return rc;
  if (surrogate && (rc = sur_ensure(P, n, stride))) return rc;
  P->last.n = n;
  P->last.stride = stride;
  P->last.chunk = chunk_for(P, mixed);
  P->last.mixed = mixed;
  P->last.exact = exact;
  return eval_enqueue(P, P->ws, params, n, np, np_uniform, stride, F_hat, F_part, part_stride,
                      mixed, s, skip, allow_profile, surrogate, exact, amps);
}

// ---- autotuner --------------------------------------------------------------
static std::string tune_key(const fstat_plan_s* P, int32_t np, bool mixed) {
  hipDeviceProp_t prop;
  std::string arch = "gpu";
  if (hipGetDeviceProperties(&prop, P->device) == hipSuccess) arch = prop.gcnArchName;
  int npc = 1;
  while (npc < np) npc <<= 1;
  int nbc = 0;
  while ((1ll << nbc) < P->grid.nbins) ++nbc;
  char buf[256], chs[16] = "";
  if (P->grid.chan.n > 1) snprintf(chs, sizeof(chs), " ch%d", P->grid.chan.n);
  snprintf(buf, sizeof(buf), "%s nbins2^%d np%d%s %s", arch.c_str(), nbc, npc, chs,
           mixed ? "mixed" : "fp64");
  for (char* c = buf; *c; ++c)
    if (*c == ':') *c = '_';
  return buf;
}

// Choices made in this process, keyed like the cache file.
static std::mutex g_tune_mu;
static std::map<std::string, std::array<int, 3>> g_tune_mem;

// (chunk, grid multiplier, 1 when the exact loop won) of a key
static bool tune_cache_get(const std::string& key, int* chunk, int* mult, int* ex) {
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_mem.find(key);
    if (it != g_tune_mem.end()) {
      *chunk = it->second[0]; *mult = it->second[1]; *ex = it->second[2];
      return true;
    }
  }
  const char* path = getenv("FSTAT_TUNE_CACHE");
  if (!path || !*path) return false;
  FILE* fp = fopen(path, "r");
  if (!fp) return false;
  char line[512];
  bool found = false;
  while (fgets(line, sizeof(line), fp)) {
    char k[400];
    int c, m, e = 0;
    const int got = sscanf(line, "%399[^|]|%d %d %d", k, &c, &m, &e);
    if (got >= 3 && key == k) {
      *chunk = c; *mult = m; *ex = got == 4 ? e : 0; found = true;   // last entry wins
    }
  }
  fclose(fp);
  return found;
}

static void tune_cache_put(const std::string& key, int chunk, int mult, int ex) {
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_mem[key] = {chunk, mult, ex};
  }
  const char* path = getenv("FSTAT_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* fp = fopen(path, "a");
  if (!fp) return;
  fprintf(fp, "%s|%d %d %d\n", key.c_str(), chunk, mult, ex);
  fclose(fp);
}

}  // namespace fstat

extern "C" {

int fstat_autotune(fstat_plan_t P, const double* params, int64_t n, int32_t np_uniform,
                   const int32_t* np, int32_t part_stride, uint32_t flags, int32_t* best_chunk,
                   int32_t* best_mult, double* best_ms, void* hip_stream) {
  g_err.clear();
  if (!P || !params || n < 1) return set_error(FSTAT_EINVAL, "fstat_autotune: bad arguments");
  if (np ? (part_stride < 1 || part_stride > 65536) : (np_uniform < 1 || np_uniform > 65536))
    return set_error(FSTAT_EINVAL, "fstat_autotune: np_uniform or part_stride out of range");
  if (!(flags & FSTAT_DEVICE_PTRS)) return set_error(FSTAT_EINVAL, "fstat_autotune needs device pointers");
  const bool mixed = (flags & FSTAT_EVAL_MIXED) != 0;
  const bool exact = (flags & FSTAT_EVAL_EXACT) != 0;
  const bool mode = (flags & FSTAT_AUTOTUNE_MODE) != 0 && !exact;
  if (mixed ? !(P->prec & FSTAT_MIXED) : !(P->prec & FSTAT_FP64))
    return set_error(FSTAT_EINVAL, "precision not built into the plan");
  hipStream_t s = (hipStream_t)hip_stream;
  const int32_t stride = np ? part_stride : np_uniform;
  const std::string key = tune_key(P, stride, mixed) + (np ? " npmix" : "") +
                          (exact ? " exact" : (mode ? " mode" : ""));
  bool& prefer = mixed ? P->prefer_exact_mixed : P->prefer_exact_fp64;
  int c = 0, m = 0, e = 0;
  double ms_best = -1.0;
  if (!(flags & FSTAT_AUTOTUNE_FORCE) && tune_cache_get(key, &c, &m, &e) && c >= 64 && m >= 1) {
    // cached
  } else {
    static const int chunks[] = {256, 512, 1024, 2048, 2560, 4096, 4608, 8192};
    static const int mults[] = {1, 2, 4};
    double* F = nullptr;
    int rc = hip_check(hipMalloc(&F, sizeof(double) * n), "alloc tune out");
    hipEvent_t e0, e1;
    if (!rc) rc = hip_check(hipEventCreate(&e0), "event");
    if (!rc) rc = hip_check(hipEventCreate(&e1), "event");
    const int save_c = P->chunk, save_cm = P->chunk_mixed;
    const int save_m = mixed ? P->grid_mult_mixed : P->grid_mult_fp64;
    const bool save_p = prefer;
    prefer = false;     // each candidate below runs the loop it names
    // interpolating loop (unless exact is requested), then the exact loop
    // (when requested, or when the mode is tuned as well)
    for (int ex = exact ? 1 : 0; ex <= ((exact || mode) ? 1 : 0) && !rc; ++ex)
      for (int ci = 0; ci < (int)(sizeof(chunks) / sizeof(chunks[0])) && !rc; ++ci)
        for (int mi = 0; mi < 3 && !rc; ++mi) {
          if (!ex && chunks[ci] > interp_max_tile(mixed)) continue;
          if (mixed) { P->chunk_mixed = chunks[ci]; P->grid_mult_mixed = mults[mi]; }
          else { P->chunk = chunks[ci]; P->grid_mult_fp64 = mults[mi]; }
          double t_min = 1e300;
          for (int rep = 0; rep < 3 && !rc; ++rep) {
            rc = hip_check(hipEventRecord(e0, s), "record");
            if (!rc) rc = eval_device(P, params, n, np, np_uniform, stride, F, nullptr, 0,
                                      mixed, s, nullptr, false, false, ex != 0);
            if (!rc) rc = hip_check(hipEventRecord(e1, s), "record");
            if (!rc) rc = hip_check(hipEventSynchronize(e1), "sync");
            float ms = 0.f;
            if (!rc) rc = hip_check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
            if (rep > 0 && ms < t_min) t_min = ms;   // first repetition is a warm-up
          }
          if (!rc && (ms_best < 0 || t_min < ms_best)) {
            ms_best = t_min; c = chunks[ci]; m = mults[mi]; e = ex;
          }
        }
    P->chunk = save_c; P->chunk_mixed = save_cm;
    if (mixed) P->grid_mult_mixed = save_m; else P->grid_mult_fp64 = save_m;
    prefer = save_p;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (F) (void)hipFree(F);
    if (rc) return rc;
    tune_cache_put(key, c, m, e);
  }
  if (mixed) { P->chunk_mixed = c; P->grid_mult_mixed = m; }
  else { P->chunk = c; P->grid_mult_fp64 = m; }
  if (!exact) prefer = mode && e != 0;
  if (best_chunk) *best_chunk = c;
  if (best_mult) *best_mult = m;
  if (best_ms) *best_ms = ms_best;
  return FSTAT_OK;
}


const char* fstat_last_error(void) { return g_err.c_str(); }

int fstat_plan_create(fstat_plan_t* out, const fstat_data_desc* d, const fstat_opts* opts,
                      void* hip_stream) {
  g_err.clear();
  if (!out || !d) return set_error(FSTAT_EINVAL, "null plan or data descriptor");
  *out = nullptr;
  if (d->nbins < 1 || d->nbins > INT32_MAX - 1) return set_error(FSTAT_EINVAL, "nbins out of range");
  if (!(d->df > 0.0) || !std::isfinite(d->df)) return set_error(FSTAT_EINVAL, "df must be > 0");
  if (d->k_lo < 1) return set_error(FSTAT_EINVAL, "k_lo must be >= 1");
  if (!(d->T_obs > 0.0) || !std::isfinite(d->T_obs)) return set_error(FSTAT_EINVAL, "T_obs must be > 0");
  if (!d->data || !d->psd) return set_error(FSTAT_EINVAL, "null data or psd");
  uint32_t flags = opts ? opts->flags : 0u;
  int prec = opts ? opts->precision : 0;
  if (prec == 0) prec = FSTAT_FP64 | FSTAT_MIXED;
  if (prec & ~(FSTAT_FP64 | FSTAT_MIXED)) return set_error(FSTAT_EINVAL, "bad precision mask");
  int chunk = (opts && opts->chunk > 0) ? opts->chunk : 2048;
  const double budget = (opts && opts->refine_budget != 0.0) ? opts->refine_budget : 5e-10;
  if (!std::isfinite(budget)) return set_error(FSTAT_EINVAL, "refine_budget must be finite");
  if (chunk < 64 || chunk > (1 << 24)) return set_error(FSTAT_EINVAL, "chunk out of range");
  const bool dev = (flags & FSTAT_DEVICE_PTRS) != 0;
  const int64_t nb = d->nbins;
  Channels chan;
  chan.n = d->n_channels > 0 ? d->n_channels : 1;
  if (chan.n > kMaxChannels) return set_error(FSTAT_EINVAL, "at most %d channels", kMaxChannels);
  for (int c = 0; c < chan.n; ++c) {
    chan.code[c] = d->channels ? d->channels[c] : FSTAT_CHANNEL_X;
    if (chan.code[c] < FSTAT_CHANNEL_X || chan.code[c] > FSTAT_CHANNEL_T)
      return set_error(FSTAT_EINVAL, "channels[%d] = %d is not a channel code", c, chan.code[c]);
    for (int e = 0; e < c; ++e)
      if (chan.code[e] == chan.code[c])
        return set_error(FSTAT_EINVAL, "channel %d listed twice", chan.code[c]);
  }
  const int64_t nbc = nb * chan.n;   // bins of all channels
  if (nbc > (int64_t)INT32_MAX) return set_error(FSTAT_EINVAL, "nbins x channels out of range");
  if (!dev) {
    for (int64_t j = 0; j < nbc; ++j) {
      if (!(d->psd[j] > 0.0) || !std::isfinite(d->psd[j]))
        return set_error(FSTAT_EINVAL, "psd[%lld] must be finite and > 0", (long long)j);
      if (!std::isfinite(d->data[2 * j]) || !std::isfinite(d->data[2 * j + 1]))
        return set_error(FSTAT_EINVAL, "data[%lld] is not finite", (long long)j);
    }
  }
  hipStream_t s = (hipStream_t)hip_stream;
  fstat_plan_s* P = new fstat_plan_s();
  P->grid = Grid{d->df, d->T_obs, d->k_lo, nb};
  P->grid.chan = chan;
  P->prec = prec;
  P->chunk = chunk;
  P->refine_budget = budget;
  int rc = hip_check(hipGetDevice(&P->device), "hipGetDevice");
  if (!rc) rc = hip_check(hipDeviceGetAttribute(&P->num_cu, hipDeviceAttributeMultiprocessorCount,
                                                P->device), "device attribute");
  if (!rc && interp_tables_init() != 0)
    rc = set_error(FSTAT_EDEVICE, "could not upload the interpolation tables");
  if (!rc) rc = scratch_init(P->device);
  double *dd = nullptr, *dp = nullptr;
  if (!rc) rc = dev_alloc(&P->b64.wr, nbc, "alloc wr");
  if (!rc) rc = dev_alloc(&P->b64.wi, nbc, "alloc wi");
  if (!rc) rc = dev_alloc(&P->b64.u, nbc, "alloc u");
  if (!rc) rc = dev_alloc(&P->b64.s0, nb, "alloc s0");
  if (!rc) rc = dev_alloc(&P->b64.c0, nb, "alloc c0");
  if (!rc && (prec & FSTAT_MIXED)) {
    rc = dev_alloc(&P->b32.wr, nbc, "alloc wr32");
    if (!rc) rc = dev_alloc(&P->b32.wi, nbc, "alloc wi32");
    if (!rc) rc = dev_alloc(&P->b32.u, nbc, "alloc u32");
    if (!rc) rc = dev_alloc(&P->b32.s0, nb, "alloc s032");
    if (!rc) rc = dev_alloc(&P->b32.c0, nb, "alloc c032");
  }
  if (!rc) rc = dev_alloc(&P->umax, 1, "alloc umax");
  if (!rc && (flags & FSTAT_PROFILE)) {
    P->profile = true;
    rc = dev_alloc(&P->bin_counter, 1, "alloc counter");
    if (!rc) rc = hip_check(hipMemsetAsync(P->bin_counter, 0, sizeof(unsigned long long), s), "memset");
  }
  const double* ddata = d->data;
  const double* dpsd = d->psd;
  if (!rc && !dev) {
    rc = dev_alloc(&dd, 2 * nbc, "alloc data staging");
    if (!rc) rc = dev_alloc(&dp, nbc, "alloc psd staging");
    if (!rc) rc = hip_check(hipMemcpyAsync(dd, d->data, sizeof(double) * 2 * nbc,
                                           hipMemcpyHostToDevice, s), "copy data");
    if (!rc) rc = hip_check(hipMemcpyAsync(dp, d->psd, sizeof(double) * nbc,
                                           hipMemcpyHostToDevice, s), "copy psd");
    ddata = dd;
    dpsd = dp;
  }
  std::vector<double> ures;
  const int32_t nut_all = (int32_t)((nb + kUTile - 1) / kUTile) * chan.n;   // u-tiles, all channels
  if (!rc) {
    P->n_utiles = (int32_t)((nb + kUTile - 1) / kUTile);
    ures.assign((size_t)nut_all, 0.0);
    rc = dev_alloc(&P->ucoef, (size_t)nut_all * kUCoef, "alloc u model");
    if (!rc) rc = dev_alloc(&P->ubad, (size_t)nut_all + 1, "alloc u model flags");
  }
  if (!rc) rc = dev_alloc(&P->ures, (size_t)nut_all, "alloc u model residuals");
  double* ubsum = nullptr;
  if (!rc) rc = dev_alloc(&P->upre, (size_t)(nb + 1) * chan.n, "alloc u prefix sums");
  if (!rc) rc = dev_alloc(&ubsum, (size_t)uprefix_block_sums(nb), "alloc u prefix scratch");
  double* dres = P->ures;
  if (!rc) {
    launch_prep(P->grid, ddata, dpsd, P->b64, s);
    launch_max(P->b64.u, nbc, P->umax, s);
    launch_scale(P->grid, P->umax, P->b64, P->b32, s);
    for (int c = 0; c < chan.n; ++c)
      launch_ufit(P->b64.u + (int64_t)c * nb, nb, P->n_utiles,
                  P->ucoef + (int64_t)c * P->n_utiles * kUCoef, dres + (int64_t)c * P->n_utiles, s);
    for (int c = 0; c < chan.n; ++c)
      launch_uprefix(P->b64.u + (int64_t)c * nb, nb, ubsum, P->upre + (int64_t)c * (nb + 1), s);
    rc = hip_check(hipGetLastError(), "prep launch");
  }
  if (!rc) rc = hip_check(hipMemcpyAsync(ures.data(), dres, sizeof(double) * nut_all,
                                         hipMemcpyDeviceToHost, s), "read u model residuals");
  if (!rc) rc = hip_check(hipStreamSynchronize(s), "plan prep");
  if (!rc) {
    // prefix count of u-tiles the smooth model does not fit to within kUFitTol
    std::vector<int32_t> bad((size_t)nut_all + 1, 0);
    for (int32_t i = 0; i < nut_all; ++i) {
      const bool ok = ures[(size_t)i] <= kUFitTol;
      bad[(size_t)i + 1] = bad[(size_t)i] + (ok ? 0 : 1);
      P->n_ufit += ok ? 1 : 0;
    }
    rc = hip_check(hipMemcpyAsync(P->ubad, bad.data(), sizeof(int32_t) * bad.size(),
                                  hipMemcpyHostToDevice, s), "copy u model flags");
    if (!rc) rc = hip_check(hipStreamSynchronize(s), "plan prep");
  }
  dev_free(dd);
  dev_free(dp);
  dev_free(ubsum);
  if (rc) {
    fstat_plan_destroy(P);
    return rc;
  }
  if (!(prec & FSTAT_FP64)) {
    // the FP64 data are only needed to build the FP32 copies (the exact mixed
    // loop keeps sin, cos(pi f L) in FP64 for its FP64 response)
    dev_free(P->b64.wr); dev_free(P->b64.wi); dev_free(P->b64.u);
  }
  *out = P;
  return FSTAT_OK;
}

void fstat_plan_destroy(fstat_plan_t P) {
  if (!P) return;
  dev_free(P->b64.wr); dev_free(P->b64.wi); dev_free(P->b64.u);
  dev_free(P->b64.s0); dev_free(P->b64.c0);
  dev_free(P->b32.wr); dev_free(P->b32.wi); dev_free(P->b32.u);
  dev_free(P->b32.s0); dev_free(P->b32.c0);
  dev_free(P->ws.pc); dev_free(P->ws.bounds); dev_free(P->ws.cnt); dev_free(P->ws.off);
  dev_free(P->ws.total); dev_free(P->ws.items); dev_free(P->ws.partials); dev_free(P->ws.Fl);
  dev_free(P->ws.direct); dev_free(P->ws.ndirect); dev_free(P->ws.bsum);
  dev_free(P->ws.tcnt); dev_free(P->ws.tcur); dev_free(P->ws.toff); dev_free(P->ws.uoff);
  dev_free(P->ws.tile_items);
  dev_free(P->ws.tile_ctr); dev_free(P->ws.xflag); dev_free(P->ws.rec); dev_free(P->ws.xerr); dev_free(P->ws.refine); dev_free(P->ws.nrefine);
  dev_free(P->io.params); dev_free(P->io.np); dev_free(P->io.F_hat); dev_free(P->io.F_part);
  dev_free(P->io.amps); dev_free(P->umax); dev_free(P->ucoef); dev_free(P->ubad);
  dev_free(P->ures); dev_free(P->upre); dev_free(P->orb_coef);
  pso_release(P);
  sur_release(P);
  for (auto& e : P->events)
    for (auto x : e) (void)hipEventDestroy(x);
  dev_free(P->bin_counter);
  delete P;
}

int fstat_interp_stats(fstat_plan_t P, int64_t* items, int64_t* rejected, int64_t* refined,
                       int64_t* bin_mix, void* hip_stream) {
  g_err.clear();
  if (!P || !P->ws.total || !P->ws.ndirect || !P->ws.nrefine || P->last.stride < 1)
    return set_error(FSTAT_EINVAL, "no evaluation yet");
  hipStream_t s = (hipStream_t)hip_stream;
  int rc0 = FSTAT_OK;
  if (bin_mix) {
    unsigned long long* d = nullptr;
    unsigned long long h[kBinMix] = {};
    rc0 = hip_check(hipMalloc(&d, sizeof(h)), "alloc bin mix");
    if (!rc0) rc0 = hip_check(hipMemcpyAsync(d, h, sizeof(h), hipMemcpyHostToDevice, s), "clear bin mix");
    if (!rc0 && P->last.exact) {
      // every item went through the exact loop: count them all as exact bins
      rc0 = set_error(FSTAT_EINVAL, "the last evaluation used the exact loop only");
    }
    if (!rc0) {
      launch_bin_mix(P->last.mixed, P->last.stride, P->last.chunk, P->grid.chan.n, P->ws, d, s);
      rc0 = hip_check(hipGetLastError(), "bin mix launch");
    }
    if (!rc0) rc0 = hip_check(hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, s), "read bin mix");
    if (!rc0) rc0 = hip_check(hipStreamSynchronize(s), "bin mix");
    if (d) (void)hipFree(d);
    if (rc0) return rc0;
    for (int i = 0; i < kBinMix; ++i) bin_mix[i] = (int64_t)h[i];
  }
  int32_t v[3] = {0, 0, 0};
  int rc = hip_check(hipMemcpyAsync(&v[0], P->ws.total, sizeof(int32_t), hipMemcpyDeviceToHost, s),
                     "read total");
  if (!rc) rc = hip_check(hipMemcpyAsync(&v[1], P->ws.ndirect, sizeof(int32_t),
                                         hipMemcpyDeviceToHost, s), "read ndirect");
  if (!rc) rc = hip_check(hipMemcpyAsync(&v[2], P->ws.nrefine, sizeof(int32_t),
                                         hipMemcpyDeviceToHost, s), "read nrefine");
  if (!rc) rc = hip_check(hipStreamSynchronize(s), "interp stats");
  if (rc) return rc;
  if (items) *items = v[0];
  if (rejected) *rejected = v[1];
  if (refined) *refined = v[2];
  return FSTAT_OK;
}

int fstat_profile_read(fstat_plan_t P, int reset, double* kernel_ms, double* main_ms,
                       int64_t* launches, int64_t* bin_templates) {
  g_err.clear();
  if (!P || !P->profile) return set_error(FSTAT_EINVAL, "plan was not created with FSTAT_PROFILE");
  double tot = 0.0, tmain = 0.0;
  for (auto& e : P->events) {
    int rc = hip_check(hipEventSynchronize(e[3]), "event sync");
    if (rc) return rc;
    float ms = 0.f, mm = 0.f;
    if ((rc = hip_check(hipEventElapsedTime(&ms, e[0], e[3]), "elapsed"))) return rc;
    if ((rc = hip_check(hipEventElapsedTime(&mm, e[1], e[2]), "elapsed"))) return rc;
    tot += ms;
    tmain += mm;
  }
  unsigned long long bins = 0;
  int rc = hip_check(hipMemcpy(&bins, P->bin_counter, sizeof(bins), hipMemcpyDeviceToHost), "read counter");
  if (rc) return rc;
  if (kernel_ms) *kernel_ms = tot;
  if (main_ms) *main_ms = tmain;
  if (launches) *launches = (int64_t)P->events.size();
  if (bin_templates) *bin_templates = (int64_t)bins;
  if (reset) {
    for (auto& e : P->events)
      for (auto x : e) (void)hipEventDestroy(x);
    P->events.clear();
    rc = hip_check(hipMemset(P->bin_counter, 0, sizeof(unsigned long long)), "reset counter");
  }
  return rc;
}

int fstat_eval(fstat_plan_t P, const double* params, int64_t n, const int32_t* np,
               int32_t np_uniform, double* F_hat, double* F_part, double* amps,
               int64_t part_stride, uint32_t flags, void* hip_stream) {
  g_err.clear();
  if (!P) return set_error(FSTAT_EINVAL, "null plan");
  if (n < 0) return set_error(FSTAT_EINVAL, "n < 0");
  if (n == 0) return FSTAT_OK;
  if (!params || !F_hat) return set_error(FSTAT_EINVAL, "null params or F_hat");
  const bool mixed = (flags & FSTAT_EVAL_MIXED) != 0;
  const bool dev = (flags & FSTAT_DEVICE_PTRS) != 0;
  const bool sur = (flags & FSTAT_EVAL_SURROGATE) != 0;
  const bool exact = (flags & FSTAT_EVAL_EXACT) != 0;
  if (sur && !P->sur_trained) return set_error(FSTAT_EINVAL, "surrogate requested but not trained");
  if (mixed && !(P->prec & FSTAT_MIXED)) return set_error(FSTAT_EINVAL, "plan has no mixed data");
  if (!mixed && !(P->prec & FSTAT_FP64)) return set_error(FSTAT_EINVAL, "plan has no FP64 data");
  int32_t stride;
  if (np) {
    if (part_stride < 1 || part_stride > 65536)
      return set_error(FSTAT_EINVAL, "part_stride must give the largest np (1..65536)");
    stride = (int32_t)part_stride;
  } else {
    if (np_uniform < 1 || np_uniform > 65536) return set_error(FSTAT_EINVAL, "np_uniform out of range");
    if ((F_part || amps) && part_stride < np_uniform)
      return set_error(FSTAT_EINVAL, "part_stride < np");
    stride = np_uniform;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  if (dev)
    return eval_device(P, params, n, np, np_uniform, stride, F_hat, F_part, part_stride, mixed, s,
                       nullptr, true, sur, exact, amps);
  // host pointers: validate, stage, run, copy back
  for (int64_t i = 0; i < n; ++i) {
    const double* t = params + 6 * i;
    bool ok = true;
    for (int k = 0; k < 6; ++k) ok = ok && std::isfinite(t[k]);
    if (!ok || !(t[1] > 0.0) || !(std::fabs(t[2]) < 1.0) || !(t[5] >= 0.0))
      return set_error(FSTAT_EINVAL, "particle %lld has invalid parameters", (long long)i);
    if (np && (np[i] < 1 || np[i] > stride))
      return set_error(FSTAT_EINVAL, "np[%lld] = %d outside 1..part_stride", (long long)i, np[i]);
  }
  int rc;
  if ((rc = ensure(&P->io.params, &P->cap.params, (size_t)n * 6, "alloc params"))) return rc;
  if ((rc = ensure(&P->io.np, &P->cap.np, (size_t)n, "alloc np"))) return rc;
  if ((rc = ensure(&P->io.F_hat, &P->cap.F_hat, (size_t)n, "alloc F_hat"))) return rc;
  int64_t ps = (F_part || amps) ? part_stride : 0;
  if (F_part && (rc = ensure(&P->io.F_part, &P->cap.F_part, (size_t)n * ps, "alloc F_part"))) return rc;
  if (amps && (rc = ensure(&P->io.amps, &P->cap.amps, (size_t)n * ps * 4, "alloc amps"))) return rc;
  if ((rc = hip_check(hipMemcpyAsync(P->io.params, params, sizeof(double) * 6 * n,
                                     hipMemcpyHostToDevice, s), "copy params"))) return rc;
  if (np && (rc = hip_check(hipMemcpyAsync(P->io.np, np, sizeof(int32_t) * n,
                                           hipMemcpyHostToDevice, s), "copy np"))) return rc;
  if (F_part && (rc = hip_check(hipMemcpyAsync(P->io.F_part, F_part, sizeof(double) * n * ps,
                                               hipMemcpyHostToDevice, s), "copy F_part"))) return rc;
  if (amps && (rc = hip_check(hipMemcpyAsync(P->io.amps, amps, sizeof(double) * n * ps * 4,
                                             hipMemcpyHostToDevice, s), "copy amps"))) return rc;
  rc = eval_device(P, P->io.params, n, np ? P->io.np : nullptr, np_uniform, stride, P->io.F_hat,
                   F_part ? P->io.F_part : nullptr, ps, mixed, s, nullptr, true, sur, exact,
                   amps ? P->io.amps : nullptr);
  if (rc) return rc;
  if ((rc = hip_check(hipMemcpyAsync(F_hat, P->io.F_hat, sizeof(double) * n,
                                     hipMemcpyDeviceToHost, s), "copy F_hat"))) return rc;
  if (F_part && (rc = hip_check(hipMemcpyAsync(F_part, P->io.F_part, sizeof(double) * n * ps,
                                               hipMemcpyDeviceToHost, s), "copy F_part"))) return rc;
  if (amps && (rc = hip_check(hipMemcpyAsync(amps, P->io.amps, sizeof(double) * n * ps * 4,
                                             hipMemcpyDeviceToHost, s), "copy amps"))) return rc;
  return hip_check(hipStreamSynchronize(s), "eval");
}

int fstat_eval_noalloc(fstat_plan_t P, const double* params, int64_t n, const int32_t* np,
                       int32_t np_uniform, double* F_hat, double* F_part, double* amps,
                       int64_t part_stride, uint32_t flags, void* hip_stream) {
  g_err.clear();
  if (!P) return set_error(FSTAT_EINVAL, "null plan");
  if (n < 0) return set_error(FSTAT_EINVAL, "n < 0");
  if (n == 0) return FSTAT_OK;
  if (!params || !F_hat) return set_error(FSTAT_EINVAL, "null params or F_hat");
  if (flags & FSTAT_EVAL_SURROGATE)
    return set_error(FSTAT_EUNSUPPORTED, "fstat_eval_noalloc does not run the surrogate");
  const bool mixed = (flags & FSTAT_EVAL_MIXED) != 0;
  const bool exact = (flags & FSTAT_EVAL_EXACT) != 0 ||
                     (mixed ? P->prefer_exact_mixed : P->prefer_exact_fp64);
  if (mixed && !(P->prec & FSTAT_MIXED)) return set_error(FSTAT_EINVAL, "plan has no mixed data");
  if (!mixed && !(P->prec & FSTAT_FP64)) return set_error(FSTAT_EINVAL, "plan has no FP64 data");
  int32_t stride;
  if (np) {
    if (part_stride < 1 || part_stride > 65536)
      return set_error(FSTAT_EINVAL, "part_stride must give the largest np (1..65536)");
    stride = (int32_t)part_stride;
  } else {
    if (np_uniform < 1 || np_uniform > 65536) return set_error(FSTAT_EINVAL, "np_uniform out of range");
    if ((F_part || amps) && part_stride < np_uniform)
      return set_error(FSTAT_EINVAL, "part_stride < np");
    stride = np_uniform;
  }
  int rc = check_chunk(P, mixed, exact);
  if (rc) return rc;
  int dev = -1;
  if ((rc = hip_check(hipGetDevice(&dev), "hipGetDevice"))) return rc;
  if (dev != P->device)
    return set_error(FSTAT_EINVAL, "the plan lives on device %d, device %d is current", P->device, dev);
  char* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    base = (dev >= 0 && dev < 64) ? g_scratch_dev[dev] : nullptr;
  }
  if (!base) return set_error(FSTAT_EDEVICE, "scratch of device %d was not set up", dev);
  if ((size_t)n * (size_t)stride > (size_t)4096 * 4096)
    return set_error(FSTAT_EINVAL, "n * stride above 16.7M partitions");
  const int chunk = chunk_for(P, mixed);
  const size_t need = carve_workspace(P, n, stride, chunk, nullptr, nullptr);
  if (need > kScratchBytes)
    return set_error(FSTAT_EINVAL, "fstat_eval_noalloc: %lld particles x (%d partitions + bin tiles) "
                     "need %zu bytes of scratch, above its fixed %zu bytes (use fstat_eval, or "
                     "fewer particles per call)", (long long)n, stride, need, kScratchBytes);
  WorkSpace ws{};
  carve_workspace(P, n, stride, chunk, base, &ws);
  return eval_enqueue(P, ws, params, n, np, np_uniform, stride, F_hat, F_part, part_stride, mixed,
                      (hipStream_t)hip_stream, nullptr, false, false, exact, amps);
}

int fstat_waveform(double T_obs, double df, int64_t k_lo, int64_t nbins, const double* params6,
                   const double* amps4, double* out, uint32_t flags, void* hip_stream) {
  g_err.clear();
  if (nbins < 1 || nbins > INT32_MAX - 1 || !(df > 0.0) || k_lo < 1 || !(T_obs > 0.0))
    return set_error(FSTAT_EINVAL, "bad grid");
  if (!params6 || !amps4 || !out) return set_error(FSTAT_EINVAL, "null argument");
  const bool dev = (flags & FSTAT_DEVICE_PTRS) != 0;
  if (!dev) {
    bool ok = true;
    for (int k = 0; k < 6; ++k) ok = ok && std::isfinite(params6[k]);
    for (int k = 0; k < 4; ++k) ok = ok && std::isfinite(amps4[k]);
    if (!ok || !(params6[1] > 0.0) || !(std::fabs(params6[2]) < 1.0) || !(params6[5] >= 0.0))
      return set_error(FSTAT_EINVAL, "invalid parameters");
  }
  const int code = (int)((flags >> 8) & 0xffu);
  if (code > FSTAT_CHANNEL_T) return set_error(FSTAT_EINVAL, "bad channel code %d", code);
  hipStream_t s = (hipStream_t)hip_stream;
  Grid g{df, T_obs, k_lo, nbins};
  g.chan.code[0] = code;
  WorkSpace ws{};
  double *dpar = nullptr, *damp = nullptr, *dout = nullptr;
  int rc = dev_alloc(&ws.pc, 1, "alloc pc");
  if (!rc) rc = dev_alloc(&ws.bounds, 2, "alloc bounds");
  if (!rc) rc = dev_alloc(&ws.cnt, 1, "alloc cnt");
  const double* pp = params6;
  const double* ap = amps4;
  double* op = out;
  if (!rc && !dev) {
    rc = dev_alloc(&dpar, 6, "alloc params");
    if (!rc) rc = dev_alloc(&damp, 4, "alloc amps");
    if (!rc) rc = dev_alloc(&dout, 2 * nbins, "alloc out");
    if (!rc) rc = hip_check(hipMemcpyAsync(dpar, params6, 6 * sizeof(double), hipMemcpyHostToDevice, s), "copy");
    if (!rc) rc = hip_check(hipMemcpyAsync(damp, amps4, 4 * sizeof(double), hipMemcpyHostToDevice, s), "copy");
    pp = dpar; ap = damp; op = dout;
  }
  if (!rc) {
      launch_setup(g, pp, 1, nullptr, 1, 1, 1 << 24, nullptr, ws, s);
    launch_waveform(g, ws.pc, ap, op, s);
    rc = hip_check(hipGetLastError(), "waveform launch");
  }
  if (!rc && !dev)
    rc = hip_check(hipMemcpyAsync(out, dout, sizeof(double) * 2 * nbins, hipMemcpyDeviceToHost, s), "copy out");
  if (!rc) rc = hip_check(hipStreamSynchronize(s), "waveform");
  dev_free(ws.pc); dev_free(ws.bounds); dev_free(ws.cnt);
  dev_free(dpar); dev_free(damp); dev_free(dout);
  return rc;
}

int fstat_plan_set_orbit(fstat_plan_t P, double t0, double dt, int32_t n_seg, const double* nodes,
                         uint32_t flags, void* hip_stream) {
  g_err.clear();
  if (!P) return set_error(FSTAT_EINVAL, "null plan");
  hipStream_t s = (hipStream_t)hip_stream;
  if (n_seg == 0) {   // back to the analytic orbit
    int rc = hip_check(hipStreamSynchronize(s), "orbit");
    dev_free(P->orb_coef);
    P->orb_coef = nullptr;
    P->grid.orb = OrbitTable{};
    return rc;
  }
  if (n_seg < 0 || !nodes) return set_error(FSTAT_EINVAL, "n_seg < 0 or null nodes");
  if (!(dt > 0.0) || !std::isfinite(dt) || !std::isfinite(t0))
    return set_error(FSTAT_EINVAL, "t0 must be finite and dt > 0");
  if (t0 > 0.0 || t0 + dt * n_seg < P->grid.T_obs)
    return set_error(FSTAT_EINVAL, "the table must cover [0, T_obs]");
  const size_t nv = (size_t)n_seg * 90;
  std::vector<double> v(nv), c(nv);
  int rc = 0;
  if (flags & FSTAT_DEVICE_PTRS) {
    if ((rc = hip_check(hipMemcpyAsync(v.data(), nodes, sizeof(double) * nv, hipMemcpyDeviceToHost, s),
                        "copy orbit")) ||
        (rc = hip_check(hipStreamSynchronize(s), "copy orbit")))
      return rc;
  } else {
    memcpy(v.data(), nodes, sizeof(double) * nv);
  }
  for (size_t i = 0; i < nv; ++i)
    if (!std::isfinite(v[i])) return set_error(FSTAT_EINVAL, "orbit node %zu is not finite", i);
  // node values at s_k = cos(pi (k + 1/2) / 10) -> Chebyshev coefficients
  const long double pi = 3.141592653589793238462643383279502884L;
  for (size_t sq = 0; sq < (size_t)n_seg * 9; ++sq)
    for (int j = 0; j < 10; ++j) {
      long double a = 0.0L;
      for (int k = 0; k < 10; ++k) a += (long double)v[sq * 10 + k] * cosl(pi * j * (k + 0.5L) / 10.0L);
      c[sq * 10 + j] = (double)(a * (j == 0 ? 1.0L : 2.0L) / 10.0L);
    }
  double* dc = nullptr;
  if ((rc = dev_alloc(&dc, nv, "alloc orbit"))) return rc;
  rc = hip_check(hipMemcpyAsync(dc, c.data(), sizeof(double) * nv, hipMemcpyHostToDevice, s), "copy orbit");
  if (!rc) rc = hip_check(hipStreamSynchronize(s), "copy orbit");
  if (rc) { dev_free(dc); return rc; }
  dev_free(P->orb_coef);
  P->orb_coef = dc;
  P->grid.orb.coef = dc;
  P->grid.orb.nseg = n_seg;
  P->grid.orb.t0 = t0;
  P->grid.orb.dt = dt;
  return FSTAT_OK;
}

int fstat_extrinsic(const double* amps, const double* params, int64_t n, double* out,
                    uint32_t flags, void* hip_stream) {
  g_err.clear();
  if (n < 0) return set_error(FSTAT_EINVAL, "n < 0");
  if (n == 0) return FSTAT_OK;
  if (!amps || !out) return set_error(FSTAT_EINVAL, "null amps or out");
  const bool dev = (flags & FSTAT_DEVICE_PTRS) != 0;
  hipStream_t s = (hipStream_t)hip_stream;
  if (dev) {
    launch_extrinsic(amps, params, n, out, s);
    return hip_check(hipGetLastError(), "extrinsic launch");
  }
  if (params)
    for (int64_t i = 0; i < n; ++i)
      if (!(params[6 * i + 1] > 0.0) || !std::isfinite(params[6 * i + 1]))
        return set_error(FSTAT_EINVAL, "particle %lld has an invalid chirp mass", (long long)i);
  double *da = nullptr, *dpar = nullptr, *dout = nullptr;
  int rc = dev_alloc(&da, (size_t)n * 4, "alloc amps");
  if (!rc) rc = dev_alloc(&dout, (size_t)n * 4, "alloc out");
  if (!rc && params) rc = dev_alloc(&dpar, (size_t)n * 6, "alloc params");
  if (!rc) rc = hip_check(hipMemcpyAsync(da, amps, sizeof(double) * 4 * n, hipMemcpyHostToDevice, s),
                          "copy amps");
  if (!rc && params)
    rc = hip_check(hipMemcpyAsync(dpar, params, sizeof(double) * 6 * n, hipMemcpyHostToDevice, s),
                   "copy params");
  if (!rc) {
    launch_extrinsic(da, dpar, n, dout, s);
    rc = hip_check(hipGetLastError(), "extrinsic launch");
  }
  if (!rc) rc = hip_check(hipMemcpyAsync(out, dout, sizeof(double) * 4 * n, hipMemcpyDeviceToHost, s),
                          "copy out");
  if (!rc) rc = hip_check(hipStreamSynchronize(s), "extrinsic");
  dev_free(da); dev_free(dpar); dev_free(dout);
  return rc;
}

}  // extern "C"
