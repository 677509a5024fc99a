// search.hip -- the three-stage hierarchical search of Sec. III.B (Fig. 2) on
// top of the batched PSO stage: t_c slices -> (t_c, Mc) boxes around each
// slice's best -> two narrow boxes around the single best and its theta
// mirror, then the amplitudes and extrinsic parameters of the estimate
// (App. B).  Host code only: every statistic evaluation is a pso_stage or
// fstat_eval launch.
//
// Checkpoint file (text, one stage per block, values printed with 17
// significant digits so that they read back exactly):
//   fstat_search 1 <key, 16 hex digits>
//   stage <s> <n>
//   <x_0> ... <x_5> <F_hat>            (n lines: the best of each space)
// The key is an FNV-1a hash of every descriptor field that changes results
// and of the plan's grid.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fstat.h"
#include "fstat_api_internal.h"

static_assert(sizeof(fstat_search_desc) == 280, "fstat_search_desc layout");
static_assert(sizeof(fstat_search_result) == 320, "fstat_search_result layout");

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr uint64_t kStageSeedStep = 0x9E3779B97F4A7C15ull;

struct Best {
  double x[6];
  double F;
};

int check_desc(const fstat_search_desc* d) {
  using fstat::set_error;
  if (!d) return set_error(FSTAT_EINVAL, "null search descriptor");
  for (int j = 0; j < 6; ++j)
    if (!std::isfinite(d->box[j][0]) || !std::isfinite(d->box[j][1]) || !(d->box[j][1] >= d->box[j][0]))
      return set_error(FSTAT_EINVAL, "box[%d] is not a finite interval", j);
  if (d->n_slices < 1 || d->n_slices > 4096) return set_error(FSTAT_EINVAL, "n_slices outside 1..4096");
  for (int s = 0; s < 3; ++s) {
    if (d->runs[s] < 1 || d->iters[s] < 0 || d->np[s] < 1 || d->np[s] > 65536)
      return set_error(FSTAT_EINVAL, "stage %d: runs >= 1, iters >= 0, np in 1..65536", s + 1);
  }
  if (d->n_part < 1 || d->n_part > 1024) return set_error(FSTAT_EINVAL, "n_part outside 1..1024");
  for (int j = 0; j < 2; ++j)
    if (!(d->width2[j] > 0.0) || !std::isfinite(d->width2[j]))
      return set_error(FSTAT_EINVAL, "width2[%d] must be finite and > 0", j);
  for (int j = 0; j < 5; ++j)
    if (!(d->width3[j] > 0.0) || !std::isfinite(d->width3[j]))
      return set_error(FSTAT_EINVAL, "width3[%d] must be finite and > 0", j);
  if (d->max_stage < 0 || d->max_stage > 3) return set_error(FSTAT_EINVAL, "max_stage outside 0..3");
  return FSTAT_OK;
}

// [lo, hi] = c -+ w/2 clipped to the full range of parameter j (phi is left
// unclipped when the full range covers the circle: the statistic is periodic).
void centred(const fstat_search_desc* d, int j, double c, double w, double* lohi) {
  double lo = c - 0.5 * w, hi = c + 0.5 * w;
  const bool circle = (j == 4) && (d->box[4][1] - d->box[4][0] >= 2.0 * kPi);
  if (!circle) {
    lo = std::fmax(lo, d->box[j][0]);
    hi = std::fmin(hi, d->box[j][1]);
    if (hi < lo) lo = hi = std::fmin(std::fmax(c, d->box[j][0]), d->box[j][1]);
  }
  lohi[0] = lo;
  lohi[1] = hi;
}

int make_boxes(const fstat_search_desc* d, int stage, const double* centres, int n_centres,
               std::vector<double>& out) {
  if (stage == 1) {
    const int n = d->n_slices;
    out.assign((size_t)n * 12, 0.0);
    const double lo = d->box[0][0], hi = d->box[0][1];
    for (int k = 0; k < n; ++k) {
      double* b = &out[(size_t)k * 12];
      for (int j = 0; j < 6; ++j) { b[2 * j] = d->box[j][0]; b[2 * j + 1] = d->box[j][1]; }
      b[0] = lo + (hi - lo) * (double)k / (double)n;
      b[1] = (k + 1 == n) ? hi : lo + (hi - lo) * (double)(k + 1) / (double)n;
    }
    return n;
  }
  if (!centres || n_centres < 1) return -1;
  if (stage == 2) {
    out.assign((size_t)n_centres * 12, 0.0);
    for (int k = 0; k < n_centres; ++k) {
      double* b = &out[(size_t)k * 12];
      const double* c = centres + 6 * k;
      for (int j = 0; j < 6; ++j) { b[2 * j] = d->box[j][0]; b[2 * j + 1] = d->box[j][1]; }
      centred(d, 0, c[0], d->width2[0], b);
      centred(d, 1, c[1], d->width2[1], b + 2);
    }
    return n_centres;
  }
  if (stage == 3) {
    out.assign(24, 0.0);
    const double* c = centres;
    for (int m = 0; m < 2; ++m) {
      double* b = &out[(size_t)m * 12];
      b[4] = d->box[2][0];
      b[5] = d->box[2][1];
      centred(d, 0, c[0], d->width3[0], b);
      centred(d, 1, c[1], d->width3[1], b + 2);
      centred(d, 3, m ? kPi - c[3] : c[3], d->width3[2], b + 6);
      centred(d, 4, c[4], d->width3[3], b + 8);
      centred(d, 5, c[5], d->width3[4], b + 10);
    }
    return 2;
  }
  return -1;
}

uint64_t fnv(uint64_t h, const void* p, size_t n) {
  const unsigned char* c = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) { h ^= c[i]; h *= 0x100000001b3ull; }
  return h;
}

uint64_t desc_key(const fstat_search_desc* d, const fstat_plan_s* P) {
  uint64_t h = 0xcbf29ce484222325ull;
  h = fnv(h, d->box, sizeof(d->box));
  h = fnv(h, &d->n_slices, sizeof(d->n_slices));
  h = fnv(h, d->runs, sizeof(d->runs));
  h = fnv(h, d->iters, sizeof(d->iters));
  h = fnv(h, d->np, sizeof(d->np));
  h = fnv(h, &d->n_part, sizeof(d->n_part));
  h = fnv(h, &d->ring_k, sizeof(d->ring_k));
  const double c[5] = {d->w_start, d->w_end, d->c1, d->c2, d->vmax};
  h = fnv(h, c, sizeof(c));
  h = fnv(h, d->width2, sizeof(d->width2));
  h = fnv(h, d->width3, sizeof(d->width3));
  h = fnv(h, &d->seed, sizeof(d->seed));
  h = fnv(h, d->flags, sizeof(d->flags));
  const double g[3] = {P->grid.df, P->grid.T_obs, (double)P->grid.k_lo};
  h = fnv(h, g, sizeof(g));
  h = fnv(h, &P->grid.nbins, sizeof(P->grid.nbins));
  return h;
}

// Reads the finished stages of a checkpoint written for `key`.  Returns the
// number of stages read (0 if the file does not exist), or an error.
int read_checkpoint(const char* path, uint64_t key, std::vector<Best> (&st)[3]) {
  FILE* f = fopen(path, "r");
  if (!f) return 0;
  char magic[32];
  int ver = 0;
  unsigned long long k = 0;
  int got = 0;
  if (fscanf(f, "%31s %d %llx", magic, &ver, &k) != 3 || strcmp(magic, "fstat_search") != 0 || ver != 1) {
    fclose(f);
    return fstat::set_error(FSTAT_EINVAL, "%s is not a search checkpoint", path);
  }
  if ((uint64_t)k != key) {
    fclose(f);
    return fstat::set_error(FSTAT_EINVAL, "%s was written for another search or grid", path);
  }
  for (;;) {
    char word[16];
    int s = 0, n = 0;
    if (fscanf(f, "%15s %d %d", word, &s, &n) != 3) break;
    if (strcmp(word, "stage") != 0 || s != got + 1 || n < 1 || n > 65536) {
      fclose(f);
      return fstat::set_error(FSTAT_EINVAL, "%s: malformed stage record", path);
    }
    std::vector<Best> v((size_t)n);
    for (int i = 0; i < n; ++i) {
      char tok[7][64];
      if (fscanf(f, "%63s %63s %63s %63s %63s %63s %63s", tok[0], tok[1], tok[2], tok[3], tok[4],
                 tok[5], tok[6]) != 7) {
        fclose(f);
        return fstat::set_error(FSTAT_EINVAL, "%s: truncated stage %d", path, s);
      }
      for (int j = 0; j < 6; ++j) v[i].x[j] = strtod(tok[j], nullptr);
      v[i].F = strtod(tok[6], nullptr);
    }
    st[s - 1] = std::move(v);
    got = s;
    if (got == 3) break;
  }
  fclose(f);
  return got;
}

int write_checkpoint(const char* path, uint64_t key, const std::vector<Best> (&st)[3], int done) {
  std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return fstat::set_error(FSTAT_EINVAL, "cannot write %s", tmp.c_str());
  fprintf(f, "fstat_search 1 %016llx\n", (unsigned long long)key);
  for (int s = 0; s < done; ++s) {
    fprintf(f, "stage %d %d\n", s + 1, (int)st[s].size());
    for (const Best& b : st[s]) {
      for (int j = 0; j < 6; ++j) fprintf(f, "%.17g ", b.x[j]);
      fprintf(f, "%.17g\n", b.F);
    }
  }
  const bool ok = fflush(f) == 0;
  fclose(f);
  if (!ok || rename(tmp.c_str(), path) != 0)
    return fstat::set_error(FSTAT_EINVAL, "cannot write %s", path);
  return FSTAT_OK;
}

// One stage: `nb` spaces (boxes [nb][6][2]) with `runs` PSO runs each in one
// pso_stage call; the best of each space (first of equal values; a space
// whose runs found no finite value reports its box centre and -inf).
int run_stage(fstat_plan_t P, const fstat_search_desc* d, int stage, const std::vector<double>& boxes,
              int nb, void* stream, std::vector<Best>& best) {
  const int runs = d->runs[stage - 1];
  const int R = nb * runs;
  std::vector<double> box((size_t)R * 12);
  for (int sp = 0; sp < nb; ++sp)
    for (int k = 0; k < runs; ++k)
      memcpy(&box[((size_t)sp * runs + k) * 12], &boxes[(size_t)sp * 12], 12 * sizeof(double));
  std::vector<int32_t> np((size_t)R, d->np[stage - 1]);
  std::vector<double> bx((size_t)R * 6), bF((size_t)R);
  pso_stage_desc pd{};
  pd.n_runs = R;
  pd.n_part = d->n_part;
  pd.iters = d->iters[stage - 1];
  pd.ring_k = d->ring_k;
  pd.w_start = d->w_start;
  pd.w_end = d->w_end;
  pd.c1 = d->c1;
  pd.c2 = d->c2;
  pd.vmax = d->vmax;
  pd.seed = d->seed + (uint64_t)stage * kStageSeedStep;
  pd.box = box.data();
  pd.np = np.data();
  pd.flags = d->flags[stage - 1];
  pd.use_graph = d->use_graph;
  pso_result pr{};
  pr.best_x = bx.data();
  pr.best_F = bF.data();
  int rc = pso_stage(P, &pd, &pr, stream);
  if (rc) return rc;
  best.assign((size_t)nb, Best{});
  for (int sp = 0; sp < nb; ++sp) {
    int arg = -1;
    double F = -INFINITY;
    for (int k = 0; k < runs; ++k) {
      const double v = bF[(size_t)sp * runs + k];
      if (v > F) { F = v; arg = sp * runs + k; }
    }
    Best& b = best[(size_t)sp];
    b.F = F;
    for (int j = 0; j < 6; ++j)
      b.x[j] = arg >= 0 ? bx[(size_t)arg * 6 + j]
                        : 0.5 * (boxes[(size_t)sp * 12 + 2 * j] + boxes[(size_t)sp * 12 + 2 * j + 1]);
  }
  return FSTAT_OK;
}

int argmax(const std::vector<Best>& v) {
  int a = 0;
  for (int i = 1; i < (int)v.size(); ++i)
    if (v[i].F > v[a].F) a = i;
  return a;
}

}  // namespace

extern "C" int fstat_search_boxes(const fstat_search_desc* d, int32_t stage, const double* centres,
                                  int32_t n_centres, double* boxes_out) {
  int rc = check_desc(d);
  if (rc) return rc;
  if (!boxes_out) return fstat::set_error(FSTAT_EINVAL, "null boxes_out");
  std::vector<double> b;
  int n = make_boxes(d, stage, centres, n_centres, b);
  if (n < 0) return fstat::set_error(FSTAT_EINVAL, "stage must be 1..3 with centres for 2 and 3");
  memcpy(boxes_out, b.data(), b.size() * sizeof(double));
  return n;
}

extern "C" int fstat_search(fstat_plan_t P, const fstat_search_desc* d, fstat_search_result* r,
                            void* hip_stream) {
  using clock = std::chrono::steady_clock;
  if (!P || !r) return fstat::set_error(FSTAT_EINVAL, "null plan or result");
  int rc = check_desc(d);
  if (rc) return rc;
  const int last = d->max_stage ? d->max_stage : 3;
  const uint64_t key = desc_key(d, P);
  std::vector<Best> st[3];
  int done = 0;
  if (d->checkpoint) {
    done = read_checkpoint(d->checkpoint, key, st);
    if (done < 0) return done;
    if (done >= 1 && (int)st[0].size() != d->n_slices)
      return fstat::set_error(FSTAT_EINVAL, "checkpoint stage 1 has %d spaces", (int)st[0].size());
  }
  r->stages_resumed = done;
  for (int s = 0; s < 3; ++s) {
    r->stage_ms[s] = 0.0;
    r->evals[s] = 0;
  }
  for (int stage = done + 1; stage <= last; ++stage) {
    std::vector<double> boxes;
    int nb = 0;
    if (stage == 1) {
      nb = make_boxes(d, 1, nullptr, 0, boxes);
    } else if (stage == 2) {
      std::vector<double> c(st[0].size() * 6);
      for (size_t i = 0; i < st[0].size(); ++i) memcpy(&c[i * 6], st[0][i].x, 6 * sizeof(double));
      nb = make_boxes(d, 2, c.data(), (int)st[0].size(), boxes);
    } else {
      nb = make_boxes(d, 3, st[1][(size_t)argmax(st[1])].x, 1, boxes);
    }
    const auto t0 = clock::now();
    if ((rc = run_stage(P, d, stage, boxes, nb, hip_stream, st[stage - 1]))) return rc;
    r->stage_ms[stage - 1] = std::chrono::duration<double, std::milli>(clock::now() - t0).count();
    r->evals[stage - 1] = (int64_t)nb * d->runs[stage - 1] * d->n_part * d->iters[stage - 1];
    done = stage;
    if (d->checkpoint && (rc = write_checkpoint(d->checkpoint, key, st, done))) return rc;
  }
  r->stages_done = done;
  for (int s = 0; s < 2; ++s) {
    double* x = s == 0 ? r->stage1_x : r->stage2_x;
    double* F = s == 0 ? r->stage1_F : r->stage2_F;
    for (size_t i = 0; i < st[s].size(); ++i) {
      if (x) memcpy(x + 6 * i, st[s][i].x, 6 * sizeof(double));
      if (F) F[i] = st[s][i].F;
    }
  }
  for (int m = 0; m < 2; ++m) {
    const bool have = st[2].size() == 2;
    for (int j = 0; j < 6; ++j) r->stage3_x[m][j] = have ? st[2][(size_t)m].x[j] : NAN;
    r->stage3_F[m] = have ? st[2][(size_t)m].F : NAN;
  }
  for (int k = 0; k < 4; ++k) r->amps[k] = r->extrinsic[k] = NAN;
  if (done == 0) {
    for (int j = 0; j < 6; ++j) r->best_x[j] = NAN;
    r->best_F = NAN;
    return FSTAT_OK;
  }
  const Best& b = st[done - 1][(size_t)argmax(st[done - 1])];
  memcpy(r->best_x, b.x, sizeof(r->best_x));
  r->best_F = b.F;
  if (done < 3 || !std::isfinite(b.F)) return FSTAT_OK;
  // amplitudes of the estimate (fully coherent) and the App. B extrinsics
  double F1 = 0.0;
  const uint32_t fl = (P->prec & FSTAT_FP64) ? 0u : (uint32_t)FSTAT_EVAL_MIXED;
  if ((rc = fstat_eval(P, r->best_x, 1, nullptr, 1, &F1, nullptr, r->amps, 1, fl, hip_stream)))
    return rc;
  return fstat_extrinsic(r->amps, r->best_x, 1, r->extrinsic, 0, hip_stream);
}
