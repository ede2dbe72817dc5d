// Ragged batches: many alignment problems with different plans run as one
// unit of work on one stream -- shared per-lane workspaces sized once, a
// cost-ordered deal of the stacks over lanes, optional capture into one
// hipGraph, and an autotuner over the launch shapes of ftk_tuning_t.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "plan_internal.h"

using namespace ftkint;

namespace {

// Cost model of one stack: Step 1 + Step 3 flop of all its pairs plus the
// transform of its images (the quantities of eq. fbk3 with the sizes of the
// plan), used to order stacks and to deal them over lanes.
double stack_gflop(const ftk_stack& st) {
  const ftk_plan* p = st.plan;
  const double H = p->t.H, M = p->M, QH = p->Qa / 2, N = p->N;
  const double pairs = static_cast<double>(st.nA) * st.nB;
  const double per_pair = 8.0 * H * M * (QH + 1) + 8.0 * N * H * QH + 2.5 * N * p->Qa * std::log2(p->Qa);
  const double nf = p->sk.nf;
  const double per_img = 10.0 * nf * nf * std::log2(nf) + 8.0 * p->M * p->Qa * p->sk.w * p->sk.w;
  return (pairs * per_pair + (st.nA + st.nB) * per_img) * 1e-9;
}

void needs_max(Needs& a, const Needs& b) {
  a.tr_h = std::max(a.tr_h, b.tr_h);
  a.tr_g = std::max(a.tr_g, b.tr_g);
  a.coef_a = std::max(a.coef_a, b.coef_a);
  a.coef_b = std::max(a.coef_b, b.coef_b);
  a.stage = std::max(a.stage, b.stage);
  a.keys = std::max(a.keys, b.keys);
  a.tmpl = std::max(a.tmpl, b.tmpl);
  a.scales = std::max(a.scales, b.scales);
  a.xhat = std::max(a.xhat, b.xhat);
}

hipError_t ensure_all(Workspace& w, const Needs& d) {
  hipError_t e;
  if ((e = w.tr_h.ensure(d.tr_h)) != hipSuccess) return e;
  if ((e = w.tr_g.ensure(d.tr_g)) != hipSuccess) return e;
  if ((e = w.coef_a.ensure(d.coef_a)) != hipSuccess) return e;
  if ((e = w.coef_b.ensure(d.coef_b)) != hipSuccess) return e;
  if ((e = w.stage.ensure(d.stage)) != hipSuccess) return e;
  if ((e = w.keys.ensure(d.keys)) != hipSuccess) return e;
  if ((e = w.tmpl.ensure(d.tmpl)) != hipSuccess) return e;
  if ((e = w.xhat.ensure(d.xhat)) != hipSuccess) return e;
  return w.scales.ensure(d.scales);
}

// ---- autotuner cache -------------------------------------------------------
// Key: the sizes that decide the kernels' shapes and grids.
using TuneKey = std::tuple<int, int, int, int, int, int, int>;

TuneKey tune_key(const ftk_stack& st, int slice_pairs) {
  const ftk_plan* p = st.plan;
  int lg = 0;
  while ((1 << (lg + 1)) <= slice_pairs) ++lg;
  return TuneKey(p->n, p->M, p->Qa, p->H_pad, p->N_pad, p->precision, lg);
}

std::mutex g_tune_mu;
std::map<TuneKey, ftk_tuning_t> g_tune_cache;
bool g_tune_file_read = false;

const char* tune_file() {
  const char* f = std::getenv("FTK_TUNE_CACHE");
  return (f && *f) ? f : nullptr;
}

void tune_cache_load_locked() {
  if (g_tune_file_read) return;
  g_tune_file_read = true;
  const char* path = tune_file();
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  int k[7];
  ftk_tuning_t t;
  while (std::fscanf(f, "%d %d %d %d %d %d %d %d %d %d %d", &k[0], &k[1], &k[2], &k[3], &k[4], &k[5], &k[6],
                     &t.step3_waves, &t.step1_zblk, &t.step1_wgs, &t.stage_mib) == 11)
    g_tune_cache[TuneKey(k[0], k[1], k[2], k[3], k[4], k[5], k[6])] = t;
  std::fclose(f);
}

void tune_cache_store_locked(const TuneKey& k, const ftk_tuning_t& t) {
  g_tune_cache[k] = t;
  const char* path = tune_file();
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%d %d %d %d %d %d %d %d %d %d %d\n", std::get<0>(k), std::get<1>(k), std::get<2>(k),
               std::get<3>(k), std::get<4>(k), std::get<5>(k), std::get<6>(k), t.step3_waves, t.step1_zblk,
               t.step1_wgs, t.stage_mib);
  std::fclose(f);
}

}  // namespace

struct ftk_batch {
  std::vector<ftk_stack> stacks;       // run order (cost descending)
  std::vector<int> lane;               // lane of each stack
  std::vector<ftk_tuning_t> tune;      // launch shapes of each stack
  std::vector<double> cost;            // cost model, GFLOP
  int lanes = 1;
  int flags = 0;
  std::vector<Workspace> ws;           // one per lane
  std::vector<hipStream_t> streams;    // lanes 1.. (lane 0 runs on the caller's stream)
  hipEvent_t ev_fork = nullptr;
  std::vector<hipEvent_t> ev_join;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_nodes = 0;
  double tune_ms = 0.0;
  DevBuf tune_best;                    // poses of the autotuner's slices

  void release() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    for (hipStream_t s : streams) (void)hipStreamDestroy(s);
    streams.clear();
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    ev_fork = nullptr;
    for (hipEvent_t e : ev_join) (void)hipEventDestroy(e);
    ev_join.clear();
    for (auto& w : ws) w.release();
    tune_best.release();
  }
};

namespace {

// One stack's launches on `s`, with the batch's workspace and tuning lent to
// the plan for the duration of the (asynchronous) enqueue.
int run_stack(ftk_batch* b, size_t i, hipStream_t s, bool timers_off) {
  const ftk_stack& st = b->stacks[i];
  ftk_plan* p = st.plan;
  if (st.nA == 0 || st.nB == 0) return FTK_OK;
  Workspace* own = p->ws;
  const ftk_tuning_t saved = p->tune;
  const bool timer_on = p->timer.on;
  p->ws = &b->ws[b->lane[i]];
  p->tune = b->tune[i];
  if (timers_off) p->timer.on = false;
  const int rc = ftk_align(p, st.images, st.nA, st.templates, st.nB, st.X, st.best, s);
  p->timer.on = timer_on;
  p->tune = saved;
  p->ws = own;
  return rc;
}

// Enqueue the whole batch: fork the lanes from `s`, run every stack on its
// lane, join back into `s`.
int enqueue(ftk_batch* b, hipStream_t s, bool capturing) {
  hipError_t e;
  if (b->lanes > 1) {
    if ((e = hipEventRecord(b->ev_fork, s)) != hipSuccess) return hip_fail(e, "ftk_batch: fork");
    for (hipStream_t ls : b->streams)
      if ((e = hipStreamWaitEvent(ls, b->ev_fork, 0)) != hipSuccess) return hip_fail(e, "ftk_batch: fork");
  }
  for (size_t i = 0; i < b->stacks.size(); ++i) {
    const int l = b->lane[i];
    const int rc = run_stack(b, i, l == 0 ? s : b->streams[l - 1], capturing);
    if (rc != FTK_OK) return rc;
  }
  if (b->lanes > 1) {
    for (int l = 1; l < b->lanes; ++l) {
      if ((e = hipEventRecord(b->ev_join[l - 1], b->streams[l - 1])) != hipSuccess) return hip_fail(e, "ftk_batch: join");
      if ((e = hipStreamWaitEvent(s, b->ev_join[l - 1], 0)) != hipSuccess) return hip_fail(e, "ftk_batch: join");
    }
  }
  return FTK_OK;
}

// Candidate launch shapes, explored one coordinate at a time from the
// plan's current tuning; duplicates (same resolved shapes) are skipped.
int autotune_stack(ftk_batch* b, size_t i, hipStream_t s) {
  const ftk_stack& st = b->stacks[i];
  ftk_plan* p = st.plan;
  if (st.nA == 0 || st.nB == 0) return FTK_OK;
  const int slice_nB = std::min(st.nB, 8192);
  const int slice_nA = std::min(st.nA, std::max(1, 8192 / slice_nB));
  const TuneKey key = tune_key(st, slice_nA * slice_nB);
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    tune_cache_load_locked();
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      b->tune[i] = it->second;
      return FTK_OK;
    }
  }
  Workspace* own = p->ws;
  const ftk_tuning_t saved = p->tune;
  const bool timer_on = p->timer.on;
  p->ws = &b->ws[0];
  p->timer.on = false;
  int rc = FTK_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ftk_tuning_t best_t = b->tune[i];
  float best_ms = 0.f;
  auto restore = [&]() {
    p->timer.on = timer_on;
    p->tune = saved;
    p->ws = own;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  hipError_t e;
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
    restore();
    return hip_fail(e, "ftk_batch: autotune events");
  }
  // coefficients of the slice, once
  const Workspace& w = b->ws[0];
  rc = ftk_transform(p, st.images, slice_nA, w.coef_a.ptr, s);
  if (rc == FTK_OK) rc = ftk_transform(p, st.templates, slice_nB, w.coef_b.ptr, s);
  auto time_one = [&](const ftk_tuning_t& t, float* ms) -> int {
    p->tune = t;
    int r = ftk_align_coeffs(p, w.coef_a.ptr, slice_nA, w.coef_b.ptr, slice_nB, nullptr,
                             b->tune_best.as<ftk_pose>(), s);  // warm
    if (r != FTK_OK) return r;
    hipError_t he;
    if ((he = hipEventRecord(e0, s)) != hipSuccess) return hip_fail(he, "ftk_batch: autotune");
    r = ftk_align_coeffs(p, w.coef_a.ptr, slice_nA, w.coef_b.ptr, slice_nB, nullptr, b->tune_best.as<ftk_pose>(), s);
    if (r != FTK_OK) return r;
    if ((he = hipEventRecord(e1, s)) != hipSuccess) return hip_fail(he, "ftk_batch: autotune");
    if ((he = hipEventSynchronize(e1)) != hipSuccess) return hip_fail(he, "ftk_batch: autotune");
    if ((he = hipEventElapsedTime(ms, e0, e1)) != hipSuccess) return hip_fail(he, "ftk_batch: autotune");
    return FTK_OK;
  };
  auto resolved = [&](const ftk_tuning_t& t) {
    p->tune = t;
    return std::make_pair(step3_waves(p), step1_zblk(p));
  };
  if (rc == FTK_OK) rc = time_one(best_t, &best_ms);
  if (rc == FTK_OK) {
    const int waves[] = {4, 8, 16};
    const int zblks[] = {64, 128};
    const int wgs[] = {1024, 16384};
    for (int pass = 0; pass < 3 && rc == FTK_OK; ++pass) {
      std::vector<ftk_tuning_t> cands;
      if (pass == 0)
        for (int v : waves) {
          ftk_tuning_t t = best_t;
          t.step3_waves = v;
          cands.push_back(t);
        }
      if (pass == 1)
        for (int v : zblks) {
          ftk_tuning_t t = best_t;
          t.step1_zblk = v;
          cands.push_back(t);
        }
      if (pass == 2)
        for (int v : wgs) {
          ftk_tuning_t t = best_t;
          t.step1_wgs = v;
          cands.push_back(t);
        }
      for (const auto& t : cands) {
        if (pass < 2 && resolved(t) == resolved(best_t)) continue;
        if (pass == 2 && t.step1_wgs == best_t.step1_wgs) continue;
        float ms = 0.f;
        rc = time_one(t, &ms);
        if (rc != FTK_OK) break;
        if (ms < 0.97f * best_ms) {  // a clear win only
          best_ms = ms;
          best_t = t;
        }
      }
    }
  }
  restore();
  if (rc != FTK_OK) return rc;
  b->tune[i] = best_t;
  std::lock_guard<std::mutex> g(g_tune_mu);
  tune_cache_store_locked(key, best_t);
  return FTK_OK;
}

int check_stack(const ftk_stack& st, int idx) {
  const std::string at = "ftk_batch_create: stack " + std::to_string(idx) + ": ";
  if (!st.plan) return fail(FTK_EINVAL, at + "NULL plan");
  if (st.nA < 0 || st.nB < 0) return fail(FTK_EINVAL, at + "negative count");
  if (st.plan->N <= 0) return fail(FTK_ESTATE, at + "shifts not set");
  if (st.nA == 0 || st.nB == 0) return FTK_OK;
  if (!st.images || !st.templates) return fail(FTK_EINVAL, at + "NULL images");
  if (!st.X && !st.best) return fail(FTK_EINVAL, at + "X and best are both NULL");
  return FTK_OK;
}

}  // namespace

extern "C" {

int ftk_batch_create(ftk_batch** out, const ftk_stack* stacks, int count, int lanes, int flags, void* stream) {
  if (!out) return fail(FTK_EINVAL, "ftk_batch_create: out is NULL");
  *out = nullptr;
  if (count < 0 || (count > 0 && !stacks)) return fail(FTK_EINVAL, "ftk_batch_create: invalid stack array");
  if (lanes < 1 || lanes > 4) return fail(FTK_EINVAL, "ftk_batch_create: lanes must be 1 to 4");
  if (flags & ~(FTK_BATCH_GRAPH | FTK_BATCH_AUTOTUNE)) return fail(FTK_EINVAL, "ftk_batch_create: unknown flag");
  for (int i = 0; i < count; ++i) {
    const int rc = check_stack(stacks[i], i);
    if (rc != FTK_OK) return rc;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  ftk_batch* b = nullptr;
  try {
    b = new ftk_batch();
    b->lanes = lanes;
    b->flags = flags;
    // cost order, largest first; ties keep the caller's order
    std::vector<int> order(count);
    std::vector<double> cost(count);
    for (int i = 0; i < count; ++i) {
      order[i] = i;
      cost[i] = stack_gflop(stacks[i]);
    }
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    std::vector<double> load(lanes, 0.0);
    for (int i : order) {
      b->stacks.push_back(stacks[i]);
      b->cost.push_back(cost[i]);
      b->tune.push_back(stacks[i].plan->tune);
      const int l = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
      b->lane.push_back(l);
      load[l] += cost[i];
    }
    b->ws.resize(lanes);
  } catch (const std::bad_alloc&) {
    delete b;
    return fail(FTK_ENOMEM, "ftk_batch_create: host allocation failed");
  }
  hipError_t e = hipSuccess;
  for (int l = 1; l < lanes && e == hipSuccess; ++l) {
    hipStream_t ls = nullptr;
    if ((e = hipStreamCreateWithFlags(&ls, hipStreamNonBlocking)) == hipSuccess) b->streams.push_back(ls);
    hipEvent_t ev = nullptr;
    if (e == hipSuccess && (e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) == hipSuccess)
      b->ev_join.push_back(ev);
  }
  if (e == hipSuccess && lanes > 1) e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
  if (e != hipSuccess) {
    b->release();
    delete b;
    return hip_fail(e, "ftk_batch_create: streams");
  }
  int rc = FTK_OK;
  if (flags & FTK_BATCH_AUTOTUNE) {
    // the slices run in lane 0's workspace before it is sized for the batch
    const auto t0 = std::chrono::steady_clock::now();
    Needs need0;
    size_t max_slice = 1;
    for (const auto& st : b->stacks) {
      if (st.nA == 0 || st.nB == 0) continue;
      const int snB = std::min(st.nB, 8192);
      const int snA = std::min(st.nA, std::max(1, 8192 / snB));
      ftk_plan* p = st.plan;
      needs_max(need0, plan_needs(p, snA, snB, true));
      max_slice = std::max(max_slice, static_cast<size_t>(snA) * snB);
    }
    if ((e = ensure_all(b->ws[0], need0)) != hipSuccess || (e = b->tune_best.ensure(max_slice * sizeof(ftk_pose))) != hipSuccess)
      rc = fail(FTK_ENOMEM, "ftk_batch_create: autotune workspace");
    for (size_t i = 0; i < b->stacks.size() && rc == FTK_OK; ++i) {
      ftk_plan* p = b->stacks[i].plan;
      const ftk_tuning_t keep = p->tune;
      p->tune = b->tune[i];
      rc = autotune_stack(b, i, s);
      p->tune = keep;
    }
    b->tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  // size every lane's workspace for its largest stack, so runs allocate nothing
  for (int l = 0; l < lanes && rc == FTK_OK; ++l) {
    Needs need;
    for (size_t i = 0; i < b->stacks.size(); ++i) {
      if (b->lane[i] != l) continue;
      const ftk_stack& st = b->stacks[i];
      ftk_plan* p = st.plan;
      const ftk_tuning_t keep = p->tune;
      p->tune = b->tune[i];
      needs_max(need, plan_needs(p, st.nA, st.nB, true));
      p->tune = keep;
    }
    if (ensure_all(b->ws[l], need) != hipSuccess) rc = fail(FTK_ENOMEM, "ftk_batch_create: workspace");
  }
  if (rc != FTK_OK) {
    (void)hipStreamSynchronize(s);
    b->release();
    delete b;
    return rc;
  }
  *out = b;
  return FTK_OK;
}

int ftk_batch_run(ftk_batch* b, void* stream) {
  if (!b) return fail(FTK_EINVAL, "ftk_batch_run: NULL batch");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!(b->flags & FTK_BATCH_GRAPH)) return enqueue(b, s, false);
  hipError_t e;
  if (!b->exec) {
    if (!s) return fail(FTK_EINVAL, "ftk_batch_run: graph capture needs a stream other than the null stream");
    if ((e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      return hip_fail(e, "ftk_batch_run: begin capture");
    const int rc = enqueue(b, s, true);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s, &g);
    if (rc != FTK_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "ftk_batch_run: end capture");
    size_t nodes = 0;
    (void)hipGraphGetNodes(g, nullptr, &nodes);
    hipGraphExec_t x = nullptr;
    if ((e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0)) != hipSuccess) {
      (void)hipGraphDestroy(g);
      return hip_fail(e, "ftk_batch_run: instantiate");
    }
    b->graph = g;
    b->exec = x;
    b->graph_nodes = static_cast<int>(nodes);
  }
  if ((e = hipGraphLaunch(b->exec, s)) != hipSuccess) return hip_fail(e, "ftk_batch_run: graph launch");
  return FTK_OK;
}

int ftk_batch_info(const ftk_batch* b, ftk_batch_info_t* out) {
  if (!b || !out) return fail(FTK_EINVAL, "ftk_batch_info: NULL argument");
  out->count = static_cast<int>(b->stacks.size());
  out->lanes = b->lanes;
  out->graph_nodes = b->graph_nodes;
  size_t bytes = 0;
  for (const auto& w : b->ws) bytes += w.bytes();
  out->workspace_bytes = bytes;
  double c = 0.0;
  for (double x : b->cost) c += x;
  out->cost_gflop = c;
  out->tune_ms = b->tune_ms;
  return FTK_OK;
}

void ftk_batch_destroy(ftk_batch* b) {
  if (!b) return;
  b->release();
  delete b;
}

}  // extern "C"
