// Uneven batches (one persistent launch, optionally replayed from a hipGraph)
// and the autotuner.
//
// Batching follows the paper's batch-size study (Ablation Study - Batch
// Size): many independent polynomials share one launch so that small sizes
// still fill the machine. Here every job is planned on its own (its pass
// split and engine come from the context, tuned or default), all passes of
// all jobs go into one table, and persistent grids of resident workgroups
// pull (pass, workgroup) items from a device queue: one launch per stage (the
// first passes of all jobs, then the second passes, ...), all captured in one
// hipGraph by ntt_batch_graph. The launch boundary orders a job's passes.
// (A single launch whose items wait on per-pass counters needs an
// agent-scope release and acquire around every item; those fences write
// back and invalidate the L2 of the workgroup's XCD each time, and cost more
// than the stages' launch boundaries.)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "frntt_internal.hpp"

namespace frntt {

namespace {

struct BatchBuild {
  std::vector<PassParams> passes;
  std::vector<int64_t> pass_wgs;
  std::vector<int64_t> item_pass;
  std::vector<int64_t> item_wg;
  std::vector<int> item_cnt;
  std::vector<int64_t> stage_begin;  // first item of each stage, then the item count
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct DevLayout {
  size_t tables, passes, item_pass, item_wg, item_cnt, counters, total;
};

DevLayout layout_for(size_t np, size_t ni, size_t n_stages) {
  DevLayout L;
  size_t off = 0;
  L.tables = off;
  off = align256(off + sizeof(DevTables));
  L.passes = off;
  off = align256(off + np * sizeof(PassParams));
  L.item_pass = off;
  off = align256(off + ni * sizeof(int64_t));
  L.item_wg = off;
  off = align256(off + ni * sizeof(int64_t));
  L.item_cnt = off;
  off = align256(off + ni * sizeof(int));
  L.counters = off;  // queue head of each stage
  off = align256(off + n_stages * sizeof(unsigned int));
  L.total = off;
  return L;
}

// Validate the jobs, fix the algorithm and plan of each (read once, so that a
// concurrent plan change cannot make the scratch layout and the passes
// disagree) unless `given` supplies them, and compute the scratch needs
// (bytes, per job offset).
int check_jobs(frntt_ctx* ctx, const frntt_job* jobs, int n_jobs, std::vector<size_t>* scratch_off,
               size_t* scratch_total, std::vector<JobPlan>* plans, const JobPlan* given = nullptr) {
  if (!ctx || n_jobs < 0 || (n_jobs > 0 && !jobs)) return FRNTT_EINVAL;
  scratch_off->assign((size_t)n_jobs, 0);
  plans->assign((size_t)n_jobs, JobPlan{});
  size_t tot = 0;
  for (int j = 0; j < n_jobs; ++j) {
    const frntt_job& jb = jobs[j];
    if (!jb.data) return FRNTT_EINVAL;
    if (jb.kind < FRNTT_FWD || jb.kind > FRNTT_COSET_INV) return FRNTT_EINVAL;
    if (jb.log_n < 0 || jb.log_n > ctx->max_log_n) return FRNTT_ERANGE;
    if (((uintptr_t)jb.data & 31) != 0) return FRNTT_EALIGN;
    if (jb.log_n == 0) continue;
    JobPlan& jp = (*plans)[(size_t)j];
    if (given) jp = given[j];
    else resolve_plan(ctx, FRNTT_ALGO_AUTO, jb.log_n, &jp.algo, &jp.plan);
    if (check_plan_valid(jp.plan, jb.log_n) != FRNTT_OK) return FRNTT_EINVAL;
    (*scratch_off)[j] = tot;
    tot += scratch_bytes_for(jb.log_n, 1, jp.plan.n_pass);
  }
  *scratch_total = tot;
  return FRNTT_OK;
}

// Tiles (workgroups of one pass) per work item.
constexpr int64_t kTilesPerItem = 4;

int build_batch(frntt_ctx* ctx, const frntt_job* jobs, int n_jobs, const std::vector<void*>& scratch,
                const std::vector<JobPlan>& plans, BatchBuild* B, bool capturing) {
  std::vector<std::vector<int>> job_passes((size_t)n_jobs);
  int max_pass = 0;
  for (int j = 0; j < n_jobs; ++j) {
    const frntt_job& jb = jobs[j];
    if (jb.log_n == 0) continue;
    const int algo = plans[(size_t)j].algo;
    const Plan& plan = plans[(size_t)j].plan;
    std::vector<PassParams> pp;
    if (plan.n_pass > 1 && !scratch[(size_t)j]) return FRNTT_EINVAL;
    int rc = build_passes(ctx, plan, jb.log_n, 1, jb.kind, jb.data, scratch[(size_t)j], &pp, algo, capturing);
    if (rc) return rc;
    for (PassParams& P : pp) {
      P.xcd_remap = 0;  // the queue decides placement
      const int idx = (int)B->passes.size();
      B->passes.push_back(P);
      B->pass_wgs.push_back(P.wg_count);
      job_passes[(size_t)j].push_back(idx);
    }
    max_pass = std::max(max_pass, (int)pp.size());
  }
  // items in pass order: every first pass, then every second pass, ...
  // (largest jobs first inside a stage, so long items start early)
  std::vector<int> order((size_t)n_jobs);
  for (int j = 0; j < n_jobs; ++j) order[(size_t)j] = j;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return jobs[a].log_n > jobs[b].log_n; });
  for (int s = 0; s < max_pass; ++s) {
    B->stage_begin.push_back((int64_t)B->item_pass.size());
    for (int j : order) {
      if ((int)job_passes[(size_t)j].size() <= s) continue;
      const int p = job_passes[(size_t)j][(size_t)s];
      // items of up to kTilesPerItem consecutive tiles: a workgroup runs
      // them in one call (one set of register saves, one staging of the
      // constant blocks)
      const int64_t wgs = B->pass_wgs[(size_t)p];
      for (int64_t w = 0; w < wgs; w += kTilesPerItem) {
        B->item_pass.push_back(p);
        B->item_wg.push_back(w);
        B->item_cnt.push_back((int)std::min<int64_t>(kTilesPerItem, wgs - w));
      }
    }
  }
  B->stage_begin.push_back((int64_t)B->item_pass.size());
  return FRNTT_OK;
}

void fill_host(uint8_t* h, const DevLayout& L, const BatchBuild& B, const DevTables& T) {
  const size_t np = B.passes.size(), ni = B.item_pass.size();
  std::memcpy(h + L.tables, &T, sizeof(DevTables));
  std::memcpy(h + L.passes, B.passes.data(), np * sizeof(PassParams));
  std::memcpy(h + L.item_pass, B.item_pass.data(), ni * sizeof(int64_t));
  std::memcpy(h + L.item_wg, B.item_wg.data(), ni * sizeof(int64_t));
  std::memcpy(h + L.item_cnt, B.item_cnt.data(), ni * sizeof(int));
  std::memset(h + L.counters, 0, (B.stage_begin.size() - 1) * sizeof(unsigned int));
}

BatchParams params_for(uint8_t* d, const DevLayout& L, const BatchBuild& B) {
  BatchParams P;
  P.tables = (const DevTables*)(d + L.tables);
  P.passes = (const PassParams*)(d + L.passes);
  P.item_pass = (const int64_t*)(d + L.item_pass);
  P.item_wg = (const int64_t*)(d + L.item_wg);
  P.item_cnt = (const int*)(d + L.item_cnt);
  P.item_begin = 0;
  P.item_end = 0;
  P.queue = (unsigned int*)(d + L.counters);
  return P;
}

// Zero the stage counters, then launch one persistent grid per stage (all
// graph-capturable: kernels only).
int launch_batch(frntt_ctx* ctx, const BatchParams& P0, const std::vector<int64_t>& stage_begin,
                 hipStream_t stream) {
  const int64_t n_stages = (int64_t)stage_begin.size() - 1;
  if (n_stages <= 0) return FRNTT_OK;
  hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)((n_stages + 255) / 256)), dim3(256), 0, stream, P0.queue,
                     n_stages);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_hip_error(ctx, e);
  for (int64_t s = 0; s < n_stages; ++s) {
    BatchParams P = P0;
    P.item_begin = stage_begin[(size_t)s];
    P.item_end = stage_begin[(size_t)s + 1];
    P.queue = P0.queue + s;
    // one resident workgroup per CU (LDS bound); never more than there are items
    const int64_t grid = std::min<int64_t>(P.item_end - P.item_begin, (int64_t)ctx->cu_count);
    if (grid <= 0) continue;
    hipLaunchKernelGGL(ntt_batch_kernel, dim3((unsigned)grid), dim3(kMfmaThreads), 0, stream, P);
    e = hipGetLastError();
    if (e != hipSuccess) return set_hip_error(ctx, e);
  }
  return FRNTT_OK;
}

bool same_plan(const JobPlan& a, const JobPlan& b) {
  if (a.algo != b.algo || a.plan.n_pass != b.plan.n_pass || a.plan.log_t != b.plan.log_t) return false;
  for (int p = 0; p < 4; ++p) {
    if (a.plan.pass_log[p] != b.plan.pass_log[p] || a.plan.nlev[p] != b.plan.nlev[p] ||
        a.plan.lev_set[p] != b.plan.lev_set[p])
      return false;
    for (int l = 0; l < kMaxLevels; ++l)
      if (a.plan.lev_log[p][l] != b.plan.lev_log[p][l]) return false;
  }
  return true;
}

// The captured graph of an entry serves a call with the same job list whose
// jobs still resolve to the same form and plan.
bool same_jobs(const GraphEntry& g, const frntt_job* b, const std::vector<JobPlan>& plans, int n) {
  if ((int)g.jobs.size() != n) return false;
  for (int i = 0; i < n; ++i)
    if (g.jobs[(size_t)i].data != b[i].data || g.jobs[(size_t)i].log_n != b[i].log_n ||
        g.jobs[(size_t)i].kind != b[i].kind || !same_plan(g.plans[(size_t)i], plans[(size_t)i]))
      return false;
  return true;
}

}  // namespace

static int batch_launch_common(frntt_ctx* ctx, const frntt_job* jobs, int n_jobs,
                               const std::vector<void*>& scratch, const std::vector<JobPlan>& plans,
                               hipStream_t stream);

int batch_impl(frntt_ctx* ctx, const frntt_job* jobs, int n_jobs, hipStream_t stream) {
  std::vector<size_t> soff;
  std::vector<JobPlan> plans;
  size_t stot = 0;
  int rc = check_jobs(ctx, jobs, n_jobs, &soff, &stot, &plans);
  if (rc) return rc;
  if (n_jobs == 0) return FRNTT_OK;
  // the descriptor upload allocates and waits on the host: not capturable
  // (ntt_batch_graph is the graph form)
  if (stream_capturing(stream)) return FRNTT_ESTATE;
  void* base = nullptr;
  rc = get_scratch(ctx, stream, stot, &base);
  if (rc) return rc;
  std::vector<void*> scratch((size_t)n_jobs, nullptr);
  for (int j = 0; j < n_jobs; ++j) scratch[(size_t)j] = base ? (uint8_t*)base + soff[(size_t)j] : nullptr;
  return batch_launch_common(ctx, jobs, n_jobs, scratch, plans, stream);
}

// As batch_impl with caller-provided scratch and plan per job (scratch NULL
// for single-pass plans); used by the server, whose request buffers carry
// their scratch, sized for the plan fixed when the request was submitted.
int batch_impl_ws(frntt_ctx* ctx, const frntt_job* jobs, void* const* scratch_in, const JobPlan* given, int n_jobs,
                  hipStream_t stream) {
  std::vector<size_t> soff;
  std::vector<JobPlan> plans;
  size_t stot = 0;
  int rc = check_jobs(ctx, jobs, n_jobs, &soff, &stot, &plans, given);
  if (rc) return rc;
  if (n_jobs == 0) return FRNTT_OK;
  std::vector<void*> scratch(scratch_in, scratch_in + n_jobs);
  return batch_launch_common(ctx, jobs, n_jobs, scratch, plans, stream);
}

static int batch_launch_common(frntt_ctx* ctx, const frntt_job* jobs, int n_jobs,
                               const std::vector<void*>& scratch, const std::vector<JobPlan>& plans,
                               hipStream_t stream) {
  int rc;
  BatchBuild B;
  rc = build_batch(ctx, jobs, n_jobs, scratch, plans, &B, false);
  if (rc) return rc;
  if (B.item_pass.empty()) return FRNTT_OK;
  const DevLayout L = layout_for(B.passes.size(), B.item_pass.size(), B.stage_begin.size() - 1);
  std::lock_guard<std::mutex> lk(ctx->mu);
  BatchBuffers& bb = ctx->batch_bufs[stream];
  // the previous batch on this stream may still read the buffers: wait for
  // its upload to finish before reusing the host staging, and keep the device
  // buffer stream-ordered
  if (bb.event) {
    hipError_t e = hipEventSynchronize(bb.event);
    if (e != hipSuccess) return set_hip_error(ctx, e);
  } else if (hipEventCreateWithFlags(&bb.event, hipEventDisableTiming) != hipSuccess) {
    return FRNTT_EHIP;
  }
  if (bb.host_bytes < L.total) {
    if (bb.host) hipHostFree(bb.host);
    bb.host = nullptr;
    bb.host_bytes = 0;
    if (hipHostMalloc(&bb.host, L.total, 0) != hipSuccess) return FRNTT_ENOMEM;
    bb.host_bytes = L.total;
  }
  if (bb.dev_bytes < L.total) {
    if (bb.dev) {
      hipError_t e = hipStreamSynchronize(stream);
      if (e != hipSuccess) return set_hip_error(ctx, e);
      hipFree(bb.dev);
    }
    bb.dev = nullptr;
    bb.dev_bytes = 0;
    if (hipMalloc(&bb.dev, L.total) != hipSuccess) return FRNTT_ENOMEM;
    bb.dev_bytes = L.total;
  }
  fill_host((uint8_t*)bb.host, L, B, ctx->tables);
  hipError_t e = hipMemcpyAsync(bb.dev, bb.host, L.total, hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return set_hip_error(ctx, e);
  e = hipEventRecord(bb.event, stream);
  if (e != hipSuccess) return set_hip_error(ctx, e);
  const BatchParams P = params_for((uint8_t*)bb.dev, L, B);
  return launch_batch(ctx, P, B.stage_begin, stream);
}

int batch_graph_impl(frntt_ctx* ctx, const frntt_job* jobs, int n_jobs, hipStream_t stream) {
  std::vector<size_t> soff;
  std::vector<JobPlan> plans;
  size_t stot = 0;
  int rc = check_jobs(ctx, jobs, n_jobs, &soff, &stot, &plans);
  if (rc) return rc;
  if (n_jobs == 0) return FRNTT_OK;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (GraphEntry& g : ctx->graphs)
      if (same_jobs(g, jobs, plans, n_jobs)) {
        hipError_t e = hipGraphLaunch(g.exec, stream);
        return set_hip_error(ctx, e);
      }
  }
  // a new job list allocates and captures: not possible inside a capture
  if (stream_capturing(stream)) return FRNTT_ESTATE;
  // new entry: dedicated scratch and descriptors, captured once
  GraphEntry g;
  g.jobs.assign(jobs, jobs + n_jobs);
  g.plans = plans;
  hipError_t e;
  if (stot) {
    e = hipMalloc(&g.scratch, stot);
    if (e != hipSuccess) return FRNTT_ENOMEM;
  }
  BatchBuild B;
  std::vector<void*> scratch((size_t)n_jobs, nullptr);
  for (int j = 0; j < n_jobs; ++j) scratch[(size_t)j] = g.scratch ? (uint8_t*)g.scratch + soff[(size_t)j] : nullptr;
  rc = build_batch(ctx, jobs, n_jobs, scratch, plans, &B, false);
  if (rc || B.item_pass.empty()) {  // nothing to run: every job has log_n 0
    if (g.scratch) hipFree(g.scratch);
    return rc;
  }
  const DevLayout L = layout_for(B.passes.size(), B.item_pass.size(), B.stage_begin.size() - 1);
  std::vector<uint8_t> host(L.total);
  fill_host(host.data(), L, B, ctx->tables);
  e = hipMalloc(&g.dev_buf, L.total);
  if (e != hipSuccess) {
    if (g.scratch) hipFree(g.scratch);
    return FRNTT_ENOMEM;
  }
  e = hipMemcpy(g.dev_buf, host.data(), L.total, hipMemcpyHostToDevice);
  hipStream_t cap = nullptr;
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    const BatchParams P = params_for((uint8_t*)g.dev_buf, L, B);
    rc = launch_batch(ctx, P, B.stage_begin, cap);
    hipError_t e2 = hipStreamEndCapture(cap, &g.graph);
    if (rc == FRNTT_OK && e2 != hipSuccess) e = e2;
    if (rc != FRNTT_OK && e == hipSuccess) e = hipErrorUnknown;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
  if (cap) hipStreamDestroy(cap);
  if (e != hipSuccess) {
    if (g.exec) hipGraphExecDestroy(g.exec);
    if (g.graph) hipGraphDestroy(g.graph);
    hipFree(g.dev_buf);
    if (g.scratch) hipFree(g.scratch);
    return set_hip_error(ctx, e);
  }
  e = hipGraphLaunch(g.exec, stream);
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->graphs.push_back(g);
  return set_hip_error(ctx, e);
}

// ---------------------------------------------------------------- tuning

namespace {

void candidate_splits(int log_n, std::vector<std::vector<int>>* out) {
  out->clear();
  if (log_n <= 12) out->push_back({log_n});
  for (int a = 1; a <= 12; ++a) {
    const int b = log_n - a;
    if (b >= 1 && b <= 12 && a >= 4 && b >= 4) out->push_back({a, b});
  }
  if (log_n >= 15)
    for (int a = 5; a <= 12; ++a)
      for (int b = 5; b <= 12; ++b) {
        const int c = log_n - a - b;
        if (c >= 5 && c <= 12 && std::abs(a - b) <= 2 && std::abs(b - c) <= 2) out->push_back({a, b, c});
      }
}

// The level orders the tuner tries for a pass radix 2^l (each has a plan
// kernel; the first is the default split), or none.
const std::vector<std::vector<int>>& level_orders(int l) {
  static const std::vector<std::vector<int>> none, o10{{4, 3, 3}, {3, 4, 3}, {3, 3, 4}},
      o11{{4, 4, 3}, {3, 4, 4}, {4, 3, 4}};
  return l == 10 ? o10 : l == 11 ? o11 : none;
}

}  // namespace

int tune_impl(frntt_ctx* ctx, int log_n, int batch, int* best_algo, int* best_passes, float* best_ms,
              hipStream_t stream) {
  if (!ctx || batch < 1) return FRNTT_EINVAL;
  if (log_n < 1 || log_n > ctx->max_log_n) return FRNTT_ERANGE;
  const size_t count = (size_t)batch << log_n;
  void* buf = nullptr;
  if (hipMalloc(&buf, count * 32) != hipSuccess) return FRNTT_ENOMEM;
  int rc = frntt_generate(ctx, buf, 7, 0, 0, count, stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  std::vector<std::vector<int>> splits;
  candidate_splits(log_n, &splits);
  TuneEntry best;
  best.ms = 1e30f;
  bool found = false;
  const std::vector<int> tables_before = pass_table_keys(ctx);
  // candidates run with explicit plans: the context's overrides and tuned
  // plans are not touched until the winner is stored under ctx->mu
  for (int algo = FRNTT_ALGO_BUTTERFLY; rc == FRNTT_OK && algo <= FRNTT_ALGO_FOURSTEP_MFMA; ++algo) {
    for (const auto& sp : splits) {
      // the matrix form also tries every level order of its 2^10 and 2^11 passes
      std::vector<Plan> cands;
      Plan base;
      base.n_pass = (int)sp.size();
      for (int i = 0; i < base.n_pass; ++i) base.pass_log[i] = sp[(size_t)i];
      cands.push_back(base);
      if (algo == FRNTT_ALGO_FOURSTEP_MFMA)
        for (int p = 0; p < base.n_pass; ++p) {
          const std::vector<std::vector<int>>& orders = level_orders(base.pass_log[p]);
          if (orders.empty()) continue;
          std::vector<Plan> grown;
          for (const Plan& c : cands)
            for (const auto& o : orders) {
              Plan g = c;
              g.lev_set[p] = true;
              g.nlev[p] = (int)o.size();
              for (int i = 0; i < (int)o.size(); ++i) g.lev_log[p][i] = o[(size_t)i];
              grown.push_back(g);
            }
          cands.swap(grown);
        }
      for (const Plan& cand : cands) {
        // warm-up, then the median of 5
        rc = transform_plan(ctx, buf, log_n, batch, FRNTT_FWD, algo, cand, stream, nullptr, 0);
        if (rc) break;
        float t[5];
        for (int r = 0; r < 5 && rc == FRNTT_OK; ++r) {
          hipEventRecord(e0, stream);
          rc = transform_plan(ctx, buf, log_n, batch, FRNTT_FWD, algo, cand, stream, nullptr, 0);
          hipEventRecord(e1, stream);
          hipEventSynchronize(e1);
          hipEventElapsedTime(&t[r], e0, e1);
        }
        if (rc) break;
        std::sort(t, t + 5);
        if (t[2] < best.ms) {
          best = TuneEntry{};
          best.ms = t[2];
          best.algo = algo;
          best.n_pass = cand.n_pass;
          for (int i = 0; i < 4; ++i) {
            best.pass_log[i] = i < cand.n_pass ? cand.pass_log[i] : 0;
            best.nlev[i] = cand.lev_set[i] ? cand.nlev[i] : 0;
            for (int j = 0; j < 3; ++j) best.lev_log[i][j] = cand.lev_set[i] ? cand.lev_log[i][j] : 0;
          }
          found = true;
        }
      }
      if (rc) break;
    }
  }
  hipStreamSynchronize(stream);
  if (found) {
    // release the pass-twiddle tables that only the losing candidates built
    Plan chosen;
    chosen.n_pass = best.n_pass;
    for (int i = 0; i < 4; ++i) chosen.pass_log[i] = best.pass_log[i];
    release_tuning_tables(ctx, tables_before, chosen);
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipFree(buf);
  if (rc) return rc;
  if (!found) return FRNTT_EINVAL;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->tuned[log_n] = best;
    ctx->has_tuned[log_n] = true;
  }
  if (best_algo) *best_algo = best.algo;
  if (best_passes) *best_passes = best.n_pass;
  if (best_ms) *best_ms = best.ms;
  return FRNTT_OK;
}

int tune_save_impl(const frntt_ctx* ctx, const char* path) {
  if (!ctx || !path) return FRNTT_EINVAL;
  FILE* f = std::fopen(path, "w");
  if (!f) return FRNTT_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  std::fprintf(f, "{\"format\": \"frntt-tune-1\", \"entries\": [");
  bool first = true;
  for (int l = 0; l <= 28; ++l) {
    if (!ctx->has_tuned[l]) continue;
    const TuneEntry& t = ctx->tuned[l];
    std::fprintf(f, "%s\n  {\"log_n\": %d, \"algo\": %d, \"passes\": [", first ? "" : ",", l, t.algo);
    for (int i = 0; i < t.n_pass; ++i) std::fprintf(f, "%s%d", i ? ", " : "", t.pass_log[i]);
    std::fprintf(f, "], \"ms\": %.6f, \"levels\": [", t.ms);
    for (int i = 0; i < t.n_pass; ++i) {
      std::fprintf(f, "%s[", i ? ", " : "");
      for (int j = 0; j < t.nlev[i]; ++j) std::fprintf(f, "%s%d", j ? ", " : "", t.lev_log[i][j]);
      std::fprintf(f, "]");
    }
    std::fprintf(f, "]}");
    first = false;
  }
  std::fprintf(f, "\n]}\n");
  std::fclose(f);
  return FRNTT_OK;
}

int tune_load_impl(frntt_ctx* ctx, const char* path) {
  if (!ctx || !path) return FRNTT_EINVAL;
  FILE* f = std::fopen(path, "r");
  if (!f) return FRNTT_EINVAL;
  std::string s;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, n);
  std::fclose(f);
  if (s.find("\"frntt-tune-1\"") == std::string::npos) return FRNTT_EINVAL;
  size_t pos = 0;
  int loaded = 0;
  while ((pos = s.find("{\"log_n\":", pos)) != std::string::npos) {
    int l = -1, algo = 0, p[4] = {0, 0, 0, 0};
    float ms = 0;
    const char* c = s.c_str() + pos;
    int np = std::sscanf(c, "{\"log_n\": %d, \"algo\": %d, \"passes\": [%d, %d, %d, %d", &l, &algo, &p[0], &p[1],
                         &p[2], &p[3]);
    if (np < 3 || l < 1 || l > 28 || algo < 1 || algo > 2) return FRNTT_EINVAL;
    const size_t close = s.find(']', pos);
    const size_t msp = s.find("\"ms\":", pos);
    if (msp != std::string::npos) std::sscanf(s.c_str() + msp, "\"ms\": %f", &ms);
    TuneEntry t;
    t.algo = algo;
    t.n_pass = np - 2;
    // count the entries actually inside the brackets
    int cnt = 1;
    for (size_t i = s.find('[', pos); i < close; ++i) cnt += s[i] == ',';
    t.n_pass = std::min(cnt, 4);
    for (int i = 0; i < 4; ++i) t.pass_log[i] = i < t.n_pass ? p[i] : 0;
    t.ms = ms;
    Plan check;
    check.n_pass = t.n_pass;
    for (int i = 0; i < 4; ++i) check.pass_log[i] = t.pass_log[i];
    if (check_plan_valid(check, l) != FRNTT_OK) return FRNTT_EINVAL;
    // optional level splits: "levels": [[4, 3, 3], [], ...], one list per pass
    const size_t next = s.find("{\"log_n\":", pos + 1);
    const size_t lv = s.find("\"levels\":", pos);
    if (lv != std::string::npos && lv < next) {
      size_t i = s.find('[', lv) + 1;
      for (int pass = 0; pass < t.n_pass; ++pass) {
        i = s.find('[', i);
        const size_t end = s.find(']', i);
        if (i == std::string::npos || end == std::string::npos || (next != std::string::npos && end > next))
          return FRNTT_EINVAL;
        int v[3] = {0, 0, 0};
        const int got = std::sscanf(s.c_str() + i, "[%d, %d, %d", &v[0], &v[1], &v[2]);
        const int nl = end == i + 1 ? 0 : std::max(got, 0);
        int sum = 0;
        for (int j = 0; j < nl; ++j) sum += v[j];
        if (nl > 0 && sum != t.pass_log[pass]) return FRNTT_EINVAL;
        t.nlev[pass] = nl;
        for (int j = 0; j < 3; ++j) t.lev_log[pass][j] = j < nl ? v[j] : 0;
        i = end + 1;
      }
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->tuned[l] = t;
    ctx->has_tuned[l] = true;
    ++loaded;
    pos = close;
  }
  return loaded > 0 ? FRNTT_OK : FRNTT_EINVAL;
}

}  // namespace frntt

using namespace frntt;

extern "C" {

int ntt_batch(frntt_ctx* ctx, const frntt_job* jobs, int n_jobs, void* stream) {
  return batch_impl(ctx, jobs, n_jobs, (hipStream_t)stream);
}

int ntt_batch_graph(frntt_ctx* ctx, const frntt_job* jobs, int n_jobs, void* stream) {
  return batch_graph_impl(ctx, jobs, n_jobs, (hipStream_t)stream);
}

int frntt_tune(frntt_ctx* ctx, int log_n, int batch, int* best_algo, int* best_passes, float* best_ms,
               void* stream) {
  return tune_impl(ctx, log_n, batch, best_algo, best_passes, best_ms, (hipStream_t)stream);
}

int frntt_tune_save(const frntt_ctx* ctx, const char* path) { return tune_save_impl(ctx, path); }

int frntt_tune_load(frntt_ctx* ctx, const char* path) { return tune_load_impl(ctx, path); }

}  // extern "C"
