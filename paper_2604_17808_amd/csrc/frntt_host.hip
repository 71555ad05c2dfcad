// Host side of libfrntt: contexts, plans, scratch, launches and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>

#include "frntt_internal.hpp"

namespace frntt {

int build_tables(frntt_ctx* ctx);

int set_hip_error(const frntt_ctx* ctx, hipError_t e) {
  if (ctx) ctx->last_hip_error = (int)e;
  return e == hipSuccess ? FRNTT_OK : FRNTT_EHIP;
}

// RAII guard that makes `dev` current and restores the caller's device.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) hipSetDevice(prev);
  }
};

// ------------------------------------------------------------------ plans

// Split a pass radix 2^l into levels of at most 2^max_m, as even as possible.
// Returns the level count; writes the levels only if they fit kMaxLevels.
static int split_levels(int l, int max_m, int* out) {
  int n = (l + max_m - 1) / max_m;
  if (n < 1) n = 1;
  if (n > kMaxLevels) return n;
  int base = l / n, extra = l % n;
  for (int i = 0; i < n; ++i) out[i] = base + (i < extra ? 1 : 0);
  return n;
}

// Can level m of a pass with 2^log_t staged elements run on MFMA? The
// matrix form runs on full 4096-element tiles only: each of the 8 waves of a
// workgroup takes the same number TPW = 2^(4 - m) of 32-vector tiles, so that
// a wave's data fragments take 64 registers.
bool mfma_level_ok(int m, int log_t) { return m >= 1 && m <= 4 && log_t == kMaxLogT; }

// Levels of pass p for the MFMA engine: radices of at most 16, as even as
// possible (the smallest first when there are three), with a plan kernel for
// the split. Returns false if the pass cannot
// run on MFMA (a tile below 4096 elements); it then runs on the butterfly
// engine.
static bool plan_levels(Plan& plan, int p, int log_t_pass) {
  const int l = plan.pass_log[p];
  int levs[kMaxLevels];
  int n = split_levels(l, 4, levs);
  if (n == 3) {
    // three levels: the smallest radix first ([3,4,3] for 2^10, [3,4,4] for
    // 2^11), measured 1-2% faster than the largest first
    const int last = levs[2];
    levs[2] = levs[1];
    levs[1] = levs[0];
    levs[0] = last;
  }
  if (plan.lev_set[p] && log_t_pass == kMaxLogT) {
    // the requested split, if it covers the pass and has a plan kernel
    int sum = 0;
    for (int i = 0; i < plan.nlev[p] && i < 3; ++i) sum += plan.lev_log[p][i];
    if (plan.nlev[p] >= 1 && plan.nlev[p] <= 3 && sum == l && mfma_plan_kernel(plan.nlev[p], plan.lev_log[p])) {
      n = plan.nlev[p];
      for (int i = 0; i < n; ++i) levs[i] = plan.lev_log[p][i];
    }
  }
  bool ok = n <= 3;
  for (int i = 0; i < n && ok; ++i) ok = mfma_level_ok(levs[i], log_t_pass);
  ok = ok && mfma_plan_kernel(n, levs) != nullptr;
  plan.nlev[p] = ok ? n : 0;
  for (int i = 0; i < kMaxLevels; ++i) plan.lev_log[p][i] = ok && i < n ? levs[i] : 0;
  return ok;
}

static void default_pass_split(int log_n, int* n_pass, int* pl) {
  if (log_n <= 12) {
    *n_pass = 1;
    pl[0] = log_n;
  } else if (log_n <= 24) {
    *n_pass = 2;
    pl[0] = (log_n + 1) / 2;
    pl[1] = log_n / 2;
  } else {
    *n_pass = 3;
    pl[0] = (log_n + 2) / 3;
    pl[1] = (log_n + 1) / 3;
    pl[2] = log_n / 3;
  }
}

int check_plan_valid(const Plan& p, int log_n) {
  if (p.n_pass < 1 || p.n_pass > 4) return FRNTT_EINVAL;
  int s = 0;
  for (int i = 0; i < p.n_pass; ++i) {
    if (p.pass_log[i] < 1 || p.pass_log[i] > kMaxLogT) return FRNTT_EINVAL;
    s += p.pass_log[i];
  }
  return s == log_n ? FRNTT_OK : FRNTT_EINVAL;
}

static Plan plan_for_locked(const frntt_ctx* ctx, int algo, int log_n) {
  Plan plan;
  if (ctx && ctx->has_override[algo][log_n]) {
    plan = ctx->plan_override[algo][log_n];
  } else if (ctx && ctx->has_tuned[log_n] && ctx->tuned[log_n].algo == algo) {
    const TuneEntry& t = ctx->tuned[log_n];
    plan.n_pass = t.n_pass;
    for (int i = 0; i < 4; ++i) {
      plan.pass_log[i] = t.pass_log[i];
      plan.lev_set[i] = t.nlev[i] > 0;
      plan.nlev[i] = t.nlev[i];
      for (int j = 0; j < 3; ++j) plan.lev_log[i][j] = t.lev_log[i][j];
    }
  } else {
    default_pass_split(log_n, &plan.n_pass, plan.pass_log);
  }
  return plan;
}

static int effective_algo_locked(const frntt_ctx* ctx, int log_n, int requested) {
  int a = requested;
  if (a == FRNTT_ALGO_AUTO) a = ctx->algo;
  if (a == FRNTT_ALGO_AUTO) {
    if (ctx->has_tuned[log_n]) a = ctx->tuned[log_n].algo;
    else a = FRNTT_ALGO_FOURSTEP_MFMA;
  }
  return a;
}

Plan plan_for(const frntt_ctx* ctx, int algo, int log_n) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  return plan_for_locked(ctx, algo, log_n);
}

int effective_algo(const frntt_ctx* ctx, int log_n, int requested) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  return effective_algo_locked(ctx, log_n, requested);
}

void resolve_plan(const frntt_ctx* ctx, int algo_req, int log_n, int* algo, Plan* plan) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  *algo = effective_algo_locked(ctx, log_n, algo_req);
  *plan = plan_for_locked(ctx, *algo, log_n);
}

bool stream_capturing(hipStream_t stream) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &st) != hipSuccess) return false;
  return st != hipStreamCaptureStatusNone;
}

size_t scratch_bytes_for(int log_n, int batch, int n_pass) {
  if (n_pass <= 1) return 0;
  return ((size_t)batch << log_n) * 32;
}

// Lines per workgroup for pass p: fill 2^12 staged elements, but never span
// more lines than one contiguous group holds, and divide the line count.
static int pass_log_g(const Plan& plan, int p, int log_n, int batch) {
  const int l = plan.pass_log[p];
  int lg = kMaxLogT - l;
  const bool last = (p == plan.n_pass - 1);
  int s = 0;
  for (int q = p + 1; q < plan.n_pass; ++q) s += plan.pass_log[q];
  int d = log_n - l - s;
  if (!last) {
    lg = std::min(lg, s);
  } else if (plan.n_pass > 1) {
    lg = std::min(lg, d);
  } else {
    // single pass: lines are whole polynomials; G must divide the batch
    int b = batch, tz = 0;
    while (b > 0 && (b & 1) == 0 && tz < 30) {
      b >>= 1;
      ++tz;
    }
    lg = std::min(lg, tz);
  }
  return std::max(lg, 0);
}

int build_passes(frntt_ctx* ctx, const Plan& plan_in, int log_n, int batch, int kind, void* data,
                 void* scratch, std::vector<PassParams>* out, int algo, bool capturing, bool no_tables) {
  PassParams pp[4];
  int n = 0;
  const int rc = build_passes_into(ctx, plan_in, log_n, batch, kind, data, scratch, pp, &n, algo, capturing,
                                   no_tables);
  out->assign(pp, pp + (rc == FRNTT_OK ? n : 0));
  return rc;
}

int build_passes_into(frntt_ctx* ctx, const Plan& plan_in, int log_n, int batch, int kind, void* data,
                      void* scratch, PassParams* out, int* n_out, int algo, bool capturing, bool no_tables) {
  Plan plan = plan_in;
  *n_out = 0;
  if (plan.n_pass < 1 || plan.n_pass > 4) return FRNTT_EINVAL;
  const int dir = (kind == FRNTT_INV || kind == FRNTT_COSET_INV) ? 1 : 0;
  const bool scaled = !no_tables && first_pass_scaled(ctx, plan);
  // an inverse transform whose first pass reads a twiddle table takes N^-1
  // from that table, and its last pass skips the N^-1 product
  const bool fold = dir == 1 && scaled;
  // a coset transform whose first pass reads a twiddle table takes the
  // per-line part of g^n from that table and the rest from its tail
  const bool coset_fold = kind == FRNTT_COSET && scaled;
  // a two-pass coset INTT also takes g^-k of the first pass's output digit
  // from that table and the rest of g^-K from its tail
  const bool coset_inv_fold = kind == FRNTT_COSET_INV && plan.n_pass == 2 && scaled;
  const u32x4* first_tw = nullptr;
  int d = 0;
  for (int p = 0; p < plan.n_pass; ++p) {
    const int l = plan.pass_log[p];
    int s = 0;
    for (int q = p + 1; q < plan.n_pass; ++q) s += plan.pass_log[q];
    const int lg = pass_log_g(plan, p, log_n, batch);
    const int log_t = l + lg;
    const bool mfma_ok = plan_levels(plan, p, log_t);
    PassParams P{};
    const bool first = p == 0, last = p == plan.n_pass - 1;
    P.src = (const u32x4*)(first ? data : scratch);
    P.dst = (u32x4*)(last ? data : scratch);
    P.log_n = log_n;
    P.log_r = l;
    P.log_s = s;
    P.log_d = d;
    P.log_g = lg;
    P.log_t = log_t;
    P.is_last = last ? 1 : 0;
    P.n_pass = plan.n_pass;
    for (int i = 0; i < 4; ++i) P.pass_log[i] = plan.pass_log[i];
    P.nlev = plan.nlev[p];
    for (int i = 0; i < kMaxLevels; ++i) P.lev_log[i] = plan.lev_log[p][i];
    P.engine = (algo == FRNTT_ALGO_FOURSTEP_MFMA && mfma_ok) ? 1 : 0;
    P.dir = dir;
    P.coset_pre = (first && kind == FRNTT_COSET) ? (coset_fold ? 2 : 1) : 0;
    P.post = 0;
    if (last && kind == FRNTT_INV) P.post = fold ? 0 : 1;
    if (last && kind == FRNTT_COSET_INV) P.post = coset_inv_fold ? 4 : fold ? 3 : 2;
    P.post_tw = P.post == 4 ? first_tw + 2 * ((int64_t)1 << log_n) : nullptr;
    const int64_t lines = ((int64_t)batch << log_n) >> l;
    P.wg_count = lines >> lg;
    P.xcd_remap = 1;
    P.pass_tw = nullptr;
    if (!last && !no_tables) {
      int rc = FRNTT_OK;
      const int coset = !first ? 0 : coset_fold ? 1 : coset_inv_fold ? 2 : 0;
      P.pass_tw = pass_table(ctx, dir, l, s, first && fold ? log_n : -1, coset, &rc, !capturing);
      if (first) first_tw = P.pass_tw;
      if (rc != FRNTT_OK) return rc;
    }
    out[(*n_out)++] = P;
    d += l;
  }
  // The matrix form leaves the outputs of a non-last pass below 2r, which
  // only its own first level reads: all passes of a transform run on one
  // engine. (With a full tile every pass has a plan kernel, so this only
  // guards the rule.)
  bool all_mfma = true;
  for (int i = 0; i < *n_out; ++i) all_mfma = all_mfma && out[i].engine == 1;
  if (!all_mfma)
    for (int i = 0; i < *n_out; ++i) out[i].engine = 0;
  return FRNTT_OK;
}

bool pass_tables_on(const frntt_ctx* ctx, int log_r, int log_s) {
  return !(ctx->flags & FRNTT_SPLIT_TWIDDLES) && log_r + log_s <= kPassTableMaxLog;
}

bool first_pass_scaled(const frntt_ctx* ctx, const Plan& plan) {
  if (plan.n_pass < 2 || (ctx->flags & FRNTT_SPLIT_TWIDDLES)) return false;
  int log_n = 0;
  for (int p = 0; p < plan.n_pass; ++p) log_n += plan.pass_log[p];
  return log_n <= kPassTableMaxLog;
}

static int pass_table_key(int dir, int log_r, int log_s, int scale_log, int coset) {
  return (coset << 26) | ((scale_log + 1) << 20) | (dir << 16) | (log_r << 8) | log_s;
}

static size_t pass_table_entries(int log_r, int log_s, int coset) {
  return ((size_t)1 << (log_r + log_s)) + (coset == 1 ? ((size_t)1 << log_r) : coset == 2 ? ((size_t)1 << log_s) : 0);
}

const u32x4* pass_table(frntt_ctx* ctx, int dir, int log_r, int log_s, int scale_log, int coset, int* rc,
                        bool may_build) {
  *rc = FRNTT_OK;
  if (!pass_tables_on(ctx, log_r, log_s)) return nullptr;
  const int key = pass_table_key(dir, log_r, log_s, scale_log, coset);
  std::lock_guard<std::mutex> lk(ctx->tw_mu);
  auto it = ctx->pass_tw.find(key);
  if (it != ctx->pass_tw.end()) return (const u32x4*)it->second;
  if (!may_build) {
    // a graph capture must not allocate or synchronise: frntt_prepare first
    *rc = FRNTT_ESTATE;
    return nullptr;
  }
  const size_t bytes = 32 * pass_table_entries(log_r, log_s, coset);
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    set_hip_error(ctx, e);
    *rc = FRNTT_ENOMEM;
    return nullptr;
  }
  // built once, on a private stream, before any transform uses it
  hipStream_t st = nullptr;
  e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (e == hipSuccess) {
    const int64_t n = (int64_t)pass_table_entries(log_r, log_s, coset);
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(pass_twiddle_kernel, dim3(grid), dim3(256), 0, st, (u32x4*)p, ctx->tables, dir, log_r,
                       log_s, scale_log, coset);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    hipStreamDestroy(st);
  }
  if (e != hipSuccess) {
    hipFree(p);
    *rc = set_hip_error(ctx, e);
    return nullptr;
  }
  ctx->pass_tw[key] = p;
  ctx->table_bytes += bytes;
  return (const u32x4*)p;
}

std::vector<int> pass_table_keys(frntt_ctx* ctx) {
  std::lock_guard<std::mutex> lk(ctx->tw_mu);
  std::vector<int> keys;
  for (const auto& kv : ctx->pass_tw) keys.push_back(kv.first);
  return keys;
}

void release_tuning_tables(frntt_ctx* ctx, const std::vector<int>& before, const Plan& chosen) {
  // keys of the forward tables of the chosen plan
  std::vector<int> keep(before);
  for (int p = 0; p + 1 < chosen.n_pass; ++p) {
    int s = 0;
    for (int q = p + 1; q < chosen.n_pass; ++q) s += chosen.pass_log[q];
    keep.push_back(pass_table_key(0, chosen.pass_log[p], s, -1, 0));
  }
  std::vector<std::pair<void*, size_t>> drop;
  {
    std::lock_guard<std::mutex> lk(ctx->tw_mu);
    for (auto it = ctx->pass_tw.begin(); it != ctx->pass_tw.end();) {
      if (std::find(keep.begin(), keep.end(), it->first) == keep.end()) {
        const int key = it->first;  // (coset << 26) | ... | (log_r << 8) | log_s
        drop.push_back({it->second, 32 * pass_table_entries((key >> 8) & 0xff, key & 0xff, key >> 26)});
        it = ctx->pass_tw.erase(it);
      } else {
        ++it;
      }
    }
  }
  if (drop.empty()) return;
  // no transform can still be reading them once the device is idle
  (void)hipDeviceSynchronize();
  for (const auto& d : drop) {
    ctx->table_bytes -= d.second;
    (void)hipFree(d.first);
  }
}

size_t pending_pass_table_bytes(frntt_ctx* ctx, const Plan& plan, int kind) {
  const int dir = (kind == FRNTT_INV || kind == FRNTT_COSET_INV) ? 1 : 0;
  const bool fold = dir == 1 && first_pass_scaled(ctx, plan);
  const bool coset_fold = kind == FRNTT_COSET && first_pass_scaled(ctx, plan);
  const bool coset_inv_fold = kind == FRNTT_COSET_INV && plan.n_pass == 2 && first_pass_scaled(ctx, plan);
  size_t bytes = 0;
  std::lock_guard<std::mutex> lk(ctx->tw_mu);
  for (int p = 0; p + 1 < plan.n_pass; ++p) {
    int s = 0;
    for (int q = p + 1; q < plan.n_pass; ++q) s += plan.pass_log[q];
    const int l = plan.pass_log[p];
    if (!pass_tables_on(ctx, l, s)) continue;
    const int scale_log = p == 0 && fold ? l + s : -1;
    const int coset = p != 0 ? 0 : coset_fold ? 1 : coset_inv_fold ? 2 : 0;
    if (!ctx->pass_tw.count(pass_table_key(dir, l, s, scale_log, coset)))
      bytes += 32 * pass_table_entries(l, s, coset);
  }
  return bytes;
}

int get_scratch(frntt_ctx* ctx, hipStream_t stream, size_t bytes, void** out) {
  *out = nullptr;
  if (bytes == 0) return FRNTT_OK;
  const bool capturing = stream_capturing(stream);
  std::lock_guard<std::mutex> lk(ctx->mu);
  Scratch& s = ctx->scratch[stream];
  if (s.bytes < bytes && capturing) return FRNTT_ESTATE;  // no allocation inside a capture
  if (s.bytes < bytes) {
    if (s.ptr) {
      // the old buffer may still be in use by work queued on this stream
      hipError_t e = hipStreamSynchronize(stream);
      if (e != hipSuccess) return set_hip_error(ctx, e);
      hipFree(s.ptr);
      s.ptr = nullptr;
      s.bytes = 0;
    }
    hipError_t e = hipMalloc(&s.ptr, bytes);
    if (e != hipSuccess) {
      s.ptr = nullptr;
      set_hip_error(ctx, e);
      return FRNTT_ENOMEM;
    }
    s.bytes = bytes;
  }
  *out = s.ptr;
  return FRNTT_OK;
}

int launch_passes(frntt_ctx* ctx, const std::vector<PassParams>& passes, int algo, hipStream_t stream) {
  return launch_passes(ctx, passes.data(), (int)passes.size(), algo, stream);
}

int launch_passes(frntt_ctx* ctx, const PassParams* passes, int n, int algo, hipStream_t stream) {
  for (int i = 0; i < n; ++i) {
    const PassParams& P = passes[i];
    if (P.wg_count <= 0) continue;
    (void)algo;
    MfmaPassKernel plan_k = P.engine == 1 ? mfma_plan_kernel(P.nlev, P.lev_log) : nullptr;
    if (plan_k)
      hipLaunchKernelGGL(plan_k, dim3((unsigned)P.wg_count), dim3(kMfmaThreads), 0, stream, P, ctx->tables);
    else
      hipLaunchKernelGGL(ntt_pass_bfly_kernel, dim3((unsigned)P.wg_count), dim3(kBflyThreads), 0, stream, P,
                         ctx->tables);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_hip_error(ctx, e);
  }
  return FRNTT_OK;
}

static int validate_inputs(frntt_ctx* ctx, void* data, int log_n, int batch, hipStream_t stream) {
  const uint64_t count = (uint64_t)batch << log_n;
  const unsigned blocks = (unsigned)((count + 255) / 256);
  hipLaunchKernelGGL(validate_kernel, dim3(blocks), dim3(256), 0, stream, (const u32x4*)data, count,
                     ctx->valid_flag);
  return set_hip_error(ctx, hipGetLastError());
}

int transform_impl(frntt_ctx* ctx, void* data, int log_n, int batch, int kind, int algo_req,
                   hipStream_t stream, void* workspace, size_t ws_bytes) {
  if (!ctx || (!data && batch > 0)) return FRNTT_EINVAL;
  if (batch < 0 || kind < FRNTT_FWD || kind > FRNTT_COSET_INV) return FRNTT_EINVAL;
  if (algo_req < FRNTT_ALGO_AUTO || algo_req > FRNTT_ALGO_FOURSTEP_MFMA) return FRNTT_EINVAL;
  if (log_n < 0 || log_n > ctx->max_log_n || log_n > kMasterLog) return FRNTT_ERANGE;
  if (((uintptr_t)data & 31) != 0) return FRNTT_EALIGN;
  if (batch == 0) return FRNTT_OK;
  if ((((int64_t)batch) << log_n) > ((int64_t)1 << 40)) return FRNTT_ERANGE;
  DeviceGuard guard(ctx->device);
  if (ctx->flags & FRNTT_VALIDATE) {
    int rc = validate_inputs(ctx, data, log_n, batch, stream);
    if (rc) return rc;
  }
  if (log_n == 0) return FRNTT_OK;  // identity (N^-1 = 1, g^0 = 1)
  int algo = 0;
  Plan plan;
  resolve_plan(ctx, algo_req, log_n, &algo, &plan);
  return transform_plan(ctx, data, log_n, batch, kind, algo, plan, stream, workspace, ws_bytes);
}

int transform_plan(frntt_ctx* ctx, void* data, int log_n, int batch, int kind, int algo, const Plan& plan,
                   hipStream_t stream, void* workspace, size_t ws_bytes) {
  const size_t need = scratch_bytes_for(log_n, batch, plan.n_pass);
  void* scratch = nullptr;
  if (need) {
    if (workspace) {
      if (ws_bytes < need) return FRNTT_EINVAL;
      scratch = workspace;
    } else {
      int rc = get_scratch(ctx, stream, need, &scratch);
      if (rc) return rc;
    }
  }
  std::vector<PassParams> passes;
  int rc = build_passes(ctx, plan, log_n, batch, kind, data, scratch, &passes, algo, stream_capturing(stream));
  if (rc) return rc;
  return launch_passes(ctx, passes, algo, stream);
}

}  // namespace frntt

using namespace frntt;

// ---------------------------------------------------------------- C ABI

extern "C" {

int frntt_ctx_create(frntt_ctx** out, int hip_device, int max_log_n, unsigned flags) {
  if (!out) return FRNTT_EINVAL;
  *out = nullptr;
  if (max_log_n < 1 || max_log_n > kMasterLog) return FRNTT_ERANGE;
  if (flags & ~(unsigned)(FRNTT_VALIDATE | FRNTT_SPLIT_TWIDDLES)) return FRNTT_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev)
    return FRNTT_EINVAL;
  frntt_ctx* ctx = new (std::nothrow) frntt_ctx();
  if (!ctx) return FRNTT_ENOMEM;
  ctx->device = hip_device;
  ctx->max_log_n = max_log_n;
  ctx->flags = flags;
  DeviceGuard guard(hip_device);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, hip_device) == hipSuccess) ctx->cu_count = prop.multiProcessorCount;
  if (ctx->cu_count <= 0) ctx->cu_count = 256;
  int rc = build_tables(ctx);
  if (rc == FRNTT_OK) rc = build_rns_tables(ctx);
  if (rc == FRNTT_OK && noalloc_scratch_address(&ctx->noalloc_scratch) != 0) rc = FRNTT_EHIP;
  if (rc == FRNTT_OK) {
    hipError_t e = hipMalloc((void**)&ctx->valid_flag, 256);
    if (e != hipSuccess) rc = FRNTT_ENOMEM;
    else if (hipMemset(ctx->valid_flag, 0, 256) != hipSuccess) rc = FRNTT_EHIP;
  }
  if (rc != FRNTT_OK) {
    frntt_ctx_destroy(ctx);
    return rc;
  }
  *out = ctx;
  return FRNTT_OK;
}

int frntt_ctx_destroy(frntt_ctx* ctx) {
  if (!ctx) return FRNTT_OK;
  {
    DeviceGuard guard(ctx->device);
    hipDeviceSynchronize();
    for (auto& kv : ctx->scratch)
      if (kv.second.ptr) hipFree(kv.second.ptr);
    for (auto& g : ctx->graphs) {
      if (g.exec) hipGraphExecDestroy(g.exec);
      if (g.graph) hipGraphDestroy(g.graph);
      if (g.dev_buf) hipFree(g.dev_buf);
      if (g.scratch) hipFree(g.scratch);
    }
    for (auto& kv : ctx->batch_bufs) {
      if (kv.second.dev) hipFree(kv.second.dev);
      if (kv.second.host) hipHostFree(kv.second.host);
      if (kv.second.event) hipEventDestroy(kv.second.event);
    }
    if (ctx->valid_flag) hipFree(ctx->valid_flag);
    if (ctx->table_mem) hipFree(ctx->table_mem);
    destroy_rns_field(ctx->rns_default);
    destroy_msm_streams(ctx);
    for (auto& kv : ctx->pass_tw) hipFree(kv.second);
  }
  delete ctx;
  return FRNTT_OK;
}

int ntt_transform(frntt_ctx* ctx, void* data, int log_n, int batch, int kind, void* stream) {
  return transform_impl(ctx, data, log_n, batch, kind, FRNTT_ALGO_AUTO, (hipStream_t)stream, nullptr, 0);
}

int ntt_transform_algo(frntt_ctx* ctx, void* data, int log_n, int batch, int kind, int algo,
                       void* stream) {
  return transform_impl(ctx, data, log_n, batch, kind, algo, (hipStream_t)stream, nullptr, 0);
}

int ntt_fwd(frntt_ctx* ctx, void* data, int log_n, int batch, void* stream) {
  return ntt_transform(ctx, data, log_n, batch, FRNTT_FWD, stream);
}
int ntt_inv(frntt_ctx* ctx, void* data, int log_n, int batch, void* stream) {
  return ntt_transform(ctx, data, log_n, batch, FRNTT_INV, stream);
}
int ntt_coset(frntt_ctx* ctx, void* data, int log_n, int batch, void* stream) {
  return ntt_transform(ctx, data, log_n, batch, FRNTT_COSET, stream);
}
int ntt_coset_inv(frntt_ctx* ctx, void* data, int log_n, int batch, void* stream) {
  return ntt_transform(ctx, data, log_n, batch, FRNTT_COSET_INV, stream);
}

int frntt_set_algo(frntt_ctx* ctx, int algo) {
  if (!ctx || algo < FRNTT_ALGO_AUTO || algo > FRNTT_ALGO_FOURSTEP_MFMA) return FRNTT_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->algo = algo;
  return FRNTT_OK;
}

int frntt_get_algo(const frntt_ctx* ctx) {
  if (!ctx) return FRNTT_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  return ctx->algo;
}

int frntt_set_plan(frntt_ctx* ctx, int algo, int log_n, const int* pass_logs, int n_passes) {
  if (!ctx || algo < FRNTT_ALGO_BUTTERFLY || algo > FRNTT_ALGO_FOURSTEP_MFMA) return FRNTT_EINVAL;
  if (log_n < 1 || log_n > kMasterLog) return FRNTT_ERANGE;
  if (n_passes == 0) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->has_override[algo][log_n] = false;
    return FRNTT_OK;
  }
  if (!pass_logs || n_passes < 0 || n_passes > 4) return FRNTT_EINVAL;
  Plan p;
  p.n_pass = n_passes;
  for (int i = 0; i < n_passes; ++i) p.pass_log[i] = pass_logs[i];
  int rc = check_plan_valid(p, log_n);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->plan_override[algo][log_n] = p;
  ctx->has_override[algo][log_n] = true;
  return FRNTT_OK;
}

int frntt_get_plan(const frntt_ctx* ctx, int algo, int log_n, int* pass_logs, int cap) {
  if (!ctx || algo < FRNTT_ALGO_AUTO || algo > FRNTT_ALGO_FOURSTEP_MFMA) return FRNTT_EINVAL;
  if (log_n < 1 || log_n > kMasterLog) return FRNTT_ERANGE;
  int a = 0;
  Plan p;
  resolve_plan(ctx, algo, log_n, &a, &p);
  for (int i = 0; i < p.n_pass && i < cap; ++i)
    if (pass_logs) pass_logs[i] = p.pass_log[i];
  return p.n_pass;
}

int frntt_get_plan_levels(const frntt_ctx* ctx, int algo, int log_n, int pass, int* levels, int cap) {
  if (!ctx || algo < FRNTT_ALGO_AUTO || algo > FRNTT_ALGO_FOURSTEP_MFMA) return FRNTT_EINVAL;
  if (log_n < 1 || log_n > kMasterLog) return FRNTT_ERANGE;
  int a = 0;
  Plan p;
  resolve_plan(ctx, algo, log_n, &a, &p);
  if (pass < 0 || pass >= p.n_pass) return FRNTT_EINVAL;
  if (a != FRNTT_ALGO_FOURSTEP_MFMA) return 0;
  // the levels of a single transform (batch 1) of this size
  const int lg = pass_log_g(p, pass, log_n, 1);
  if (!plan_levels(p, pass, p.pass_log[pass] + lg)) return 0;
  for (int i = 0; i < p.nlev[pass] && i < cap; ++i)
    if (levels) levels[i] = p.lev_log[pass][i];
  return p.nlev[pass];
}

size_t frntt_scratch_bytes(int log_n, int batch) {
  if (log_n < 0 || log_n > kMasterLog || batch < 0) return 0;
  int n_pass, pl[4];
  default_pass_split(log_n, &n_pass, pl);
  return scratch_bytes_for(log_n, batch, n_pass);
}

int frntt_prepare(frntt_ctx* ctx, int log_n, int kind) {
  if (!ctx || kind < FRNTT_FWD || kind > FRNTT_COSET_INV) return FRNTT_EINVAL;
  if (log_n < 0 || log_n > ctx->max_log_n) return FRNTT_ERANGE;
  DeviceGuard guard(ctx->device);
  for (int algo = FRNTT_ALGO_BUTTERFLY; algo <= FRNTT_ALGO_FOURSTEP_MFMA; ++algo) {
    std::vector<PassParams> tmp;
    const int rc = build_passes(ctx, plan_for(ctx, algo, log_n), log_n, 1, kind, nullptr, nullptr, &tmp, algo);
    if (rc != FRNTT_OK) return rc;
  }
  return FRNTT_OK;
}

size_t frntt_table_bytes(const frntt_ctx* ctx) { return ctx ? ctx->table_bytes.load() : 0; }

int frntt_generate(frntt_ctx* ctx, void* data, uint64_t seed, uint64_t stream_id, uint64_t start,
                   uint64_t count, void* stream) {
  if (!ctx || (!data && count)) return FRNTT_EINVAL;
  if (((uintptr_t)data & 31) != 0) return FRNTT_EALIGN;
  if (count == 0) return FRNTT_OK;
  if (start + count > (1ull << 32)) return FRNTT_ERANGE;
  DeviceGuard guard(ctx->device);
  const unsigned blocks = (unsigned)((count + 255) / 256);
  hipLaunchKernelGGL(generate_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (u32x4*)data, seed,
                     stream_id, start, count);
  return set_hip_error(ctx, hipGetLastError());
}

int frntt_check_inputs(frntt_ctx* ctx) {
  if (!ctx) return FRNTT_EINVAL;
  if (!(ctx->flags & FRNTT_VALIDATE)) return FRNTT_OK;
  DeviceGuard guard(ctx->device);
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return set_hip_error(ctx, e);
  unsigned int flag = 0;
  e = hipMemcpy(&flag, ctx->valid_flag, sizeof flag, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return set_hip_error(ctx, e);
  if (flag) {
    e = hipMemset(ctx->valid_flag, 0, sizeof flag);
    if (e != hipSuccess) return set_hip_error(ctx, e);
    return FRNTT_EINVAL;
  }
  return FRNTT_OK;
}

int frntt_last_hip_error(const frntt_ctx* ctx) { return ctx ? ctx->last_hip_error : 0; }

const char* frntt_strerror(int status) {
  switch (status) {
    case FRNTT_OK: return "ok";
    case FRNTT_EINVAL: return "invalid argument";
    case FRNTT_ERANGE: return "size out of range";
    case FRNTT_EALIGN: return "data pointer not 32-byte aligned";
    case FRNTT_ENOMEM: return "out of memory";
    case FRNTT_EHIP: return "HIP runtime error";
    case FRNTT_EBUSY: return "busy: over budget or queue limit";
    case FRNTT_ESTATE: return "invalid state";
  }
  return "unknown status";
}

}  // extern "C"
