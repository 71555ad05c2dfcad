// Host-side internals of libfrntt: context, plans and launch helpers.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/frntt.h"
#include "ntt_device.hpp"
#include "rns_lazy.hpp"

namespace frntt {

struct MsmStreams;
__global__ void ntt_pass_bfly_kernel(PassParams P, DevTables T);

__global__ void ntt_batch_kernel(BatchParams B);
__global__ void generate_kernel(u32x4* out, uint64_t seed, uint64_t stream_id, uint64_t start,
                                uint64_t count);
__global__ void validate_kernel(const u32x4* data, uint64_t count, unsigned int* flag);
__global__ void zero_words_kernel(unsigned int* p, int64_t n);
__global__ void pass_twiddle_kernel(u32x4* dst, DevTables T, int dir, int log_r, int log_s, int scale_log,
                                    int coset);

// Decomposition of one transform size into passes and levels.
struct Plan {
  int n_pass = 0;
  int pass_log[4] = {0, 0, 0, 0};
  int nlev[4] = {0, 0, 0, 0};
  int lev_log[4][kMaxLevels] = {};
  // lev_set[p]: pass p asks for the level split in nlev[p] / lev_log[p] (the
  // autotuner's choice) instead of the default one; used if a plan kernel
  // exists for it and the pass runs on the matrix form
  bool lev_set[4] = {false, false, false, false};
  int log_t = 12;   // elements per workgroup (upper bound)
};

struct Scratch {
  void* ptr = nullptr;
  size_t bytes = 0;
};

struct JobPlan {
  int algo = 0;
  Plan plan;
};

struct GraphEntry {
  std::vector<frntt_job> jobs;
  std::vector<JobPlan> plans;  // the form and plan of each job when captured
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  void* dev_buf = nullptr;  // descriptors + counters used by the captured launch
  void* scratch = nullptr;  // scratch owned by the captured launch
};

// Per-stream descriptor buffers of ntt_batch.
struct BatchBuffers {
  void* dev = nullptr;
  size_t dev_bytes = 0;
  void* host = nullptr;     // pinned staging
  size_t host_bytes = 0;
  hipEvent_t event = nullptr;  // recorded after the upload from `host`
};

// Algorithm and plan fixed for one job of a batch.
struct TuneEntry {
  int algo = FRNTT_ALGO_FOURSTEP_MFMA;
  int n_pass = 0;
  int pass_log[4] = {0, 0, 0, 0};
  int nlev[4] = {0, 0, 0, 0};      // level split per pass (matrix form; 0: default)
  int lev_log[4][3] = {};
  float ms = 0.f;
};

}  // namespace frntt

struct frntt_ctx {
  int device = 0;
  int max_log_n = 0;
  unsigned flags = 0;
  int algo = FRNTT_ALGO_AUTO;       // guarded by mu
  int cu_count = 0;
  mutable int last_hip_error = 0;
  void* table_mem = nullptr;       // single device allocation holding all tables
  std::atomic<size_t> table_bytes{0};  // all context tables, including pass-twiddle tables
  frntt::DevTables tables{};
  unsigned int* valid_flag = nullptr;  // device flag for FRNTT_VALIDATE
  void* noalloc_scratch = nullptr;     // this device's static scratch of ntt_transform_noalloc
  frntt_rns_field* rns_default = nullptr;  // RNS lazy product over Fr (BN254), built at creation
  frntt::MsmStreams* msm_streams = nullptr;  // side streams of frntt_msm_batch, made on first use
  // plan overrides [algo][log_n]
  frntt::Plan plan_override[3][29];
  bool has_override[3][29] = {};
  frntt::TuneEntry tuned[29];
  bool has_tuned[29] = {};
  mutable std::mutex mu;           // guards algo, plan overrides, tuned plans, scratch, graphs
  std::map<hipStream_t, frntt::Scratch> scratch;
  std::vector<frntt::GraphEntry> graphs;
  std::map<hipStream_t, frntt::BatchBuffers> batch_bufs;
  // pass-twiddle tables, built on first use: key (dir, log_r, log_s)
  std::mutex tw_mu;
  std::map<int, void*> pass_tw;
};

namespace frntt {

int set_hip_error(const frntt_ctx* ctx, hipError_t e);
// The context's RNS lazy product over Fr (built at context creation), any
// other field's tables, and their release.
int build_rns_tables(frntt_ctx* ctx);
int create_rns_field(frntt_ctx* ctx, const uint32_t* m, int mw, frntt_rns_field** out);
void destroy_rns_field(frntt_rns_field* f);
// Release the side streams and events of frntt_msm_batch (after the device
// has been synchronised).
void destroy_msm_streams(frntt_ctx* ctx);
// Default or overridden plan for (algo, log_n); algo must be BUTTERFLY or MFMA.
// Takes ctx->mu.
Plan plan_for(const frntt_ctx* ctx, int algo, int log_n);
// The algorithm and plan a call with algorithm `algo_req` uses for this size,
// read together under ctx->mu.
void resolve_plan(const frntt_ctx* ctx, int algo_req, int log_n, int* algo, Plan* plan);
// Is work on `stream` being captured into a graph? Such calls must not
// allocate or synchronise, so they fail with FRNTT_ESTATE where they would.
bool stream_capturing(hipStream_t stream);
// Build the per-pass launch parameters of one transform. A pass-twiddle table
// that does not exist yet is built (synchronously) unless `capturing`, in
// which case the call fails with FRNTT_ESTATE.
// With no_tables every pass twiddle comes from the split tables (no table is
// looked up or built).
int build_passes(frntt_ctx* ctx, const Plan& plan, int log_n, int batch, int kind,
                 void* data, void* scratch, std::vector<PassParams>* out, int algo, bool capturing = false,
                 bool no_tables = false);
// The same into a caller's array of at least 4 entries (no host allocation).
int build_passes_into(frntt_ctx* ctx, const Plan& plan, int log_n, int batch, int kind, void* data,
                      void* scratch, PassParams* out, int* n_out, int algo, bool capturing, bool no_tables);
// Largest batch << log_n of the allocation-free entry point (its static
// device scratch holds 2^kNoallocMaxLog elements).
constexpr int kNoallocMaxLog = 20;
// Device address of this GPU's allocation-free scratch array (hipError_t).
int noalloc_scratch_address(void** out);
// One transform with an explicit plan (no plan lookup).
int transform_plan(frntt_ctx* ctx, void* data, int log_n, int batch, int kind, int algo, const Plan& plan,
                   hipStream_t stream, void* workspace, size_t ws_bytes);
// Pass-twiddle table w_(2^(log_r + log_s))^(rest * k) at [k][rest] for a
// non-last pass, times 2^-scale_log when scale_log >= 0, times g^rest with
// 2^log_r pre-scale entries (g^(2^log_s))^j appended when coset == 1, times
// g^-k with 2^log_s epilogue entries (g^-(2^log_r))^k' appended when
// coset == 2 (built
// and cached per (dir, log_r, log_s, scale_log, coset) on first use), or
// nullptr when it would
// exceed kPassTableMaxLog entries (the pass then forms each twiddle from the
// split tables).
constexpr int kPassTableMaxLog = 25;
const u32x4* pass_table(frntt_ctx* ctx, int dir, int log_r, int log_s, int scale_log, int coset, int* rc,
                        bool may_build = true);
// Does a non-last pass of radix 2^log_r and stride 2^log_s read a twiddle
// table (no FRNTT_SPLIT_TWIDDLES, at most 2^kPassTableMaxLog entries)?
bool pass_tables_on(const frntt_ctx* ctx, int log_r, int log_s);
// Does the first pass of `plan` read a twiddle table (so that an inverse
// transform can take N^-1 from it)?
bool first_pass_scaled(const frntt_ctx* ctx, const Plan& plan);
// Bytes of the pass-twiddle tables a transform with this plan and kind would
// still have to build.
size_t pending_pass_table_bytes(frntt_ctx* ctx, const Plan& plan, int kind);
// Takes ctx->mu.
int effective_algo(const frntt_ctx* ctx, int log_n, int requested);
// Keys of the pass-twiddle tables built so far.
std::vector<int> pass_table_keys(frntt_ctx* ctx);
// After tuning: free the pass-twiddle tables built since `before` except the
// forward tables of the chosen plan (waits for the device first).
void release_tuning_tables(frntt_ctx* ctx, const std::vector<int>& before, const Plan& chosen);
size_t scratch_bytes_for(int log_n, int batch, int n_pass);
int get_scratch(frntt_ctx* ctx, hipStream_t stream, size_t bytes, void** out);
int launch_passes(frntt_ctx* ctx, const std::vector<PassParams>& passes, int algo, hipStream_t stream);
int launch_passes(frntt_ctx* ctx, const PassParams* passes, int n, int algo, hipStream_t stream);
bool mfma_level_ok(int m, int log_t);
int transform_impl(frntt_ctx* ctx, void* data, int log_n, int batch, int kind, int algo,
                   hipStream_t stream, void* workspace, size_t ws_bytes);
int check_plan_valid(const Plan& p, int log_n);

}  // namespace frntt
