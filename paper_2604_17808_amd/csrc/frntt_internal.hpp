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

namespace frntt {

__global__ void ntt_pass_bfly_kernel(PassParams P, DevTables T);
__global__ void ntt_pass_mfma_kernel(PassParams P, DevTables T);

__global__ void ntt_batch_kernel(BatchParams B, DevTables T);
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
  int log_t = 12;   // elements per workgroup (upper bound)
};

struct Scratch {
  void* ptr = nullptr;
  size_t bytes = 0;
};

struct GraphEntry {
  std::vector<frntt_job> jobs;
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

struct TuneEntry {
  int algo = FRNTT_ALGO_FOURSTEP_MFMA;
  int n_pass = 0;
  int pass_log[4] = {0, 0, 0, 0};
  float ms = 0.f;
};

}  // namespace frntt

struct frntt_ctx {
  int device = 0;
  int max_log_n = 0;
  unsigned flags = 0;
  int algo = FRNTT_ALGO_AUTO;
  int cu_count = 0;
  mutable int last_hip_error = 0;
  void* table_mem = nullptr;       // single device allocation holding all tables
  std::atomic<size_t> table_bytes{0};  // all context tables, including pass-twiddle tables
  frntt::DevTables tables{};
  unsigned int* valid_flag = nullptr;  // device flag for FRNTT_VALIDATE
  // plan overrides [algo][log_n]
  frntt::Plan plan_override[3][29];
  bool has_override[3][29] = {};
  frntt::TuneEntry tuned[29];
  bool has_tuned[29] = {};
  std::mutex mu;                   // guards scratch, graphs, tuning state
  std::map<hipStream_t, frntt::Scratch> scratch;
  std::vector<frntt::GraphEntry> graphs;
  std::map<hipStream_t, frntt::BatchBuffers> batch_bufs;
  // pass-twiddle tables, built on first use: key (dir, log_r, log_s)
  std::mutex tw_mu;
  std::map<int, void*> pass_tw;
};

namespace frntt {

int set_hip_error(const frntt_ctx* ctx, hipError_t e);
// Default or overridden plan for (algo, log_n); algo must be BUTTERFLY or MFMA.
Plan plan_for(const frntt_ctx* ctx, int algo, int log_n);
// Build the per-pass launch parameters of one transform.
int build_passes(frntt_ctx* ctx, const Plan& plan, int log_n, int batch, int kind,
                 void* data, void* scratch, std::vector<PassParams>* out, int algo);
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
const u32x4* pass_table(frntt_ctx* ctx, int dir, int log_r, int log_s, int scale_log, int coset, int* rc);
// Does the first pass of `plan` read a twiddle table (so that an inverse
// transform can take N^-1 from it)?
bool first_pass_scaled(const Plan& plan);
// Bytes of the pass-twiddle tables a transform with this plan and kind would
// still have to build.
size_t pending_pass_table_bytes(frntt_ctx* ctx, const Plan& plan, int kind);
int effective_algo(const frntt_ctx* ctx, int log_n, int requested);
size_t scratch_bytes_for(int log_n, int batch, int n_pass);
int get_scratch(frntt_ctx* ctx, hipStream_t stream, size_t bytes, void** out);
int launch_passes(frntt_ctx* ctx, const std::vector<PassParams>& passes, int algo, hipStream_t stream);
bool mfma_level_ok(int m, int log_t);
int transform_impl(frntt_ctx* ctx, void* data, int log_n, int batch, int kind, int algo,
                   hipStream_t stream, void* workspace, size_t ws_bytes);
int check_plan_valid(const Plan& p, int log_n);

}  // namespace frntt
