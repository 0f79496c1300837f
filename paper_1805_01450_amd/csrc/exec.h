// Device executor of the per-item contraction program (host-side API).
#pragma once
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "host.h"

namespace qgm {

// Wide-engine descriptors on the device (plus the host copy of the step
// records, read when launching).
struct WideDev {
  void* steps = nullptr;
  void* ops = nullptr;
  int n_steps = 0;
  std::vector<int32_t> host_steps;
  void* module = nullptr;  // generated kernels (hipModule_t), or null: prebuilt per-step kernels
  // generated item kernels, one per level of independent steps, in order
  struct Level {
    void* fn;                   // hipFunction_t
    unsigned long long blocks;  // blocks per 64-item group
    int threads;                // threads per block
  };
  std::vector<Level> levels;
  // profiling: when set, levels.size() + 1 events recorded on the launch
  // stream around the level launches of the first pass of a run
  mutable void* const* level_events = nullptr;
  // constant steps: runs of small steps in one single-block launch (indices
  // in const_list[first, first + count)), large steps alone (first = step)
  struct ConstLaunch {
    int block, first, count;
    void* fn;  // generated kernel (hipFunction_t) or null for the prebuilt ones
    unsigned long long elems;
  };
  std::vector<ConstLaunch> const_plan;
  void* const_list = nullptr;
};

// Device-resident copy of a compiled program (owned by a plan).
struct DevProgram {
  int device = -1;
  void* raw = nullptr;     // double2 per raw entry
  void* rawp = nullptr;    // int per raw entry (RZ parameter index or -1)
  void* rawb = nullptr;    // int per raw entry (RZ variable value)
  void* rawd = nullptr;    // int per raw entry (1 = RZ derivative table)
  void* slot_param = nullptr;  // int per gradient slot: parameter index
  void* steps = nullptr;
  void* leaves = nullptr;
  void* optab = nullptr;
  int n_steps = 0, n_const_steps = 0;
  int n_cu = 0;
  size_t max_lds = 0;
  WideDev wide;            // wide engine (empty otherwise)
  void* module = nullptr;  // hipModule_t of the generated chain kernel
  void* chain_fn = nullptr;  // hipFunction_t "qgm_chain"
  int chain_waves = 1;       // wavefronts per block of the generated kernel
  int chain_persistent = 0;  // 1: the generated kernel pulls chunks from a work queue (resident grid)
  // Constant area computed once per plan (plans without RZ angles): the raw
  // tables and every constant step, contracted at upload; runs then read it
  // instead of rebuilding the constants in their workspace.
  void* cst_cache = nullptr;
  int cst_cached = 0;
};

// Precision of the slice contraction: 0 = complex128, 1 = complex64.
struct LaunchCfg {
  int prec;
  int generated;        // 1 = generated chain kernel
  int wide;             // 1 = wide engine (one kernel per step, tensors in HBM)
  size_t wide_budget;   // bytes of HBM the wide engine may use for item tensors
  int n_qubits;
  int n_bs;             // bitstrings
  uint64_t s_begin;     // first slice index
  uint64_t n_s;         // slices per bitstring in this call
  int n_params;
};

struct WsLayout {
  size_t cst, bits, res, gres, counter, chunks, scratch, total;
  int fused;            // generated kernel sums each block's 64 slices itself
  int wide_groups;      // wide engine: 64-item groups resident per pass
  int use_lds;
  int grid;             // persistent workgroups (one wave each)
  size_t lds_bytes;     // dynamic LDS per workgroup
};

// All functions return 0 or a negative qgm status; `err` gets a message.
// Uploads the program tables and, when `code` is not empty, loads the
// generated kernel's code object on the current device.
int dev_upload(const Program& prog, const std::vector<char>& code, const WideProgram* wide, DevProgram& dp,
               std::string& err, const std::vector<char>* wide_code = nullptr,
               const std::vector<WideKernel>* wide_kernels = nullptr);
void dev_free(DevProgram& dp);
int dev_layout(const Program& prog, const DevProgram& dp, const LaunchCfg& cfg, WsLayout& ws, std::string& err);
// Runs prologue, persistent chain and slice reduction on `stream`.  Device
// inputs: bits (n_bs x n_qubits bytes), params (n_params doubles or null).
// Device output: partial (n_bs x 4 doubles: sum re, sum im, comp re, comp im)
// and, for gradient programs when d_grad_partial is not null, grad_partial
// (n_bs x n_params x 4 doubles, same layout per parameter).
// events: null, or 4 HIP events recorded before the prologue, before the
// chain, after the chain and after the reduction.
int dev_run(const Program& prog, const DevProgram& dp, const LaunchCfg& cfg, const WsLayout& ws,
            const uint8_t* d_bits, const double* d_params, void* d_ws, void* stream, double* d_partial,
            double* d_grad_partial, void* const* events, std::string& err);
int dev_query(int& n_cu, size_t& max_lds, std::string& err);
// Contract the constant steps of a plan without RZ angles once into
// plan-owned device memory (synchronous, on a private stream).
int dev_cache_constants(const Program& prog, DevProgram& dp, int prec, int wide, std::string& err);

}  // namespace qgm
