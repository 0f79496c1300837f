// Device executor: prologue (tables, constant steps), persistent per-item
// contraction chain, and the FP64 compensated slice reduction.
//
// Work items are (bitstring b, slice s) pairs.  A wavefront runs 64 items
// at once, one per lane, all following the same program; every operand
// offset is therefore wave-uniform and is read with scalar loads.  Item
// tensors live in LDS as [element][lane] rows, so each wavefront access is a
// contiguous, conflict-free 64-lane row.  Constant tensors (those that depend
// on no fixed variable) are computed once per call and read through the
// scalar cache.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "bfx3.h"
#include "exec.h"

namespace qgm {

template <typename R>
int wide_launch_steps(const WideDev& wd, int first_group, int n_groups, const void* cst, void* mem,
                      uint64_t group_elems, const uint64_t* packed, int n_bs, uint64_t s_begin, uint64_t n_s,
                      uint64_t n_items, void* res, void* gres, bool const_steps, hipStream_t stream);

namespace {

struct DevStep {
  int kind, out, r, ns, m, ops, leaf, grad_slot;
};

// A leaf: up to four free variables (strides fs) and four fixed ones
// (source 0 = output bit, 1 = slice bit; bit; stride ds).
struct DevLeaf {
  int nfree, ndep, table, pad;
  int fs[4], src[4], bit[4], ds[4];
};

template <typename R>
struct cx {
  R x, y;
};

template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
  cx<R> c;
  c.x = a.x * b.x - a.y * b.y;
  c.y = a.x * b.y + a.y * b.x;
  return c;
}

constexpr uint32_t kConst = 0x80000000u;
constexpr int kLanes = 64;

#define HIP_OK(expr)                                                   \
  do {                                                                 \
    hipError_t e_ = (expr);                                            \
    if (e_ != hipSuccess) {                                            \
      err = std::string(#expr) + ": " + hipGetErrorString(e_);         \
      return -6;                                                       \
    }                                                                  \
  } while (0)

// ---------------------------------------------------------------- prologue
// One workgroup.  Zeroes the work counter, packs the bitstrings, writes the
// raw factor tables in the working precision (RZ(theta) entries
// e^{i theta (2u-1)/2} from the angles), then runs the constant steps in
// order.
template <typename R>
__global__ void __launch_bounds__(256) prologue_kernel(const double* __restrict__ raw, const int* __restrict__ rawp,
                                                       const int* __restrict__ rawb, const int* __restrict__ rawd,
                                                       int n_raw,
                                                       const double* __restrict__ params,
                                                       const DevStep* __restrict__ steps, int n_const_steps,
                                                       const uint32_t* __restrict__ optab, cx<R>* __restrict__ cst,
                                                       const uint8_t* __restrict__ bits, int n_bs, int n_qubits,
                                                       uint64_t* __restrict__ packed, unsigned* __restrict__ counter) {
  const int tid = threadIdx.x;
  if (tid == 0 && counter) *counter = 0u;
  for (int b = tid; b < n_bs; b += blockDim.x) {
    uint64_t w = 0;
    for (int q = 0; q < n_qubits; ++q) w |= (uint64_t)(bits[(size_t)b * n_qubits + q] & 1) << q;
    packed[b] = w;
  }
  for (int e = tid; e < n_raw; e += blockDim.x) {
    cx<R> v;
    int p = rawp[e];
    if (p >= 0) {
      // RZ(theta) entry e^{i phi}, phi = theta (2u - 1) / 2; derivative tables
      // hold d/dtheta of it, (i/2)(2u - 1) e^{i phi}.
      const double sgn = 2.0 * rawb[e] - 1.0;
      const double phi = 0.5 * params[p] * sgn;
      double sn, cs;
      sincos(phi, &sn, &cs);
      if (rawd[e]) {
        v.x = (R)(-0.5 * sgn * sn);
        v.y = (R)(0.5 * sgn * cs);
      } else {
        v.x = (R)cs;
        v.y = (R)sn;
      }
    } else {
      v.x = (R)raw[2 * e];
      v.y = (R)raw[2 * e + 1];
    }
    cst[e] = v;
  }
  __syncthreads();
  for (int si = 0; si < n_const_steps; ++si) {
    const DevStep st = steps[si];
    const int nc = 1 << st.r, nsum = 1 << st.ns;
    for (int c = tid; c < nc; c += blockDim.x) {
      cx<R> acc{0, 0};
      const uint32_t* op = optab + st.ops + (size_t)c * nsum * st.m;
      for (int s = 0; s < nsum; ++s) {
        cx<R> prod = cst[op[0] & ~kConst];
        for (int i = 1; i < st.m; ++i) prod = cmul(prod, cst[op[i] & ~kConst]);
        op += st.m;
        acc.x += prod.x;
        acc.y += prod.y;
      }
      cst[st.out + c] = acc;
    }
    __syncthreads();
  }
}

// --------------------------------------------------------- chain (per item)
template <typename R, bool LDS>
__global__ void __launch_bounds__(64) chain_kernel(const DevStep* __restrict__ steps, int first_step, int n_steps,
                                                   const DevLeaf* __restrict__ leaves,
                                                   const uint32_t* __restrict__ optab,
                                                   const cx<R>* __restrict__ cst,
                                                   const uint64_t* __restrict__ packed, int n_bs,
                                                   uint64_t s_begin, uint64_t n_s, uint64_t n_items,
                                                   unsigned* __restrict__ counter, cx<R>* __restrict__ res,
                                                   cx<R>* __restrict__ gres, cx<R>* __restrict__ gscratch,
                                                   int item_elems) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  cx<R>* mem = LDS ? reinterpret_cast<cx<R>*>(lds_raw)
                   : gscratch + (size_t)blockIdx.x * (size_t)item_elems * kLanes;
  const int lane = threadIdx.x;
  __shared__ unsigned chunk_sh;
  const uint64_t n_chunks = (n_items + kLanes - 1) / kLanes;
  for (;;) {
    if (lane == 0) chunk_sh = atomicAdd(counter, 1u);
    __syncthreads();
    const uint64_t chunk = chunk_sh;
    __syncthreads();
    if (chunk >= n_chunks) break;
    uint64_t item = chunk * kLanes + lane;
    const bool valid = item < n_items;
    if (!valid) item = n_items - 1;
    const uint64_t b = item / n_s;
    const uint64_t sl = item - b * n_s;
    const uint64_t s = s_begin + sl;
    const uint64_t xb = packed[b];
    for (int si = first_step; si < n_steps; ++si) {
      const DevStep st = steps[si];
      if (st.kind == 0) {
        const DevLeaf L = leaves[st.leaf];
        int lane_off = 0;
        for (int j = 0; j < L.ndep; ++j) {
          const uint64_t w = L.src[j] ? s : xb;
          lane_off += (int)((w >> L.bit[j]) & 1) * L.ds[j];
        }
        const int nc = 1 << st.r;
        for (int c = 0; c < nc; ++c) {
          int off = L.table + lane_off;
          for (int j = 0; j < L.nfree; ++j) off += ((c >> j) & 1) * L.fs[j];
          mem[(size_t)(st.out + c) * kLanes + lane] = cst[off];
        }
      } else {
        const int nc = 1 << st.r, nsum = 1 << st.ns;
        const uint32_t* op = optab + st.ops;
        for (int c = 0; c < nc; ++c) {
          cx<R> acc{0, 0};
          for (int s2 = 0; s2 < nsum; ++s2) {
            cx<R> prod{1, 0};
            for (int i = 0; i < st.m; ++i) {
              const uint32_t e = op[i];
              cx<R> v;
              if (e & kConst)
                v = cst[e & ~kConst];
              else
                v = mem[(size_t)e * kLanes + lane];
              prod = (i == 0) ? v : cmul(prod, v);
            }
            op += st.m;
            acc.x += prod.x;
            acc.y += prod.y;
          }
          if (st.kind == 2) {  // rank r: 2^r amplitudes per item (open outputs)
            if (valid) res[((sl * (uint64_t)n_bs + b) << st.r) + c] = acc;
          } else if (st.kind == 3) {
            if (valid) gres[((uint64_t)st.grad_slot * n_s + sl) * (uint64_t)n_bs + b] = acc;
          } else {
            mem[(size_t)(st.out + c) * kLanes + lane] = acc;
          }
        }
      }
    }
  }
}

// ------------------------------------------------------------ reduction
// alpha_x = sum over slices, ascending s, in FP64 with Neumaier's
// compensation (improved Kahan summation).  partial = (sum, comp) per part.
__device__ __forceinline__ void neumaier(double& sum, double& comp, double x) {
  double t = sum + x;
  if (fabs(sum) >= fabs(x))
    comp += (sum - t) + x;
  else
    comp += (x - t) + sum;
  sum = t;
}

// Knuth's TwoSum: s + e equals a + b exactly.
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bv = s - a;
  e = (a - (s - bv)) + (b - bv);
}

// Compensated butterfly over the 64 lanes of a wavefront (partners lane ^ 1,
// ^ 2, ..., ^ 32).  Every lane ends with the same (sum, comp); sum + comp is
// the total of the 64 inputs.  Addition is commutative and TwoSum's error is
// exact, so partners compute identical values and the order is fixed.
__device__ __forceinline__ void wave_sum(double& s, double& c) {
  for (int m = 1; m < 64; m <<= 1) {
    const double so = __shfl_xor(s, m);
    const double co = __shfl_xor(c, m);
    double t, e;
    two_sum(s, so, t, e);
    s = t;
    c = (c + co) + e;
  }
}

// Slice sums, one order for every path: slices are taken in chunks of 64
// consecutive s (the last chunk padded with zeros); a chunk is summed by the
// compensated butterfly into (sum_c, comp_c); the chunk sums are then added in
// ascending chunk order with Neumaier's compensation and the chunk
// compensations are accumulated alongside.  One 64-lane block per bitstring.
template <typename R>
__global__ void __launch_bounds__(64) reduce_kernel(const cx<R>* __restrict__ res, int n_bs, uint64_t n_s,
                                                    double* __restrict__ partial) {
  const int b = blockIdx.x, lane = threadIdx.x;
  double S[2] = {0, 0}, SC[2] = {0, 0}, CC[2] = {0, 0};
  for (uint64_t c0 = 0; c0 < n_s; c0 += 64) {
    double v[2] = {0, 0}, c[2] = {0, 0};
    if (c0 + lane < n_s) {
      cx<R> x = res[(c0 + lane) * (uint64_t)n_bs + b];
      v[0] = (double)x.x;
      v[1] = (double)x.y;
    }
    for (int k = 0; k < 2; ++k) {
      wave_sum(v[k], c[k]);
      neumaier(S[k], SC[k], v[k]);
      CC[k] += c[k];
    }
  }
  if (lane == 0) {
    partial[4 * b + 0] = S[0];
    partial[4 * b + 1] = S[1];
    partial[4 * b + 2] = SC[0] + CC[0];
    partial[4 * b + 3] = SC[1] + CC[1];
  }
}

// Chunk partials [b][chunk][4] written by the generated kernel (same chunk
// sums as above) -> per-bitstring partial.
// Resets the persistent chain kernel's work-queue counter (a fill kernel
// rather than a memset, so captured graphs replay it correctly).
__global__ void zero_counter_kernel(unsigned* __restrict__ counter) { *counter = 0u; }

__global__ void combine_kernel(const double* __restrict__ chunks, int n_bs, uint64_t per_bs,
                               double* __restrict__ partial) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_bs) return;
  double S[2] = {0, 0}, SC[2] = {0, 0}, CC[2] = {0, 0};
  const double* p = chunks + (size_t)b * per_bs * 4;
  for (uint64_t c = 0; c < per_bs; ++c) {
    for (int j = 0; j < 2; ++j) {
      neumaier(S[j], SC[j], p[4 * c + j]);
      CC[j] += p[4 * c + 2 + j];
    }
  }
  partial[4 * b + 0] = S[0];
  partial[4 * b + 1] = S[1];
  partial[4 * b + 2] = SC[0] + CC[0];
  partial[4 * b + 3] = SC[1] + CC[1];
}

// d alpha / d theta_j per bitstring: every gradient slot of parameter j
// (slots ascending) is summed over the slices in the order used for the
// amplitudes.  One 64-lane block per (bitstring, parameter).
template <typename R>
__global__ void __launch_bounds__(64) grad_reduce_kernel(const cx<R>* __restrict__ gres, int n_bs, uint64_t n_s,
                                                         int n_slots, const int* __restrict__ slot_param,
                                                         int n_params, double* __restrict__ out) {
  const int t = blockIdx.x, lane = threadIdx.x;
  const int b = t / n_params, j = t - b * n_params;
  double S[2] = {0, 0}, SC[2] = {0, 0}, CC[2] = {0, 0};
  for (int g = 0; g < n_slots; ++g) {
    if (slot_param[g] != j) continue;
    const cx<R>* base = gres + (uint64_t)g * n_s * (uint64_t)n_bs;
    for (uint64_t c0 = 0; c0 < n_s; c0 += 64) {
      double v[2] = {0, 0}, c[2] = {0, 0};
      if (c0 + lane < n_s) {
        cx<R> x = base[(c0 + lane) * (uint64_t)n_bs + b];
        v[0] = (double)x.x;
        v[1] = (double)x.y;
      }
      for (int k = 0; k < 2; ++k) {
        wave_sum(v[k], c[k]);
        neumaier(S[k], SC[k], v[k]);
        CC[k] += c[k];
      }
    }
  }
  if (lane == 0) {
    out[4 * (size_t)t + 0] = S[0];
    out[4 * (size_t)t + 1] = S[1];
    out[4 * (size_t)t + 2] = SC[0] + CC[0];
    out[4 * (size_t)t + 3] = SC[1] + CC[1];
  }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

int dev_query(int& n_cu, size_t& max_lds, std::string& err) {
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  HIP_OK(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  int lds = 0;
  HIP_OK(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  max_lds = (size_t)lds;
  return 0;
}

int dev_upload(const Program& prog, const std::vector<char>& code, const WideProgram* wide, DevProgram& dp,
               std::string& err, const std::vector<char>* wide_code, const std::vector<WideKernel>* wide_kernels) {
  if (dp.steps) return 0;
  if (wide && wide_code && !wide_code->empty() && wide_kernels) {
    hipModule_t mod = nullptr;
    HIP_OK(hipModuleLoadData(&mod, wide_code->data()));
    dp.wide.module = mod;
    for (const WideKernel& k : *wide_kernels) {
      hipFunction_t fn = nullptr;
      HIP_OK(hipModuleGetFunction(&fn, mod, k.name.c_str()));
      if (k.kind == 0)
        dp.wide.levels.push_back({fn, k.blocks, k.threads});
      else  // generated constant-step kernels, in step order
        dp.wide.const_plan.push_back({k.kind == 1 ? 1 : 0, k.steps.front(), (int)k.steps.size(), fn, k.blocks});
    }
  }
  if (wide) {
    HIP_OK(hipMalloc(&dp.wide.steps, std::max<size_t>(wide->steps.size() * sizeof(int32_t), 16)));
    HIP_OK(hipMalloc(&dp.wide.ops, std::max<size_t>(wide->ops.size() * sizeof(int32_t), 16)));
    if (!wide->steps.empty())
      HIP_OK(hipMemcpy(dp.wide.steps, wide->steps.data(), wide->steps.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    if (!wide->ops.empty())
      HIP_OK(hipMemcpy(dp.wide.ops, wide->ops.data(), wide->ops.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    dp.wide.n_steps = wide->n_steps;
    dp.wide.host_steps = wide->steps;
    std::vector<int32_t> list;
    if (dp.wide.const_plan.empty()) {  // no generated constant kernels: prebuilt ones
      for (int si = 0; si < wide->n_steps; ++si) {
        if (!wide->steps[8 * si + 7]) continue;
        if (wide->steps[8 * si + 2] <= 14) {
          if (dp.wide.const_plan.empty() || !dp.wide.const_plan.back().block)
            dp.wide.const_plan.push_back({1, (int)list.size(), 0, nullptr, 0});
          list.push_back(si);
          dp.wide.const_plan.back().count++;
        } else {
          dp.wide.const_plan.push_back({0, si, 1, nullptr, 0});
        }
      }
    }
    HIP_OK(hipMalloc(&dp.wide.const_list, std::max<size_t>(list.size() * sizeof(int32_t), 16)));
    if (!list.empty())
      HIP_OK(hipMemcpy(dp.wide.const_list, list.data(), list.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  }
  if (!code.empty()) {
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;
    HIP_OK(hipModuleLoadData(&mod, code.data()));
    hipError_t e = hipModuleGetFunction(&fn, mod, "qgm_chain");
    if (e != hipSuccess) {
      (void)hipModuleUnload(mod);
      err = std::string("hipModuleGetFunction: ") + hipGetErrorString(e);
      return -6;
    }
    dp.module = mod;
    dp.chain_fn = fn;
  }
  HIP_OK(hipGetDevice(&dp.device));
  int rc = dev_query(dp.n_cu, dp.max_lds, err);
  if (rc) return rc;
  std::vector<DevStep> ds(prog.steps.size());
  for (size_t i = 0; i < prog.steps.size(); ++i) {
    const Step& s = prog.steps[i];
    ds[i] = DevStep{s.kind, s.out, s.r, s.ns, s.m, s.ops, s.leaf, s.grad_slot};
  }
  std::vector<DevLeaf> dl(prog.leaves.size());
  for (size_t i = 0; i < prog.leaves.size(); ++i) {
    const Leaf& L = prog.leaves[i];
    DevLeaf d{};
    d.nfree = L.nfree;
    d.ndep = L.ndep;
    d.table = L.table;
    for (int j = 0; j < 4; ++j) {
      d.fs[j] = j < L.nfree ? L.free_stride[j] : 0;
      d.src[j] = j < L.ndep ? L.dep_src[j] : 0;
      d.bit[j] = j < L.ndep ? L.dep_bit[j] : 0;
      d.ds[j] = j < L.ndep ? L.dep_stride[j] : 0;
    }
    dl[i] = d;
  }
  auto up = [&](void** dst, const void* src, size_t bytes) -> int {
    HIP_OK(hipMalloc(dst, std::max<size_t>(bytes, 16)));
    if (bytes) HIP_OK(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
    return 0;
  };
  if ((rc = up(&dp.raw, prog.raw.data(), prog.raw.size() * sizeof(double)))) return rc;
  if ((rc = up(&dp.rawp, prog.raw_param.data(), prog.raw_param.size() * sizeof(int)))) return rc;
  if ((rc = up(&dp.rawb, prog.raw_bit.data(), prog.raw_bit.size() * sizeof(int)))) return rc;
  if ((rc = up(&dp.rawd, prog.raw_deriv.data(), prog.raw_deriv.size() * sizeof(int)))) return rc;
  if ((rc = up(&dp.slot_param, prog.grad_param.data(), prog.grad_param.size() * sizeof(int)))) return rc;
  if ((rc = up(&dp.leaves, dl.data(), dl.size() * sizeof(DevLeaf)))) return rc;
  if ((rc = up(&dp.optab, prog.optab.data(), prog.optab.size() * sizeof(uint32_t)))) return rc;
  if ((rc = up(&dp.steps, ds.data(), ds.size() * sizeof(DevStep)))) return rc;
  dp.n_steps = (int)prog.steps.size();
  dp.n_const_steps = prog.n_const_steps;
  return 0;
}

namespace {
template <typename R>
int cache_constants_typed(const Program& prog, DevProgram& dp, int wide, std::string& err) {
  const size_t bytes = std::max<size_t>((size_t)std::max(prog.n_const, 1) * sizeof(cx<R>), 256);
  HIP_OK(hipMalloc(&dp.cst_cache, bytes));
  hipStream_t st = nullptr;
  HIP_OK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  auto* cst = (cx<R>*)dp.cst_cache;
  // no bitstrings: the prologue writes the raw tables and runs the constant
  // steps (the interpreter's); the wide engine's constant kernels follow
  hipLaunchKernelGGL(prologue_kernel<R>, dim3(1), dim3(256), 0, st, (const double*)dp.raw, (const int*)dp.rawp,
                     (const int*)dp.rawb, (const int*)dp.rawd, prog.n_raw, (const double*)nullptr,
                     (const DevStep*)dp.steps, wide ? 0 : dp.n_const_steps, (const uint32_t*)dp.optab, cst,
                     (const uint8_t*)nullptr, 0, 0, (uint64_t*)nullptr, (unsigned*)nullptr);
  int rc = 0;
  if (wide && wide_launch_steps<R>(dp.wide, 0, 0, cst, nullptr, 0, nullptr, 0, 0, 1, 0, nullptr, nullptr, true, st))
    rc = -6;
  hipError_t e = hipStreamSynchronize(st);
  (void)hipStreamDestroy(st);
  if (rc || e != hipSuccess) {
    err = "constant steps at upload failed";
    return -6;
  }
  dp.cst_cached = 1;
  return 0;
}
}  // namespace

int dev_cache_constants(const Program& prog, DevProgram& dp, int prec, int wide, std::string& err) {
  if (dp.cst_cached) return 0;
  return prec == 0 ? cache_constants_typed<double>(prog, dp, wide, err)
                   : prec == 2 ? cache_constants_typed<bfx3>(prog, dp, wide, err)
                               : cache_constants_typed<float>(prog, dp, wide, err);
}

void dev_free(DevProgram& dp) {
  void* ps[] = {dp.raw, dp.rawp, dp.rawb, dp.rawd, dp.slot_param, dp.steps, dp.leaves, dp.optab};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  if (dp.module) (void)hipModuleUnload((hipModule_t)dp.module);
  if (dp.wide.steps) (void)hipFree(dp.wide.steps);
  if (dp.wide.const_list) (void)hipFree(dp.wide.const_list);
  if (dp.wide.module) (void)hipModuleUnload((hipModule_t)dp.wide.module);
  if (dp.wide.ops) (void)hipFree(dp.wide.ops);
  if (dp.cst_cache) (void)hipFree(dp.cst_cache);
  dp = DevProgram();
}

int dev_layout(const Program& prog, const DevProgram& dp, const LaunchCfg& cfg, WsLayout& ws, std::string& err) {
  const size_t el = cfg.prec == 0 ? 16 : 8;
  const uint64_t n_items = (uint64_t)cfg.n_bs * cfg.n_s;
  const uint64_t n_chunks = (n_items + kLanes - 1) / kLanes;
  ws.fused = (cfg.generated && cfg.n_s % kLanes == 0 && prog.n_open == 0) ? 1 : 0;
  size_t lds = (size_t)prog.item_elems * kLanes * el;
  if (cfg.generated) lds = 0;
  // 64 bytes of headroom for the kernel's static LDS (the work-queue slot)
  if (cfg.wide) lds = 0;
  ws.use_lds = (!cfg.generated && !cfg.wide && lds + 64 <= dp.max_lds) ? 1 : 0;
  ws.lds_bytes = ws.use_lds ? lds : 0;
  int per_cu = 8;
  if (ws.use_lds) {
    int occ = 0;
    hipError_t e = cfg.prec == 0   ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, chain_kernel<double, true>, 64, lds)
                   : cfg.prec == 2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, chain_kernel<bfx3, true>, 64, lds)
                                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, chain_kernel<float, true>, 64, lds);
    if (e != hipSuccess || occ <= 0) occ = (int)std::max<size_t>(1, dp.max_lds / std::max<size_t>(lds, 1));
    per_cu = std::min(occ, 8);
    if (lds > 65536) {
      if (cfg.prec == 0)
        (void)hipFuncSetAttribute((const void*)chain_kernel<double, true>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      else if (cfg.prec == 2)
        (void)hipFuncSetAttribute((const void*)chain_kernel<bfx3, true>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      else
        (void)hipFuncSetAttribute((const void*)chain_kernel<float, true>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    }
  }
  uint64_t grid = (uint64_t)std::max(1, dp.n_cu) * per_cu;
  if (grid > n_chunks) grid = n_chunks;
  if (grid == 0) grid = 1;
  ws.grid = (int)grid;
  size_t off = 0;
  ws.cst = off;
  off = align256(off + (size_t)std::max(prog.n_const, 1) * el);
  ws.bits = off;
  off = align256(off + (size_t)std::max(cfg.n_bs, 1) * 8);
  ws.res = off;  // 2^n_open amplitudes per item (open outputs)
  off = align256(off + ((size_t)std::max<uint64_t>(n_items, 1) << prog.n_open) * el);
  ws.gres = off;
  off = align256(off + (size_t)prog.n_grad_slots * n_items * el);
  ws.counter = off;
  off = align256(off + 256);
  ws.chunks = off;
  off = align256(off + (size_t)std::max<uint64_t>(n_chunks, 1) * 4 * sizeof(double));
  ws.scratch = off;
  ws.wide_groups = 0;
  if (cfg.wide) {
    const uint64_t groups = std::max<uint64_t>(n_chunks, 1);
    const size_t per_group = (size_t)prog.item_elems * kLanes * el;
    uint64_t fit = cfg.wide_budget / std::max<size_t>(per_group, 1);
    if (fit < 1) {
      err = "one 64-item group needs " + std::to_string(per_group) + " bytes of item memory, over the budget";
      return -5;
    }
    ws.wide_groups = (int)std::min<uint64_t>(groups, std::min<uint64_t>(fit, 65535));
    off = align256(off + (size_t)ws.wide_groups * per_group);
  } else if (!cfg.generated && !ws.use_lds) {
    off = align256(off + (size_t)ws.grid * prog.item_elems * kLanes * el);
  }
  ws.total = off;
  (void)err;
  return 0;
}

namespace {

template <typename R>
int run_typed(const Program& prog, const DevProgram& dp, const LaunchCfg& cfg, const WsLayout& ws,
              const uint8_t* d_bits, const double* d_params, char* base, hipStream_t stream, double* d_partial,
              double* d_grad_partial, void* const* events, std::string& err) {
  auto mark = [&](int i) {
    if (events) (void)hipEventRecord((hipEvent_t)events[i], stream);
  };
  const uint64_t n_items = (uint64_t)cfg.n_bs * cfg.n_s;
  // amplitudes per call: 2^n_open per bitstring, item results laid out as
  // [slice][bitstring][amplitude], so each amplitude reduces like a bitstring
  const int n_amp_bs = cfg.n_bs << prog.n_open;
  auto* packed = (uint64_t*)(base + ws.bits);
  auto* counter = (unsigned*)(base + ws.counter);
  // plans without angles read the constants contracted at upload
  auto* cst = dp.cst_cached ? (cx<R>*)dp.cst_cache : (cx<R>*)(base + ws.cst);
  auto* res = (cx<R>*)(base + ws.res);
  auto* gres = (cx<R>*)(base + ws.gres);
  auto* scr = (cx<R>*)(base + ws.scratch);
  auto* chunks = (double*)(base + ws.chunks);
  const int first = dp.n_const_steps;
  const dim3 red_grid((cfg.n_bs + 63) / 64);
  const bool grads = prog.n_grad_slots > 0 && d_grad_partial != nullptr;
  auto grad_reduce = [&]() {
    if (!grads) return;
    const int n = cfg.n_bs * cfg.n_params;
    hipLaunchKernelGGL(grad_reduce_kernel<R>, dim3(n), dim3(64), 0, stream, gres, cfg.n_bs, cfg.n_s,
                       prog.n_grad_slots, (const int*)dp.slot_param, cfg.n_params, d_grad_partial);
  };
  mark(0);
  // The generated kernel reads the FP64 tables and the bitstring bytes itself.
  // (with cached constants only the bitstrings are packed)
  if (!cfg.generated || n_items == 0)
    hipLaunchKernelGGL(prologue_kernel<R>, dim3(1), dim3(256), 0, stream, (const double*)dp.raw, (const int*)dp.rawp,
                       (const int*)dp.rawb, (const int*)dp.rawd, dp.cst_cached ? 0 : prog.n_raw, d_params,
                       (const DevStep*)dp.steps, (cfg.wide || dp.cst_cached) ? 0 : dp.n_const_steps,
                       (const uint32_t*)dp.optab, cst, d_bits, cfg.n_bs, cfg.n_qubits, packed, counter);
  if (cfg.wide && !dp.cst_cached &&
      wide_launch_steps<R>(dp.wide, 0, 0, cst, nullptr, 0, packed, cfg.n_bs, cfg.s_begin, cfg.n_s, n_items, res,
                           gres, true, stream)) {
    err = "wide constant steps: launch failed";
    return -6;
  }
  mark(1);
  if (n_items == 0) {
    mark(2);
    hipLaunchKernelGGL(reduce_kernel<R>, dim3(n_amp_bs), dim3(64), 0, stream, res, n_amp_bs, cfg.n_s, d_partial);
    grad_reduce();
    mark(3);
    HIP_OK(hipGetLastError());
    return 0;
  }
  if (cfg.wide) {
    const uint64_t n_groups = (n_items + kLanes - 1) / kLanes;
    for (uint64_t g0 = 0; g0 < n_groups; g0 += (uint64_t)ws.wide_groups) {
      const int ng = (int)std::min<uint64_t>((uint64_t)ws.wide_groups, n_groups - g0);
      if (wide_launch_steps<R>(dp.wide, (int)g0, ng, cst, scr, (uint64_t)prog.item_elems, packed, cfg.n_bs,
                               cfg.s_begin, cfg.n_s, n_items, res, gres, false, stream)) {
        err = "wide steps: launch failed";
        return -6;
      }
    }
    mark(2);
    hipLaunchKernelGGL(reduce_kernel<R>, dim3(n_amp_bs), dim3(64), 0, stream, res, n_amp_bs, cfg.n_s, d_partial);
    grad_reduce();
    mark(3);
  } else if (cfg.generated) {
    const uint64_t n_blocks = (n_items + kLanes - 1) / kLanes;
    const uint64_t per_bs = cfg.n_s / kLanes;
    // With one block per bitstring the block partial is the final partial.
    double* part = (ws.fused && per_bs == 1) ? d_partial : chunks;
    unsigned long long a_nbs = (unsigned long long)cfg.n_bs, a_sb = cfg.s_begin, a_ns = cfg.n_s, a_ni = n_items;
    const void* a_raw = dp.raw;
    const void* a_par = d_params;
    const void* a_bits = d_bits;
    int a_nq = cfg.n_qubits;
    void* a_res = res;
    void* a_gres = gres;
    void* a_part = part;
    int a_fused = ws.fused;
    int a_log2 = (cfg.n_s & (cfg.n_s - 1)) == 0 ? __builtin_ctzll(cfg.n_s) : -1;
    void* a_queue = counter;
    void* args[] = {&a_bits, &a_ns, &a_sb, &a_ni, &a_nbs, &a_nq, &a_fused, &a_log2, &a_par, &a_res, &a_gres, &a_part,
                    &a_raw, &a_queue};
    uint64_t grid = n_blocks;
    if (dp.chain_persistent) {
      // resident blocks only; the rest of the chunks come from the queue
      int occ = 0;
      if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (hipFunction_t)dp.chain_fn,
                                                             kLanes * dp.chain_waves, 0) != hipSuccess || occ < 1)
        occ = 1;
      grid = std::min<uint64_t>(n_blocks, (uint64_t)std::max(1, dp.n_cu) * (uint64_t)occ);
      hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(1), 0, stream, counter);
    }
    HIP_OK(hipModuleLaunchKernel((hipFunction_t)dp.chain_fn, (unsigned)grid, 1, 1, kLanes * dp.chain_waves, 1,
                                 1, 0, stream, args, nullptr));
    mark(2);
    if (!ws.fused)
      hipLaunchKernelGGL(reduce_kernel<R>, dim3(n_amp_bs), dim3(64), 0, stream, res, n_amp_bs, cfg.n_s, d_partial);
    else if (per_bs > 1)
      hipLaunchKernelGGL(combine_kernel, red_grid, dim3(64), 0, stream, chunks, cfg.n_bs, per_bs, d_partial);
    grad_reduce();
    mark(3);
  } else {
    if (ws.use_lds)
      hipLaunchKernelGGL((chain_kernel<R, true>), dim3(ws.grid), dim3(64), ws.lds_bytes, stream,
                         (const DevStep*)dp.steps, first, dp.n_steps, (const DevLeaf*)dp.leaves,
                         (const uint32_t*)dp.optab, cst, packed, cfg.n_bs, cfg.s_begin, cfg.n_s, n_items, counter, res,
                         gres, scr, prog.item_elems);
    else
      hipLaunchKernelGGL((chain_kernel<R, false>), dim3(ws.grid), dim3(64), 0, stream, (const DevStep*)dp.steps,
                         first, dp.n_steps, (const DevLeaf*)dp.leaves, (const uint32_t*)dp.optab, cst, packed,
                         cfg.n_bs, cfg.s_begin, cfg.n_s, n_items, counter, res, gres, scr, prog.item_elems);
    mark(2);
    hipLaunchKernelGGL(reduce_kernel<R>, dim3(n_amp_bs), dim3(64), 0, stream, res, n_amp_bs, cfg.n_s, d_partial);
    grad_reduce();
    mark(3);
  }
  HIP_OK(hipGetLastError());
  return 0;
}

}  // namespace

int dev_run(const Program& prog, const DevProgram& dp, const LaunchCfg& cfg, const WsLayout& ws,
            const uint8_t* d_bits, const double* d_params, void* d_ws, void* stream_, double* d_partial,
            double* d_grad_partial, void* const* events, std::string& err) {
  if (cfg.n_bs == 0) return 0;
  if (cfg.wide && !dp.wide.steps) {
    err = "wide engine descriptors not loaded";
    return -6;
  }
  if (cfg.generated && !dp.chain_fn) {
    err = "generated kernel not loaded";
    return -6;
  }
  hipStream_t stream = (hipStream_t)stream_;
  if (cfg.prec == 2)
    return run_typed<bfx3>(prog, dp, cfg, ws, d_bits, d_params, (char*)d_ws, stream, d_partial, d_grad_partial, events,
                           err);
  if (cfg.prec == 0)
    return run_typed<double>(prog, dp, cfg, ws, d_bits, d_params, (char*)d_ws, stream, d_partial, d_grad_partial,
                             events, err);
  return run_typed<float>(prog, dp, cfg, ws, d_bits, d_params, (char*)d_ws, stream, d_partial, d_grad_partial, events,
                          err);
}

}  // namespace qgm
