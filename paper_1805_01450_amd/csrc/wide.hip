// Wide engine kernels: one launch per elimination step for plans whose
// tensors are too large for registers or LDS.
//
// Item tensors live in HBM as [element][64 items] rows (items = the
// (bitstring, slice) pairs of a group of 64), so every wavefront load or
// store is one contiguous 64-lane row whatever the tensor's variable order:
// no permutation is ever needed.  A wavefront computes `cpw` consecutive
// output elements for its 64 items; operand offsets are wave-uniform.
// Constant steps (no fixed variable) run with one thread per output element.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "bfx3.h"
#include "exec.h"

namespace qgm {

namespace {

template <typename R>
struct cw {
  R x, y;
};

template <typename R>
__device__ __forceinline__ cw<R> wmul(cw<R> a, cw<R> b) {
  cw<R> c;
  c.x = a.x * b.x - a.y * b.y;
  c.y = a.x * b.y + a.y * b.x;
  return c;
}

constexpr int kOp = kWideOpInts;
constexpr int kMaxOps = 64;  // operands whose high-bit offset is cached per wave

template <typename R>
__global__ void __launch_bounds__(256) wide_step_kernel(const int* __restrict__ steps, int si,
                                                        const int* __restrict__ ops, const cw<R>* __restrict__ cst,
                                                        cw<R>* __restrict__ mem, uint64_t group_elems, int group0,
                                                        const uint64_t* __restrict__ packed, int n_bs,
                                                        uint64_t s_begin, uint64_t n_s, uint64_t n_items,
                                                        cw<R>* __restrict__ res, cw<R>* __restrict__ gres,
                                                        int cpw_log2) {
  const int lane = threadIdx.x & 63;
  const int wib = threadIdx.x >> 6;
  const uint64_t wave = (uint64_t)blockIdx.x * 4 + wib;
  const int* st = steps + 8 * si;
  const int kind = st[0], out = st[1], r = st[2], ns = st[3], m = st[4], slot = st[5], ob = st[6];
  const uint64_t nc = 1ull << r;
  const uint64_t c_begin = wave << cpw_log2;
  // per-wave offset of each operand at c_begin (high bits); lanes share it
  __shared__ long long hoff[4][kMaxOps];
  if (lane < m && lane < kMaxOps && c_begin < nc) {
    const int* op = ops + (size_t)(ob + lane) * kOp;
    long long off = op[1];
    for (int j = cpw_log2; j < r; ++j)
      if ((c_begin >> j) & 1) off += op[16 + j];
    hoff[wib][lane] = off;
  }
  __syncthreads();
  if (c_begin >= nc) return;
  const uint64_t c_end = c_begin + (1ull << cpw_log2) < nc ? c_begin + (1ull << cpw_log2) : nc;
  const uint64_t g = (uint64_t)group0 + blockIdx.y;
  uint64_t item = g * 64 + lane;
  const bool valid = item < n_items;
  if (!valid) item = n_items - 1;
  const uint64_t b = item / n_s;
  const uint64_t sl = item - b * n_s;
  const uint64_t s = s_begin + sl;
  const uint64_t xb = packed[b];
  cw<R>* gmem = mem + (uint64_t)blockIdx.y * group_elems * 64;
  for (uint64_t c = c_begin; c < c_end; ++c) {
    const int lo = (int)(c - c_begin);
    cw<R> acc{0, 0};
    for (int s2 = 0; s2 < (1 << ns); ++s2) {
      cw<R> prod{1, 0};
      for (int i = 0; i < m; ++i) {
        const int* op = ops + (size_t)(ob + i) * kOp;
        long long off;
        if (i < kMaxOps) {
          off = hoff[wib][i];
          for (int j = 0; j < cpw_log2; ++j)
            if ((lo >> j) & 1) off += op[16 + j];
        } else {
          off = op[1];
          for (int j = 0; j < r; ++j)
            if ((c >> j) & 1) off += op[16 + j];
        }
        for (int j = 0; j < ns; ++j)
          if ((s2 >> j) & 1) off += op[48 + j];
        cw<R> v;
        const int k = op[0];
        if (k == WOP_ITEM) {
          v = gmem[(uint64_t)off * 64 + lane];
        } else if (k == WOP_CONST) {
          v = cst[off];
        } else {
          long long d = 0;
          for (int j = 0; j < op[2]; ++j) {
            const uint64_t w = op[3 + j] ? s : xb;
            d += (long long)((w >> op[7 + j]) & 1) * op[11 + j];
          }
          v = cst[off + d];
        }
        prod = i == 0 ? v : wmul(prod, v);
      }
      acc.x += prod.x;
      acc.y += prod.y;
    }
    if (kind == ST_ELIM)
      gmem[(uint64_t)(out + c) * 64 + lane] = acc;
    else if (kind == ST_FINAL) {  // rank r: 2^r amplitudes per item (open outputs)
      if (valid) res[((sl * (uint64_t)n_bs + b) << r) + c] = acc;
    } else if (kind == ST_GRAD) {
      if (valid) gres[((uint64_t)slot * n_s + sl) * (uint64_t)n_bs + b] = acc;
    }
  }
}

template <typename R>
__global__ void __launch_bounds__(256) const_step_kernel(const int* __restrict__ steps, int si,
                                                         const int* __restrict__ ops, cw<R>* __restrict__ cst) {
  const int* st = steps + 8 * si;
  const int out = st[1], r = st[2], ns = st[3], m = st[4], ob = st[6];
  const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (1ull << r)) return;
  cw<R> acc{0, 0};
  for (int s2 = 0; s2 < (1 << ns); ++s2) {
    cw<R> prod{1, 0};
    for (int i = 0; i < m; ++i) {
      const int* op = ops + (size_t)(ob + i) * kOp;
      long long off = op[1];
      for (int j = 0; j < r; ++j)
        if ((c >> j) & 1) off += op[16 + j];
      for (int j = 0; j < ns; ++j)
        if ((s2 >> j) & 1) off += op[48 + j];
      const cw<R> v = cst[off];
      prod = i == 0 ? v : wmul(prod, v);
    }
    acc.x += prod.x;
    acc.y += prod.y;
  }
  cst[out + c] = acc;
}

// A run of small constant steps in one block of 1024 threads, one step after
// the other (each step reads only constants written before it).
template <typename R>
__global__ void __launch_bounds__(1024) const_block_kernel(const int* __restrict__ steps, const int* __restrict__ list,
                                                           int n_list, const int* __restrict__ ops,
                                                           cw<R>* __restrict__ cst) {
  for (int li = 0; li < n_list; ++li) {
    const int* st = steps + 8 * list[li];
    const int out = st[1], r = st[2], ns = st[3], m = st[4], ob = st[6];
    for (uint64_t c = threadIdx.x; c < (1ull << r); c += blockDim.x) {
      cw<R> acc{0, 0};
      for (int s2 = 0; s2 < (1 << ns); ++s2) {
        cw<R> prod{1, 0};
        for (int i = 0; i < m; ++i) {
          const int* op = ops + (size_t)(ob + i) * kOp;
          long long off = op[1];
          for (int j = 0; j < r; ++j)
            if ((c >> j) & 1) off += op[16 + j];
          for (int j = 0; j < ns; ++j)
            if ((s2 >> j) & 1) off += op[48 + j];
          const cw<R> v = cst[off];
          prod = i == 0 ? v : wmul(prod, v);
        }
        acc.x += prod.x;
        acc.y += prod.y;
      }
      cst[out + c] = acc;
    }
    __syncthreads();
  }
}

}  // namespace

int wide_cpw_log2(int r) {
  // enough wavefronts per step to fill the GPU, up to 64 elements each
  int l = r - 13;
  return l < 0 ? 0 : (l > 6 ? 6 : l);
}

template <typename R>
int wide_launch_steps(const WideDev& wd, int first_group, int n_groups, const void* cst, void* mem,
                      uint64_t group_elems, const uint64_t* packed, int n_bs, uint64_t s_begin, uint64_t n_s,
                      uint64_t n_items, void* res, void* gres, bool const_steps, hipStream_t stream) {
  if (const_steps) {
    // runs of small constant steps share one single-block launch; large ones
    // get a launch of their own (plan made at upload, in step order)
    for (const WideDev::ConstLaunch& cl : wd.const_plan) {
      if (cl.fn) {
        void* a_cst = const_cast<void*>(cst);
        void* args[] = {&a_cst};
        const unsigned blocks = cl.block ? 1u : (unsigned)((cl.elems + 255) / 256);
        if (hipModuleLaunchKernel((hipFunction_t)cl.fn, blocks, 1, 1, cl.block ? 1024 : 256, 1, 1, 0, stream, args,
                                  nullptr) != hipSuccess)
          return -6;
      } else if (cl.block) {
        hipLaunchKernelGGL(const_block_kernel<R>, dim3(1), dim3(1024), 0, stream, (const int*)wd.steps,
                           (const int*)wd.const_list + cl.first, cl.count, (const int*)wd.ops, (cw<R>*)cst);
      } else {
        const uint64_t nc = 1ull << wd.host_steps[8 * cl.first + 2];
        hipLaunchKernelGGL(const_step_kernel<R>, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, stream,
                           (const int*)wd.steps, cl.first, (const int*)wd.ops, (cw<R>*)cst);
      }
    }
    return hipGetLastError() == hipSuccess ? 0 : -6;
  }
  if (!wd.levels.empty()) {
    // generated kernels: one launch per level of independent steps
    void* a_mem = mem;
    const void* a_cst = cst;
    const void* a_packed = packed;
    unsigned long long a_ge = group_elems, a_sb = s_begin, a_ns = n_s, a_ni = n_items, a_nbs = (unsigned)n_bs;
    int a_g0 = first_group;
    int a_log2 = (n_s & (n_s - 1)) == 0 ? __builtin_ctzll(n_s) : -1;
    void* a_res = res;
    void* a_gres = gres;
    // group sharing: steps that depend on none of these fixed variables run
    // in group 0 of the pass only, and the other groups read their results
    unsigned long long a_vary = group_vary_mask((uint64_t)first_group, n_groups, s_begin, n_s);
    void* args[] = {&a_mem, &a_cst, &a_packed, &a_ge, &a_sb, &a_ns, &a_g0, &a_log2, &a_ni, &a_nbs, &a_res, &a_gres,
                    &a_vary};
    void* const* ev = first_group == 0 ? wd.level_events : nullptr;
    for (size_t li = 0; li < wd.levels.size(); ++li) {
      const WideDev::Level& lv = wd.levels[li];
      if (ev && hipEventRecord((hipEvent_t)ev[li], stream) != hipSuccess) return -6;
      if (hipModuleLaunchKernel((hipFunction_t)lv.fn, (unsigned)lv.blocks, (unsigned)n_groups, 1, (unsigned)lv.threads, 1,
                                1, 0, stream,
                                args, nullptr) != hipSuccess)
        return -6;
    }
    if (ev && hipEventRecord((hipEvent_t)ev[wd.levels.size()], stream) != hipSuccess) return -6;
    return hipGetLastError() == hipSuccess ? 0 : -6;
  }
  for (int si = 0; si < wd.n_steps; ++si) {
    const int r = wd.host_steps[8 * si + 2], is_const = wd.host_steps[8 * si + 7];
    if (is_const) continue;
    const int cl = wide_cpw_log2(r);
    const uint64_t waves = ((1ull << r) + (1ull << cl) - 1) >> cl;
    hipLaunchKernelGGL(wide_step_kernel<R>, dim3((unsigned)((waves + 3) / 4), (unsigned)n_groups), dim3(256), 0,
                       stream, (const int*)wd.steps, si, (const int*)wd.ops, (const cw<R>*)cst, (cw<R>*)mem,
                       group_elems, first_group, packed, n_bs, s_begin, n_s, n_items, (cw<R>*)res, (cw<R>*)gres, cl);
  }
  return hipGetLastError() == hipSuccess ? 0 : -6;
}

template int wide_launch_steps<float>(const WideDev&, int, int, const void*, void*, uint64_t, const uint64_t*, int,
                                      uint64_t, uint64_t, uint64_t, void*, void*, bool, hipStream_t);
template int wide_launch_steps<bfx3>(const WideDev&, int, int, const void*, void*, uint64_t, const uint64_t*, int,
                                     uint64_t, uint64_t, uint64_t, void*, void*, bool, hipStream_t);
template int wide_launch_steps<double>(const WideDev&, int, int, const void*, void*, uint64_t, const uint64_t*, int,
                                       uint64_t, uint64_t, uint64_t, void*, void*, bool, hipStream_t);

}  // namespace qgm
