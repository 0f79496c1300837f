// Straight-line HIP source for the per-item program of one plan.
//
// The program is static, so every operand's element index is known when the
// plan is made.  Each step becomes register arithmetic on local variables
// named after the tensor and element (t<id>_<e>); the compiler's register
// allocator sees the whole data flow.  One lane is one work item (a
// bitstring and a slice); a block runs 64 items.
//
//   * Output bits are unpacked in the kernel (the row length is a constant).
//   * Gate-table entries that do not depend on an angle are exact constants
//     of the plan and appear as hexadecimal literals, so multiplications by
//     0 and +-1 (the whole CZ table, for instance) compile away.
//   * RZ entries e^{i theta (2u-1)/2} and their theta-derivatives come from a
//     per-block table built from the angles; constant steps (those
//     independent of the output and slice bits) are evaluated from the FP64
//     tables in device memory, each just before its first use.
//   * In every product an item tensor comes first, so no product of two
//     constants exists to be folded at compile time.
//   * Amplitude programs form a tree (every tensor has one consumer).  The
//     tree is cut into subtrees that run on different wavefronts of the block
//     for the same 64 items; their root tensors go through LDS to wavefront
//     0, which runs the top of the tree after a barrier.
//   * When the block's 64 items are 64 consecutive slices of one bitstring
//     the block sums them (FP64, compensated butterfly) into one partial.
#include <algorithm>
#include <cstdio>
#include <functional>
#include <map>
#include <set>
#include <sstream>
#include <string>
#include <vector>

#include "host.h"

namespace qgm {

namespace {

std::string literal(double v) {
  char buf[64];
  std::snprintf(buf, sizeof(buf), "(R)%a", v);
  return buf;
}

std::string tvar(int tid, int e) { return "t" + std::to_string(tid) + "_" + std::to_string(e); }

// Emits code into one wavefront branch; constants are (re)computed per branch.
class Branch {
 public:
  Branch(const Program& p, std::ostringstream& o) : prog(p), o(o), done(p.n_const, 0) {}

  std::string const_ref(int k) {
    if (k < prog.n_raw) {
      if (prog.raw_param[k] < 0) return "C2{" + literal(prog.raw[2 * k]) + ", " + literal(prog.raw[2 * k + 1]) + "}";
      ensure_param(k);
      return "p" + std::to_string(k);
    }
    ensure_const(k);
    return "q" + std::to_string(k);
  }

  std::string runtime_ref(int k) {
    if (k < prog.n_raw) {
      if (prog.raw_param[k] < 0) {
        ensure_raw(k);
        return "r" + std::to_string(k);
      }
      ensure_param(k);
      return "p" + std::to_string(k);
    }
    ensure_const(k);
    return "q" + std::to_string(k);
  }

  void ensure_raw(int k) {
    if (done[k]) return;
    done[k] = 1;
    o << "  const C2 r" << k << " = C2{(R)rawd[" << 2 * k << "], (R)rawd[" << 2 * k + 1 << "]};\n";
  }

  void ensure_param(int k) {
    if (done[k]) return;
    done[k] = 1;
    o << "  const C2 p" << k << " = ptab[" << 4 * prog.raw_param[k] + 2 * prog.raw_deriv[k] + prog.raw_bit[k]
      << "];\n";
  }

  // constant steps in order until element k exists
  void ensure_const(int k) {
    while (!done[k] && next_const < prog.n_const_steps) {
      const Step& st = prog.steps[next_const++];
      emit_products(st, [&](const Operand& op, int e) { return runtime_ref(op.storage + e); },
                    [&](int c) { return "q" + std::to_string(st.out + c); }, true);
      for (int c = 0; c < (1 << st.r); ++c) done[st.out + c] = 1;
    }
  }

  // out[c] = sum_s prod_i operand_i(c, s); `ref` names an operand element,
  // `dst` the destination of output element c.
  template <typename Ref, typename Dst>
  void emit_products(const Step& st, Ref ref, Dst dst, bool declare) {
    std::map<int, int> bitpos;
    std::map<int, int> from_s;
    for (int j = 0; j < st.r; ++j) {
      bitpos[st.out_vars[j]] = j;
      from_s[st.out_vars[j]] = 0;
    }
    for (int j = 0; j < st.ns; ++j) {
      bitpos[st.sum_vars[j]] = j;
      from_s[st.sum_vars[j]] = 1;
    }
    // item operands first: every multiplication involves a run-time value
    std::vector<const Operand*> ops;
    for (const Operand& op : st.opnd)
      if (!op.is_const) ops.push_back(&op);
    for (const Operand& op : st.opnd)
      if (op.is_const) ops.push_back(&op);
    for (int c = 0; c < (1 << st.r); ++c) {
      std::vector<std::string> terms;
      for (int s = 0; s < (1 << st.ns); ++s) {
        std::string cur = st.m == 0 ? "C2{(R)1, (R)0}" : "";
        for (size_t i = 0; i < ops.size(); ++i) {
          int e = 0;
          for (size_t j = 0; j < ops[i]->vars.size(); ++j) {
            const int u = ops[i]->vars[j];
            const int val = from_s[u] ? (s >> bitpos[u]) & 1 : (c >> bitpos[u]) & 1;
            e |= val << j;
          }
          const std::string v = ref(*ops[i], e);
          cur = i == 0 ? v : "cm(" + cur + ", " + v + ")";
        }
        terms.push_back(cur);
      }
      const std::string d = dst(c);
      o << "  " << (declare ? "C2 " : "") << d << " = " << terms[0] << ";\n";
      for (size_t t = 1; t < terms.size(); ++t) o << "  " << d << " = cad(" << d << ", " << terms[t] << ");\n";
    }
  }

  const Program& prog;
  std::ostringstream& o;
  std::vector<char> done;
  int next_const = 0;
};

// Tree cut of the item steps: which wavefront runs each step (-1 = top part
// on wavefront 0 after the barrier) and which tensors cross through LDS.
struct Cut {
  int waves = 1;
  std::vector<int> wave_of;        // per item step index (into prog.steps)
  std::set<int> exchanged;         // tensor ids written to LDS by a subtree
};

// force_waves > 0 asks for exactly that many wavefronts (when the tree and
// the LDS budget allow it); 0 lets the cost model choose.
Cut cut_tree(const Program& prog, int max_waves, size_t elem_bytes, int force_waves) {
  // LDS for the exchanged tensors stays under this, so several blocks share a CU
  const size_t kMaxExchangeBytes = force_waves > 0 ? 64 * 1024 : 40 * 1024;
  if (force_waves > 0) max_waves = force_waves;
  Cut cut;
  const int n = (int)prog.steps.size();
  cut.wave_of.assign(n, 0);
  if (max_waves <= 1) return cut;
  std::map<int, int> producer;  // tensor id -> step index
  std::vector<int> uses_count(0);
  std::map<int, int> uses;
  int root = -1;
  for (int i = prog.n_const_steps; i < n; ++i) {
    const Step& st = prog.steps[i];
    if (st.kind == ST_GRAD) return cut;  // gradient programs are not trees
    if (st.kind == ST_FINAL) root = i;
    if (st.kind == ST_LEAF || st.kind == ST_ELIM) producer[st.out_tid] = i;
    for (const Operand& op : st.opnd)
      if (!op.is_const && ++uses[op.tid] > 1) return cut;
  }
  if (root < 0) return cut;
  std::vector<std::vector<int>> children(n);
  for (int i = prog.n_const_steps; i < n; ++i)
    for (const Operand& op : prog.steps[i].opnd)
      if (!op.is_const) children[i].push_back(producer.at(op.tid));
  std::vector<double> cost(n, 0), sub(n, 0);
  std::function<double(int)> subtree = [&](int i) {
    const Step& st = prog.steps[i];
    cost[i] = st.kind == ST_LEAF ? (double)(1 << st.r) * 2 : st.flops;
    double s = cost[i];
    for (int c : children[i]) s += subtree(c);
    sub[i] = s;
    return s;
  };
  const double total = subtree(root);
  int best_w = 1;
  double best_span = total;
  std::vector<int> best_front, best_assign;
  for (int w = force_waves > 1 ? force_waves : 2; w <= max_waves; w *= 2) {
    std::vector<int> front{root};
    double top = 0;
    const double target = total / w;
    for (;;) {
      auto it = std::max_element(front.begin(), front.end(), [&](int a, int b) { return sub[a] < sub[b]; });
      const int f = *it;
      if (sub[f] <= 1.05 * target || children[f].empty()) break;
      front.erase(it);
      top += cost[f];
      for (int c : children[f]) front.push_back(c);
    }
    std::sort(front.begin(), front.end(), [&](int a, int b) { return sub[a] > sub[b]; });
    std::vector<double> bins(w, 0);
    std::vector<int> assign(front.size());
    for (size_t k = 0; k < front.size(); ++k) {
      const int b = (int)(std::min_element(bins.begin(), bins.end()) - bins.begin());
      bins[b] += sub[front[k]];
      assign[k] = b;
    }
    // a barrier and an LDS round trip per exchanged element cost a little
    const double span = *std::max_element(bins.begin(), bins.end()) + top + 400.0 * w;
    size_t xbytes = 0;
    for (int f : front) xbytes += ((size_t)1 << prog.steps[f].r) * 64 * elem_bytes;
    if (xbytes > kMaxExchangeBytes) continue;
    if (span < 0.8 * best_span || force_waves > 1) {
      best_span = span;
      best_w = w;
      best_front = front;
      best_assign = assign;
    }
  }
  if (best_w == 1) return cut;
  cut.waves = best_w;
  std::fill(cut.wave_of.begin(), cut.wave_of.end(), -1);
  std::function<void(int, int)> mark = [&](int i, int w) {
    cut.wave_of[i] = w;
    for (int c : children[i]) mark(c, w);
  };
  for (size_t k = 0; k < best_front.size(); ++k) {
    mark(best_front[k], best_assign[k]);
    const Step& st = prog.steps[best_front[k]];
    cut.exchanged.insert(st.out_tid);
  }
  return cut;
}

}  // namespace

std::string generate_chain_source(const Program& prog, int prec, int n_qubits, int* waves_out, int force_waves) {
  std::ostringstream head, o;
  const char* R = prec == 0 ? "double" : "float";
  const Cut cut = cut_tree(prog, 4, prec == 0 ? 16 : 8, force_waves);
  // BF16x3: products from bf16 hi/lo splits with FP32 accumulation
  const std::string mul = prec == 2
      ? std::string("static __device__ __forceinline__ float bh(float x) { unsigned u = __float_as_uint(x); "
                    "u += 0x7FFFu + ((u >> 16) & 1u); return __uint_as_float(u & 0xFFFF0000u); }\n"
                    "static __device__ __forceinline__ float m3(float a, float b) { const float ah = bh(a), "
                    "al = bh(a - ah), bh_ = bh(b), bl = bh(b - bh_); return ah * bh_ + (ah * bl + al * bh_); }\n"
                    "static __device__ __forceinline__ C2 cm(C2 a, C2 b) { C2 c; c.x = m3(a.x, b.x) - m3(a.y, b.y); "
                    "c.y = m3(a.x, b.y) + m3(a.y, b.x); return c; }\n")
      : std::string("static __device__ __forceinline__ C2 cm(C2 a, C2 b) { C2 c; c.x = a.x * b.x - a.y * b.y; "
                    "c.y = a.x * b.y + a.y * b.x; return c; }\n");
  const int W = cut.waves;
  if (waves_out) *waves_out = W;
  head << "typedef " << R << " R;\n"
       << "struct C2 { R x, y; };\n"
       << mul
       << "static __device__ __forceinline__ C2 cad(C2 a, C2 b) { C2 c; c.x = a.x + b.x; c.y = a.y + b.y; return c; }\n"
       << "static __device__ __forceinline__ C2 sel(bool t, C2 a1, C2 a0) { C2 c; c.x = t ? a1.x : a0.x; "
          "c.y = t ? a1.y : a0.y; return c; }\n"
       << "static __device__ __forceinline__ void wave_sum(double& s, double& c) { for (int m = 1; m < 64; m <<= 1) "
          "{ const double so = __shfl_xor(s, m); const double co = __shfl_xor(c, m); const double t = s + so; "
          "const double bv = t - s; const double e = (s - (t - bv)) + (so - bv); s = t; c = (c + co) + e; } }\n"
       << "extern \"C\" __global__ void __launch_bounds__(" << 64 * W
       << ") qgm_chain(const double* __restrict__ rawd, "
          "const double* __restrict__ params, const unsigned char* __restrict__ bits, int n_qubits, "
          "unsigned long long n_bs, unsigned long long s_begin, unsigned long long n_s, unsigned long long n_items, "
          "C2* __restrict__ res, C2* __restrict__ gres, double* __restrict__ part, int fused) {\n"
       << "  (void)rawd; (void)params; (void)gres;\n"
       << "  const int lane = threadIdx.x & 63;\n"
       << "  const int wave = threadIdx.x >> 6;\n"
       << "  (void)wave;\n"
       << "  unsigned long long item = (unsigned long long)blockIdx.x * 64ull + lane;\n"
       << "  const bool valid = item < n_items;\n"
       << "  if (!valid) item = n_items - 1;\n"
       << "  const unsigned long long b = item / n_s;\n"
       << "  const unsigned long long sl = item - b * n_s;\n"
       << "  const unsigned long long s = s_begin + sl;\n"
       << "  const unsigned char* xrow = bits + b * (unsigned long long)n_qubits;\n"
       << "  unsigned long long xb = 0;\n";
  for (int q = 0; q < n_qubits; ++q)
    head << "  xb |= (unsigned long long)(xrow[" << q << "] & 1) << " << q << ";\n";
  head << "  (void)s; (void)xb; (void)xrow;\n";
  int n_params = 0;
  for (int k = 0; k < prog.n_raw; ++k) n_params = std::max(n_params, prog.raw_param[k] + 1);
  if (n_params > 0) {
    // Per angle theta_j, u = 0, 1: RZ entries e^{-+i h} (h = theta_j / 2)
    // and their theta-derivatives (i/2)(2u - 1) e^{i (2u - 1) h}; the threads
    // of the block share the work, one angle per thread.
    head << "  __shared__ C2 ptab[" << 4 * n_params << "];\n"
         << "  for (int j = threadIdx.x; j < " << n_params << "; j += blockDim.x) {\n"
         << "    double sn, cs;\n"
         << "    sincos(0.5 * params[j], &sn, &cs);\n"
         << "    ptab[4 * j] = C2{(R)cs, (R)(-sn)};\n"
         << "    ptab[4 * j + 1] = C2{(R)cs, (R)sn};\n"
         << "    ptab[4 * j + 2] = C2{(R)(-0.5 * sn), (R)(-0.5 * cs)};\n"
         << "    ptab[4 * j + 3] = C2{(R)(-0.5 * sn), (R)(0.5 * cs)};\n"
         << "  }\n"
         << "  __syncthreads();\n";
  }
  // LDS slots of the exchanged tensors
  std::map<int, int> xoff;
  int xn = 0;
  if (W > 1) {
    for (int i = prog.n_const_steps; i < (int)prog.steps.size(); ++i) {
      const Step& st = prog.steps[i];
      if ((st.kind == ST_LEAF || st.kind == ST_ELIM) && cut.exchanged.count(st.out_tid)) {
        xoff[st.out_tid] = xn;
        xn += 1 << st.r;
      }
    }
    head << "  __shared__ C2 xch[" << std::max(1, xn) << "][64];\n";
  }

  auto emit_step = [&](Branch& br, const Step& st, std::set<int>* loaded) {
    if (st.kind == ST_LEAF) {
      const Leaf& L = prog.leaves[st.leaf];
      std::string d[2];
      for (int j = 0; j < L.ndep; ++j)
        d[j] = std::string("((") + (L.dep_src[j] ? "s" : "xb") + " >> " + std::to_string(L.dep_bit[j]) + ") & 1ull) != 0ull";
      for (int c = 0; c < (1 << st.r); ++c) {
        int base = L.table + ((c & 1) ? L.free_stride[0] : 0) + ((c & 2) ? L.free_stride[1] : 0);
        auto T = [&](int k) { return br.const_ref(k); };
        std::string v;
        if (L.ndep == 1) {
          v = "sel(" + d[0] + ", " + T(base + L.dep_stride[0]) + ", " + T(base) + ")";
        } else {
          v = "sel(" + d[1] + ", sel(" + d[0] + ", " + T(base + L.dep_stride[0] + L.dep_stride[1]) + ", " +
              T(base + L.dep_stride[1]) + "), sel(" + d[0] + ", " + T(base + L.dep_stride[0]) + ", " + T(base) + "))";
        }
        o << "  const C2 " << tvar(st.out_tid, c) << " = " << v << ";\n";
      }
      return;
    }
    // operands crossing from another wavefront are read from LDS once
    if (loaded) {
      for (const Operand& op : st.opnd) {
        if (op.is_const || !xoff.count(op.tid) || loaded->count(op.tid)) continue;
        loaded->insert(op.tid);
        for (int e = 0; e < (1 << op.vars.size()); ++e)
          o << "  const C2 " << tvar(op.tid, e) << " = xch[" << xoff[op.tid] + e << "][lane];\n";
      }
    }
    auto ref = [&](const Operand& op, int e) -> std::string {
      if (op.is_const) return br.const_ref(op.storage + e);
      return tvar(op.tid, e);
    };
    // resolve constant references before the statement that uses them
    for (const Operand& op : st.opnd)
      if (op.is_const)
        for (int e = 0; e < (1 << op.vars.size()); ++e) br.const_ref(op.storage + e);
    if (st.kind == ST_FINAL) {
      br.emit_products(st, ref, [](int) { return std::string("amp"); }, false);
    } else if (st.kind == ST_GRAD) {
      const std::string g = "g" + std::to_string(st.grad_slot);
      br.emit_products(st, ref, [&](int) { return g; }, true);
      o << "  if (valid) gres[(" << st.grad_slot << "ull * n_s + sl) * n_bs + b] = " << g << ";\n";
    } else {
      br.emit_products(st, ref, [&](int c) { return tvar(st.out_tid, c); }, true);
    }
  };

  o << "  C2 amp;\n";
  if (W == 1) {
    Branch br(prog, o);
    for (int i = prog.n_const_steps; i < (int)prog.steps.size(); ++i) emit_step(br, prog.steps[i], nullptr);
  } else {
    for (int w = 0; w < W; ++w) {
      o << "  if (wave == " << w << ") {\n";
      Branch br(prog, o);
      for (int i = prog.n_const_steps; i < (int)prog.steps.size(); ++i) {
        if (cut.wave_of[i] != w) continue;
        const Step& st = prog.steps[i];
        emit_step(br, st, nullptr);
        if (cut.exchanged.count(st.out_tid))
          for (int e = 0; e < (1 << st.r); ++e)
            o << "  xch[" << xoff[st.out_tid] + e << "][lane] = " << tvar(st.out_tid, e) << ";\n";
      }
      o << "  }\n";
    }
    o << "  __syncthreads();\n"
      << "  if (wave != 0) return;\n";
    Branch br(prog, o);
    std::set<int> loaded;
    for (int i = prog.n_const_steps; i < (int)prog.steps.size(); ++i)
      if (cut.wave_of[i] < 0) emit_step(br, prog.steps[i], &loaded);
  }
  // fused slice sum of the block's 64 slices: the compensated butterfly that
  // the reduction kernels use for each chunk of 64 slices
  o << "  if (!fused) {\n"
    << "    if (valid) res[sl * n_bs + b] = amp;\n"
    << "    return;\n"
    << "  }\n"
    << "  double sr = (double)amp.x, si = (double)amp.y, cr = 0.0, ci = 0.0;\n"
    << "  wave_sum(sr, cr);\n"
    << "  wave_sum(si, ci);\n"
    << "  if (lane == 0) {\n"
    << "    const unsigned long long chunk = item / 64ull;\n"
    << "    part[4 * chunk + 0] = sr;\n"
    << "    part[4 * chunk + 1] = si;\n"
    << "    part[4 * chunk + 2] = cr;\n"
    << "    part[4 * chunk + 3] = ci;\n"
    << "  }\n"
    << "}\n";
  return head.str() + o.str();
}

}  // namespace qgm
