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
//     per-block table built from the angles.  Constant steps (those
//     independent of the output and slice bits) are written out with the
//     same literals, just before their first use, so those without angles
//     fold at compile time.
//   * In every product of an item step an item tensor comes first.
//   * Amplitude programs form a tree (every tensor has one consumer).  The
//     tree is cut into pieces that run on different wavefronts of the block
//     for the same 64 items; the piece roots go through LDS to the wavefront
//     that runs the top of the tree after a barrier.
//   * When the block's 64 items are 64 consecutive slices of one bitstring
//     the block sums them (FP64, compensated butterfly) into one partial.
#include <algorithm>
#include <cmath>
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

  // Operands of the constant steps: gate entries are literals too, so a
  // constant sub-network without angles folds at compile time (no table
  // loads in the middle of a wavefront); angle entries come from the table
  // the block builds.
  std::string runtime_ref(int k) { return const_ref(k); }

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

// Multi-wavefront schedule of the item steps (amplitude programs are trees:
// every tensor has one consumer).  The tree is cut into pieces (subtrees)
// that run on the wavefronts of the block for the same 64 items; the piece
// roots go to LDS, one block barrier follows, and one wavefront runs the
// steps above the cut (the top) reading them.  Point-to-point exchange
// through LDS flags, and list schedules with many exchanges, measured slower
// than this single barrier on gfx950 for these trees.
struct Sched {
  int waves = 1;
  std::vector<int> wave_of;           // per step index (item steps); -1 otherwise
  std::vector<std::vector<int>> seq;  // per wavefront: step indices in execution order
  std::vector<char> top;              // per step: runs after the barrier on top_wave
  int top_wave = 0;
  std::map<int, int> xch;             // piece root tensor id -> LDS element offset
  int lds_elems = 0;
  double makespan = 0;
};

// Estimated VALU instructions of one item step as generated: a product term
// with an exact-zero gate entry vanishes, a factor +-1 or +-i is free, a
// real or imaginary constant costs 2, any other factor 4 (a complex multiply
// is two multiplies and two fused multiply-adds), each added term 2; a leaf
// costs two selects per element whose alternatives differ.
double step_cost(const Program& prog, const Step& st) {
  auto raw_kind = [&](int k) -> int {  // 0 zero, 1 unit, 2 real/imaginary, 3 general
    if (k >= prog.n_raw || prog.raw_param[k] >= 0) return 3;
    const double re = prog.raw[2 * k], im = prog.raw[2 * k + 1];
    if (re == 0 && im == 0) return 0;
    if ((std::fabs(re) == 1 && im == 0) || (re == 0 && std::fabs(im) == 1)) return 1;
    if (re == 0 || im == 0) return 2;
    return 3;
  };
  if (st.kind == ST_LEAF) {
    const Leaf& L = prog.leaves[st.leaf];
    double c = 0;
    if (L.ndep == 0) return 0;
    for (int e = 0; e < (1 << st.r); ++e) {
      int base = L.table, alt = L.table;
      for (int j = 0; j < L.nfree; ++j)
        if ((e >> j) & 1) base += L.free_stride[j];
      alt = base;
      for (int j = 0; j < L.ndep; ++j) alt += L.dep_stride[j];
      c += (prog.raw[2 * base] != prog.raw[2 * alt] || prog.raw[2 * base + 1] != prog.raw[2 * alt + 1]) ? 2.0 : 0.0;
      c += 2.0 * (L.ndep - 1);
    }
    return c;
  }
  std::map<int, int> bitpos, from_s;
  for (int j = 0; j < st.r; ++j) {
    bitpos[st.out_vars[j]] = j;
    from_s[st.out_vars[j]] = 0;
  }
  for (int j = 0; j < st.ns; ++j) {
    bitpos[st.sum_vars[j]] = j;
    from_s[st.sum_vars[j]] = 1;
  }
  double c = 0;
  for (int o = 0; o < (1 << st.r); ++o) {
    int terms = 0;
    for (int sm = 0; sm < (1 << st.ns); ++sm) {
      double t = 0;
      bool zero = false;
      int n_item = 0;
      for (const Operand& op : st.opnd) {
        int e = 0;
        for (size_t j = 0; j < op.vars.size(); ++j) {
          const int u = op.vars[j];
          e |= (from_s[u] ? (sm >> bitpos[u]) & 1 : (o >> bitpos[u]) & 1) << j;
        }
        if (!op.is_const) {
          if (n_item++) t += 4;
          continue;
        }
        const int kind = raw_kind(op.storage + e);
        if (kind == 0) zero = true;
        t += kind == 3 ? 4 : kind == 2 ? 2 : 0;
      }
      if (zero) continue;
      c += t;
      ++terms;
    }
    c += 2.0 * std::max(0, terms - 1);
  }
  return c;
}

// Cut on W wavefronts: the largest subtrees are split until every piece is
// at most total / W; pieces (leaves excepted) are packed onto the
// wavefronts, largest first onto the least loaded; the top runs on the
// least loaded one after the barrier, with the leaves it reads.  Returns
// waves = 0 when the program is not a tree.
Sched schedule_cut(const Program& prog, int W) {
  Sched sc;
  const int n = (int)prog.steps.size();
  std::vector<double> cost(n, 0), sub(n, 0);
  std::vector<std::vector<int>> preds(n);
  std::vector<int> succ(n, -1);
  std::map<int, int> producer;
  int root = -1;
  for (int i = prog.n_const_steps; i < n; ++i) {
    const Step& st = prog.steps[i];
    if (st.kind == ST_GRAD) return sc;
    if (st.kind == ST_FINAL) root = i;
    if (st.kind == ST_LEAF || st.kind == ST_ELIM) producer[st.out_tid] = i;
    cost[i] = step_cost(prog, st);
    sub[i] = cost[i];
    for (const Operand& op : st.opnd)
      if (!op.is_const) {
        const int p = producer.at(op.tid);
        if (succ[p] >= 0) return sc;  // a tensor with two consumers: not a tree
        succ[p] = i;
        preds[i].push_back(p);
        sub[i] += sub[p];
      }
  }
  if (root < 0) return sc;
  sc.waves = W;
  sc.wave_of.assign(n, -1);
  sc.seq.assign(W, {});
  sc.top.assign(n, 0);
  const double target = sub[root] / W;
  std::vector<int> front{root};
  for (;;) {
    auto it = std::max_element(front.begin(), front.end(), [&](int a, int b) { return sub[a] < sub[b]; });
    const int f = *it;
    if (sub[f] <= 1.05 * target || preds[f].empty()) break;
    front.erase(it);
    sc.top[f] = 1;
    for (int p : preds[f]) front.push_back(p);
  }
  std::sort(front.begin(), front.end(), [&](int a, int b) { return sub[a] > sub[b]; });
  std::vector<double> bins(W, 0);
  std::vector<int> piece_wave(n, -1);
  for (int f : front) {
    if (prog.steps[f].kind == ST_LEAF) continue;
    const int b = (int)(std::min_element(bins.begin(), bins.end()) - bins.begin());
    bins[b] += sub[f];
    piece_wave[f] = b;
  }
  sc.top_wave = (int)(std::min_element(bins.begin(), bins.end()) - bins.begin());
  for (int f : front)
    if (prog.steps[f].kind == ST_LEAF) sc.top[f] = 1;  // leaves under the cut are read by the top itself
  for (int i = n - 1; i >= prog.n_const_steps; --i) {
    if (sc.top[i]) {
      sc.wave_of[i] = sc.top_wave;
      continue;
    }
    sc.wave_of[i] = piece_wave[i] >= 0 ? piece_wave[i] : sc.wave_of[succ[i]];
  }
  for (int i = prog.n_const_steps; i < n; ++i)
    if (!sc.top[i]) sc.seq[sc.wave_of[i]].push_back(i);
  for (int i = prog.n_const_steps; i < n; ++i)
    if (sc.top[i]) sc.seq[sc.top_wave].push_back(i);
  // LDS slots of the piece roots
  for (int i = prog.n_const_steps; i < n; ++i) {
    if (sc.top[i]) continue;
    if (succ[i] >= 0 && sc.top[succ[i]]) {
      sc.xch[prog.steps[i].out_tid] = sc.lds_elems;
      sc.lds_elems += 1 << prog.steps[i].r;
    }
  }
  // estimated time: slowest wavefront's pieces (plus root writes), one
  // exchange latency, the root reads and the top
  const double kBarrier = 200.0, kPerElem = 2.0;
  double bar = 0, topc = 0;
  for (int w = 0; w < W; ++w) {
    double c = 0;
    for (int i : sc.seq[w]) {
      if (sc.top[i]) {
        topc += cost[i];
        continue;
      }
      c += cost[i];
      if (sc.xch.count(prog.steps[i].out_tid)) c += kPerElem * (double)(1 << prog.steps[i].r);
    }
    bar = std::max(bar, c);
  }
  sc.makespan = bar + kBarrier + kPerElem * sc.lds_elems + topc;
  return sc;
}

// Wavefront count: force_waves when given (falling back to fewer when the
// exchange does not fit in LDS), else the count with the shortest estimated
// time that beats the next smaller one by 10 %.
Sched choose_schedule(const Program& prog, size_t elem_bytes, int force_waves) {
  Sched one;
  one.waves = 1;
  one.wave_of.assign(prog.steps.size(), -1);
  one.seq.assign(1, {});
  one.top.assign(prog.steps.size(), 0);
  for (int i = prog.n_const_steps; i < (int)prog.steps.size(); ++i) {
    one.wave_of[i] = 0;
    one.seq[0].push_back(i);
    one.makespan += step_cost(prog, prog.steps[i]);
  }
  if (force_waves == 1) return one;
  // exchange slots in LDS, 64 lanes per element (gfx950 gives a block up to
  // 160 KiB; multi-wavefront schedules are for batches of few blocks, where
  // blocks per CU do not matter)
  const size_t kMaxExchangeBytes = 128 * 1024;
  const size_t max_elems = kMaxExchangeBytes / (64 * elem_bytes);
  Sched best = one;
  const int lo = force_waves > 1 ? force_waves : 2, hi = force_waves > 1 ? force_waves : 8;
  for (int w = lo; w <= hi; w *= 2) {
    Sched sc = schedule_cut(prog, w);
    if (sc.waves != w || (size_t)sc.lds_elems > max_elems) continue;
    if (force_waves > 1 || sc.makespan < 0.9 * best.makespan) best = sc;
  }
  return best;
}

}  // namespace

std::string generate_chain_source(const Program& prog, int prec, int n_qubits, int* waves_out, int force_waves,
                                  bool persistent) {
  std::ostringstream head, item_head, blockhead, o;
  // persistent: the block loops over 64-item chunks taken from a device work
  // queue; the per-chunk code leaves through `qnext` instead of returning
  const std::string leave = persistent ? "goto qnext;" : "return;";
  const char* R = prec == 0 ? "double" : "float";
  const Sched sch = choose_schedule(prog, prec == 0 ? 16 : 8, force_waves);
  // BF16x3: products from bf16 hi/lo splits with FP32 accumulation
  const std::string mul = prec == 2
      ? std::string("typedef float bf_f32x2 __attribute__((ext_vector_type(2)));\n"
                    "typedef __bf16 bf_bf16x2 __attribute__((ext_vector_type(2)));\n"
                    // two floats rounded to bfloat16 (nearest even) in one
                    // pack-convert; the halves read back as floats
                    "static __device__ __forceinline__ unsigned pkb(float a, float b) { return __builtin_bit_cast("
                    "unsigned, __builtin_convertvector((bf_f32x2){a, b}, bf_bf16x2)); }\n"
                    "static __device__ __forceinline__ float lo16(unsigned p) { return __uint_as_float(p << 16); }\n"
                    "static __device__ __forceinline__ float hi16(unsigned p) { return __uint_as_float(p & 0xFFFF0000u); }\n"
                    // x*y = xh*yh + (xh*yl + xl*yh), x = xh + xl
                    "static __device__ __forceinline__ C2 cm(C2 a, C2 b) { "
                    "const unsigned ah = pkb(a.x, a.y), bh = pkb(b.x, b.y); "
                    "const float arh = lo16(ah), aih = hi16(ah), brh = lo16(bh), bih = hi16(bh); "
                    "const unsigned al = pkb(a.x - arh, a.y - aih), bl = pkb(b.x - brh, b.y - bih); "
                    "const float arl = lo16(al), ail = hi16(al), brl = lo16(bl), bil = hi16(bl); C2 c; "
                    "c.x = (arh * brh + (arh * brl + arl * brh)) - (aih * bih + (aih * bil + ail * bih)); "
                    "c.y = (arh * bih + (arh * bil + arl * bih)) + (aih * brh + (aih * brl + ail * brh)); return c; }\n")
      : std::string("static __device__ __forceinline__ C2 cm(C2 a, C2 b) { C2 c; c.x = a.x * b.x - a.y * b.y; "
                    "c.y = a.x * b.y + a.y * b.x; return c; }\n");
  const int W = sch.waves;
  if (waves_out) *waves_out = W;
  head << "typedef " << R << " R;\n"
       << "struct C2 { R x, y; };\n"
       << mul
       << "static __device__ __forceinline__ C2 cad(C2 a, C2 b) { C2 c; c.x = a.x + b.x; c.y = a.y + b.y; return c; }\n"
       << "static __device__ __forceinline__ C2 sel(bool t, C2 a1, C2 a0) { C2 c; c.x = t ? a1.x : a0.x; "
          "c.y = t ? a1.y : a0.y; return c; }\n"
       // Compensated butterfly over the 64 lanes.  At level m every lane adds
       // the sum of the other aligned group of m lanes, as the xor butterfly
       // of the reduction kernels does; the partner group is reached by DPP
       // (quad permutations, half-row and row mirrors) and by the gfx950
       // row and half-wave swaps instead of LDS permutes.  TwoSum and the
       // compensation sum are symmetric in their operands, so every lane
       // ends with the xor butterfly's values bit for bit.
       << "template <int C> static __device__ __forceinline__ double dppd(double v) { "
          "const long long u = __double_as_longlong(v); "
          "const int lo = __builtin_amdgcn_update_dpp(0, (int)u, C, 0xF, 0xF, false); "
          "const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), C, 0xF, 0xF, false); "
          "return __longlong_as_double(((long long)hi << 32) | (unsigned)lo); }\n"
       << "static __device__ __forceinline__ void two_add(double& s, double& c, double so, double co) { "
          "const double t = s + so; const double bv = t - s; const double e = (s - (t - bv)) + (so - bv); s = t; "
          "c = (c + co) + e; }\n"
       << "static __device__ __forceinline__ void swap16(double& a, double& b) { "
          "const long long u = __double_as_longlong(a); "
          "const auto l = __builtin_amdgcn_permlane16_swap((unsigned)u, (unsigned)u, false, false); "
          "const auto h = __builtin_amdgcn_permlane16_swap((unsigned)(u >> 32), (unsigned)(u >> 32), false, false); "
          "a = __longlong_as_double(((long long)h[0] << 32) | l[0]); "
          "b = __longlong_as_double(((long long)h[1] << 32) | l[1]); }\n"
       << "static __device__ __forceinline__ void swap32(double& a, double& b) { "
          "const long long u = __double_as_longlong(a); "
          "const auto l = __builtin_amdgcn_permlane32_swap((unsigned)u, (unsigned)u, false, false); "
          "const auto h = __builtin_amdgcn_permlane32_swap((unsigned)(u >> 32), (unsigned)(u >> 32), false, false); "
          "a = __longlong_as_double(((long long)h[0] << 32) | l[0]); "
          "b = __longlong_as_double(((long long)h[1] << 32) | l[1]); }\n"
       << "static __device__ __forceinline__ void wave_sum(double& s, double& c) {\n"
          "  two_add(s, c, dppd<0xB1>(s), dppd<0xB1>(c));\n"    // quad_perm [1,0,3,2]: lane ^ 1
          "  two_add(s, c, dppd<0x4E>(s), dppd<0x4E>(c));\n"    // quad_perm [2,3,0,1]: lane ^ 2
          "  two_add(s, c, dppd<0x141>(s), dppd<0x141>(c));\n"  // half-row mirror: other 4 of 8
          "  two_add(s, c, dppd<0x140>(s), dppd<0x140>(c));\n"  // row mirror: other 8 of 16
          "  double s0 = s, s1, c0 = c, c1;\n"
          "  swap16(s0, s1); swap16(c0, c1);\n"                  // rows 2j and 2j+1
          "  s = s0; c = c0; two_add(s, c, s1, c1);\n"
          "  s0 = s; c0 = c;\n"
          "  swap32(s0, s1); swap32(c0, c1);\n"                  // lanes 0-31 and 32-63
          "  s = s0; c = c0; two_add(s, c, s1, c1);\n"
          "}\n"
       // the arguments needed first lead the list, so that they arrive in
       // preloaded SGPRs rather than through a scalar load at wave start
       << "extern \"C\" __global__ void __launch_bounds__(" << 64 * W
       << ") qgm_chain(const unsigned char* __restrict__ bits, unsigned long long n_s, unsigned long long s_begin, "
          "unsigned long long n_items, unsigned long long n_bs, int n_qubits, int fused, int ns_log2, "
          "const double* __restrict__ params, C2* __restrict__ res, C2* __restrict__ gres, "
          "double* __restrict__ part, const double* __restrict__ rawd, unsigned* __restrict__ queue) {\n"
       << "  (void)rawd; (void)params; (void)gres; (void)queue;\n"
       << "  const int lane = threadIdx.x & 63;\n"
       << "  const int wave = threadIdx.x >> 6;\n"
       << "  (void)wave;\n";
  if (persistent)
    item_head << "  unsigned long long item = chunk * 64ull + lane;\n";
  else
    item_head << "  unsigned long long item = (unsigned long long)blockIdx.x * 64ull + lane;\n";
  item_head
       << "  const bool valid = item < n_items;\n"
       << "  if (!valid) item = n_items - 1;\n"
       // no 64-bit division when the slice count is a power of two
       << "  unsigned long long b, sl;\n"
       << "  if (ns_log2 >= 0) {\n"
       << "    b = item >> ns_log2;\n"
       << "    sl = item & (n_s - 1ull);\n"
       << "  } else if (n_items <= 0xFFFFFFFFull) {\n"
       << "    b = (unsigned)item / (unsigned)n_s;\n"
       << "    sl = item - b * n_s;\n"
       << "  } else {\n"
       << "    b = item / n_s;\n"
       << "    sl = item - b * n_s;\n"
       << "  }\n"
       << "  const unsigned long long s = s_begin + sl;\n"
       << "  unsigned long long xb = 0;\n"
       // fused blocks hold 64 slices of one bitstring: lane q reads qubit q,
       // and a ballot packs the row once the steps that do not need it are
       // done; otherwise each lane reads its own row
       << "  unsigned xlane = 0;\n"
       << "  if (fused) {\n"
       << "    const unsigned long long bu = (unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)b) | "
          "((unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)(b >> 32)) << 32);\n"
       << "    const int q = lane < n_qubits ? lane : 0;\n"
       << "    xlane = bits[bu * (unsigned long long)n_qubits + q];\n"
       << "  } else {\n"
       << "    const unsigned char* xrow = bits + b * (unsigned long long)n_qubits;\n";
  for (int q = 0; q < n_qubits; ++q)
    item_head << "    xb |= (unsigned long long)(xrow[" << q << "] & 1) << " << q << ";\n";
  item_head << "  }\n"
            << "  (void)s; (void)xb; (void)xlane;\n";
  // (the empty asm pins the first use of the loaded byte here, so the
  // compiler cannot move the test, and with it the wait, up to the load)
  const std::string pack_bits =
      "  if (fused) {\n    asm volatile(\"\" : \"+v\"(xlane));\n"
      "    xb = __ballot(lane < n_qubits && (xlane & 1u));\n  }\n";
  // LDS slots of the piece roots of the multi-wavefront schedule
  if (W > 1) blockhead << "  __shared__ C2 xch[" << std::max(1, sch.lds_elems) << "][64];\n";
  int n_params = 0;
  for (int k = 0; k < prog.n_raw; ++k) n_params = std::max(n_params, prog.raw_param[k] + 1);
  if (n_params > 0) {
    // Per angle theta_j, u = 0, 1: RZ entries e^{-+i h} (h = theta_j / 2)
    // and their theta-derivatives (i/2)(2u - 1) e^{i (2u - 1) h}; the threads
    // of the block share the work, one angle per thread.
    blockhead << "  __shared__ C2 ptab[" << 4 * n_params << "];\n"
         << "  for (int j = threadIdx.x; j < " << n_params << "; j += blockDim.x) {\n"
         << "    double sn, cs;\n"
         << "    sincos(0.5 * params[j], &sn, &cs);\n"
         << "    ptab[4 * j] = C2{(R)cs, (R)(-sn)};\n"
         << "    ptab[4 * j + 1] = C2{(R)cs, (R)sn};\n"
         << "    ptab[4 * j + 2] = C2{(R)(-0.5 * sn), (R)(-0.5 * cs)};\n"
         << "    ptab[4 * j + 3] = C2{(R)(-0.5 * sn), (R)(0.5 * cs)};\n"
         << "  }\n";
  }
  if (n_params > 0) blockhead << "  __syncthreads();\n";

  auto emit_step = [&](Branch& br, const Step& st) {
    if (st.kind == ST_LEAF) {
      const Leaf& L = prog.leaves[st.leaf];
      std::string d[4];
      for (int j = 0; j < L.ndep; ++j)
        d[j] = std::string("((") + (L.dep_src[j] ? "s" : "xb") + " >> " + std::to_string(L.dep_bit[j]) + ") & 1ull) != 0ull";
      for (int c = 0; c < (1 << st.r); ++c) {
        int base = L.table;
        for (int j = 0; j < L.nfree; ++j)
          if ((c >> j) & 1) base += L.free_stride[j];
        auto T = [&](int k) { return br.const_ref(k); };
        // the entry at the item's fixed bits: a select per fixed variable,
        // the last one outermost
        std::function<std::string(int, int)> pick = [&](int j, int off) -> std::string {
          if (j < 0) return T(base + off);
          return "sel(" + d[j] + ", " + pick(j - 1, off + L.dep_stride[j]) + ", " + pick(j - 1, off) + ")";
        };
        // (built before the statement: a table reference may first emit the
        // declaration it needs)
        const std::string v = pick(L.ndep - 1, 0);
        o << "  const C2 " << tvar(st.out_tid, c) << " = " << v << ";\n";
      }
      return;
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
      // open outputs: 2^r amplitudes per item
      if (st.r > 0)
        br.emit_products(st, ref, [](int c) { return "amp_" + std::to_string(c); }, false);
      else
        br.emit_products(st, ref, [](int) { return std::string("amp"); }, false);
    } else if (st.kind == ST_GRAD) {
      const std::string g = "g" + std::to_string(st.grad_slot);
      br.emit_products(st, ref, [&](int) { return g; }, true);
      o << "  if (valid) gres[(" << st.grad_slot << "ull * n_s + sl) * n_bs + b] = " << g << ";\n";
    } else {
      br.emit_products(st, ref, [&](int c) { return tvar(st.out_tid, c); }, true);
    }
  };

  // Emission order: within each wavefront's part, the steps that do not
  // depend on the output bits come first (they depend only on such steps),
  // so they run while the bitstring load is in flight.
  std::vector<int> seq;
  std::vector<char> xdep(prog.steps.size(), 0);
  {
    std::map<int, bool> xdep_t;
    std::vector<int> later;
    for (int i = prog.n_const_steps; i < (int)prog.steps.size(); ++i) {
      const Step& st = prog.steps[i];
      bool d = false;
      if (st.kind == ST_LEAF) {
        const Leaf& L = prog.leaves[st.leaf];
        for (int j = 0; j < L.ndep; ++j) d = d || L.dep_src[j] == 0;
      } else {
        for (const Operand& op : st.opnd) d = d || (!op.is_const && xdep_t[op.tid]);
      }
      if (st.kind == ST_LEAF || st.kind == ST_ELIM) xdep_t[st.out_tid] = d;
      xdep[i] = d;
      (d && prog.n_grad_slots == 0 ? later : seq).push_back(i);
    }
    seq.insert(seq.end(), later.begin(), later.end());
  }
  const int n_amp = 1 << prog.n_open;  // amplitudes per item (open outputs)
  if (prog.n_open == 0)
    o << "  C2 amp;\n";
  else
    for (int c = 0; c < n_amp; ++c) o << "  C2 amp_" << c << ";\n";
  // the packed row is formed before the first step that reads it
  bool packed = false;
  auto need_bits = [&](int i) {
    if (!packed && xdep[i]) {
      o << pack_bits;
      packed = true;
    }
  };
  if (W == 1) {
    Branch br(prog, o);
    for (int i : seq) {
      need_bits(i);
      emit_step(br, prog.steps[i]);
    }
  } else {
    for (int w = 0; w < W; ++w) {
      o << "  if (wave == " << w << ") {\n";
      Branch br(prog, o);
      packed = false;
      for (int i : sch.seq[w]) {
        if (sch.top[i]) continue;
        const Step& st = prog.steps[i];
        need_bits(i);
        emit_step(br, st);
        auto x = sch.xch.find(st.out_tid);
        if (x != sch.xch.end())
          for (int e = 0; e < (1 << st.r); ++e)
            o << "  xch[" << x->second + e << "][lane] = " << tvar(st.out_tid, e) << ";\n";
      }
      // the top wavefront continues after the barrier and needs the row there
      if (!packed && w == sch.top_wave) o << pack_bits;
      o << "  }\n";
    }
    o << "  __syncthreads();\n"
      << "  if (wave != " << sch.top_wave << ") " << leave << "\n";
    Branch br(prog, o);
    std::set<int> loaded;
    for (int i : sch.seq[sch.top_wave]) {
      if (!sch.top[i]) continue;
      const Step& st = prog.steps[i];
      for (const Operand& op : st.opnd) {
        if (op.is_const || loaded.count(op.tid)) continue;
        auto x = sch.xch.find(op.tid);
        if (x == sch.xch.end()) continue;
        loaded.insert(op.tid);
        for (int e = 0; e < (1 << op.vars.size()); ++e)
          o << "  const C2 " << tvar(op.tid, e) << " = xch[" << x->second + e << "][lane];\n";
      }
      emit_step(br, st);
    }
  }
  // fused slice sum of the block's 64 slices: the compensated butterfly that
  // the reduction kernels use for each chunk of 64 slices
  if (prog.n_open > 0) {
    // open outputs: every amplitude goes to the per-item results (the
    // slice sum runs in the reduction kernel; blocks never fuse it)
    for (int c = 0; c < n_amp; ++c)
      o << "  if (valid) res[((sl * n_bs + b) << " << prog.n_open << ") + " << c << "] = amp_" << c << ";\n";
    o << "  " << leave << "\n";
  } else {
    o << "  if (!fused) {\n"
      << "    if (valid) res[sl * n_bs + b] = amp;\n"
      << "    " << leave << "\n"
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
      << "  }\n";
  }
  if (!persistent) {
    o << "}\n";
    return head.str() + item_head.str() + blockhead.str() + o.str();
  }
  // Persistent form: a block's first chunk is its block index, later ones
  // come from the queue counter (zero at launch), offset by the grid size.
  // Every wave of the block passes the same barriers each round, so the
  // exchange slots and the shared chunk index are free for the next round.
  std::ostringstream loop;
  loop << "  __shared__ unsigned long long q_chunk;\n"
       << "  const unsigned long long n_chunks = (n_items + 63ull) / 64ull;\n"
       << "  unsigned long long chunk = blockIdx.x;\n"
       << "  while (chunk < n_chunks) {\n"
       << "  {\n";
  o << "  }\n"
    << "  qnext:\n"
    << "  __syncthreads();\n"
    << "  if (threadIdx.x == 0) q_chunk = (unsigned long long)gridDim.x + atomicAdd(queue, 1u);\n"
    << "  __syncthreads();\n"
    << "  chunk = q_chunk;\n"
    << "  }\n"
    << "}\n";
  return head.str() + blockhead.str() + loop.str() + item_head.str() + o.str();
}

}  // namespace qgm
