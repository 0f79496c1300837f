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
//   * Amplitude programs form a tree (every tensor has one consumer).  Its
//     steps are list-scheduled onto the wavefronts of a block, which work on
//     the same 64 items; a tensor consumed on another wavefront crosses
//     through LDS with a release/acquire publish counter per wavefront.
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

// Multi-wavefront schedule of the item steps.  Every step runs on one
// wavefront of the block for the block's 64 items.  A tensor consumed on
// another wavefront goes through LDS: the producer writes it, then raises its
// publish counter (release); the consumer waits until the counter reaches
// the tensor's publish number (acquire) and reads it.  Each wavefront runs
// its steps in the order they were scheduled, which is a topological order
// of the whole program, so every wait is for a step that precedes the
// waiting one in that order; schedules are also checked by simulating the
// waits before any code is emitted.
struct Sched {
  int waves = 1;
  std::vector<int> wave_of;           // per step index (item steps); -1 otherwise
  std::vector<std::vector<int>> seq;  // per wavefront: step indices in execution order
  struct Xch {
    int slot, wave, number;           // LDS element offset, producer, publish number (1-based)
  };
  std::map<int, Xch> xch;             // exchanged tensor id -> LDS slot and publish number
  int lds_elems = 0;
  double makespan = 0;
};

// Earliest-start list scheduling: steps in order of decreasing bottom level
// (the longest cost path from the step to the end of the program); each goes
// to the wavefront where it can start first, counting a fixed latency plus a
// per-element cost for operands that cross wavefronts.
Sched schedule_waves(const Program& prog, int W, double comm, double per_elem, size_t max_lds_elems) {
  Sched sc;
  const int n = (int)prog.steps.size();
  sc.wave_of.assign(n, -1);
  std::map<int, int> producer;
  std::vector<std::vector<int>> preds(n), succs(n);
  std::vector<double> cost(n, 0), bl(n, 0);
  for (int i = prog.n_const_steps; i < n; ++i) {
    const Step& st = prog.steps[i];
    if (st.kind == ST_LEAF || st.kind == ST_ELIM) producer[st.out_tid] = i;
    cost[i] = st.kind == ST_LEAF ? (double)(1 << st.r) * 2 : st.flops;
    for (const Operand& op : st.opnd)
      if (!op.is_const) {
        const int p = producer.at(op.tid);
        preds[i].push_back(p);
        succs[p].push_back(i);
      }
  }
  for (int i = n - 1; i >= prog.n_const_steps; --i) {
    double m = 0;
    for (int s : succs[i]) m = std::max(m, bl[s]);
    bl[i] = cost[i] + m;
  }
  std::vector<int> pending(n, 0);
  std::vector<int> ready;
  for (int i = prog.n_const_steps; i < n; ++i) {
    pending[i] = (int)preds[i].size();
    if (!pending[i]) ready.push_back(i);
  }
  std::vector<double> fin(n, 0), free_at(W, 0);
  sc.waves = W;
  sc.seq.assign(W, {});
  std::vector<int> n_pub(W, 0);
  while (!ready.empty()) {
    auto it = std::max_element(ready.begin(), ready.end(), [&](int a, int b) {
      return bl[a] < bl[b] || (bl[a] == bl[b] && a > b);
    });
    const int i = *it;
    ready.erase(it);
    int best_w = -1;
    double best_start = 0, best_local = 0;
    for (int w = 0; w < W; ++w) {
      double start = free_at[w], xtra = 0, local = 0;
      for (int p : preds[i]) {
        if (sc.wave_of[p] == w) {
          start = std::max(start, fin[p]);
          local += cost[p];
        } else {
          const double e = (double)(1 << prog.steps[p].r);
          start = std::max(start, fin[p] + comm + per_elem * e);
          xtra += per_elem * e;
        }
      }
      start += xtra;
      if (best_w < 0 || start < best_start || (start == best_start && local > best_local)) {
        best_w = w;
        best_start = start;
        best_local = local;
      }
    }
    sc.wave_of[i] = best_w;
    sc.seq[best_w].push_back(i);
    fin[i] = best_start + cost[i];
    free_at[best_w] = fin[i];
    sc.makespan = std::max(sc.makespan, fin[i]);
    for (int p : preds[i])
      if (sc.wave_of[p] != best_w && !sc.xch.count(prog.steps[p].out_tid))
        sc.xch[prog.steps[p].out_tid] = {-1, sc.wave_of[p], 0};
    for (int s : succs[i])
      if (--pending[s] == 0) ready.push_back(s);
  }
  // publish numbers follow each producer's execution order
  for (int w = 0; w < W; ++w)
    for (int i : sc.seq[w]) {
      const Step& st = prog.steps[i];
      auto x = sc.xch.find(st.out_tid);
      if ((st.kind == ST_LEAF || st.kind == ST_ELIM) && x != sc.xch.end()) x->second.number = ++n_pub[w];
    }
  (void)max_lds_elems;
  return sc;
}

// Simulates the wavefronts' waits and assigns the LDS slots.  Returns false
// unless every wavefront runs to the end (no wait can block for ever) and
// every operand is available where it is read (produced earlier on the same
// wavefront, or published by another).  Slots are reused: a tensor may take
// the slot of one already read when that read happens before the write in
// every execution, which vector clocks over the publish/wait edges decide
// (the clock of a wavefront counts the steps of each wavefront known to be
// complete; a wait merges in the clock the producer had when publishing).
bool finalize_schedule(const Program& prog, Sched& sc) {
  const int W = sc.waves;
  std::map<int, int> producer;
  for (int i = prog.n_const_steps; i < (int)prog.steps.size(); ++i) {
    const Step& st = prog.steps[i];
    if (st.kind == ST_LEAF || st.kind == ST_ELIM) producer[st.out_tid] = i;
  }
  std::vector<size_t> pos(W, 0);
  std::vector<int> published(W, 0);
  std::vector<char> done(prog.steps.size(), 0);
  std::vector<std::vector<int>> vc(W, std::vector<int>(W, 0));
  std::vector<std::vector<std::vector<int>>> pub_vc(W);  // per wave, per publish: clock
  std::vector<std::map<int, int>> waited(W);            // as the emitted code: max number waited
  struct Slot {
    int offset, size, tid;  // tid: current occupant
  };
  std::vector<Slot> slots;
  std::map<int, std::pair<int, int>> read_at;  // tensor id -> (wave, position) of its read
  sc.lds_elems = 0;
  size_t left = 0;
  for (int w = 0; w < W; ++w) left += sc.seq[w].size();
  for (;;) {
    bool moved = false;
    for (int w = 0; w < W; ++w) {
      while (pos[w] < sc.seq[w].size()) {
        const int i = sc.seq[w][pos[w]];
        const Step& st = prog.steps[i];
        bool ok = true;
        for (const Operand& op : st.opnd) {
          if (op.is_const) continue;
          const int p = producer.at(op.tid);
          if (sc.wave_of[p] == w) {
            if (!done[p]) return false;  // same wavefront: must come earlier
          } else {
            auto x = sc.xch.find(op.tid);
            if (x == sc.xch.end() || x->second.wave != sc.wave_of[p]) return false;
            if (published[x->second.wave] < x->second.number) ok = false;
          }
        }
        if (!ok) break;
        // the waits and reads of this step
        for (const Operand& op : st.opnd) {
          if (op.is_const) continue;
          auto x = sc.xch.find(op.tid);
          if (x == sc.xch.end() || x->second.wave == w) continue;
          const int q = x->second.wave, nmb = x->second.number;
          if (waited[w][q] < nmb) {
            waited[w][q] = nmb;
            for (int v = 0; v < W; ++v) vc[w][v] = std::max(vc[w][v], pub_vc[q][nmb - 1][v]);
          }
          read_at[op.tid] = {w, (int)pos[w]};
        }
        done[i] = 1;
        vc[w][w] = (int)pos[w] + 1;
        if ((st.kind == ST_LEAF || st.kind == ST_ELIM) && sc.xch.count(st.out_tid)) {
          Sched::Xch& x = sc.xch.at(st.out_tid);
          if (x.number != published[w] + 1) return false;
          // the smallest slot large enough whose occupant's read happened
          // before this write
          const int size = 1 << st.r;
          int chosen = -1;
          for (size_t k = 0; k < slots.size(); ++k) {
            if (slots[k].size < size || (chosen >= 0 && slots[k].size >= slots[chosen].size)) continue;
            auto r = read_at.find(slots[k].tid);
            if (r == read_at.end()) continue;
            if (vc[w][r->second.first] >= r->second.second + 1) chosen = (int)k;
          }
          if (chosen < 0) {
            slots.push_back({sc.lds_elems, size, st.out_tid});
            sc.lds_elems += size;
            chosen = (int)slots.size() - 1;
          }
          slots[chosen].tid = st.out_tid;
          x.slot = slots[chosen].offset;
          published[w]++;
          pub_vc[w].push_back(vc[w]);
        }
        ++pos[w];
        --left;
        moved = true;
      }
    }
    if (!left) return true;
    if (!moved) return false;  // every unfinished wavefront waits
  }
}

// Wavefront count: force_waves when given (falling back to fewer when the
// exchange does not fit in LDS), else the count with the shortest estimated
// time that clearly beats the next smaller one.
Sched choose_schedule(const Program& prog, size_t elem_bytes, int force_waves, double comm0) {
  Sched one;
  one.waves = 1;
  one.wave_of.assign(prog.steps.size(), -1);
  one.seq.assign(1, {});
  for (int i = prog.n_const_steps; i < (int)prog.steps.size(); ++i) {
    one.wave_of[i] = 0;
    one.seq[0].push_back(i);
  }
  // gradient programs are not trees (a tensor may feed several steps)
  for (const Step& st : prog.steps)
    if (st.kind == ST_GRAD) return one;
  // exchange slots in LDS, 64 lanes per element (gfx950 gives a block up to
  // 160 KiB; multi-wavefront schedules are for batches of few blocks, where
  // blocks per CU do not matter)
  const size_t kMaxExchangeBytes = 128 * 1024;
  const size_t max_elems = kMaxExchangeBytes / (64 * elem_bytes);
  double total = 0;
  for (int i = prog.n_const_steps; i < (int)prog.steps.size(); ++i) {
    const Step& st = prog.steps[i];
    total += st.kind == ST_LEAF ? (double)(1 << st.r) * 2 : st.flops;
  }
  Sched best = one;
  best.makespan = total;
  const int lo = force_waves > 1 ? force_waves : 2, hi = force_waves > 1 ? force_waves : 8;
  for (int w = lo; w <= hi; w *= 2) {
    // exchange latency and per-element cost in flops; a higher latency
    // estimate trades parallelism for fewer exchanges when LDS is short
    for (double comm : {comm0, 2.5 * comm0, 6.0 * comm0}) {
      Sched sc = schedule_waves(prog, w, comm, 4.0, max_elems);
      if (!finalize_schedule(prog, sc) || (size_t)sc.lds_elems > max_elems) continue;
      if (force_waves > 1 ? (best.waves != w || sc.makespan < best.makespan) : sc.makespan < 0.85 * best.makespan)
        best = sc;
      break;
    }
  }
  return best;
}

}  // namespace

std::string generate_chain_source(const Program& prog, int prec, int n_qubits, int* waves_out, int force_waves,
                                  double comm) {
  std::ostringstream head, o;
  const char* R = prec == 0 ? "double" : "float";
  const Sched sch = choose_schedule(prog, prec == 0 ? 16 : 8, force_waves, comm > 0 ? comm : kDefaultExchangeCost);
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
       // cross-wavefront exchange: publish counters in LDS; a wait gives up
       // (and flags the block's result as NaN) after about a second
       << "static __device__ __forceinline__ void xwait(unsigned* c, unsigned n, unsigned* err) { unsigned it = 0; "
          "while (__hip_atomic_load(c, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < n) "
          "if (++it > (1u << 24)) { *err = 1u; break; } }\n"
       << "static __device__ __forceinline__ void xpub(unsigned* c, unsigned n) { "
          "__hip_atomic_store(c, n, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP); }\n"
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
          "double* __restrict__ part, const double* __restrict__ rawd) {\n"
       << "  (void)rawd; (void)params; (void)gres;\n"
       << "  const int lane = threadIdx.x & 63;\n"
       << "  const int wave = threadIdx.x >> 6;\n"
       << "  (void)wave;\n"
       << "  unsigned long long item = (unsigned long long)blockIdx.x * 64ull + lane;\n"
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
    head << "    xb |= (unsigned long long)(xrow[" << q << "] & 1) << " << q << ";\n";
  head << "  }\n"
       << "  (void)s; (void)xb; (void)xlane;\n";
  // (the empty asm pins the first use of the loaded byte here, so the
  // compiler cannot move the test, and with it the wait, up to the load)
  const std::string pack_bits =
      "  if (fused) {\n    asm volatile(\"\" : \"+v\"(xlane));\n"
      "    xb = __ballot(lane < n_qubits && (xlane & 1u));\n  }\n";
  // LDS exchange of the multi-wavefront schedule: slots, per-wavefront
  // publish counters (zeroed before the barrier below), error flag
  if (W > 1)
    head << "  __shared__ C2 xch[" << std::max(1, sch.lds_elems) << "][64];\n"
         << "  __shared__ unsigned xcnt[" << W << "];\n"
         << "  __shared__ unsigned xerr;\n"
         << "  if (lane == 0) xcnt[wave] = 0u;\n"
         << "  if (threadIdx.x == 0) xerr = 0u;\n";
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
         << "  }\n";
  }
  if (n_params > 0 || W > 1) head << "  __syncthreads();\n";

  auto emit_step = [&](Branch& br, const Step& st) {
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
  o << "  C2 amp;\n";
  // the packed row is formed before the first step that reads it
  bool packed = false;
  auto need_bits = [&](int i) {
    if (!packed && xdep[i]) {
      o << pack_bits;
      packed = true;
    }
  };
  int final_wave = 0;
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
      std::map<int, int> waited;  // producer wavefront -> publish number already waited for
      for (int i : sch.seq[w]) {
        const Step& st = prog.steps[i];
        need_bits(i);
        // operands from other wavefronts: wait for their publication, read once
        for (const Operand& op : st.opnd) {
          if (op.is_const) continue;
          auto x = sch.xch.find(op.tid);
          if (x == sch.xch.end() || x->second.wave == w) continue;
          if (waited[x->second.wave] < x->second.number) {
            o << "  xwait(&xcnt[" << x->second.wave << "], " << x->second.number << "u, &xerr);\n";
            waited[x->second.wave] = x->second.number;
          }
          for (int e = 0; e < (1 << op.vars.size()); ++e)
            o << "  const C2 " << tvar(op.tid, e) << " = xch[" << x->second.slot + e << "][lane];\n";
        }
        emit_step(br, st);
        if (st.kind == ST_FINAL) final_wave = w;
        auto x = sch.xch.find(st.out_tid);
        if ((st.kind == ST_LEAF || st.kind == ST_ELIM) && x != sch.xch.end()) {
          for (int e = 0; e < (1 << st.r); ++e)
            o << "  xch[" << x->second.slot + e << "][lane] = " << tvar(st.out_tid, e) << ";\n";
          o << "  xpub(&xcnt[" << w << "], " << x->second.number << "u);\n";
        }
      }
      o << "  }\n";
    }
    o << "  if (wave != " << final_wave << ") return;\n"
      << "  if (xerr) amp.x = amp.y = __builtin_nanf(\"\");\n";
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
