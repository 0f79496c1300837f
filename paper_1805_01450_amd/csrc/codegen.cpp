// Straight-line HIP source for the per-item program of one plan.
//
// The program is static, so every operand offset is known when the plan is
// made.  The generator turns each step into register arithmetic: item
// tensors become local variables (one per element of the packed item
// memory, so buffer reuse is register reuse) and leaves select among their
// table entries with the item's output and slice bits.  One lane is one
// work item; the kernel needs no other launch:
//   * output bits are packed from the bitstring bytes in the kernel;
//   * gate-table entries that do not depend on an angle are exact constants
//     of the plan and appear as hexadecimal literals, so multiplications by
//     0 and +-1 (the whole CZ table, for instance) compile away;
//   * RZ entries e^{i theta (2u-1)/2} are evaluated from the angles, and the
//     constant steps (those independent of the output and slice bits) are
//     evaluated from the FP64 tables in device memory, each just before its
//     first use;
//   * in every product an item tensor comes first, so no product of two
//     constants exists to be folded at compile time;
//   * when a block's 64 items are 64 consecutive slices of one bitstring the
//     block sums them (FP64, Neumaier, ascending s) into one partial.
#include <algorithm>
#include <cstdio>
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

class Gen {
 public:
  Gen(const Program& p, std::ostringstream& o) : prog(p), o(o), done_const(p.n_const, 0) {}

  // Constant-area element k as an expression usable in an item step.
  std::string const_ref(int k) {
    if (k < prog.n_raw) {
      if (prog.raw_param[k] < 0) return "C2{" + literal(prog.raw[2 * k]) + ", " + literal(prog.raw[2 * k + 1]) + "}";
      ensure_param(k);
      return "p" + std::to_string(k);
    }
    ensure_const(k);
    return "q" + std::to_string(k);
  }

  // Constant-area element k as a run-time value (for constant steps).
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

  std::string item_operand(uint32_t e) {
    if (e & OP_CONST) return const_ref((int)(e & ~OP_CONST));
    return "m" + std::to_string(e);
  }

  void ensure_raw(int k) {
    if (done_const[k]) return;
    done_const[k] = 1;
    o << "  const C2 r" << k << " = C2{(R)rawd[" << 2 * k << "], (R)rawd[" << 2 * k + 1 << "]};\n";
  }

  // RZ entries come from the block's table of e^{-+i theta/2} (see below).
  void ensure_param(int k) {
    if (done_const[k]) return;
    done_const[k] = 1;
    o << "  const C2 p" << k << " = ptab[" << 4 * prog.raw_param[k] + 2 * prog.raw_deriv[k] + prog.raw_bit[k]
      << "];\n";
  }

  // Emit constant steps in order until element k exists.
  void ensure_const(int k) {
    while (!done_const[k] && next_const < prog.n_const_steps) {
      const Step& st = prog.steps[next_const++];
      const int nsum = 1 << st.ns;
      size_t p = st.ops;
      for (int c = 0; c < (1 << st.r); ++c) {
        std::vector<std::string> terms;
        for (int s = 0; s < nsum; ++s) {
          std::string cur;
          for (int i = 0; i < st.m; ++i) {
            std::string v = runtime_ref((int)(prog.optab[p + i] & ~OP_CONST));
            cur = i == 0 ? v : "cm(" + cur + ", " + v + ")";
          }
          p += st.m;
          terms.push_back(cur);
        }
        o << "  C2 q" << (st.out + c) << " = " << terms[0] << ";\n";
        for (size_t t = 1; t < terms.size(); ++t) o << "  q" << (st.out + c) << " = cad(q" << (st.out + c) << ", " << terms[t] << ");\n";
        done_const[st.out + c] = 1;
      }
    }
  }

  const Program& prog;
  std::ostringstream& o;
  std::vector<char> done_const;
  int next_const = 0;
};

}  // namespace

std::string generate_chain_source(const Program& prog, int prec, int n_qubits) {
  std::ostringstream head, o;
  const char* R = prec == 0 ? "double" : "float";
  head << "typedef " << R << " R;\n"
       << "struct C2 { R x, y; };\n"
       << "static __device__ __forceinline__ C2 cm(C2 a, C2 b) { C2 c; c.x = a.x * b.x - a.y * b.y; "
          "c.y = a.x * b.y + a.y * b.x; return c; }\n"
       << "static __device__ __forceinline__ C2 cad(C2 a, C2 b) { C2 c; c.x = a.x + b.x; c.y = a.y + b.y; return c; }\n"
       << "static __device__ __forceinline__ C2 sel(bool t, C2 a1, C2 a0) { C2 c; c.x = t ? a1.x : a0.x; "
          "c.y = t ? a1.y : a0.y; return c; }\n"

       << "static __device__ __forceinline__ void wave_sum(double& s, double& c) { for (int m = 1; m < 64; m <<= 1) "
          "{ const double so = __shfl_xor(s, m); const double co = __shfl_xor(c, m); const double t = s + so; "
          "const double bv = t - s; const double e = (s - (t - bv)) + (so - bv); s = t; c = (c + co) + e; } }\n"
       << "extern \"C\" __global__ void __launch_bounds__(64) qgm_chain(const double* __restrict__ rawd, "
          "const double* __restrict__ params, const unsigned char* __restrict__ bits, int n_qubits, "
          "unsigned long long n_bs, unsigned long long s_begin, unsigned long long n_s, unsigned long long n_items, "
          "C2* __restrict__ res, C2* __restrict__ gres, double* __restrict__ part, int fused) {\n"
       << "  (void)rawd; (void)params;\n"
       << "  const int lane = threadIdx.x;\n"
       << "  unsigned long long item = (unsigned long long)blockIdx.x * 64ull + lane;\n"
       << "  const bool valid = item < n_items;\n"
       << "  if (!valid) item = n_items - 1;\n"
       << "  const unsigned long long b = item / n_s;\n"
       << "  const unsigned long long sl = item - b * n_s;\n"
       << "  const unsigned long long s = s_begin + sl;\n"
       << "  const unsigned char* xrow = bits + b * (unsigned long long)n_qubits;\n"
       << "  unsigned long long xb = 0;\n";
  // the row length is a constant of the plan: independent loads, no loop
  for (int q = 0; q < n_qubits; ++q)
    head << "  xb |= (unsigned long long)(xrow[" << q << "] & 1) << " << q << ";\n";
  head << "  (void)s; (void)xb; (void)xrow;\n";
  int n_params = 0;
  for (int k = 0; k < prog.n_raw; ++k) n_params = std::max(n_params, prog.raw_param[k] + 1);
  if (n_params > 0) {
    // Per angle theta_j, u = 0, 1: RZ entries e^{-+i h} (h = theta_j / 2)
    // and their theta-derivatives (i/2)(2u - 1) e^{i (2u - 1) h}; the lanes
    // of the block share the work, one angle per lane.
    head << "  __shared__ C2 ptab[" << 4 * n_params << "];\n"
         << "  for (int j = lane; j < " << n_params << "; j += 64) {\n"
         << "    double sn, cs;\n"
         << "    sincos(0.5 * params[j], &sn, &cs);\n"
         << "    ptab[4 * j] = C2{(R)cs, (R)(-sn)};\n"
         << "    ptab[4 * j + 1] = C2{(R)cs, (R)sn};\n"
         << "    ptab[4 * j + 2] = C2{(R)(-0.5 * sn), (R)(-0.5 * cs)};\n"
         << "    ptab[4 * j + 3] = C2{(R)(-0.5 * sn), (R)(0.5 * cs)};\n"
         << "  }\n"
         << "  __syncthreads();\n";
  }
  for (int e = 0; e < prog.item_elems; ++e) head << "  C2 m" << e << ";\n";
  head << "  C2 amp;\n";
  Gen g(prog, o);
  for (size_t si = (size_t)prog.n_const_steps; si < prog.steps.size(); ++si) {
    const Step& st = prog.steps[si];
    if (st.kind == ST_LEAF) {
      const Leaf& L = prog.leaves[st.leaf];
      std::string d[2];
      for (int j = 0; j < L.ndep; ++j)
        d[j] = std::string("((") + (L.dep_src[j] ? "s" : "xb") + " >> " + std::to_string(L.dep_bit[j]) + ") & 1ull) != 0ull";
      for (int c = 0; c < (1 << st.r); ++c) {
        int base = L.table + ((c & 1) ? L.free_stride[0] : 0) + ((c & 2) ? L.free_stride[1] : 0);
        auto T = [&](int k) { return g.const_ref(k); };
        std::string v;
        if (L.ndep == 1) {
          v = "sel(" + d[0] + ", " + T(base + L.dep_stride[0]) + ", " + T(base) + ")";
        } else {
          v = "sel(" + d[1] + ", sel(" + d[0] + ", " + T(base + L.dep_stride[0] + L.dep_stride[1]) + ", " +
              T(base + L.dep_stride[1]) + "), sel(" + d[0] + ", " + T(base + L.dep_stride[0]) + ", " + T(base) + "))";
        }
        o << "  m" << (st.out + c) << " = " << v << ";\n";
      }
      continue;
    }
    const int nsum = 1 << st.ns;
    size_t p = st.ops;
    for (int c = 0; c < (1 << st.r); ++c) {
      std::vector<std::string> terms;
      for (int s = 0; s < nsum; ++s) {
        // item operands first: every multiplication involves a run-time value
        std::vector<uint32_t> ops(prog.optab.begin() + p, prog.optab.begin() + p + st.m);
        std::stable_partition(ops.begin(), ops.end(), [](uint32_t e) { return !(e & OP_CONST); });
        std::string cur = st.m == 0 ? "C2{(R)1, (R)0}" : "";
        for (int i = 0; i < st.m; ++i) {
          std::string v = g.item_operand(ops[i]);
          cur = i == 0 ? v : "cm(" + cur + ", " + v + ")";
        }
        p += st.m;
        terms.push_back(cur);
      }
      o << "  { C2 a = " << terms[0] << ";";
      for (size_t t = 1; t < terms.size(); ++t) o << " a = cad(a, " << terms[t] << ");";
      if (st.kind == ST_FINAL)
        o << " amp = a; }\n";
      else if (st.kind == ST_GRAD)
        o << " if (valid) gres[(" << st.grad_slot << "ull * n_s + sl) * n_bs + b] = a; }\n";
      else
        o << " m" << (st.out + c) << " = a; }\n";
    }
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
