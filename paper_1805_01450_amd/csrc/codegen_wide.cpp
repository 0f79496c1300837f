// Generated kernels for the wide engine: one kernel per level of mutually
// independent item steps.
//
// Item tensors live in HBM as [element][64 items] rows.  A wavefront owns a
// tile of 2^L consecutive output elements of a step for the 64 items of a
// group.  The offset of operand i at output element c and summed index s is
//   base_i + sum_j c_j * out_stride_ij + sum_j s_j * sum_stride_ij;
// the high output bits (the tile index) give a per-wavefront base computed
// once, and everything inside the tile (the low L output bits, the summed
// bits, the operands) is unrolled with compile-time offsets, so all loads of
// an output row are independent and issued together.
#include <algorithm>
#include <cstdio>
#include <sstream>
#include <string>
#include <vector>

#include "host.h"

namespace qgm {

namespace {

std::string lit(double v) {
  char buf[64];
  std::snprintf(buf, sizeof(buf), "(R)%a", v);
  return buf;
}

}  // namespace

std::string generate_wide_source(const Program& prog, const WideProgram& wide, int prec,
                                 std::vector<WideKernel>& kernels) {
  kernels.clear();
  std::ostringstream o;
  o << "typedef " << (prec == 0 ? "double" : "float") << " R;\n"
    << "struct C2 { R x, y; };\n";
  if (prec == 2)
    o << "static __device__ __forceinline__ float bh(float x) { unsigned u = __float_as_uint(x); "
         "u += 0x7FFFu + ((u >> 16) & 1u); return __uint_as_float(u & 0xFFFF0000u); }\n"
         "static __device__ __forceinline__ float m3(float a, float b) { const float ah = bh(a), al = bh(a - ah), "
         "bh_ = bh(b), bl = bh(b - bh_); return ah * bh_ + (ah * bl + al * bh_); }\n"
         "static __device__ __forceinline__ C2 cm(C2 a, C2 b) { C2 c; c.x = m3(a.x, b.x) - m3(a.y, b.y); "
         "c.y = m3(a.x, b.y) + m3(a.y, b.x); return c; }\n";
  else
    o << "static __device__ __forceinline__ C2 cm(C2 a, C2 b) { C2 c; c.x = a.x * b.x - a.y * b.y; "
         "c.y = a.x * b.y + a.y * b.x; return c; }\n";
  o << "static __device__ __forceinline__ C2 cad(C2 a, C2 b) { C2 c; c.x = a.x + b.x; c.y = a.y + b.y; return c; }\n";

  // Levels: an item step joins the launch after the last earlier step it
  // conflicts with, i.e. one that produces an operand it reads (RAW), reads
  // the memory its output overwrites (WAR) or writes that memory too (WAW);
  // item memory is packed by lifetime, so later tensors reuse earlier
  // buffers.  Steps of one level are independent and share one launch.
  std::vector<int> level(wide.n_steps, -1);
  std::vector<std::vector<std::pair<long long, long long>>> reads(wide.n_steps);
  std::vector<std::pair<long long, long long>> writes(wide.n_steps, {0, 0});
  int n_levels = 0;
  for (int si = 0; si < wide.n_steps; ++si) {
    const int32_t* sr = &wide.steps[8 * si];
    if (sr[7]) continue;
    for (int i = 0; i < sr[4]; ++i) {
      const int32_t* rc = &wide.ops[(size_t)(sr[6] + i) * kWideOpInts];
      if (rc[0] != WOP_ITEM) continue;
      long long span = 1;
      for (int j = 0; j < 32; ++j) span += rc[16 + j];
      for (int j = 0; j < 16; ++j) span += rc[48 + j];
      reads[si].push_back({rc[1], rc[1] + span});
    }
    if (sr[0] == ST_ELIM) writes[si] = {sr[1], sr[1] + (1ll << sr[2])};
    auto overlap = [](std::pair<long long, long long> a, std::pair<long long, long long> b) {
      return a.first < b.second && b.first < a.second;
    };
    int lev = 0;
    for (int pj = 0; pj < si; ++pj) {
      if (level[pj] < 0 || level[pj] + 1 <= lev) continue;
      bool conflict = writes[si].second > writes[si].first && overlap(writes[si], writes[pj]);
      for (auto& r : reads[si]) conflict = conflict || overlap(r, writes[pj]);
      for (auto& r : reads[pj]) conflict = conflict || overlap(r, writes[si]);
      if (conflict) lev = level[pj] + 1;
    }
    level[si] = lev;
    n_levels = std::max(n_levels, lev + 1);
  }
  // one kernel per level; a block runs 4 wavefront tiles of one of its steps
  for (int lev = 0; lev < n_levels; ++lev) {
    WideKernel k;
    k.kind = 0;
    k.name = "wl" + std::to_string(lev);
    k.blocks = 0;
    o << "extern \"C\" __global__ void __launch_bounds__(256) " << k.name
      << "(C2* __restrict__ mem, const C2* __restrict__ cst, const unsigned long long* __restrict__ packed, "
         "unsigned long long group_elems, unsigned long long s_begin, unsigned long long n_s, int group0, "
         "int ns_log2, unsigned long long n_items, unsigned long long n_bs, C2* __restrict__ res, "
         "C2* __restrict__ gres) {\n"
      << "  const int lane = threadIdx.x & 63;\n"
      << "  const unsigned long long wv = (unsigned)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);\n"
      << "  unsigned long long item = (unsigned long long)(group0 + blockIdx.y) * 64ull + lane;\n"
      << "  const bool valid = item < n_items;\n"
      << "  if (!valid) item = n_items - 1;\n"
      << "  unsigned long long b, sl;\n"
      << "  if (ns_log2 >= 0) {\n"
      << "    b = item >> ns_log2;\n"
      << "    sl = item & (n_s - 1ull);\n"
      << "  } else {\n"
      << "    b = item / n_s;\n"
      << "    sl = item - b * n_s;\n"
      << "  }\n"
      << "  const unsigned long long s = s_begin + sl;\n"
      << "  const unsigned long long xb = packed[b];\n"
      << "  (void)s; (void)xb; (void)res; (void)gres; (void)valid; (void)sl; (void)n_bs;\n"
      << "  C2* gm = mem + (unsigned long long)blockIdx.y * group_elems * 64ull;\n"
      << "  (void)gm;\n"
      << "  const unsigned long long blk = blockIdx.x;\n";
    for (int si = 0; si < wide.n_steps; ++si) {
      if (level[si] != lev) continue;
      const int32_t* sr = &wide.steps[8 * si];
      const int kind = sr[0], out = sr[1], r = sr[2], ns = sr[3], m = sr[4], slot = sr[5], ob = sr[6];
      // tile width: unrolled loads per wavefront stay moderate, tiles stay many
      int L = std::min(r, 4);
      while (L > 0 && ((m << (L + ns)) > 192)) --L;
      while (L > 0 && r - L < 12 && (1 << (r - L)) < 2048) --L;
      const unsigned long long tiles = 1ull << (r - L);
      const unsigned long long nb = (tiles + 3) / 4;
      k.steps.push_back(si);
      o << "  if (blk >= " << k.blocks << "ull && blk < " << k.blocks + nb << "ull) {\n"
        << "  // step " << si << "\n"
        << "  const unsigned long long t = (blk - " << k.blocks << "ull) * 4ull + wv;\n"
        << "  if (t >= " << tiles << "ull) return;\n";
      k.blocks += nb;
      // per-operand base offsets from the tile index
      std::vector<const int32_t*> rec(m);
      for (int i = 0; i < m; ++i) {
        rec[i] = &wide.ops[(size_t)(ob + i) * kWideOpInts];
        o << "  const long long o" << i << " = " << rec[i][1] << "ll";
        for (int j = L; j < r; ++j)
          if (rec[i][16 + j]) o << " + (long long)((t >> " << (j - L) << ") & 1ull) * " << rec[i][16 + j] << "ll";
        if (rec[i][0] == WOP_LEAF)
          for (int d = 0; d < rec[i][2]; ++d)
            o << " + (long long)(((" << (rec[i][3 + d] ? "s" : "xb") << " >> " << rec[i][5 + d] << ") & 1ull) * "
              << rec[i][7 + d] << "ll)";
        o << ";\n";
      }
      // item operands first in every product
      std::vector<int> order;
      for (int i = 0; i < m; ++i)
        if (rec[i][0] == WOP_ITEM) order.push_back(i);
      for (int i = 0; i < m; ++i)
        if (rec[i][0] != WOP_ITEM) order.push_back(i);
      for (int lo = 0; lo < (1 << L); ++lo) {
        o << "  {\n    C2 a;\n";
        // per summed index: the operand loads, then their product
        for (int s2 = 0; s2 < (1 << ns); ++s2) {
          o << "    {\n";
          for (int i : order) {
            long long off = 0;
            for (int j = 0; j < L; ++j)
              if ((lo >> j) & 1) off += rec[i][16 + j];
            for (int j = 0; j < ns; ++j)
              if ((s2 >> j) & 1) off += rec[i][48 + j];
            o << "      const C2 v" << i << " = ";
            if (rec[i][0] == WOP_ITEM)
              o << "gm[(o" << i << " + " << off << "ll) * 64ll + lane];\n";
            else
              o << "cst[o" << i << " + " << off << "ll];\n";
          }
          std::string cur = m == 0 ? "C2{(R)1, (R)0}" : "";
          for (size_t q = 0; q < order.size(); ++q) {
            const std::string v = "v" + std::to_string(order[q]);
            cur = q == 0 ? v : "cm(" + cur + ", " + v + ")";
          }
          o << "      " << (s2 == 0 ? "a = " + cur : "a = cad(a, " + cur + ")") << ";\n    }\n";
        }
        if (kind == ST_ELIM)
          o << "    gm[(" << out << "ll + ((long long)t << " << L << ") + " << lo << "ll) * 64ll + lane] = a;\n";
        else if (kind == ST_FINAL)
          o << "    if (valid) res[sl * n_bs + b] = a;\n";
        else
          o << "    if (valid) gres[(" << slot << "ull * n_s + sl) * n_bs + b] = a;\n";
        o << "  }\n";
      }
      o << "  return;\n  }\n";
    }
    o << "}\n";
    kernels.push_back(k);
  }
  // constant steps (no fixed variable): one thread per output element,
  // strides as constants.  Runs of small steps share a single-block kernel
  // (a barrier between steps); large steps get a grid of their own.
  auto const_body = [&](int si, const std::string& c_expr) {
    const int32_t* sr = &wide.steps[8 * si];
    const int out = sr[1], r = sr[2], ns = sr[3], m = sr[4], ob = sr[6];
    for (int i = 0; i < m; ++i) {
      const int32_t* rc = &wide.ops[(size_t)(ob + i) * kWideOpInts];
      o << "    const long long o" << i << " = " << rc[1] << "ll";
      for (int j = 0; j < r; ++j)
        if (rc[16 + j]) o << " + (long long)((" << c_expr << " >> " << j << ") & 1ull) * " << rc[16 + j] << "ll";
      o << ";\n";
    }
    o << "    C2 a;\n";
    for (int s2 = 0; s2 < (1 << ns); ++s2) {
      std::string cur = m == 0 ? "C2{(R)1, (R)0}" : "";
      for (int i = 0; i < m; ++i) {
        const int32_t* rc = &wide.ops[(size_t)(ob + i) * kWideOpInts];
        long long off = 0;
        for (int j = 0; j < ns; ++j)
          if ((s2 >> j) & 1) off += rc[48 + j];
        const std::string v = "cst[o" + std::to_string(i) + " + " + std::to_string(off) + "ll]";
        cur = i == 0 ? v : "cm(" + cur + ", " + v + ")";
      }
      o << "    " << (s2 == 0 ? "a = " + cur : "a = cad(a, " + cur + ")") << ";\n";
    }
    o << "    cst[" << out << "ll + (long long)" << c_expr << "] = a;\n";
  };
  std::vector<int> run;
  auto flush_run = [&]() {
    if (run.empty()) return;
    WideKernel k;
    k.kind = 1;
    k.name = "qcb" + std::to_string(run.front());
    k.blocks = 1;
    k.steps = run;
    kernels.push_back(k);
    o << "extern \"C\" __global__ void __launch_bounds__(1024) " << k.name << "(C2* __restrict__ cst) {\n";
    for (int si : run) {
      const int r = wide.steps[8 * si + 2];
      o << "  for (unsigned long long c = threadIdx.x; c < " << (1ull << r) << "ull; c += 1024ull) {\n";
      const_body(si, "c");
      o << "  }\n  __syncthreads();\n";
    }
    o << "}\n";
    run.clear();
  };
  for (int si = 0; si < wide.n_steps; ++si) {
    if (!wide.steps[8 * si + 7]) continue;
    const int r = wide.steps[8 * si + 2];
    if (r <= 14) {
      run.push_back(si);
      continue;
    }
    flush_run();
    WideKernel k;
    k.kind = 2;
    k.name = "qc" + std::to_string(si);
    k.blocks = 1ull << r;
    k.steps = {si};
    kernels.push_back(k);
    o << "extern \"C\" __global__ void __launch_bounds__(256) " << k.name << "(C2* __restrict__ cst) {\n"
      << "  const unsigned long long c = (unsigned long long)blockIdx.x * 256ull + threadIdx.x;\n"
      << "  if (c >= " << (1ull << r) << "ull) return;\n  {\n";
    const_body(si, "c");
    o << "  }\n}\n";
  }
  flush_run();
  (void)lit;
  (void)prog;
  return o.str();
}

}  // namespace qgm
