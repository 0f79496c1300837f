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
#include <cstdlib>
#include <functional>
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

// A two-operand contraction step out[b, i, j] = sum_k A[b, i, k] B[b, k, j]
// (b: output bits both operands carry, i: those only A carries, j: only B,
// k: summed bits, carried by both) is, for each item, a batch of complex
// GEMMs.  With at least 5 i bits and 5 j bits it runs on the matrix cores
// (complex64): v_mfma_f32_32x32x1_2b_f32 computes two independent 32x32
// rank-1 updates, one per item of a pair, so a wavefront keeps a 32x32 tile
// of two item pairs (four items) and walks k, loading per k and item one
// A row element per tile row and one B row element per tile column (lane a
// of the A operand: item a / 32 of the pair, tile row a % 32; lane b of the
// B operand likewise with the tile column).  Real parts: Cr += ar br - ai bi,
// Ci += ar bi + ai br (four MFMAs per k).  Result register r of a lane l
// holds item r / 16 of the pair, tile row 8 (r % 16 / 4) + 4 (l / 32) +
// r % 4 and tile column l % 32.  A block of four wavefronts covers 16 items;
// the grid covers item quarters (fastest), the remaining j bits, the
// remaining i bits and the b bits.  Returns false when the step does not
// qualify.
bool emit_mfma_step(std::ostringstream& o, WideKernel& k, int si, int kind, int out, int r, int ns,
                    const std::vector<const int32_t*>& rec) {
  if (kind != ST_ELIM || rec.size() != 2 || rec[0][0] != WOP_ITEM || rec[1][0] != WOP_ITEM) return false;
  const int32_t* A = rec[0];
  const int32_t* B = rec[1];
  std::vector<int> bb, bi, bj, bk;
  for (int j = 0; j < r; ++j) {
    const bool a = A[16 + j] != 0, b = B[16 + j] != 0;
    if (a && b) bb.push_back(j);
    else if (a) bi.push_back(j);
    else if (b) bj.push_back(j);
    else return false;
  }
  for (int j = 0; j < ns; ++j) {
    if (A[48 + j] == 0 || B[48 + j] == 0) return false;
    bk.push_back(j);
  }
  if (bi.size() < 5 || bj.size() < 5 || bk.empty()) return false;
  // grid: item quarter (2 bits), remaining j bits, remaining i bits, b bits
  std::vector<int> gj(bj.begin() + 5, bj.end()), gi(bi.begin() + 5, bi.end());
  const int grid_bits = 2 + (int)gj.size() + (int)gi.size() + (int)bb.size();
  const unsigned long long nb = 1ull << grid_bits;
  o << "  if (blk >= " << k.blocks << "ull && blk < " << k.blocks + nb << "ull) {\n"
    << "  // step " << si << " (matrix cores)\n"
    << "  const unsigned long long g = blk - " << k.blocks << "ull;\n"
    << "  const int lid = threadIdx.x & 63;\n"
    << "  const int q0 = (int)(g & 3ull) * 16 + (int)wv * 4;\n";  // first item of the wavefront
  k.blocks += nb;
  k.steps.push_back(si);
  k.mfma_steps += 1;
  k.mfma_flops += 8.0 * (double)(1ull << (r + ns));
  // block bases of A, B and the output from the grid bits
  auto grid_sum = [&](const std::function<long long(int)>& stride_of_out_bit) {
    std::string e;
    int pos = 2;
    for (int j : gj) {
      if (stride_of_out_bit(j)) e += " + (long long)((g >> " + std::to_string(pos) + ") & 1ull) * " +
                                     std::to_string(stride_of_out_bit(j)) + "ll";
      ++pos;
    }
    for (int j : gi) {
      if (stride_of_out_bit(j)) e += " + (long long)((g >> " + std::to_string(pos) + ") & 1ull) * " +
                                     std::to_string(stride_of_out_bit(j)) + "ll";
      ++pos;
    }
    for (int j : bb) {
      if (stride_of_out_bit(j)) e += " + (long long)((g >> " + std::to_string(pos) + ") & 1ull) * " +
                                     std::to_string(stride_of_out_bit(j)) + "ll";
      ++pos;
    }
    return e;
  };
  o << "  const long long ba = " << A[1] << "ll" << grid_sum([&](int j) { return (long long)A[16 + j]; }) << ";\n"
    << "  const long long bbv = " << B[1] << "ll" << grid_sum([&](int j) { return (long long)B[16 + j]; }) << ";\n"
    << "  const long long bo = " << out << "ll" << grid_sum([&](int j) { return 1ll << j; }) << ";\n";
  // per-lane tile row of A and tile column of B
  o << "  const int tr = lid & 31;\n"
    << "  const long long la = ba";
  for (int t = 0; t < 5; ++t) o << " + (long long)((tr >> " << t << ") & 1) * " << A[16 + bi[t]] << "ll";
  o << ";\n  const long long lb = bbv";
  for (int t = 0; t < 5; ++t) o << " + (long long)((tr >> " << t << ") & 1) * " << B[16 + bj[t]] << "ll";
  o << ";\n  const int hi = lid >> 5;\n"
    << "  f32x32 cr0 = {}, ci0 = {}, cr1 = {}, ci1 = {};\n"
    << "  #pragma unroll 2\n"
    << "  for (int kk = 0; kk < " << (1 << ns) << "; ++kk) {\n"
    << "    const long long ka = la";
  for (size_t t = 0; t < bk.size(); ++t) o << " + (long long)((kk >> " << t << ") & 1) * " << A[48 + bk[t]] << "ll";
  o << ";\n    const long long kb = lb";
  for (size_t t = 0; t < bk.size(); ++t) o << " + (long long)((kk >> " << t << ") & 1) * " << B[48 + bk[t]] << "ll";
  o << ";\n"
    << "    const C2 a0 = gm[ka * 64ll + q0 + hi];\n"
    << "    const C2 b0 = gm[kb * 64ll + q0 + hi];\n"
    << "    const C2 a1 = gm[ka * 64ll + q0 + 2 + hi];\n"
    << "    const C2 b1 = gm[kb * 64ll + q0 + 2 + hi];\n"
    << "    cr0 = __builtin_amdgcn_mfma_f32_32x32x1f32(a0.x, b0.x, cr0, 0, 0, 0);\n"
    << "    ci0 = __builtin_amdgcn_mfma_f32_32x32x1f32(a0.x, b0.y, ci0, 0, 0, 0);\n"
    << "    cr1 = __builtin_amdgcn_mfma_f32_32x32x1f32(a1.x, b1.x, cr1, 0, 0, 0);\n"
    << "    ci1 = __builtin_amdgcn_mfma_f32_32x32x1f32(a1.x, b1.y, ci1, 0, 0, 0);\n"
    << "    cr0 = __builtin_amdgcn_mfma_f32_32x32x1f32(-a0.y, b0.y, cr0, 0, 0, 0);\n"
    << "    ci0 = __builtin_amdgcn_mfma_f32_32x32x1f32(a0.y, b0.x, ci0, 0, 0, 0);\n"
    << "    cr1 = __builtin_amdgcn_mfma_f32_32x32x1f32(-a1.y, b1.y, cr1, 0, 0, 0);\n"
    << "    ci1 = __builtin_amdgcn_mfma_f32_32x32x1f32(a1.y, b1.x, ci1, 0, 0, 0);\n"
    << "  }\n";
  // results: register r -> item r / 16 of the pair, tile row
  // 8 (r % 16 / 4) + 4 hi + r % 4, tile column lid % 32
  o << "  const long long oc = bo";
  for (int t = 0; t < 5; ++t) o << " + (long long)((tr >> " << t << ") & 1) * " << (1ll << bj[t]) << "ll";
  o << ";\n  const long long oh = hi ? " << (1ll << bi[2]) << "ll : 0ll;\n";
  for (int rr = 0; rr < 32; ++rr) {
    const int row = 8 * ((rr % 16) / 4) + (rr % 4);  // without the 4 hi term
    long long off = 0;
    for (int t = 0; t < 5; ++t)
      if ((row >> t) & 1) off += 1ll << bi[t];
    const int item = rr / 16;
    o << "  gm[(oc + oh + " << off << "ll) * 64ll + q0 + " << item << "] = C2{cr0[" << rr << "], ci0[" << rr
      << "]};\n"
      << "  gm[(oc + oh + " << off << "ll) * 64ll + q0 + 2 + " << item << "] = C2{cr1[" << rr << "], ci1[" << rr
      << "]};\n";
  }
  o << "  return;\n  }\n";
  return true;
}

std::string generate_wide_source(const Program& prog, const WideProgram& wide, int prec,
                                 std::vector<WideKernel>& kernels, bool mfma) {
  kernels.clear();
  std::ostringstream o;
  o << "typedef " << (prec == 0 ? "double" : "float") << " R;\n"
    << "struct C2 { R x, y; };\n"
    << "typedef float f32x32 __attribute__((ext_vector_type(32)));\n";
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
      std::vector<const int32_t*> rec(m);
      for (int i = 0; i < m; ++i) rec[i] = &wide.ops[(size_t)(ob + i) * kWideOpInts];
      if (prec == 1 && mfma && emit_mfma_step(o, k, si, kind, out, r, ns, rec)) continue;
      // Iteration order of the output bits: those that fewer item operands
      // depend on come first (inside the tile, then across neighbouring
      // wavefronts), so an operand row is reused within a tile or soon after
      // by the next tiles while it is still in cache; the bits every large
      // operand shares vary slowest.  perm[k] is the output bit at position k.
      std::vector<int> perm(r), weight(r, 0);
      for (int j = 0; j < r; ++j) {
        perm[j] = j;
        for (int i = 0; i < m; ++i) weight[j] += rec[i][0] == WOP_ITEM && rec[i][16 + j] != 0;
      }
      std::stable_sort(perm.begin(), perm.end(), [&](int x, int y) { return weight[x] < weight[y]; });
      // Tile: the first L bits of perm.  A wavefront keeps 2^L accumulators
      // (64 items each) and, per summed index, loads each operand row the
      // tile needs once: a register-blocked contraction.  L grows while the
      // accumulators and the rows per summed index stay within budget and
      // enough tiles remain to fill the GPU.
      auto rows_for = [&](int L) {
        int n = 0;
        for (int i = 0; i < m; ++i) {
          int d = 0;
          for (int k2 = 0; k2 < L; ++k2) d += rec[i][16 + perm[k2]] != 0;
          n += 1 << d;
        }
        return n;
      };
      const int max_acc = prec == 0 ? 32 : 64, max_rows = 40;
      int L = 0;
      while (L < r && (2 << L) <= max_acc && rows_for(L + 1) <= max_rows && (r - L - 1 >= 13 || (1 << (r - L - 1)) >= 2048))
        ++L;
      const unsigned long long tiles = 1ull << (r - L);
      const unsigned long long nb = (tiles + 3) / 4;
      k.steps.push_back(si);
      o << "  if (blk >= " << k.blocks << "ull && blk < " << k.blocks + nb << "ull) {\n"
        << "  // step " << si << "\n"
        << "  const unsigned long long t = (blk - " << k.blocks << "ull) * 4ull + wv;\n"
        << "  if (t >= " << tiles << "ull) return;\n";
      k.blocks += nb;
      // per-operand base offsets from the tile index
      for (int i = 0; i < m; ++i) {
        o << "  const long long o" << i << " = " << rec[i][1] << "ll";
        for (int k2 = L; k2 < r; ++k2)
          if (rec[i][16 + perm[k2]])
            o << " + (long long)((t >> " << (k2 - L) << ") & 1ull) * " << rec[i][16 + perm[k2]] << "ll";
        if (rec[i][0] == WOP_LEAF)
          for (int d = 0; d < rec[i][2]; ++d)
            o << " + (long long)(((" << (rec[i][3 + d] ? "s" : "xb") << " >> " << rec[i][5 + d] << ") & 1ull) * "
              << rec[i][7 + d] << "ll)";
        o << ";\n";
      }
      if (kind == ST_ELIM) {
        o << "  const long long ob = " << out << "ll";
        for (int k2 = L; k2 < r; ++k2)
          o << " + (long long)((t >> " << (k2 - L) << ") & 1ull) * " << (1ll << perm[k2]) << "ll";
        o << ";\n";
      }
      // item operands first in every product
      std::vector<int> order;
      for (int i = 0; i < m; ++i)
        if (rec[i][0] == WOP_ITEM) order.push_back(i);
      for (int i = 0; i < m; ++i)
        if (rec[i][0] != WOP_ITEM) order.push_back(i);
      // tile bits each operand depends on, and its row index for output lo
      std::vector<std::vector<int>> dep(m);
      for (int i = 0; i < m; ++i)
        for (int k2 = 0; k2 < L; ++k2)
          if (rec[i][16 + perm[k2]]) dep[i].push_back(k2);
      auto row_of = [&](int i, int lo) {
        int e = 0;
        for (size_t d = 0; d < dep[i].size(); ++d) e |= ((lo >> dep[i][d]) & 1) << d;
        return e;
      };
      for (int lo = 0; lo < (1 << L); ++lo) o << "  C2 a" << lo << " = C2{(R)0, (R)0};\n";
      // summed index: a loop (two iterations per pass) unless short
      const int nsum = 1 << ns;
      if (nsum > 4) o << "  #pragma unroll 2\n";
      o << "  for (int q = 0; q < " << nsum << "; ++q) {\n";
      for (int i = 0; i < m; ++i) {
        o << "    const long long p" << i << " = o" << i;
        for (int j = 0; j < ns; ++j)
          if (rec[i][48 + j]) o << " + (long long)((q >> " << j << ") & 1) * " << rec[i][48 + j] << "ll";
        o << ";\n";
      }
      for (int i : order)
        for (int e = 0; e < (1 << dep[i].size()); ++e) {
          long long off = 0;
          for (size_t d = 0; d < dep[i].size(); ++d)
            if ((e >> d) & 1) off += rec[i][16 + perm[dep[i][d]]];
          o << "    const C2 v" << i << "_" << e << " = ";
          if (rec[i][0] == WOP_ITEM)
            o << "gm[(p" << i << " + " << off << "ll) * 64ll + lane];\n";
          else
            o << "cst[p" << i << " + " << off << "ll];\n";
        }
      for (int lo = 0; lo < (1 << L); ++lo) {
        std::string cur = m == 0 ? "C2{(R)1, (R)0}" : "";
        for (size_t q2 = 0; q2 < order.size(); ++q2) {
          const int i = order[q2];
          const std::string v = "v" + std::to_string(i) + "_" + std::to_string(row_of(i, lo));
          cur = q2 == 0 ? v : "cm(" + cur + ", " + v + ")";
        }
        o << "    a" << lo << " = cad(a" << lo << ", " << cur << ");\n";
      }
      o << "  }\n";
      for (int lo = 0; lo < (1 << L); ++lo) {
        if (kind == ST_ELIM) {
          long long lo_off = 0;
          for (int j = 0; j < L; ++j)
            if ((lo >> j) & 1) lo_off += 1ll << perm[j];
          o << "  gm[(ob + " << lo_off << "ll) * 64ll + lane] = a" << lo << ";\n";
        } else if (kind == ST_FINAL) {
          o << "  if (valid) res[sl * n_bs + b] = a" << lo << ";\n";
        } else {
          o << "  if (valid) gres[(" << slot << "ull * n_s + sl) * n_bs + b] = a" << lo << ";\n";
        }
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
