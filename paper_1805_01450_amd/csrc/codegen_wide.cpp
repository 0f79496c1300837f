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
#include <cmath>
#include <cstdlib>
#include <cstring>
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
// k: summed bits, carried by both) is, per item, a batch of complex GEMMs.
// With at least 4 i bits and 4 j bits it runs on the matrix cores in the
// 16-block 4x4 forms, whose lanes match the item-major memory rows: lane l
// of an operand holds item l / 4 and tile row (A) or column (B) l % 4, and
// result register r of lane l is row r, column l % 4 of item l / 4.
//   complex64: v_mfma_f32_4x4x1_16b_f32, four real rank-1 updates per k
//     (Cr += ar br - ai bi, Ci += ar bi + ai br);
//   BF16x3: v_mfma_f32_4x4x4_16b_bf16 with each real product split into the
//     three bfloat16 products hi*hi + hi*lo + lo*hi (x = hi + lo, hi and lo
//     rounded to bfloat16; lo*lo is dropped).  A k step contributes six
//     terms to Cr and six to Ci; two k steps fill three 4-term MFMAs of each.
// A wavefront owns a 16 x 16 tile (4 x 4 MFMA blocks) of 16 items; the four
// wavefronts of a block cover 2 x 2 tiles of the same items when there are
// at least 5 i and 5 j bits, else more items.  The operand rows a block
// needs for two k (a "unit") are copied from HBM straight into LDS (16
// bytes per lane, no registers) through a ring of P stages (at most 52 KiB,
// so three blocks share a CU); P - 1 units of loads are in flight behind the
// matrix-core work, and each unit costs one block barrier.  Operand slots
// are swizzled so the LDS reads are free of bank conflicts (see the copy
// mapping below).  Blocks are numbered so that each XCD (block
// index mod 8) runs a contiguous range of tiles, j fastest within bands of
// 4 j blocks, so the operand panels a band shares stay in that XCD's L2.
// Returns false when the step does not qualify; lds_bytes receives the LDS
// the step needs.
// Output bits of a two-operand item step split into batch (both operands),
// row (A only) and column (B only) bits; false unless the step is a
// complex64 / BF16x3 two-operand contraction of the matrix-core shape.
static bool mfma_bits(int kind, int r, int ns, int prec, const std::vector<const int32_t*>& rec, std::vector<int>& bb,
                      std::vector<int>& bi, std::vector<int>& bj) {
  if (kind != ST_ELIM || rec.size() < 2 || rec.size() > 3 || rec[0][0] != WOP_ITEM || rec[1][0] != WOP_ITEM)
    return false;
  if (ns < 1 || (prec != 1 && prec != 2)) return false;
  if (rec.size() == 3) {
    // a constant scale of the output (no summed variable), applied to the results
    if (rec[2][0] != WOP_CONST) return false;
    for (int j = 0; j < ns; ++j)
      if (rec[2][48 + j] != 0) return false;
  }
  const int32_t* A = rec[0];
  const int32_t* B = rec[1];
  for (int j = 0; j < r; ++j) {
    const bool a = A[16 + j] != 0, b = B[16 + j] != 0;
    if (a && b) bb.push_back(j);
    else if (a) bi.push_back(j);
    else if (b) bj.push_back(j);
    else return false;
  }
  for (int j = 0; j < ns; ++j)
    if (A[48 + j] == 0 || B[48 + j] == 0) return false;
  return bi.size() >= 4 && bj.size() >= 4;
}

bool mfma_step_shape(const WideProgram& wide, int si, int prec, int& nb, int& ni, int& nj, int& nk) {
  const int32_t* sr = &wide.steps[8 * si];
  if (sr[7]) return false;
  std::vector<const int32_t*> rec(sr[4]);
  for (int i = 0; i < sr[4]; ++i) rec[i] = &wide.ops[(size_t)(sr[6] + i) * kWideOpInts];
  std::vector<int> bb, bi, bj;
  if (!mfma_bits(sr[0], sr[2], sr[3], prec, rec, bb, bi, bj)) return false;
  nb = (int)bb.size();
  ni = (int)bi.size();
  nj = (int)bj.size();
  nk = sr[3];
  return true;
}

// BF16x3 steps in the per-item 16 x 16 x 32 form (v_mfma_f32_16x16x32_bf16,
// the full-rate bfloat16 shape of gfx950).  Its operands are one 16 x 16
// GEMM tile of one matrix, so a wavefront owns one item: a block's four
// wavefronts take four neighbouring items (a 32-byte piece of each operand
// row) and the same TM x TN output tile of each (TM = 16 WM rows, TN = 16 WN
// columns, up to 64 x 64).  Lane l of an operand holds row (A) or column
// (B) l % 16 and eight consecutive k slots 8 (l / 16) .. 8 (l / 16) + 7; the
// result register e of lane l is row 4 (l / 16) + e, column l % 16.
// Complex k values map to slot groups: the 8 slots of lane group l / 16
// belong to complex k = 4 t + l / 16 of K step t.  With x = hi + lo (hi and
// lo rounded to bfloat16), the slots hold
//   A:          (ar_hi, ai_hi, ar_lo, ai_lo, ar_hi, ai_hi, ar_lo, ai_lo)
//   B for Cr:   (br_hi, -bi_hi, br_hi, -bi_hi, br_lo, -bi_lo, 0, 0)
//   B for Ci:   (bi_hi,  br_hi, bi_hi,  br_hi, bi_lo,  br_lo, 0, 0)
// so one MFMA pair forms, for four complex k, the six products hi*hi +
// lo*hi + hi*lo of ar br - ai bi and of ar bi + ai br: the BF16x3 terms,
// lo*lo dropped.  The A slots are the two pack-converts of the element,
// used twice; the B slots cost four pack-converts.
// Operand rows reach LDS through global_load_lds (16 bytes per lane = two
// items) in a ring of P stages of K_u complex k; LDS row slot s (32 bytes,
// four items) keeps its two item pairs swapped when bit 3 of s is set, so
// the 16 rows a lane group reads land on 16 different 8-byte bank pairs.
// Tiles are numbered with the four item quads of a 128-byte line fastest
// (they read the same lines at the same time), then j tiles, i tiles, b
// bits and the four lines of a row; each XCD takes a contiguous range.
static bool emit_mfma16_step(std::ostringstream* o_, const std::string& pre, WideKernel& k, int si, int out, int r,
                             int ns, int IT, int prec,
                             const int32_t* A, const int32_t* B, const int32_t* Sc, const std::vector<int>& bb,
                             const std::vector<int>& bi, const std::vector<int>& bj, const MfmaTile& tp,
                             bool from_table, int& lds_bytes) {
  const int ni = (int)bi.size(), nj = (int)bj.size();
  if (ni < 4 || nj < 4 || ns < 2 || (IT != 4 && IT != 8) || (prec != 1 && prec != 2)) return false;
  // IT items per block, one per wavefront: an operand row slot holds
  // SB = 8 IT bytes (LPR lanes of 16 bytes), a copy instruction RPI rows
  const int SB = 8 * IT, LPR = IT / 2, RPI = 64 / LPR, lg = IT == 4 ? 1 : 2;
  int WM = std::min(4, 1 << (ni - 4)), WN = std::min(4, 1 << (nj - 4));
  const int lay = tp.layout & 7;
  // complex64, layout + 32: the three-multiplication complex product
  const bool m3 = prec == 1 && (tp.layout & 32);
  if (lay == 4) WM = std::min(WM, 2);
  else if (lay == 5) WN = std::min(WN, 2);
  else if (lay == 6) WM = std::min(WM, 2), WN = std::min(WN, 2);
  const int nk = 1 << ns;
  // complex k per stage: 4 per K step, times the table's steps per stage
  // (at most the whole sum), and more when the copies of a stage do not
  // split evenly over the four wavefronts (32 rows per copy); a short sum
  // takes narrower tiles instead
  auto min_ku = [&]() {
    int v = 4;
    while (((16 * (WM + WN)) * v / RPI) % IT) v *= 2;
    return v;
  };
  while (min_ku() > nk && (WM > 1 || WN > 1)) {
    if (WM >= WN) WM /= 2;
    else WN /= 2;
  }
  int ku = std::max(min_ku(), std::min(nk, 4 * std::max(1, std::min(4, from_table ? tp.per : 1))));
  if (ku > nk) return false;
  const int TM = 16 * WM, TN = 16 * WN;
  const int li = 4 + (WM == 4 ? 2 : WM == 2 ? 1 : 0), lj = 4 + (WN == 4 ? 2 : WN == 2 ? 1 : 0);
  const int nbi = ni - li, nbj = nj - lj, nbb = (int)bb.size();
  // results from registers straight to HBM (table jband 1) or through LDS
  const bool direct_stores = from_table && tp.jband == 1;
  const int kub = ku == 4 ? 2 : ku == 8 ? 3 : ku == 16 ? 4 : 5;
  const int nu = nk / ku;
  const int stage = (TM + TN) * ku * SB;
  const int n_ins = (TM + TN) * ku / RPI, per_wave = n_ins / IT;
  int P = std::max(2, std::min(8, (from_table ? tp.lds_budget : 65536) / stage));
  P = std::min(P, 2 + 63 / std::max(1, per_wave));
  if (P * stage > 163840) return false;
  lds_bytes = P * stage;
  if (!o_) return true;  // shape check only
  std::ostringstream& o = *o_;
  // tile index bits, fastest first: item quads inside a 128-byte line, j
  // tiles, i tiles, b bits, the line of the 512-byte row
  std::vector<std::pair<int, int>> bits;  // (0 = j, 1 = i, 2 = b, 3 = item group; bit)
  for (int t = 0; t < (IT == 4 ? 2 : 1); ++t) bits.push_back({3, t});
  for (int t = 0; t < nbj; ++t) bits.push_back({0, bj[lj + t]});
  for (int t = 0; t < nbi; ++t) bits.push_back({1, bi[li + t]});
  for (int t = 0; t < nbb; ++t) bits.push_back({2, bb[t]});
  bits.push_back({3, 8});
  bits.push_back({3, 9});
  const unsigned long long nb = 1ull << bits.size();
  k.blocks = (k.blocks + 7) & ~7ull;
  o << "  if (blk >= " << k.blocks << "ull && blk < " << k.blocks + nb << "ull) {\n"
    << "  // step " << si << " (matrix cores, per item) b " << nbb << " i " << ni << " j " << nj << " k " << ns
    << (prec == 1 ? " fp32" : " bf16x3") << "\n"
    << pre
    << "  const unsigned long long g = blk - " << k.blocks << "ull;\n"
    << "  const unsigned long long tx = (g & 7ull) * " << (nb >> 3) << "ull + (g >> 3);\n";
  k.blocks += nb;
  k.steps.push_back(si);
  k.mfma_steps += 1;
  k.mfma_flops += 8.0 * (double)(1ull << (r + ns));
  auto sum_of = [&](const std::function<long long(int, int)>& stride) {
    std::string e;
    for (size_t p = 0; p < bits.size(); ++p) {
      if (bits[p].first == 3) continue;
      const long long s = stride(bits[p].first, bits[p].second);
      if (s) e += " + (long long)((tx >> " + std::to_string(p) + ") & 1ull) * " + std::to_string(s) + "ll";
    }
    return e;
  };
  const size_t qhi = bits.size() - 2;
  auto idx_off = [&](const int32_t* X, const std::vector<int>& v, const std::string& x, int nbits) {
    std::string e;
    for (int t = 0; t < nbits; ++t)
      e += " + (long long)(((" + x + ") >> " + std::to_string(t) + ") & 1) * " + std::to_string(X[16 + v[t]]) + "ll";
    return e;
  };
  // k offset of the low kub bits (inside a stage) and of the stage index
  auto koff = [&](const int32_t* X, const std::string& kv, int t0, int t1) {
    std::string e;
    for (int t = t0; t < t1 && t < ns; ++t)
      e += " + (long long)(((" + kv + ") >> " + std::to_string(t - t0) + ") & 1) * " + std::to_string(X[48 + t]) + "ll";
    return e;
  };
  o << "  const int lid = threadIdx.x & 63, w4 = (int)wv;\n"
    << "  const long long itb = (long long)(((tx >> " << qhi << ") & 3ull) * 16ull + (tx & " << 16 / IT - 1 << "ull) * "
    << IT << "ull);\n"
    << "  const long long ba = " << A[1] << "ll" << sum_of([&](int kd, int b) { return kd == 0 ? 0ll : (long long)A[16 + b]; })
    << ";\n"
    << "  const long long bbk = " << B[1] << "ll" << sum_of([&](int kd, int b) { return kd == 1 ? 0ll : (long long)B[16 + b]; })
    << ";\n"
    << "  const long long lo = " << out << "ll" << sum_of([&](int, int b) { return 1ll << b; }) << ";\n";
  if (Sc) {
    // the scale's element of this lane's results: tile part, then rows
    // 4 (l / 16) + .. and column l % 16
    o << "  const long long scl = " << Sc[1] << "ll" << sum_of([&](int, int b) { return (long long)Sc[16 + b]; })
      << " + (long long)((lid >> 4) & 1) * " << Sc[16 + bi[2]] << "ll + (long long)((lid >> 5) & 1) * "
      << Sc[16 + bi[3]] << "ll";
    for (int t = 0; t < 4; ++t) o << " + (long long)((lid >> " << t << ") & 1) * " << Sc[16 + bj[t]] << "ll";
    o << ";\n";
  }
  // offset in the scale of register e of tile (f, g), beyond scl
  auto sc_off = [&](int f, int g, int e) {
    long long off = 0;
    if (e & 1) off += Sc[16 + bi[0]];
    if (e & 2) off += Sc[16 + bi[1]];
    if (f & 1) off += Sc[16 + bi[4]];
    if (f & 2) off += Sc[16 + bi[5]];
    if (g & 1) off += Sc[16 + bj[4]];
    if (g & 2) off += Sc[16 + bj[5]];
    return off;
  };
  // the value stored for register e of tile C (f, g)
  auto result = [&](const std::string& C, int f, int g, int e) {
    const std::string v = "C2{cr" + C + "[" + std::to_string(e) + "], ci" + C + "[" + std::to_string(e) + "]}";
    return Sc ? "cm(" + v + ", cst[scl + " + std::to_string(sc_off(f, g, e)) + "ll])" : v;
  };
  // copies: instruction c = IT q + wave covers row slots RPI c .. RPI c +
  // RPI - 1; lane l fills 16-byte part l % LPR of slot RPI c + l / LPR with
  // the item pair (l % LPR) ^ swz(slot): swz = bit 3 of the slot for four
  // items per slot, bits 2..3 for eight.  Slots 0 .. ku TM - 1 are A rows (k
  // major), then ku TN B rows.
  const std::string swz_sl = IT == 4 ? " >> 3) & 1)" : " >> 2) & 3)";
  for (int q = 0; q < per_wave; ++q) {
    const std::string Q = std::to_string(q);
    o << "  const int sl" << Q << " = " << RPI * IT * q << " + " << RPI << " * w4 + (lid >> " << lg << ");\n"
      << "  const bool isa" << Q << " = sl" << Q << " < " << ku * TM << ";\n"
      << "  const int sr" << Q << " = isa" << Q << " ? sl" << Q << " : sl" << Q << " - " << ku * TM << ";\n"
      << "  const int kl" << Q << " = isa" << Q << " ? sr" << Q << " / " << TM << " : sr" << Q << " / " << TN << ";\n"
      << "  const int rw" << Q << " = isa" << Q << " ? sr" << Q << " % " << TM << " : sr" << Q << " % " << TN << ";\n"
      << "  const long long eo" << Q << " = isa" << Q << " ? ba" << idx_off(A, bi, "rw" + Q, li) << koff(A, "kl" + Q, 0, kub)
      << " : bbk" << idx_off(B, bj, "rw" + Q, lj) << koff(B, "kl" + Q, 0, kub) << ";\n"
      << "  const long long src" << Q << " = itb + 2 * ((lid & " << LPR - 1 << ") ^ ((sl" << Q << swz_sl << ");\n";
  }
  auto issue = [&](const std::string& unit, const std::string& stg) {
    o << "    {\n"
      << "    const long long ka = 0ll" << koff(A, unit, kub, ns) << ";\n"
      << "    const long long kb = 0ll" << koff(B, unit, kub, ns) << ";\n";
    for (int q = 0; q < per_wave; ++q) {
      const std::string Q = std::to_string(q);
      o << "    __builtin_amdgcn_global_load_lds((const void*)((isa" << Q << " ? gq0 : gq1) + (eo" << Q << " + (isa" << Q
        << " ? ka : kb)) * 64ll + src" << Q << "), (__attribute__((address_space(3))) void*)(lds + (" << stg << ") * "
        << stage << " + " << IT * 1024 * q << " + 1024 * w4), 16, 0, 0);\n";
    }
    o << "    }\n";
  };
  for (int f = 0; f < WM; ++f)
    for (int g = 0; g < WN; ++g)
      o << "  f32x4 cr" << f << "_" << g << " = {}, ci" << f << "_" << g << " = {}"
        << (m3 ? ", cs" + std::to_string(f) + "_" + std::to_string(g) + " = {}" : "") << ";\n";
  for (int s = 0; s < P - 1; ++s) issue(std::to_string(std::min(s, nu - 1)), std::to_string(s));
  // lane read offsets: slot (4 t + l / 16) TM + 16 f + l % 16 of A, item pair
  // (w4 / 2) ^ swz(slot) (swz from the low bits of l % 16), item w4 & 1 of
  // the pair
  o << "  const int rdx = " << SB << " * (lid & 15) + 16 * ((w4 >> 1) ^ ((lid" << swz_sl << ") + 8 * (w4 & 1);\n"
    << "  const int rda = rdx + " << SB * TM << " * (lid >> 4);\n"
    << "  const int rdb = rdx + " << SB * TN << " * (lid >> 4) + " << SB * ku * TM << ";\n";
  const int N = (P - 2) * per_wave;
  const int wait_imm = (N & 15) | (7 << 4) | (0 << 8) | ((N >> 4) << 14);
  o << "  for (int u = 0; u < " << nu << "; ++u) {\n"
    << "    __builtin_amdgcn_s_waitcnt(" << wait_imm << ");\n"
    << "    __asm__ volatile(\"\" ::: \"memory\");  // LDS reads of unit u - 1 stay above the barrier\n"
    << "    __builtin_amdgcn_s_barrier();  // every wave's copies of unit u are in LDS\n"
    << "    __asm__ volatile(\"\" ::: \"memory\");  // and this unit's reads below it\n"
    << "    {\n"
    << "    const int un = u + " << P - 1 << " < " << nu << " ? u + " << P - 1 << " : " << nu - 1 << ";\n";
  issue("un", "(u + " + std::to_string(P - 1) + ") % " + std::to_string(P));
  o << "    }\n"
    << "    const char* sb = lds + (u % " << P << ") * " << stage << ";\n";
  for (int t = 0; t < ku / 4 && m3; ++t) {
    // complex64, three-multiplication form: Cr += ar br, Cs += ai bi, Ci +=
    // (ar + ai)(br + bi) per tile and K step; after the sum Re = Cr - Cs and
    // Im = Ci - Cr - Cs (three FP32 16 x 16 x 4 products instead of four)
    const std::string T = std::to_string(t);
    for (int f = 0; f < WM; ++f) {
      const std::string F = T + "_" + std::to_string(f);
      o << "    const C2 a" << F << " = *(const C2*)(sb + rda + " << SB * (4 * t * TM + 16 * f) << ");\n"
        << "    const float sa" << F << " = a" << F << ".x + a" << F << ".y;\n";
    }
    for (int g = 0; g < WN; ++g) {
      const std::string G = T + "_" + std::to_string(g);
      o << "    const C2 b" << G << " = *(const C2*)(sb + rdb + " << SB * (4 * t * TN + 16 * g) << ");\n"
        << "    const float sb" << G << " = b" << G << ".x + b" << G << ".y;\n";
    }
    for (int f = 0; f < WM; ++f)
      for (int g = 0; g < WN; ++g) {
        const std::string C = std::to_string(f) + "_" + std::to_string(g);
        const std::string F = T + "_" + std::to_string(f), G = T + "_" + std::to_string(g);
        o << "    cr" << C << " = __builtin_amdgcn_mfma_f32_16x16x4f32(a" << F << ".x, b" << G << ".x, cr" << C
          << ", 0, 0, 0);\n"
          << "    cs" << C << " = __builtin_amdgcn_mfma_f32_16x16x4f32(a" << F << ".y, b" << G << ".y, cs" << C
          << ", 0, 0, 0);\n"
          << "    ci" << C << " = __builtin_amdgcn_mfma_f32_16x16x4f32(sa" << F << ", sb" << G << ", ci" << C
          << ", 0, 0, 0);\n";
      }
  }
  for (int t = 0; t < ku / 4 && prec == 1 && !m3; ++t) {
    // complex64: four FP32 16 x 16 x 4 products per tile and K step, lane
    // group l / 16 holding complex k = 4 t + l / 16 (Cr += ar br - ai bi,
    // Ci += ar bi + ai br)
    const std::string T = std::to_string(t);
    for (int f = 0; f < WM; ++f) {
      const std::string F = T + "_" + std::to_string(f);
      o << "    const C2 a" << F << " = *(const C2*)(sb + rda + " << SB * (4 * t * TM + 16 * f) << ");\n"
        << "    const float na" << F << " = -a" << F << ".y;\n";
    }
    for (int g = 0; g < WN; ++g) {
      const std::string G = T + "_" + std::to_string(g);
      o << "    const C2 b" << G << " = *(const C2*)(sb + rdb + " << SB * (4 * t * TN + 16 * g) << ");\n";
    }
    for (int f = 0; f < WM; ++f)
      for (int g = 0; g < WN; ++g) {
        const std::string C = std::to_string(f) + "_" + std::to_string(g);
        const std::string F = T + "_" + std::to_string(f), G = T + "_" + std::to_string(g);
        o << "    cr" << C << " = __builtin_amdgcn_mfma_f32_16x16x4f32(a" << F << ".x, b" << G << ".x, cr" << C
          << ", 0, 0, 0);\n"
          << "    cr" << C << " = __builtin_amdgcn_mfma_f32_16x16x4f32(na" << F << ", b" << G << ".y, cr" << C
          << ", 0, 0, 0);\n"
          << "    ci" << C << " = __builtin_amdgcn_mfma_f32_16x16x4f32(a" << F << ".x, b" << G << ".y, ci" << C
          << ", 0, 0, 0);\n"
          << "    ci" << C << " = __builtin_amdgcn_mfma_f32_16x16x4f32(a" << F << ".y, b" << G << ".x, ci" << C
          << ", 0, 0, 0);\n";
      }
  }
  for (int t = 0; t < ku / 4 && prec == 2; ++t) {
    const std::string T = std::to_string(t);
    for (int f = 0; f < WM; ++f) {
      const std::string F = T + "_" + std::to_string(f);
      o << "    const C2 a" << F << " = *(const C2*)(sb + rda + " << SB * (4 * t * TM + 16 * f) << ");\n"
        << "    const unsigned ap" << F << " = pk(a" << F << ".x, a" << F << ".y);\n"
        << "    const unsigned al" << F << " = pk(a" << F << ".x - lowf(ap" << F << "), a" << F << ".y - highf(ap" << F
        << "));\n"
        << "    const bf16x8 A" << F << " = __builtin_bit_cast(bf16x8, (u32x4){ap" << F << ", al" << F << ", ap" << F
        << ", al" << F << "});\n";
    }
    for (int g = 0; g < WN; ++g) {
      const std::string G = T + "_" + std::to_string(g);
      o << "    const C2 b" << G << " = *(const C2*)(sb + rdb + " << SB * (4 * t * TN + 16 * g) << ");\n"
        << "    const unsigned bq" << G << " = pk(b" << G << ".x, -b" << G << ".y);\n"
        << "    const unsigned bs" << G << " = pk(b" << G << ".y, b" << G << ".x);\n"
        << "    const float brl" << G << " = b" << G << ".x - lowf(bq" << G << "), bil" << G << " = b" << G
        << ".y - lowf(bs" << G << ");\n"
        << "    const bf16x8 R" << G << " = __builtin_bit_cast(bf16x8, (u32x4){bq" << G << ", bq" << G << ", pk(brl" << G
        << ", -bil" << G << "), 0u});\n"
        << "    const bf16x8 I" << G << " = __builtin_bit_cast(bf16x8, (u32x4){bs" << G << ", bs" << G << ", pk(bil" << G
        << ", brl" << G << "), 0u});\n";
    }
    for (int f = 0; f < WM; ++f)
      for (int g = 0; g < WN; ++g) {
        const std::string C = std::to_string(f) + "_" + std::to_string(g);
        const std::string F = T + "_" + std::to_string(f), G = T + "_" + std::to_string(g);
        o << "    cr" << C << " = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A" << F << ", R" << G << ", cr" << C
          << ", 0, 0, 0);\n"
          << "    ci" << C << " = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A" << F << ", I" << G << ", ci" << C
          << ", 0, 0, 0);\n";
      }
  }
  o << "  }\n"
    << "  __builtin_amdgcn_s_waitcnt(" << ((7 << 4) | (15 << 8)) << ");  // no copy left in flight\n";
  if (m3)
    for (int f = 0; f < WM; ++f)
      for (int g = 0; g < WN; ++g) {
        const std::string C = std::to_string(f) + "_" + std::to_string(g);
        o << "  ci" << C << " = ci" << C << " - (cr" << C << " + cs" << C << ");\n"
          << "  cr" << C << " = cr" << C << " - cs" << C << ";\n";
      }
  // results: register e of tile (f, g) is row 16 f + 4 (l / 16) + e, column
  // 16 g + l % 16, item itb + w4
  auto fg_off = [&](int f, int g) {
    long long off = 0;
    if (f & 1) off += 1ll << bi[4];
    if (f & 2) off += 1ll << bi[5];
    if (g & 1) off += 1ll << bj[4];
    if (g & 2) off += 1ll << bj[5];
    return off;
  };
  if (!direct_stores) {
    // Through LDS, ncb 16 x 16 tiles at a time: each wavefront writes its
    // item's values as [element][IT items] (8 bytes each; item slot w4 ^ f,
    // f = (element >> 3) & 3 for four items, 2 ((element >> 2) & 3) for
    // eight, so that a lane group's writes spread over the banks); then each
    // thread stores 16 bytes (two items of one element), neighbouring
    // threads the parts of one element's 8 IT-byte piece.
    int ncb = 1;  // tiles per round: a power of two that divides WM WN
    while (2 * ncb <= WM * WN && 2 * ncb * 2048 * IT <= lds_bytes) ncb *= 2;
    o << "  const int wre = 64 * (lid >> 4);\n"
      << "  const int tt = threadIdx.x;\n"
      << "  const long long seo = lo";
    for (int t = 0; t < 3; ++t) o << " + (long long)((tt >> " << lg + 4 + t << ") & 1) * " << (1ll << bi[t]) << "ll";
    for (int t = 0; t < 4; ++t) o << " + (long long)((tt >> " << lg + t << ") & 1) * " << (1ll << bj[t]) << "ll";
    o << ";\n";
    if (IT == 4)
      o << "  const long long sit = itb + 2 * ((tt & 1) ^ ((tt >> 5) & 1));\n"
        << "  const bool sws = (tt >> 4) & 1;\n";
    else
      o << "  const long long sit = itb + 2 * ((tt & 3) ^ ((tt >> 4) & 3));\n";
    for (int c0 = 0; c0 < WM * WN; c0 += ncb) {
      o << "  __syncthreads();\n";
      for (int cb = 0; cb < ncb; ++cb) {
        const int f = (c0 + cb) / WN, g = (c0 + cb) % WN;
        const std::string C = std::to_string(f) + "_" + std::to_string(g);
        for (int e = 0; e < 4; ++e) {
          o << "  *(C2*)(lds + ((" << 256 * cb + 16 * e << " + wre + (lid & 15)) * " << IT << " + (w4 ^ ";
          if (IT == 4)
            o << "((" << 2 * e << " + ((lid >> 3) & 1)) & 3)";
          else
            o << "(2 * ((lid >> 2) & 3))";
          o << ")) * 8) = " << result(C, f, g, e) << ";\n";
        }
      }
      o << "  __syncthreads();\n";
      for (int it = 0; it < 2 * ncb; ++it) {
        const int cb = it >> 1, f = (c0 + cb) / WN, g = (c0 + cb) % WN;
        long long off = fg_off(f, g) + ((it & 1) ? 1ll << bi[3] : 0);
        o << "  {\n"
          << "  const f32x4 v = *(const f32x4*)(lds + " << 1024 * IT * it << " + 16 * tt);\n"
          << "  *(f32x4*)(gm + (seo + " << off << "ll) * 64ll + sit) = "
          << (IT == 4 ? "sws ? (f32x4){v[2], v[3], v[0], v[1]} : v;\n" : "v;\n")
          << "  }\n";
      }
    }
  } else {
    o << "  const long long so = lo" << " + (long long)((lid >> 4) & 1) * " << (1ll << bi[2]) << "ll + (long long)((lid >> 5) & 1) * "
      << (1ll << bi[3]) << "ll";
    for (int t = 0; t < 4; ++t) o << " + (long long)((lid >> " << t << ") & 1) * " << (1ll << bj[t]) << "ll";
    o << ";\n"
      << "  const long long sit = itb + w4;\n";
    for (int f = 0; f < WM; ++f)
      for (int g = 0; g < WN; ++g)
        for (int e = 0; e < 4; ++e) {
          long long off = fg_off(f, g);
          if (e & 1) off += 1ll << bi[0];
          if (e & 2) off += 1ll << bi[1];
          const std::string C = std::to_string(f) + "_" + std::to_string(g);
          o << "  gm[(so + " << off << "ll) * 64ll + sit] = " << result(C, f, g, e) << ";\n";
        }
  }
  o << "  return;\n  }\n";
  return true;
}

// The tile table entry of a matrix-core step's shape, if any.
static bool table_tile(const TileTable* tiles, int prec, int ni, int nj, int ns, MfmaTile& tp) {
  if (!tiles) return false;
  auto it = tiles->find(TileKey{prec, ni, nj, ns});
  if (it == tiles->end()) return false;
  tp = it->second;
  return true;
}

// Form choice of a matrix-core step.  Table layouts: 1, 2, 3 = 16-item
// variants (7 = their built-in choice); 0, 4, 5, 6 = per-item full tile,
// at most 32 rows, 32 columns, both (BF16x3), or the same plus 16 (either
// precision); + 8 = eight items per block.  Built in: BF16x3 per-item for
// sums of 32 or more k (on shorter sums, where the results' stores
// dominate, the 16-item forms store whole 128-byte lines and were as fast
// or faster), complex64 the 16-item form.
static bool per_item_choice(int prec, bool from_table, const MfmaTile& tp, int ns, MfmaTile& t16, int& it_pref) {
  const int lay = tp.layout & 7;
  const bool variant = lay == 0 || (lay >= 4 && lay <= 6);
  bool per_item;
  if (prec == 2)
    per_item = from_table ? (tp.layout & 16) || variant : ns >= 5;
  else
    per_item = prec == 1 && from_table && (tp.layout & 16) && variant;
  t16 = from_table ? tp : MfmaTile{2, 65536, 0, 0};
  t16.layout = lay | (tp.layout & 32);
  it_pref = from_table && (tp.layout & 8) ? 8 : 4;
  return per_item;
}

// Block sizes a step can run at in a level kernel: bit 0 = four wavefronts,
// bit 1 = eight, bit 2 = it asks for eight (a per-item step whose table
// entry has eight items per block).  Vector steps take either; 16-item
// matrix-core steps need four.
static int step_waves(int kind, int r, int ns, int prec, const std::vector<const int32_t*>& rec, bool mfma,
                      const TileTable* tiles) {
  std::vector<int> bb, bi, bj;
  if (!mfma || !mfma_bits(kind, r, ns, prec, rec, bb, bi, bj)) return 3;
  MfmaTile tp, t16;
  const bool from_table = table_tile(tiles, prec, (int)bi.size(), (int)bj.size(), ns, tp);
  int it_pref = 4, lds = 0;
  if (!per_item_choice(prec, from_table, tp, ns, t16, it_pref)) return 1;
  WideKernel scratch;
  const bool ok8 = emit_mfma16_step(nullptr, std::string(), scratch, 0, 0, r, ns, 8, prec, rec[0], rec[1], nullptr, bb,
                                    bi, bj, t16, true, lds);
  return 1 | (ok8 ? 2 : 0) | (ok8 && it_pref == 8 ? 4 : 0);
}

bool emit_mfma_step(std::ostringstream& o, const std::string& pre, WideKernel& k, int si, int kind, int out, int r,
                    int ns, int prec,
                    const std::vector<const int32_t*>& rec, int& lds_bytes, const TileTable* tiles, int W) {
  std::vector<int> bb, bi, bj;
  if (!mfma_bits(kind, r, ns, prec, rec, bb, bi, bj)) return false;
  const int32_t* A = rec[0];
  const int32_t* B = rec[1];
  const int32_t* Sc = rec.size() == 3 ? rec[2] : nullptr;  // constant scale of the results
  // Tile parameters: a tuned table entry for this shape, else the built-in
  // choice (2 x 2 tiles of 16 items when both sides have 5 bits, two k per
  // unit, a ring of at most 52 KiB, bands of four j blocks).
  MfmaTile tp;
  const bool from_table = table_tile(tiles, prec, (int)bi.size(), (int)bj.size(), ns, tp);
  // the per-item form, as many items per block as the level kernel has
  // wavefronts, or the 16-item forms, which need four wavefronts
  {
    MfmaTile t16;
    int it_pref = 4;
    if (per_item_choice(prec, from_table, tp, ns, t16, it_pref) &&
        emit_mfma16_step(&o, pre, k, si, out, r, ns, W, prec, A, B, Sc, bb, bi, bj, t16, true, lds_bytes))
      return true;
  }
  if (W != 4) return false;
  tp.layout &= 7;
  if (tp.layout >= 4) tp.layout = 0;
  int WI = bi.size() >= 5 ? 2 : 1, WJ = bj.size() >= 5 ? 2 : 1;
  if (tp.layout == 1) WI = WJ = 1;                                   // four item groups
  else if (tp.layout == 2 && bi.size() >= 5) WI = 2, WJ = 1;         // two i tiles x two item groups
  else if (tp.layout == 3 && bj.size() >= 5) WI = 1, WJ = 2;         // two j tiles x two item groups
  const int WQ = 4 / (WI * WJ);
  const int li = WI == 2 ? 5 : 4, lj = WJ == 2 ? 5 : 4;  // i / j bits inside a block
  const int nbi = (int)bi.size() - li, nbj = (int)bj.size() - lj, nbb = (int)bb.size();
  const int nqg = 4 / WQ;  // item groups of 16 * WQ items
  const int grid_bits = nbj + nbi + nbb + (nqg == 4 ? 2 : nqg == 2 ? 1 : 0);
  const unsigned long long nb = 1ull << grid_bits;
  const int nk = 1 << ns;
  // k steps per unit (one barrier each); BF16x3 pairs the k steps
  int per = std::min(nk, std::max(prec == 2 ? 2 : 1, tp.per));
  if (prec == 2 && per % 2) per = 2;
  const int nu = nk / per;                            // units
  const int a_bytes = 16 * WI * 16 * WQ * 8;          // A rows of one k
  const int b_bytes = 16 * WJ * 16 * WQ * 8;
  const int stage = per * (a_bytes + b_bytes);
  const int nA = a_bytes / 1024, nB = b_bytes / 1024;  // 1 KiB copies per k
  const int n_ins = per * (nA + nB), per_wave = n_ins / 4;
  // ring depth: what the LDS budget holds, 2..8 stages, and at most what the
  // 6-bit load counter can wait for ((P - 2) copies per wave in flight)
  int P = std::max(2, std::min(8, tp.lds_budget / stage));
  P = std::min(P, 2 + 63 / std::max(1, per_wave));
  if (P * stage > 163840) return false;
  lds_bytes = P * stage;
  // block ranges start at multiples of 8 so that blk & 7 is the XCD
  k.blocks = (k.blocks + 7) & ~7ull;
  o << "  if (blk >= " << k.blocks << "ull && blk < " << k.blocks + nb << "ull) {\n"
    << "  // step " << si << " (matrix cores) b " << nbb << " i " << bi.size() << " j " << bj.size() << " k " << ns << "\n"
    << pre
    << "  const unsigned long long g = blk - " << k.blocks << "ull;\n";
  if (nb >= 8)
    o << "  const unsigned long long tx = (g & 7ull) * " << (nb >> 3) << "ull + (g >> 3);\n";
  else
    o << "  const unsigned long long tx = g;\n";
  k.blocks += nb;
  k.steps.push_back(si);
  k.mfma_steps += 1;
  k.mfma_flops += 8.0 * (double)(1ull << (r + ns));
  // tile index bits, fastest first: j blocks inside a band of up to
  // 2^jband, i blocks, the remaining j bits (bands), b bits, item groups
  const int jband = std::min(nbj, tp.jband);
  std::vector<std::pair<int, int>> bits;  // (kind 0 = j, 1 = i, 2 = b; out bit)
  for (int t = 0; t < jband; ++t) bits.push_back({0, bj[lj + t]});
  for (int t = 0; t < nbi; ++t) bits.push_back({1, bi[li + t]});
  for (int t = jband; t < nbj; ++t) bits.push_back({0, bj[lj + t]});
  for (int t = 0; t < nbb; ++t) bits.push_back({2, bb[t]});
  auto sum_of = [&](const std::function<long long(int, int)>& stride) {
    std::string e;
    for (size_t p = 0; p < bits.size(); ++p) {
      const long long s = stride(bits[p].first, bits[p].second);
      if (s) e += " + (long long)((tx >> " + std::to_string(p) + ") & 1ull) * " + std::to_string(s) + "ll";
    }
    return e;
  };
  const size_t qpos = bits.size();
  // row (A) / column (B) offset of block-local index x over the operand's
  // bits v[0..]
  auto idx_off = [&](const int32_t* X, const std::vector<int>& v, const std::string& x, int nbits) {
    std::string e;
    for (int t = 0; t < nbits; ++t)
      e += " + (long long)(((" + x + ") >> " + std::to_string(t) + ") & 1) * " + std::to_string(X[16 + v[t]]) + "ll";
    return e;
  };
  auto koff = [&](const int32_t* X, const std::string& kv) {
    std::string e;
    for (int t = 0; t < ns; ++t)
      e += " + (long long)(((" + kv + ") >> " + std::to_string(t) + ") & 1) * " + std::to_string(X[48 + t]) + "ll";
    return e;
  };
  o << "  const int lid = threadIdx.x & 63, sub = lid & 3, w4 = (int)wv;\n"
    << "  const int wi = " << (WI == 2 ? "w4 & 1" : "0") << ", wj = "
    << (WJ == 2 ? (WI == 2 ? "(w4 >> 1) & 1" : "w4 & 1") : "0")
    << ", wq = " << (WQ == 1 ? "0" : WI * WJ == 2 ? "w4 >> 1" : "w4") << ";\n"
    << "  const long long itb = (long long)(" << (nqg > 1 ? "(tx >> " + std::to_string(qpos) + ")" : "0ull")
    << " * " << 16 * WQ << "ull);\n"
    << "  const long long ba = " << A[1] << "ll" << sum_of([&](int kd, int b) { return kd == 0 ? 0ll : (long long)A[16 + b]; })
    << ";\n"
    << "  const long long bbk = " << B[1] << "ll" << sum_of([&](int kd, int b) { return kd == 1 ? 0ll : (long long)B[16 + b]; })
    << ";\n"
    << "  const long long lo = " << out << "ll" << sum_of([&](int, int b) { return 1ll << b; })
    << (WI == 2 ? " + (long long)wi * " + std::to_string(1ll << bi[4]) + "ll" : "")
    << (WJ == 2 ? " + (long long)wj * " + std::to_string(1ll << bj[4]) + "ll" : "")
    << " + (long long)(sub & 1) * " << (1ll << bj[0]) << "ll + (long long)(sub >> 1) * " << (1ll << bj[1]) << "ll;\n"
    << "  const int it = (int)itb + wq * 16 + (lid >> 2);\n";
  if (Sc)  // the scale's element of this lane's results (as lo, with the scale's strides)
    o << "  const long long scl = " << Sc[1] << "ll" << sum_of([&](int, int b) { return (long long)Sc[16 + b]; })
      << (WI == 2 ? " + (long long)wi * " + std::to_string(Sc[16 + bi[4]]) + "ll" : "")
      << (WJ == 2 ? " + (long long)wj * " + std::to_string(Sc[16 + bj[4]]) + "ll" : "")
      << " + (long long)(sub & 1) * " << Sc[16 + bj[0]] << "ll + (long long)(sub >> 1) * " << Sc[16 + bj[1]]
      << "ll;\n";
  // Copies: instruction j = 4 q + wave of a unit; j < per nA: A rows, else
  // B rows.  A copy moves 1 KiB = 1024 / (128 WQ) rows of 16 WQ items into
  // LDS slots of 16 bytes (two items of one row), 8 WQ slots per row: lane
  // l fills slot l % (8 WQ) of row l / (8 WQ) of the copy.  Slot t of row r
  // holds the item pair t ^ 2 (r % 4): the operand reads of 16 lanes (4
  // rows x 4 items) then fall on 16 different 8-byte bank pairs (without
  // the swizzle the 4 rows, 8 WQ slots apart, share banks).  Per copy: the
  // lane's element offset without the k part, its item pair and the LDS
  // byte offset inside a stage.
  const int rows_per = 8 / WQ;
  o << "  const int lrow = lid / " << 8 * WQ << ", lch = lid % " << 8 * WQ << ";\n"
    << "  const int xo = ((((16 * wq + (lid >> 2)) >> 1) ^ (2 * sub)) * 16) + ((lid >> 2) & 1) * 8;\n";
  for (int q = 0; q < per_wave; ++q) {
    o << "  const int j" << q << " = " << 4 * q << " + w4;\n";
    // which operand and which k of the unit: the A copies come first
    o << "  const bool isa" << q << " = j" << q << " < " << per * nA << ";\n"
      << "  const int jr" << q << " = isa" << q << " ? j" << q << " : j" << q << " - " << per * nA << ";\n"
      << "  const int h" << q << " = isa" << q << " ? jr" << q << " / " << nA << " : jr" << q << " / " << nB << ";\n"
      << "  const int c" << q << " = isa" << q << " ? jr" << q << " % " << nA << " : jr" << q << " % " << nB << ";\n"
      << "  const int rw" << q << " = c" << q << " * " << rows_per << " + lrow;\n"
      << "  const int pq" << q << " = lch ^ (2 * (rw" << q << " & 3));\n"
      << "  const long long eo" << q << " = isa" << q << " ? ba" << idx_off(A, bi, "rw" + std::to_string(q), li)
      << " : bbk" << idx_off(B, bj, "rw" + std::to_string(q), lj) << ";\n"
      << "  const unsigned lds" << q << " = (unsigned)(h" << q << " * " << (a_bytes + b_bytes) << " + (isa" << q
      << " ? 0 : " << a_bytes << ") + c" << q << " * 1024);\n";
  }
  auto issue = [&](const std::string& unit, const std::string& stg) {
    for (int q = 0; q < per_wave; ++q) {
      const std::string Q = std::to_string(q);
      const std::string kv = per == 1 ? "(" + unit + ")" : "(" + std::to_string(per) + " * (" + unit + ") + h" + Q + ")";
      o << "    {\n"
        << "    const long long e = eo" << Q << " + (isa" << Q << " ? 0ll" << koff(A, kv) << " : 0ll" << koff(B, kv)
        << ");\n"
        << "    __builtin_amdgcn_global_load_lds((const void*)((isa" << Q << " ? gq0 : gq1) + e * 64ll + itb + 2 * pq" << Q
        << "), "
        << "(__attribute__((address_space(3))) void*)(lds + (" << stg << ") * " << stage << " + lds" << Q
        << "), 16, 0, 0);\n"
        << "    }\n";
    }
  };
  for (int g = 0; g < 4; ++g)
    o << "  f32x4 cr" << g << "_0 = {}, cr" << g << "_1 = {}, cr" << g << "_2 = {}, cr" << g << "_3 = {};\n"
      << "  f32x4 ci" << g << "_0 = {}, ci" << g << "_1 = {}, ci" << g << "_2 = {}, ci" << g << "_3 = {};\n";
  // prologue: units 0 .. P - 2 (clamped to the last unit)
  for (int s = 0; s < P - 1; ++s) issue(std::to_string(std::min(s, nu - 1)), std::to_string(s));
  // vmcnt(N) and lgkmcnt(0): this wave's copies of unit u have landed and
  // its LDS reads of unit u - 1 have completed (a read still in flight at
  // the barrier could see the copy another wave issues right after it into
  // that stage)
  const int N = (P - 2) * per_wave;
  const int wait_imm = (N & 15) | (7 << 4) | (0 << 8) | ((N >> 4) << 14);
  o << "  for (int u = 0; u < " << nu << "; ++u) {\n"
    << "    __builtin_amdgcn_s_waitcnt(" << wait_imm << ");\n"
    << "    __asm__ volatile(\"\" ::: \"memory\");  // LDS reads of unit u - 1 stay above the barrier\n"
    << "    __builtin_amdgcn_s_barrier();  // every wave's copies of unit u are in LDS\n"
    << "    __asm__ volatile(\"\" ::: \"memory\");  // and this unit's reads below it\n"
    << "    {\n"
    << "    const int un = u + " << P - 1 << " < " << nu << " ? u + " << P - 1 << " : " << nu - 1 << ";\n";
  issue("un", "(u + " + std::to_string(P - 1) + ") % " + std::to_string(P));
  o << "    }\n"
    << "    const char* sb = lds + (u % " << P << ") * " << stage << ";\n";
  // operand reads: A row 16 wi + 4 rg + sub, B column 16 wj + 4 cg + sub,
  // item 16 wq + lid / 4, in slot (item / 2) ^ 2 sub of its row
  for (int h = 0; h < per; ++h) {
    for (int g = 0; g < 4; ++g)
      o << "    const C2 a" << h << "_" << g << " = *(const C2*)(sb + " << h * (a_bytes + b_bytes) << " + (16 * wi + "
        << 4 * g << " + sub) * " << 128 * WQ << " + xo);\n";
    for (int g = 0; g < 4; ++g)
      o << "    const C2 b" << h << "_" << g << " = *(const C2*)(sb + " << h * (a_bytes + b_bytes) + a_bytes
        << " + (16 * wj + " << 4 * g << " + sub) * " << 128 * WQ << " + xo);\n";
  }
  if (prec == 1) {
    for (int h = 0; h < per; ++h) {
      const std::string H = std::to_string(h);
      for (int g = 0; g < 4; ++g) o << "    const float na" << H << g << " = -a" << H << "_" << g << ".y;\n";
      for (int rg = 0; rg < 4; ++rg)
        for (int cg = 0; cg < 4; ++cg) {
          const std::string cr = "cr" + std::to_string(rg) + "_" + std::to_string(cg);
          const std::string ci = "ci" + std::to_string(rg) + "_" + std::to_string(cg);
          const std::string a = "a" + H + "_" + std::to_string(rg), b = "b" + H + "_" + std::to_string(cg);
          o << "    " << cr << " = __builtin_amdgcn_mfma_f32_4x4x1f32(" << a << ".x, " << b << ".x, " << cr << ", 0, 0, 0);\n"
            << "    " << ci << " = __builtin_amdgcn_mfma_f32_4x4x1f32(" << a << ".x, " << b << ".y, " << ci << ", 0, 0, 0);\n"
            << "    " << cr << " = __builtin_amdgcn_mfma_f32_4x4x1f32(na" << H << rg << ", " << b << ".y, " << cr
            << ", 0, 0, 0);\n"
            << "    " << ci << " = __builtin_amdgcn_mfma_f32_4x4x1f32(" << a << ".y, " << b << ".x, " << ci << ", 0, 0, 0);\n";
        }
    }
  } else {
    // k steps in pairs: 12 terms for Cr and 12 for Ci in three 4-slot
    // bfloat16 operands each; the A slots are shared by Cr and Ci.
    //   A: (rh rh rl ih | ih il) per k;  B for Cr: (rh rl rh -ih | -il -ih);
    //   B for Ci: (ih il ih rh | rl rh)   (r = real, i = imaginary part)
    for (int hp = 0; hp < per / 2; ++hp) {
      const std::string h0 = std::to_string(2 * hp), h1 = std::to_string(2 * hp + 1);
      for (int g = 0; g < 4; ++g) {
        const std::string G = std::to_string(g);
        const std::string S = std::to_string(hp) + "_" + G;  // pair, group
        o << "    s16x4 A" << S << "_0, A" << S << "_1, A" << S << "_2;\n"
          << "    bsplit(a" << h0 << "_" << G << ", a" << h1 << "_" << G << ", A" << S << "_0, A" << S << "_1, A" << S
          << "_2);\n"
          << "    s16x4 R" << S << "_0, R" << S << "_1, R" << S << "_2, I" << S << "_0, I" << S << "_1, I" << S << "_2;\n"
          << "    bsplitb(b" << h0 << "_" << G << ", b" << h1 << "_" << G << ", R" << S << "_0, R" << S << "_1, R" << S
          << "_2, I" << S << "_0, I" << S << "_1, I" << S << "_2);\n";
      }
      for (int rg = 0; rg < 4; ++rg)
        for (int cg = 0; cg < 4; ++cg) {
          const std::string cr = "cr" + std::to_string(rg) + "_" + std::to_string(cg);
          const std::string ci = "ci" + std::to_string(rg) + "_" + std::to_string(cg);
          for (int t = 0; t < 3; ++t) {
            const std::string T = "_" + std::to_string(t);
            const std::string a = "A" + std::to_string(hp) + "_" + std::to_string(rg) + T;
            const std::string rr = "R" + std::to_string(hp) + "_" + std::to_string(cg) + T;
            const std::string ii = "I" + std::to_string(hp) + "_" + std::to_string(cg) + T;
            o << "    " << cr << " = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(" << a << ", " << rr << ", " << cr
              << ", 0, 0, 0);\n"
              << "    " << ci << " = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(" << a << ", " << ii << ", " << ci
              << ", 0, 0, 0);\n";
          }
        }
    }
  }
  o << "  }\n"
    << "  __builtin_amdgcn_s_waitcnt(" << ((7 << 4) | (15 << 8)) << ");  // no copy left in flight\n";
  // results: register e of block (rg, cg) -> row bits (e, rg) on i bits
  // 0..3, column bits (sub, cg) on j bits 0..3, item it
  for (int rg = 0; rg < 4; ++rg)
    for (int cg = 0; cg < 4; ++cg)
      for (int e = 0; e < 4; ++e) {
        const int row = e + 4 * rg;
        long long off = 0;
        for (int t = 0; t < 4; ++t)
          if ((row >> t) & 1) off += 1ll << bi[t];
        if (cg & 1) off += 1ll << bj[2];
        if (cg & 2) off += 1ll << bj[3];
        const std::string v = "C2{cr" + std::to_string(rg) + "_" + std::to_string(cg) + "[" + std::to_string(e) +
                              "], ci" + std::to_string(rg) + "_" + std::to_string(cg) + "[" + std::to_string(e) + "]}";
        if (Sc) {
          long long soff = 0;
          for (int t = 0; t < 4; ++t)
            if ((row >> t) & 1) soff += Sc[16 + bi[t]];
          if (cg & 1) soff += Sc[16 + bj[2]];
          if (cg & 2) soff += Sc[16 + bj[3]];
          o << "  gm[(lo + " << off << "ll) * 64ll + it] = cm(" << v << ", cst[scl + " << soff << "ll]);\n";
        } else {
          o << "  gm[(lo + " << off << "ll) * 64ll + it] = " << v << ";\n";
        }
      }
  o << "  return;\n  }\n";
  return true;
}

bool read_tile_table(const std::string& path, TileTable& t, std::string& err) {
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) {
    err = "cannot open tile table " + path;
    return false;
  }
  char line[512];
  int ln = 0;
  bool ok = true;
  while (ok && std::fgets(line, sizeof(line), f)) {
    ++ln;
    char* hash = std::strchr(line, '#');
    if (hash) *hash = 0;
    int v[8];
    int n = std::sscanf(line, "%d %d %d %d %d %d %d %d", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5], &v[6], &v[7]);
    if (n <= 0) continue;  // blank or comment
    if (n != 8 || v[0] < 0 || v[0] > 2 || v[1] < 4 || v[2] < 4 || v[3] < 1 || v[3] > 16 || v[4] < 1 || v[4] > 16 ||
        (v[4] & (v[4] - 1)) || v[5] < 1024 || v[5] > 163840 || v[6] < 0 || v[6] > 8 || v[7] < 0 || v[7] > 63) {
      err = "tile table " + path + " line " + std::to_string(ln) + ": expected prec ni nj nk per lds_budget jband layout";
      ok = false;
      break;
    }
    t[TileKey{v[0], v[1], v[2], v[3]}] = MfmaTile{v[4], v[5], v[6], v[7]};
  }
  std::fclose(f);
  return ok;
}

bool write_tile_table(const std::string& path, const TileTable& t, std::string& err) {
  FILE* f = std::fopen(path.c_str(), "w");
  if (!f) {
    err = "cannot write tile table " + path;
    return false;
  }
  std::fprintf(f, "# qgm matrix-core tile table: prec ni nj nk per lds_budget jband layout\n");
  for (const auto& e : t)
    std::fprintf(f, "%d %d %d %d %d %d %d %d\n", e.first.prec, e.first.ni, e.first.nj, e.first.nk, e.second.per,
                 e.second.lds_budget, e.second.jband, e.second.layout);
  const bool ok = std::fclose(f) == 0;
  if (!ok) err = "write failed: " + path;
  return ok;
}

std::string generate_wide_source(const Program& prog, const WideProgram& wide, int prec,
                                 std::vector<WideKernel>& kernels, bool mfma, const TileTable* tiles) {
  kernels.clear();
  std::ostringstream o;
  o << "typedef " << (prec == 0 ? "double" : "float") << " R;\n"
    << "struct C2 { R x, y; };\n"
    << "typedef float f32x4 __attribute__((ext_vector_type(4)));\n"
    << "typedef short s16x4 __attribute__((ext_vector_type(4)));\n";
  if (prec == 2)
    o << "typedef float bf_f32x2 __attribute__((ext_vector_type(2)));\n"
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
         "c.y = (arh * bih + (arh * bil + arl * bih)) + (aih * brh + (aih * brl + ail * brh)); return c; }\n"
         // bfloat16 halves for the matrix-core form: x = hi + lo, hi and lo
         // rounded to nearest even (the hardware pack-convert, two at a
         // time); operands as packed 4 x bfloat16
         "typedef float f32x2 __attribute__((ext_vector_type(2)));\n"
         "typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));\n"
         "static __device__ __forceinline__ unsigned pk(float a, float b) { "
         "return __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){a, b}, bf16x2)); }\n"
         "static __device__ __forceinline__ float lowf(unsigned p) { return __uint_as_float(p << 16); }\n"
         "static __device__ __forceinline__ float highf(unsigned p) { return __uint_as_float(p & 0xFFFF0000u); }\n"
         "typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;\n"
         "typedef unsigned u32x4 __attribute__((ext_vector_type(4)));\n"
         "static __device__ __forceinline__ s16x4 v4(unsigned lo, unsigned hi) { "
         "return __builtin_bit_cast(s16x4, (unsigned long long)lo | ((unsigned long long)hi << 32)); }\n"
         // A slots (rh rh rl ih | ih il) per k, k = p then q
         "static __device__ __forceinline__ void bsplit(C2 p, C2 q, s16x4& A0, s16x4& A1, s16x4& A2) { "
         "const unsigned prr = pk(p.x, p.x), pii = pk(p.y, p.y), qrr = pk(q.x, q.x), qii = pk(q.y, q.y); "
         "const float prl = p.x - lowf(prr), pil = p.y - lowf(pii), qrl = q.x - lowf(qrr), qil = q.y - lowf(qii); "
         "A0 = v4(prr, pk(prl, p.y)); A1 = v4(pk(p.y, pil), qrr); A2 = v4(pk(qrl, q.y), pk(q.y, qil)); }\n"
         // B slots for Cr (rh rl rh -ih | -il -ih) and for Ci (ih il ih rh | rl rh)
         "static __device__ __forceinline__ void bsplitb(C2 p, C2 q, s16x4& R0, s16x4& R1, s16x4& R2, s16x4& I0, "
         "s16x4& I1, s16x4& I2) { "
         "const unsigned prr = pk(p.x, p.x), pii = pk(p.y, p.y), qrr = pk(q.x, q.x), qii = pk(q.y, q.y); "
         "const float prl = p.x - lowf(prr), pil = p.y - lowf(pii), qrl = q.x - lowf(qrr), qil = q.y - lowf(qii); "
         "R0 = v4(pk(p.x, prl), pk(p.x, -p.y)); R1 = v4(pk(-pil, -p.y), pk(q.x, qrl)); "
         "R2 = v4(pk(q.x, -q.y), pk(-qil, -q.y)); "
         "I0 = v4(pk(p.y, pil), pk(p.y, p.x)); I1 = v4(pk(prl, p.x), pk(q.y, qil)); "
         "I2 = v4(pk(q.y, q.x), pk(qrl, q.x)); }\n";
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
  // one kernel per level; a block runs W wavefront tiles of one of its
  // steps (W = 4, or 8 when every step of the level can and one asks for it)
  std::vector<int> level_lds(n_levels, 0);  // LDS of the level's matrix-core steps
  for (int lev = 0; lev < n_levels; ++lev) {
    WideKernel k;
    k.kind = 0;
    k.name = "wl" + std::to_string(lev);
    k.blocks = 0;
    int all8 = 1, want8 = 0;
    for (int si = 0; si < wide.n_steps; ++si) {
      if (level[si] != lev) continue;
      const int32_t* sr = &wide.steps[8 * si];
      std::vector<const int32_t*> rec(sr[4]);
      for (int i = 0; i < sr[4]; ++i) rec[i] = &wide.ops[(size_t)(sr[6] + i) * kWideOpInts];
      const int wmask = step_waves(sr[0], sr[2], sr[3], prec, rec, mfma, tiles);
      all8 &= (wmask >> 1) & 1;
      want8 |= (wmask >> 2) & 1;
    }
    const int W = all8 && want8 ? 8 : 4;
    k.threads = 64 * W;
    // Two wavefronts per SIMD: caps a wavefront at 256 registers, which
    // also makes the compiler keep matrix-core accumulators in ordinary
    // VGPRs (with 512 it places them in AGPRs and copies them between
    // register sets inside the K loops).
    o << "extern \"C\" __global__ void __launch_bounds__(" << 64 * W << ") "
      << (mfma && prec != 0 ? "__attribute__((amdgpu_waves_per_eu(2))) " : "") << k.name
      << "(C2* __restrict__ mem, const C2* __restrict__ cst, const unsigned long long* __restrict__ packed, "
         "unsigned long long group_elems, unsigned long long s_begin, unsigned long long n_s, int group0, "
         "int ns_log2, unsigned long long n_items, unsigned long long n_bs, C2* __restrict__ res, "
         "C2* __restrict__ gres, unsigned long long vary) {\n"
      << "/*LDS" << lev << "*/\n"
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
      << "  (void)s; (void)xb; (void)res; (void)gres; (void)valid; (void)sl; (void)n_bs; (void)vary;\n"
      << "  C2* gm = mem + (unsigned long long)blockIdx.y * group_elems * 64ull;\n"
      << "  (void)gm;\n"
      << "  const unsigned long long blk = blockIdx.x;\n";
    for (int si = 0; si < wide.n_steps; ++si) {
      if (level[si] != lev) continue;
      const int32_t* sr = &wide.steps[8 * si];
      const int kind = sr[0], out = sr[1], r = sr[2], ns = sr[3], m = sr[4], slot = sr[5], ob = sr[6];
      std::vector<const int32_t*> rec(m);
      for (int i = 0; i < m; ++i) rec[i] = &wide.ops[(size_t)(ob + i) * kWideOpInts];
      // operands that carry no summed bit multiply each sum once
      std::vector<char> has_sum(m, 0);
      int m_in = 0;
      for (int i = 0; i < m; ++i) {
        for (int j = 0; j < ns; ++j) has_sum[i] |= rec[i][48 + j] != 0;
        m_in += has_sum[i];
      }
      const bool factor_out = ns >= 1 && m_in >= 1 && m_in < m;
      if (kind == ST_ELIM || kind == ST_FINAL) {
        const double sflops = step_flops(r, ns, factor_out ? m_in : m, factor_out ? m - m_in : 0);
        k.flops += sflops;
        // every operand and the output once, 8 B per element
        double elems = (double)(1ull << r);
        for (int i = 0; i < m; ++i) {
          int nv = 0;
          for (int j = 0; j < r; ++j) nv += rec[i][16 + j] != 0;
          for (int j = 0; j < ns; ++j) nv += rec[i][48 + j] != 0;
          elems += (double)(1ull << nv);
        }
        k.bytes += 8.0 * elems;
        k.step_flops.push_back(sflops);
        k.step_bytes.push_back(8.0 * elems);
        k.step_fix.push_back(wide.step_fix.empty() ? ~0ull : wide.step_fix[si]);
      }
      // Group sharing: a step whose values depend on none of the fixed
      // variables that differ between the groups of a pass (`vary`, set by
      // the host per pass) runs in group 0 only, and every group reads such
      // an operand from group 0's memory (the same offsets in every group).
      std::string pre;
      {
        char line[160];
        const uint64_t sf = wide.step_fix.empty() ? ~0ull : wide.step_fix[si];
        if (sf != ~0ull) {
          std::snprintf(line, sizeof(line), "  if ((0x%llxull & vary) == 0ull && blockIdx.y != 0u) return;\n",
                        (unsigned long long)sf);
          pre += line;
        }
        for (int i = 0; i < m; ++i) {
          if (rec[i][0] != WOP_ITEM) continue;
          const uint64_t of = wide.op_fix.empty() ? ~0ull : wide.op_fix[(size_t)ob + i];
          if (of == ~0ull)
            std::snprintf(line, sizeof(line), "  C2* const gq%d = gm;\n", i);
          else
            std::snprintf(line, sizeof(line), "  C2* const gq%d = (0x%llxull & vary) == 0ull ? mem : gm;\n", i,
                          (unsigned long long)of);
          pre += line;
        }
      }
      int lds_bytes = 0;
      if (mfma && emit_mfma_step(o, pre, k, si, kind, out, r, ns, prec, rec, lds_bytes, tiles, W)) {
        level_lds[lev] = std::max(level_lds[lev], lds_bytes);
        continue;
      }
      // Iteration order of the output bits: those that fewer item operands
      // depend on come first (inside the tile, then across neighbouring
      // wavefronts), so an operand row is reused within a tile or soon after
      // by the next tiles while it is still in cache; the bits every large
      // operand shares vary slowest.  perm[k] is the output bit at position k.
      std::vector<int> perm(r), weight(r, 0);
      std::vector<double> wbytes(r, 0.0);
      for (int j = 0; j < r; ++j) {
        perm[j] = j;
        for (int i = 0; i < m; ++i) weight[j] += rec[i][0] == WOP_ITEM && rec[i][16 + j] != 0;
      }
      {
        // A streaming step (at most 3 summed bits) whose largest item
        // operand is at least 8 times larger than every other: ties are
        // broken by the size of the operands a bit indexes, so the bits the
        // large operand does not carry vary first and its rows are reused
        // by the neighbouring tiles of one block instead of being fetched
        // again by tiles on other XCDs.  GEMM-shaped steps keep the plain
        // order (the size order made such complex128 steps up to 2.3x
        // slower).
        std::vector<double> sz;
        for (int i = 0; i < m; ++i) {
          if (rec[i][0] != WOP_ITEM) continue;
          int nv = 0;
          for (int j = 0; j < r; ++j) nv += rec[i][16 + j] != 0;
          for (int j = 0; j < ns; ++j) nv += rec[i][48 + j] != 0;
          sz.push_back(std::ldexp(1.0, nv));
        }
        std::sort(sz.rbegin(), sz.rend());
        if (ns <= 3 && sz.size() >= 2 && sz[0] >= 8 * sz[1])
          for (int i = 0; i < m; ++i) {
            if (rec[i][0] != WOP_ITEM) continue;
            int nv = 0;
            for (int j = 0; j < r; ++j) nv += rec[i][16 + j] != 0;
            for (int j = 0; j < ns; ++j) nv += rec[i][48 + j] != 0;
            for (int j = 0; j < r; ++j)
              if (rec[i][16 + j]) wbytes[j] += std::ldexp(1.0, nv);
          }
      }
      std::stable_sort(perm.begin(), perm.end(), [&](int x, int y) {
        return weight[x] != weight[y] ? weight[x] < weight[y] : wbytes[x] < wbytes[y];
      });
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
      const unsigned long long nb = (tiles + W - 1) / W;
      k.steps.push_back(si);
      o << "  if (blk >= " << k.blocks << "ull && blk < " << k.blocks + nb << "ull) {\n"
        << "  // step " << si << "\n"
        << pre
        << "  const unsigned long long t = (blk - " << k.blocks << "ull) * " << W << "ull + wv;\n";
      o << "  if (t >= " << tiles << "ull) return;\n";
      k.blocks += nb;
      // per-operand base offsets from the tile index
      for (int i = 0; i < m; ++i) {
        o << "  const long long o" << i << " = " << rec[i][1] << "ll";
        for (int k2 = L; k2 < r; ++k2)
          if (rec[i][16 + perm[k2]])
            o << " + (long long)((t >> " << (k2 - L) << ") & 1ull) * " << rec[i][16 + perm[k2]] << "ll";
        if (rec[i][0] == WOP_LEAF)
          for (int d = 0; d < rec[i][2]; ++d)
            o << " + (long long)(((" << (rec[i][3 + d] ? "s" : "xb") << " >> " << rec[i][7 + d] << ") & 1ull) * "
              << rec[i][11 + d] << "ll)";
        o << ";\n";
      }
      if (kind == ST_ELIM || kind == ST_FINAL) {
        // (FINAL: the element index of the amplitude among the item's 2^r)
        o << "  const long long ob = " << (kind == ST_ELIM ? out : 0) << "ll";
        for (int k2 = L; k2 < r; ++k2)
          o << " + (long long)((t >> " << (k2 - L) << ") & 1ull) * " << (1ll << perm[k2]) << "ll";
        o << ";\n";
      }
      // item operands first in every product; operands with no summed bit
      // (factor_out) multiply each sum after the loop
      std::vector<int> order, after;
      for (int i = 0; i < m; ++i)
        if (rec[i][0] == WOP_ITEM) (factor_out && !has_sum[i] ? after : order).push_back(i);
      for (int i = 0; i < m; ++i)
        if (rec[i][0] != WOP_ITEM) (factor_out && !has_sum[i] ? after : order).push_back(i);
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
      for (int i : order) {
        o << "    const long long p" << i << " = o" << i;
        for (int j = 0; j < ns; ++j)
          if (rec[i][48 + j]) o << " + (long long)((q >> " << j << ") & 1) * " << rec[i][48 + j] << "ll";
        o << ";\n";
      }
      // operand i's values at this tile's rows, from base p<i> (in the loop)
      // or o<i> (after it)
      auto load_rows = [&](int i, const std::string& ind, const std::string& base) {
        for (int e = 0; e < (1 << dep[i].size()); ++e) {
          long long off = 0;
          for (size_t d = 0; d < dep[i].size(); ++d)
            if ((e >> d) & 1) off += rec[i][16 + perm[dep[i][d]]];
          o << ind << "const C2 v" << i << "_" << e << " = ";
          if (rec[i][0] == WOP_ITEM)
            o << "gq" << i << "[(" << base << i << " + " << off << "ll) * 64ll + lane];\n";
          else
            o << "cst[" << base << i << " + " << off << "ll];\n";
        }
      };
      for (int i : order) load_rows(i, "    ", "p");
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
      for (int i : after) load_rows(i, "  ", "o");
      for (int lo = 0; lo < (1 << L) && !after.empty(); ++lo) {
        o << "  a" << lo << " = ";
        std::string cur = "a" + std::to_string(lo);
        for (int i : after) cur = "cm(" + cur + ", v" + std::to_string(i) + "_" + std::to_string(row_of(i, lo)) + ")";
        o << cur << ";\n";
      }
      for (int lo = 0; lo < (1 << L); ++lo) {
        if (kind == ST_ELIM) {
          long long lo_off = 0;
          for (int j = 0; j < L; ++j)
            if ((lo >> j) & 1) lo_off += 1ll << perm[j];
          o << "  gm[(ob + " << lo_off << "ll) * 64ll + lane] = a" << lo << ";\n";
        } else if (kind == ST_FINAL) {
          long long lo_off = 0;
          for (int j = 0; j < L; ++j)
            if ((lo >> j) & 1) lo_off += 1ll << perm[j];
          o << "  if (valid) res[((sl * n_bs + b) << " << r << ") + ob + " << lo_off << "ll] = a" << lo << ";\n";
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
  // the LDS ring of each level kernel with matrix-core steps
  std::string src = o.str();
  for (int lev = 0; lev < n_levels; ++lev) {
    const std::string mark = "/*LDS" + std::to_string(lev) + "*/";
    const size_t at = src.find(mark);
    if (at == std::string::npos) continue;
    src.replace(at, mark.size(),
                level_lds[lev] ? "  __shared__ __attribute__((aligned(16))) char lds[" + std::to_string(level_lds[lev]) + "];"
                               : std::string());
  }
  return src;
}

}  // namespace qgm
