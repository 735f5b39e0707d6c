// Batched complex GEMM on the CDNA4 matrix cores for the slice propagator.
//
// C_w = diag(rs) [alpha op(A_w) op(B_w) + beta C_w + cI I + c1 P1_w + c2 P2_w + c3 P3_w] diag(cs),
// with up to four extra outputs formed from the same product and the same P_w.  The
// epilogue builds the Paterson-Stockmeyer blocks of the Taylor series of e^V and applies
// the half-step kinetic factors of the symmetric Trotter propagator (eq. B) without
// extra passes over memory.  A single epilogue operand is prefetched during the last
// k-tile (tiles of at most 4 blocks per wave); 16 x 16 blocks outside the m x n result issue no
// MFMAs.
//
// Tiling: a BM x BN output tile per workgroup of (BM/WM) x (BN/WN) waves, each wave a WM x WN
// tile of 16 x 16 MFMA blocks; K staged through LDS BK at a time, double-buffered: the next
// k-tile's global loads are in flight during the current k-tile's MFMAs (for the FP32-MFMA
// propagator products every load is unconditional, so that none of them is waited for early).  Several
// tile shapes are built; the library times them on the real problem size at start-up and
// keeps the fastest per system and precision (see gemm_tile_count / the tile field).
// Complex products use four real MFMAs: re += a.re b.re - a.im b.im,
// im += a.re b.im + a.im b.re.  FP64 path: v_mfma_f64_16x16x4f64; mixed path:
// v_mfma_f32_16x16x4f32 with complex64 operands and FP32 accumulation.
// Matrices are [W][ld][ld] (or any lda/ldb/ldc) with zero padding beyond M;
// every load is bounds-guarded against M, every store against Mpad.
#include "common.h"
#include "kernels.h"
#include <type_traits>

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

namespace {

constexpr int PAD = 1;   // LDS row padding (complex elements)

template <int BM_, int BN_, int BK_, int WM_, int WN_> struct Tile {
  static constexpr int BM = BM_, BN = BN_, BK = BK_, WM = WM_, WN = WN_;
  static constexpr int WGM = BM / WM, WGN = BN / WN, NT = 64 * WGM * WGN;
  static constexpr int FM = WM / 16, FN = WN / 16;
  static constexpr int EA = BM * BK / NT, EB = BK * BN / NT;
  static_assert(EA * NT == BM * BK && EB * NT == BK * BN, "tile loads must split evenly");
};

template <typename ACC> struct Mfma;
template <> struct Mfma<double> {
  typedef d4v acc_t;
  static FT_DEV acc_t mma(double a, double b, acc_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  // output register v of lane l holds row 4v + l/16, column l%16 of the 16x16 block
  static FT_DEV int row(int lane, int v) { return 4 * v + (lane >> 4); }
};
template <> struct Mfma<float> {
  typedef f4v acc_t;
  static FT_DEV acc_t mma(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  // output register v of lane l holds row 4(l/16) + v, column l%16
  static FT_DEV int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

template <typename T> FT_DEV double2 ld_c(const T* p) { return to_d2(*p); }

// The 16-wave 64 x 64 propagator tile is held to 8 waves per SIMD (two workgroups per CU): in FP64
// that costs a few spilled registers and gains 7-10% (M = 171, 485); the dense linear algebra
// keeps its registers (a spilling update kernel was 24% slower).
template <typename TA, typename TB, typename TC, typename ACC, int ROLE, typename TL>
__global__ __launch_bounds__(TL::NT, (ROLE == 0 && TL::NT >= 1024 && TL::WM == 16 && TL::WN == 16) ? 8 : 1) void zgemm_kernel(GemmParams p) {
  typedef typename cplx_of<ACC>::type cacc;
  typedef typename Mfma<ACC>::acc_t acc_t;
  constexpr int BM = TL::BM, BN = TL::BN, BK = TL::BK, FM = TL::FM, FN = TL::FN, NT = TL::NT;
  // A is staged k-contiguous (As[m][k]: the coalesced loads store without a transpose), B as stored
  __shared__ cacc As[2][BM][BK + PAD];
  __shared__ cacc Bs[2][BK][BN + PAD];
  // the propagator products use A and B as stored; only the dense linear algebra takes A^H
  const int opA = ROLE == 1 ? p.opA : 0, opB = ROLE == 1 ? p.opB : 0;
  // unconditional tile and epilogue loads (below) for the FP32-MFMA propagator products
  constexpr bool UNCOND = ROLE == 0 && sizeof(ACC) == 4;

  int w, tile;
  if (!xcd_walker_tile(blockIdx.x, p.W, p.tiles_m * p.tiles_n, &w, &tile)) return;
  const int tm = tile / p.tiles_n, tn = tile - tm * p.tiles_n;
  const int m0 = tm * BM, n0 = tn * BN;
  // Hermitian result: the tiles above the diagonal are written by their mirror images
  constexpr bool SQUARE = BM == BN;
  const bool herm = ROLE == 1 && SQUARE && p.herm;
  if (herm && tn > tm) return;   // uniform over the workgroup, before any barrier
  // the wave index is scalar, so that the per-block tests below are scalar branches
  const int t = threadIdx.x, lane = t & 63, wid = __builtin_amdgcn_readfirstlane(t >> 6);
  const int wr = wid / TL::WGN, wc = wid % TL::WGN;
  const int Mr = p.m, Nc = p.n, Kd = p.k;

  const TA* A = (const TA*)p.A + (long long)w * p.sA;
  const TB* B = (const TB*)p.B + (long long)w * p.sB;

  acc_t accR[FM][FN], accI[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) { accR[i][j][v] = 0; accI[i][j][v] = 0; }

  // FP32-MFMA propagator products (A and B as stored): tile entries are kept as stored
  // (complex64, or complex128 converted at once).  Every load is unconditional, at a clamped address (an entry outside the matrix
  // reads its first element), so that all the loads of a k-tile are in flight together during
  // the MFMAs; the bounds select and the conversion to the MFMA type happen when the tile is
  // staged in LDS.  (A load behind a bounds branch was waited for at once: the k-tile's loads
  // ran one after another before the MFMAs.)
  // Operands stored wider than the MFMA type (the complex128 Y of the mixed apply) would hold
  // twice the registers across the MFMAs; those are converted right after their loads instead
  // (all of the tile's loads are issued first, so they still wait only once).
  typedef typename std::conditional<sizeof(TA) == sizeof(cacc), TA, cacc>::type RA;
  typedef typename std::conditional<sizeof(TB) == sizeof(cacc), TB, cacc>::type RB;
  RA ra[TL::EA];
  RB rb[TL::EB];
  bool oka[TL::EA], okb[TL::EB];
  auto load_tile = [&](int kt) {
    const int k0 = kt * BK;
    TA ta[TL::EA];
    TB tb[TL::EB];
#pragma unroll
    for (int q = 0; q < TL::EA; ++q) {
      const int e = t + q * NT;
      int gm, gk;
      if (opA == 0) { gm = m0 + e / BK; gk = k0 + e % BK; }
      else            { gk = k0 + e / BM; gm = m0 + e % BM; }
      oka[q] = gm < Mr && gk < Kd;
      const long long off = opA == 0 ? (long long)gm * p.lda + gk : (long long)gk * p.lda + gm;
      ta[q] = A[oka[q] ? off : 0];
    }
#pragma unroll
    for (int q = 0; q < TL::EB; ++q) {
      const int e = t + q * NT;
      int gk, gn;
      if (opB == 0) { gk = k0 + e / BN; gn = n0 + e % BN; }
      else            { gn = n0 + e / BK; gk = k0 + e % BK; }
      okb[q] = gn < Nc && gk < Kd;
      const long long off = opB == 0 ? (long long)gk * p.ldb + gn : (long long)gn * p.ldb + gk;
      tb[q] = B[okb[q] ? off : 0];
    }
#pragma unroll
    for (int q = 0; q < TL::EA; ++q) {
      if constexpr (sizeof(TA) == sizeof(cacc)) ra[q] = ta[q];
      else ra[q] = cvt<ACC>(ta[q]);
    }
#pragma unroll
    for (int q = 0; q < TL::EB; ++q) {
      if constexpr (sizeof(TB) == sizeof(cacc)) rb[q] = tb[q];
      else rb[q] = cvt<ACC>(tb[q]);
    }
  };
  // The FP64 tiles (the FP64 propagator and the dense linear algebra) load behind the bounds
  // test, converting and conjugating at the load: there the unconditional form above was 3-7%
  // slower (FP64 update tile 90.6 -> 93.4 us, FP64 propagator tile 226 -> 241 us at M=171).
  auto load_tile_la = [&](int kt) {
    const int k0 = kt * BK;
#pragma unroll
    for (int q = 0; q < TL::EA; ++q) {
      const int e = t + q * NT;
      int gm, gk;
      if (opA == 0) { gm = m0 + e / BK; gk = k0 + e % BK; }
      else            { gk = k0 + e / BM; gm = m0 + e % BM; }
      double2 v = make_double2(0.0, 0.0);
      if (gm < Mr && gk < Kd)
        v = opA == 0 ? ld_c(A + (long long)gm * p.lda + gk) : cconj(ld_c(A + (long long)gk * p.lda + gm));
      ra[q] = cvt<ACC>(v);
      oka[q] = true;
    }
#pragma unroll
    for (int q = 0; q < TL::EB; ++q) {
      const int e = t + q * NT;
      int gk, gn;
      if (opB == 0) { gk = k0 + e / BN; gn = n0 + e % BN; }
      else            { gn = n0 + e / BK; gk = k0 + e % BK; }
      double2 v = make_double2(0.0, 0.0);
      if (gn < Nc && gk < Kd)
        v = opB == 0 ? ld_c(B + (long long)gk * p.ldb + gn) : cconj(ld_c(B + (long long)gn * p.ldb + gk));
      rb[q] = cvt<ACC>(v);
      okb[q] = true;
    }
  };
  auto staged = [&](auto raw, bool ok) {
    cacc v = cvt<ACC>(raw);
    if (!ok) { v.x = 0; v.y = 0; }
    return v;
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int q = 0; q < TL::EA; ++q) {
      const int e = t + q * NT;
      const cacc v = staged(ra[q], oka[q]);
      if (opA == 0) As[buf][e / BK][e % BK] = v;
      else          As[buf][e % BM][e / BM] = v;
    }
#pragma unroll
    for (int q = 0; q < TL::EB; ++q) {
      const int e = t + q * NT;
      const cacc v = staged(rb[q], okb[q]);
      if (opB == 0) Bs[buf][e / BN][e % BN] = v;
      else          Bs[buf][e % BK][e / BK] = v;
    }
  };

  const int nk = (Kd + BK - 1) / BK;
  TC* C = (TC*)p.C + (long long)w * p.sC;
  const TC* P1 = p.P1 ? (const TC*)p.P1 + (long long)w * p.sP : nullptr;
  const TC* P2 = p.P2 ? (const TC*)p.P2 + (long long)w * p.sP : nullptr;
  const TC* P3 = p.P3 ? (const TC*)p.P3 + (long long)w * p.sP : nullptr;
  // One epilogue operand (P1 alone, or C when beta != 0) is loaded during the last k-tile
  // so that its latency overlaps the MFMAs.
  // (tiles of more than 4 blocks per wave keep no prefetched operand: it would not fit in registers)
  constexpr bool PREF = FM * FN <= 4;
  const bool pre_p1 = PREF && P1 && !P2 && !P3 && p.beta == 0.0;
  const bool pre_c = PREF && !P1 && p.beta != 0.0;
  const TC* PRE = pre_p1 ? P1 : (pre_c ? (const TC*)C : nullptr);
  const int pre_ld = pre_p1 ? p.ldp : p.ldc;
  TC pre[PREF ? FM : 1][PREF ? FN : 1][4];   // kept in the output precision (complex64 in the mixed path)
  const int li = lane & 15, lk = lane >> 4;
  // 16 x 16 blocks entirely outside the m x n result are skipped (uniform per wave)
  bool live[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) live[i][j] = (m0 + wr * TL::WM + i * 16 < Mr) && (n0 + wc * TL::WN + j * 16 < Nc);

  auto load = [&](int kt) {
    if constexpr (UNCOND) load_tile(kt);
    else load_tile_la(kt);
  };
  // upper-triangular A: the k-tiles left of this row tile hold only zeros of A
  const int kt0 = (ROLE == 1 && p.tri_a) ? (m0 / BK < nk ? m0 / BK : nk) : 0;
  if (kt0 < nk) {
    load(kt0);
    store_tile(kt0 & 1);
  }
  __syncthreads();
  for (int kt = kt0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load(kt + 1);
    if (kt + 1 == nk && PRE) {
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int gi = m0 + wr * TL::WM + i * 16 + Mfma<ACC>::row(lane, v);
            const int gj = n0 + wc * TL::WN + j * 16 + li;
            if constexpr (PREF) pre[i][j][v] = (gi < Mr && gj < Nc) ? PRE[(long long)gi * pre_ld + gj] : TC{};
          }
    }
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      cacc a[FM], b[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) a[i] = As[buf][wr * TL::WM + i * 16 + li][ks + lk];
#pragma unroll
      for (int j = 0; j < FN; ++j) b[j] = Bs[buf][ks + lk][wc * TL::WN + j * 16 + li];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        const ACC nai = -a[i].y;
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          if (!live[i][j]) continue;
          accR[i][j] = Mfma<ACC>::mma(a[i].x, b[j].x, accR[i][j]);
          accR[i][j] = Mfma<ACC>::mma(nai, b[j].y, accR[i][j]);
          accI[i][j] = Mfma<ACC>::mma(a[i].x, b[j].y, accI[i][j]);
          accI[i][j] = Mfma<ACC>::mma(a[i].y, b[j].x, accI[i][j]);
        }
      }
    }
    if (kt + 1 < nk) store_tile(buf ^ 1);
    __syncthreads();
  }

  if constexpr (UNCOND) {
    // epilogue: the operand loads of EV entries (the addends, C when beta != 0, the row and
    // column factors) are issued together, unconditionally at a clamped address for entries
    // outside the result, before any of them is used.  Two entries for the 192 x 192 tile (its
    // spill shrank from 36 to 12 bytes), one for the others: four made the register-capped
    // tiles spill inside the k-loop.
    constexpr int EV = TL::BM == 192 ? 2 : 1;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int v0 = 0; v0 < 4; v0 += EV) {
          const int gj = n0 + wc * TL::WN + j * 16 + li;
          int gi[EV];
          bool in[EV];
          TC q1r[EV], q2r[EV], q3r[EV], qcr[EV];
          double rsv[EV], csv = 1.0;
#pragma unroll
          for (int u = 0; u < EV; ++u) {
            gi[u] = m0 + wr * TL::WM + i * 16 + Mfma<ACC>::row(lane, v0 + u);
            in[u] = gi[u] < Mr && gj < Nc;
            const long long offp = in[u] ? (long long)gi[u] * p.ldp + gj : 0;
            const long long off = in[u] ? (long long)gi[u] * p.ldc + gj : 0;
            q1r[u] = q2r[u] = q3r[u] = qcr[u] = TC{};
            rsv[u] = 1.0;
            if (P1 && !pre_p1) q1r[u] = P1[offp];
            if (P2) q2r[u] = P2[offp];
            if (P3) q3r[u] = P3[offp];
            if (!pre_c && p.beta != 0.0) qcr[u] = C[off];
            if (p.rs) rsv[u] = p.rs[in[u] ? gi[u] : 0];
          }
          if (p.cs) csv = p.cs[gj < Nc ? gj : 0];
#pragma unroll
          for (int u = 0; u < EV; ++u) {
            const int v = v0 + u;
            if (gi[u] >= p.mpad || gj >= p.npad) continue;
            if (ROLE == 1 && gi[u] >= p.skip0 && gi[u] < p.skip1) continue;   // rows left untouched
            const long long off = (long long)gi[u] * p.ldc + gj;
            const double2 acc = make_double2((double)accR[i][j][v], (double)accI[i][j][v]);
            double2 q1 = to_d2(q1r[u]), q2 = to_d2(q2r[u]), q3 = to_d2(q3r[u]), qc = to_d2(qcr[u]);
            if constexpr (PREF) {
              if (pre_p1) q1 = to_d2(pre[i][j][v]);
              if (pre_c) qc = to_d2(pre[i][j][v]);
            }
            const double di = (gi[u] == gj) ? 1.0 : 0.0;
            double2 out = make_double2(0.0, 0.0);
            if (in[u]) {
              out = cscale(acc, p.alpha);
              if (p.beta != 0.0) out = cadd(out, cscale(qc, p.beta));
              out.x += p.cI * di;
              out = cadd(out, cadd(cscale(q1, p.c1), cadd(cscale(q2, p.c2), cscale(q3, p.c3))));
              if (p.rs) out = cscale(out, rsv[u]);
              if (p.cs) out = cscale(out, csv);
            }
            store_c(C + off, out);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              if (e >= p.nextra) break;
              const GemmOut& o = p.extra[e];
              double2 x = make_double2(0.0, 0.0);
              if (in[u]) {
                x = cscale(acc, o.cacc);
                x.x += o.cI * di;
                x = cadd(x, cadd(cscale(q1, o.c1), cadd(cscale(q2, o.c2), cscale(q3, o.c3))));
              }
              store_c((TC*)o.ptr + (long long)w * p.sC + off, x);
            }
          }
        }
  } else {
    // the FP64 tiles keep the plain per-entry epilogue
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int gi = m0 + wr * TL::WM + i * 16 + Mfma<ACC>::row(lane, v);
          const int gj = n0 + wc * TL::WN + j * 16 + li;
          if (gi >= p.mpad || gj >= p.npad) continue;
          if (ROLE == 1 && gi >= p.skip0 && gi < p.skip1) continue;   // rows left untouched
          const long long off = (long long)gi * p.ldc + gj;
          const bool in = gi < Mr && gj < Nc;
          const double2 acc = make_double2((double)accR[i][j][v], (double)accI[i][j][v]);
          double2 q1 = make_double2(0.0, 0.0), q2 = q1, q3 = q1, qc = q1;
          if (in) {
            const long long offp = (long long)gi * p.ldp + gj;
            if (pre_p1) { if constexpr (PREF) q1 = to_d2(pre[i][j][v]); }
            else if (P1) q1 = ld_c(P1 + offp);
            if (P2) q2 = ld_c(P2 + offp);
            if (P3) q3 = ld_c(P3 + offp);
            if (pre_c) { if constexpr (PREF) qc = to_d2(pre[i][j][v]); }
            else if (p.beta != 0.0) qc = ld_c(C + off);
          }
          const double di = (gi == gj) ? 1.0 : 0.0;
          double2 out = make_double2(0.0, 0.0);
          if (in) {
            out = cscale(acc, p.alpha);
            if (p.beta != 0.0) out = cadd(out, cscale(qc, p.beta));
            out.x += p.cI * di;
            out = cadd(out, cadd(cscale(q1, p.c1), cadd(cscale(q2, p.c2), cscale(q3, p.c3))));
            if (p.rs) out = cscale(out, p.rs[gi]);
            if (p.cs) out = cscale(out, p.cs[gj]);
          }
          store_c(C + off, out);
          if (herm && tn < tm && gj < p.mpad && gi < p.npad) store_c(C + (long long)gj * p.ldc + gi, cconj(out));
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            if (e >= p.nextra) break;
            const GemmOut& o = p.extra[e];
            double2 x = make_double2(0.0, 0.0);
            if (in) {
              x = cscale(acc, o.cacc);
              x.x += o.cI * di;
              x = cadd(x, cadd(cscale(q1, o.c1), cadd(cscale(q2, o.c2), cscale(q3, o.c3))));
            }
            store_c((TC*)o.ptr + (long long)w * p.sC + off, x);
          }
        }
  }
}

typedef Tile<64, 64, 16, 32, 32> T64x64;     // 4 waves of 32 x 32
typedef Tile<64, 128, 16, 32, 64> T64x128;   // 4 waves of 32 x 64
typedef Tile<128, 64, 16, 64, 32> T128x64;   // 4 waves of 64 x 32
typedef Tile<32, 64, 16, 16, 32> T32x64;     // 4 waves of 16 x 32
typedef Tile<32, 32, 16, 16, 16> T32x32;     // 4 waves of 16 x 16
// 16 waves of small per-wave tiles: few registers per wave (high occupancy) while the
// 64-row / 64- or 128-column workgroup tile still shares every LDS-staged operand.
typedef Tile<64, 64, 16, 16, 16> T64x64w16;
typedef Tile<64, 128, 16, 16, 32> T64x128w16;
// dense linear algebra with at most 32 result rows (the pivot-block products): 8 waves
typedef Tile<32, 64, 16, 16, 16> T32x64w8;
// 8 waves of 16 x 32: fewer workgroup barriers per MFMA (the FP64 products at M ~ 170 prefer it)
typedef Tile<64, 64, 16, 16, 32> T64x64w8;
// One walker's whole product at M <= 192 (complex64 only: 101 KB of LDS, 128 VGPRs): 16 waves of
// 48 x 48 (3 x 3 blocks), nine times the MFMAs per k-tile barrier of the 64 x 64 tile, one
// workgroup per walker and CU; the 16 x 16 blocks beyond M issue no MFMAs.
typedef Tile<192, 192, 16, 48, 48> T192w16;

template <typename TA, typename TB, typename TC, typename ACC, int ROLE, typename TL>
hipError_t launch_tile(GemmParams p, hipStream_t s) {
  p.tiles_m = (p.mpad + TL::BM - 1) / TL::BM;
  p.tiles_n = (p.npad + TL::BN - 1) / TL::BN;
  const int blocks = ((p.W + 7) / 8) * 8 * p.tiles_m * p.tiles_n;
  if (blocks == 0) return hipSuccess;
  zgemm_kernel<TA, TB, TC, ACC, ROLE, TL><<<blocks, TL::NT, 0, s>>>(p);
  return hipGetLastError();
}

template <typename TA, typename TB, typename TC, typename ACC, int ROLE>
hipError_t launch_shape(const GemmParams& p, hipStream_t s) {
  switch (p.tile) {
    case 0: return launch_tile<TA, TB, TC, ACC, ROLE, T64x64>(p, s);
    case 1: return launch_tile<TA, TB, TC, ACC, ROLE, T64x128>(p, s);
    case 2: return launch_tile<TA, TB, TC, ACC, ROLE, T128x64>(p, s);
    case 3: return launch_tile<TA, TB, TC, ACC, ROLE, T32x64>(p, s);
    case 4: return launch_tile<TA, TB, TC, ACC, ROLE, T32x32>(p, s);
    case 5: return launch_tile<TA, TB, TC, ACC, ROLE, T64x64w16>(p, s);
    case 6: return launch_tile<TA, TB, TC, ACC, ROLE, T64x128w16>(p, s);
    case 7: return launch_tile<TA, TB, TC, ACC, ROLE, T64x64w8>(p, s);
    case 8:
      if constexpr (sizeof(ACC) == 4) return launch_tile<TA, TB, TC, ACC, ROLE, T192w16>(p, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int gemm_tile_count() { return 9; }
bool gemm_tile_walker_sized(int tile) { return tile == 8; }
bool gemm_tile_supported(int tile, int prec) {
  if (tile < 0 || tile >= gemm_tile_count()) return false;
  return tile != 8 || prec == GEMM_C32 || prec == GEMM_C32_Z64B;   // the 192 x 192 tile: FP32 MFMA only
}

hipError_t launch_zgemm(const GemmParams& p, int prec, hipStream_t s) {
  if (p.m <= 0 || p.n <= 0) return hipSuccess;
  if (p.mpad < p.m || p.npad < p.n) return hipErrorInvalidValue;
  switch (prec * 2 + (p.role ? 1 : 0)) {
    case 2 * GEMM_Z64:       // complex128 in and out, FP64 MFMA (propagator chain)
      return launch_shape<double2, double2, double2, double, 0>(p, s);
    case 2 * GEMM_Z64 + 1:   // the same for the dense linear algebra (64 x 64 tiles, 16 waves)
      if (p.mpad <= 32) return launch_tile<double2, double2, double2, double, 1, T32x64w8>(p, s);
      return launch_tile<double2, double2, double2, double, 1, T64x64w16>(p, s);
    case 2 * GEMM_C32:       // complex64 in and out, FP32 MFMA
      return launch_shape<float2, float2, float2, float, 0>(p, s);
    case 2 * GEMM_C32_Z64B:  // complex64 A, complex128 B (rounded to complex64), complex128 out
      return launch_shape<float2, double2, double2, float, 0>(p, s);
    default: return hipErrorInvalidValue;
  }
}
