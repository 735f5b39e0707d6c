// Blocked Gaussian elimination on per-walker augmented matrices [A | R], batched over walkers.
//
// Used for three solves of the slice path:
//   * the Green's function (eq. green) in scale-split form: A = X^T, R = (Ti D_b)^T with
//     partial pivoting, by blocked Gauss-Jordan, so R becomes X^{-T} (Ti D_b)^T;
//   * the Cholesky factor of S = Y^H Y in the QR stabilisation: no pivoting, forward
//     only; the left block becomes U = D L^H (S = L D L^H) and R becomes L^{-1} R;
//   * the update of T^{-1} by a unit triangular factor (again forward only).
// NB = 32 columns per panel (64 for the Gauss-Jordan steps where at most 256 rows are left),
// one kernel sequence for all walkers:
//   panel   one workgroup per walker.  Forward elimination: one row per thread, LU of the panel
//           with LDS broadcasts of the pivot row, then L11^{-1}.  Gauss-Jordan: in-place
//           Gauss-Jordan inversion of the pivot block inside the column loop, either with one
//           row per thread (the row rotated in registers so the runtime column loop stays
//           small) or, by default, column-split: each wave owns 8 columns of every row, the
//           owning wave searches a column's pivot alone and passes the multipliers through
//           LDS (row exchange = relabelling in both);
//   swap    the panel's row exchanges composed into one permutation of at most 2 x the panel
//           width rows;
// Forward elimination (LU, right-looking):
//   trsm    U12 = L11^{-1} A12 as a small in-place MFMA GEMM (each workgroup owns whole
//           columns and reads them completely before it writes);
//   update  A22 -= L21 U12 as a batched MFMA GEMM over the contiguous column range
//           [j0+NB, rhs_off+nrhs) (the zero padding between the two blocks stays zero).
//   Above 256 rows two panels make one step with K = 64 (the combined inverse of the 64-column
//   unit lower block from the combine kernel); with a lower-triangular left block (the T^{-1}
//   update) the products cover the right-hand block only.
// Gauss-Jordan (the solve with right-hand sides): the panel kernel leaves the panel columns
// untouched and returns A11^{-1} of the pivot block; the row exchanges run
// over the panel columns too, the pivot rows become P = A11^{-1} [A12 | R1] in place, and every
// other row, above and below, takes row_i -= A_i1 P.  After the last panel the right-hand block
// holds the solution in natural order: row exchanges only reorder equations.
// ln det of the left block is the sum of the logs of the pivots plus i pi per row exchange.
#include "common.h"
#include "kernels.h"
#include <climits>
#include <cstdlib>
#include <cstring>

namespace {

constexpr int NB = 32;

struct PanelParams {
  double2* aug; long long stride; int lda;
  int M, j0, jb, W, pivot;
  int gj;         // Gauss-Jordan: keep the panel columns, return A11^{-1} instead of L11^{-1}
  int* piv; int ld;
  double2* lndet; int* status;
  double2* tri;   // [W][tri_stride]: NB x NB L11^{-1} (forward) or A11^{-1} (Gauss-Jordan) at tri
  long long tri_stride;
};

// Per-walker pivot-block workspace (complex entries from the walker's start): the inverses of
// the two 32-column sub-panels of a 64-column Gauss-Jordan step, then the combined operator.
constexpr long long TRI_T1 = 0, TRI_T2 = NB * NB, TRI_TL = 2 * NB * NB;
constexpr long long TRI_ELEMS = 2 * NB * NB + 4 * NB * NB;
constexpr int GJ_WIDE_MIN_M = 256;      // 64-column Gauss-Jordan steps above this order (measured)

// The order above which the solve takes 64-column steps; FTAFQMC_GJ_WIDE_MIN_M=<order> in the
// environment overrides it (for experiments; read at every solve).
int gj_wide_min_m() {
  const char* env = std::getenv("FTAFQMC_GJ_WIDE_MIN_M");
  return env ? std::atoi(env) : GJ_WIDE_MIN_M;
}

template <int NT>
struct PanelShared {
  double2 curRow[2][NB];            // row `col`, double-buffered by column parity
  double2 pivv[NB];                 // pivots of this panel
  double2 Ls[NB][NB + 1];           // unit lower L11
};

// DPP move of a double within 16-lane rows (CTRL is a row-local pattern, every source exists).
template <int CTRL> FT_DEV double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

struct PanelCtx {
  int t, myrow, M, j0, jb;
};

// Column C of the forward (unpivoted) panel, compile-time so that every register index is
// static.  One barrier per column: the owner of row col publishes it.
template <int NT, int C>
FT_DEV void panel_column(double2 (&a)[NB], PanelCtx& x, PanelShared<NT>& sh) {
  if (C >= x.jb) return;                 // uniform over the workgroup
  const int col = x.j0 + C, buf = C & 1;
  if (x.myrow == col) {
#pragma unroll
    for (int i = C; i < NB; ++i) sh.curRow[buf][i] = a[i];
  }
  __syncthreads();
  const double2* pr = sh.curRow[buf];
  const double2 pv = pr[C];
  if (x.t == 0) sh.pivv[C] = pv;
  if (x.myrow > col && x.myrow < x.M) {
    const double2 l = cdiv(a[C], pv);
    a[C] = l;
#pragma unroll
    for (int i = C + 1; i < NB; ++i) a[i] = cfnms(a[i], l, pr[i]);
  }
}

template <int NT, int C> struct PanelColumns {
  static FT_DEV void run(double2 (&a)[NB], PanelCtx& x, PanelShared<NT>& sh) {
    panel_column<NT, C>(a, x, sh);
    PanelColumns<NT, C + 1>::run(a, x, sh);
  }
};
template <int NT> struct PanelColumns<NT, NB> {
  static FT_DEV void run(double2 (&)[NB], PanelCtx&, PanelShared<NT>&) {}
};

// Forward elimination: one workgroup per walker factors rows [j0, M) x columns [j0, j0+jb)
// without pivoting, one row per thread, writes L21 and U11 back and L11^{-1} to tri (one
// column of the inverse per thread).
template <int NT>
__global__ __launch_bounds__(NT) void panel_kernel(PanelParams p) {
  __shared__ PanelShared<NT> sh;
  const int w = blockIdx.x;
  if (w >= p.W) return;
  double2* aug = p.aug + (long long)w * p.stride;
  const int t = threadIdx.x;
  const int M = p.M, j0 = p.j0, jb = p.jb, lda = p.lda;
  const int r = j0 + t;                    // the row this thread holds (M - j0 <= NT)
  double2 a[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) a[c] = (r < M && c < jb) ? aug[(long long)r * lda + j0 + c] : make_double2(0.0, 0.0);
  PanelCtx x;
  x.t = t; x.myrow = r; x.M = M; x.j0 = j0; x.jb = jb;
  PanelColumns<NT, 0>::run(a, x, sh);
  if (r < M) {
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < jb) aug[(long long)r * lda + j0 + c] = a[c];
  }
  // rows j0..j0+jb hold L11 in their strictly lower part; rows beyond jb are the identity
  if (r >= j0 && r < j0 + NB) {
    const int i = r - j0;
#pragma unroll
    for (int c = 0; c < NB; ++c) sh.Ls[i][c] = (c < i && i < jb) ? a[c] : make_double2(0.0, 0.0);
  }
  for (int i = jb + t; i < NB; i += NT)
    for (int c = 0; c < NB; ++c) sh.Ls[i][c] = make_double2(0.0, 0.0);
  __syncthreads();
  // ln det contribution and pivot checks (wave 0 holds all jb <= 32 pivots)
  double lx = 0.0, ly = 0.0, badv = 0.0;
  if (t < jb) {
    const double2 pv = sh.pivv[t];
    const double2 lg = clog(pv);
    lx = lg.x;
    ly = lg.y;
    if (!(cabs2(pv) > 0.0) || !isfinite(pv.x) || !isfinite(pv.y)) badv = 1.0;
  }
  if (t < 64) {
    lx = wave_sum(lx); ly = wave_sum(ly); badv = wave_sum(badv);
  }
  // column t of L11^{-1} by forward substitution on e_t
  double2* tri = p.tri + (long long)w * p.tri_stride;
  if (t < NB) {
    double2 xcol[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      double2 v = make_double2(i == t ? 1.0 : 0.0, 0.0);
#pragma unroll
      for (int k = 0; k < i; ++k) v = cfnms(v, sh.Ls[i][k], xcol[k]);
      xcol[i] = v;
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) tri[i * NB + t] = xcol[i];
  }
  if (t == 0) {
    if (p.lndet) {
      double2 acc = j0 == 0 ? make_double2(0.0, 0.0) : p.lndet[w];
      acc.x += lx;
      acc.y += ly;
      p.lndet[w] = acc;
    }
    if (badv > 0.0 && p.status) p.status[w] = 2;
  }
}

// ---------------------------------------------------------------------------------------
// Gauss-Jordan panel: the pivot block's inverse by in-place elimination inside the column loop.
//
// One thread per row holds the row's NB panel entries in registers.  Column C (a runtime
// loop, so the loop body stays in the instruction cache) picks the pivot p among the rows not
// yet chosen, then every other row r takes
//     g = a_r[C] / a_p[C],   a_r[i] -= g a_p[i]  (i != C),   a_r[C] = -g,
// and the pivot row keeps its entries except a_p[C] = 1.  This is Gauss-Jordan on
// [A11 | I] stored in place with the pivot rows left unnormalised: after the last column the
// row chosen for column c holds pv_c times row c of A11^{-1} (A11 = the chosen rows in the
// order chosen, pv_c its pivot), so one division per row finishes the inverse.  Rows never
// chosen carry the same updates and are discarded.  The pivots equal those of LU with the
// same partial pivoting.

// Maximum of an int over the wave, uniform: row maxima by DPP, then the four rows by readlane.
template <int CTRL> FT_DEV int dpp_i(int v) { return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xF, 0xF, false); }
FT_DEV int wave_max_int(int v) {
  v = max(v, dpp_i<0xB1>(v));     // quad_perm [1,0,3,2]
  v = max(v, dpp_i<0x4E>(v));     // quad_perm [2,3,0,1]
  v = max(v, dpp_i<0x124>(v));    // row_ror:4
  v = max(v, dpp_i<0x128>(v));    // row_ror:8
  const int r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
  const int r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
  return max(max(r0, r1), max(r2, r3));
}

// 1 / b = conj(b) / |b|^2 with b scaled by a power of two (|b|^2 stays in range) and the
// hardware reciprocal estimate refined by two Newton steps (quadratic convergence: full double
// precision).  Zero or non-finite b gives NaN or Inf entries.
FT_DEV double2 crecip_newton(double2 b) {
  int e;
  (void)frexp(fmax(fabs(b.x), fabs(b.y)), &e);
  const double xs = ldexp(b.x, -e), ys = ldexp(b.y, -e);
  const double d = xs * xs + ys * ys;
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  r = fma(r, fma(-d, r, 1.0), r);
  return make_double2(ldexp(xs * r, -e), ldexp(-ys * r, -e));
}

constexpr int GJ_CH = 8;              // panel columns staged through LDS per step of the load

template <int NT>
struct GjShared {
  double2 stage[NT][GJ_CH];         // coalesced load of the panel
  double2 candRow[2][NT / 64][NB];  // each wave's best row, double-buffered by column parity
  int candKey[2][NT / 64];
  int candIdx[2][NT / 64];
  double2 pivv[NB];                 // pivots of this panel
  int swapped[NB];
};

// 1 / b by Smith's scaling (two real divisions), for the one pivot of a column.
FT_DEV double2 crecip(double2 b) {
  if (fabs(b.x) >= fabs(b.y)) {
    const double r = b.y / b.x, s = 1.0 / (b.x + b.y * r);
    return make_double2(s, -r * s);
  } else {
    const double r = b.x / b.y, s = 1.0 / (b.y + b.x * r);
    return make_double2(r * s, -s);
  }
}

// One workgroup per walker: rows [j0, M) x panel columns [j0, j0+jb).  Writes the pivot rows
// (piv), A11^{-1} (tri, [NB][NB], the leading jb x jb used), ln det and the status; the panel
// columns in memory are left as they are.
template <int NT>
__global__ __launch_bounds__(NT) void panel_gj_kernel(PanelParams p) {
  __shared__ GjShared<NT> sh;
  const int w = blockIdx.x;
  if (w >= p.W) return;
  double2* aug = p.aug + (long long)w * p.stride;
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const int M = p.M, j0 = p.j0, jb = p.jb, lda = p.lda;
  const int r = j0 + t;                    // M - j0 <= NT
  // a[k] holds panel column (C + k) mod NB while column C is processed: the row rotates by one
  // entry per column, so every register index is static; after NB steps it is back in order.
  double2 a[NB];
  {
    // the panel goes through LDS GJ_CH columns at a time: consecutive lanes read consecutive
    // entries of a row (coalesced), then every thread takes its own row from LDS
    // (every load is unconditional, so that all GJ_CH of them are in flight at once: entries
    // outside the panel read the pivot block's corner, which always exists, and become zero;
    // the next chunk's loads are issued before this chunk goes through LDS)
    const int rows = M - j0;
    double2 v[2][GJ_CH];
    auto load = [&](int q, double2 (&dst)[GJ_CH]) {
#pragma unroll
      for (int e0 = 0; e0 < GJ_CH; ++e0) {
        const int e = t + e0 * NT, rr = e / GJ_CH, c = q * GJ_CH + e % GJ_CH;
        const bool in = rr < rows && c < jb;
        dst[e0] = aug[(long long)(j0 + (in ? rr : 0)) * lda + j0 + (in ? c : 0)];
        if (!in) dst[e0] = make_double2(0.0, 0.0);
      }
    };
    load(0, v[0]);
#pragma unroll
    for (int q = 0; q < NB / GJ_CH; ++q) {
      if (q + 1 < NB / GJ_CH) load(q + 1, v[(q + 1) & 1]);
#pragma unroll
      for (int e0 = 0; e0 < GJ_CH; ++e0) {
        const int e = t + e0 * NT;
        sh.stage[e / GJ_CH][e % GJ_CH] = v[q & 1][e0];
      }
      __syncthreads();
#pragma unroll
      for (int c = 0; c < GJ_CH; ++c) a[q * GJ_CH + c] = sh.stage[t][c];
      __syncthreads();
    }
  }
  int* piv = p.piv + (long long)w * p.ld;
  int myrow = r;
  bool chosen = false;
  double2 mypv = make_double2(1.0, 0.0);
  // one column: a[0] is column C on entry; the row rotates by one entry on exit
  auto column = [&](int C) {
    const int col = j0 + C, buf = C & 1;
    const double2 f = a[0];
    const bool cand = myrow >= col && myrow < M;
    // search key: the high word of |a|^2 (orders non-negative doubles; candidates equal in their
    // leading 20 mantissa bits count as ties); -1 for non-candidates and NaN entries
    const double bv = cabs2(f);
    const int key = (cand && bv == bv) ? __double2hiint(bv) : -1;
    const int mk = wave_max_int(key);
    const unsigned long long hit = __ballot(cand && key == mk && mk >= 0);
    if (hit) {
      const int lead = __ffsll((long long)hit) - 1;   // lowest lane among the maxima
      if (lane == lead) {
#pragma unroll
        for (int i = 0; i < NB; ++i) sh.candRow[buf][wid][i] = a[i];
        sh.candKey[buf][wid] = mk;
        sh.candIdx[buf][wid] = myrow;
      }
    } else if (lane == 0) {
      sh.candKey[buf][wid] = -1;
      sh.candIdx[buf][wid] = INT_MAX;
    }
    __syncthreads();
    int bk = sh.candKey[buf][0], bi = sh.candIdx[buf][0], win = 0;
#pragma unroll
    for (int k = 1; k < NT / 64; ++k) {
      const int v = sh.candKey[buf][k], ix = sh.candIdx[buf][k];
      const bool better = v > bk || (v == bk && ix < bi);
      bk = better ? v : bk;
      bi = better ? ix : bi;
      win = better ? k : win;
    }
    // no usable pivot (every candidate NaN): the walker is marked failed and the column keeps
    // its row, so that the row exchanges stay a valid permutation; nothing is updated
    const bool ok = bk >= 0;
    const double2* pr = sh.candRow[buf][win];
    const int prow = ok ? bi : col;
    const double2 pv = ok ? pr[0] : make_double2(NAN, NAN);
    if (t == 0) {
      piv[col] = prow;
      sh.pivv[C] = pv;
      sh.swapped[C] = prow != col;
    }
    const bool ispiv = ok && myrow == prow;
    if (ispiv) { myrow = col; chosen = true; mypv = pv; }
    else if (ok && myrow == col) myrow = prow;
    // branch-free: the pivot row and padding rows take g = 0 and keep their entries (a failed
    // column leaves garbage in a walker that is marked failed)
    const bool upd = ok && r < M && !ispiv;
    const double2 q = cmul(f, crecip_newton(pv));
    const double2 g = upd ? q : make_double2(0.0, 0.0);
    // eight entries at a time, the reads of the next eight in flight during the updates (the
    // pivot row's reads are not all hoisted at once)
    double2 pb[2][8];
#pragma unroll
    for (int i = 0; i < 8; ++i) pb[0][i] = pr[1 + i];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (k < 3) {
#pragma unroll
        for (int i = 0; i < 8; ++i)
          if (9 + 8 * k + i < NB) pb[(k + 1) & 1][i] = pr[9 + 8 * k + i];
      }
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (1 + 8 * k + i < NB) a[1 + 8 * k + i] = cfnms(a[1 + 8 * k + i], g, pb[k & 1][i]);
      __builtin_amdgcn_sched_barrier(0);
    }
    const double2 a0 = upd ? make_double2(-g.x, -g.y) : (ispiv ? make_double2(1.0, 0.0) : f);
#pragma unroll
    for (int i = 0; i < NB - 1; ++i) a[i] = a[i + 1];
    a[NB - 1] = a0;
  };
  int C = 0;
#pragma unroll 1
  for (; C + 4 <= jb; C += 4) {
    column(C);
    column(C + 1);
    column(C + 2);
    column(C + 3);
  }
#pragma unroll 1
  for (; C < jb; ++C) column(C);
#pragma unroll 1
  for (; C < NB; ++C) {                   // the zero columns beyond jb only rotate
    const double2 a0 = a[0];
#pragma unroll
    for (int i = 0; i < NB - 1; ++i) a[i] = a[i + 1];
    a[NB - 1] = a0;
  }
  // the row chosen for column c holds pv_c times row c of A11^{-1}
  double2* tri = p.tri + (long long)w * p.tri_stride;
  if (chosen) {
    const int c = myrow - j0;
    const double2 s = crecip(mypv);
#pragma unroll
    for (int i = 0; i < NB; ++i) tri[c * NB + i] = i < jb ? cmul(a[i], s) : make_double2(0.0, 0.0);
  }
  __syncthreads();                         // pivv / swapped of the last column
  // ln det contribution and pivot checks (wave 0 holds all jb <= 32 pivots)
  double lx = 0.0, ly = 0.0, nsw = 0.0, badv = 0.0;
  if (t < jb) {
    const double2 pv = sh.pivv[t];
    const double2 lg = clog(pv);
    lx = lg.x;
    ly = lg.y;
    nsw = sh.swapped[t] ? 1.0 : 0.0;
    if (!(cabs2(pv) > 0.0) || !isfinite(pv.x) || !isfinite(pv.y)) badv = 1.0;
  }
  if (wid == 0) {
    lx = wave_sum(lx); ly = wave_sum(ly); nsw = wave_sum(nsw); badv = wave_sum(badv);
  }
  const bool bad = badv > 0.0;
  if (t == 0) {
    if (p.lndet) {
      double2 acc = j0 == 0 ? make_double2(0.0, 0.0) : p.lndet[w];
      acc.x += lx;
      acc.y += ly + 3.14159265358979323846 * nsw;
      p.lndet[w] = acc;
    }
    if (bad && p.status) p.status[w] = 2;
  }
}

// ---------------------------------------------------------------------------------------
// Gauss-Jordan panel, column-split layout.  The same elimination as panel_gj_kernel with the
// work laid out the other way: a panel of PW = 32 or 64 columns, NW = PW / CPW waves, wave w
// holding panel columns
// [w CPW, (w+1) CPW) of every row (lane l, slot s: row j0 + l + 64 s).  Column C belongs to
// one wave, which searches the pivot alone (no cross-wave reduction) and computes the
// multiplier of every row; the multipliers reach the other waves through LDS, one entry per
// row, and each wave takes the pivot row's entries in its own columns from its own registers
// (readlane).  Per column that moves one entry per row through LDS instead of the whole pivot
// row to every thread.  The pivot choice (per group of 64 rows the lowest row among the
// largest keys, then the lowest label among the groups), the multipliers and every update are
// those of panel_gj_kernel, operation for operation, so the two give identical results.
template <int SL, int PW>
struct GjSplitShared {
  double2 g[2][SL][64];             // multipliers of column C, by column parity
  double2 pv[2];
  int info[2][4];                   // pivot label, its lane and slot, found
  double2 pivv[PW];
  int swapped[PW];
};

FT_DEV double readlane_d(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}
FT_DEV int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <int SL, int CPW, int PW>
__global__ __launch_bounds__(64 * (PW / CPW)) void panel_gj_split_kernel(PanelParams p) {
  constexpr int NW = PW / CPW;
  __shared__ GjSplitShared<SL, PW> sh;
  const int w = blockIdx.x;
  if (w >= p.W) return;
  double2* aug = p.aug + (long long)w * p.stride;
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const int M = p.M, j0 = p.j0, jb = p.jb, lda = p.lda;
  const int cw = wid * CPW;                // this wave's first panel column
  double2 a[SL][CPW];
  int label[SL];
  bool chosen[SL];
  double2 mypv[SL];
#pragma unroll
  for (int s = 0; s < SL; ++s) {
    const int r = j0 + lane + 64 * s;
    label[s] = r;
    chosen[s] = false;
    mypv[s] = make_double2(1.0, 0.0);
#pragma unroll
    for (int i = 0; i < CPW; ++i)
      a[s][i] = (r < M && cw + i < jb) ? aug[(long long)r * lda + j0 + cw + i] : make_double2(0.0, 0.0);
  }
  int* piv = p.piv + (long long)w * p.ld;
#pragma unroll 1
  for (int grp = 0; grp < NW && grp * CPW < jb; ++grp) {
#pragma unroll
    for (int cc = 0; cc < CPW; ++cc) {
      const int C = grp * CPW + cc;
      if (C >= jb) break;                  // uniform
      const int col = j0 + C, buf = C & 1;
      double2 g[SL], ncol[SL];
      if (wid == grp) {                    // the wave holding column C
        double2 f[SL];
        int key[SL], kmax = -1;
#pragma unroll
        for (int s = 0; s < SL; ++s) {
          f[s] = a[s][cc];
          const bool cand = label[s] >= col && label[s] < M;
          const double bv = cabs2(f[s]);
          key[s] = (cand && bv == bv) ? __double2hiint(bv) : -1;
          kmax = max(kmax, key[s]);
        }
        const int mk = wave_max_int(kmax);
        int bi = INT_MAX, bl = 0, bs = 0;
        const bool ok = mk >= 0;
        if (ok) {
#pragma unroll
          for (int s = 0; s < SL; ++s) {
            const unsigned long long hit = __ballot(key[s] == mk);
            if (hit) {
              const int lead = __ffsll((long long)hit) - 1;
              const int ix = __builtin_amdgcn_readlane(label[s], lead);
              if (ix < bi) { bi = ix; bl = lead; bs = s; }
            }
          }
        }
        const int prow = ok ? bi : col;
        double2 pv = make_double2(NAN, NAN);
        if (ok) {
#pragma unroll
          for (int s = 0; s < SL; ++s)
            if (s == bs) pv = make_double2(readlane_d(f[s].x, bl), readlane_d(f[s].y, bl));
        }
        const double2 rc = crecip_newton(pv);
#pragma unroll
        for (int s = 0; s < SL; ++s) {
          const bool ispiv = ok && label[s] == prow;
          const bool upd = ok && j0 + lane + 64 * s < M && !ispiv;
          const double2 q = cmul(f[s], rc);
          g[s] = upd ? q : make_double2(0.0, 0.0);
          sh.g[buf][s][lane] = g[s];
          ncol[s] = upd ? make_double2(-g[s].x, -g[s].y) : (ispiv ? make_double2(1.0, 0.0) : f[s]);
        }
        if (lane == 0) {
          sh.info[buf][0] = prow;
          sh.info[buf][1] = bl;
          sh.info[buf][2] = bs;
          sh.info[buf][3] = ok ? 1 : 0;
          sh.pv[buf] = pv;
          piv[col] = prow;
          sh.pivv[C] = pv;
          sh.swapped[C] = prow != col;
        }
      }
      __syncthreads();
      const int prow = uniform_i(sh.info[buf][0]), bl = uniform_i(sh.info[buf][1]);
      const int bs = uniform_i(sh.info[buf][2]);
      const bool ok = uniform_i(sh.info[buf][3]) != 0;
      const double2 pv = sh.pv[buf];
      if (wid != grp) {
#pragma unroll
        for (int s = 0; s < SL; ++s) g[s] = sh.g[buf][s][lane];
      }
      // the pivot row's entries in this wave's columns (it is not updated in this column)
      double2 pr[CPW];
#pragma unroll
      for (int i = 0; i < CPW; ++i) pr[i] = make_double2(0.0, 0.0);
      if (ok) {
#pragma unroll
        for (int s = 0; s < SL; ++s)
          if (s == bs) {
#pragma unroll
            for (int i = 0; i < CPW; ++i) pr[i] = make_double2(readlane_d(a[s][i].x, bl), readlane_d(a[s][i].y, bl));
          }
      }
#pragma unroll
      for (int s = 0; s < SL; ++s) {
#pragma unroll
        for (int i = 0; i < CPW; ++i) a[s][i] = cfnms(a[s][i], g[s], pr[i]);
      }
      if (wid == grp) {
#pragma unroll
        for (int s = 0; s < SL; ++s) a[s][cc] = ncol[s];
      }
#pragma unroll
      for (int s = 0; s < SL; ++s) {
        const bool ispiv = ok && label[s] == prow;
        if (ispiv) { label[s] = col; chosen[s] = true; mypv[s] = pv; }
        else if (ok && label[s] == col) label[s] = prow;
      }
    }
  }
  // the row chosen for column c holds pv_c times row c of A11^{-1}
  double2* tri = p.tri + (long long)w * p.tri_stride;
#pragma unroll
  for (int s = 0; s < SL; ++s) {
    if (chosen[s]) {
      const int c = label[s] - j0;
      const double2 sc = crecip(mypv[s]);
#pragma unroll
      for (int i = 0; i < CPW; ++i) tri[c * PW + cw + i] = cw + i < jb ? cmul(a[s][i], sc) : make_double2(0.0, 0.0);
    }
  }
  __syncthreads();                         // pivv / swapped of the last column
  double lx = 0.0, ly = 0.0, nsw = 0.0, badv = 0.0;
  if (t < jb) {
    const double2 pvt = sh.pivv[t];
    const double2 lg = clog(pvt);
    lx = lg.x;
    ly = lg.y;
    nsw = sh.swapped[t] ? 1.0 : 0.0;
    if (!(cabs2(pvt) > 0.0) || !isfinite(pvt.x) || !isfinite(pvt.y)) badv = 1.0;
  }
  if (wid == 0) {
    lx = wave_sum(lx); ly = wave_sum(ly); nsw = wave_sum(nsw); badv = wave_sum(badv);
  }
  if (t == 0) {
    if (p.lndet) {
      double2 acc = j0 == 0 ? make_double2(0.0, 0.0) : p.lndet[w];
      acc.x += lx;
      acc.y += ly + 3.14159265358979323846 * nsw;
      p.lndet[w] = acc;
    }
    if (badv > 0.0 && p.status) p.status[w] = 2;
  }
}

// Combined operator of a 64-column Gauss-Jordan step from its two 32-column halves.  With the
// first half's pivot block A11 (inverse T1), the second half's pivot rows A21 (original values
// in the first half's columns) and the inverse T2 of the second half's block after the first
// half's step, the pivot rows' trailing entries R1, R2 become
//     X = [[T1, 0], [-T2 A21 T1, T2]] [R1; R2]
// (X1 = T1 R1 is the first half's result, X2 the second's); every other row takes
// row -= A_i,[j0, j0+kb) X, and the first half's rows then take X1 - P1 X2 with P1 = T1 A12.
// One workgroup per walker; writes the kb x kb operator (row stride 2 NB) at TRI_TL.
struct CombineParams {
  const double2* aug; long long stride; int lda;
  double2* tri; long long tri_stride;
  int j0, jb2, W;
};

__global__ __launch_bounds__(256) void gj_combine_kernel(CombineParams c) {
  __shared__ double2 T1[NB][NB + 1], A21[NB][NB + 1], T2[NB][NB + 1], M21[NB][NB + 1];
  const int w = blockIdx.x;
  if (w >= c.W) return;
  double2* tri = c.tri + (long long)w * c.tri_stride;
  const double2* aug = c.aug + (long long)w * c.stride;
  const int t = threadIdx.x, jb2 = c.jb2, j0 = c.j0;
  for (int e = t; e < NB * NB; e += 256) {
    const int i = e / NB, j = e - i * NB;
    T1[i][j] = tri[TRI_T1 + e];
    T2[i][j] = (i < jb2 && j < jb2) ? tri[TRI_T2 + e] : make_double2(0.0, 0.0);
    A21[i][j] = i < jb2 ? aug[(long long)(j0 + NB + i) * c.lda + j0 + j] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int e = t; e < NB * NB; e += 256) {   // M21 = A21 T1
    const int i = e / NB, j = e - i * NB;
    double2 acc = make_double2(0.0, 0.0);
    for (int k = 0; k < NB; ++k) acc = cadd(acc, cmul(A21[i][k], T1[k][j]));
    M21[i][j] = acc;
  }
  __syncthreads();
  double2* tl = tri + TRI_TL;
  for (int e = t; e < 4 * NB * NB; e += 256) {
    const int i = e / (2 * NB), j = e - i * (2 * NB);
    double2 v = make_double2(0.0, 0.0);
    if (i < NB) {
      if (j < NB) v = T1[i][j];
    } else if (i - NB < jb2) {
      const int ii = i - NB;
      if (j < NB) {
        for (int k = 0; k < jb2; ++k) v = cfnms(v, T2[ii][k], M21[k][j]);
      } else if (j - NB < jb2) {
        v = T2[ii][j - NB];
      }
    }
    tl[e] = v;
  }
}

// Row exchanges of panel j0 for columns [c0, c1).  The jb exchanges compose into one
// permutation that moves at most 2 jb rows: the workgroup first finds, for every moved row, the
// row whose contents it receives (tracing the exchanges backwards), then each thread reads its
// column of all moved rows into registers (every load in flight at once), and after a barrier
// writes them to their new places.  64 columns per workgroup, one per lane, four row groups.
// PW is the panel width (32, or 64 for the 64-column Gauss-Jordan panel).
constexpr int SWAP_COLS = 64, SWAP_GROUPS = 4;
template <int PW>
__global__ __launch_bounds__(256) void swap_kernel(PanelParams p, int c0, int c1, int chunks) {
  constexpr int SWAP_PER = 2 * PW / SWAP_GROUPS;
  __shared__ int pv[PW];
  __shared__ int src[2 * PW], dst[2 * PW];
  __shared__ int nmov;
  const int w = blockIdx.x / chunks, ch = blockIdx.x - w * chunks;
  if (w >= p.W) return;
  const int t = threadIdx.x, j0 = p.j0, jb = p.jb, lda = p.lda;
  if (t < PW) pv[t] = t < jb ? p.piv[(long long)w * p.ld + j0 + t] : j0 + t;
  if (t == 0) nmov = 0;
  __syncthreads();
  if (t < 2 * jb) {
    // candidate position: a pivot row of the panel or the row it was exchanged with
    const int pos = t < jb ? j0 + t : pv[t - jb];
    bool first = true;
    if (t >= jb) {
      if (pos < j0 + jb) first = false;                     // listed by the first half
      for (int u = 0; u < t - jb; ++u) first = first && pv[u] != pos;
    }
    int from = pos;
    for (int c = jb - 1; c >= 0; --c) {
      const int a = j0 + c, b = pv[c];
      from = from == a ? b : (from == b ? a : from);
    }
    if (first && from != pos) {
      const int k = atomicAdd(&nmov, 1);
      src[k] = from;
      dst[k] = pos;
    }
  }
  __syncthreads();
  const int n = nmov, lane = t & (SWAP_COLS - 1);
  const int g = __builtin_amdgcn_readfirstlane(t / SWAP_COLS);   // row group = wave
  if (n == 0) return;                                     // uniform over the workgroup
  // lanes past c1 repeat the last column: the same value to the same address, no predicate
  const int cc = c0 + ch * SWAP_COLS + lane, col = cc < c1 ? cc : c1 - 1;
  double2* aug = p.aug + (long long)w * p.stride + col;
  double2 v[SWAP_PER];
#pragma unroll
  for (int i = 0; i < SWAP_PER; ++i) {
    const int r = g + i * SWAP_GROUPS;
    v[i] = r < n ? aug[(long long)src[r] * lda] : make_double2(0.0, 0.0);
  }
  __syncthreads();   // a moved row may be the source of another row in the same column
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): every load has returned before the stores
#pragma unroll
  for (int i = 0; i < SWAP_PER; ++i) {
    const int r = g + i * SWAP_GROUPS;
    if (r < n) aug[(long long)dst[r] * lda] = v[i];
  }
}

GemmParams aug_params(const ElimParams& e) {
  GemmParams g;
  memset(&g, 0, sizeof(g));
  g.sA = g.sB = g.sC = g.sP = e.stride;
  g.lda = g.ldb = g.ldc = g.ldp = e.lda;
  g.W = e.W;
  g.role = 1;
  return g;
}

// aug[row0.., col0..] -= aug[row0.., k0..k0+kb] aug[k0..k0+kb, col0..]
GemmParams update_params(const ElimParams& e, int row0, int nrows, int k0, int kb, int col0, int ncols) {
  GemmParams g = aug_params(e);
  g.A = e.aug + (long long)row0 * e.lda + k0;
  g.B = e.aug + (long long)k0 * e.lda + col0;
  g.C = e.aug + (long long)row0 * e.lda + col0;
  g.m = nrows; g.n = ncols; g.k = kb; g.mpad = nrows; g.npad = ncols;
  g.alpha = -1.0;
  g.beta = 1.0;
  return g;
}

// Rows the FP64 update GEMM computes for `rows` rows of C: a 32-row tile up to 32 rows, 64-row
// tiles above.
int update_row_work(int rows) { return rows <= 0 ? 0 : rows <= 32 ? 32 : 64 * ((rows + 63) / 64); }

// aug[r, c0..c0+ncols) -= aug[r, j0..j0+kb) aug[j0..j0+kb, c0..c0+ncols) for every row r but
// the pivot rows [j0, j0 + kb): two GEMMs over the rows above and below the pivot rows where
// they cover fewer tile rows than one GEMM over all M rows whose epilogue skips the pivot rows
// (a 64-column step at j0 = 64 c computes two tile rows of three at M = 171).  Every entry takes
// the same k-ordered sum either way.
hipError_t update_except(const ElimParams& e, int j0, int kb, int c0, int ncols, hipStream_t s) {
  const int M = e.M, below = M - j0 - kb;
  hipError_t err;
  if (update_row_work(j0) + update_row_work(below) < update_row_work(M)) {
    if (j0 > 0 && (err = launch_zgemm(update_params(e, 0, j0, j0, kb, c0, ncols), GEMM_Z64, s)) != hipSuccess)
      return err;
    return below > 0 ? launch_zgemm(update_params(e, j0 + kb, below, j0, kb, c0, ncols), GEMM_Z64, s) : hipSuccess;
  }
  GemmParams g = update_params(e, 0, M, j0, kb, c0, ncols);
  g.skip0 = j0;
  g.skip1 = j0 + kb;
  return launch_zgemm(g, GEMM_Z64, s);
}

// aug[row0..row0+kb, col0..] <- T aug[row0..row0+kb, col0..] with a per-walker kb x kb T (in place)
GemmParams tri_params(const ElimParams& e, const double2* T, int ldT, int row0, int kb, int col0, int ncols) {
  GemmParams g = aug_params(e);
  g.A = T; g.sA = TRI_ELEMS; g.lda = ldT;
  g.B = e.aug + (long long)row0 * e.lda + col0;
  g.C = e.aug + (long long)row0 * e.lda + col0;
  g.m = kb; g.n = ncols; g.k = kb; g.mpad = kb; g.npad = ncols;
  g.alpha = 1.0;
  return g;
}

}  // namespace

size_t elim_tri_elems(int) { return (size_t)TRI_ELEMS; }

namespace {

template <typename K64, typename K128, typename K256, typename K512>
hipError_t launch_panel(int rows, int W, const PanelParams& p, hipStream_t s, K64 k64, K128 k128, K256 k256, K512 k512) {
  if (rows <= 64) k64<<<W, 64, 0, s>>>(p);
  else if (rows <= 128) k128<<<W, 128, 0, s>>>(p);
  else if (rows <= 256) k256<<<W, 256, 0, s>>>(p);
  else k512<<<W, 512, 0, s>>>(p);
  return hipGetLastError();
}

// FTAFQMC_GJ_ROW_PANEL=1 in the environment selects the row-per-thread panel kernel (for
// comparisons: the two give identical results; read at every solve).
bool gj_row_panel() {
  const char* env = std::getenv("FTAFQMC_GJ_ROW_PANEL");
  return env && std::atoi(env) == 1;
}

hipError_t gj_panel(const PanelParams& p, int M, int W, bool row_panel, hipStream_t s) {
  const int rows = M - p.j0;
  if (row_panel)
    return launch_panel(rows, W, p, s, panel_gj_kernel<64>, panel_gj_kernel<128>, panel_gj_kernel<256>,
                        panel_gj_kernel<512>);
  if (rows <= 64) panel_gj_split_kernel<1, 8, NB><<<W, 256, 0, s>>>(p);
  else if (rows <= 128) panel_gj_split_kernel<2, 8, NB><<<W, 256, 0, s>>>(p);
  else if (rows <= 192) panel_gj_split_kernel<3, 8, NB><<<W, 256, 0, s>>>(p);
  else if (rows <= 256) panel_gj_split_kernel<4, 8, NB><<<W, 256, 0, s>>>(p);
  else if (rows <= 384) panel_gj_split_kernel<6, 4, NB><<<W, 512, 0, s>>>(p);
  else panel_gj_split_kernel<8, 4, NB><<<W, 512, 0, s>>>(p);
  return hipGetLastError();
}

// A 64-column panel (at most 256 rows): 8 waves of 8 columns, pivot block inverse at TRI_TL
// (row stride 64).
hipError_t gj_panel64(const PanelParams& p, int M, int W, hipStream_t s) {
  const int rows = M - p.j0;
  if (rows <= 64) panel_gj_split_kernel<1, 8, 2 * NB><<<W, 512, 0, s>>>(p);
  else if (rows <= 128) panel_gj_split_kernel<2, 8, 2 * NB><<<W, 512, 0, s>>>(p);
  else if (rows <= 192) panel_gj_split_kernel<3, 8, 2 * NB><<<W, 512, 0, s>>>(p);
  else if (rows <= 256) panel_gj_split_kernel<4, 8, 2 * NB><<<W, 512, 0, s>>>(p);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// FTAFQMC_GJ_PANEL64=0 in the environment keeps the solve on 32-column panels (read at every
// solve).
bool gj_panel64_on() {
  const char* env = std::getenv("FTAFQMC_GJ_PANEL64");
  return !env || std::atoi(env) != 0;
}

hipError_t swap_rows(const PanelParams& p, int W, int c0, int c1, hipStream_t s) {
  const int chunks = (c1 - c0 + SWAP_COLS - 1) / SWAP_COLS;
  if (p.jb > NB) swap_kernel<2 * NB><<<W * chunks, SWAP_COLS * SWAP_GROUPS, 0, s>>>(p, c0, c1, chunks);
  else swap_kernel<NB><<<W * chunks, SWAP_COLS * SWAP_GROUPS, 0, s>>>(p, c0, c1, chunks);
  return hipGetLastError();
}

// Gauss-Jordan with row pivoting over the augmented matrix.  With `wide`, 64 columns per step
// where two 32-column panels fit: one trailing update with K = 64 instead of two with K = 32
// halves the passes over the right-hand columns, for a small combine kernel and two 32-row
// products.  That pays where the updates are bound by memory traffic (large M); for small M
// they are bound by the FP64 matrix cores and 32-column steps are faster.
hipError_t launch_gj(const ElimParams& e, PanelParams p, int cend, bool wide, hipStream_t s) {
  const int M = e.M;
  const bool row_panel = gj_row_panel();
  const bool p64 = !row_panel && gj_panel64_on();
  hipError_t err;
  for (int j0 = 0; j0 < M;) {
    if (p64 && M - j0 > NB && M - j0 <= 256) {
      // one 64-column panel, its row exchanges, the pivot rows' product and one K = 64 update
      const int jb = M - j0 < 2 * NB ? M - j0 : 2 * NB, c0 = j0 + jb, ncols = cend - c0;
      p.j0 = j0; p.jb = jb; p.tri = e.tri + TRI_TL;
      if ((err = gj_panel64(p, M, e.W, s)) != hipSuccess) return err;
      if ((err = swap_rows(p, e.W, j0, cend, s)) != hipSuccess) return err;
      if (ncols > 0) {
        if ((err = launch_zgemm(tri_params(e, e.tri + TRI_TL, 2 * NB, j0, jb, c0, ncols), GEMM_Z64, s)) != hipSuccess) return err;
        if ((err = update_except(e, j0, jb, c0, ncols, s)) != hipSuccess) return err;
      }
      j0 += jb;
      continue;
    }
    if (!wide || M - j0 <= NB) {
      const int jb = M - j0 < NB ? M - j0 : NB, c0 = j0 + jb, ncols = cend - c0;
      p.j0 = j0; p.jb = jb; p.tri = e.tri + TRI_T1;
      if ((err = gj_panel(p, M, e.W, row_panel, s)) != hipSuccess) return err;
      if ((err = swap_rows(p, e.W, j0, cend, s)) != hipSuccess) return err;   // panel columns too
      if (ncols > 0) {
        if ((err = launch_zgemm(tri_params(e, e.tri + TRI_T1, NB, j0, jb, c0, ncols), GEMM_Z64, s)) != hipSuccess) return err;
        if ((err = update_except(e, j0, jb, c0, ncols, s)) != hipSuccess) return err;
      }
      j0 += jb;
      continue;
    }
    const int jb2 = M - j0 - NB < NB ? M - j0 - NB : NB, kb = NB + jb2;
    const int c2 = j0 + NB;               // the second half's columns [c2, c2 + jb2)
    // first half: pivots, T1, its step on the second half's columns only
    p.j0 = j0; p.jb = NB; p.tri = e.tri + TRI_T1;
    if ((err = gj_panel(p, M, e.W, row_panel, s)) != hipSuccess) return err;
    if ((err = swap_rows(p, e.W, j0, cend, s)) != hipSuccess) return err;
    if ((err = launch_zgemm(tri_params(e, e.tri + TRI_T1, NB, j0, NB, c2, jb2), GEMM_Z64, s)) != hipSuccess) return err;
    if ((err = update_except(e, j0, NB, c2, jb2, s)) != hipSuccess) return err;
    // second half: pivots among rows [c2, M), T2; its exchanges cover the first half's columns
    p.j0 = c2; p.jb = jb2; p.tri = e.tri + TRI_T2;
    if ((err = gj_panel(p, M, e.W, row_panel, s)) != hipSuccess) return err;
    if ((err = swap_rows(p, e.W, j0, cend, s)) != hipSuccess) return err;
    CombineParams cp;
    cp.aug = e.aug; cp.stride = e.stride; cp.lda = e.lda; cp.tri = e.tri; cp.tri_stride = TRI_ELEMS;
    cp.j0 = j0; cp.jb2 = jb2; cp.W = e.W;
    gj_combine_kernel<<<e.W, 256, 0, s>>>(cp);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    const int c0 = j0 + kb, ncols = cend - c0;
    if (ncols > 0) {
      if ((err = launch_zgemm(tri_params(e, e.tri + TRI_TL, 2 * NB, j0, kb, c0, ncols), GEMM_Z64, s)) != hipSuccess) return err;
      if ((err = update_except(e, j0, kb, c0, ncols, s)) != hipSuccess) return err;
      // first half's rows: X1 - P1 X2 (P1 in their second-half columns, X2 in the second half's rows)
      if ((err = launch_zgemm(update_params(e, j0, NB, c2, jb2, c0, ncols), GEMM_Z64, s)) != hipSuccess) return err;
    }
    j0 += kb;
  }
  return hipSuccess;
}

}  // namespace

namespace {
hipError_t forward_panel(const ElimParams& e, PanelParams p, int j0, int jb, double2* tri, hipStream_t s) {
  p.j0 = j0; p.jb = jb; p.tri = tri;
  return launch_panel(e.M - j0, e.W, p, s, panel_kernel<64>, panel_kernel<128>, panel_kernel<256>,
                      panel_kernel<512>);
}

// Forward elimination without pivoting; with `lower_left` the left block is lower triangular, so
// the pivot rows' entries right of the panel inside the left block are zeros and so is every
// left-block product: the pivot-block products and trailing updates cover the right-hand block only.
// Above GJ_WIDE_MIN_M rows (as for the solve) two 32-column panels make one step with a K = 64
// trailing update: the first panel's step reaches the second half's columns only, and the
// combined inverse of the 64-column unit lower block, [[T1, 0], [-T2 L21 T1, T2]], comes from the
// combine kernel (L21 being the first panel's multipliers in the second half's rows).
hipError_t launch_forward(const ElimParams& e, PanelParams p, bool lower_left, hipStream_t s) {
  const int M = e.M, cend = e.rhs_off + e.nrhs;
  const bool wide = M > gj_wide_min_m();
  hipError_t err;
  for (int j0 = 0; j0 < M;) {
    if (wide && M - j0 > NB) {
      const int jb2 = M - j0 - NB < NB ? M - j0 - NB : NB, kb = NB + jb2, c2 = j0 + NB;
      if ((err = forward_panel(e, p, j0, NB, e.tri + TRI_T1, s)) != hipSuccess) return err;
      if (!lower_left) {                   // (lower triangular: those columns of the pivot rows are zero)
        if ((err = launch_zgemm(tri_params(e, e.tri + TRI_T1, NB, j0, NB, c2, jb2), GEMM_Z64, s)) != hipSuccess) return err;
        if ((err = launch_zgemm(update_params(e, c2, M - c2, j0, NB, c2, jb2), GEMM_Z64, s)) != hipSuccess) return err;
      }
      if ((err = forward_panel(e, p, c2, jb2, e.tri + TRI_T2, s)) != hipSuccess) return err;
      CombineParams cp;
      cp.aug = e.aug; cp.stride = e.stride; cp.lda = e.lda; cp.tri = e.tri; cp.tri_stride = TRI_ELEMS;
      cp.j0 = j0; cp.jb2 = jb2; cp.W = e.W;
      gj_combine_kernel<<<e.W, 256, 0, s>>>(cp);
      if ((err = hipGetLastError()) != hipSuccess) return err;
      const int c0 = lower_left ? e.rhs_off : j0 + kb, ncols = cend - c0;
      if (ncols > 0) {
        if ((err = launch_zgemm(tri_params(e, e.tri + TRI_TL, 2 * NB, j0, kb, c0, ncols), GEMM_Z64, s)) != hipSuccess)
          return err;
        if (M - j0 - kb > 0 &&
            (err = launch_zgemm(update_params(e, j0 + kb, M - j0 - kb, j0, kb, c0, ncols), GEMM_Z64, s)) != hipSuccess)
          return err;
      }
      j0 += kb;
      continue;
    }
    const int jb = M - j0 < NB ? M - j0 : NB;
    if ((err = forward_panel(e, p, j0, jb, e.tri + TRI_T1, s)) != hipSuccess) return err;
    const int c0 = lower_left ? e.rhs_off : j0 + jb, ncols = cend - c0;
    if (ncols > 0) {
      if ((err = launch_zgemm(tri_params(e, e.tri + TRI_T1, NB, j0, jb, c0, ncols), GEMM_Z64, s)) != hipSuccess)
        return err;
      if (M - j0 - jb > 0 &&
          (err = launch_zgemm(update_params(e, j0 + jb, M - j0 - jb, j0, jb, c0, ncols), GEMM_Z64, s)) != hipSuccess)
        return err;
    }
    j0 += jb;
  }
  return hipSuccess;
}

PanelParams panel_params(const ElimParams& e) {
  PanelParams p;
  p.aug = e.aug; p.stride = e.stride; p.lda = e.lda; p.M = e.M; p.W = e.W; p.pivot = e.pivot;
  p.piv = e.piv; p.ld = e.ld; p.lndet = e.lndet; p.status = e.status; p.gj = e.backsub != 0 ? 1 : 0;
  p.tri = e.tri;
  p.tri_stride = TRI_ELEMS;
  return p;
}
}  // namespace

hipError_t launch_elim_lower(const ElimParams& e, hipStream_t s) {
  if (e.W <= 0 || e.M <= 0) return hipSuccess;
  if (e.M > 512 || !e.tri || e.pivot || e.backsub || e.rhs_off < e.M) return hipErrorInvalidValue;
  return launch_forward(e, panel_params(e), true, s);
}

hipError_t launch_elim(const ElimParams& e, hipStream_t s) {
  if (e.W <= 0 || e.M <= 0) return hipSuccess;
  if (e.M > 512 || !e.tri) return hipErrorInvalidValue;
  if ((e.pivot != 0) != (e.backsub != 0)) return hipErrorInvalidValue;   // the two modes built
  const int cend = e.rhs_off + e.nrhs;   // trailing columns run up to the end of the right-hand sides
  const PanelParams p = panel_params(e);
  if (e.backsub) return launch_gj(e, p, cend, e.M > gj_wide_min_m(), s);   // a solve: Gauss-Jordan
  return launch_forward(e, p, false, s);
}
