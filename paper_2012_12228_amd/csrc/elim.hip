// Blocked Gaussian elimination on per-walker augmented matrices [A | R], batched over walkers.
//
// Used for three solves of the slice path:
//   * the Green's function (eq. green) in scale-split form: A = X^T, R = (Ti D_b)^T with
//     partial pivoting, by blocked Gauss-Jordan, so R becomes X^{-T} (Ti D_b)^T;
//   * the Cholesky factor of S = Y^H Y in the QR stabilisation: no pivoting, forward
//     only; the left block becomes U = D L^H (S = L D L^H) and R becomes L^{-1} R;
//   * the update of T^{-1} by a unit triangular factor (again forward only).
// NB = 32 columns per panel, one kernel sequence for all walkers:
//   panel   one workgroup per walker factors the panel with partial pivoting, one row per
//           thread (pivot search = workgroup reduction, row exchange and rank-1 updates =
//           register operations with LDS broadcasts), then inverts the triangular factors of
//           the pivot block in LDS;
//   swap    column-parallel row exchanges;
// Forward elimination (LU, right-looking):
//   trsm    U12 = L11^{-1} A12 as a small in-place MFMA GEMM (each workgroup owns whole
//           columns and reads them completely before it writes);
//   update  A22 -= L21 U12 as a batched MFMA GEMM over the contiguous column range
//           [j0+NB, rhs_off+nrhs) (the zero padding between the two blocks stays zero).
// Gauss-Jordan (the solve with right-hand sides): the panel kernel leaves the panel columns
// untouched and returns A11^{-1} = U11^{-1} L11^{-1} of the pivot block; the row exchanges run
// over the panel columns too, the pivot rows become P = A11^{-1} [A12 | R1] in place, and every
// other row, above and below, takes row_i -= A_i1 P.  After the last panel the right-hand block
// holds the solution in natural order: row exchanges only reorder equations.
// ln det of the left block is the sum of the logs of the pivots plus i pi per row exchange.
#include "common.h"
#include "kernels.h"
#include <climits>
#include <cstring>

namespace {

constexpr int NB = 32;

struct PanelParams {
  double2* aug; long long stride; int lda;
  int M, j0, jb, W, pivot;
  int gj;         // Gauss-Jordan: keep the panel columns, return A11^{-1} instead of L11^{-1}
  int* piv; int ld;
  double2* lndet; int* status;
  double2* tri;   // [W][NB][NB] inverse of the unit lower L11 of this panel
};

template <int NT>
struct PanelShared {
  double2 candRow[2][NT / 64][NB];  // each wave's best row, double-buffered by column parity
  double candVal[2][NT / 64];
  int candIdx[2][NT / 64];
  double2 curRow[2][NB];            // logical row `col` (used without pivoting)
  double2 pivv[NB];                 // pivots of this panel
  int swapped[NB];
  double2 Ls[NB][NB + 1];           // unit lower L11, then its inverse
  double2 Us[NB][NB + 1];           // upper U11, then its inverse (Gauss-Jordan)
  double2 rpiv[NB];                 // 1 / U11_ii
};

// DPP move of a double within 16-lane rows (CTRL is a row-local pattern, every source exists).
template <int CTRL> FT_DEV double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
// Maximum over the 64 lanes of a wave, returned to every lane.
FT_DEV double wave_max(double v) {
  v = fmax(v, dpp_d<0xB1>(v));    // quad_perm [1,0,3,2]
  v = fmax(v, dpp_d<0x4E>(v));    // quad_perm [2,3,0,1]
  v = fmax(v, dpp_d<0x124>(v));   // row_ror:4
  v = fmax(v, dpp_d<0x128>(v));   // row_ror:8
  v = fmax(v, __shfl_xor(v, 16, 64));
  v = fmax(v, __shfl_xor(v, 32, 64));
  return v;
}

struct PanelCtx {
  int t, lane, wid, myrow, M, j0, jb, pivot;
  int* piv;
};

// Column C of the panel (compile-time, so every register index is static).  Row exchanges
// only relabel threads: the thread holding logical row prow becomes logical row col and vice
// versa; rows go to their final positions when the panel is written back.  One barrier per
// column: each wave publishes its best candidate (value, logical row, entries C..NB-1), and
// the owner of row col publishes that row for the unpivoted case.
template <int NT, int C>
FT_DEV void panel_column(double2 (&a)[NB], PanelCtx& x, PanelShared<NT>& sh) {
  if (C >= x.jb) return;                 // uniform over the workgroup
  const int col = x.j0 + C, buf = C & 1, M = x.M;
  const bool cand = x.myrow >= col && x.myrow < M;
  if (x.pivot) {
    double bv = cand ? cabs2(a[C]) : -1.0;
    if (!(bv == bv)) bv = -1.0;          // a NaN entry never wins the search
    const double mv = wave_max(bv);
    // lowest lane among the maxima; ties go to the smaller logical row
    int best = cand && bv == mv ? x.myrow : INT_MAX;
    for (int o = 32; o > 0; o >>= 1) best = min(best, __shfl_xor(best, o, 64));
    if (cand && bv == mv && x.myrow == best) {
#pragma unroll
      for (int i = C; i < NB; ++i) sh.candRow[buf][x.wid][i] = a[i];
    }
    if (x.lane == 0) { sh.candVal[buf][x.wid] = mv; sh.candIdx[buf][x.wid] = best; }
  } else if (x.myrow == col) {
#pragma unroll
    for (int i = C; i < NB; ++i) sh.curRow[buf][i] = a[i];
  }
  __syncthreads();
  int prow = col;
  const double2* pr = sh.curRow[buf];
  if (x.pivot) {
    double bv = sh.candVal[buf][0];
    int bi = sh.candIdx[buf][0], win = 0;
#pragma unroll
    for (int k = 1; k < NT / 64; ++k) {
      const double v = sh.candVal[buf][k];
      const int ix = sh.candIdx[buf][k];
      if (v > bv || (v == bv && ix < bi)) { bv = v; bi = ix; win = k; }
    }
    prow = (bi >= col && bi < M) ? bi : col;
    pr = sh.candRow[buf][win];
    if (prow == col && !(bi >= col && bi < M)) {
      // no usable candidate (all NaN): the diagonal row stays; its entries are its own
      pr = nullptr;
    }
    if (x.myrow == prow) x.myrow = col;
    else if (x.myrow == col) x.myrow = prow;
  }
  double2 pv;
  if (pr) pv = pr[C];
  else pv = make_double2(NAN, NAN);
  if (x.t == 0) {
    if (x.pivot) x.piv[col] = prow;
    sh.pivv[C] = pv;
    sh.swapped[C] = prow != col;
  }
  if (x.myrow > col && x.myrow < M && pr) {
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

// One workgroup per walker factors rows [j0, M) x columns [j0, j0+jb) with partial pivoting,
// one row per thread, then inverts the unit lower L11 (one column of the inverse per thread).
template <int NT>
__global__ __launch_bounds__(NT) void panel_kernel(PanelParams p) {
  __shared__ PanelShared<NT> sh;
  const int w = blockIdx.x;
  if (w >= p.W) return;
  double2* aug = p.aug + (long long)w * p.stride;
  const int t = threadIdx.x;
  const int M = p.M, j0 = p.j0, jb = p.jb, lda = p.lda;
  const int r = j0 + t;                    // the row this thread loads (M - j0 <= NT)
  double2 a[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) a[c] = (r < M && c < jb) ? aug[(long long)r * lda + j0 + c] : make_double2(0.0, 0.0);
  PanelCtx x;
  x.t = t; x.lane = t & 63; x.wid = t >> 6; x.myrow = r; x.M = M; x.j0 = j0; x.jb = jb; x.pivot = p.pivot;
  x.piv = p.piv + (long long)w * p.ld;
  PanelColumns<NT, 0>::run(a, x, sh);
  const int myrow = x.myrow;
  if (myrow < M && !p.gj) {
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < jb) aug[(long long)myrow * lda + j0 + c] = a[c];
  }
  // logical rows j0..j0+jb hold L11 in their strictly lower part and U11 in the rest
  if (myrow >= j0 && myrow < j0 + NB) {
    const int i = myrow - j0;
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      sh.Ls[i][c] = (c < i && i < jb) ? a[c] : make_double2(0.0, 0.0);
      sh.Us[i][c] = (c >= i && i < jb && c < jb) ? a[c] : make_double2(0.0, 0.0);
    }
  }
  // rows of the pivot block beyond jb (last panel) are the identity
  for (int i = jb + t; i < NB; i += NT)
    for (int c = 0; c < NB; ++c) {
      sh.Ls[i][c] = make_double2(0.0, 0.0);
      sh.Us[i][c] = make_double2(c == i ? 1.0 : 0.0, 0.0);
    }
  __syncthreads();
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
  if (x.wid == 0) {
    lx = wave_sum(lx); ly = wave_sum(ly); nsw = wave_sum(nsw); badv = wave_sum(badv);
  }
  // column t of L11^{-1} by forward substitution on e_t
  double2* tri = p.tri + (long long)w * NB * NB;
  if (t < NB) {
    double2 xcol[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      double2 v = make_double2(i == t ? 1.0 : 0.0, 0.0);
#pragma unroll
      for (int k = 0; k < i; ++k) v = cfnms(v, sh.Ls[i][k], xcol[k]);
      xcol[i] = v;
    }
    if (!p.gj) {
#pragma unroll
      for (int i = 0; i < NB; ++i) tri[i * NB + t] = xcol[i];
    } else {
      // threads 0..NB-1 are one wave: every read of Ls above precedes these writes
#pragma unroll
      for (int i = 0; i < NB; ++i) sh.Ls[i][t] = xcol[i];
      sh.rpiv[t] = cdiv(make_double2(1.0, 0.0), sh.Us[t][t]);
    }
  }
  if (p.gj) {
    __syncthreads();
    // column t of U11^{-1} by back substitution on e_t (again one wave, in place)
    if (t < NB) {
      double2 xcol[NB];
#pragma unroll
      for (int i = NB - 1; i >= 0; --i) {
        double2 v = make_double2(i == t ? 1.0 : 0.0, 0.0);
#pragma unroll
        for (int k = i + 1; k < NB; ++k) v = cfnms(v, sh.Us[i][k], xcol[k]);
        xcol[i] = cmul(v, sh.rpiv[i]);
      }
#pragma unroll
      for (int i = 0; i < NB; ++i) sh.Us[i][t] = xcol[i];
    }
    __syncthreads();
    // A11^{-1} = U11^{-1} L11^{-1}
    for (int e = t; e < NB * NB; e += NT) {
      const int i = e / NB, j = e - i * NB;
      double2 acc = make_double2(0.0, 0.0);
      for (int k = (i > j ? i : j); k < NB; ++k) acc = cadd(acc, cmul(sh.Us[i][k], sh.Ls[k][j]));
      tri[e] = acc;
    }
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

// Row exchanges of panel j0 for columns [c0, c1), one column per thread.
__global__ __launch_bounds__(256) void swap_kernel(PanelParams p, int c0, int c1, int chunks) {
  __shared__ int pv[NB];
  const int w = blockIdx.x / chunks, ch = blockIdx.x - w * chunks;
  if (w >= p.W) return;
  const int t = threadIdx.x, j0 = p.j0, jb = p.jb, lda = p.lda;
  if (t < NB) pv[t] = t < jb ? p.piv[(long long)w * p.ld + j0 + t] : j0 + t;
  __syncthreads();
  const int col = c0 + ch * 256 + t;
  if (col >= c1) return;
  double2* aug = p.aug + (long long)w * p.stride;
  for (int c = 0; c < jb; ++c) {
    const int pr = pv[c];
    if (pr != j0 + c) {
      const double2 u = aug[(long long)(j0 + c) * lda + col];
      aug[(long long)(j0 + c) * lda + col] = aug[(long long)pr * lda + col];
      aug[(long long)pr * lda + col] = u;
    }
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

// aug[row0..row0+kb, col0..] <- T aug[row0..row0+kb, col0..] with a per-walker kb x kb T (in place)
GemmParams tri_params(const ElimParams& e, const double2* T, long long sT, int row0, int kb, int col0, int ncols) {
  GemmParams g = aug_params(e);
  g.A = T; g.sA = sT; g.lda = NB;
  g.B = e.aug + (long long)row0 * e.lda + col0;
  g.C = e.aug + (long long)row0 * e.lda + col0;
  g.m = kb; g.n = ncols; g.k = kb; g.mpad = kb; g.npad = ncols;
  g.alpha = 1.0;
  return g;
}

}  // namespace

size_t elim_tri_elems(int) { return (size_t)NB * NB; }

hipError_t launch_elim(const ElimParams& e, hipStream_t s) {
  if (e.W <= 0 || e.M <= 0) return hipSuccess;
  if (e.M > 512 || !e.tri) return hipErrorInvalidValue;
  const int M = e.M;
  const int cend = e.rhs_off + e.nrhs;   // trailing columns run up to the end of the right-hand sides
  const bool gj = e.backsub != 0;        // a solve: Gauss-Jordan, no back substitution
  PanelParams p;
  p.aug = e.aug; p.stride = e.stride; p.lda = e.lda; p.M = M; p.W = e.W; p.pivot = e.pivot;
  p.piv = e.piv; p.ld = e.ld; p.lndet = e.lndet; p.status = e.status; p.gj = gj ? 1 : 0;
  p.tri = e.tri;                          // [W][NB][NB]: L11^{-1} (forward) or A11^{-1} (Gauss-Jordan)
  hipError_t err;
  for (int j0 = 0; j0 < M; j0 += NB) {
    const int jb = M - j0 < NB ? M - j0 : NB;
    p.j0 = j0; p.jb = jb;
    if (M - j0 <= 64) panel_kernel<64><<<e.W, 64, 0, s>>>(p);
    else if (M - j0 <= 128) panel_kernel<128><<<e.W, 128, 0, s>>>(p);
    else if (M - j0 <= 256) panel_kernel<256><<<e.W, 256, 0, s>>>(p);
    else panel_kernel<512><<<e.W, 512, 0, s>>>(p);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    const int c0 = j0 + jb;
    const int ncols = cend - c0;
    if (ncols <= 0) continue;
    if (e.pivot) {
      const int s0 = gj ? j0 : c0;        // Gauss-Jordan keeps the panel columns in memory: swap them too
      const int chunks = (cend - s0 + 255) / 256;
      swap_kernel<<<e.W * chunks, 256, 0, s>>>(p, s0, cend, chunks);
      if ((err = hipGetLastError()) != hipSuccess) return err;
    }
    if ((err = launch_zgemm(tri_params(e, e.tri, (long long)NB * NB, j0, jb, c0, ncols), GEMM_Z64, s)) != hipSuccess)
      return err;
    if (gj) {
      GemmParams g = update_params(e, 0, M, j0, jb, c0, ncols);   // every row but the pivot rows
      g.skip0 = j0;
      g.skip1 = j0 + jb;
      if ((err = launch_zgemm(g, GEMM_Z64, s)) != hipSuccess) return err;
    } else if (M - c0 > 0 && (err = launch_zgemm(update_params(e, c0, M - c0, j0, jb, c0, ncols), GEMM_Z64, s)) != hipSuccess) {
      return err;
    }
  }
  return hipSuccess;
}
