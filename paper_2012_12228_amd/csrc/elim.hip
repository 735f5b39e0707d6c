// Blocked Gaussian elimination on per-walker augmented matrices [A | R], batched over walkers.
//
// Used for three solves of the slice path:
//   * the Green's function (eq. green) in scale-split form: A = X^T, R = (Ti D_b)^T with
//     partial pivoting and back substitution, so R becomes X^{-T} (Ti D_b)^T;
//   * the Cholesky factor of S = Y^H Y in the QR stabilisation: no pivoting, forward
//     only; the left block becomes U = D L^H (S = L D L^H) and R becomes L^{-1} R;
//   * the update of T^{-1} by a unit triangular factor (again forward only).
// Right-looking with NB = 32 columns per panel, one kernel sequence for all walkers:
//   panel   one workgroup per walker factors the panel with partial pivoting, one row per
//           thread (pivot search = workgroup reduction, row exchange and rank-1 updates =
//           register operations with LDS broadcasts), then inverts the unit lower L11 in LDS;
//   swap    column-parallel row exchanges of the trailing columns and right-hand sides;
//   trsm    U12 = L11^{-1} A12 as a small in-place MFMA GEMM (each workgroup owns whole
//           columns and reads them completely before it writes);
//   update  A22 -= L21 U12 as a batched MFMA GEMM over the contiguous column range
//           [j0+NB, rhs_off+nrhs) (the zero padding between the two blocks stays zero).
// Back substitution: the inverses of the diagonal blocks of U in one launch, then by
// blocks from the bottom an in-place GEMM H_i = U_ii^{-1} R_i and the update of the rows
// above.  ln det of the left block is the sum of the logs of the pivots plus i pi per
// row exchange.
#include "common.h"
#include "kernels.h"
#include <climits>
#include <cstring>

namespace {

constexpr int NB = 32;

struct PanelParams {
  double2* aug; long long stride; int lda;
  int M, j0, jb, W, pivot;
  int* piv; int ld;
  double2* lndet; int* status;
  double2* tri;   // [W][NB][NB] inverse of the unit lower L11 of this panel
};

struct PanelCtx {
  int t, lane, wid, r, M, j0, jb, pivot, nswaps;
  bool bad;
  double2 lsum;
  int* piv;          // this walker's pivot rows
};

template <int NT>
struct PanelShared {
  double2 bufP[NB];
  double2 bufC[NB];
  double redv[NT / 64];
  int redi[NT / 64];
  double2 Ls[NB][NB + 1];
  double2 Li[NB][NB + 1];
};

// Elimination step of panel column C (a compile-time index, so the row stays in registers).
template <int NT, int C>
FT_DEV void panel_column(double2 (&a)[NB], PanelCtx& x, PanelShared<NT>& sh) {
  if (C >= x.jb) return;                 // uniform over the workgroup
  const int col = x.j0 + C, r = x.r, M = x.M;
  int prow = col;
  if (x.pivot) {
    double bv = (r >= col && r < M) ? cabs2(a[C]) : -1.0;
    int bi = (r >= col && r < M) ? r : INT_MAX;
    if (!(bv == bv)) bv = -1.0;          // a NaN entry never wins the search
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(bv, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
    }
    if (x.lane == 0) { sh.redv[x.wid] = bv; sh.redi[x.wid] = bi; }
    __syncthreads();
    bv = sh.redv[0]; bi = sh.redi[0];
#pragma unroll
    for (int k = 1; k < NT / 64; ++k)
      if (sh.redv[k] > bv || (sh.redv[k] == bv && sh.redi[k] < bi)) { bv = sh.redv[k]; bi = sh.redi[k]; }
    prow = (bi >= col && bi < M) ? bi : col;
  }
  if (r == prow) {
#pragma unroll
    for (int c2 = 0; c2 < NB; ++c2) sh.bufP[c2] = a[c2];
  }
  if (prow != col && r == col) {
#pragma unroll
    for (int c2 = 0; c2 < NB; ++c2) sh.bufC[c2] = a[c2];
  }
  __syncthreads();
  if (prow != col) {
    if (r == prow) {
#pragma unroll
      for (int c2 = 0; c2 < NB; ++c2) a[c2] = sh.bufC[c2];
    }
    if (r == col) {
#pragma unroll
      for (int c2 = 0; c2 < NB; ++c2) a[c2] = sh.bufP[c2];
    }
  }
  const double2 pv = sh.bufP[C];
  if (x.t == 0) {
    if (x.pivot) x.piv[col] = prow;
    if (!(cabs2(pv) > 0.0) || !isfinite(pv.x) || !isfinite(pv.y)) x.bad = true;
    const double2 lg = clog(pv);
    x.lsum.x += lg.x;
    x.lsum.y += lg.y;
    if (prow != col) ++x.nswaps;
  }
  if (r > col && r < M) {
    const double2 l = cdiv(a[C], pv);
    a[C] = l;
#pragma unroll
    for (int c2 = C + 1; c2 < NB; ++c2) a[c2] = cfnms(a[c2], l, sh.bufP[c2]);
  }
  __syncthreads();
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

template <int NT>
__global__ __launch_bounds__(NT) void panel_kernel(PanelParams p) {
  __shared__ PanelShared<NT> sh;
  const int w = blockIdx.x;
  if (w >= p.W) return;
  double2* aug = p.aug + (long long)w * p.stride;
  const int t = threadIdx.x;
  const int M = p.M, j0 = p.j0, jb = p.jb, lda = p.lda;
  const int r = j0 + t;                    // one panel row per thread (M - j0 <= NT)
  double2 a[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) a[c] = (r < M && c < jb) ? aug[(long long)r * lda + j0 + c] : make_double2(0.0, 0.0);
  PanelCtx x;
  x.t = t; x.lane = t & 63; x.wid = t >> 6; x.r = r; x.M = M; x.j0 = j0; x.jb = jb; x.pivot = p.pivot;
  x.nswaps = 0; x.bad = false; x.lsum = make_double2(0.0, 0.0);
  x.piv = p.piv + (long long)w * p.ld;
  PanelColumns<NT, 0>::run(a, x, sh);
  double2 lsum = x.lsum;
  const int nswaps = x.nswaps;
  const bool bad = x.bad;
  if (r < M) {
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < jb) aug[(long long)r * lda + j0 + c] = a[c];
  }
  // inverse of the unit lower L11 (rows j0..j0+jb are threads 0..jb-1)
  if (t < NB) {
#pragma unroll
    for (int c = 0; c < NB; ++c) sh.Ls[t][c] = (c < t && t < jb) ? a[c] : make_double2(0.0, 0.0);
  }
  for (int e = t; e < NB * NB; e += NT) {
    const int i = e / NB, c = e - i * NB;
    sh.Li[i][c] = make_double2(i == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int k = 0; k < jb - 1; ++k) {      // row i of L^{-1} -= L[i][k] * row k, for i > k
    for (int e = t; e < NB * NB; e += NT) {
      const int i = e / NB, c = e - i * NB;
      if (i > k && c <= k) sh.Li[i][c] = cfnms(sh.Li[i][c], sh.Ls[i][k], sh.Li[k][c]);
    }
    __syncthreads();
  }
  double2* tri = p.tri + (long long)w * NB * NB;
  for (int e = t; e < NB * NB; e += NT) tri[e] = sh.Li[e / NB][e % NB];
  if (t == 0) {
    if (p.lndet) {
      double2 acc = j0 == 0 ? make_double2(0.0, 0.0) : p.lndet[w];
      acc.x += lsum.x;
      acc.y += lsum.y + 3.14159265358979323846 * (double)nswaps;
      p.lndet[w] = acc;
    }
    if (bad && p.status) p.status[w] = 2;
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

// Inverses of the upper triangular diagonal blocks U_bb, one workgroup per (walker, block).
__global__ __launch_bounds__(256) void tri_inv_upper_kernel(PanelParams p, int nblk, double2* uinv) {
  __shared__ double2 U[NB][NB + 1];
  __shared__ double2 X[NB][NB + 1];
  const int w = blockIdx.x / nblk, b = blockIdx.x - w * nblk;
  if (w >= p.W) return;
  const int i0 = b * NB, ib = min(NB, p.M - i0), t = threadIdx.x;
  const double2* aug = p.aug + (long long)w * p.stride;
  for (int e = t; e < NB * NB; e += 256) {
    const int i = e / NB, c = e - i * NB;
    U[i][c] = (i < ib && c < ib && c >= i) ? aug[(long long)(i0 + i) * p.lda + i0 + c]
                                            : make_double2(i == c ? 1.0 : 0.0, 0.0);
    X[i][c] = make_double2(i == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  // U X = I from the last row up: X[k][:] = (I[k][:] - sum_{m>k} U[k][m] X[m][:]) / U[k][k]
  for (int k = NB - 1; k >= 0; --k) {
    if (t < NB) {
      double2 v = X[k][t];
      for (int m = k + 1; m < NB; ++m) v = cfnms(v, U[k][m], X[m][t]);
      X[k][t] = cdiv(v, U[k][k]);
    }
    __syncthreads();
  }
  double2* out = uinv + ((long long)w * nblk + b) * NB * NB;
  for (int e = t; e < NB * NB; e += 256) out[e] = X[e / NB][e % NB];
}

GemmParams aug_params(const ElimParams& e) {
  GemmParams g;
  memset(&g, 0, sizeof(g));
  g.sA = g.sB = g.sC = g.sP = e.stride;
  g.lda = g.ldb = g.ldc = g.ldp = e.lda;
  g.W = e.W;
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

size_t elim_tri_elems(int M) { return (size_t)((M + NB - 1) / NB) * NB * NB; }

hipError_t launch_elim(const ElimParams& e, hipStream_t s) {
  if (e.W <= 0 || e.M <= 0) return hipSuccess;
  if (e.M > 512 || !e.tri) return hipErrorInvalidValue;
  const int M = e.M;
  const int cend = e.rhs_off + e.nrhs;   // trailing columns run up to the end of the right-hand sides
  const int nblk = (M + NB - 1) / NB;
  double2* linv = e.tri;                  // forward phase: [W][NB][NB], the current panel's L11^{-1}
  double2* uinv = e.tri;                  // back substitution: [W][nblk][NB][NB], the U_bb^{-1}
  PanelParams p;
  p.aug = e.aug; p.stride = e.stride; p.lda = e.lda; p.M = M; p.W = e.W; p.pivot = e.pivot;
  p.piv = e.piv; p.ld = e.ld; p.lndet = e.lndet; p.status = e.status;
  hipError_t err;
  for (int j0 = 0; j0 < M; j0 += NB) {
    const int jb = M - j0 < NB ? M - j0 : NB;
    p.j0 = j0; p.jb = jb;
    p.tri = linv;                         // L11^{-1} of walker w at linv + w * NB * NB
    if (M - j0 <= 64) panel_kernel<64><<<e.W, 64, 0, s>>>(p);
    else if (M - j0 <= 256) panel_kernel<256><<<e.W, 256, 0, s>>>(p);
    else panel_kernel<512><<<e.W, 512, 0, s>>>(p);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    const int c0 = j0 + jb;
    const int ncols = cend - c0;
    if (ncols <= 0) continue;
    if (e.pivot) {
      const int chunks = (ncols + 255) / 256;
      swap_kernel<<<e.W * chunks, 256, 0, s>>>(p, c0, cend, chunks);
      if ((err = hipGetLastError()) != hipSuccess) return err;
    }
    if ((err = launch_zgemm(tri_params(e, linv, (long long)NB * NB, j0, jb, c0, ncols), GEMM_Z64, s)) != hipSuccess)
      return err;
    if (M - c0 > 0 && (err = launch_zgemm(update_params(e, c0, M - c0, j0, jb, c0, ncols), GEMM_Z64, s)) != hipSuccess)
      return err;
  }
  if (e.backsub) {
    tri_inv_upper_kernel<<<e.W * nblk, 256, 0, s>>>(p, nblk, uinv);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    for (int b = nblk - 1; b >= 0; --b) {
      const int i0 = b * NB, ib = M - i0 < NB ? M - i0 : NB;
      GemmParams g = tri_params(e, uinv + (long long)b * NB * NB, (long long)nblk * NB * NB, i0, ib, e.rhs_off, e.nrhs);
      if ((err = launch_zgemm(g, GEMM_Z64, s)) != hipSuccess) return err;
      if (i0 > 0 && (err = launch_zgemm(update_params(e, 0, i0, i0, ib, e.rhs_off, e.nrhs), GEMM_Z64, s)) != hipSuccess)
        return err;
    }
  }
  return hipSuccess;
}
