// Blocked Gaussian elimination on per-walker augmented matrices [A | R], batched over walkers.
//
// Used for three solves of the slice path:
//   * the Green's function (eq. green) in scale-split form: A = X^T, R = (Ti D_b)^T with
//     partial pivoting and back substitution, so R becomes X^{-T} (Ti D_b)^T;
//   * the Cholesky factor of S = Y^H Y in the QR stabilisation: no pivoting, forward
//     only; the left block becomes U = D L^H (S = L D L^H) and R becomes L^{-1} R;
//   * the update of T^{-1} by a unit triangular factor (again forward only).
// Right-looking with NB = 32 columns per panel, one kernel sequence for all walkers:
//   panel      one workgroup per walker factors the M x NB panel with partial pivoting,
//              one row per thread (the pivot search is a workgroup reduction, the row
//              exchange and the rank-1 updates are register operations with LDS broadcasts);
//   swap/trsm  column-parallel: applies the panel's row exchanges to the trailing
//              columns and right-hand sides and solves with the unit lower L11;
//   update     the trailing update A22 -= L21 U12 as a batched complex GEMM on MFMA,
//              over the contiguous column range [j0+NB, rhs_off+nrhs) (the zero padding
//              between the blocks stays zero);
// then the back substitution by blocks from the bottom (column-parallel triangular solve
// with U_ii, GEMM update of the rows above).  ln det of the left block is the sum of the
// logs of the pivots plus i pi per row exchange.
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
};

template <int NT>
__global__ __launch_bounds__(NT) void panel_kernel(PanelParams p) {
  __shared__ double2 bufP[NB];
  __shared__ double2 bufC[NB];
  __shared__ double redv[NT / 64];
  __shared__ int redi[NT / 64];
  const int w = blockIdx.x;
  if (w >= p.W) return;
  double2* aug = p.aug + (long long)w * p.stride;
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const int M = p.M, j0 = p.j0, jb = p.jb, lda = p.lda;
  const int r = j0 + t;                    // one panel row per thread (M - j0 <= NT)
  double2 a[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) a[c] = (r < M && c < jb) ? aug[(long long)r * lda + j0 + c] : make_double2(0.0, 0.0);
  double2 lsum = make_double2(0.0, 0.0);
  int nswaps = 0;
  bool bad = false;
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    if (c >= jb) break;
    const int col = j0 + c;
    int prow = col;
    if (p.pivot) {
      double bv = (r >= col && r < M) ? cabs2(a[c]) : -1.0;
      int bi = (r >= col && r < M) ? r : INT_MAX;
      if (!(bv == bv)) bv = -1.0;          // a NaN entry never wins the search
      for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(bv, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
      }
      if (lane == 0) { redv[wid] = bv; redi[wid] = bi; }
      __syncthreads();
      bv = redv[0]; bi = redi[0];
#pragma unroll
      for (int k = 1; k < NT / 64; ++k)
        if (redv[k] > bv || (redv[k] == bv && redi[k] < bi)) { bv = redv[k]; bi = redi[k]; }
      prow = (bi >= col && bi < M) ? bi : col;
    }
    if (r == prow) {
#pragma unroll
      for (int c2 = 0; c2 < NB; ++c2) bufP[c2] = a[c2];
    }
    if (prow != col && r == col) {
#pragma unroll
      for (int c2 = 0; c2 < NB; ++c2) bufC[c2] = a[c2];
    }
    __syncthreads();
    if (prow != col) {
      if (r == prow) {
#pragma unroll
        for (int c2 = 0; c2 < NB; ++c2) a[c2] = bufC[c2];
      }
      if (r == col) {
#pragma unroll
        for (int c2 = 0; c2 < NB; ++c2) a[c2] = bufP[c2];
      }
    }
    const double2 pv = bufP[c];
    if (t == 0) {
      if (p.pivot) p.piv[(long long)w * p.ld + col] = prow;
      if (!(cabs2(pv) > 0.0) || !isfinite(pv.x) || !isfinite(pv.y)) bad = true;
      const double2 lg = clog(pv);
      lsum.x += lg.x;
      lsum.y += lg.y;
      if (prow != col) ++nswaps;
    }
    if (r > col && r < M) {
      const double2 l = cdiv(a[c], pv);
      a[c] = l;
#pragma unroll
      for (int c2 = 0; c2 < NB; ++c2)
        if (c2 > c) a[c2] = cfnms(a[c2], l, bufP[c2]);
    }
    __syncthreads();
  }
  if (r < M) {
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < jb) aug[(long long)r * lda + j0 + c] = a[c];
  }
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

// Row exchanges of panel j0 and U12 = L11^{-1} A12 for columns [c0, c1) (one column per thread).
__global__ __launch_bounds__(256) void swap_trsm_kernel(PanelParams p, int c0, int c1, int chunks) {
  __shared__ double2 L11[NB][NB + 1];
  __shared__ int pv[NB];
  const int w = blockIdx.x / chunks, ch = blockIdx.x - w * chunks;
  if (w >= p.W) return;
  double2* aug = p.aug + (long long)w * p.stride;
  const int t = threadIdx.x, j0 = p.j0, jb = p.jb, lda = p.lda;
  for (int e = t; e < NB * NB; e += 256) {
    const int i = e / NB, m = e - i * NB;
    L11[i][m] = (i < jb && m < i) ? aug[(long long)(j0 + i) * lda + j0 + m] : make_double2(0.0, 0.0);
  }
  if (t < NB) pv[t] = (p.pivot && t < jb) ? p.piv[(long long)w * p.ld + j0 + t] : j0 + t;
  __syncthreads();
  const int col = c0 + ch * 256 + t;
  if (col >= c1) return;
  for (int c = 0; c < jb; ++c) {
    const int pr = pv[c];
    if (pr != j0 + c) {
      const double2 u = aug[(long long)(j0 + c) * lda + col];
      aug[(long long)(j0 + c) * lda + col] = aug[(long long)pr * lda + col];
      aug[(long long)pr * lda + col] = u;
    }
  }
  double2 x[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) x[i] = i < jb ? aug[(long long)(j0 + i) * lda + col] : make_double2(0.0, 0.0);
#pragma unroll
  for (int i = 1; i < NB; ++i)
#pragma unroll
    for (int m = 0; m < NB; ++m)
      if (m < i) x[i] = cfnms(x[i], L11[i][m], x[m]);
#pragma unroll
  for (int i = 0; i < NB; ++i)
    if (i < jb) aug[(long long)(j0 + i) * lda + col] = x[i];
}

// Back substitution with the upper block U_ii (rows/cols i0..i0+ib) for columns [c0, c1).
__global__ __launch_bounds__(256) void trsm_upper_kernel(PanelParams p, int i0, int ib, int c0, int c1, int chunks) {
  __shared__ double2 U[NB][NB + 1];
  const int w = blockIdx.x / chunks, ch = blockIdx.x - w * chunks;
  if (w >= p.W) return;
  double2* aug = p.aug + (long long)w * p.stride;
  const int t = threadIdx.x, lda = p.lda;
  for (int e = t; e < NB * NB; e += 256) {
    const int i = e / NB, m = e - i * NB;
    U[i][m] = (i < ib && m < ib && m >= i) ? aug[(long long)(i0 + i) * lda + i0 + m] : make_double2(i == m ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  const int col = c0 + ch * 256 + t;
  if (col >= c1) return;
  double2 x[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) x[i] = i < ib ? aug[(long long)(i0 + i) * lda + col] : make_double2(0.0, 0.0);
#pragma unroll
  for (int i = NB - 1; i >= 0; --i) {
#pragma unroll
    for (int m = 0; m < NB; ++m)
      if (m > i) x[i] = cfnms(x[i], U[i][m], x[m]);
    x[i] = cdiv(x[i], U[i][i]);
  }
#pragma unroll
  for (int i = 0; i < NB; ++i)
    if (i < ib) aug[(long long)(i0 + i) * lda + col] = x[i];
}

GemmParams update_params(const ElimParams& e, int row0, int nrows, int k0, int kb, int col0, int ncols) {
  // aug[row0.., col0..] -= aug[row0.., k0..k0+kb] aug[k0..k0+kb, col0..]
  GemmParams g;
  memset(&g, 0, sizeof(g));
  g.A = e.aug + (long long)row0 * e.lda + k0;
  g.B = e.aug + (long long)k0 * e.lda + col0;
  g.C = e.aug + (long long)row0 * e.lda + col0;
  g.sA = g.sB = g.sC = g.sP = e.stride;
  g.lda = g.ldb = g.ldc = g.ldp = e.lda;
  g.m = nrows; g.n = ncols; g.k = kb; g.mpad = nrows; g.npad = ncols; g.W = e.W;
  g.alpha = -1.0;
  g.beta = 1.0;
  return g;
}

}  // namespace

hipError_t launch_elim(const ElimParams& e, hipStream_t s) {
  if (e.W <= 0 || e.M <= 0) return hipSuccess;
  if (e.M > 512) return hipErrorInvalidValue;
  const int M = e.M;
  const int cend = e.rhs_off + e.nrhs;   // trailing columns run up to the end of the right-hand sides
  PanelParams p;
  p.aug = e.aug; p.stride = e.stride; p.lda = e.lda; p.M = M; p.W = e.W; p.pivot = e.pivot;
  p.piv = e.piv; p.ld = e.ld; p.lndet = e.lndet; p.status = e.status;
  for (int j0 = 0; j0 < M; j0 += NB) {
    const int jb = M - j0 < NB ? M - j0 : NB;
    p.j0 = j0; p.jb = jb;
    if (M - j0 <= 64) panel_kernel<64><<<e.W, 64, 0, s>>>(p);
    else if (M - j0 <= 256) panel_kernel<256><<<e.W, 256, 0, s>>>(p);
    else panel_kernel<512><<<e.W, 512, 0, s>>>(p);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    const int c0 = j0 + jb;
    const int ncols = cend - c0;
    if (ncols <= 0) continue;
    const int chunks = (ncols + 255) / 256;
    swap_trsm_kernel<<<e.W * chunks, 256, 0, s>>>(p, c0, cend, chunks);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    if (M - c0 > 0) {
      err = launch_zgemm(update_params(e, c0, M - c0, j0, jb, c0, ncols), GEMM_Z64, s);
      if (err != hipSuccess) return err;
    }
  }
  if (e.backsub) {
    const int chunks = (e.nrhs + 255) / 256;
    for (int i0 = ((M - 1) / NB) * NB; i0 >= 0; i0 -= NB) {
      const int ib = M - i0 < NB ? M - i0 : NB;
      trsm_upper_kernel<<<e.W * chunks, 256, 0, s>>>(p, i0, ib, e.rhs_off, cend, chunks);
      hipError_t err = hipGetLastError();
      if (err != hipSuccess) return err;
      if (i0 > 0) {
        err = launch_zgemm(update_params(e, 0, i0, i0, ib, e.rhs_off, e.nrhs), GEMM_Z64, s);
        if (err != hipSuccess) return err;
      }
    }
  }
  return hipSuccess;
}
