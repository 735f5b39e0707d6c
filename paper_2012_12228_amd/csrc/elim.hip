// Per-walker blocked Gaussian elimination on an augmented matrix [A | R].
//
// Used for three solves of the slice path, all by one 256-thread workgroup per walker:
//   * the Green's function (eq. green) in scale-split form: A = X^T, R = U^T with
//     partial pivoting and back substitution, so R becomes X^{-T} U^T;
//   * the Cholesky factor of S = Y^H Y for the QR stabilisation: without pivoting
//     and without back substitution, the left block becomes U = D L^H (S = L D L^H)
//     and R becomes L^{-1} R;
//   * the update of T^{-1} by a unit triangular factor (again forward only).
// Right-looking, NB = 16 columns per panel.  The panel lives in registers, one row
// per thread (two when M > 256), so the pivot search, the row exchange and the
// rank-1 updates of the panel need only LDS broadcasts.  Row exchanges are
// applied to the trailing columns and the right-hand sides (the multipliers of
// earlier panels are never read again).  The trailing update stages 16 x 64 blocks
// of L21 and U12 in LDS and keeps a 4 x 4 complex register tile per thread.
// ln det of the left block is the sum of the logs of the pivots plus i pi per swap.
#include "common.h"
#include "kernels.h"
#include <climits>

namespace {

constexpr int NB = 16, NT = 256, UT = 64;

struct ElimShared {
  double2 bufP[NB];
  double2 bufC[NB];
  double2 L11[NB][NB + 1];
  double2 Ls[NB][UT + 1];
  double2 Us[NB][UT + 1];
  double redv[4];
  int redi[4];
  int swp[NB];
};

FT_DEV int phys_col(int lc, int c_begin, int nc1, int rhs_off) {
  return lc < nc1 ? c_begin + lc : rhs_off + (lc - nc1);
}

// aug[r][pc] -= sum_{k<kb} aug[r][k0+k] aug[k0+k][pc] for r in [r_lo, r_hi) and the
// logical columns [0, ncols) (first nc1 map to c_begin.., the rest to rhs_off..).
FT_DEV void block_update(double2* aug, int lda, int r_lo, int r_hi, int k0, int kb,
                         int c_begin, int nc1, int rhs_off, int ncols, ElimShared& sh) {
  const int t = threadIdx.x;
  if (r_hi <= r_lo || ncols <= 0) return;
  const int nrt = (r_hi - r_lo + UT - 1) / UT, nct = (ncols + UT - 1) / UT;
  const int tr = t >> 4, tc = t & 15;
  for (int tile = 0; tile < nrt * nct; ++tile) {
    const int rt = tile / nct, ct = tile - rt * nct;
    const int rb = r_lo + rt * UT, cb = ct * UT;
    for (int e = t; e < NB * UT; e += NT) {
      const int x = e / NB, k = e - x * NB;          // Ls: row x of the tile, column k
      const int r = rb + x;
      sh.Ls[k][x] = (k < kb && r < r_hi) ? aug[(long long)r * lda + k0 + k] : make_double2(0.0, 0.0);
      const int k2 = e / UT, x2 = e - k2 * UT;       // Us: row k2, tile column x2
      const int lc = cb + x2;
      sh.Us[k2][x2] = (k2 < kb && lc < ncols)
                          ? aug[(long long)(k0 + k2) * lda + phys_col(lc, c_begin, nc1, rhs_off)]
                          : make_double2(0.0, 0.0);
    }
    __syncthreads();
    double2 acc[4][4];
    int pc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int lc = cb + tc * 4 + j;
      pc[j] = lc < ncols ? phys_col(lc, c_begin, nc1, rhs_off) : -1;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = rb + tr * 4 + i;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j] = (r < r_hi && pc[j] >= 0) ? aug[(long long)r * lda + pc[j]] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      double2 l[4], u[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) l[i] = sh.Ls[k][tr * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) u[j] = sh.Us[k][tc * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = cfnms(acc[i][j], l[i], u[j]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = rb + tr * 4 + i;
      if (r >= r_hi) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (pc[j] >= 0) aug[(long long)r * lda + pc[j]] = acc[i][j];
    }
    __syncthreads();
  }
}

template <int RPT>
__global__ __launch_bounds__(NT) void elim_kernel(ElimParams p) {
  __shared__ ElimShared sh;
  const int w = blockIdx.x;
  if (w >= p.W) return;
  double2* aug = p.aug + (long long)w * p.stride;
  const int M = p.M, lda = p.lda, t = threadIdx.x, lane = t & 63, wid = t >> 6;
  double2 lsum = make_double2(0.0, 0.0);
  int nswaps = 0;
  bool bad = false;

  for (int j0 = 0; j0 < M; j0 += NB) {
    const int jb = min(NB, M - j0);
    double2 a[RPT][NB];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = j0 + t + q * NT;
#pragma unroll
      for (int c = 0; c < NB; ++c)
        a[q][c] = (r < M && c < jb) ? aug[(long long)r * lda + j0 + c] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      if (c >= jb) break;
      const int col = j0 + c;
      int prow = col;
      if (p.pivot) {
        double bv = -1.0;
        int bi = INT_MAX;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const int r = j0 + t + q * NT;
          if (r >= col && r < M) {
            const double v = cabs2(a[q][c]);
            if (v > bv || (v == bv && r < bi)) { bv = v; bi = r; }
          }
        }
        for (int o = 32; o > 0; o >>= 1) {
          const double ov = __shfl_xor(bv, o, 64);
          const int oi = __shfl_xor(bi, o, 64);
          if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        }
        if (lane == 0) { sh.redv[wid] = bv; sh.redi[wid] = bi; }
        __syncthreads();
        bv = sh.redv[0]; bi = sh.redi[0];
#pragma unroll
        for (int k = 1; k < 4; ++k)
          if (sh.redv[k] > bv || (sh.redv[k] == bv && sh.redi[k] < bi)) { bv = sh.redv[k]; bi = sh.redi[k]; }
        prow = (bi >= col && bi < M) ? bi : col;   // all-NaN column: keep the diagonal
      }
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int r = j0 + t + q * NT;
        if (r == prow) {
#pragma unroll
          for (int c2 = 0; c2 < NB; ++c2) sh.bufP[c2] = a[q][c2];
        }
        if (prow != col && r == col) {
#pragma unroll
          for (int c2 = 0; c2 < NB; ++c2) sh.bufC[c2] = a[q][c2];
        }
      }
      __syncthreads();
      if (prow != col) {
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const int r = j0 + t + q * NT;
          if (r == prow) {
#pragma unroll
            for (int c2 = 0; c2 < NB; ++c2) a[q][c2] = sh.bufC[c2];
          }
          if (r == col) {
#pragma unroll
            for (int c2 = 0; c2 < NB; ++c2) a[q][c2] = sh.bufP[c2];
          }
        }
      }
      const double2 piv = sh.bufP[c];
      if (t == 0) {
        sh.swp[c] = prow;
        if (!(cabs2(piv) > 0.0) || !isfinite(piv.x) || !isfinite(piv.y)) bad = true;
        const double2 lg = clog(piv);
        lsum.x += lg.x;
        lsum.y += lg.y;
        if (prow != col) ++nswaps;
      }
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int r = j0 + t + q * NT;
        if (r > col && r < M) {
          const double2 l = cdiv(a[q][c], piv);
          a[q][c] = l;
#pragma unroll
          for (int c2 = 0; c2 < NB; ++c2)
            if (c2 > c) a[q][c2] = cfnms(a[q][c2], l, sh.bufP[c2]);
        }
      }
      __syncthreads();
    }
    // panel back to memory; unit-lower L11 into LDS
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = j0 + t + q * NT;
      if (r < M) {
#pragma unroll
        for (int c = 0; c < NB; ++c)
          if (c < jb) aug[(long long)r * lda + j0 + c] = a[q][c];
      }
    }
    if (t < NB) {
#pragma unroll
      for (int c = 0; c < NB; ++c) sh.L11[t][c] = (t < jb) ? a[0][c] : make_double2(0.0, 0.0);
    }
    __syncthreads();

    const int nc1 = M - j0 - jb, ncols = nc1 + p.nrhs, cbeg = j0 + jb;
    // row exchanges and U12 = L11^{-1} A12 on the trailing columns and the right-hand sides
    for (int lc = t; lc < ncols; lc += NT) {
      const int pc = phys_col(lc, cbeg, nc1, p.rhs_off);
      for (int c = 0; c < jb; ++c) {
        const int pr = sh.swp[c];
        if (pr != j0 + c) {
          const double2 u = aug[(long long)(j0 + c) * lda + pc];
          aug[(long long)(j0 + c) * lda + pc] = aug[(long long)pr * lda + pc];
          aug[(long long)pr * lda + pc] = u;
        }
      }
      double2 x[NB];
#pragma unroll
      for (int i = 0; i < NB; ++i) x[i] = i < jb ? aug[(long long)(j0 + i) * lda + pc] : make_double2(0.0, 0.0);
#pragma unroll
      for (int i = 1; i < NB; ++i)
#pragma unroll
        for (int m = 0; m < NB; ++m)
          if (m < i) x[i] = cfnms(x[i], sh.L11[i][m], x[m]);
#pragma unroll
      for (int i = 0; i < NB; ++i)
        if (i < jb) aug[(long long)(j0 + i) * lda + pc] = x[i];
    }
    __syncthreads();
    block_update(aug, lda, j0 + jb, M, j0, jb, cbeg, nc1, p.rhs_off, ncols, sh);
    __syncthreads();
  }

  if (p.backsub) {
    for (int i0 = ((M - 1) / NB) * NB; i0 >= 0; i0 -= NB) {
      const int ib = min(NB, M - i0);
      for (int e = t; e < NB * NB; e += NT) {
        const int i = e / NB, m = e - i * NB;
        sh.L11[i][m] = (i < ib && m < ib) ? aug[(long long)(i0 + i) * lda + i0 + m] : make_double2(0.0, 0.0);
      }
      __syncthreads();
      for (int lc = t; lc < p.nrhs; lc += NT) {
        const int pc = p.rhs_off + lc;
        double2 x[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) x[i] = i < ib ? aug[(long long)(i0 + i) * lda + pc] : make_double2(0.0, 0.0);
#pragma unroll
        for (int i = NB - 1; i >= 0; --i) {
          if (i < ib) {
#pragma unroll
            for (int m = 0; m < NB; ++m)
              if (m > i) x[i] = cfnms(x[i], sh.L11[i][m], x[m]);
            x[i] = cdiv(x[i], sh.L11[i][i]);
          }
        }
#pragma unroll
        for (int i = 0; i < NB; ++i)
          if (i < ib) aug[(long long)(i0 + i) * lda + pc] = x[i];
      }
      __syncthreads();
      if (i0 > 0) block_update(aug, lda, 0, i0, i0, ib, 0, 0, p.rhs_off, p.nrhs, sh);
      __syncthreads();
    }
  }

  if (t == 0) {
    if (p.lndet) p.lndet[w] = make_double2(lsum.x, lsum.y + 3.14159265358979323846 * (double)nswaps);
    if (bad && p.status) p.status[w] = 2;
  }
}

}  // namespace

hipError_t launch_elim(const ElimParams& p, hipStream_t s) {
  if (p.W <= 0 || p.M <= 0) return hipSuccess;
  if (p.M <= NT) elim_kernel<1><<<p.W, NT, 0, s>>>(p);
  else if (p.M <= 2 * NT) elim_kernel<2><<<p.W, NT, 0, s>>>(p);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}
