// Frozen-path derivatives of the weight and the local energy in mu and the kinetic scale lambda.
//
// With the sampled path (the shifted coefficients c_Q of every slice) held fixed, mu and lambda
// enter only through the half-step factors K = exp(-dtau/2 (lambda eps + h - mu)) of every
// B_k = K e^{V_k} K (eq. B) and through the kinetic term of the local energy.
//   * mu: K carries e^{dtau mu/2} on both sides, so A_k = B_T^{n-k} B_k..B_1 scales as
//     e^{k dtau mu}: d ln det(I + A_k) = k dtau tr(I - G_k), dG_n = -beta (I - G_n) G_n.
//   * lambda: dB_ij = -dtau/2 (eps_i + eps_j) B_ij does not commute with the path.  The product
//     and its derivative are carried together as the doubled product
//     Rd = [[R, dR], [0, R]] = Yd diag(Dd) Td, re-factorised by the pre-pivoted Cholesky-QR
//     every slice.  The ratio of the step that inserts B_{k+1} is the M x M determinant
//     det(I + Phi), Phi = (B B_T^{-1} - I)(I - Gc), with the cyclic Green's function
//     Gc = (I + B_T R_k B_T^{n-k-1})^{-1}; its derivative uses the off-diagonal block of the
//     doubled Gc.  At tau = beta, dG_n is the off-diagonal block of (I + Rd)^{-1}.
// Both doubled inverses are taken transposed, in the left-graded form of the forward path:
//   Gc^T = (I + L Td^T Dd (Yd^T B_T))^{-1}, Yd unitary right after the re-factorisation, so
//   Gc = L_b Z with X'^T Z = D_b Yd^H B_T^{-1},  X'^T = D_b Yd^H B_T^{-1} L_b + D_s Td L_s
// (L = B_T^{n-k-1}; at tau = beta L = B_T = I).
#include "common.h"
#include "kernels.h"

namespace {

constexpr int NT = 256;
constexpr int TT = 32;
constexpr double PI = 3.14159265358979323846;

FT_DEV double2 zero2() { return make_double2(0.0, 0.0); }

FT_DEV void split_val(double lnv, double* b, double* s) {   // v = e^lnv = s / b, b = 1/max(1,v)
  *b = exp(-fmax(lnv, 0.0));
  *s = exp(fmin(lnv, 0.0));
}
FT_DEV void split_D(double d, double* db, double* ds) {
  const double a = fabs(d);
  if (a > 1.0) { *db = 1.0 / a; *ds = d / a; }
  else { *db = 1.0; *ds = d; }
}

// V[w] from the recorded coefficients of slice k (the gather of the forward path).
constexpr int RV_ROWS = 16;               // rows of V per workgroup
__global__ __launch_bounds__(NT) void coef_replay_kernel(SysDev s, int k, int chunks) {
  int w, ch;
  if (!xcd_walker_tile(blockIdx.x, s.W, chunks, &w, &ch)) return;
  const double2* c = s.rec_c + ((long long)w * s.n + k) * s.NQ;
  double2* Vw = (double2*)s.V + (long long)w * s.mat_stride;
  const int ld = s.ld, M = s.M, i0 = ch * RV_ROWS;
  for (int e = threadIdx.x; e < RV_ROWS * ld; e += NT) {
    const int i = i0 + e / ld, j = e - (e / ld) * ld;
    if (i >= ld) break;
    double2 v = zero2();
    if (i < M && j < M && i != j) v = c[s.idx[i * M + j]];
    Vw[(long long)i * ld + j] = v;
  }
}

// Yd = I, Td = I, Dd = 1, derivative accumulators cleared.
__global__ __launch_bounds__(NT) void tan_init_kernel(SysDev s, TanDev t) {
  const long long mat = (long long)t.ld2 * t.ld2;
  const long long total = (long long)s.W * mat;
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < total; e += (long long)gridDim.x * NT) {
    const long long loc = e % mat;
    const int i = (int)(loc / t.ld2), j = (int)(loc % t.ld2);
    const double2 v = (i == j && i < t.M2) ? make_double2(1.0, 0.0) : zero2();
    t.dd.Y[e] = v;
    t.Td[e] = v;
  }
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < (long long)s.W * t.ld2; e += (long long)gridDim.x * NT)
    t.dd.D[e] = ((int)(e % t.ld2) < t.M2) ? 1.0 : 0.0;
  for (long long w = (long long)blockIdx.x * NT + threadIdx.x; w < s.W; w += (long long)gridDim.x * NT) {
    t.dlnw[2 * w] = 0.0;
    t.dlnw[2 * w + 1] = 0.0;
    t.alive[w] = 1;
    t.tstat[w] = 0;
    t.lndet_dummy[w] = zero2();
  }
}

// Bcat = [B | dB], Fcat = [dB B_T^{-1} | B B_T^{-1} - I] with dB_ij = -dtau/2 (eps_i + eps_j) B_ij.
__global__ __launch_bounds__(NT) void tan_prep_kernel(SysDev s, TanDev t, const double2* B) {
  const long long per = (long long)s.ld * t.ld2;
  const long long total = (long long)s.W * per;
  const int M = s.M;
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < total; e += (long long)gridDim.x * NT) {
    const long long w = e / per;
    const int loc = (int)(e - w * per);
    const int i = loc / t.ld2, c = loc - i * t.ld2;
    double2 bc = zero2(), fc = zero2();
    if (i < M && c < 2 * M) {
      const int j = c < M ? c : c - M;
      const double2 b = B[w * s.mat_stride + (long long)i * s.ld + j];
      const double btinv = exp(-s.lnbt[j]);
      const double2 db = cscale(b, -0.5 * s.dtau * (s.eps[i] + s.eps[j]));
      if (c < M) { bc = b; fc = cscale(db, btinv); }
      else { bc = db; fc = cscale(b, btinv); if (i == j) fc.x -= 1.0; }
    }
    t.Bcat[e] = bc;
    t.Fcat[e] = fc;
  }
}

// Doubled augmented system [X'^T | D_b Yd^H B_T^{-1}] (see the header comment), through LDS tiles.
// literal = 1: the Green's function at tau = beta, L = B_T = I.
__global__ __launch_bounds__(NT) void cyc_form_kernel(SysDev s, TanDev t, int k, int literal) {
  __shared__ double2 tY[TT][TT + 1];
  const int ld2 = t.ld2, M2 = t.M2, M = s.M;
  const int nt = (ld2 + TT - 1) / TT;
  int w, tile;
  if (!xcd_walker_tile(blockIdx.x, s.W, nt * nt, &w, &tile)) return;
  const int ti = tile / nt, tj = tile - ti * nt;   // aug rows ti.., cols tj..
  const double2* Y = t.dd.Y + (long long)w * t.dd.mat_stride;
  const double2* T = t.Td + (long long)w * t.dd.mat_stride;
  const double* D = t.dd.D + (long long)w * ld2;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int yy = ty; yy < TT; yy += 8) {
    const int row = tj * TT + yy, col = ti * TT + tx;   // Yd[row = j][col = i]
    tY[yy][tx] = (row < M2 && col < M2) ? Y[(long long)row * ld2 + col] : zero2();
  }
  __syncthreads();
  double2* aug = t.caug + (long long)w * t.dd.aug_stride;
  for (int yy = ty; yy < TT; yy += 8) {
    const int i = ti * TT + yy, j = tj * TT + tx;
    if (i >= ld2 || j >= ld2) continue;
    double2 left = zero2(), right = zero2();
    if (i < M2 && j < M2) {
      const int jj = j < M ? j : j - M;
      double lb = 1.0, ls = 1.0, btinv = 1.0;
      if (!literal) {
        split_val((double)(s.n - k - 1) * s.lnbt[jj], &lb, &ls);
        btinv = exp(-s.lnbt[jj]);
      }
      double db, ds;
      split_D(D[i], &db, &ds);
      const double2 yc = cconj(tY[tx][yy]);          // conj(Yd[j][i])
      right = cscale(yc, db * btinv);
      const double2 tv = T[(long long)i * ld2 + j];
      left = make_double2(right.x * lb + ds * ls * tv.x, right.y * lb + ds * ls * tv.y);
    }
    aug[(long long)i * 2 * ld2 + j] = left;
    aug[(long long)i * 2 * ld2 + ld2 + j] = right;
  }
}

// After the elimination, Z = aug right block and Gc = L_b Z.
// literal = 0: Gst[r][j] = Gc[r][j] (r < M), Gc[r - M][M + j] (M <= r < 2M), j < M.
// literal = 1: dG (lambda slot)[i][j] = Gd[i][M + j].
__global__ __launch_bounds__(NT) void cyc_post_kernel(SysDev s, TanDev t, int k, int literal) {
  const int M = s.M, ld = s.ld, ld2 = t.ld2;
  const long long per = literal ? (long long)ld * ld : (long long)ld2 * ld;
  const long long total = (long long)s.W * per;
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < total; e += (long long)gridDim.x * NT) {
    const long long w = e / per;
    const int loc = (int)(e - w * per);
    const int r = loc / ld, j = loc - r * ld;
    const double2* Z = t.caug + w * t.dd.aug_stride + ld2;     // Z[i][c] at i * 2 ld2 + c
    double2 v = zero2();
    if (literal) {
      if (r < M && j < M) v = Z[(long long)r * 2 * ld2 + M + j];
      t.dG[(long long)s.W * ld * ld + e] = v;
    } else {
      if (r < 2 * M && j < M) {
        const int i = r < M ? r : r - M;
        const int c = r < M ? j : M + j;
        double lb, ls;
        split_val((double)(s.n - k - 1) * s.lnbt[i], &lb, &ls);
        v = cscale(Z[(long long)i * 2 * ld2 + c], lb);
      }
      t.Gst[e] = v;
    }
  }
}

// d ln S_k along lambda = 2 tr((I + Phi)^{-1} dPhi) (aug right block after the solve) and along
// mu from the recorded traces; d ln w += Re d ln S - tan(theta_k) Im d ln S while the walker
// survives the slice (the forward kills it when cos theta_k <= 0).
__global__ __launch_bounds__(NT) void tan_weight_kernel(SysDev s, TanDev t, int k) {
  __shared__ double red[8];
  const int w = blockIdx.x;
  if (w >= s.W) return;
  const double2* aug = s.aug + (long long)w * s.aug_stride;
  double2 tr = zero2();
  for (int i = threadIdx.x; i < s.M; i += NT) tr = cadd(tr, aug[(long long)i * 2 * s.ld + s.ld + i]);
  tr = block_csum_256(tr, red);
  if (threadIdx.x != 0 || !t.alive[w]) return;
  const double th = s.slice_theta[(long long)w * s.n + k];
  const double cth = cos(th);
  const double2 g0 = s.rec_trG[(long long)w * (s.n + 1) + k], g1 = s.rec_trG[(long long)w * (s.n + 1) + k + 1];
  // d ln det(I + A_j)/dmu = j dtau (M - tr G_j)
  const double2 dmu = make_double2(2.0 * s.dtau * ((k + 1) * (s.M - g1.x) - k * (s.M - g0.x)),
                                   2.0 * s.dtau * (-(k + 1) * g1.y + k * g0.y));
  const double2 dlam = cscale(tr, 2.0);
  if (!(cth > 0.0) || !isfinite(dlam.x) || !isfinite(dlam.y)) { t.alive[w] = 0; return; }
  const double tn = tan(th);
  t.dlnw[2 * w] += dmu.x - tn * dmu.y;
  t.dlnw[2 * w + 1] += dlam.x - tn * dlam.y;
}

// dd.E0 = Td[perm[i], :] (the row order of the new triangular factor)
__global__ __launch_bounds__(NT) void permute_rows_kernel(TanDev t) {
  const long long mat = t.dd.mat_stride;
  const long long total = (long long)t.dd.W * mat;
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < total; e += (long long)gridDim.x * NT) {
    const long long w = e / mat;
    const int loc = (int)(e - w * mat);
    const int i = loc / t.ld2, j = loc - i * t.ld2;
    double2 v = zero2();
    if (i < t.M2) v = t.Td[w * mat + (long long)t.dd.perm[w * t.ld2 + i] * t.ld2 + j];
    ((double2*)t.dd.E0)[e] = v;
  }
}

// Exchange part of the energy derivative: sum_{a != d} v(K_a - K_d) sum_b (dP_ab P_cd + P_ab dP_cd)
// with K_c = K_b - K_a + K_d, P = I - G^T, dP = -dG^T.  One workgroup per (walker, a).
__global__ __launch_bounds__(NT) void exchange_tangent_kernel(SysDev s, TanDev t, int dir) {
  extern __shared__ char dyn[];
  double2* pcol = (double2*)dyn;                    // [M] P_ab
  double2* dcol = pcol + s.M;                       // [M] dP_ab
  short* grid = (short*)(dcol + s.M);
  __shared__ double red[8];
  int w, a;
  if (!xcd_walker_tile(blockIdx.x, s.W, s.M, &w, &a)) return;
  const int M = s.M, ld = s.ld;
  const double2* G = s.G + (long long)w * s.mat_stride;
  const double2* dG = t.dG + ((long long)dir * s.W + w) * s.mat_stride;
  const int g3 = s.grid_dim * s.grid_dim * s.grid_dim;
  for (int e = threadIdx.x; e < g3; e += NT) grid[e] = s.grid[e];
  for (int b = threadIdx.x; b < M; b += NT) {
    double2 v = cscale(G[(long long)b * ld + a], -1.0);
    if (b == a) v.x += 1.0;
    pcol[b] = v;
    dcol[b] = cscale(dG[(long long)b * ld + a], -1.0);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double2 acc = zero2();
  for (int d = wid; d < M; d += 4) {
    if (d == a) continue;
    const double v = s.vq[s.idx[a * M + d]];
    const double2* Gd = G + (long long)d * ld;
    const double2* dGd = dG + (long long)d * ld;
    const int off = s.flat[d] - s.flat[a] + s.grid_c0;
    double2 part = zero2();
    for (int b = lane; b < M; b += 64) {
      const int c = grid[s.flat[b] + off];
      if (c >= 0) {
        double2 pcd = cscale(Gd[c], -1.0);
        if (c == d) pcd.x += 1.0;
        const double2 dpcd = cscale(dGd[c], -1.0);
        part = cadd(part, cadd(cmul(dcol[b], pcd), cmul(pcol[b], dpcd)));
      }
    }
    acc.x += v * part.x;
    acc.y += v * part.y;
  }
  acc = block_csum_256(acc, red);
  if (threadIdx.x == 0) t.exch[(long long)w * ld + a] = acc;
}

// dE1 = 2 lambda sum eps dP_KK (+ 2 sum eps P_KK along lambda), dN = 2 sum dP_KK,
// dE2 = 2 sum_Q v_Q (dr_Q r_-Q + r_Q dr_-Q) - (exchange part), dr_Q = -sum over pairs dG_rp.
__global__ __launch_bounds__(NT) void energy_tangent_kernel(SysDev s, TanDev t, int dir) {
  extern __shared__ double2 drs[];                 // [NQ]
  __shared__ double red[8];
  const int w = blockIdx.x;
  if (w >= s.W) return;
  const double2* G = s.G + (long long)w * s.mat_stride;
  const double2* dG = t.dG + ((long long)dir * s.W + w) * s.mat_stride;
  const double2* r = s.r + (long long)w * s.NQ;
  for (int q = threadIdx.x; q < s.NQ; q += NT) {
    double2 acc = zero2();
    for (int e = s.qptr[q]; e < s.qptr[q + 1]; ++e) acc = csub(acc, dG[s.qpair[e]]);
    drs[q] = acc;
  }
  __syncthreads();
  double2 de1 = zero2(), dn = zero2(), e1x = zero2(), hart = zero2(), ex = zero2();
  for (int i = threadIdx.x; i < s.M; i += NT) {
    const double2 g = G[(long long)i * s.ld + i];
    const double2 dpkk = cscale(dG[(long long)i * s.ld + i], -1.0);
    de1 = cadd(de1, cscale(dpkk, s.eps[i]));
    dn = cadd(dn, dpkk);
    e1x = cadd(e1x, cscale(make_double2(1.0 - g.x, -g.y), s.eps[i]));
    ex = cadd(ex, t.exch[(long long)w * s.ld + i]);
  }
  for (int q = threadIdx.x; q < s.NQ; q += NT) {
    const int nq = s.neg[q];
    hart = cadd(hart, cscale(cadd(cmul(drs[q], r[nq]), cmul(r[q], drs[nq])), s.vq[q]));
  }
  de1 = block_csum_256(de1, red);
  dn = block_csum_256(dn, red);
  e1x = block_csum_256(e1x, red);
  hart = block_csum_256(hart, red);
  ex = block_csum_256(ex, red);
  if (threadIdx.x != 0) return;
  double2 dE1 = cscale(de1, 2.0 * s.kscale);
  if (dir == 1) dE1 = cadd(dE1, cscale(e1x, 2.0));
  const double2 dE2 = csub(cscale(hart, 2.0), ex);
  double2* out = t.dloc + ((long long)w * 2 + dir) * 4;
  out[0] = dE1;
  out[1] = dE2;
  out[2] = cadd(dE1, dE2);
  out[3] = cscale(dn, 2.0);
}

// Weighted means over live walkers and their derivatives:
// d<O> = sum_w f_w (dO_w + (O_w - <O>) d ln w_w) / sum_w f_w, f_w = e^{ln w_w - max}.
// jac = (d<E>/dmu, d<N>/dmu, d<E>/dlambda, d<N>/dlambda); grad = cot . Re(jac) per parameter;
// walker[w] = (d ln w, dE, dN) along mu then lambda (NaN where a doubled factorisation failed).
__global__ __launch_bounds__(NT) void tan_mean_kernel(SysDev s, TanDev t, const double* cot, double2* jac,
                                                      double* grad, double2* walker) {
  __shared__ double red[8];
  __shared__ double mxs[4];
  __shared__ double2 means[2];
  const int W = s.W;
  auto live = [&](int w) { return s.status[w] == 0 && isfinite(s.logw[w]); };
  double mx = -INFINITY;
  for (int w = threadIdx.x; w < W; w += NT)
    if (live(w)) mx = fmax(mx, s.logw[w]);
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  if ((threadIdx.x & 63) == 0) mxs[threadIdx.x >> 6] = mx;
  __syncthreads();
  mx = fmax(fmax(mxs[0], mxs[1]), fmax(mxs[2], mxs[3]));
  double ws = 0.0;
  double2 sE = zero2(), sN = zero2();
  for (int w = threadIdx.x; w < W; w += NT) {
    if (!live(w)) continue;
    const double f = exp(s.logw[w] - mx);
    ws += f;
    sE = cadd(sE, cscale(s.local[(long long)w * 4 + 2], f));
    sN = cadd(sN, cscale(s.local[(long long)w * 4 + 3], f));
  }
  ws = block_sum_256(ws, red);
  sE = block_csum_256(sE, red);
  sN = block_csum_256(sN, red);
  if (threadIdx.x == 0) { means[0] = cscale(sE, 1.0 / ws); means[1] = cscale(sN, 1.0 / ws); }
  __syncthreads();
  const double2 mE = means[0], mN = means[1];
  double2 acc[4] = {zero2(), zero2(), zero2(), zero2()};
  for (int w = threadIdx.x; w < W; w += NT) {
    const bool bad = t.tstat[w] != 0;
    if (walker) {
      for (int dir = 0; dir < 2; ++dir) {
        const double2* dl = t.dloc + ((long long)w * 2 + dir) * 4;
        double2* o = walker + (long long)w * 6 + 3 * dir;
        o[0] = bad ? make_double2(NAN, NAN) : make_double2(t.dlnw[2 * w + dir], 0.0);
        o[1] = bad ? make_double2(NAN, NAN) : dl[2];
        o[2] = bad ? make_double2(NAN, NAN) : dl[3];
      }
    }
    if (!live(w)) continue;
    const double f = exp(s.logw[w] - mx);
    const double2 E = s.local[(long long)w * 4 + 2], N = s.local[(long long)w * 4 + 3];
    for (int dir = 0; dir < 2; ++dir) {
      const double2* dl = t.dloc + ((long long)w * 2 + dir) * 4;
      const double dlw = bad ? NAN : t.dlnw[2 * w + dir];
      acc[2 * dir] = cadd(acc[2 * dir], cscale(cadd(dl[2], cscale(csub(E, mE), dlw)), f));
      acc[2 * dir + 1] = cadd(acc[2 * dir + 1], cscale(cadd(dl[3], cscale(csub(N, mN), dlw)), f));
    }
  }
  for (int c = 0; c < 4; ++c) acc[c] = block_csum_256(acc[c], red);
  if (threadIdx.x != 0) return;
  double2 j[4];
  for (int c = 0; c < 4; ++c) j[c] = ws > 0.0 ? cscale(acc[c], 1.0 / ws) : make_double2(NAN, NAN);
  if (jac)
    for (int c = 0; c < 4; ++c) jac[c] = j[c];
  if (grad && cot) {
    grad[0] = cot[0] * j[0].x + cot[1] * j[1].x;
    grad[1] = cot[0] * j[2].x + cot[1] * j[3].x;
  }
}

// ------------------------------------------------------------ pathwise ---
// Raw fields held fixed while mu or lambda moves: the force bias of every slice follows G_k, so
// V_k, e^{V_k} (Frechet derivative), B_k and the exponent of eq. import move too.  One pass per
// direction carries the doubled product with its inverse triangular factor Tid (so that the
// literal doubled Green's function (I + diag(L, L) Rd)^{-1} at every slice comes from the forward
// path's own scale-split solve), whose blocks are G_k and dG_k.

__global__ __launch_bounds__(NT) void pw_reset_kernel(SysDev s, TanDev t) {
  const long long mat = (long long)t.ld2 * t.ld2;
  const long long total = (long long)s.W * mat;
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < total; e += (long long)gridDim.x * NT) {
    const long long loc = e % mat;
    const int i = (int)(loc / t.ld2), j = (int)(loc % t.ld2);
    const double2 v = (i == j && i < t.M2) ? make_double2(1.0, 0.0) : zero2();
    t.dd.Y[e] = v;
    t.Td[e] = v;
    t.Tid[e] = v;
  }
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < (long long)s.W * t.ld2; e += (long long)gridDim.x * NT)
    t.dd.D[e] = ((int)(e % t.ld2) < t.M2) ? 1.0 : 0.0;
  for (long long w = (long long)blockIdx.x * NT + threadIdx.x; w < s.W; w += (long long)gridDim.x * NT) {
    t.alive[w] = 1;
    t.lndet_dummy[w] = zero2();
  }
}

// Gk = Gd[:M, :M], dGk = Gd[:M, M:2M] (and dG_out = dGk when given)
__global__ __launch_bounds__(NT) void pw_extract_kernel(SysDev s, TanDev t, double2* dG_out) {
  const long long per = (long long)s.ld * s.ld;
  const long long total = (long long)s.W * per;
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < total; e += (long long)gridDim.x * NT) {
    const long long w = e / per;
    const int loc = (int)(e - w * per);
    const int i = loc / s.ld, j = loc - i * s.ld;
    double2 g = zero2(), dg = zero2();
    if (i < s.M && j < s.M) {
      const double2* Gd = t.Gd + w * t.dd.mat_stride + (long long)i * t.ld2;
      g = Gd[j];
      dg = Gd[s.M + j];
    }
    t.Gk[e] = g;
    t.dGk[e] = dg;
    if (dG_out) dG_out[e] = dg;
  }
}

// dc_Q = -2 dtau v_Q dr_-Q (the derivative of c_Q = i s_Q (z_Q + conj z_-Q) - 2 dtau v_Q r_-Q) and
// d(exponent) = sum_Q (x_A - xbar_A) dxbar_A + (x_B - xbar_B) dxbar_B with
// xbar_A = -2i s_Q (r_Q + r_-Q), xbar_B = 2 s_Q (r_Q - r_-Q) and their derivatives in dr.
__global__ __launch_bounds__(NT) void pw_coef_kernel(SysDev s, TanDev t, const double2* fields, int k) {
  __shared__ double red[8];
  const int w = blockIdx.x;
  if (w >= s.W) return;
  const double2* z = fields + ((long long)w * s.n + k) * s.NQ;
  const double2* r = t.rk + (long long)w * s.NQ;
  const double2* dr = t.drk + (long long)w * s.NQ;
  double2 acc = zero2();
  for (int q = threadIdx.x; q < s.NQ; q += NT) {
    const int nq = s.neg[q];
    const double sqv = s.sq[q];
    const double2 rq = r[q], rn = r[nq], dq = dr[q], dn = dr[nq], zq = z[q];
    t.dcq[(long long)w * s.NQ + q] = cscale(dn, -2.0 * s.dtau * s.vq[q]);
    const double2 sp = cadd(rq, rn), sm = csub(rq, rn), dsp = cadd(dq, dn), dsm = csub(dq, dn);
    const double2 xa = make_double2(2.0 * sqv * sp.y, -2.0 * sqv * sp.x);      // -2i s (r_q + r_-q)
    const double2 xb = cscale(sm, 2.0 * sqv);
    const double2 dxa = make_double2(2.0 * sqv * dsp.y, -2.0 * sqv * dsp.x);
    const double2 dxb = cscale(dsm, 2.0 * sqv);
    const double2 ua = make_double2(zq.x - xa.x, -xa.y), ub = make_double2(zq.y - xb.x, -xb.y);
    acc = cadd(acc, cadd(cmul(ua, dxa), cmul(ub, dxb)));
  }
  acc = block_csum_256(acc, red);
  if (threadIdx.x == 0) t.dexpo[w] = acc;
}

// dB_k = c[k][1] dV + c[k][2] dV2 + c[k][3] dV3 for k < nb - 1 (into dBk[k]); the top term
// c[nb-1][0] dV4 + c[nb-1][1] dV + c[nb-1][2] dV2 + c[nb-1][3] dV3 into dE0.
__global__ __launch_bounds__(NT) void pw_blocks_kernel(SysDev s, TanDev t, PwBlocks b) {
  const long long total = (long long)s.W * s.mat_stride;
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < total; e += (long long)gridDim.x * NT) {
    const double2 v1 = t.dV[e], v2 = t.dV2[e], v3 = t.dV3[e], v4 = t.dV4[e];
    for (int k = 0; k < b.nb; ++k) {
      double2 x = cadd(cscale(v1, b.c[k][1]), cadd(cscale(v2, b.c[k][2]), cscale(v3, b.c[k][3])));
      if (k == b.nb - 1) t.dE0[e] = cadd(x, cscale(v4, b.c[k][0]));
      else t.dBk[k][e] = x;
    }
  }
}

// Bcat = [B | dB], Fcat = [dB B_T^{-1} | B B_T^{-1} - I] with dB = K dE K + dK E K + K E dK:
// along mu (dir 0) dK = dtau/2 K, along lambda (dir 1) dK = -dtau/2 eps K.
__global__ __launch_bounds__(NT) void pw_prep_kernel(SysDev s, TanDev t, const double2* B, const double2* KdEK, int dir) {
  const long long per = (long long)s.ld * t.ld2;
  const long long total = (long long)s.W * per;
  const int M = s.M;
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < total; e += (long long)gridDim.x * NT) {
    const long long w = e / per;
    const int loc = (int)(e - w * per);
    const int i = loc / t.ld2, c = loc - i * t.ld2;
    double2 bc = zero2(), fc = zero2();
    if (i < M && c < 2 * M) {
      const int j = c < M ? c : c - M;
      const long long o = w * s.mat_stride + (long long)i * s.ld + j;
      const double2 b = B[o];
      const double btinv = exp(-s.lnbt[j]);
      const double f = dir == 0 ? s.dtau : -0.5 * s.dtau * (s.eps[i] + s.eps[j]);
      const double2 db = cadd(cscale(b, f), KdEK[o]);
      if (c < M) { bc = b; fc = cscale(db, btinv); }
      else { bc = db; fc = cscale(b, btinv); if (i == j) fc.x -= 1.0; }
    }
    t.Bcat[e] = bc;
    t.Fcat[e] = fc;
  }
}

// d ln S_k = 2 tr((I + Phi)^{-1} dPhi) from the solve; d ln w (direction dir) +=
// Re d ln S + Re d(exponent) - tan(theta_k) Im d ln S while the walker survives the slice.
__global__ __launch_bounds__(NT) void pw_weight_kernel(SysDev s, TanDev t, int k, int dir) {
  __shared__ double red[8];
  const int w = blockIdx.x;
  if (w >= s.W) return;
  const double2* aug = s.aug + (long long)w * s.aug_stride;
  double2 tr = zero2();
  for (int i = threadIdx.x; i < s.M; i += NT) tr = cadd(tr, aug[(long long)i * 2 * s.ld + s.ld + i]);
  tr = block_csum_256(tr, red);
  if (threadIdx.x != 0 || !t.alive[w]) return;
  const double th = s.slice_theta[(long long)w * s.n + k];
  const double2 d = cscale(tr, 2.0);
  const double2 de = t.dexpo[w];
  if (!(cos(th) > 0.0) || !isfinite(d.x) || !isfinite(d.y)) { t.alive[w] = 0; return; }
  t.dlnw[2 * w + dir] += d.x + de.x - tan(th) * d.y;
}

// flags[w] = 1 when the smallest cos(theta_k) over the slices walker w survived is below
// `threshold` (its weight is not differentiable at a phaseless kill), else 0.
__global__ __launch_bounds__(NT) void kink_kernel(SysDev s, double threshold, int* flags) {
  const int w = blockIdx.x * NT + threadIdx.x;
  if (w >= s.W) return;
  int f = 0;
  for (int k = 0; k < s.n; ++k) {
    const double c = cos(s.slice_theta[(long long)w * s.n + k]);
    if (!(c > 0.0)) break;                      // the forward killed it here
    if (c < threshold) { f = 1; break; }
  }
  flags[w] = f;
}

int grid_for(long long total) {
  const long long b = (total + NT - 1) / NT;
  return (int)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace

hipError_t launch_coef_replay(const SysDev& s, int k, hipStream_t st) {
  const int chunks = (s.ld + RV_ROWS - 1) / RV_ROWS;
  coef_replay_kernel<<<((s.W + 7) / 8) * 8 * chunks, NT, 0, st>>>(s, k, chunks);
  return hipGetLastError();
}
hipError_t launch_tan_init(const SysDev& s, const TanDev& t, hipStream_t st) {
  tan_init_kernel<<<grid_for((long long)s.W * t.ld2 * t.ld2), NT, 0, st>>>(s, t);
  return hipGetLastError();
}
hipError_t launch_tan_prep(const SysDev& s, const TanDev& t, const double2* B, hipStream_t st) {
  tan_prep_kernel<<<grid_for((long long)s.W * s.ld * t.ld2), NT, 0, st>>>(s, t, B);
  return hipGetLastError();
}
hipError_t launch_cyc_form(const SysDev& s, const TanDev& t, int k, int literal, hipStream_t st) {
  const int nt = (t.ld2 + TT - 1) / TT;
  cyc_form_kernel<<<((s.W + 7) / 8) * 8 * nt * nt, NT, 0, st>>>(s, t, k, literal);
  return hipGetLastError();
}
hipError_t launch_cyc_post(const SysDev& s, const TanDev& t, int k, int literal, hipStream_t st) {
  const long long per = literal ? (long long)s.ld * s.ld : (long long)t.ld2 * s.ld;
  cyc_post_kernel<<<grid_for((long long)s.W * per), NT, 0, st>>>(s, t, k, literal);
  return hipGetLastError();
}
hipError_t launch_tan_weight(const SysDev& s, const TanDev& t, int k, hipStream_t st) {
  tan_weight_kernel<<<s.W, NT, 0, st>>>(s, t, k);
  return hipGetLastError();
}
hipError_t launch_permute_rows(const TanDev& t, hipStream_t st) {
  permute_rows_kernel<<<grid_for((long long)t.dd.W * t.dd.mat_stride), NT, 0, st>>>(t);
  return hipGetLastError();
}
hipError_t launch_energy_tangent(const SysDev& s, const TanDev& t, int dir, hipStream_t st) {
  const size_t shm = 2 * (size_t)s.M * sizeof(double2) +
                     (size_t)s.grid_dim * s.grid_dim * s.grid_dim * sizeof(short) + 16;
  exchange_tangent_kernel<<<((s.W + 7) / 8) * 8 * s.M, NT, shm, st>>>(s, t, dir);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  energy_tangent_kernel<<<s.W, NT, (size_t)s.NQ * sizeof(double2), st>>>(s, t, dir);
  return hipGetLastError();
}
hipError_t launch_tan_mean(const SysDev& s, const TanDev& t, const double* cot, double2* jac, double* grad,
                           double2* walker, hipStream_t st) {
  tan_mean_kernel<<<1, NT, 0, st>>>(s, t, cot, jac, grad, walker);
  return hipGetLastError();
}
hipError_t launch_pw_reset(const SysDev& s, const TanDev& t, hipStream_t st) {
  pw_reset_kernel<<<grid_for((long long)s.W * t.ld2 * t.ld2), NT, 0, st>>>(s, t);
  return hipGetLastError();
}
hipError_t launch_pw_extract(const SysDev& s, const TanDev& t, double2* dG_out, hipStream_t st) {
  pw_extract_kernel<<<grid_for((long long)s.W * s.ld * s.ld), NT, 0, st>>>(s, t, dG_out);
  return hipGetLastError();
}
hipError_t launch_pw_coef(const SysDev& s, const TanDev& t, const double2* fields, int k, hipStream_t st) {
  pw_coef_kernel<<<s.W, NT, 0, st>>>(s, t, fields, k);
  return hipGetLastError();
}
hipError_t launch_pw_blocks(const SysDev& s, const TanDev& t, const PwBlocks& b, hipStream_t st) {
  if (b.nb < 1 || b.nb > 6) return hipErrorInvalidValue;
  pw_blocks_kernel<<<grid_for((long long)s.W * s.mat_stride), NT, 0, st>>>(s, t, b);
  return hipGetLastError();
}
hipError_t launch_pw_prep(const SysDev& s, const TanDev& t, const double2* B, const double2* KdEK, int dir,
                          hipStream_t st) {
  pw_prep_kernel<<<grid_for((long long)s.W * s.ld * t.ld2), NT, 0, st>>>(s, t, B, KdEK, dir);
  return hipGetLastError();
}
hipError_t launch_pw_weight(const SysDev& s, const TanDev& t, int k, int dir, hipStream_t st) {
  pw_weight_kernel<<<s.W, NT, 0, st>>>(s, t, k, dir);
  return hipGetLastError();
}
hipError_t launch_kink_flags(const SysDev& s, double threshold, int* flags, hipStream_t st) {
  kink_kernel<<<(s.W + NT - 1) / NT, NT, 0, st>>>(s, threshold, flags);
  return hipGetLastError();
}
