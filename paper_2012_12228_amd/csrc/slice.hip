// Slice-path kernels other than the GEMMs and the elimination.
//
// Notation: per walker the sampled product is R_k = Y diag(D) T with Ti = T^{-1}; the
// constrained product is A_k = L_k R_k with the diagonal trial block
// L_k = B_T^{n-k} (eq. Abrenda).  Scale splitting: L = L_s / L_b and D = D_s / D_b
// with L_b = 1/max(1,|L|), D_b = 1/max(1,|D|) (Sec. "Numerical Stabilization"), so
//   I + A = L_b^{-1} X D_b^{-1} T,   X = L_b Ti D_b + L_s Y D_s,
//   G = (I + A)^{-1} = (Ti D_b) X^{-1} L_b,
//   ln det(I + A) = ln det X + ln det T - sum ln L_b - sum ln D_b.
#include "common.h"
#include "kernels.h"

namespace {

constexpr int NT = 256;
constexpr int TT = 32;  // transpose tile
constexpr double PI = 3.14159265358979323846;

FT_DEV double2 zero2() { return make_double2(0.0, 0.0); }

// ------------------------------------------------------------------ init ---
__global__ __launch_bounds__(NT) void init_state_kernel(SysDev s) {
  const long long total = (long long)s.W * s.mat_stride;
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < total; e += (long long)gridDim.x * NT) {
    const long long loc = e % s.mat_stride;
    const int i = (int)(loc / s.ld), j = (int)(loc % s.ld);
    const double2 v = (i == j && i < s.M) ? make_double2(1.0, 0.0) : zero2();
    s.Y[e] = v;
    s.Ti[e] = v;
  }
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < (long long)s.W * s.ld; e += (long long)gridDim.x * NT)
    s.D[e] = ((int)(e % s.ld) < s.M) ? 1.0 : 0.0;
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < s.W; e += (long long)gridDim.x * NT) {
    s.lndetT[e] = zero2();
    s.logw[e] = 0.0;
    s.status[e] = 0;
    s.expo[e] = zero2();
  }
}

// ------------------------------------------------- force-bias shifted V ---
// c_Q = i s_Q (z_Q + conj z_{-Q}) - 2 dtau v_Q r_{-Q}: the coefficient of rho(Q) in
// sqrt(dtau) (x - xbar).v with xbar_A = -2i s_Q (r_Q + r_{-Q}), xbar_B = 2 s_Q (r_Q - r_{-Q}),
// r_Q = <rho(Q)> per spin; the weight exponent is sum_Q [x.xbar - xbar.xbar/2].
// One workgroup per walker: c_Q into cq (and the path record) and the weight exponent.
__global__ __launch_bounds__(NT) void coef_kernel(SysDev s, const double2* fields, int k) {
  __shared__ double red[8];
  const int w = blockIdx.x;
  if (w >= s.W) return;
  const double2* z = fields + ((long long)w * s.n + k) * s.NQ;
  const double2* r = s.rb + (long long)w * s.NQ;     // the force bias's <rho_Q>
  double2* cq = s.cq + (long long)w * s.NQ;
  double2 ex = zero2();
  for (int q = threadIdx.x; q < s.NQ; q += NT) {
    const int nq = s.neg[q];
    const double2 zq = z[q], zn = z[nq], rq = r[q], rn = r[nq];
    const double sqv = s.sq[q], vqv = s.vq[q];
    // i s (z_q + conj z_-q)
    const double2 u = make_double2(zq.x + zn.x, zq.y - zn.y);
    double2 c = make_double2(-sqv * u.y, sqv * u.x);
    c.x -= 2.0 * s.dtau * vqv * rn.x;
    c.y -= 2.0 * s.dtau * vqv * rn.y;
    cq[q] = c;
    if (s.rec_c) s.rec_c[((long long)w * s.n + k) * s.NQ + q] = c;
    // xbar_A = -2i s (r_q + r_-q), xbar_B = 2 s (r_q - r_-q)
    const double2 sp = make_double2(rq.x + rn.x, rq.y + rn.y), sm = make_double2(rq.x - rn.x, rq.y - rn.y);
    const double2 xa = make_double2(2.0 * sqv * sp.y, -2.0 * sqv * sp.x);
    const double2 xb = make_double2(2.0 * sqv * sm.x, 2.0 * sqv * sm.y);
    const double2 xa2 = cmul(xa, xa), xb2 = cmul(xb, xb);
    ex.x += zq.x * xa.x + zq.y * xb.x - 0.5 * (xa2.x + xb2.x);
    ex.y += zq.x * xa.y + zq.y * xb.y - 0.5 * (xa2.y + xb2.y);
  }
  ex = block_csum_256(ex, red);
  if (threadIdx.x == 0) s.expo[w] = ex;
}

// V_ij = c_{Q = K_i - K_j} (zero on the diagonal and in the padding), V_ROWS rows per
// workgroup, the workgroups of a walker on one XCD (its c_Q stay in that L2).
constexpr int V_ROWS = 16;
template <typename TV>
__global__ __launch_bounds__(NT) void fill_v_kernel(SysDev s, TV* V, int chunks) {
  int w, c;
  if (!xcd_walker_tile(blockIdx.x, s.W, chunks, &w, &c)) return;
  const double2* cq = s.cq + (long long)w * s.NQ;
  TV* Vw = V + (long long)w * s.mat_stride;
  const int ld = s.ld, M = s.M, i0 = c * V_ROWS;
  for (int e = threadIdx.x; e < V_ROWS * ld; e += NT) {
    const int i = i0 + e / ld, j = e - (e / ld) * ld;
    if (i >= ld) break;
    double2 v = zero2();
    if (i < M && j < M && i != j) v = cq[s.idx[i * M + j]];
    store_c(Vw + (long long)i * ld + j, v);
  }
}

// -------------------------------------------- Taylor truncation check ---
// Column 1-norms of V and of V^4 (the Paterson-Stockmeyer chain's own V^4): 64 columns per
// workgroup, the rows shared by the 4 waves; the maximum over the chunk's columns goes to
// tnorm[w][c] (V) and tnorm[w][8 + c] (V^4).  A NaN entry makes the norm NaN.
template <typename TV>
__global__ __launch_bounds__(NT) void taylor_norms_kernel(SysDev s, const TV* V, const TV* V4, int chunks) {
  __shared__ double part[2][NT / 64][64];
  int w, c;
  if (!xcd_walker_tile(blockIdx.x, s.W, chunks, &w, &c)) return;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int M = s.M, ld = s.ld, j = c * 64 + lane;
  const TV* Vw = V + (long long)w * s.mat_stride;
  const TV* V4w = V4 + (long long)w * s.mat_stride;
  double a = 0.0, b = 0.0;
  if (j < M) {
#pragma unroll 4
    for (int i = wid; i < M; i += NT / 64) {
      const double2 x = to_d2(Vw[(long long)i * ld + j]), y = to_d2(V4w[(long long)i * ld + j]);
      a += sqrt(cabs2(x));
      b += sqrt(cabs2(y));
    }
  }
  part[0][wid][lane] = a;
  part[1][wid][lane] = b;
  __syncthreads();
  if (wid == 0) {
    a = (part[0][0][lane] + part[0][1][lane]) + (part[0][2][lane] + part[0][3][lane]);
    b = (part[1][0][lane] + part[1][1][lane]) + (part[1][2][lane] + part[1][3][lane]);
    for (int o = 32; o > 0; o >>= 1) {
      const double a2 = __shfl_xor(a, o, 64), b2 = __shfl_xor(b, o, 64);
      a = (a2 > a || a2 != a2) ? a2 : a;       // a NaN wins
      b = (b2 > b || b2 != b2) ? b2 : b;
    }
    if (lane == 0) {
      s.tnorm[(long long)w * 16 + c] = a;
      s.tnorm[(long long)w * 16 + 8 + c] = b;
    }
  }
}

// Bound on the Taylor remainder sum_{j > p} ||V^j|| / j! with ||V^{4q+b}|| <= ||V^4||^q ||V||^b
// (1-norms, submultiplicative), from the chunk maxima in tnorm.  NaN if a norm is NaN.
FT_DEV double taylor_tail(const SysDev& s, int w) {
  double n1 = 0.0, n4 = 0.0;
  const int chunks = (s.M + 63) / 64;
  for (int c = 0; c < chunks; ++c) {
    const double a = s.tnorm[(long long)w * 16 + c], b = s.tnorm[(long long)w * 16 + 8 + c];
    n1 = (a > n1 || a != a) ? a : n1;
    n4 = (b > n4 || b != b) ? b : n4;
  }
  if (n1 != n1 || n4 != n4) return NAN;
  if (n4 == 0.0) return 0.0;
  const double l1 = n1 > 0.0 ? log(n1) : -INFINITY, l4 = log(n4);
  double lf = 0.0;                                   // ln j!
  for (int j = 2; j <= s.taylor_deg; ++j) lf += log((double)j);
  double tail = 0.0;
  for (int j = s.taylor_deg + 1; j <= s.taylor_deg + 80; ++j) {
    lf += log((double)j);
    const int q = j >> 2, b = j & 3;
    const double t = exp((double)q * l4 + (b ? (double)b * l1 : 0.0) - lf);
    tail += t;
    if (t < 1e-30 * tail) break;
  }
  return tail;
}

// Lower Taylor blocks B_k = c[k][0] I + c[k][1] V + c[k][2] V^2 + c[k][3] V^3, k < t.nlo.
template <typename TV>
__global__ __launch_bounds__(NT) void taylor_blocks_kernel(SysDev s, TaylorLow t) {
  const long long total = (long long)s.W * s.mat_stride;
  const TV* V = (const TV*)s.V;
  const TV* V2 = (const TV*)s.V2;
  const TV* V3 = (const TV*)s.V3;
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < total; e += (long long)gridDim.x * NT) {
    const long long loc = e % s.mat_stride;
    const int i = (int)(loc / s.ld), j = (int)(loc % s.ld);
    const double di = (i == j && i < s.M) ? 1.0 : 0.0;
    const double2 v1 = to_d2(V[e]), v2 = to_d2(V2[e]), v3 = to_d2(V3[e]);
    for (int k = 0; k < t.nlo; ++k) {
      double2 b = make_double2(t.c[k][0] * di, 0.0);
      b = cadd(b, cadd(cscale(v1, t.c[k][1]), cadd(cscale(v2, t.c[k][2]), cscale(v3, t.c[k][3]))));
      store_c((TV*)s.Bk[k] + e, b);
    }
  }
}

// ------------------------------------------------------ Green's function ---
FT_DEV void split_L(const SysDev& s, int i, int lexp, double* lb, double* ls) {
  const double lnl = (double)lexp * s.lnbt[i];
  *lb = exp(-fmax(lnl, 0.0));
  *ls = exp(fmin(lnl, 0.0));
}
FT_DEV void split_D(double d, double* db, double* ds) {
  const double a = fabs(d);
  if (a > 1.0) { *db = 1.0 / a; *ds = d / a; }
  else { *db = 1.0; *ds = d; }
}

// aug[i][j] = X[j][i], aug[i][ld + j] = (Ti D_b)[j][i]  (transposed through LDS).
// Low-rank truncation (eq. thresh) of the diagonal left block: plane waves with B_T^lexp below the
// threshold drop out (L_s = 0: their rows of X are those of Ti D_b, so the same rows of G are the
// identity and their columns of the solution are known); only the lr_mL kept plane waves, in
// lr_order, are right-hand sides.
__global__ __launch_bounds__(NT) void greens_form_kernel(SysDev s, int lexp) {
  __shared__ double2 tX[TT][TT + 1];
  __shared__ double2 tU[TT][TT + 1];
  const int nt = (s.ld + TT - 1) / TT;
  int w, tile;
  if (!xcd_walker_tile(blockIdx.x, s.W, nt * nt, &w, &tile)) return;
  const int ti = tile / nt, tj = tile - ti * nt;   // aug rows ti*TT.., aug cols tj*TT..
  const double2* Y = s.Y + (long long)w * s.mat_stride;
  const double2* Ti = s.Ti + (long long)w * s.mat_stride;
  const double* D = s.D + (long long)w * s.ld;
  const bool lr = s.lr_order != nullptr;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  for (int yy = ty; yy < TT; yy += 8) {
    const int row = tj * TT + yy, col = ti * TT + tx;   // element (row=j, col=i) of Y and Ti
    double2 x = zero2(), u = zero2();
    if (row < s.M && col < s.M) {
      double lb, ls, db, ds;
      split_L(s, row, lexp, &lb, &ls);
      split_D(D[col], &db, &ds);
      if (lr && (double)lexp * s.lnbt[row] < s.lr_lnthr) ls = 0.0;
      const double2 tv = Ti[(long long)row * s.ld + col], yv = Y[(long long)row * s.ld + col];
      u = cscale(tv, db);
      x = make_double2(lb * u.x + ls * ds * yv.x, lb * u.y + ls * ds * yv.y);
      if (lr) u = row < s.lr_mL ? cscale(Ti[(long long)s.lr_order[row] * s.ld + col], db) : zero2();
    }
    tX[yy][tx] = x;
    tU[yy][tx] = u;
  }
  __syncthreads();
  double2* aug = s.aug + (long long)w * s.aug_stride;
  for (int yy = ty; yy < TT; yy += 8) {
    const int i = ti * TT + yy, j = tj * TT + tx;
    if (i < s.ld && j < s.ld) {
      aug[(long long)i * 2 * s.ld + j] = tX[tx][yy];
      aug[(long long)i * 2 * s.ld + s.ld + j] = tU[tx][yy];
    }
  }
}

// G[i][j] = H[j][i] L_b[j] with H = aug right block (= X^{-T} (Ti D_b)^T).  Low-rank: column i of
// H is solved column lr_pos[i] when i is kept, else e_i (row i of G is the identity).
__global__ __launch_bounds__(NT) void greens_post_kernel(SysDev s, int lexp) {
  __shared__ double2 tH[TT][TT + 1];
  const int nt = (s.ld + TT - 1) / TT;
  int w, tile;
  if (!xcd_walker_tile(blockIdx.x, s.W, nt * nt, &w, &tile)) return;
  const int ti = tile / nt, tj = tile - ti * nt;   // G rows ti.., cols tj..
  const double2* aug = s.aug + (long long)w * s.aug_stride;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int yy = ty; yy < TT; yy += 8) {
    const int row = tj * TT + yy, col = ti * TT + tx;   // H[row=j][col=i]
    double2 h = zero2();
    if (row < s.M && col < s.M) {
      double lb, ls;
      split_L(s, row, lexp, &lb, &ls);
      int c = col;
      if (s.lr_order) c = s.lr_pos[col] < s.lr_mL ? s.lr_pos[col] : -1;
      if (c >= 0) h = cscale(aug[(long long)row * 2 * s.ld + s.ld + c], lb);
      else if (row == col) h = make_double2(lb, 0.0);
    }
    tH[yy][tx] = h;
  }
  __syncthreads();
  double2* G = s.G + (long long)w * s.mat_stride;
  for (int yy = ty; yy < TT; yy += 8) {
    const int i = ti * TT + yy, j = tj * TT + tx;
    if (i < s.ld && j < s.ld) G[(long long)i * s.ld + j] = tH[tx][yy];
  }
}

// Right rank of the Green's function formed after slice k: the columns with |D| >= threshold.
__global__ __launch_bounds__(NT) void lr_rank_kernel(SysDev s, int k) {
  __shared__ double red[8];
  const int w = blockIdx.x;
  if (w >= s.W) return;
  const double* D = s.D + (long long)w * s.ld;
  double c = 0.0;
  for (int i = threadIdx.x; i < s.M; i += NT) c += fabs(D[i]) >= s.lr_thr ? 1.0 : 0.0;
  c = block_sum_256(c, red);
  if (threadIdx.x == 0) s.lr_mR[(long long)w * (s.n + 1) + k] = (int)c;
}

// r_Q = sum over pairs K_p - K_r = Q of P_pr = -G_rp: one Q per thread, NT Q per workgroup, the
// workgroups of a walker on one XCD (its G stays in that L2); eight partial sums keep eight
// gathers in flight.
__global__ __launch_bounds__(NT) void rq_kernel(SysDev s, int chunks) {
  int w, c;
  if (!xcd_walker_tile(blockIdx.x, s.W, chunks, &w, &c)) return;
  const int q = c * NT + threadIdx.x;
  if (q >= s.NQ) return;
  const double2* G = s.G + (long long)w * s.mat_stride;
  const int e0 = s.qptr[q], e1 = s.qptr[q + 1];
  double2 acc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) acc[k] = zero2();
  int e = e0;
  for (; e + 8 <= e1; e += 8) {
    int ix[8];
    double2 g[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) ix[k] = s.qpair[e + k];
#pragma unroll
    for (int k = 0; k < 8; ++k) g[k] = G[ix[k]];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = csub(acc[k], g[k]);
  }
  for (; e < e1; ++e) acc[0] = csub(acc[0], G[s.qpair[e]]);
  s.r[(long long)w * s.NQ + q] =
      cadd(cadd(cadd(acc[0], acc[1]), cadd(acc[2], acc[3])), cadd(cadd(acc[4], acc[5]), cadd(acc[6], acc[7])));
}

// r_Q with G streamed through LDS: one workgroup per walker (block w runs on XCD w mod 8, the
// XCD whose L2 holds walker w's G).  G goes through LDS one block of rows at a time with
// coalesced loads, together with the block's pair list; each thread then gathers the pairs of
// its Qs in that block from LDS.  The next block's loads are in flight during the gathers.
// Every Q sums its pairs block by block and row by row: a fixed order.
constexpr int RQ_NT = 1024, RQ_ELEMS = 4096, RQ_QPT = 4, RQ_PER = RQ_ELEMS / RQ_NT;
__global__ __launch_bounds__(RQ_NT) void rq_stream_kernel(SysDev s) {
  __shared__ double2 Gs[RQ_ELEMS];
  __shared__ int Is[RQ_ELEMS];
  const int w = blockIdx.x;
  if (w >= s.W) return;
  const int t = threadIdx.x, NQ = s.NQ, ld = s.ld, npair = s.M * (s.M - 1);
  const double2* G = s.G + (long long)w * s.mat_stride;
  // Block b's rows of G are contiguous (nr ld <= RQ_ELEMS entries).  Its pair list starts where
  // block b-1's ends (so no load waits for another) and has fewer than nr ld entries.  The index
  // loads are unconditional, at a clamped index: entries of Is past the block's own are loaded
  // but never read.
  double2 gv[RQ_PER];
  int iv[RQ_PER], qs[RQ_QPT], qe[RQ_QPT], iend = 0;
  auto fetch = [&](int b, int i0) {
    const int r0 = b * s.rq_rows, nr = min(s.rq_rows, s.M - r0), n = nr * ld;
    const double2* gb = G + (long long)r0 * ld;
    const int* bp = s.rbptr + (long long)b * (NQ + 1);
#pragma unroll
    for (int k = 0; k < RQ_PER; ++k) {
      const int e = t + k * RQ_NT;
      gv[k] = e < n ? gb[e] : zero2();
      iv[k] = s.rbidx[min(i0 + e, npair - 1)];
    }
#pragma unroll
    for (int i = 0; i < RQ_QPT; ++i) {
      const int q = t + i * RQ_NT, qc = q < NQ ? q : 0;
      qs[i] = bp[qc];                  // absolute offsets; made relative when used
      qe[i] = bp[qc + 1];
    }
    iend = bp[NQ];
  };
  double2 acc[RQ_QPT];
#pragma unroll
  for (int i = 0; i < RQ_QPT; ++i) acc[i] = zero2();
  int i0 = 0;                          // start of the current block's pair list
  fetch(0, 0);
  for (int b = 0; b < s.rq_nblk; ++b) {
    __syncthreads();                 // every gather of the previous block is done
#pragma unroll
    for (int k = 0; k < RQ_PER; ++k) {
      Gs[t + k * RQ_NT] = gv[k];
      Is[t + k * RQ_NT] = iv[k];
    }
    int cs[RQ_QPT], ce[RQ_QPT];
#pragma unroll
    for (int i = 0; i < RQ_QPT; ++i) {
      const bool mine = t + i * RQ_NT < NQ;
      cs[i] = mine ? qs[i] - i0 : 0;
      ce[i] = mine ? qe[i] - i0 : 0;
    }
    const int inext = iend;
    __syncthreads();
    if (b + 1 < s.rq_nblk) fetch(b + 1, inext);
#pragma unroll
    for (int i = 0; i < RQ_QPT; ++i)
      for (int e = cs[i]; e < ce[i]; ++e) acc[i] = csub(acc[i], Gs[Is[e]]);
    i0 = inext;
  }
#pragma unroll
  for (int i = 0; i < RQ_QPT; ++i) {
    const int q = t + i * RQ_NT;
    if (q < NQ) s.r[(long long)w * NQ + q] = acc[i];
  }
}

// ln det(I + A_k) and the phaseless weight (after rq_kernel).
__global__ __launch_bounds__(NT) void weight_kernel(SysDev s, int k, double sum_lnLb, int init) {
  __shared__ double red[8];
  const int w = blockIdx.x;
  if (w >= s.W) return;
  const double2* G = s.G + (long long)w * s.mat_stride;
  const double2* r = s.r + (long long)w * s.NQ;
  double bad = 0.0;
  for (int q = threadIdx.x; q < s.NQ; q += NT) {
    const double2 v = r[q];
    if (!isfinite(v.x) || !isfinite(v.y)) bad = 1.0;
  }
  double sdb = 0.0;
  const double* D = s.D + (long long)w * s.ld;
  for (int i = threadIdx.x; i < s.M; i += NT) sdb += log(fmax(fabs(D[i]), 1.0));   // -ln D_b
  sdb = block_sum_256(sdb, red);
  bad = block_sum_256(bad, red);
  if (s.rec_trG) {                       // tr G_k, kept for the frozen-path derivative in mu
    double2 tr = zero2();
    for (int i = threadIdx.x; i < s.M; i += NT) tr = cadd(tr, G[(long long)i * s.ld + i]);
    tr = block_csum_256(tr, red);
    if (threadIdx.x == 0) s.rec_trG[(long long)w * (s.n + 1) + k] = tr;
  }
  if (threadIdx.x != 0) return;
  const double2 lx = s.lndetX[w], lt = s.lndetT[w];
  // ln det(I + A) = ln det X + ln det T - sum ln L_b - sum ln D_b
  const double2 ell = make_double2(lx.x + lt.x - sum_lnLb + sdb, lx.y + lt.y);
  int st = s.status[w];
  if (init) {
    s.ell[w] = ell;
    if (!(isfinite(ell.x) && isfinite(ell.y)) || bad > 0.0) s.status[w] = 2;
    return;
  }
  const double2 old = s.ell[w];
  s.ell[w] = ell;
  // S = det(I + A_{k+1})^2 / det(I + A_k)^2 ; theta = arg S in (-pi, pi]
  const double2 lnS = make_double2(2.0 * (ell.x - old.x), 2.0 * (ell.y - old.y));
  double th = remainder(lnS.y, 2.0 * PI);
  if (th <= -PI) th += 2.0 * PI;
  const double lnI = lnS.x + s.expo[w].x;
  s.slice_lnS[(long long)w * s.n + (k - 1)] = lnS;
  s.slice_theta[(long long)w * s.n + (k - 1)] = th;
  if (st == 0) {
    const double cth = cos(th);
    // the slice's e^V is trusted only while its Taylor remainder bound is below the tolerance
    const double tail = s.tnorm ? taylor_tail(s, w) : 0.0;
    if (!(isfinite(lnI) && isfinite(ell.x) && isfinite(ell.y)) || bad > 0.0 || !(tail <= s.taylor_tol)) {
      s.status[w] = 2;
      s.logw[w] = -INFINITY;
    }
    else if (cth <= 0.0) { s.status[w] = 1; s.logw[w] = -INFINITY; }
    else s.logw[w] += lnI + log(cth);
  }
}

// ------------------------------------------------------- stabilisation ---
// Column norms |Y e_j| |D_j| into scratch: 64 columns per workgroup, the rows shared by the 4
// waves; a NaN norm becomes -1 (it ranks last, so ranks stay a permutation).
__global__ __launch_bounds__(NT) void stab_norm_kernel(SysDev s, int chunks) {
  __shared__ double part[NT / 64][64];
  int w, c;
  if (!xcd_walker_tile(blockIdx.x, s.W, chunks, &w, &c)) return;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int M = s.M, ld = s.ld, j = c * 64 + lane;
  const double2* Y = s.Y + (long long)w * s.mat_stride;
  double a = 0.0;
  if (j < M)
    for (int i = wid; i < M; i += NT / 64) a += cabs2(Y[(long long)i * ld + j]);
  part[wid][lane] = a;
  __syncthreads();
  if (wid == 0 && j < M) {
    const double t = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
    const double v = sqrt(t) * fabs(s.D[(long long)w * ld + j]);
    s.scratch[(long long)w * ld + j] = (v == v) ? v : -1.0;
  }
}

// Pre-pivoting: order the columns of Y diag(D) by decreasing norm (ties by index); the parity of
// the permutation (from its inversions) goes into ln det T.
__global__ __launch_bounds__(NT) void stab_perm_kernel(SysDev s) {
  extern __shared__ double nrm[];           // [M], then perm [M] as int
  __shared__ double red[8];
  const int w = blockIdx.x;
  if (w >= s.W) return;
  const double* D = s.D + (long long)w * s.ld;
  const int M = s.M, ld = s.ld;
  int* psh = (int*)(nrm + M);
  for (int j = threadIdx.x; j < M; j += NT) nrm[j] = s.scratch[(long long)w * ld + j];
  __syncthreads();
  int* perm = s.perm + (long long)w * ld;
  double* Dpi = s.Dpi + (long long)w * ld;
  for (int j = threadIdx.x; j < M; j += NT) {
    const double v = nrm[j];
    int rank = 0;
    for (int i = 0; i < M; ++i) {
      const double u = nrm[i];
      rank += (u > v || (u == v && i < j)) ? 1 : 0;
    }
    perm[rank] = j;
    psh[rank] = j;
  }
  __syncthreads();
  double inv = 0.0;
  for (int j = threadIdx.x; j < M; j += NT) {
    Dpi[j] = D[psh[j]];
    const int pj = psh[j];
    int c = 0;
    for (int i = 0; i < j; ++i) c += psh[i] > pj ? 1 : 0;
    inv += (double)c;
  }
  inv = block_sum_256(inv, red);
  if (threadIdx.x == 0 && ((long long)inv & 1)) s.lndetT[w].y += PI;
}

// E0 = Y[:, perm]; aug right block = E0^H
__global__ __launch_bounds__(NT) void stab_gather_kernel(SysDev s) {
  __shared__ double2 tile_sh[TT][TT + 1];
  const int nt = (s.ld + TT - 1) / TT;
  int w, tile;
  if (!xcd_walker_tile(blockIdx.x, s.W, nt * nt, &w, &tile)) return;
  const int ti = tile / nt, tj = tile - ti * nt;   // E0 rows ti.., cols tj..
  const double2* Y = s.Y + (long long)w * s.mat_stride;
  const int* perm = s.perm + (long long)w * s.ld;
  double2* E0 = (double2*)s.E0 + (long long)w * s.mat_stride;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int yy = ty; yy < TT; yy += 8) {
    const int i = ti * TT + yy, j = tj * TT + tx;
    double2 v = zero2();
    if (i < s.M && j < s.M) v = Y[(long long)i * s.ld + perm[j]];
    if (i < s.ld && j < s.ld) E0[(long long)i * s.ld + j] = v;
    tile_sh[yy][tx] = v;
  }
  __syncthreads();
  double2* aug = s.aug + (long long)w * s.aug_stride;
  for (int yy = ty; yy < TT; yy += 8) {
    const int j = tj * TT + yy, i = ti * TT + tx;    // aug[j][ld + i] = conj(E0[i][j])
    if (i < s.ld && j < s.ld) aug[(long long)j * 2 * s.ld + s.ld + i] = cconj(tile_sh[tx][yy]);
  }
}

// After the Cholesky elimination of [S | E0^H]: U = aug left (S = L D L^H, U = D L^H),
// aug right = L'^{-1} E0^H with L' unit lower.  R1 = D^{-1/2} U, Q^H = D^{-1/2} (aug right).
// Writes Y = Q, D_new = sqrt(d) D_pi, and Ru = D_new^{-1} R1 D_pi (unit upper) into E1.
__global__ __launch_bounds__(NT) void stab_finish_a_kernel(SysDev s) {
  __shared__ double2 tile_sh[TT][TT + 1];
  const int nt = (s.ld + TT - 1) / TT;
  int w, tile;
  if (!xcd_walker_tile(blockIdx.x, s.W, nt * nt, &w, &tile)) return;
  const int ti = tile / nt, tj = tile - ti * nt;   // aug rows ti.., cols tj..
  const double2* aug = s.aug + (long long)w * s.aug_stride;
  const double* Dpi = s.Dpi + (long long)w * s.ld;
  double2* Ru = (double2*)s.E1 + (long long)w * s.mat_stride;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int ld2 = 2 * s.ld;
  for (int yy = ty; yy < TT; yy += 8) {
    const int i = ti * TT + yy, j = tj * TT + tx;
    double2 q = zero2(), ru = zero2();
    if (i < s.M && j < s.M) {
      const double d = aug[(long long)i * ld2 + i].x;
      const double sd = sqrt(d);
      q = cscale(aug[(long long)i * ld2 + s.ld + j], 1.0 / sd);
      if (j == i) ru = make_double2(1.0, 0.0);
      else if (j > i) ru = cscale(aug[(long long)i * ld2 + j], Dpi[j] / (d * Dpi[i]));
    }
    if (i < s.ld && j < s.ld) Ru[(long long)i * s.ld + j] = ru;
    tile_sh[yy][tx] = q;
  }
  __syncthreads();
  double2* Y = s.Y + (long long)w * s.mat_stride;
  for (int yy = ty; yy < TT; yy += 8) {
    const int j = tj * TT + yy, i = ti * TT + tx;   // Y[j][i] = conj(Q^H[i][j])
    if (i < s.ld && j < s.ld) Y[(long long)j * s.ld + i] = cconj(tile_sh[tx][yy]);
  }
}

// New D from the pivots d_i of the Cholesky (LDL^H) step, and the conditioning test of the pass:
// rho = min_i d_i / S_ii is the smallest squared sine between a pre-pivoted column of Y and the
// span of the columns before it (S = E0^H E0, S_ii = |Y e_perm(i)|^2 from the pre-pivot norms).
// Cholesky-QR loses orthogonality like eps / rho; below STAB_MIN_RHO (or at a non-positive or
// non-finite pivot) the walker is flagged numeric instead of carrying a non-orthogonal Q.
constexpr double STAB_MIN_RHO = 1e-5;
__global__ __launch_bounds__(NT) void stab_newd_kernel(SysDev s) {
  __shared__ double red[8];
  const int w = blockIdx.x;
  if (w >= s.W) return;
  const double2* aug = s.aug + (long long)w * s.aug_stride;
  const double* Dpi = s.Dpi + (long long)w * s.ld;
  const int* perm = s.perm + (long long)w * s.ld;
  const double* nrm = s.scratch + (long long)w * s.ld;      // |Y e_j| |D_j| from the pre-pivot
  double* D = s.D + (long long)w * s.ld;
  double bad = 0.0;
  for (int i = threadIdx.x; i < s.ld; i += NT) {
    double v = 0.0;
    if (i < s.M) {
      const double d = aug[(long long)i * 2 * s.ld + i].x;
      const double cn = nrm[perm[i]] / fabs(Dpi[i]);
      const double rho = d / (cn * cn);
      if (!(d > 0.0) || !isfinite(d) || !(rho >= STAB_MIN_RHO)) bad = 1.0;
      v = sqrt(d) * Dpi[i];
    }
    D[i] = v;
  }
  bad = block_sum_256(bad, red);
  if (threadIdx.x == 0 && bad > 0.0 && s.status[w] == 0) {
    s.status[w] = 2;   // the partial product was too ill-conditioned for one Cholesky-QR pass
    if (s.logw) s.logw[w] = -INFINITY;
  }
}

// aug = [Ru^T | (Ti[:, perm])^T]
__global__ __launch_bounds__(NT) void stab_build_ti_kernel(SysDev s) {
  __shared__ double2 tR[TT][TT + 1];
  __shared__ double2 tT[TT][TT + 1];
  const int nt = (s.ld + TT - 1) / TT;
  int w, tile;
  if (!xcd_walker_tile(blockIdx.x, s.W, nt * nt, &w, &tile)) return;
  const int ti = tile / nt, tj = tile - ti * nt;   // aug rows ti.., cols tj..
  const double2* Ru = (const double2*)s.E1 + (long long)w * s.mat_stride;
  const double2* Ti = s.Ti + (long long)w * s.mat_stride;
  const int* perm = s.perm + (long long)w * s.ld;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int yy = ty; yy < TT; yy += 8) {
    const int row = tj * TT + yy, col = ti * TT + tx;   // source element (row=j, col=i)
    double2 a = zero2(), b = zero2();
    if (row < s.M && col < s.M) {
      a = Ru[(long long)row * s.ld + col];
      b = Ti[(long long)row * s.ld + perm[col]];
    }
    tR[yy][tx] = a;
    tT[yy][tx] = b;
  }
  __syncthreads();
  double2* aug = s.aug + (long long)w * s.aug_stride;
  for (int yy = ty; yy < TT; yy += 8) {
    const int i = ti * TT + yy, j = tj * TT + tx;
    if (i < s.ld && j < s.ld) {
      aug[(long long)i * 2 * s.ld + j] = tR[tx][yy];
      aug[(long long)i * 2 * s.ld + s.ld + j] = tT[tx][yy];
    }
  }
}

// Ti[i][j] = aug[j][ld + i]
__global__ __launch_bounds__(NT) void stab_finish_b_kernel(SysDev s) {
  __shared__ double2 tile_sh[TT][TT + 1];
  const int nt = (s.ld + TT - 1) / TT;
  int w, tile;
  if (!xcd_walker_tile(blockIdx.x, s.W, nt * nt, &w, &tile)) return;
  const int ti = tile / nt, tj = tile - ti * nt;   // Ti rows ti.., cols tj..
  const double2* aug = s.aug + (long long)w * s.aug_stride;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int yy = ty; yy < TT; yy += 8) {
    const int row = tj * TT + yy, col = ti * TT + tx;   // aug[row=j][ld + col=i]
    double2 v = zero2();
    if (row < s.M && col < s.M) v = aug[(long long)row * 2 * s.ld + s.ld + col];
    tile_sh[yy][tx] = v;
  }
  __syncthreads();
  double2* Ti = s.Ti + (long long)w * s.mat_stride;
  for (int yy = ty; yy < TT; yy += 8) {
    const int i = ti * TT + yy, j = tj * TT + tx;
    if (i < s.ld && j < s.ld) Ti[(long long)i * s.ld + j] = tile_sh[tx][yy];
  }
}

// ---------------------------------------------------------------- energy ---
// Exchange: sum_Q v_Q Lambda_Q = sum_{a != d} v(K_a - K_d) sum_b P_ab P_cd with
// K_c = K_b - (K_a - K_d), P = I - G^T.  One workgroup per (walker, a), the d shared over the
// waves, b over the lanes; the lookup tables sit in LDS and each lane's (at most 8) gathers
// of row d are issued together.  P_cd = delta_cd - G_dc, and c = d only for b = a, so the sum
// over b is P_aa - sum_b P_ab G_dc: the delta term leaves the loop as P_aa sum_{d != a} v(K_a - K_d).
// The wave index is scalar, so row d's address is scalar and each gather is one offset; the row
// v(K_a - K_d) over d sits in LDS with the tables.
// With X: the sum over b for every pair (a, d) also goes to X[w][a][d] (for <rho(Q) rho(-Q)>).
template <int EX_B, bool WITHX>                     // b per lane: M <= 64 EX_B
__global__ __launch_bounds__(NT) void exchange_kernel(SysDev s, double2* X) {
  extern __shared__ char dyn[];
  const int M = s.M, ld = s.ld;
  double2* pcol = (double2*)dyn;                    // [M]: P_ab = delta_ab - G_ba
  double* vrow = (double*)(pcol + M);               // [M]: v(K_a - K_d), 0 at d = a
  int* flat = (int*)(vrow + M);                     // [M]
  short* grid = (short*)(flat + M);                 // [grid_dim^3]
  __shared__ double red[8];
  int w, a;
  if (!xcd_walker_tile(blockIdx.x, s.W, s.M, &w, &a)) return;
  const double2* G = s.G + (long long)w * s.mat_stride;
  const int g3 = s.grid_dim * s.grid_dim * s.grid_dim;
  for (int e = threadIdx.x; e < g3; e += NT) grid[e] = s.grid[e];
  for (int b = threadIdx.x; b < M; b += NT) {
    double2 v = cscale(G[(long long)b * ld + a], -1.0);
    if (b == a) v.x += 1.0;
    pcol[b] = v;
    flat[b] = s.flat[b];
    vrow[b] = b == a ? 0.0 : s.vq[s.idx[a * M + b]];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // this lane's b and their grid offsets do not depend on d
  int fb[EX_B];
  double2 pb[EX_B];
#pragma unroll
  for (int k = 0; k < EX_B; ++k) {
    const int b = lane + 64 * k;
    fb[k] = b < M ? flat[b] - flat[a] + s.grid_c0 : -1;
    pb[k] = b < M ? pcol[b] : zero2();
  }
  const double2 paa = pcol[a];
  double2 acc = zero2();
  double vsum = 0.0;                                // sum of v(K_a - K_d) over this wave's d
  for (int d = wid; d < M; d += NT / 64) {
    if (d == a) continue;
    const double v = vrow[d];
    const double2* Gd = G + (long long)d * ld;
    const int fd = flat[d];
    int c[EX_B];
    double2 g[EX_B];
#pragma unroll
    for (int k = 0; k < EX_B; ++k) c[k] = fb[k] >= 0 ? grid[fb[k] + fd] : -1;   // K_b - K_a + K_d
#pragma unroll
    for (int k = 0; k < EX_B; ++k) g[k] = c[k] >= 0 ? Gd[c[k]] : zero2();
    double2 part = zero2();                         // sum_b P_ab G_dc
#pragma unroll
    for (int k = 0; k < EX_B; ++k) {
      part.x = fma(pb[k].x, g[k].x, part.x);
      part.x = fma(-pb[k].y, g[k].y, part.x);
      part.y = fma(pb[k].x, g[k].y, part.y);
      part.y = fma(pb[k].y, g[k].x, part.y);
    }
    acc.x -= v * part.x;
    acc.y -= v * part.y;
    vsum += v;
    if constexpr (WITHX) {
      const double px = wave_sum(part.x), py = wave_sum(part.y);
      if (lane == 0) X[(long long)w * s.mat_stride + (long long)a * ld + d] = make_double2(paa.x - px, paa.y - py);
    }
  }
  if (lane == 0) {                                  // the delta term
    acc.x += paa.x * vsum;
    acc.y += paa.y * vsum;
  }
  acc = block_csum_256(acc, red);
  if (threadIdx.x == 0) s.exch[(long long)w * ld + a] = acc;
}

// <rho(Q) rho(-Q)> = 4 r_Q r_-Q + 2 (n_Q - Lambda_Q) per walker and Q (Wick's theorem with both
// spins), with Lambda_Q = sum over the pairs (p, r) of Q (K_p - K_r = Q) of X[p][r] and
// n_Q = sum over the same pairs of P_pp = 1 - G_pp.  One thread per (walker, Q).
__global__ __launch_bounds__(NT) void density_corr_kernel(SysDev s, const double2* X, double2* out, int chunks) {
  int w, c;
  if (!xcd_walker_tile(blockIdx.x, s.W, chunks, &w, &c)) return;
  const int q = c * NT + threadIdx.x;
  if (q >= s.NQ) return;
  const double2* G = s.G + (long long)w * s.mat_stride;
  const double2* Xw = X + (long long)w * s.mat_stride;
  double2 lam = zero2(), nq = zero2();
  for (int e = s.qptr[q]; e < s.qptr[q + 1]; ++e) {
    const int f = s.qpair[e];                     // r ld + p
    const int r = f / s.ld, p = f - r * s.ld;
    lam = cadd(lam, Xw[(long long)p * s.ld + r]);
    const double2 g = G[(long long)p * s.ld + p];
    nq = cadd(nq, make_double2(1.0 - g.x, -g.y));
  }
  const double2* rr = s.r + (long long)w * s.NQ;
  const double2 h = cmul(rr[q], rr[s.neg[q]]);
  out[(long long)w * s.NQ + q] = make_double2(4.0 * h.x + 2.0 * (nq.x - lam.x), 4.0 * h.y + 2.0 * (nq.y - lam.y));
}

// Weighted mean over live walkers of per-walker values v [W][n] into mean [n].
__global__ __launch_bounds__(NT) void weighted_mean_kernel(const double2* v, int n, const double* logw,
                                                           const int* status, int W, double2* mean) {
  const int q = blockIdx.x * NT + threadIdx.x;
  if (q >= n) return;
  double mx = -INFINITY;
  for (int w = 0; w < W; ++w)
    if (status[w] == 0 && isfinite(logw[w])) mx = fmax(mx, logw[w]);
  double ws = 0.0;
  double2 acc = zero2();
  for (int w = 0; w < W; ++w)
    if (status[w] == 0 && isfinite(logw[w])) {
      const double f = exp(logw[w] - mx);
      ws += f;
      acc = cadd(acc, cscale(v[(long long)w * n + q], f));
    }
  mean[q] = ws > 0.0 ? cscale(acc, 1.0 / ws) : make_double2(NAN, NAN);
}

// E1 = 2 lambda sum eps P_KK, N = 2 sum P_KK, Hartree = (1/2) sum v_Q 4 r_Q r_-Q,
// E2 = Hartree - sum_Q v_Q Lambda_Q, E = E1 + E2 + E_M.
__global__ __launch_bounds__(NT) void energy_finish_kernel(SysDev s, int rec) {
  __shared__ double red[8];
  const int w = blockIdx.x;
  if (w >= s.W) return;
  const double2* G = s.G + (long long)w * s.mat_stride;
  const double2* r = s.r + (long long)w * s.NQ;
  double2 e1 = zero2(), nn = zero2(), hart = zero2(), ex = zero2();
  for (int i = threadIdx.x; i < s.M; i += NT) {
    const double2 g = G[(long long)i * s.ld + i];
    const double2 pkk = make_double2(1.0 - g.x, -g.y);
    e1 = cadd(e1, cscale(pkk, s.eps[i]));
    nn = cadd(nn, pkk);
    ex = cadd(ex, s.exch[(long long)w * s.ld + i]);
  }
  for (int q = threadIdx.x; q < s.NQ; q += NT) hart = cadd(hart, cscale(cmul(r[q], r[s.neg[q]]), s.vq[q]));
  e1 = block_csum_256(e1, red);
  nn = block_csum_256(nn, red);
  hart = block_csum_256(hart, red);
  ex = block_csum_256(ex, red);
  if (threadIdx.x != 0) return;
  const double2 E1 = cscale(e1, 2.0 * s.kscale);
  const double2 N = cscale(nn, 2.0);
  const double2 E2 = csub(cscale(hart, 2.0), ex);
  const double2 E = make_double2(E1.x + E2.x + s.e_madelung, E1.y + E2.y);
  double2* out = s.local + (long long)w * 4;
  out[0] = E1; out[1] = E2; out[2] = E; out[3] = N;
  if (rec >= 0) {
    const long long rw = (long long)rec * s.rec_W + s.w_off + w;   // records span all walkers of the system
    double2* ro = s.rec_E + rw * 4;
    ro[0] = E1; ro[1] = E2; ro[2] = E; ro[3] = N;
    s.rec_logw[rw] = s.logw[w];
    s.rec_status[rw] = s.status[w];
  }
}

// weighted means over live walkers: sum_w e^{logw - max} O_w / sum_w e^{logw - max}
__global__ __launch_bounds__(NT) void energy_mean_kernel(const double2* local, const double* logw,
                                                         const int* status, int W, double2* mean) {
  __shared__ double red[8];
  double mx = -INFINITY;
  for (int w = threadIdx.x; w < W; w += NT)
    if (status[w] == 0 && isfinite(logw[w])) mx = fmax(mx, logw[w]);
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  __shared__ double mxs[4];
  if ((threadIdx.x & 63) == 0) mxs[threadIdx.x >> 6] = mx;
  __syncthreads();
  mx = fmax(fmax(mxs[0], mxs[1]), fmax(mxs[2], mxs[3]));
  __syncthreads();
  double ws = 0.0;
  double2 acc[4] = {zero2(), zero2(), zero2(), zero2()};
  for (int w = threadIdx.x; w < W; w += NT) {
    if (status[w] == 0 && isfinite(logw[w])) {
      const double f = exp(logw[w] - mx);
      ws += f;
      for (int c = 0; c < 4; ++c) acc[c] = cadd(acc[c], cscale(local[(long long)w * 4 + c], f));
    }
  }
  ws = block_sum_256(ws, red);
  for (int c = 0; c < 4; ++c) acc[c] = block_csum_256(acc[c], red);
  if (threadIdx.x == 0)
    for (int c = 0; c < 4; ++c)
      mean[c] = ws > 0.0 ? cscale(acc[c], 1.0 / ws) : make_double2(NAN, NAN);
}

template <typename TO>
__global__ __launch_bounds__(NT) void copy_greens_kernel(SysDev s, TO* out) {
  const long long total = (long long)s.W * s.M * s.M;
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < total; e += (long long)gridDim.x * NT) {
    const long long w = e / ((long long)s.M * s.M);
    const int loc = (int)(e - w * s.M * s.M);
    const int i = loc / s.M, j = loc - i * s.M;
    store_c(out + e, s.G[w * s.mat_stride + (long long)i * s.ld + j]);
  }
}

__global__ __launch_bounds__(NT) void copy_state_kernel(SysDev s, double2* local, double* logw, int* status) {
  for (int w = blockIdx.x * NT + threadIdx.x; w < s.W; w += gridDim.x * NT) {
    if (local)
      for (int c = 0; c < 4; ++c) local[(long long)w * 4 + c] = s.local[(long long)w * 4 + c];
    if (logw) logw[w] = s.logw[w];
    if (status) status[w] = s.status[w];
  }
}

int tiles_blocks(const SysDev& s, int per_walker) { return ((s.W + 7) / 8) * 8 * per_walker; }
int tt_tiles(const SysDev& s) { const int nt = (s.ld + TT - 1) / TT; return nt * nt; }

}  // namespace

hipError_t launch_init_state(const SysDev& s, hipStream_t st) {
  init_state_kernel<<<1024, NT, 0, st>>>(s);
  return hipGetLastError();
}
hipError_t launch_fill_v(const SysDev& s, void* V, int mixed, hipStream_t st) {
  const int chunks = (s.ld + V_ROWS - 1) / V_ROWS;
  if (mixed) fill_v_kernel<float2><<<tiles_blocks(s, chunks), NT, 0, st>>>(s, (float2*)V, chunks);
  else fill_v_kernel<double2><<<tiles_blocks(s, chunks), NT, 0, st>>>(s, (double2*)V, chunks);
  return hipGetLastError();
}
hipError_t launch_coef_v(const SysDev& s, const double2* fields, int k, int mixed, hipStream_t st) {
  coef_kernel<<<s.W, NT, 0, st>>>(s, fields, k);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int chunks = (s.ld + V_ROWS - 1) / V_ROWS;
  if (mixed) fill_v_kernel<float2><<<tiles_blocks(s, chunks), NT, 0, st>>>(s, (float2*)s.V, chunks);
  else fill_v_kernel<double2><<<tiles_blocks(s, chunks), NT, 0, st>>>(s, (double2*)s.V, chunks);
  return hipGetLastError();
}
hipError_t launch_taylor_norms(const SysDev& s, int mixed, hipStream_t st) {
  const int chunks = (s.M + 63) / 64;
  if (chunks > 8) return hipErrorInvalidValue;
  if (mixed) taylor_norms_kernel<float2><<<tiles_blocks(s, chunks), NT, 0, st>>>(s, (const float2*)s.V, (const float2*)s.V4, chunks);
  else taylor_norms_kernel<double2><<<tiles_blocks(s, chunks), NT, 0, st>>>(s, (const double2*)s.V, (const double2*)s.V4, chunks);
  return hipGetLastError();
}
hipError_t launch_taylor_blocks(const SysDev& s, int mixed, const TaylorLow& t, hipStream_t st) {
  if (t.nlo < 0 || t.nlo > 2) return hipErrorInvalidValue;
  if (t.nlo == 0) return hipSuccess;
  if (mixed) taylor_blocks_kernel<float2><<<2048, NT, 0, st>>>(s, t);
  else taylor_blocks_kernel<double2><<<2048, NT, 0, st>>>(s, t);
  return hipGetLastError();
}
hipError_t launch_greens_form(const SysDev& s, int lexp, hipStream_t st) {
  greens_form_kernel<<<tiles_blocks(s, tt_tiles(s)), NT, 0, st>>>(s, lexp);
  return hipGetLastError();
}
hipError_t launch_greens_post(const SysDev& s, int lexp, hipStream_t st) {
  greens_post_kernel<<<tiles_blocks(s, tt_tiles(s)), NT, 0, st>>>(s, lexp);
  return hipGetLastError();
}
hipError_t launch_lr_rank(const SysDev& s, int k, hipStream_t st) {
  if (!s.lr_mR) return hipSuccess;
  lr_rank_kernel<<<s.W, NT, 0, st>>>(s, k);
  return hipGetLastError();
}
int rq_block_elems() { return RQ_ELEMS; }
hipError_t launch_rq(const SysDev& s, hipStream_t st) {
  if (!s.rq_gather && s.NQ > 0 && s.NQ <= RQ_QPT * RQ_NT && s.rq_rows * s.ld <= RQ_ELEMS) {
    rq_stream_kernel<<<s.W, RQ_NT, 0, st>>>(s);
  } else {
    const int chunks = (s.NQ + NT - 1) / NT;
    rq_kernel<<<tiles_blocks(s, chunks), NT, 0, st>>>(s, chunks);
  }
  return hipGetLastError();
}
hipError_t launch_weight(const SysDev& s, int k, double sum_lnLb, int init, hipStream_t st) {
  hipError_t e = launch_rq(s, st);
  if (e != hipSuccess) return e;
  weight_kernel<<<s.W, NT, 0, st>>>(s, k, sum_lnLb, init);
  return hipGetLastError();
}
hipError_t launch_stab_perm(const SysDev& s, hipStream_t st) {
  const int chunks = (s.M + 63) / 64;
  stab_norm_kernel<<<tiles_blocks(s, chunks), NT, 0, st>>>(s, chunks);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  stab_perm_kernel<<<s.W, NT, (size_t)s.M * (sizeof(double) + sizeof(int)), st>>>(s);
  return hipGetLastError();
}
hipError_t launch_stab_gather(const SysDev& s, hipStream_t st) {
  stab_gather_kernel<<<tiles_blocks(s, tt_tiles(s)), NT, 0, st>>>(s);
  return hipGetLastError();
}
hipError_t launch_stab_finish_a(const SysDev& s, hipStream_t st) {
  stab_finish_a_kernel<<<tiles_blocks(s, tt_tiles(s)), NT, 0, st>>>(s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  stab_newd_kernel<<<s.W, NT, 0, st>>>(s);
  return hipGetLastError();
}
hipError_t launch_stab_build_ti(const SysDev& s, hipStream_t st) {
  stab_build_ti_kernel<<<tiles_blocks(s, tt_tiles(s)), NT, 0, st>>>(s);
  return hipGetLastError();
}
hipError_t launch_stab_finish_b(const SysDev& s, hipStream_t st) {
  stab_finish_b_kernel<<<tiles_blocks(s, tt_tiles(s)), NT, 0, st>>>(s);
  return hipGetLastError();
}
template <bool WITHX> hipError_t launch_exchange(const SysDev& s, double2* X, hipStream_t st) {
  const size_t shm = (size_t)s.M * (sizeof(double2) + sizeof(double) + sizeof(int)) +
                     (size_t)s.grid_dim * s.grid_dim * s.grid_dim * sizeof(short) + 16;
  if (s.M <= 64 * 2) exchange_kernel<2, WITHX><<<tiles_blocks(s, s.M), NT, shm, st>>>(s, X);
  else if (s.M <= 64 * 3) exchange_kernel<3, WITHX><<<tiles_blocks(s, s.M), NT, shm, st>>>(s, X);
  else if (s.M <= 64 * 4) exchange_kernel<4, WITHX><<<tiles_blocks(s, s.M), NT, shm, st>>>(s, X);
  else if (s.M <= 64 * 6) exchange_kernel<6, WITHX><<<tiles_blocks(s, s.M), NT, shm, st>>>(s, X);
  else if (s.M <= 64 * 8) exchange_kernel<8, WITHX><<<tiles_blocks(s, s.M), NT, shm, st>>>(s, X);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}
hipError_t launch_density_correlation(const SysDev& s, double2* X, double2* out, double2* mean, hipStream_t st) {
  hipError_t e = launch_exchange<true>(s, X, st);
  if (e != hipSuccess) return e;
  const int chunks = (s.NQ + NT - 1) / NT;
  density_corr_kernel<<<tiles_blocks(s, chunks), NT, 0, st>>>(s, X, out, chunks);
  e = hipGetLastError();
  if (e != hipSuccess || !mean) return e;
  weighted_mean_kernel<<<(s.NQ + NT - 1) / NT, NT, 0, st>>>(out, s.NQ, s.logw, s.status, s.W, mean);
  return hipGetLastError();
}
hipError_t launch_energy(const SysDev& s, int rec, hipStream_t st) {
  hipError_t e0 = launch_exchange<false>(s, nullptr, st);
  if (e0 != hipSuccess) return e0;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  energy_finish_kernel<<<s.W, NT, 0, st>>>(s, rec);
  return hipGetLastError();
}
hipError_t launch_energy_mean(const SysDev& s, const double2* local, const double* logw, const int* status,
                              double2* mean, hipStream_t st) {
  energy_mean_kernel<<<1, NT, 0, st>>>(local, logw, status, s.W, mean);
  return hipGetLastError();
}
hipError_t launch_copy_greens(const SysDev& s, void* out, int dtype, hipStream_t st) {
  if (dtype == 0) copy_greens_kernel<double2><<<1024, NT, 0, st>>>(s, (double2*)out);
  else copy_greens_kernel<float2><<<1024, NT, 0, st>>>(s, (float2*)out);
  return hipGetLastError();
}
hipError_t launch_copy_state(const SysDev& s, double2* local_out, double* logw_out, int* status_out,
                             hipStream_t st) {
  copy_state_kernel<<<(s.W + NT - 1) / NT, NT, 0, st>>>(s, local_out, logw_out, status_out);
  return hipGetLastError();
}
