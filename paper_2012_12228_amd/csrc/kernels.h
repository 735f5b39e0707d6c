// Launch interfaces of the slice-path kernels (host <-> device boundary inside the library).
#pragma once
#include <hip/hip_runtime.h>

enum { GEMM_Z64 = 0, GEMM_C32 = 1, GEMM_C32_Z64B = 2 };

// Primary output: C = diag(rs) [alpha op(A) op(B) + beta C + cI I + c1 P1 + c2 P2 + c3 P3] diag(cs).
// Extra outputs X_e = cacc op(A) op(B) + cI I + c1 P1 + c2 P2 + c3 P3 (same layout as C, unscaled).
// C is m x n with inner size k; entries with m <= i < mpad or n <= j < npad are written as zero.
struct GemmOut { void* ptr; double cacc, cI, c1, c2, c3; };
struct GemmParams {
  const void* A; const void* B; void* C;
  const void* P1; const void* P2; const void* P3;
  const double* rs; const double* cs;
  long long sA, sB, sC, sP;  // walker strides in elements
  int lda, ldb, ldc, ldp;
  int m, n, k, mpad, npad, W;
  int opA, opB;              // 0 = as stored, 1 = conjugate transpose
  double alpha, beta, cI, c1, c2, c3;
  int nextra;                // 0..4 extra outputs
  GemmOut extra[4];
  int role;                  // 0 = propagator chain, 1 = elimination / stabilisation (separate kernel symbols)
  int tile;                  // tile shape index (0 .. gemm_tile_count()-1) for role 0
  int tiles_m, tiles_n;      // set by the launcher
  int skip0, skip1;          // role 1: rows [skip0, skip1) of C are not written
  int tri_a;                 // role 1: A is upper triangular (zero below the diagonal): k starts at the row tile
  int herm;                  // role 1: C is Hermitian (A^H A): only the tiles on and below the diagonal are
                             // computed, each one below also stored conjugate-transposed above
};
hipError_t launch_zgemm(const GemmParams& p, int prec, hipStream_t s);
// The mixed propagator's products on the BF16 matrix cores with three-way split operands
// (complex64 A; B complex128 when wide_b, else complex64; C as B); role 0, A and B as stored.
hipError_t launch_zgemm_bf16x6(const GemmParams& p, bool wide_b, hipStream_t s);
int gemm_tile_count();
bool gemm_tile_supported(int tile, int prec);   // shapes built for this precision
bool gemm_tile_walker_sized(int tile);           // one workgroup per walker (fills every CU at W >= 256)

// Blocked Gaussian elimination on a per-walker augmented matrix [A | R] (M x M
// left block, nrhs right-hand sides starting at column rhs_off, row stride lda).
struct ElimParams {
  double2* aug; long long stride; int lda;
  int M, rhs_off, nrhs, W;
  int pivot;    // partial (row) pivoting
  int backsub;  // solve: Gauss-Jordan to the solution in the right-hand block (else forward only)
  double2* lndet;  // [W] sum of log pivots + i pi (row swaps); may be null
  int* status;     // [W] set to 2 on a zero or non-finite pivot; may be null
  int* piv;        // [W][ld] pivot rows (workspace)
  int ld;          // stride of piv
  double2* tri;    // [W][elim_tri_elems(M)] inverse of the current pivot block (workspace)
};
hipError_t launch_elim(const ElimParams& p, hipStream_t s);
// Forward elimination (no pivoting, no back-substitution) of [L | R] with L lower triangular:
// the same result as launch_elim, the products over L's zero upper part skipped.
hipError_t launch_elim_lower(const ElimParams& p, hipStream_t s);
size_t elim_tri_elems(int M);

// Per-system constant tables and per-walker state, as device pointers.
struct SysDev {
  int M, ld, NQ, W, n, grid_dim;
  int grid_c0;            // flat lookup offset of the zero vector
  double dtau, kscale, e_madelung;
  // tables
  const int* idx;         // [M][M] momentum-transfer index of K_i - K_j, -1 on the diagonal
  const int* neg;         // [NQ] index of -Q
  const double* vq;       // [NQ] 4 pi / (Omega Q^2)
  const double* sq;       // [NQ] sqrt(pi dtau / (Omega Q^2))
  const double* eps;      // [ld] |K|^2 / 2 (0 beyond M)
  const double* kh;       // [ld] exp(-dtau/2 (lambda eps + h - mu)) (0 beyond M)
  const double* lnbt;     // [ld] -dtau (eps - mu_T)
  const int* qptr;        // [NQ+1] CSR offsets of the pairs of each Q
  const int* qpair;       // [M(M-1)] flat index r*ld + p of G_{r p} for pairs K_p - K_r = Q
  // the same pairs by blocks of rq_rows rows of G: block b's pairs grouped by Q (rows ascending
  // within a Q), each as (r - b rq_rows) ld + p, with CSR offsets rbptr[b (NQ+1) + q]
  const int* rbptr;       // [rq_nblk (NQ+1)]
  const int* rbidx;       // [M(M-1)]
  int rq_rows, rq_nblk;
  int rq_gather;          // 1: r_Q by the per-Q gather kernel even where the LDS-streamed one applies
  const short* grid;      // [grid_dim^3] basis index of an integer vector, -1 outside
  const int* flat;        // [M] flat offset of each basis vector in the lookup grid
  // state
  double2* Y; double2* Ti; double2* G; double2* aug;
  void* V; void* V2; void* V3; void* V4; void* E0; void* E1;  // complex128 or complex64
  void* Bk[5];            // Paterson-Stockmeyer blocks B_0..B_{nb-2} (complex128 or complex64)
  double2* Ynew;
  double* D; double* Dpi; int* perm; int* piv;
  double2* tri;           // [W][elim_tri_elems(M)]
  double2* r;             // [W][NQ] <rho_Q> per spin of the current G
  double2* rb;            // [W][NQ] <rho_Q> that the force bias uses (= r, or of Gt)
  double2* Gt;            // [W][ld][ld] G of the constraint product (= G, or the eq. ztfix one)
  double2* cq;            // [W][NQ] shifted coefficients c_Q of the current slice
  double2* expo;          // [W] weight exponent of the current slice
  double2* ell;           // [W] ln det(I + A_k)
  double2* lndetT;        // [W] ln det T
  double2* lndetX;        // [W] ln det of the eliminated block
  double* logw; int* status;
  double2* slice_lnS; double* slice_theta;   // [W][n] per-slice trace
  double2* exch;          // [W][ld] exchange partial sums
  double2* local;         // [W][4]
  double2* rec_E;         // [nrec_max][W][4]
  double* rec_logw;       // [nrec_max][W]
  int* rec_status;        // [nrec_max][W]
  double* scratch;        // [W][ld] reals
  double* tnorm;          // [W][16] per 64-column chunk: max column 1-norm of V (0..7) and of V^4 (8..15)
  int* pop_parent;        // [W] population control: walker copied into each slot
  double* pop_logw;       // [W] population control: new ln w of each slot
  int taylor_deg;         // degree of the Taylor polynomial of e^V (a multiple of 4)
  double taylor_tol;      // a walker whose truncation bound exceeds this is flagged numeric
  // low-rank truncation (eq. thresh), or lr_order == null: the kept left plane waves are the first
  // lr_mL of lr_order (decreasing ln B_T); lr_pos is its inverse; lr_thr counts the right rank
  const int* lr_order;    // [M]
  const int* lr_pos;      // [M]
  int lr_mL;              // left rank of the current solve
  double lr_thr, lr_lnthr;
  int* lr_mR;             // [W][n+1] right rank at every Green's function formation, or null
  double2* rec_c;         // [W][n][NQ] shifted coefficients c_Q of every slice (path record), or null
  double2* rec_trG;       // [W][n+1] tr G_k of every slice, or null
  int w_off, rec_W;       // walker offset of this view and walker count of the record arrays
  long long mat_stride;   // ld*ld
  long long aug_stride;   // ld*2*ld
};

// Frozen-path tangent state of one system: the doubled product [[R, dR], [0, R]] (2M x 2M,
// stored with leading dimension ld2) in the form Yd diag(Dd) Td, re-factorised every slice.
// dd is the doubled system seen as a SysDev (M = 2M, ld = ld2) so that the stabilisation and
// elimination launchers serve it unchanged.
struct TanDev {
  int M2, ld2;
  SysDev dd;              // Y = Yd, D = Dd, E0/E1/aug/perm/piv/tri/Dpi doubled scratch, status = tstat
  double2* Ydn;           // [W][ld2][ld2] product before re-factorisation
  double2* Td;            // [W][ld2][ld2]
  double2* Bcat;          // [W][ld][ld2] = [B | dB] of the current slice (rows < M)
  double2* Fcat;          // [W][ld][ld2] = [dB B_T^{-1} | B B_T^{-1} - I]
  double2* Gst;           // [W][ld2][ld] = cyclic Green's function rows stacked: [Gc_11 ; Gc_12]
  double2* dG;            // [2][W][ld][ld] dG at tau = beta along mu and lambda
  double2* exch;          // [W][ld]
  double* dlnw;           // [W][2]
  double2* dloc;          // [W][2][4] (dE1, dE2, dE, dN) along mu and lambda
  int* alive;             // [W]
  int* tstat;             // [W] 0, or 2 when a doubled factorisation broke down
  double2* lndet_dummy;   // [W] (the stabilisation records a permutation parity there)
  long long bc_stride;    // ld*ld2
  long long gs_stride;    // ld2*ld
  // pathwise mode (raw fields fixed, force bias recomputed)
  double2* Tid;           // [W][ld2][ld2] inverse of Td (carried like the forward's T^{-1})
  double2* Gd;            // [W][ld2][ld2] literal doubled Green's function at the current slice
  double* lnbt2;          // [ld2] ln diag B_T repeated for both halves
  double2* lndetX2;       // [W] (the elimination records its ln det there)
  // the cyclic doubled solve's own augmented system and elimination scratch, so that it can run
  // beside the re-factorisation of the doubled product (which uses dd.aug, dd.piv, dd.tri)
  double2* caug;          // [W][ld2][2 ld2]
  int* cpiv;              // [W][ld2]
  double2* ctri;          // [W][elim_tri_elems(2M)]
  double2* Gk; double2* dGk;   // [W][ld][ld] G_k and dG_k (blocks of Gd)
  double2* rk; double2* drk;   // [W][NQ] r_Q of G_k and its derivative
  double2* dcq;           // [W][NQ] derivative of the shifted coefficients
  double2* dexpo;         // [W] derivative of the exponent of eq. import for the current slice
  double2* dV; double2* dV2; double2* dV3; double2* dV4;   // [W][ld][ld] derivatives of V^j
  double2* dE0; double2* dE1;                               // [W][ld][ld] Horner derivatives
  double2* dBk[5];        // [W][ld][ld] derivatives of the Paterson-Stockmeyer blocks
};

hipError_t launch_coef_replay(const SysDev& s, int k, hipStream_t st);             // V from rec_c[k]
hipError_t launch_tan_init(const SysDev& s, const TanDev& t, hipStream_t st);
hipError_t launch_tan_prep(const SysDev& s, const TanDev& t, const double2* B, hipStream_t st);
hipError_t launch_cyc_form(const SysDev& s, const TanDev& t, int k, int literal, hipStream_t st);
hipError_t launch_cyc_post(const SysDev& s, const TanDev& t, int k, int literal, hipStream_t st);
hipError_t launch_tan_weight(const SysDev& s, const TanDev& t, int k, hipStream_t st);
hipError_t launch_permute_rows(const TanDev& t, hipStream_t st);                 // dd.E0 = Td[perm, :]
hipError_t launch_energy_tangent(const SysDev& s, const TanDev& t, int dir, hipStream_t st);
hipError_t launch_tan_mean(const SysDev& s, const TanDev& t, const double* cot, double2* jac,
                           double* grad, double2* walker, hipStream_t st);
// pathwise mode
hipError_t launch_pw_reset(const SysDev& s, const TanDev& t, hipStream_t st);   // Yd, Td, Tid = I, Dd = 1
hipError_t launch_pw_extract(const SysDev& s, const TanDev& t, double2* dG_out, hipStream_t st);  // Gk, dGk
hipError_t launch_pw_coef(const SysDev& s, const TanDev& t, const double2* fields, int k, hipStream_t st);
struct PwBlocks { int nb; double c[6][4]; };   // dB_k = c1 dV + c2 dV2 + c3 dV3 (+ c0 dV4 for the top)
hipError_t launch_pw_blocks(const SysDev& s, const TanDev& t, const PwBlocks& b, hipStream_t st);
hipError_t launch_pw_prep(const SysDev& s, const TanDev& t, const double2* B, const double2* KdEK, int dir,
                          hipStream_t st);
hipError_t launch_pw_weight(const SysDev& s, const TanDev& t, int k, int dir, hipStream_t st);
hipError_t launch_kink_flags(const SysDev& s, double threshold, int* flags, hipStream_t st);

// Truncation check of the Taylor polynomial of e^V: per-chunk column 1-norms of V and V^4 into
// tnorm (the weight kernel turns them into a bound on the remainder and flags the walker).
hipError_t launch_taylor_norms(const SysDev& s, int mixed, hipStream_t st);
// Lower Paterson-Stockmeyer blocks B_k = sum_{r<4} c[k][r] V^r (identity for r = 0) for k < nlo,
// written to s.Bk[k] (used when the V^4 product's epilogue cannot write them all).
struct TaylorLow { int nlo; double c[2][4]; };
hipError_t launch_taylor_blocks(const SysDev& s, int mixed, const TaylorLow& t, hipStream_t st);
// Population control (method 0 comb, 1 pair branch) with uniforms u; parent / newlogw [W].
hipError_t launch_population_control(const SysDev& s, int method, const double* u, int* parent, double* newlogw,
                                     hipStream_t st);
size_t pop_select_lds(int W);
// Weighted statistics of the nrec energy records into stats [nrec][8] (and their averages into avg [3]).
hipError_t launch_record_stats(const SysDev& s, int nrec, double* stats, double* avg, hipStream_t st);
hipError_t launch_init_state(const SysDev& s, hipStream_t st);
hipError_t launch_coef_v(const SysDev& s, const double2* fields, int k, int mixed, hipStream_t st);
hipError_t launch_fill_v(const SysDev& s, void* V, int mixed, hipStream_t st);   // V from s.cq
// G of (I + B_T^lexp R)^{-1}: the transposed augmented system, and G from its solution
hipError_t launch_greens_form(const SysDev& s, int lexp, hipStream_t st);
hipError_t launch_greens_post(const SysDev& s, int lexp, hipStream_t st);
hipError_t launch_lr_rank(const SysDev& s, int k, hipStream_t st);   // right rank into lr_mR[w][k]
hipError_t launch_rq(const SysDev& s, hipStream_t st);                // r_Q of s.G into s.r
hipError_t launch_weight(const SysDev& s, int k, double sum_lnLb, int init, hipStream_t st);
int rq_block_elems();     // complex entries of G per row block of the r_Q kernel (rows * ld at most)
hipError_t launch_stab_perm(const SysDev& s, hipStream_t st);
hipError_t launch_stab_gather(const SysDev& s, hipStream_t st);       // E0 = Y[:, perm], aug right = E0^H
hipError_t launch_stab_finish_a(const SysDev& s, hipStream_t st);     // Y, D, Ru (E1) from the Cholesky step
hipError_t launch_stab_build_ti(const SysDev& s, hipStream_t st);     // aug = [Ru^T | Ti_pi^T]
hipError_t launch_stab_finish_b(const SysDev& s, hipStream_t st);     // Ti = (aug right)^T
hipError_t launch_energy(const SysDev& s, int rec, hipStream_t st);   // local energies (+ record)
// <rho(Q) rho(-Q)> per walker into out [W][NQ] (X: [W][ld][ld] scratch), weighted mean into mean [NQ]
hipError_t launch_density_correlation(const SysDev& s, double2* X, double2* out, double2* mean, hipStream_t st);
hipError_t launch_energy_mean(const SysDev& s, const double2* local, const double* logw,
                              const int* status, double2* mean, hipStream_t st);
hipError_t launch_copy_greens(const SysDev& s, void* out, int dtype, hipStream_t st);
hipError_t launch_copy_state(const SysDev& s, double2* local_out, double* logw_out, int* status_out,
                             hipStream_t st);
