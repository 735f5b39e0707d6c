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
};
hipError_t launch_zgemm(const GemmParams& p, int prec, hipStream_t s);
int gemm_tile_count();

// Blocked Gaussian elimination on a per-walker augmented matrix [A | R] (M x M
// left block, nrhs right-hand sides starting at column rhs_off, row stride lda).
struct ElimParams {
  double2* aug; long long stride; int lda;
  int M, rhs_off, nrhs, W;
  int pivot;    // partial (row) pivoting
  int backsub;  // solve the upper triangle after the forward elimination
  double2* lndet;  // [W] sum of log pivots + i pi (row swaps); may be null
  int* status;     // [W] set to 2 on a zero or non-finite pivot; may be null
  int* piv;        // [W][ld] pivot rows (workspace)
  int ld;          // stride of piv
  double2* tri;    // [W][elim_tri_elems(M)] triangular-block inverses (workspace)
};
hipError_t launch_elim(const ElimParams& p, hipStream_t s);
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
  const short* grid;      // [grid_dim^3] basis index of an integer vector, -1 outside
  const int* flat;        // [M] flat offset of each basis vector in the lookup grid
  // state
  double2* Y; double2* Ti; double2* G; double2* aug;
  void* V; void* V2; void* V3; void* V4; void* E0; void* E1;  // complex128 or complex64
  void* Bk[3];            // Paterson-Stockmeyer blocks B_0..B_2 (complex128 or complex64)
  double2* Ynew;
  double* D; double* Dpi; int* perm; int* piv;
  double2* tri;           // [W][elim_tri_elems(M)]
  double2* r;             // [W][NQ] <rho_Q> per spin of the current G
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
  long long mat_stride;   // ld*ld
  long long aug_stride;   // ld*2*ld
};

hipError_t launch_init_state(const SysDev& s, hipStream_t st);
hipError_t launch_coef_v(const SysDev& s, const double2* fields, int k, int mixed, hipStream_t st);
hipError_t launch_greens_form(const SysDev& s, int k, hipStream_t st);
hipError_t launch_greens_post(const SysDev& s, int k, hipStream_t st);
hipError_t launch_weight(const SysDev& s, int k, double sum_lnLb, int init, hipStream_t st);
hipError_t launch_stab_perm(const SysDev& s, hipStream_t st);
hipError_t launch_stab_gather(const SysDev& s, hipStream_t st);       // E0 = Y[:, perm], aug right = E0^H
hipError_t launch_stab_finish_a(const SysDev& s, hipStream_t st);     // Y, D, Ru (E1) from the Cholesky step
hipError_t launch_stab_build_ti(const SysDev& s, hipStream_t st);     // aug = [Ru^T | Ti_pi^T]
hipError_t launch_stab_finish_b(const SysDev& s, hipStream_t st);     // Ti = (aug right)^T
hipError_t launch_energy(const SysDev& s, int rec, hipStream_t st);   // local energies (+ record)
hipError_t launch_energy_mean(const SysDev& s, const double2* local, const double* logw,
                              const int* status, double2* mean, hipStream_t st);
hipError_t launch_copy_greens(const SysDev& s, void* out, int dtype, hipStream_t st);
hipError_t launch_copy_state(const SysDev& s, double2* local_out, double* logw_out, int* status_out,
                             hipStream_t st);
