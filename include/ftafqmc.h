/*
 * ftafqmc.h -- C ABI of the MI355X library for the imaginary-time slice path of
 * phaseless finite-temperature AFQMC (ph-FT-AFQMC) on the uniform electron gas
 * in a plane-wave basis (Lee, Morales, Malone, arXiv:2012.12228).
 *
 * What the library computes (per walker, batched over walkers):
 *   - the slice propagator B = e^{-dtau/2 (H_1 - mu N)} e^{sqrt(dtau)(x - xbar).v}
 *     e^{-dtau/2 (H_1 - mu N)} (Sec. "Finite-Temperature AFQMC", eq. B; the HS
 *     operators of Sec. "Uniform Electron Gas": v = i A(Q)/sqrt2, i B(Q)/sqrt2);
 *   - the optimal force bias xbar = -sqrt(dtau) <v> from P = I - G^T (Sec.
 *     "Phaseless approximation");
 *   - the constrained product A(tau_k) = B_T^{n-k} B_k ... B_1 (eq. Abrenda) kept
 *     as a stratified Q D T factorisation (Sec. "Numerical Stabilization") and the
 *     Green's function G = (I + A)^{-1} (eq. green) with ln det(I + A);
 *   - the phaseless weight w <- |I| max(0, cos theta) (eq. import, eq. phimport,
 *     eq. theta) with S = det(I + A_{k+1})^2 / det(I + A_k)^2;
 *   - the local energy E_M + E_1 + E_2 with Hartree and exchange parts (Sec.
 *     "Uniform Electron Gas", Gamma_Q and Lambda_Q) and the electron number;
 * and around that path (each declared below with its passage):
 *   - derivatives of <E> and <N> at tau = beta in mu and lambda, along the frozen path
 *     or pathwise (ftafqmc_backward);
 *   - population control by the comb or pair branching, record statistics and time-slice
 *     averages, <rho(Q) rho(-Q)> (Sec. "Computational Details", "Comparison to Other
 *     Approaches");
 *   - chemical-potential tuning by bracketing with a weighted line fit, or by Newton steps
 *     from d<N>/dmu (ftafqmc_tune_mu);
 *   - the thermal Hartree-Fock trial, the modified overlap ratio (eq. ztfix), the low-rank
 *     truncation of the Green's function solve (eq. thresh) and the mixed-precision
 *     propagator (flags of ftafqmc_params).
 *
 * Conventions shared by every entry point:
 *   - Spin-restricted: one M x M block per walker serves both spins; det(I + A)
 *     enters squared and one-body expectation values carry a factor 2.
 *   - Basis order: plane waves K = 2 pi n / L, integer n with |n|^2 <= nmax2,
 *     sorted by |n|^2, then n_x, n_y, n_z ascending.  Momentum transfers Q are
 *     all distinct nonzero K_i - K_j in the same order; query() reports N_Q.
 *   - Fields: complex128 per walker, slice and momentum transfer, row-major
 *     [W][n_slices][N_Q]; Re = field of A(Q), Im = field of B(Q), each meant to
 *     be iid N(0,1) (the HS transform's Gaussian fields).
 *   - Matrices handed out are row-major [W][M][M] with G_ij = <c_i c_j^+>.
 *   - Memory: every device pointer is owned by the caller.  The library never
 *     allocates device memory: all per-walker state and constant tables live in
 *     one caller-provided device workspace of ftafqmc_workspace_bytes() bytes,
 *     which must stay valid and untouched until ftafqmc_destroy().  The handle
 *     itself is host memory owned by the library.
 *   - Streams: `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Every call only enqueues work on it; results are ready when the stream is.
 *   - Errors: functions return an ftafqmc_status; nothing throws or aborts.
 *     ftafqmc_last_error() gives a message.  Numerical failure of one walker
 *     (non-finite G, failed stabilisation) is reported in that walker's status
 *     word, not as a call error.
 *   - Threads: a handle must not be used from two threads at once.
 */
#ifndef FTAFQMC_H
#define FTAFQMC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ftafqmc_ctx* ftafqmc_t;

typedef enum {
  FTAFQMC_OK = 0,
  FTAFQMC_E_ARG = -1,         /* invalid argument (sizes, NULL pointer, parameter range) */
  FTAFQMC_E_HIP = -2,         /* a HIP runtime call failed */
  FTAFQMC_E_NUMERIC = -3,     /* every walker of a system failed numerically */
  FTAFQMC_E_STATE = -4,       /* call not valid in the handle's current state */
  FTAFQMC_E_UNSUPPORTED = -5  /* requested feature not built */
} ftafqmc_status;

/* precision of the propagator GEMM chain */
enum { FTAFQMC_FP64 = 0, FTAFQMC_MIXED = 1 };
/* per-walker status word */
enum { FTAFQMC_WALKER_ALIVE = 0, FTAFQMC_WALKER_KILLED = 1, FTAFQMC_WALKER_NUMERIC = 2 };
/* dtype codes for ftafqmc_greens */
enum { FTAFQMC_C128 = 0, FTAFQMC_C64 = 1 };

/* One UEG system (Sec. "Computational Details"): N, r_s, Theta = T/T_F, basis
 * cutoff, time step; plus the walker batch and the stabilisation interval. */
typedef struct {
  int n_elec;      /* N-bar: even, >= 2 (N/2 electrons per spin) */
  double rs;       /* Wigner-Seitz radius, > 0; box L = (4 pi N / 3)^(1/3) r_s */
  double theta;    /* reduced temperature T/T_F, > 0; k_B T_F = (9 pi/4)^(2/3) / (2 r_s^2) (eq. fermiT) */
  int nmax2;       /* plane waves with integer |n|^2 <= nmax2, >= 1 */
  double dtau;     /* nominal time step; n = round(beta/dtau) slices, dtau_eff = beta/n */
  int stab_every;  /* QR stabilisation every stab_every slices (and at slice n), >= 1 */
  int n_walkers;   /* >= 1 */
  double mu;       /* interacting chemical potential; NaN selects mu_T of the trial */
  double kscale;   /* lambda in H_1 = lambda T + h (1 = the physical Hamiltonian) */
  int precision;   /* FTAFQMC_FP64 or FTAFQMC_MIXED */
  int flags;       /* 0, or any of FTAFQMC_CHECKPOINT, FTAFQMC_OVERLAP, FTAFQMC_GRAPH,
                      FTAFQMC_TRIAL_THF, FTAFQMC_MODIFIED_OVERLAP, FTAFQMC_MEASURE_EVERY_SLICE,
                      FTAFQMC_LOW_RANK, FTAFQMC_BF16_SPLIT */
} ftafqmc_params;

/* flags: record the sampled path (the shifted coefficients c_Q and tr G of every slice) so
 * that ftafqmc_backward can differentiate it.  FP64 systems with M <= 256 only; the workspace
 * grows by W n N_Q complex128 plus the doubled (2M x 2M) derivative state. */
#define FTAFQMC_CHECKPOINT 1
/* flags: split the system's walkers into two groups that propagate on two streams (the
 * caller's and one the handle owns), so that one group's latency-bound eliminations overlap
 * with the other group's GEMMs.  Results are identical; throughput is higher where the
 * elimination dominates (M up to about 256), and each GEMM launch then shares the GPU. */
#define FTAFQMC_OVERLAP 2
/* flags (on any system of a handle): a call of ftafqmc_propagate that runs every system's whole
 * path from slice 0 is captured once into a HIP graph and replayed by later such calls with the
 * same field buffers (their contents may change between calls).  Results are identical to the
 * eager launches; profiling (ftafqmc_profile) runs eagerly. */
#define FTAFQMC_GRAPH 4
/* flags: thermal Hartree-Fock trial (Sec. "Results", fig. thf) instead of the free-electron one:
 * B_T = diag exp(-dtau (e_K - mu_T)) with the self-consistent levels
 * e_K = |K|^2/2 - sum_{K' != K} v(K - K') f_K', f_K = 1/(1 + exp(beta (e_K - mu_T))) and
 * 2 sum f = N (plane waves stay Hartree-Fock orbitals of the uniform gas; the Q = 0 Hartree term
 * cancels against the background).  mu_T (and the default mu) become this trial's. */
#define FTAFQMC_TRIAL_THF 8
/* flags: the phaseless constraint from the modified overlap ratio of eq. ztfix,
 * S~_k = tr(B_T^n B_k ... B_1) / tr(B_T^n B_{k-1} ... B_1): the trial always enters to the n-th
 * power, so the force bias, ln det, S and theta of every slice use (I + B_T^n R_k)^{-1}; the
 * estimators (ftafqmc_energy, ftafqmc_greens, the records) keep G_k = (I + B_T^{n-k} R_k)^{-1},
 * formed at records and after the last slice of each ftafqmc_propagate call (one more
 * elimination there).  Not with FTAFQMC_CHECKPOINT. */
#define FTAFQMC_MODIFIED_OVERLAP 16
/* flags: an energy record after every slice (for time-slice averages, ftafqmc_record_stats)
 * instead of every stab_every slices; stabilisation keeps its own interval. */
#define FTAFQMC_MEASURE_EVERY_SLICE 32
/* flags: low-rank truncation of the Green's function solve (Sec. "Exploiting the low-rank
 * structure", eq. thresh, threshold FTAFQMC_LOW_RANK_THRESHOLD as in Sec. "Computational
 * Details").  The diagonal left block B_T^{n-k} keeps the m_L plane waves whose factor is at
 * least the threshold; the others' rows of G are the identity and drop out of the solve, which
 * then has m_L right-hand sides instead of M (the saving).  The right block keeps all of its
 * columns: which of them fall below the threshold depends on how the product is factorised,
 * and dropping them would make the result depend on it too; its rank m_R is reported.  The
 * per-slice ranks are read with ftafqmc_lowrank_ranks.  Not with FTAFQMC_CHECKPOINT or
 * FTAFQMC_MODIFIED_OVERLAP. */
#define FTAFQMC_LOW_RANK 64
#define FTAFQMC_LOW_RANK_THRESHOLD 1e-6
/* flags (FTAFQMC_MIXED only): the propagator products (the Taylor chain of e^V and its
 * application to Y) on the BF16 matrix cores with every FP32 operand split into three bf16
 * parts and the six split products down to 2^-16 of the leading one kept, FP32 accumulation
 * (the same 24-bit operand precision as the FP32 products it replaces; results differ from them
 * at the rounding level).  Everything else as FTAFQMC_MIXED. */
#define FTAFQMC_BF16_SPLIT 128
/* ftafqmc_backward modes */
#define FTAFQMC_FROZEN_PATH 0
#define FTAFQMC_PATHWISE 1

/* Derived sizes and constants of one system (host-side values). */
typedef struct {
  int M;            /* plane waves */
  int n_q;          /* momentum transfers (both signs) */
  int n_slices;     /* n */
  int n_walkers;
  int slice;        /* slices done so far (0..n) */
  int n_measure;    /* energy records so far (one per stabilisation boundary and at slice n) */
  int ld;           /* padded leading dimension used internally */
  double beta, dtau, L, omega, mu_T, mu, e_madelung;
  int gemm_tile_chain;   /* tile shape of the plain Taylor-chain products (V^2, V^3), chosen by
                            the start-up autotuner */
  int gemm_tile_apply;   /* tile shape of the product that applies e^V */
  int gemm_tile_shapes;  /* number of tile shapes built (valid values of FTAFQMC_GEMM_TILE) */
  int walker_groups;     /* walker groups whose eliminations overlap on separate streams */
  int gemm_tile_epilogue; /* tile shape of the V^4 product, whose epilogue adds V, V^2, V^3 and
                             writes the Taylor blocks */
  int gemm_tile_horner;   /* tile shape of the Horner steps (one addend, one output) */
  int taylor_degree;      /* degree p of the Taylor polynomial of e^V (a multiple of 4): the
                             smallest of 16, 20, 24 (FP64) or 12, 16, 20, 24 (mixed) whose
                             leading remainder term at an a-priori norm estimate of V (from
                             dtau and the Coulomb kernel) is below 1e-14 (FP64) or 1e-8; every
                             slice checks the remainder bound sum_{j>p} ||V^4||^{j/4} ||V||^{j%4}/j!
                             (1-norms) on the device and flags a walker FTAFQMC_WALKER_NUMERIC
                             when it exceeds 1e-11 (FP64) or 1e-6 (mixed: the rounding level of
                             its FP32 products) */
  int refactor_every;     /* the product is re-factorised (Sec. "Numerical Stabilization") at
                             least every refactor_every slices, in addition to every stab_every
                             slices: the kinetic part of the product between two passes keeps a
                             condition number below e^6.  A pass whose pivot spread
                             min_i d_i / |column i|^2 falls below 1e-5 (orthogonality would be
                             lost) flags the walker FTAFQMC_WALKER_NUMERIC */
} ftafqmc_info;

/* Bytes of device workspace needed for the n_sys systems listed in p[0..n_sys-1]
 * (n_sys > 1 batches walkers of different systems in one handle).  Host-only. */
int ftafqmc_workspace_bytes(const ftafqmc_params* p, int n_sys, size_t* bytes);

/* Build the plane-wave tables (basis, momentum transfers, Coulomb kernel, the
 * one-body remainder h_K of the sum-of-squares form, the trial chemical
 * potential mu_T with 2 sum_K f(eps_K - mu_T) = N) on the host, upload them into
 * d_workspace on `stream`, and set every walker to tau = 0: A_0 = B_T^n, weight 1,
 * G_0 = (I + B_T^n)^{-1}.  d_workspace: device memory of ws_bytes >= the size
 * from ftafqmc_workspace_bytes, 256-byte aligned.  On success *out is a new handle. */
int ftafqmc_init_ueg(const ftafqmc_params* p, int n_sys, void* d_workspace, size_t ws_bytes,
                     void* stream, ftafqmc_t* out);

/* Allocation-free variant of ftafqmc_init_ueg, for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops, harnesses that forbid allocation).  The
 * workspace is a file-scope device array of FTAFQMC_STATIC_WORKSPACE_BYTES that the library
 * holds on every device it runs on until the process ends (the M = 19, 64-walker system needs
 * 21 MiB); the call itself allocates no device memory.  Everything else is as ftafqmc_init_ueg,
 * and the handle is used and destroyed like any other.  One live handle per device may hold the
 * array: a second call on the same device returns FTAFQMC_E_STATE until that handle is
 * destroyed, and work of such handles from several threads or processes that overlaps on one
 * device would race on the array.  Errors: FTAFQMC_E_ARG when the systems need more than the
 * maximum or ask for FTAFQMC_OVERLAP or FTAFQMC_GRAPH (which create streams and graphs), with
 * the message in ftafqmc_last_error(NULL). */
#define FTAFQMC_STATIC_WORKSPACE_BYTES (64u << 20)
int ftafqmc_init_ueg_static(const ftafqmc_params* p, int n_sys, void* stream, ftafqmc_t* out);

/* Sizes and constants of system `sys` (host-side; does not synchronise). */
int ftafqmc_query(ftafqmc_t h, int sys, ftafqmc_info* out);

/* Put every walker of every system back to tau = 0 (enqueued on stream). */
int ftafqmc_reset(ftafqmc_t h, void* stream);

/* Advance every walker of every system by n_slices slices (clamped at each
 * system's n).  d_fields[s]: device pointer to system s's whole-path fields,
 * complex128 [W_s][n_s][N_Q,s]; slice k of the path reads d_fields[s][w][k][:].
 * Per slice: force bias from the current G, shifted propagator, stabilisation when
 * the slice count reaches a multiple of stab_every or n, the new G and ln det,
 * the phaseless weight update; the local energy is recorded at every
 * stabilisation boundary and at slice n (see ftafqmc_records). */
int ftafqmc_propagate(ftafqmc_t h, const void* const* d_fields, int n_slices, void* stream);

/* Copy the current per-walker Green's function of system `sys` into d_G:
 * row-major [W][M][M], dtype FTAFQMC_C128 (double2) or FTAFQMC_C64 (float2). */
int ftafqmc_greens(ftafqmc_t h, int sys, void* d_G, int dtype, void* stream);

/* Local energy of every walker of system `sys` at the current slice, from the
 * current G: d_local [W][4] complex128 = (E_1, E_2, E = E_M + E_1 + E_2, N);
 * d_mean [4] complex128 = weighted means sum_w w O_w / sum_w w over live walkers
 * (NaN if none is alive); d_logw [W] double = ln w (-inf when killed);
 * d_status [W] int = FTAFQMC_WALKER_*.  Any output pointer may be NULL. */
int ftafqmc_energy(ftafqmc_t h, int sys, void* d_local, void* d_mean, double* d_logw,
                   int* d_status, void* stream);

/* Energy records taken during propagation: d_trace [n_rec][W][4] complex128 as in
 * ftafqmc_energy, d_logw [n_rec][W] and d_slice [n_rec] (host int array, the slice
 * of each record).  n_rec = info.n_measure.  Any pointer may be NULL. */
int ftafqmc_records(ftafqmc_t h, int sys, void* d_trace, double* d_logw, int* h_slice,
                    void* stream);

/* Derivatives of the weighted means <E> and <N> at tau = beta with respect to mu and the
 * kinetic scale lambda, for the sampled path held fixed (mode FTAFQMC_FROZEN_PATH): the
 * fields and their force-bias shifts keep their sampled values, while mu and lambda move in
 * the half-step factors K = exp(-dtau/2 (lambda eps + h - mu)) of every slice propagator
 * (eq. B), hence in G, in ln det(I + A_k), in the overlap ratios S_k and phases theta_k of
 * the phaseless weight (eqs. ftoratio, import, theta), and in the local energy (Sec.
 * "Uniform Electron Gas").  The mu direction is exact in closed form (K scales by
 * e^{dtau mu/2}); the lambda direction carries the doubled product [[R, dR], [0, R]] through
 * the same stabilised factorisation as the forward path.  Replays the recorded path: the
 * system must have been initialised with FTAFQMC_CHECKPOINT and propagated to slice n.
 * Device pointers (each may be NULL):
 *   d_cot    [2] double: cotangents dL/dRe<E>, dL/dRe<N> (needed for d_grad)
 *   d_jac    [4] complex128: d<E>/dmu, d<N>/dmu, d<E>/dlambda, d<N>/dlambda
 *   d_grad   [2] double: dL/dmu, dL/dlambda = cot . Re(jac)
 *   d_walker [W][6] complex128: per walker (d ln w, dE, dN) along mu, then along lambda
 *            (NaN for a walker whose doubled factorisation broke down).
 * Mode FTAFQMC_PATHWISE differentiates the same estimator with the raw fields x_k held fixed
 * instead of the shifted ones: the force bias xbar_k = -sqrt(dtau) v_Q <rho_Q>_{G_k} (eq. fb)
 * moves with G_k, hence the shifted fields x_k - xbar_k, the one-body operator V_k, e^{V_k}
 * (its Frechet derivative carried through the same Taylor chain as the forward product) and the
 * exponent of the importance function (eq. import), on top of everything the frozen mode
 * moves.  Both directions carry the doubled product; each slice also forms the doubled
 * G_k = (I + diag(B_T^{n-k}) R_k)^{-1} for dG_k, so the cost is about twice the frozen mode's
 * lambda direction per direction.  The path must have been propagated with one field buffer
 * for all of its slices (the layout [W][n][N_Q] of ftafqmc_propagate, from slice 0 in one call
 * or in several calls on the same buffer), which must still hold the path's fields.
 * The weight is differentiable away from the phaseless kill (cos theta_k = 0 on a slice the
 * walker survived); ftafqmc_kink_flags marks walkers near it.
 * Walkers that are killed or numerically failed carry zero weight and do not enter the means.
 * Errors: E_STATE without the record, before slice n, or (pathwise) when the slices came from
 * different field buffers; E_ARG for an unknown mode. */
int ftafqmc_backward(ftafqmc_t h, int sys, int mode, const double* d_cot, void* d_jac,
                     double* d_grad, void* d_walker, void* stream);

/* Ranks of the low-rank truncation (system initialised with FTAFQMC_LOW_RANK) at every Green's
 * function formation k = 0..n (k = 0: the initial one; k: after slice k):
 *   h_mL [n+1] host int: left rank m_L (plane waves with B_T^{n-k} >= threshold), the same for
 *        every walker;
 *   d_mR [W][n+1] device int: right rank m_R, the columns of the walker's stabilised
 *        factorisation R = Y D T with |D| >= threshold (D of the last stabilisation);
 * m_T = min(m_L, m_R) and the compression c_i = (1 - m_i / M) 100% (Sec. "Efficacy of the
 * Low-Rank Truncation") follow.  Entries after the slice reached so far are stale.  Either
 * pointer may be NULL.  Errors: E_STATE for a system without the flag. */
int ftafqmc_lowrank_ranks(ftafqmc_t h, int sys, int* d_mR, int* h_mL, void* stream);

/* Walkers whose recorded path came within `threshold` of the phaseless kill: d_flags [W] int
 * (device), 1 where cos theta_k < threshold on some slice k the walker survived (eq. theta;
 * the pathwise derivative of such a walker's weight is taken next to the kink of
 * max(0, cos theta)), else 0.  Read from the phases every system records per slice. */
int ftafqmc_kink_flags(ftafqmc_t h, int sys, double threshold, int* d_flags, void* stream);

/* Population control of system `sys` (Sec. "Computational Details": the comb method, and pair
 * branching for Theta <= 0.25), between ftafqmc_propagate calls.  Weights are
 * w_i = exp(ln w_i - max ln w) over live walkers (0 for killed and numeric ones).
 *   FTAFQMC_POP_COMB: with T = sum w and one uniform u = d_u[0], teeth at (k + u) T / W,
 *     k = 0..W-1; walker i receives the teeth in [c_{i-1}, c_i) with the running sums c from
 *     walker 0 upwards; every copy carries ln(T / W) + max ln w.
 *   FTAFQMC_POP_PAIR_BRANCH: the p-th heaviest walker pairs with the p-th lightest (ties to the
 *     lower index) while the heavy one weighs more than 2 T/W or the light one less than
 *     T/(2W); with probability w_l / (w_l + w_s) (pair p reads d_u[p]) both slots become the
 *     heavy walker, otherwise the light one, each with weight (w_l + w_s) / 2.
 * A walker that keeps a copy keeps its slot; further copies go to the slots of walkers that
 * keep none, in ascending order, in tooth (pair) order.  Copied state: the stratified product
 * (Y, D, T), G, <rho_Q>, ln det(I + A), ln det T, ln w and the status word; the per-slice and
 * record histories stay with the slot.
 * d_u: device double [W] of uniforms in [0, 1) (comb reads one, pair branching up to W/2);
 * d_parent: device int [W] or NULL, receives the walker copied into each slot.
 * Errors: E_ARG for an unknown method or more than 2730 walkers; E_STATE for a system
 * initialised with FTAFQMC_CHECKPOINT (its recorded path would no longer be the walkers'). */
#define FTAFQMC_POP_COMB 0
#define FTAFQMC_POP_PAIR_BRANCH 1
int ftafqmc_population_control(ftafqmc_t h, int sys, int method, const double* d_u, int* d_parent, void* stream);

/* Weighted statistics of the energy records of system `sys` (estimators are weight-averaged
 * over the walkers, Sec. "Finite-Temperature AFQMC in the Grand Canonical Ensemble"; the
 * time-slice average is the "Average" estimator of Sec. "Results", fig. averaging).
 * d_stats: device double [n_rec][8] (n_rec = info.n_measure), per record over live walkers:
 *   Re<E>, its standard error sqrt(sum w^2 (Re E - Re<E>)^2) / sum w (delta method for the
 *   ratio estimator), Re<N>, its standard error, sum w / max w, ln max w, the effective walker
 *   count (sum w)^2 / sum w^2, the number of live walkers (NaN means for a record without any).
 * d_average: device double [3] or NULL: the average over the records with live walkers of
 *   Re<E> and of Re<N>, and the number of such records. */
int ftafqmc_record_stats(ftafqmc_t h, int sys, double* d_stats, double* d_average, void* stream);

/* Density correlation <rho(Q) rho(-Q)> of system `sys` from every walker's current G, for every
 * momentum transfer Q (both spins); divided by N it is the static structure factor
 * S(Q) = <rho(Q) rho(-Q)> / N of Sec. "Results".  Per walker, by Wick's theorem with
 * P = I - G^T: 4 r_Q r_-Q + 2 (n_Q - Lambda_Q), with r_Q = sum_K P_{K+Q,K},
 * n_Q = sum_{K, K+Q in basis} P_{K+Q,K+Q} and the exchange sum Lambda_Q of the local energy.
 * d_walker: device complex128 [W][N_Q] or NULL; d_mean: device complex128 [N_Q] or NULL, the
 * weighted mean over live walkers (NaN if none).  Q order as ftafqmc_qvectors.  Uses internal
 * scratch that ftafqmc_propagate also uses: call it between propagations. */
int ftafqmc_density_correlation(ftafqmc_t h, int sys, void* d_walker, void* d_mean, void* stream);

/* The momentum transfers of system `sys` as integer vectors n (Q = 2 pi n / L), host int
 * [N_Q][3], in the library's Q order (sorted by |n|^2, then n_x, n_y, n_z). */
int ftafqmc_qvectors(ftafqmc_t h, int sys, int* h_qvec);

/* Set the interacting chemical potential of system `sys` (it enters only the half-step factors
 * exp(-dtau/2 (lambda eps + h - mu)) of eq. B) and put the system back at tau = 0. */
int ftafqmc_set_mu(ftafqmc_t h, int sys, double mu, void* stream);

/* Tune mu of system `sys` so that the ensemble's <N> at tau = beta matches n_target (Sec.
 * "Computational Details").  Every run is the whole path of every walker on the same fields
 * d_fields (device complex128 [W][n][N_Q], common random numbers); <N> is the weighted mean of
 * Re N over live walkers and its standard error is that of ftafqmc_record_stats.  Starting from
 * the system's current mu:
 *   FTAFQMC_MU_BRACKET_FIT: the paper's procedure.  Steps of 0.05 scale (doubled) until <N> - n
 *     changes sign, bisection until the bracket is below 1% of scale = max(|mu|, 1/beta), mu~
 *     its midpoint; five runs at mu~ + scale {-0.025, -0.0125, 0, 0.0125, 0.025}; a straight line
 *     N = a + b mu by least squares with weights 1/sigma^2 (equal weights if a sigma is 0);
 *     mu* = (n_target - a) / b.
 *   FTAFQMC_MU_NEWTON: mu <- mu - (<N> - n_target) / (d<N>/dmu) with the frozen-path derivative
 *     of ftafqmc_backward (the system needs FTAFQMC_CHECKPOINT) until |<N> - n_target| <=
 *     tol n_target.
 * h_trace: host double [max_runs][4] or NULL: mu, <N>, its standard error, d<N>/dmu (0 when not
 * taken) of every run.  The system is left at the tuned mu and reset to tau = 0.  Synchronises
 * the stream after every run.  Errors: E_NUMERIC when max_runs runs do not suffice or no walker
 * survives a run; E_STATE for Newton without FTAFQMC_CHECKPOINT or on a handle with a captured
 * graph or profiling on. */
#define FTAFQMC_MU_BRACKET_FIT 0
#define FTAFQMC_MU_NEWTON 1
typedef struct {
  double mu;        /* the tuned chemical potential */
  double mu_tilde;  /* bracketing: midpoint of the 1% bracket; Newton: the tuned mu */
  double n_mean;    /* <N> of the last run and its standard error */
  double n_stderr;
  int runs;         /* whole-path runs made */
} ftafqmc_mu_result;
int ftafqmc_tune_mu(ftafqmc_t h, int sys, const void* d_fields, int method, double n_target, double tol,
                    int max_runs, double* h_trace, ftafqmc_mu_result* out, void* stream);

/* Wall time in milliseconds of each system's share of the last eager ftafqmc_propagate call
 * (h_ms: host double [n_sys]), from events on the system's first stream before its first slice
 * and after its last.  The systems of a handle run concurrently, each on streams of its own (the
 * caller's stream and side streams the handle owns, default priority), enqueued slice by slice
 * in order of decreasing per-slice work M^3 W; their sum over the call's wall time says how
 * much they overlapped.  E_STATE before any eager call (graph replays record no times). */
int ftafqmc_system_times(ftafqmc_t h, double* h_ms);

/* Kernel-class timing with HIP events recorded on the caller's stream around every
 * launch (instrumentation).  enable = 1 starts recording every class;
 * enable = FTAFQMC_PROFILE_ONLY | (bit c for each class c) records only those classes (fewer
 * events in flight: the other launches run as without profiling); any other nonzero value is
 * E_ARG.  enable = 0 stops, waits for the recorded events and writes, per class, the summed
 * milliseconds into h_ms[FTAFQMC_PROF_CLASSES] and the launch counts into h_count (host
 * arrays, may be NULL).  Classes: the propagator GEMMs, the Green's-function elimination,
 * the transposes around it, the weight/force-bias kernel, the coefficient/V gather,
 * the stabilisation, the energy, the derivative replay (ftafqmc_backward). */
enum { FTAFQMC_PROF_GEMM = 0, FTAFQMC_PROF_ELIM = 1, FTAFQMC_PROF_GREENS = 2, FTAFQMC_PROF_WEIGHT = 3,
       FTAFQMC_PROF_COEF = 4, FTAFQMC_PROF_STAB = 5, FTAFQMC_PROF_ENERGY = 6, FTAFQMC_PROF_BACKWARD = 7,
       FTAFQMC_PROF_CLASSES = 8 };
#define FTAFQMC_PROFILE_ONLY 256
int ftafqmc_profile(ftafqmc_t h, int enable, double* h_ms, long long* h_count);

/* Message of the last error on this handle ("" if none); valid until the next call.  With
 * h = NULL: the message of the last failed ftafqmc_init_ueg / ftafqmc_init_ueg_static call on
 * this thread. */
const char* ftafqmc_last_error(ftafqmc_t h);

/* Release the handle (host memory only; the caller frees the workspace). */
void ftafqmc_destroy(ftafqmc_t h);

#ifdef __cplusplus
}
#endif
#endif /* FTAFQMC_H */
