// Host side of the library: UEG tables, workspace layout, slice orchestration and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/ftafqmc.h"
#include "internal.h"
#include "kernels.h"

namespace {

thread_local std::string init_err;       // message of the last failed initialisation on this thread

constexpr double PI = 3.14159265358979323846;
constexpr double MADELUNG = 2.837297;  // Sec. "Uniform Electron Gas"
constexpr int MAX_M = 512;             // the elimination keeps a panel row per thread, two per thread at most
constexpr int MAX_NQ = 8192;           // the shifted coefficients of one walker are staged in LDS
// Taylor polynomial of e^V: the smallest degree (a multiple of 4, at least 16 in FP64 and 12 in
// mixed precision, at most 24) whose leading remainder term nu^{p+1}/(p+1)! at the a-priori norm
// estimate nu is below TAYLOR_APRIORI_TOL; every slice then checks the rigorous 1-norm bound
// of the remainder on the device against TAYLOR_CHECK_TOL and flags the walker otherwise.
constexpr int TAYLOR_MAX_NB = 6;
constexpr double LOW_RANK_THRESHOLD = FTAFQMC_LOW_RANK_THRESHOLD;
constexpr double TAYLOR_APRIORI_TOL[2] = {1e-14, 1e-8};   // FP64, mixed
// The check tolerance sits at the level of each precision's own product rounding: the 1-norm
// bound is measured 50-400x above the true truncation error on the workloads (M=485: bound
// 2e-9 at degree 12, 3e-14 at degree 16), and the FP32 products of the mixed chain round at
// about 1e-7 relative.
constexpr double TAYLOR_CHECK_TOL[2] = {1e-11, 1e-6};
constexpr double TAYLOR_NU_MARGIN = 1.7;                  // measured: ||V^4||_1^{1/4} <= 1.7 x estimate
// Re-factorisation interval: the kinetic part of the product between two Cholesky-QR passes has
// condition number at most e^{STAB_KIN_RANGE} (dtau (max - min of lambda eps + h) per slice).
constexpr double STAB_KIN_RANGE = 6.0;

typedef std::array<int, 3> iv3;

bool iv_less(const iv3& a, const iv3& b) {
  const int na = a[0] * a[0] + a[1] * a[1] + a[2] * a[2], nb = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
  if (na != nb) return na < nb;
  return a < b;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct HostSys {
  ftafqmc_params p;
  int M = 0, NQ = 0, n = 0, ld = 0, rmax = 0, gdim = 0, gc0 = 0, nrec_max = 0;
  double L = 0, omega = 0, TF = 0, beta = 0, dtau = 0, muT = 0, mu = 0, EM = 0;
  std::vector<iv3> nvec, qvec;
  std::vector<int> idx, neg, qptr, qpair, flat, rbptr, rbidx;
  int rq_rows = 0, rq_nblk = 0;
  std::vector<double> vq, sq, eps, hK, kh, lnbt;
  std::vector<double> tlev;             // trial levels: eps (free electron) or thermal Hartree-Fock
  std::vector<double> lnbt2;            // ln diag B_T for both halves of the doubled system
  std::vector<short> grid;
  size_t off_begin = 0, bytes = 0;
  SysDev dev;
  double2* mean = nullptr;
  int k = 0, nrec = 0;
  std::vector<int> rec_slice;
  int tile_chain = 0, tile_apply = 0, tile_epi = 0, tile_horner = 0;   // GEMM tile shapes chosen by the start-up autotuner
  bool ckpt = false;                    // path recorded for the frozen-path derivative
  int groups = 1;                       // walker groups (streams) of ftafqmc_propagate
  double2* Y0 = nullptr;                // the buffers Y and Ynew start as at every reset
  double2* Ynew0 = nullptr;
  int M2 = 0, ld2 = 0;                  // doubled system of the derivative
  TanDev tan;
  int taylor_nb = 4;                    // Paterson-Stockmeyer blocks of 4: degree 4 taylor_nb
  bool modified = false;                // constraint from the modified overlap ratio (eq. ztfix)
  bool lowrank = false;                 // low-rank truncation of the Green's function solve (eq. thresh)
  bool bf16 = false;                    // mixed propagator products on BF16 matrix cores, split operands
  std::vector<int> lr_order, lr_pos;    // plane waves by decreasing ln B_T, and the inverse order
  std::vector<int> lr_mL;               // [n + 1] left rank of the solve after slice k
  bool every = false;                   // energy record after every slice
  double* small = nullptr;              // [32] device doubles for host-driven loops (mu tuning)
  int lane0 = 0;                        // first stream lane of this system (its groups follow)
  const void* fields = nullptr;         // field buffer of the current path (pathwise derivative)
  bool fields_ok = false;               // one buffer served every slice so far
  hipEvent_t t0 = nullptr, t1 = nullptr;  // start and end of its share of the last eager propagate call
  int stab_cap = 1;                     // re-factorise at least every stab_cap slices
};

// Logistic 1/(1+e^x) without overflow.
double fermi(double x) { return x > 0 ? std::exp(-x) / (1.0 + std::exp(-x)) : 1.0 / (1.0 + std::exp(x)); }

std::string build_tables(HostSys& s, const ftafqmc_params& p) {
  s.p = p;
  if (p.n_elec < 2 || (p.n_elec & 1)) return "n_elec must be even and >= 2";
  if (!(p.rs > 0) || !(p.theta > 0) || !(p.dtau > 0)) return "rs, theta and dtau must be positive";
  if (p.nmax2 < 1) return "nmax2 must be >= 1";
  if (p.stab_every < 1) return "stab_every must be >= 1";
  if (p.n_walkers < 1) return "n_walkers must be >= 1";
  if (p.precision != FTAFQMC_FP64 && p.precision != FTAFQMC_MIXED) return "unknown precision";
  if (!std::isfinite(p.kscale)) return "kscale must be finite";
  if (p.flags & ~(FTAFQMC_CHECKPOINT | FTAFQMC_OVERLAP | FTAFQMC_GRAPH | FTAFQMC_TRIAL_THF | FTAFQMC_MODIFIED_OVERLAP |
                  FTAFQMC_MEASURE_EVERY_SLICE | FTAFQMC_LOW_RANK | FTAFQMC_BF16_SPLIT))
    return "unknown flags";
  s.bf16 = (p.flags & FTAFQMC_BF16_SPLIT) != 0;
  if (s.bf16 && p.precision != FTAFQMC_MIXED) return "the split-BF16 products belong to the mixed precision";
  s.lowrank = (p.flags & FTAFQMC_LOW_RANK) != 0;
  if (s.lowrank && (p.flags & (FTAFQMC_CHECKPOINT | FTAFQMC_MODIFIED_OVERLAP)))
    return "the low-rank truncation is built for the standard overlap ratio without the derivative record";
  s.modified = (p.flags & FTAFQMC_MODIFIED_OVERLAP) != 0;
  s.every = (p.flags & FTAFQMC_MEASURE_EVERY_SLICE) != 0;
  if (s.modified && (p.flags & FTAFQMC_CHECKPOINT))
    return "the frozen-path derivative is built for the standard overlap ratio only";
  s.groups = (p.flags & FTAFQMC_OVERLAP) ? 2 : 1;
  s.ckpt = (p.flags & FTAFQMC_CHECKPOINT) != 0;
  if (s.ckpt && p.precision != FTAFQMC_FP64) return "the path record for derivatives needs FP64 propagation";
  // box, temperature, slices (Sec. "Computational Details", eq. fermiT)
  s.L = std::cbrt(4.0 * PI * p.n_elec / 3.0) * p.rs;
  s.omega = s.L * s.L * s.L;
  s.TF = 0.5 * std::pow(9.0 * PI / 4.0, 2.0 / 3.0) / (p.rs * p.rs);
  s.beta = 1.0 / (p.theta * s.TF);
  s.n = std::max(1, (int)std::lround(s.beta / p.dtau));
  s.dtau = s.beta / s.n;
  // basis
  s.rmax = (int)std::floor(std::sqrt((double)p.nmax2));
  while ((s.rmax + 1) * (s.rmax + 1) <= p.nmax2) ++s.rmax;
  for (int a = -s.rmax; a <= s.rmax; ++a)
    for (int b = -s.rmax; b <= s.rmax; ++b)
      for (int c = -s.rmax; c <= s.rmax; ++c)
        if (a * a + b * b + c * c <= p.nmax2) s.nvec.push_back({a, b, c});
  std::sort(s.nvec.begin(), s.nvec.end(), iv_less);
  s.M = (int)s.nvec.size();
  if (s.M > MAX_M) return "basis larger than the supported maximum of 512 plane waves";
  s.ld = (s.M + 15) / 16 * 16;
  if (s.ckpt && 2 * s.M > MAX_M) return "derivatives double the system: at most 256 plane waves";
  s.M2 = 2 * s.M;
  s.ld2 = (s.M2 + 15) / 16 * 16;
  const double k0 = 2.0 * PI / s.L;
  s.eps.assign(s.ld, 0.0);
  for (int i = 0; i < s.M; ++i) {
    const iv3& v = s.nvec[i];
    s.eps[i] = 0.5 * k0 * k0 * (double)(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  }
  // momentum transfers
  std::map<iv3, int, bool (*)(const iv3&, const iv3&)> qmap(iv_less);
  for (int i = 0; i < s.M; ++i)
    for (int j = 0; j < s.M; ++j)
      if (i != j) qmap.emplace(iv3{s.nvec[i][0] - s.nvec[j][0], s.nvec[i][1] - s.nvec[j][1], s.nvec[i][2] - s.nvec[j][2]}, 0);
  for (auto& kv : qmap) { kv.second = (int)s.qvec.size(); s.qvec.push_back(kv.first); }
  s.NQ = (int)s.qvec.size();
  if (s.NQ > MAX_NQ) return "too many momentum transfers";
  s.idx.assign((size_t)s.M * s.M, -1);
  for (int i = 0; i < s.M; ++i)
    for (int j = 0; j < s.M; ++j)
      if (i != j)
        s.idx[(size_t)i * s.M + j] = qmap.at(iv3{s.nvec[i][0] - s.nvec[j][0], s.nvec[i][1] - s.nvec[j][1], s.nvec[i][2] - s.nvec[j][2]});
  s.neg.resize(s.NQ);
  s.vq.resize(s.NQ);
  s.sq.resize(s.NQ);
  for (int q = 0; q < s.NQ; ++q) {
    const iv3& v = s.qvec[q];
    s.neg[q] = qmap.at(iv3{-v[0], -v[1], -v[2]});
    const double q2 = k0 * k0 * (double)(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    s.vq[q] = 4.0 * PI / (s.omega * q2);
    s.sq[q] = std::sqrt(PI * s.dtau / (s.omega * q2));
  }
  // one-body remainder of the sum-of-squares form: h_K = -(1/2) sum_{K' != K} v(K - K')
  s.hK.assign(s.M, 0.0);
  for (int i = 0; i < s.M; ++i) {
    double a = 0.0;
    for (int j = 0; j < s.M; ++j)
      if (j != i) a += s.vq[s.idx[(size_t)i * s.M + j]];
    s.hK[i] = -0.5 * a;
  }
  // trial levels e_K and chemical potential: 2 sum_K f(e_K - mu_T) = N by bisection, with
  // e_K = eps_K (free-electron trial) or the self-consistent thermal Hartree-Fock levels
  // e_K = eps_K - sum_{K' != K} v(K - K') f_K' (Sec. "Results", fig. thf; the uniform gas keeps
  // plane waves as Hartree-Fock orbitals, and the Q = 0 Hartree term goes with the background),
  // iterated to a fixed point with mixing 1/2
  s.tlev.assign(s.eps.begin(), s.eps.begin() + s.M);
  auto chem_pot = [&](const std::vector<double>& e, double* mu_out) -> bool {
    auto count = [&](double mu) { double c = 0; for (int i = 0; i < s.M; ++i) c += 2.0 * fermi(s.beta * (e[i] - mu)); return c; };
    const double emin = *std::min_element(e.begin(), e.end()), emax = *std::max_element(e.begin(), e.end());
    double lo = emin - 60.0 / s.beta, hi = emax + 60.0 / s.beta;
    if (!(count(lo) < p.n_elec && p.n_elec < count(hi))) return false;
    for (int it = 0; it < 400; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (count(mid) < p.n_elec) lo = mid; else hi = mid;
      if (hi - lo <= 4e-16 * std::max(1.0, std::fabs(mid))) break;
    }
    *mu_out = 0.5 * (lo + hi);
    return true;
  };
  if (!chem_pot(s.tlev, &s.muT)) return "electron number not reachable in this basis";
  if (p.flags & FTAFQMC_TRIAL_THF) {
    std::vector<double> enew(s.M), f(s.M);
    bool conv = false;
    for (int it = 0; it < 10000 && !conv; ++it) {
      double mu = 0.0;
      if (!chem_pot(s.tlev, &mu)) return "electron number not reachable in this basis";
      for (int i = 0; i < s.M; ++i) f[i] = fermi(s.beta * (s.tlev[i] - mu));
      double diff = 0.0, emax = 1.0;
      for (int i = 0; i < s.M; ++i) {
        double x = 0.0;
        for (int j = 0; j < s.M; ++j)
          if (j != i) x += s.vq[s.idx[(size_t)i * s.M + j]] * f[j];
        enew[i] = s.eps[i] - x;
        diff = std::max(diff, std::fabs(enew[i] - s.tlev[i]));
        emax = std::max(emax, std::fabs(s.tlev[i]));
      }
      if (diff <= 1e-14 * emax) { s.tlev = enew; conv = true; }
      else for (int i = 0; i < s.M; ++i) s.tlev[i] = 0.5 * (s.tlev[i] + enew[i]);
    }
    if (!conv) return "thermal Hartree-Fock trial did not converge";
    if (!chem_pot(s.tlev, &s.muT)) return "electron number not reachable in this basis";
  }
  s.mu = std::isnan(p.mu) ? s.muT : p.mu;
  s.EM = -MADELUNG * p.n_elec / (2.0 * s.L);
  s.kh.assign(s.ld, 0.0);
  s.lnbt.assign(s.ld, 0.0);
  for (int i = 0; i < s.M; ++i) {
    s.kh[i] = std::exp(-0.5 * s.dtau * (p.kscale * s.eps[i] + s.hK[i] - s.mu));
    s.lnbt[i] = -s.dtau * (s.tlev[i] - s.muT);
  }
  s.lnbt2.assign(s.ld2, 0.0);
  for (int i = 0; i < s.M2; ++i) s.lnbt2[i] = s.lnbt[i % s.M];
  if (s.lowrank) {
    // eq. thresh on the diagonal left block B_T^lexp: the kept plane waves are a prefix of the
    // order of decreasing ln B_T (lexp >= 0), of length lr_mL[n - lexp] for the solve after slice k
    s.lr_order.resize(s.M);
    for (int i = 0; i < s.M; ++i) s.lr_order[i] = i;
    std::stable_sort(s.lr_order.begin(), s.lr_order.end(), [&](int a, int b) { return s.lnbt[a] > s.lnbt[b]; });
    s.lr_pos.assign(s.M, 0);
    for (int c = 0; c < s.M; ++c) s.lr_pos[s.lr_order[c]] = c;
    s.lr_mL.assign(s.n + 1, 0);
    for (int k = 0; k <= s.n; ++k) {
      int m = 0;
      for (int i = 0; i < s.M; ++i) m += (double)(s.n - k) * s.lnbt[i] >= std::log(LOW_RANK_THRESHOLD) ? 1 : 0;
      s.lr_mL[k] = m;
    }
  }
  // pairs of each Q as flat indices of G_{r p} (K_p - K_r = Q)
  s.qptr.assign(s.NQ + 1, 0);
  for (int i = 0; i < s.M; ++i)
    for (int j = 0; j < s.M; ++j)
      if (i != j) s.qptr[s.idx[(size_t)i * s.M + j] + 1]++;
  for (int q = 0; q < s.NQ; ++q) s.qptr[q + 1] += s.qptr[q];
  s.qpair.assign(s.qptr[s.NQ], 0);
  {
    std::vector<int> fill(s.qptr.begin(), s.qptr.end() - 1);
    for (int pidx = 0; pidx < s.M; ++pidx)
      for (int r = 0; r < s.M; ++r)
        if (pidx != r) s.qpair[fill[s.idx[(size_t)pidx * s.M + r]]++] = r * s.ld + pidx;
  }
  // the pairs again by blocks of rows of G (each block fits one LDS buffer of the r_Q kernel)
  s.rq_rows = std::max(1, std::min(s.M, rq_block_elems() / s.ld));
  s.rq_nblk = (s.M + s.rq_rows - 1) / s.rq_rows;
  s.rbptr.assign((size_t)s.rq_nblk * (s.NQ + 1), 0);
  s.rbidx.assign((size_t)s.M * (s.M - 1), 0);
  {
    std::vector<int> fill(s.NQ);
    int off = 0;
    for (int b = 0; b < s.rq_nblk; ++b) {
      const int r0 = b * s.rq_rows, r1 = std::min(s.M, r0 + s.rq_rows);
      int* bp = &s.rbptr[(size_t)b * (s.NQ + 1)];
      for (int r = r0; r < r1; ++r)
        for (int pidx = 0; pidx < s.M; ++pidx)
          if (pidx != r) bp[s.idx[(size_t)pidx * s.M + r] + 1]++;
      bp[0] = off;
      for (int q = 0; q < s.NQ; ++q) bp[q + 1] += bp[q];
      for (int q = 0; q < s.NQ; ++q) fill[q] = bp[q];
      for (int r = r0; r < r1; ++r)
        for (int pidx = 0; pidx < s.M; ++pidx)
          if (pidx != r) s.rbidx[fill[s.idx[(size_t)pidx * s.M + r]]++] = (r - r0) * s.ld + pidx;
      off = bp[s.NQ];
    }
  }
  // lookup grid for K_b - K_a + K_d
  const int R = 3 * s.rmax;
  s.gdim = 2 * R + 1;
  s.gc0 = R * (s.gdim * s.gdim + s.gdim + 1);
  s.grid.assign((size_t)s.gdim * s.gdim * s.gdim, (short)-1);
  s.flat.resize(s.M);
  for (int i = 0; i < s.M; ++i) {
    const iv3& v = s.nvec[i];
    s.flat[i] = v[0] * s.gdim * s.gdim + v[1] * s.gdim + v[2];
    s.grid[(size_t)(s.flat[i] + s.gc0)] = (short)i;
  }
  s.nrec_max = (p.flags & FTAFQMC_MEASURE_EVERY_SLICE) ? s.n + 1 : s.n / p.stab_every + 2;
  // A-priori size of V = sqrt(dtau) (x - xbar).v: an entry V_ij = i s_Q (z_Q + conj z_-Q) has
  // E|V_ij|^2 = 4 s_Q^2 for unit Gaussian fields, and the norm of such a random matrix is about
  // twice the root of its largest column variance.
  {
    double colmax = 0.0;
    for (int j = 0; j < s.M; ++j) {
      double a = 0.0;
      for (int i = 0; i < s.M; ++i)
        if (i != j) { const double sv = s.sq[s.idx[(size_t)i * s.M + j]]; a += sv * sv; }
      colmax = std::max(colmax, a);
    }
    const double nu = TAYLOR_NU_MARGIN * 4.0 * std::sqrt(colmax);
    const int mixed = p.precision == FTAFQMC_MIXED;
    int nb = mixed ? 3 : 4;
    for (; nb < TAYLOR_MAX_NB; ++nb) {
      const int q = 4 * nb + 1;
      double lt = q * std::log(nu);
      for (int j = 2; j <= q; ++j) lt -= std::log((double)j);
      if (std::exp(lt) <= TAYLOR_APRIORI_TOL[mixed]) break;
    }
    s.taylor_nb = nb;
  }
  {
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < s.M; ++i) {
      const double e = p.kscale * s.eps[i] + s.hK[i];
      lo = std::min(lo, e);
      hi = std::max(hi, e);
    }
    const double per_slice = s.dtau * (hi - lo);
    s.stab_cap = per_slice > 0.0 ? std::max(1, (int)std::floor(STAB_KIN_RANGE / per_slice)) : s.n;
  }
  return "";
}

// Lay out (or only size, when base == nullptr) one system's slice of the workspace.
size_t layout(HostSys& s, char* base, size_t off) {
  const int W = s.p.n_walkers, ld = s.ld, M = s.M, NQ = s.NQ;
  const size_t mat = (size_t)ld * ld;
  const size_t velem = s.p.precision == FTAFQMC_MIXED ? sizeof(float2) : sizeof(double2);
  auto take = [&](size_t bytes) -> char* { char* r = base ? base + off : nullptr; off = align256(off + bytes); return r; };
  SysDev& d = s.dev;
  s.off_begin = off;
  d.idx = (const int*)take(sizeof(int) * M * M);
  d.neg = (const int*)take(sizeof(int) * NQ);
  d.vq = (const double*)take(sizeof(double) * NQ);
  d.sq = (const double*)take(sizeof(double) * NQ);
  d.eps = (const double*)take(sizeof(double) * ld);
  d.kh = (const double*)take(sizeof(double) * ld);
  d.lnbt = (const double*)take(sizeof(double) * ld);
  d.qptr = (const int*)take(sizeof(int) * (NQ + 1));
  d.qpair = (const int*)take(sizeof(int) * (size_t)M * (M - 1));
  d.rbptr = (const int*)take(sizeof(int) * (size_t)s.rq_nblk * (NQ + 1));
  d.rbidx = (const int*)take(sizeof(int) * (size_t)M * (M - 1));
  d.grid = (const short*)take(sizeof(short) * s.grid.size());
  d.flat = (const int*)take(sizeof(int) * M);
  if (s.lowrank) {
    d.lr_order = (const int*)take(sizeof(int) * M);
    d.lr_pos = (const int*)take(sizeof(int) * M);
    d.lr_mR = (int*)take(sizeof(int) * (size_t)W * (s.n + 1));
    d.lr_thr = LOW_RANK_THRESHOLD;
    d.lr_lnthr = std::log(LOW_RANK_THRESHOLD);
    d.lr_mL = M;
  }
  d.Y = (double2*)take(sizeof(double2) * mat * W);
  d.Ti = (double2*)take(sizeof(double2) * mat * W);
  d.G = (double2*)take(sizeof(double2) * mat * W);
  d.Ynew = (double2*)take(sizeof(double2) * mat * W);
  d.aug = (double2*)take(sizeof(double2) * 2 * mat * W);
  d.V = take(velem * mat * W);
  d.V2 = take(velem * mat * W);
  d.V3 = take(velem * mat * W);
  d.V4 = take(velem * mat * W);
  for (int k = 0; k < 5; ++k) d.Bk[k] = k < std::max(3, s.taylor_nb - 1) ? take(velem * mat * W) : nullptr;
  d.E0 = take(sizeof(double2) * mat * W);
  d.E1 = take(sizeof(double2) * mat * W);
  d.D = (double*)take(sizeof(double) * ld * W);
  d.Dpi = (double*)take(sizeof(double) * ld * W);
  d.perm = (int*)take(sizeof(int) * ld * W);
  d.piv = (int*)take(sizeof(int) * ld * W);
  d.tri = (double2*)take(sizeof(double2) * elim_tri_elems(M) * W);
  d.r = (double2*)take(sizeof(double2) * (size_t)NQ * W);
  d.rb = s.modified ? (double2*)take(sizeof(double2) * (size_t)NQ * W) : d.r;
  d.Gt = s.modified ? (double2*)take(sizeof(double2) * mat * W) : d.G;
  d.cq = (double2*)take(sizeof(double2) * (size_t)NQ * W);
  d.expo = (double2*)take(sizeof(double2) * W);
  d.ell = (double2*)take(sizeof(double2) * W);
  d.lndetT = (double2*)take(sizeof(double2) * W);
  d.lndetX = (double2*)take(sizeof(double2) * W);
  d.logw = (double*)take(sizeof(double) * W);
  d.status = (int*)take(sizeof(int) * W);
  d.slice_lnS = (double2*)take(sizeof(double2) * (size_t)W * s.n);
  d.slice_theta = (double*)take(sizeof(double) * (size_t)W * s.n);
  d.exch = (double2*)take(sizeof(double2) * (size_t)ld * W);
  d.local = (double2*)take(sizeof(double2) * 4 * W);
  d.rec_E = (double2*)take(sizeof(double2) * 4 * (size_t)W * s.nrec_max);
  d.rec_logw = (double*)take(sizeof(double) * (size_t)W * s.nrec_max);
  d.rec_status = (int*)take(sizeof(int) * (size_t)W * s.nrec_max);
  d.scratch = (double*)take(sizeof(double) * (size_t)ld * W);
  d.tnorm = (double*)take(sizeof(double) * 16 * (size_t)W);
  d.pop_parent = (int*)take(sizeof(int) * (size_t)W);
  d.pop_logw = (double*)take(sizeof(double) * (size_t)W);
  s.small = (double*)take(sizeof(double) * 32);   // statistics of one record, a Jacobian
  s.mean = (double2*)take(sizeof(double2) * 4);
  d.rec_c = nullptr;
  d.rec_trG = nullptr;
  if (s.ckpt) {
    const int ld2 = s.ld2;
    const size_t mat2 = (size_t)ld2 * ld2;
    TanDev& t = s.tan;
    d.rec_c = (double2*)take(sizeof(double2) * (size_t)W * s.n * NQ);
    d.rec_trG = (double2*)take(sizeof(double2) * (size_t)W * (s.n + 1));
    t.M2 = s.M2; t.ld2 = ld2;
    t.dd = d;                                     // tables shared; state and scratch doubled
    t.dd.M = s.M2; t.dd.ld = ld2;
    t.dd.Y = (double2*)take(sizeof(double2) * mat2 * W);
    t.dd.D = (double*)take(sizeof(double) * ld2 * W);
    t.dd.Dpi = (double*)take(sizeof(double) * ld2 * W);
    t.dd.scratch = (double*)take(sizeof(double) * ld2 * W);   // column norms of the doubled Y
    t.dd.perm = (int*)take(sizeof(int) * ld2 * W);
    t.dd.piv = (int*)take(sizeof(int) * ld2 * W);
    t.dd.tri = (double2*)take(sizeof(double2) * elim_tri_elems(s.M2) * W);
    t.dd.E0 = take(sizeof(double2) * mat2 * W);
    t.dd.E1 = take(sizeof(double2) * mat2 * W);
    t.dd.aug = (double2*)take(sizeof(double2) * 2 * mat2 * W);
    t.caug = (double2*)take(sizeof(double2) * 2 * mat2 * W);
    t.cpiv = (int*)take(sizeof(int) * ld2 * W);
    t.ctri = (double2*)take(sizeof(double2) * elim_tri_elems(s.M2) * W);
    t.tstat = (int*)take(sizeof(int) * W);
    t.lndet_dummy = (double2*)take(sizeof(double2) * W);
    t.dd.status = t.tstat;
    t.dd.lndetT = t.lndet_dummy;
    t.dd.logw = nullptr;                          // the doubled factorisation flags tstat only
    t.dd.tnorm = nullptr;
    t.dd.mat_stride = (long long)mat2;
    t.dd.aug_stride = (long long)2 * mat2;
    t.Ydn = (double2*)take(sizeof(double2) * mat2 * W);
    t.Td = (double2*)take(sizeof(double2) * mat2 * W);
    t.Bcat = (double2*)take(sizeof(double2) * (size_t)ld * ld2 * W);
    t.Fcat = (double2*)take(sizeof(double2) * (size_t)ld * ld2 * W);
    t.Gst = (double2*)take(sizeof(double2) * (size_t)ld2 * ld * W);
    t.dG = (double2*)take(sizeof(double2) * 2 * mat * W);
    t.exch = (double2*)take(sizeof(double2) * (size_t)ld * W);
    t.dlnw = (double*)take(sizeof(double) * 2 * W);
    t.dloc = (double2*)take(sizeof(double2) * 8 * W);
    t.alive = (int*)take(sizeof(int) * W);
    t.bc_stride = (long long)ld * ld2;
    t.gs_stride = (long long)ld2 * ld;
    // pathwise mode
    t.Tid = (double2*)take(sizeof(double2) * mat2 * W);
    t.Gd = (double2*)take(sizeof(double2) * mat2 * W);
    t.lnbt2 = (double*)take(sizeof(double) * ld2);
    t.lndetX2 = (double2*)take(sizeof(double2) * W);
    t.Gk = (double2*)take(sizeof(double2) * mat * W);
    t.dGk = (double2*)take(sizeof(double2) * mat * W);
    t.rk = (double2*)take(sizeof(double2) * (size_t)NQ * W);
    t.drk = (double2*)take(sizeof(double2) * (size_t)NQ * W);
    t.dcq = (double2*)take(sizeof(double2) * (size_t)NQ * W);
    t.dexpo = (double2*)take(sizeof(double2) * W);
    t.dV = (double2*)take(sizeof(double2) * mat * W);
    t.dV2 = (double2*)take(sizeof(double2) * mat * W);
    t.dV3 = (double2*)take(sizeof(double2) * mat * W);
    t.dV4 = (double2*)take(sizeof(double2) * mat * W);
    t.dE0 = (double2*)take(sizeof(double2) * mat * W);
    t.dE1 = (double2*)take(sizeof(double2) * mat * W);
    for (int k = 0; k < 5; ++k) t.dBk[k] = k < std::max(3, s.taylor_nb - 1) ? (double2*)take(sizeof(double2) * mat * W) : nullptr;
  }
  s.bytes = off - s.off_begin;
  d.M = M; d.ld = ld; d.NQ = NQ; d.W = W; d.n = s.n; d.grid_dim = s.gdim; d.grid_c0 = s.gc0;
  d.rq_rows = s.rq_rows; d.rq_nblk = s.rq_nblk;
  // the gather form of r_Q serves N_Q above 4096 (M near 512); FTAFQMC_RQ_GATHER=1 selects it
  // everywhere (its test)
  d.rq_gather = std::getenv("FTAFQMC_RQ_GATHER") && std::atoi(std::getenv("FTAFQMC_RQ_GATHER")) == 1;
  d.dtau = s.dtau; d.kscale = s.p.kscale; d.e_madelung = s.EM;
  d.taylor_deg = 4 * s.taylor_nb;
  d.taylor_tol = TAYLOR_CHECK_TOL[s.p.precision == FTAFQMC_MIXED ? 1 : 0];
  d.mat_stride = (long long)mat;
  d.aug_stride = (long long)2 * mat;
  d.w_off = 0; d.rec_W = W;
  s.Y0 = d.Y; s.Ynew0 = d.Ynew;
  if (s.ckpt) {
    SysDev& dd = s.tan.dd;
    dd.NQ = NQ; dd.W = W; dd.n = s.n; dd.grid_dim = s.gdim; dd.grid_c0 = s.gc0;
    dd.dtau = s.dtau; dd.kscale = s.p.kscale; dd.e_madelung = s.EM;
    dd.idx = d.idx; dd.neg = d.neg; dd.vq = d.vq; dd.sq = d.sq; dd.eps = d.eps; dd.kh = d.kh; dd.lnbt = d.lnbt;
    dd.qptr = d.qptr; dd.qpair = d.qpair; dd.grid = d.grid; dd.flat = d.flat;
    dd.rbptr = d.rbptr; dd.rbidx = d.rbidx; dd.rq_rows = d.rq_rows; dd.rq_nblk = d.rq_nblk;
    dd.rec_c = nullptr; dd.rec_trG = nullptr;
    dd.w_off = 0; dd.rec_W = W;
  }
  return off;
}

// The walkers [w0, w0 + nw) of a system as a SysDev of their own: every per-walker array is
// offset by w0 walkers; the tables and the record arrays (indexed through w_off, rec_W) are shared.
SysDev walker_view(const HostSys& s, int w0, int nw) {
  SysDev v = s.dev;
  const long long mat = v.mat_stride;
  const size_t velem = s.p.precision == FTAFQMC_MIXED ? sizeof(float2) : sizeof(double2);
  const long long ld = s.ld, w = w0;
  v.Y += w * mat; v.Ti += w * mat; v.G += w * mat; v.Ynew += w * mat;
  v.aug += w * v.aug_stride;
  auto offv = [&](void* q, size_t bytes) { return q ? (void*)((char*)q + (size_t)w * bytes) : nullptr; };
  v.V = offv(v.V, velem * mat); v.V2 = offv(v.V2, velem * mat);
  v.V3 = offv(v.V3, velem * mat); v.V4 = offv(v.V4, velem * mat);
  for (int k = 0; k < 5; ++k) v.Bk[k] = offv(v.Bk[k], velem * mat);
  v.E0 = offv(v.E0, sizeof(double2) * mat); v.E1 = offv(v.E1, sizeof(double2) * mat);
  v.D += w * ld; v.Dpi += w * ld; v.perm += w * ld; v.piv += w * ld;
  v.tri += w * (long long)elim_tri_elems(s.M);
  v.r += w * s.NQ;
  v.rb += w * s.NQ;
  v.Gt += w * mat;
  v.cq += w * s.NQ;
  v.expo += w; v.ell += w; v.lndetT += w; v.lndetX += w; v.logw += w; v.status += w;
  v.slice_lnS += w * s.n; v.slice_theta += w * s.n;
  v.exch += w * ld; v.local += w * 4; v.scratch += w * ld;
  if (v.tnorm) v.tnorm += w * 16;
  if (v.rec_c) v.rec_c += w * s.n * (long long)s.NQ;
  if (v.rec_trG) v.rec_trG += w * (s.n + 1);
  if (v.lr_mR) v.lr_mR += w * (s.n + 1);
  v.W = nw; v.w_off = w0; v.rec_W = s.p.n_walkers;
  return v;
}

}  // namespace

struct ProfEvent { int cls; hipEvent_t a, b; };

struct ftafqmc_ctx {
  std::vector<HostSys> sys;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  std::string err;
  bool prof = false;
  unsigned prof_mask = 0;                 // classes recorded while prof is set
  std::vector<ProfEvent> events;
  // Stream lanes: lane 0 is the caller's stream, lane L > 0 the handle's side stream side[L-1]
  // (default priority).  System i uses lanes lane0_i .. lane0_i + groups_i - 1: its own lanes when
  // the systems run concurrently, lane 0 and up for all of them when they run one after another.
  int lanes = 1;
  static constexpr int MAX_GROUPS = 4;
  static constexpr int MAX_LANES = 16;
  hipStream_t side[MAX_LANES - 1] = {};
  hipEvent_t fork = nullptr, join[MAX_LANES - 1] = {};
  bool times_valid = false;             // per-system events of the last propagate call were recorded
  // FTAFQMC_GRAPH: the launch sequence of a whole path, captured once and replayed
  bool graph = false;
  hipStream_t cap = nullptr;            // capture stream (the caller's may be the legacy default stream)
  hipGraphExec_t gexec = nullptr;
  std::vector<const void*> gfields;     // field buffers the captured path reads
  struct SysAfter { int k, nrec; std::vector<int> rec_slice; double2* Y; double2* Ynew; };
  std::vector<SysAfter> gafter;         // host-side state of every system after the path
  // ftafqmc_backward's second stream (default priority) and its fork/join events, created when a
  // system records its path and side streams are allowed
  hipStream_t bwd = nullptr;
  hipEvent_t bwd_ev[4] = {};
  int set(int code, const std::string& m) { err = m; return code; }
};

namespace {

#define HIPCHK(call)                                                             \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess) return h->set(FTAFQMC_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Launch f on st; with profiling on, bracket it with two events of class cls.
template <typename F> hipError_t timed(ftafqmc_ctx* h, int cls, hipStream_t st, F f) {
  if (!h->prof || !((h->prof_mask >> cls) & 1u)) return f();
  ProfEvent ev{cls, nullptr, nullptr};
  hipError_t e = hipEventCreate(&ev.a);
  if (e == hipSuccess) e = hipEventCreate(&ev.b);
  if (e == hipSuccess) e = hipEventRecord(ev.a, st);
  if (e != hipSuccess) return e;
  e = f();
  if (e != hipSuccess) return e;
  e = hipEventRecord(ev.b, st);
  h->events.push_back(ev);
  return e;
}

double sum_ln_lb(const HostSys& s, int lexp) {
  double a = 0.0;
  for (int i = 0; i < s.M; ++i) a += -std::max(0.0, (double)lexp * s.lnbt[i]);
  return a;
}

GemmParams gp_base(const HostSys& s, const SysDev& d) {
  GemmParams g;
  std::memset(&g, 0, sizeof(g));
  g.sA = g.sB = g.sC = g.sP = d.mat_stride;
  g.lda = g.ldb = g.ldc = g.ldp = s.ld;
  g.m = g.n = g.k = s.M; g.mpad = g.npad = s.ld; g.W = d.W;
  g.alpha = 1.0;
  return g;
}

double inv_fact(int j) { double f = 1.0; for (int i = 2; i <= j; ++i) f *= i; return 1.0 / f; }

int horner_step(ftafqmc_ctx* h, HostSys& s, SysDev& d, void* cur, void* nxt, int k, hipStream_t st);

// Y <- K e^V K Y with e^V = sum_{j<=deg} V^j / j! by Paterson-Stockmeyer with blocks of 4:
// B_k = sum_{r<4} a_{4k+r} V^r and e^V = (((a_deg V^4 + B_top) V^4 + ...) V^4 + B_0), with
// deg = 4 nb chosen per system (16 in FP64 and 12 in mixed precision on the workloads).  The
// V^4 product also writes the top Horner term and up to three lower blocks, so every Horner
// step reads one matrix; blocks below those (nb > 4) come from an elementwise pass.  With
// `check`, the column norms of V and V^4 are taken for the device-side truncation bound.
// Forms B = K e^V K from d.V; *B_out points at the buffer that holds it (E0 or E1).
// One product of the propagator chain: FP64 or FP32 MFMA, or with FTAFQMC_BF16_SPLIT the mixed
// path's products on the BF16 matrix cores with three-way split operands.
hipError_t chain_gemm(const HostSys& s, const GemmParams& g, int prec, hipStream_t st) {
  if (s.bf16 && prec != GEMM_Z64) return launch_zgemm_bf16x6(g, prec == GEMM_C32_Z64B, st);
  return launch_zgemm(g, prec, st);
}

int form_propagator(ftafqmc_ctx* h, HostSys& s, SysDev& d, hipStream_t st, void** B_out, bool check) {
  const bool mixed = s.p.precision == FTAFQMC_MIXED;
  const int prec = mixed ? GEMM_C32 : GEMM_Z64;
  const int nb = s.taylor_nb;
  const int deg = 4 * nb;
  GemmParams g = gp_base(s, d);
  g.tile = s.tile_chain;
  g.A = d.V; g.B = d.V; g.C = d.V2;
  HIPCHK(timed(h, FTAFQMC_PROF_GEMM, st, [&] { return chain_gemm(s, g, prec, st); }));   // V^2
  g.A = d.V2; g.B = d.V; g.C = d.V3;
  HIPCHK(timed(h, FTAFQMC_PROF_GEMM, st, [&] { return chain_gemm(s, g, prec, st); }));   // V^3
  g.A = d.V2; g.B = d.V2; g.C = d.V4;                                                  // V^4 and the blocks
  g.tile = s.tile_epi;
  g.P1 = d.V; g.P2 = d.V2; g.P3 = d.V3;
  const int top = 4 * (nb - 1);
  g.extra[0] = GemmOut{d.E0, inv_fact(deg), inv_fact(top), inv_fact(top + 1), inv_fact(top + 2), inv_fact(top + 3)};
  int ne = 1;
  for (int k = nb - 2; k >= 0 && ne < 4; --k, ++ne)
    g.extra[ne] = GemmOut{d.Bk[k], 0.0, inv_fact(4 * k), inv_fact(4 * k + 1), inv_fact(4 * k + 2), inv_fact(4 * k + 3)};
  g.nextra = ne;
  HIPCHK(timed(h, FTAFQMC_PROF_GEMM, st, [&] { return chain_gemm(s, g, prec, st); }));
  const int nlo = nb - ne;                      // blocks B_0 .. B_{nlo-1} not written by the epilogue
  if (nlo > 0) {
    TaylorLow t;
    t.nlo = nlo;
    for (int k = 0; k < nlo; ++k)
      for (int r = 0; r < 4; ++r) t.c[k][r] = inv_fact(4 * k + r);
    HIPCHK(timed(h, FTAFQMC_PROF_COEF, st, [&] { return launch_taylor_blocks(d, mixed, t, st); }));
  }
  if (check) HIPCHK(timed(h, FTAFQMC_PROF_COEF, st, [&] { return launch_taylor_norms(d, mixed, st); }));
  if (!B_out) return FTAFQMC_OK;              // the powers and blocks only (the pathwise chain)
  void* cur = d.E0;
  void* nxt = d.E1;
  for (int k = nb - 2; k >= 0; --k) {
    const int rc = horner_step(h, s, d, cur, nxt, k, st);
    if (rc) return rc;
    std::swap(cur, nxt);
  }
  *B_out = cur;
  return FTAFQMC_OK;
}

// One Horner step of the Taylor polynomial: nxt = cur V^4 + B_k, with K on both sides at k = 0.
int horner_step(ftafqmc_ctx* h, HostSys& s, SysDev& d, void* cur, void* nxt, int k, hipStream_t st) {
  const bool mixed = s.p.precision == FTAFQMC_MIXED;
  GemmParams e = gp_base(s, d);
  e.tile = s.tile_horner;
  e.A = cur; e.B = d.V4; e.C = nxt;
  e.P1 = d.Bk[k]; e.c1 = 1.0;
  if (k == 0) { e.rs = d.kh; e.cs = d.kh; }            // K e^V K
  HIPCHK(timed(h, FTAFQMC_PROF_GEMM, st, [&] { return chain_gemm(s, e, mixed ? GEMM_C32 : GEMM_Z64, st); }));
  return FTAFQMC_OK;
}

int apply_propagator(ftafqmc_ctx* h, HostSys& s, SysDev& d, hipStream_t st) {
  const bool mixed = s.p.precision == FTAFQMC_MIXED;
  void* cur = nullptr;
  int rc = form_propagator(h, s, d, st, &cur, true);
  if (rc) return rc;
  GemmParams a = gp_base(s, d);
  a.tile = s.tile_apply;
  a.A = cur; a.B = d.Y; a.C = d.Ynew;
  HIPCHK(timed(h, FTAFQMC_PROF_GEMM, st, [&] { return chain_gemm(s, a, mixed ? GEMM_C32_Z64B : GEMM_Z64, st); }));
  std::swap(d.Y, d.Ynew);
  return FTAFQMC_OK;
}

// Pre-pivoted QR of Y diag(D) by one Cholesky-QR pass; updates Y, D and Ti = T^{-1}.
int stabilise(ftafqmc_ctx* h, HostSys& s, SysDev& d, hipStream_t st) {
  HIPCHK(timed(h, FTAFQMC_PROF_STAB, st, [&] { return launch_stab_perm(d, st); }));
  HIPCHK(timed(h, FTAFQMC_PROF_STAB, st, [&] { return launch_stab_gather(d, st); }));
  GemmParams g = gp_base(s, d);
  g.A = d.E0; g.B = d.E0; g.C = d.aug; g.opA = 1; g.role = 1; g.herm = 1;
  g.sC = d.aug_stride; g.ldc = 2 * s.ld;
  HIPCHK(timed(h, FTAFQMC_PROF_STAB, st, [&] { return launch_zgemm(g, GEMM_Z64, st); }));  // S = E0^H E0 into the left block
  ElimParams e;
  e.aug = d.aug; e.stride = d.aug_stride; e.lda = 2 * s.ld; e.M = s.M; e.rhs_off = s.ld; e.nrhs = s.M;
  e.W = d.W; e.pivot = 0; e.backsub = 0; e.lndet = nullptr; e.status = d.status;
  e.piv = d.piv; e.ld = s.ld; e.tri = d.tri;
  HIPCHK(timed(h, FTAFQMC_PROF_STAB, st, [&] { return launch_elim(e, st); }));
  HIPCHK(timed(h, FTAFQMC_PROF_STAB, st, [&] { return launch_stab_finish_a(d, st); }));
  HIPCHK(timed(h, FTAFQMC_PROF_STAB, st, [&] { return launch_stab_build_ti(d, st); }));
  HIPCHK(timed(h, FTAFQMC_PROF_STAB, st, [&] { return launch_elim_lower(e, st); }));   // Ru^T is lower triangular
  HIPCHK(timed(h, FTAFQMC_PROF_STAB, st, [&] { return launch_stab_finish_b(d, st); }));
  return FTAFQMC_OK;
}

// (I + B_T^lexp R)^{-1} into d.G with ln det X of the eliminated block (Sec. "Numerical Stabilization").
// Low-rank: only the plane waves kept in the left block are right-hand sides.
int greens_solve(ftafqmc_ctx* h, HostSys& s, SysDev& d0, int lexp, hipStream_t st) {
  SysDev d = d0;
  if (s.lowrank) d.lr_mL = s.lr_mL[s.n - lexp];
  HIPCHK(timed(h, FTAFQMC_PROF_GREENS, st, [&] { return launch_greens_form(d, lexp, st); }));
  ElimParams e;
  e.aug = d.aug; e.stride = d.aug_stride; e.lda = 2 * s.ld; e.M = s.M; e.rhs_off = s.ld; e.nrhs = s.lowrank ? d.lr_mL : s.M;
  e.W = d.W; e.pivot = 1; e.backsub = 1; e.lndet = d.lndetX; e.status = d.status;
  e.piv = d.piv; e.ld = s.ld; e.tri = d.tri;
  HIPCHK(timed(h, FTAFQMC_PROF_ELIM, st, [&] { return launch_elim(e, st); }));
  HIPCHK(timed(h, FTAFQMC_PROF_GREENS, st, [&] { return launch_greens_post(d, lexp, st); }));
  return FTAFQMC_OK;
}

// The constraint's G, ln det(I + A_k) and the weight update of the slice that ended at k, with
// r_Q for the next force bias; A_k = B_T^{n-k} R_k (eq. Abrenda), or B_T^n R_k for the modified
// overlap ratio (eq. ztfix), whose constraint G lives in Gt.  With `measure` (or the standard
// ratio, where the two coincide) also G_k = (I + B_T^{n-k} R_k)^{-1} and its r_Q for the estimators.
int greens(ftafqmc_ctx* h, HostSys& s, SysDev& d, int k, int init, bool measure, hipStream_t st) {
  if (!s.modified) {
    int rc = greens_solve(h, s, d, s.n - k, st);
    if (rc) return rc;
    if (s.lowrank) HIPCHK(timed(h, FTAFQMC_PROF_GREENS, st, [&] { return launch_lr_rank(d, k, st); }));
    const double slb = sum_ln_lb(s, s.n - k);
    HIPCHK(timed(h, FTAFQMC_PROF_WEIGHT, st, [&] { return launch_weight(d, k, slb, init, st); }));
    return FTAFQMC_OK;
  }
  SysDev cv = d;
  cv.G = d.Gt;
  cv.r = d.rb;
  int rc = greens_solve(h, s, cv, s.n, st);
  if (rc) return rc;
  const double slb = sum_ln_lb(s, s.n);
  HIPCHK(timed(h, FTAFQMC_PROF_WEIGHT, st, [&] { return launch_weight(cv, k, slb, init, st); }));
  if (!measure) return FTAFQMC_OK;
  rc = greens_solve(h, s, d, s.n - k, st);
  if (rc) return rc;
  HIPCHK(timed(h, FTAFQMC_PROF_WEIGHT, st, [&] { return launch_rq(d, st); }));
  return FTAFQMC_OK;
}

// Start-up autotuner: time every GEMM tile shape on this system's real size (W walkers of
// M x M x M products) for each kind of product in the propagator (plain chain product, V^4 with
// the Taylor blocks, Horner step, apply), keep the fastest for each.
// FTAFQMC_GEMM_TILE=<index> in the environment forces one shape (for experiments).
std::vector<SysDev> make_views(const HostSys& s, int ngroups);

int autotune_gemm(ftafqmc_ctx* h, HostSys& s, hipStream_t st) {
  SysDev& d = s.dev;
  const bool mixed = s.p.precision == FTAFQMC_MIXED;
  const size_t velem = mixed ? sizeof(float2) : sizeof(double2);
  const size_t mat = (size_t)s.ld * s.ld * s.p.n_walkers;
  if (const char* env = std::getenv("FTAFQMC_GEMM_TILE")) {
    // a shape not built for this precision falls back to the timed choice
    const int t = std::atoi(env);
    if (gemm_tile_supported(t, mixed ? GEMM_C32 : GEMM_Z64) && (!mixed || gemm_tile_supported(t, GEMM_C32_Z64B))) {
      s.tile_chain = s.tile_apply = s.tile_epi = s.tile_horner = t;
      return FTAFQMC_OK;
    }
  }
  HIPCHK(hipMemsetAsync(d.V, 0, velem * mat, st));
  HIPCHK(hipMemsetAsync(d.V2, 0, velem * mat, st));
  HIPCHK(hipMemsetAsync(d.V3, 0, velem * mat, st));
  HIPCHK(hipMemsetAsync(d.Ynew, 0, sizeof(double2) * mat, st));
  hipEvent_t a = nullptr, b = nullptr;
  HIPCHK(hipEventCreate(&a));
  HIPCHK(hipEventCreate(&b));
  int rc = FTAFQMC_OK;
  // With walker groups the groups' kernels run side by side; a tile of one workgroup per walker
  // leaves the other group no room (measured: overlap gains 8.6% with 64 x 64 tiles, 1.4% with it).
  const bool grouped = make_views(s, s.groups).size() > 1;
  // kind 0: a plain chain product; 1: the apply; 2: the V^4 product with its three addends and
  // Taylor-block outputs; 3: a Horner step (one addend, one output)
  for (int kind = 0; kind < 4 && rc == FTAFQMC_OK; ++kind) {
    float best = 1e30f;
    int besti = 0;
    for (int t = 0; t < gemm_tile_count(); ++t) {
      GemmParams g = gp_base(s, d);
      g.tile = t;
      int prec = mixed ? GEMM_C32 : GEMM_Z64;
      if (kind == 0) { g.A = d.V; g.B = d.V; g.C = d.V2; }
      else if (kind == 1) { g.A = d.V; g.B = d.Ynew; g.C = d.E1; if (mixed) prec = GEMM_C32_Z64B; }
      else if (kind == 3) { g.A = d.V2; g.B = d.V4; g.C = d.V3; g.P1 = d.V; g.c1 = 1.0; }
      else {
        g.A = d.V2; g.B = d.V2; g.C = d.V4; g.P1 = d.V; g.P2 = d.V2; g.P3 = d.V3; g.c1 = 1.0;
        const int nb = s.taylor_nb;
        g.extra[0] = GemmOut{d.E0, 1.0, 1.0, 1.0, 1.0, 1.0};
        int e = 1;
        for (int k = nb - 2; k >= 0 && e < 4; --k, ++e) g.extra[e] = GemmOut{d.Bk[k], 0.0, 1.0, 1.0, 1.0, 1.0};
        g.nextra = e;
      }
      if (!gemm_tile_supported(t, prec) || (grouped && gemm_tile_walker_sized(t))) continue;
      hipError_t e = launch_zgemm(g, prec, st);                 // warm-up
      if (e == hipSuccess) e = hipEventRecord(a, st);
      for (int r = 0; r < 3 && e == hipSuccess; ++r) e = launch_zgemm(g, prec, st);
      if (e == hipSuccess) e = hipEventRecord(b, st);
      if (e == hipSuccess) e = hipEventSynchronize(b);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
      if (e != hipSuccess) { rc = h->set(FTAFQMC_E_HIP, std::string("autotune: ") + hipGetErrorString(e)); break; }
      // The V^4 product's heavy epilogue (three addends, four outputs) does not overlap anyone's
      // MFMAs when every CU holds one walker's workgroup: in the running path the 64 x 64 tile
      // beats the one-walker tile that ties with it here (M=171: 197 against about 223 us), so
      // a one-walker tile must win this trial by more than 5%.
      if (kind == 2 && gemm_tile_walker_sized(t)) ms *= 1.05f;
      if (ms < best) { best = ms; besti = t; }
    }
    if (kind == 0) s.tile_chain = besti;
    else if (kind == 1) s.tile_apply = besti;
    else if (kind == 2) s.tile_epi = besti;
    else s.tile_horner = besti;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return rc;
}

int reset_sys(ftafqmc_ctx* h, HostSys& s, hipStream_t st) {
  s.dev.Y = s.Y0;                       // every path starts from the same buffers (graph replay)
  s.dev.Ynew = s.Ynew0;
  HIPCHK(launch_init_state(s.dev, st));
  int rc = greens(h, s, s.dev, 0, 1, true, st);
  if (rc) return rc;
  s.k = 0;
  s.nrec = 0;
  s.rec_slice.clear();
  return FTAFQMC_OK;
}

// One slice k -> k+1 for the walkers of view d (fields of those walkers), on stream st.
// rec >= 0: energy record number rec after the slice; refac: re-factorise the product;
// last: the last slice of this propagate call (the estimators' G must be current after it).
int slice_step(ftafqmc_ctx* h, HostSys& s, SysDev& d, const double2* fields, int k, int rec, bool refac,
               bool last, hipStream_t st) {
  const int mixed = s.p.precision == FTAFQMC_MIXED;
  HIPCHK(timed(h, FTAFQMC_PROF_COEF, st, [&] { return launch_coef_v(d, fields, k, mixed, st); }));
  int rc = apply_propagator(h, s, d, st);
  if (rc) return rc;
  if (refac) { rc = stabilise(h, s, d, st); if (rc) return rc; }
  rc = greens(h, s, d, k + 1, 0, rec >= 0 || last, st);
  if (rc) return rc;
  if (rec >= 0) HIPCHK(timed(h, FTAFQMC_PROF_ENERGY, st, [&] { return launch_energy(d, rec, st); }));
  return FTAFQMC_OK;
}

// One slice for every walker of system s.  The walkers are split into groups that run on the
// caller's stream and the handle's side stream: the elimination of one group is latency bound
// (a workgroup per walker walks its pivot columns one by one) and overlaps with the GEMMs of the
// other.  Walkers are independent, so the results do not depend on the split.
int step(ftafqmc_ctx* h, HostSys& s, std::vector<SysDev>& views, const double2* fields, bool last, hipStream_t st) {
  const int k = s.k;
  const bool boundary = ((k + 1) % s.p.stab_every == 0) || (k + 1 == s.n);
  const bool record = boundary || s.every;
  const int rec = record ? s.nrec : -1;
  // records at the caller's stabilisation interval; extra re-factorisations where the kinetic
  // range of the product would make one Cholesky-QR pass lose orthogonality
  const bool refac = boundary || ((k + 1) % s.stab_cap == 0);
  for (size_t g = 0; g < views.size(); ++g) {
    SysDev& d = views[g];
    const double2* f = fields + (long long)d.w_off * s.n * s.NQ;
    const int lane = s.lane0 + (int)g;
    int rc = slice_step(h, s, d, f, k, rec, refac, last || k + 1 == s.n, lane == 0 ? st : h->side[lane - 1]);
    if (rc) return rc;
  }
  std::swap(s.dev.Y, s.dev.Ynew);           // every view swapped its own pointers once
  if (record) {
    s.rec_slice.push_back(k + 1);
    ++s.nrec;
  }
  s.k = k + 1;
  return FTAFQMC_OK;
}

// Walker groups of a system, one per stream: boundaries at multiples of 8 (the XCD count)
// nearest to g W / ng, at most W / 8 groups; empty groups are dropped.
std::vector<SysDev> make_views(const HostSys& s, int ngroups) {
  const int W = s.p.n_walkers;
  const int ng = std::max(1, std::min(ngroups, W / 8));
  std::vector<SysDev> v;
  int w0 = 0;
  for (int g = 1; g <= ng; ++g) {
    const int b = g == ng ? W : std::min(W, (g * W / ng + 4) / 8 * 8);
    if (b > w0) v.push_back(walker_view(s, w0, b - w0));
    w0 = std::max(w0, b);
  }
  return v;
}

// ------------------------------------------------------------ derivative ---
GemmParams gp_dd(const HostSys& s) {       // 2M x 2M products of the doubled system
  GemmParams g;
  std::memset(&g, 0, sizeof(g));
  g.sA = g.sB = g.sC = g.sP = s.tan.dd.mat_stride;
  g.lda = g.ldb = g.ldc = g.ldp = s.ld2;
  g.m = g.n = g.k = s.M2; g.mpad = g.npad = s.ld2; g.W = s.p.n_walkers;
  g.alpha = 1.0; g.role = 1;
  return g;
}

ElimParams ep_dd(const HostSys& s, int pivot, int backsub) {
  const SysDev& dd = s.tan.dd;
  ElimParams e;
  e.aug = dd.aug; e.stride = dd.aug_stride; e.lda = 2 * s.ld2; e.M = s.M2; e.rhs_off = s.ld2; e.nrhs = s.M2;
  e.W = dd.W; e.pivot = pivot; e.backsub = backsub; e.lndet = nullptr; e.status = dd.status;
  e.piv = dd.piv; e.ld = s.ld2; e.tri = dd.tri;
  return e;
}

// Doubled Green's function (cyclic at slice k, or literal at tau = beta) into Gst / the lambda dG,
// in its own augmented system (caug, cpiv, ctri).  The form step reads the doubled state; the
// solve step reads only caug.
int doubled_greens_form(ftafqmc_ctx* h, HostSys& s, int k, int literal, hipStream_t st) {
  HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_cyc_form(s.dev, s.tan, k, literal, st); }));
  return FTAFQMC_OK;
}
int doubled_greens_solve(ftafqmc_ctx* h, HostSys& s, int k, int literal, hipStream_t st) {
  TanDev& t = s.tan;
  ElimParams e = ep_dd(s, 1, 1);
  e.aug = t.caug; e.piv = t.cpiv; e.tri = t.ctri;
  HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_elim(e, st); }));
  HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_cyc_post(s.dev, t, k, literal, st); }));
  return FTAFQMC_OK;
}
int doubled_greens(ftafqmc_ctx* h, HostSys& s, int k, int literal, hipStream_t st) {
  int rc = doubled_greens_form(h, s, k, literal, st);
  return rc ? rc : doubled_greens_solve(h, s, k, literal, st);
}

// One slice of the doubled product: Rd <- [[B, dB], [0, B]] Rd, then the pre-pivoted
// Cholesky-QR re-factorisation Yd Dd Td with Td <- Ru Td[perm, :]; with `with_inverse` also
// Tid <- Tid[:, perm] Ru^{-1} (the inverse triangular factor, as the forward path carries it).
int doubled_push(ftafqmc_ctx* h, HostSys& s, hipStream_t st, bool with_inverse) {
  TanDev& t = s.tan;
  SysDev& dd = t.dd;
  const int M = s.M;
  GemmParams g;
  std::memset(&g, 0, sizeof(g));
  g.W = s.p.n_walkers; g.alpha = 1.0; g.role = 1;
  g.sA = t.bc_stride; g.sB = g.sC = dd.mat_stride;
  g.lda = s.ld2; g.ldb = g.ldc = s.ld2;
  g.A = t.Bcat; g.B = dd.Y; g.C = t.Ydn;                         // rows < M: [B | dB] Rd
  g.m = M; g.n = s.M2; g.k = s.M2; g.mpad = M; g.npad = s.ld2;
  HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_zgemm(g, GEMM_Z64, st); }));
  g.B = dd.Y + (size_t)M * s.ld2; g.C = t.Ydn + (size_t)M * s.ld2;  // rows >= M: B Rd_bottom
  g.k = M; g.mpad = s.ld2 - M;
  HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_zgemm(g, GEMM_Z64, st); }));
  std::swap(dd.Y, t.Ydn);
  HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_stab_perm(dd, st); }));
  HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_stab_gather(dd, st); }));
  GemmParams gs = gp_dd(s);
  gs.A = dd.E0; gs.B = dd.E0; gs.C = dd.aug; gs.opA = 1; gs.herm = 1;
  gs.sC = dd.aug_stride; gs.ldc = 2 * s.ld2;
  HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_zgemm(gs, GEMM_Z64, st); }));
  const ElimParams e = ep_dd(s, 0, 0);
  HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_elim(e, st); }));
  HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_stab_finish_a(dd, st); }));
  if (with_inverse) {
    SysDev pv = dd;
    pv.Ti = t.Tid;
    HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_stab_build_ti(pv, st); }));
    HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_elim_lower(e, st); }));   // Ru^T lower triangular
    HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_stab_finish_b(pv, st); }));
  }
  HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_permute_rows(t, st); }));
  GemmParams gt = gp_dd(s);
  gt.A = dd.E1; gt.B = dd.E0; gt.C = t.Td; gt.tri_a = 1;   // Ru is upper triangular
  HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_zgemm(gt, GEMM_Z64, st); }));
  return FTAFQMC_OK;
}

// The ratio of the step that inserts B_{k+1}: [I + Phi | dPhi] = [I + W - W Gc11 | dW - (dW Gc11 +
// W Gc12)] from Fcat = [dW | W] and the cyclic doubled Green's function, eliminated in d.aug (the
// right block then holds (I + Phi)^{-1} dPhi).
int ratio_solve(ftafqmc_ctx* h, HostSys& s, hipStream_t st) {
  SysDev& d = s.dev;
  TanDev& t = s.tan;
  const int M = s.M, ld = s.ld, W = s.p.n_walkers;
  GemmParams g;
  std::memset(&g, 0, sizeof(g));
  g.W = W; g.role = 1; g.alpha = -1.0; g.c1 = 1.0;
  g.sA = g.sP = t.bc_stride; g.sB = t.gs_stride; g.sC = d.aug_stride;
  g.lda = g.ldp = s.ld2; g.ldb = ld; g.ldc = 2 * ld;
  g.A = t.Fcat + M; g.P1 = t.Fcat + M; g.B = t.Gst; g.C = d.aug; g.cI = 1.0;
  g.m = M; g.n = M; g.k = M; g.mpad = M; g.npad = ld;
  HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_zgemm(g, GEMM_Z64, st); }));
  g.A = t.Fcat; g.P1 = t.Fcat; g.C = d.aug + ld; g.cI = 0.0; g.k = s.M2;
  HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_zgemm(g, GEMM_Z64, st); }));
  ElimParams e;
  e.aug = d.aug; e.stride = d.aug_stride; e.lda = 2 * ld; e.M = M; e.rhs_off = ld; e.nrhs = M;
  e.W = W; e.pivot = 1; e.backsub = 1; e.lndet = nullptr; e.status = t.tstat;
  e.piv = d.piv; e.ld = ld; e.tri = d.tri;
  HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_elim(e, st); }));
  return FTAFQMC_OK;
}

// Frozen-path derivatives of <E> and <N> at tau = beta in mu and lambda (replays the recorded path).
int backward(ftafqmc_ctx* h, HostSys& s, const double* cot, double2* jac, double* grad, double2* walker,
             hipStream_t st) {
  SysDev& d = s.dev;
  TanDev& t = s.tan;
  HIPCHK(launch_tan_init(d, t, st));
  // With the handle's backward stream, the re-factorisation of the doubled product (which needs
  // only B and the state) runs beside the cyclic solve and the ratio of the same slice (which
  // need only the state and their own scratch): the form step reads the state first.
  const hipStream_t side = h->bwd;
  for (int k = 0; k < s.n; ++k) {
    HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_coef_replay(d, k, st); }));
    void* B = nullptr;
    int rc = form_propagator(h, s, d, st, &B, false);
    if (rc) return rc;
    HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_tan_prep(d, t, (const double2*)B, st); }));
    if ((rc = doubled_greens_form(h, s, k, 0, st))) return rc;
    if (side) HIPCHK(hipEventRecord(h->bwd_ev[0], st));
    // the latency-bound solve is queued before the re-factorisation's GEMMs, which would
    // otherwise take every CU first
    if ((rc = doubled_greens_solve(h, s, k, 0, st))) return rc;
    if (side) {
      HIPCHK(hipStreamWaitEvent(side, h->bwd_ev[0], 0));
      if ((rc = doubled_push(h, s, side, false))) return rc;
      HIPCHK(hipEventRecord(h->bwd_ev[1], side));
    }
    if ((rc = ratio_solve(h, s, st))) return rc;
    HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_tan_weight(d, t, k, st); }));
    if (side) HIPCHK(hipStreamWaitEvent(st, h->bwd_ev[1], 0));
    else if ((rc = doubled_push(h, s, st, false))) return rc;
  }
  int rc = doubled_greens(h, s, s.n, 1, st);                      // lambda: dG_n
  if (rc) return rc;
  GemmParams g = gp_base(s, d);                                      // mu: dG_n = beta (G G - G)
  g.role = 1; g.A = d.G; g.B = d.G; g.C = t.dG; g.P1 = d.G; g.alpha = s.beta; g.c1 = -s.beta;
  HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_zgemm(g, GEMM_Z64, st); }));
  for (int dir = 0; dir < 2; ++dir)
    HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_energy_tangent(d, t, dir, st); }));
  HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_tan_mean(d, t, cot, jac, grad, walker, st); }));
  return FTAFQMC_OK;
}

hipStream_t lane_stream(ftafqmc_ctx* h, hipStream_t st, int lane) { return lane == 0 ? st : h->side[lane - 1]; }

// ------------------------------------------------------------ pathwise ---
// The literal doubled Green's function (I + diag(L, L) Rd)^{-1}, L = B_T^lexp, into Gd by the
// forward path's scale-split solve on the doubled state (Yd, Dd and the inverse factor Tid).
int pw_literal(ftafqmc_ctx* h, HostSys& s, int lexp, hipStream_t st) {
  TanDev& t = s.tan;
  SysDev pv = t.dd;
  pv.Ti = t.Tid; pv.G = t.Gd; pv.lnbt = t.lnbt2; pv.lndetX = t.lndetX2;
  HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_greens_form(pv, lexp, st); }));
  ElimParams e = ep_dd(s, 1, 1);
  e.lndet = t.lndetX2;
  HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_elim(e, st); }));
  HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_greens_post(pv, lexp, st); }));
  return FTAFQMC_OK;
}

// B = K e^V K of the recorded slice (the forward path's own products, bit-identical) and, carried
// alongside, K (d e^V) K for the Frechet derivative of e^V in the direction dV: with the
// Paterson-Stockmeyer blocks of B_k = sum_r a_{4k+r} V^r,
//   (V^2)' = V dV + dV V, (V^3)' = (V^2)' V + V^2 dV, (V^4)' = (V^2)' V^2 + V^2 (V^2)',
//   B_k' = sum_{r>0} a_{4k+r} (V^r)', and each Horner step E <- E V^4 + B_k gives
//   E' <- E' V^4 + E (V^4)' + B_k' (K on both sides at the last step).
int pw_chain(ftafqmc_ctx* h, HostSys& s, hipStream_t st, void** B_out, double2** KdEK_out) {
  SysDev& d = s.dev;
  TanDev& t = s.tan;
  int rc = form_propagator(h, s, d, st, nullptr, false);          // V^2, V^3, V^4 and the blocks
  if (rc) return rc;
  const int nb = s.taylor_nb, deg = 4 * nb;
  auto prod = [&](const void* A, const void* B, void* C, const void* P1, const double* rs) -> int {
    GemmParams g = gp_base(s, d);
    g.tile = s.tile_chain;
    g.A = A; g.B = B; g.C = C;
    if (P1 == C) g.beta = 1.0;                          // accumulate into C
    else if (P1) { g.P1 = P1; g.c1 = 1.0; }
    if (rs) { g.rs = rs; g.cs = rs; }
    HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_zgemm(g, GEMM_Z64, st); }));
    return FTAFQMC_OK;
  };
  if ((rc = prod(d.V, t.dV, t.dV2, nullptr, nullptr))) return rc;       // (V^2)'
  if ((rc = prod(t.dV, d.V, t.dV2, t.dV2, nullptr))) return rc;
  if ((rc = prod(t.dV2, d.V, t.dV3, nullptr, nullptr))) return rc;      // (V^3)'
  if ((rc = prod(d.V2, t.dV, t.dV3, t.dV3, nullptr))) return rc;
  if ((rc = prod(t.dV2, d.V2, t.dV4, nullptr, nullptr))) return rc;     // (V^4)'
  if ((rc = prod(d.V2, t.dV2, t.dV4, t.dV4, nullptr))) return rc;
  PwBlocks b;
  std::memset(&b, 0, sizeof(b));
  b.nb = nb;
  for (int k = 0; k < nb; ++k) {
    b.c[k][0] = k == nb - 1 ? inv_fact(deg) : 0.0;
    for (int r = 1; r < 4; ++r) b.c[k][r] = inv_fact(4 * k + r);
  }
  HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_pw_blocks(d, t, b, st); }));
  void* cur = d.E0;
  void* nxt = d.E1;
  double2* dcur = t.dE0;
  double2* dnxt = t.dE1;
  for (int k = nb - 2; k >= 0; --k) {
    if ((rc = prod(dcur, d.V4, dnxt, t.dBk[k], nullptr))) return rc;
    if ((rc = prod(cur, t.dV4, dnxt, dnxt, k == 0 ? d.kh : nullptr))) return rc;
    if ((rc = horner_step(h, s, d, cur, nxt, k, st))) return rc;
    std::swap(cur, nxt);
    std::swap(dcur, dnxt);
  }
  *B_out = cur;
  *KdEK_out = dcur;
  return FTAFQMC_OK;
}

// Pathwise derivatives of <E> and <N> at tau = beta in mu and lambda: the raw fields of the path
// held fixed, the force bias (hence V_k, e^{V_k} and the exponent of eq. import) following G_k.
// One pass per direction over the recorded slices.
int backward_pathwise(ftafqmc_ctx* h, HostSys& s, const double* cot, double2* jac, double* grad, double2* walker,
                      hipStream_t st) {
  SysDev& d = s.dev;
  TanDev& t = s.tan;
  const long long mat = d.mat_stride;
  const double2* fields = (const double2*)s.fields;
  HIPCHK(launch_tan_init(d, t, st));
  // With the handle's backward stream: the cyclic solve of slice k (state only) runs beside the
  // literal solve and the propagator chain; the re-factorisation (state and [B | dB]) beside the
  // ratio and the weight.
  const hipStream_t side = h->bwd;
  for (int dir = 0; dir < 2; ++dir) {
    HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_pw_reset(d, t, st); }));
    for (int k = 0; k < s.n; ++k) {
      int rc;
      if (side) {
        HIPCHK(hipEventRecord(h->bwd_ev[0], st));
        HIPCHK(hipStreamWaitEvent(side, h->bwd_ev[0], 0));
        if ((rc = doubled_greens(h, s, k, 0, side))) return rc;
        HIPCHK(hipEventRecord(h->bwd_ev[1], side));
      }
      HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_coef_replay(d, k, st); }));
      rc = pw_literal(h, s, s.n - k, st);                             // G_k and dG_k
      if (rc) return rc;
      HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_pw_extract(d, t, nullptr, st); }));
      SysDev gv = d;
      gv.G = t.Gk; gv.r = t.rk;
      HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_rq(gv, st); }));
      SysDev dv = d;
      dv.G = t.dGk; dv.r = t.drk;
      HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_rq(dv, st); }));
      HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_pw_coef(d, t, fields, k, st); }));
      SysDev fv = d;
      fv.cq = t.dcq;
      HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_fill_v(fv, t.dV, 0, st); }));
      void* B = nullptr;
      double2* KdEK = nullptr;
      if ((rc = pw_chain(h, s, st, &B, &KdEK))) return rc;
      HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_pw_prep(d, t, (const double2*)B, KdEK, dir, st); }));
      if (side) {
        HIPCHK(hipEventRecord(h->bwd_ev[2], st));
        HIPCHK(hipStreamWaitEvent(side, h->bwd_ev[2], 0));
        if ((rc = doubled_push(h, s, side, true))) return rc;
        HIPCHK(hipEventRecord(h->bwd_ev[3], side));
        HIPCHK(hipStreamWaitEvent(st, h->bwd_ev[1], 0));
      } else if ((rc = doubled_greens(h, s, k, 0, st))) {
        return rc;
      }
      if ((rc = ratio_solve(h, s, st))) return rc;
      HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_pw_weight(d, t, k, dir, st); }));
      if (side) HIPCHK(hipStreamWaitEvent(st, h->bwd_ev[3], 0));
      else if ((rc = doubled_push(h, s, st, true))) return rc;
    }
    int rc = pw_literal(h, s, 0, st);                                   // dG_n at tau = beta
    if (rc) return rc;
    HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_pw_extract(d, t, t.dG + (long long)dir * d.W * mat, st); }));
    HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_energy_tangent(d, t, dir, st); }));
  }
  HIPCHK(timed(h, FTAFQMC_PROF_BACKWARD, st, [&] { return launch_tan_mean(d, t, cot, jac, grad, walker, st); }));
  return FTAFQMC_OK;
}

// The launch sequence of ftafqmc_propagate for n_slices slices (eager, or under graph capture).
// Each system runs on its own lanes: the side lanes start after the work already queued on the
// caller's stream and the caller's stream continues after all of them (fork / join).  Within a
// slice round the systems are enqueued in order of decreasing per-slice work (M^3 W), so that
// the longest paths start first; a system that has reached its n slices drops out.
int run_slices(ftafqmc_ctx* h, const void* const* d_fields, int n_slices, hipStream_t st, bool capture) {
  std::vector<std::vector<SysDev>> views;
  for (auto& s : h->sys) views.push_back(make_views(s, s.groups));
  std::vector<int> order(h->sys.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  auto work = [&](int i) { const HostSys& s = h->sys[i]; return (double)s.M * s.M * s.M * s.p.n_walkers; };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(a) > work(b); });
  HIPCHK(hipEventRecord(h->fork, st));
  for (int l = 1; l < h->lanes; ++l) HIPCHK(hipStreamWaitEvent(h->side[l - 1], h->fork, 0));
  const bool timing = !capture;
  std::vector<char> started(h->sys.size(), 0);
  int rc = FTAFQMC_OK;
  for (int j = 0; j < n_slices && rc == FTAFQMC_OK; ++j) {
    bool any = false;
    for (int i : order) {
      HostSys& s = h->sys[i];
      if (s.k >= s.n) continue;
      any = true;
      const hipStream_t s0 = lane_stream(h, st, s.lane0);
      if (timing && !started[i]) { HIPCHK(hipEventRecord(s.t0, s0)); started[i] = 1; }
      if (s.k == 0) { s.fields = d_fields[i]; s.fields_ok = true; }
      else if (d_fields[i] != s.fields) s.fields_ok = false;
      const bool last = j + 1 == n_slices || s.k + 1 == s.n;
      rc = step(h, s, views[i], (const double2*)d_fields[i], last, st);
      if (rc) break;
      if (last) {                        // the system's share of this call ends: join its groups
        for (size_t g = 1; g < views[i].size(); ++g) {
          const int l = s.lane0 + (int)g;
          HIPCHK(hipEventRecord(h->join[l - 1], h->side[l - 1]));
          HIPCHK(hipStreamWaitEvent(s0, h->join[l - 1], 0));
        }
        if (timing) HIPCHK(hipEventRecord(s.t1, s0));
      }
    }
    if (!any) break;
  }
  for (int l = 1; l < h->lanes; ++l) {
    HIPCHK(hipEventRecord(h->join[l - 1], h->side[l - 1]));
    HIPCHK(hipStreamWaitEvent(st, h->join[l - 1], 0));
  }
  bool all = true;
  for (size_t i = 0; i < h->sys.size(); ++i) all = all && started[i];
  h->times_valid = timing && all && rc == FTAFQMC_OK;
  return rc;
}

// mu enters only the half-step factors K = exp(-dtau/2 (lambda eps + h - mu)) (eq. B).
int set_mu(ftafqmc_ctx* h, HostSys& s, double mu, hipStream_t st) {
  s.mu = mu;
  for (int i = 0; i < s.M; ++i) s.kh[i] = std::exp(-0.5 * s.dtau * (s.p.kscale * s.eps[i] + s.hK[i] - s.mu));
  HIPCHK(hipMemcpyAsync((void*)s.dev.kh, s.kh.data(), sizeof(double) * s.ld, hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));          // the host vector may change again before a later copy
  return FTAFQMC_OK;
}

// One whole path of system s at chemical potential mu on its fields: Re<N> at tau = beta, its
// standard error over the walkers, and with `deriv` the frozen-path d Re<N> / dmu.
int mu_run(ftafqmc_ctx* h, HostSys& s, const double2* fields, double mu, bool deriv, double* n, double* err,
           double* dn, hipStream_t st) {
  int rc = set_mu(h, s, mu, st);
  if (rc) return rc;
  rc = reset_sys(h, s, st);
  if (rc) return rc;
  std::vector<SysDev> views = make_views(s, s.groups);
  const hipStream_t s0 = lane_stream(h, st, s.lane0);
  HIPCHK(hipEventRecord(h->fork, st));
  for (int l = 1; l < h->lanes; ++l) HIPCHK(hipStreamWaitEvent(h->side[l - 1], h->fork, 0));
  for (int k = 0; k < s.n && rc == FTAFQMC_OK; ++k) rc = step(h, s, views, fields, k + 1 == s.n, st);
  for (int l = 1; l < h->lanes; ++l) {
    HIPCHK(hipEventRecord(h->join[l - 1], h->side[l - 1]));
    HIPCHK(hipStreamWaitEvent(st, h->join[l - 1], 0));
  }
  (void)s0;
  if (rc) return rc;
  // statistics of the last record (tau = beta): a view of that record alone
  SysDev last = s.dev;
  last.rec_E += (long long)(s.nrec - 1) * s.p.n_walkers * 4;
  last.rec_logw += (long long)(s.nrec - 1) * s.p.n_walkers;
  last.rec_status += (long long)(s.nrec - 1) * s.p.n_walkers;
  HIPCHK(launch_record_stats(last, 1, s.small, nullptr, st));
  double stats[8];
  HIPCHK(hipMemcpyAsync(stats, s.small, sizeof(stats), hipMemcpyDeviceToHost, st));
  if (deriv) {
    rc = backward(h, s, nullptr, (double2*)(s.small + 8), nullptr, nullptr, st);
    if (rc) return rc;
  }
  double jac[8] = {0};
  if (deriv) HIPCHK(hipMemcpyAsync(jac, s.small + 8, sizeof(jac), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  *n = stats[2];
  *err = stats[3];
  if (dn) *dn = deriv ? jac[2] : 0.0;          // Re d<N>/dmu (second complex entry)
  if (!(stats[7] > 0.0)) return h->set(FTAFQMC_E_NUMERIC, "mu tuning: no live walker");
  return FTAFQMC_OK;
}

int check_handle(ftafqmc_ctx* h, int sys) {
  if (!h) return FTAFQMC_E_ARG;
  if (sys < 0 || sys >= (int)h->sys.size()) return h->set(FTAFQMC_E_ARG, "system index out of range");
  return FTAFQMC_OK;
}

}  // namespace

extern "C" {

int ftafqmc_workspace_bytes(const ftafqmc_params* p, int n_sys, size_t* bytes) {
  if (!p || n_sys < 1 || !bytes) return FTAFQMC_E_ARG;
  size_t off = 0;
  for (int i = 0; i < n_sys; ++i) {
    HostSys s;
    if (!build_tables(s, p[i]).empty()) return FTAFQMC_E_ARG;
    off = layout(s, nullptr, off);
  }
  *bytes = off;
  return FTAFQMC_OK;
}

int ftafqmc_init_ueg(const ftafqmc_params* p, int n_sys, void* d_workspace, size_t ws_bytes, void* stream,
                     ftafqmc_t* out) {
  return init_ueg_impl(p, n_sys, d_workspace, ws_bytes, stream, out, false);
}

}  // extern "C"

int init_ueg_impl(const ftafqmc_params* p, int n_sys, void* d_workspace, size_t ws_bytes, void* stream,
                  ftafqmc_t* out, bool no_side_streams) {
  if (!p || n_sys < 1 || !out || !d_workspace) return lib_init_error(FTAFQMC_E_ARG, "null parameters, output or workspace");
  if (((uintptr_t)d_workspace) & 255) return lib_init_error(FTAFQMC_E_ARG, "workspace not 256-byte aligned");
  ftafqmc_ctx* h = new (std::nothrow) ftafqmc_ctx();
  if (!h) return lib_init_error(FTAFQMC_E_ARG, "out of host memory");
  h->sys.resize(n_sys);
  size_t off = 0;
  for (int i = 0; i < n_sys; ++i) {
    std::string m = build_tables(h->sys[i], p[i]);
    if (!m.empty()) { delete h; return lib_init_error(FTAFQMC_E_ARG, m.c_str()); }
    off = layout(h->sys[i], nullptr, off);
  }
  if (off > ws_bytes) { delete h; return lib_init_error(FTAFQMC_E_ARG, "workspace smaller than ftafqmc_workspace_bytes"); }
  // Systems run concurrently on lanes of their own (the small systems' latency-bound kernels
  // then overlap with the large ones'); FTAFQMC_SERIAL_SYSTEMS=1 in the environment, or the
  // static workspace (which creates no streams), runs them one after another on lane 0 and up.
  const char* serial_env = std::getenv("FTAFQMC_SERIAL_SYSTEMS");
  const bool concurrent = n_sys > 1 && !no_side_streams && !(serial_env && std::atoi(serial_env) == 1);
  h->lanes = 1;
  int next = 0;
  for (auto& s : h->sys) {
    if (s.p.flags & FTAFQMC_GRAPH) h->graph = true;
    if (const char* env = std::getenv("FTAFQMC_WALKER_GROUPS"))   // experiments: force a group count
      s.groups = std::max(1, std::min(ftafqmc_ctx::MAX_GROUPS, std::atoi(env)));
    if (no_side_streams) s.groups = 1;
    s.lane0 = concurrent ? next : 0;
    if (s.lane0 + s.groups > ftafqmc_ctx::MAX_LANES) s.lane0 = 0;   // more lanes than streams: share
    next = s.lane0 + s.groups;
    h->lanes = std::max(h->lanes, s.lane0 + s.groups);
  }
  bool ok = hipEventCreateWithFlags(&h->fork, hipEventDisableTiming) == hipSuccess;
  for (int l = 1; ok && l < h->lanes; ++l)
    ok = hipStreamCreateWithFlags(&h->side[l - 1], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&h->join[l - 1], hipEventDisableTiming) == hipSuccess;
  for (auto& s : h->sys)
    ok = ok && hipEventCreate(&s.t0) == hipSuccess && hipEventCreate(&s.t1) == hipSuccess;
  bool any_ckpt = false;
  for (auto& s : h->sys) any_ckpt = any_ckpt || s.ckpt;
  if (ok && any_ckpt && !no_side_streams && !std::getenv("FTAFQMC_SERIAL_BACKWARD")) {
    ok = hipStreamCreateWithFlags(&h->bwd, hipStreamNonBlocking) == hipSuccess;
    for (int e = 0; ok && e < 4; ++e) ok = hipEventCreateWithFlags(&h->bwd_ev[e], hipEventDisableTiming) == hipSuccess;
  }
  if (!ok) { ftafqmc_destroy(h); return lib_init_error(FTAFQMC_E_HIP, "event or stream creation failed"); }
  h->ws = (char*)d_workspace;
  h->ws_bytes = ws_bytes;
  hipStream_t st = (hipStream_t)stream;
  off = 0;
  for (int i = 0; i < n_sys; ++i) {
    HostSys& s = h->sys[i];
    off = layout(s, h->ws, off);
    const SysDev& d = s.dev;
    auto up = [&](const void* dst, const void* src, size_t n) {
      return hipMemcpyAsync((void*)dst, src, n, hipMemcpyHostToDevice, st);
    };
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = up(d.idx, s.idx.data(), sizeof(int) * s.idx.size());
    if (e == hipSuccess) e = up(d.neg, s.neg.data(), sizeof(int) * s.NQ);
    if (e == hipSuccess) e = up(d.vq, s.vq.data(), sizeof(double) * s.NQ);
    if (e == hipSuccess) e = up(d.sq, s.sq.data(), sizeof(double) * s.NQ);
    if (e == hipSuccess) e = up(d.eps, s.eps.data(), sizeof(double) * s.ld);
    if (e == hipSuccess) e = up(d.kh, s.kh.data(), sizeof(double) * s.ld);
    if (e == hipSuccess) e = up(d.lnbt, s.lnbt.data(), sizeof(double) * s.ld);
    if (e == hipSuccess) e = up(d.qptr, s.qptr.data(), sizeof(int) * (s.NQ + 1));
    if (e == hipSuccess) e = up(d.qpair, s.qpair.data(), sizeof(int) * s.qpair.size());
    if (e == hipSuccess) e = up(d.rbptr, s.rbptr.data(), sizeof(int) * s.rbptr.size());
    if (e == hipSuccess) e = up(d.rbidx, s.rbidx.data(), sizeof(int) * s.rbidx.size());
    if (e == hipSuccess) e = up(d.grid, s.grid.data(), sizeof(short) * s.grid.size());
    if (e == hipSuccess) e = up(d.flat, s.flat.data(), sizeof(int) * s.M);
    if (e == hipSuccess && s.ckpt) e = up(s.tan.lnbt2, s.lnbt2.data(), sizeof(double) * s.ld2);
    if (e == hipSuccess && s.lowrank) e = up((void*)d.lr_order, s.lr_order.data(), sizeof(int) * s.M);
    if (e == hipSuccess && s.lowrank) e = up((void*)d.lr_pos, s.lr_pos.data(), sizeof(int) * s.M);
    // the host tables are no longer needed once the copies have completed
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) { ftafqmc_destroy(h); return lib_init_error(FTAFQMC_E_HIP, "table upload failed"); }
    if (autotune_gemm(h, s, st) != FTAFQMC_OK) { ftafqmc_destroy(h); return lib_init_error(FTAFQMC_E_HIP, "GEMM autotuning failed"); }
    if (reset_sys(h, s, st) != FTAFQMC_OK) { ftafqmc_destroy(h); return lib_init_error(FTAFQMC_E_HIP, "walker initialisation failed"); }
  }
  init_err.clear();
  *out = h;
  return FTAFQMC_OK;
}

extern "C" {

int ftafqmc_query(ftafqmc_t h, int sys, ftafqmc_info* out) {
  int rc = check_handle(h, sys);
  if (rc) return rc;
  if (!out) return h->set(FTAFQMC_E_ARG, "null output");
  const HostSys& s = h->sys[sys];
  out->M = s.M; out->n_q = s.NQ; out->n_slices = s.n; out->n_walkers = s.p.n_walkers;
  out->slice = s.k; out->n_measure = s.nrec; out->ld = s.ld;
  out->beta = s.beta; out->dtau = s.dtau; out->L = s.L; out->omega = s.omega;
  out->mu_T = s.muT; out->mu = s.mu; out->e_madelung = s.EM;
  out->gemm_tile_chain = s.tile_chain; out->gemm_tile_apply = s.tile_apply; out->gemm_tile_epilogue = s.tile_epi;
  out->gemm_tile_horner = s.tile_horner;
  out->taylor_degree = 4 * s.taylor_nb;
  out->refactor_every = s.stab_cap;
  out->gemm_tile_shapes = gemm_tile_count();
  out->walker_groups = (int)make_views(s, s.groups).size();
  return FTAFQMC_OK;
}

int ftafqmc_reset(ftafqmc_t h, void* stream) {
  if (!h) return FTAFQMC_E_ARG;
  for (auto& s : h->sys) {
    int rc = reset_sys(h, s, (hipStream_t)stream);
    if (rc) return rc;
  }
  return FTAFQMC_OK;
}

int ftafqmc_propagate(ftafqmc_t h, const void* const* d_fields, int n_slices, void* stream) {
  if (!h) return FTAFQMC_E_ARG;
  if (!d_fields || n_slices < 0) return h->set(FTAFQMC_E_ARG, "bad fields or slice count");
  for (size_t i = 0; i < h->sys.size(); ++i)
    if (!d_fields[i]) return h->set(FTAFQMC_E_ARG, "null fields pointer");
  hipStream_t st = (hipStream_t)stream;
  bool whole = h->graph && !h->prof;
  for (auto& s : h->sys) whole = whole && s.k == 0 && n_slices >= s.n;
  if (!whole) return run_slices(h, d_fields, n_slices, st, false);
  std::vector<const void*> key(d_fields, d_fields + h->sys.size());
  if (!h->gexec || key != h->gfields) {
    if (h->gexec) { (void)hipGraphExecDestroy(h->gexec); h->gexec = nullptr; }
    if (!h->cap) HIPCHK(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
    // record on the capture stream (nothing runs); the instantiated graph is launched on st
    HIPCHK(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
    const int rc = run_slices(h, d_fields, n_slices, h->cap, true);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(h->cap, &g);
    if (rc != FTAFQMC_OK || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return rc != FTAFQMC_OK ? rc : h->set(FTAFQMC_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    }
    const hipError_t e2 = hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) { h->gexec = nullptr; return h->set(FTAFQMC_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(e2)); }
    h->gfields = key;
    h->gafter.clear();
    for (auto& s : h->sys) h->gafter.push_back({s.k, s.nrec, s.rec_slice, s.dev.Y, s.dev.Ynew});
  } else {
    for (size_t i = 0; i < h->sys.size(); ++i) {   // the replay leaves every system where the capture did
      HostSys& s = h->sys[i];
      const ftafqmc_ctx::SysAfter& a = h->gafter[i];
      s.k = a.k; s.nrec = a.nrec; s.rec_slice = a.rec_slice; s.dev.Y = a.Y; s.dev.Ynew = a.Ynew;
    }
  }
  HIPCHK(hipGraphLaunch(h->gexec, st));
  return FTAFQMC_OK;
}

int ftafqmc_greens(ftafqmc_t h, int sys, void* d_G, int dtype, void* stream) {
  int rc = check_handle(h, sys);
  if (rc) return rc;
  if (!d_G || (dtype != FTAFQMC_C128 && dtype != FTAFQMC_C64)) return h->set(FTAFQMC_E_ARG, "bad output");
  HIPCHK(launch_copy_greens(h->sys[sys].dev, d_G, dtype, (hipStream_t)stream));
  return FTAFQMC_OK;
}

int ftafqmc_energy(ftafqmc_t h, int sys, void* d_local, void* d_mean, double* d_logw, int* d_status,
                   void* stream) {
  int rc = check_handle(h, sys);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  HostSys& s = h->sys[sys];
  HIPCHK(launch_energy(s.dev, -1, st));
  HIPCHK(launch_energy_mean(s.dev, s.dev.local, s.dev.logw, s.dev.status, s.mean, st));
  HIPCHK(launch_copy_state(s.dev, (double2*)d_local, d_logw, d_status, st));
  if (d_mean) HIPCHK(hipMemcpyAsync(d_mean, s.mean, 4 * sizeof(double2), hipMemcpyDeviceToDevice, st));
  return FTAFQMC_OK;
}

int ftafqmc_records(ftafqmc_t h, int sys, void* d_trace, double* d_logw, int* h_slice, void* stream) {
  int rc = check_handle(h, sys);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  HostSys& s = h->sys[sys];
  const size_t W = s.p.n_walkers;
  if (d_trace && s.nrec)
    HIPCHK(hipMemcpyAsync(d_trace, s.dev.rec_E, sizeof(double2) * 4 * W * s.nrec, hipMemcpyDeviceToDevice, st));
  if (d_logw && s.nrec)
    HIPCHK(hipMemcpyAsync(d_logw, s.dev.rec_logw, sizeof(double) * W * s.nrec, hipMemcpyDeviceToDevice, st));
  if (h_slice)
    for (int i = 0; i < s.nrec; ++i) h_slice[i] = s.rec_slice[i];
  return FTAFQMC_OK;
}

int ftafqmc_backward(ftafqmc_t h, int sys, int mode, const double* d_cot, void* d_jac, double* d_grad,
                     void* d_walker, void* stream) {
  int rc = check_handle(h, sys);
  if (rc) return rc;
  if (mode != FTAFQMC_FROZEN_PATH && mode != FTAFQMC_PATHWISE) return h->set(FTAFQMC_E_ARG, "unknown mode");
  HostSys& s = h->sys[sys];
  if (!s.ckpt) return h->set(FTAFQMC_E_STATE, "the system was initialised without FTAFQMC_CHECKPOINT");
  if (s.k != s.n) return h->set(FTAFQMC_E_STATE, "the path has not reached tau = beta");
  if (d_grad && !d_cot) return h->set(FTAFQMC_E_ARG, "d_grad needs d_cot");
  if (mode == FTAFQMC_PATHWISE) {
    if (!s.fields_ok || !s.fields)
      return h->set(FTAFQMC_E_STATE, "the pathwise mode reads the path's fields: one buffer must serve every slice");
    return backward_pathwise(h, s, d_cot, (double2*)d_jac, d_grad, (double2*)d_walker, (hipStream_t)stream);
  }
  return backward(h, s, d_cot, (double2*)d_jac, d_grad, (double2*)d_walker, (hipStream_t)stream);
}

int ftafqmc_population_control(ftafqmc_t h, int sys, int method, const double* d_u, int* d_parent, void* stream) {
  int rc = check_handle(h, sys);
  if (rc) return rc;
  if (method != FTAFQMC_POP_COMB && method != FTAFQMC_POP_PAIR_BRANCH) return h->set(FTAFQMC_E_ARG, "unknown population control method");
  if (!d_u) return h->set(FTAFQMC_E_ARG, "null uniforms");
  HostSys& s = h->sys[sys];
  if (s.ckpt) return h->set(FTAFQMC_E_STATE, "population control would break the recorded path of FTAFQMC_CHECKPOINT");
  if (pop_select_lds(s.p.n_walkers) > 64 * 1024) return h->set(FTAFQMC_E_ARG, "too many walkers for population control");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(launch_population_control(s.dev, method, d_u, s.dev.pop_parent, s.dev.pop_logw, st));
  if (d_parent) HIPCHK(hipMemcpyAsync(d_parent, s.dev.pop_parent, sizeof(int) * s.p.n_walkers, hipMemcpyDeviceToDevice, st));
  return FTAFQMC_OK;
}

int ftafqmc_record_stats(ftafqmc_t h, int sys, double* d_stats, double* d_average, void* stream) {
  int rc = check_handle(h, sys);
  if (rc) return rc;
  if (!d_stats) return h->set(FTAFQMC_E_ARG, "null stats");
  HostSys& s = h->sys[sys];
  HIPCHK(launch_record_stats(s.dev, s.nrec, d_stats, d_average, (hipStream_t)stream));
  return FTAFQMC_OK;
}

int ftafqmc_density_correlation(ftafqmc_t h, int sys, void* d_walker, void* d_mean, void* stream) {
  int rc = check_handle(h, sys);
  if (rc) return rc;
  HostSys& s = h->sys[sys];
  hipStream_t st = (hipStream_t)stream;
  // the exchange partial sums per (a, d) use E0 and the per-walker values cq (both free between
  // propagate calls)
  HIPCHK(launch_density_correlation(s.dev, (double2*)s.dev.E0, s.dev.cq, (double2*)d_mean, st));
  if (d_walker)
    HIPCHK(hipMemcpyAsync(d_walker, s.dev.cq, sizeof(double2) * (size_t)s.NQ * s.p.n_walkers, hipMemcpyDeviceToDevice, st));
  return FTAFQMC_OK;
}

int ftafqmc_qvectors(ftafqmc_t h, int sys, int* h_qvec) {
  int rc = check_handle(h, sys);
  if (rc) return rc;
  if (!h_qvec) return h->set(FTAFQMC_E_ARG, "null output");
  const HostSys& s = h->sys[sys];
  for (int q = 0; q < s.NQ; ++q)
    for (int c = 0; c < 3; ++c) h_qvec[3 * q + c] = s.qvec[q][c];
  return FTAFQMC_OK;
}

int ftafqmc_set_mu(ftafqmc_t h, int sys, double mu, void* stream) {
  int rc = check_handle(h, sys);
  if (rc) return rc;
  if (!std::isfinite(mu)) return h->set(FTAFQMC_E_ARG, "mu must be finite");
  HostSys& s = h->sys[sys];
  rc = set_mu(h, s, mu, (hipStream_t)stream);
  if (rc) return rc;
  return reset_sys(h, s, (hipStream_t)stream);
}

int ftafqmc_tune_mu(ftafqmc_t h, int sys, const void* d_fields, int method, double n_target, double tol,
                    int max_runs, double* h_trace, ftafqmc_mu_result* out, void* stream) {
  int rc = check_handle(h, sys);
  if (rc) return rc;
  HostSys& s = h->sys[sys];
  if (!d_fields || !out || max_runs < 1 || !(n_target > 0.0)) return h->set(FTAFQMC_E_ARG, "bad tuning arguments");
  if (method != FTAFQMC_MU_BRACKET_FIT && method != FTAFQMC_MU_NEWTON) return h->set(FTAFQMC_E_ARG, "unknown method");
  if (method == FTAFQMC_MU_NEWTON && !s.ckpt)
    return h->set(FTAFQMC_E_STATE, "Newton steps need the derivative: initialise with FTAFQMC_CHECKPOINT");
  if (h->gexec || h->prof) return h->set(FTAFQMC_E_STATE, "tuning runs eagerly: no graph or profiling");
  hipStream_t st = (hipStream_t)stream;
  const double2* f = (const double2*)d_fields;
  int runs = 0;
  double n = 0.0, err = 0.0, dn = 0.0;
  auto run = [&](double mu, bool deriv) -> int {
    if (runs >= max_runs) return h->set(FTAFQMC_E_NUMERIC, "mu tuning exceeded its run budget");
    const int r = mu_run(h, s, f, mu, deriv, &n, &err, &dn, st);
    if (r) return r;
    if (h_trace) { h_trace[4 * runs] = mu; h_trace[4 * runs + 1] = n; h_trace[4 * runs + 2] = err; h_trace[4 * runs + 3] = dn; }
    ++runs;
    return FTAFQMC_OK;
  };
  const double mu0 = s.mu;
  if (method == FTAFQMC_MU_NEWTON) {
    double mu = mu0;
    for (;;) {
      rc = run(mu, true);
      if (rc) return rc;
      if (std::fabs(n - n_target) <= tol * n_target) break;
      if (!(dn != 0.0) || !std::isfinite(dn)) return h->set(FTAFQMC_E_NUMERIC, "mu tuning: zero or non-finite d<N>/dmu");
      mu = mu - (n - n_target) / dn;
    }
    out->mu = mu; out->mu_tilde = mu;
  } else {
    // bracket the root with single runs (error bars ignored) to 1% of max(|mu|, 1/beta), then a
    // weighted least-squares line through five runs on mu~ +- 2.5% (Sec. "Computational Details")
    const double scale0 = std::max(std::fabs(mu0), 1.0 / s.beta);
    double step = 0.05 * scale0, a, b;
    if ((rc = run(mu0, false))) return rc;
    if (n < n_target) {
      a = mu0;
      b = a + step;
      for (;;) {
        if ((rc = run(b, false))) return rc;
        if (!(n < n_target)) break;
        a = b; step = 2.0 * step; b = a + step;
      }
    } else {
      b = mu0;
      a = b - step;
      for (;;) {
        if ((rc = run(a, false))) return rc;
        if (n < n_target) break;
        b = a; step = 2.0 * step; a = b - step;
      }
    }
    while (b - a > 0.01 * std::max(std::fabs(0.5 * (a + b)), 1.0 / s.beta)) {
      const double m = 0.5 * (a + b);
      if ((rc = run(m, false))) return rc;
      if (n < n_target) a = m; else b = m;
    }
    const double mt = 0.5 * (a + b), scale = std::max(std::fabs(mt), 1.0 / s.beta);
    const double offs[5] = {-0.025, -0.0125, 0.0, 0.0125, 0.025};
    double mus[5], ns[5], es[5];
    bool pos = true;
    for (int i = 0; i < 5; ++i) {
      mus[i] = mt + offs[i] * scale;
      if ((rc = run(mus[i], false))) return rc;
      ns[i] = n; es[i] = err;
      pos = pos && err > 0.0;
    }
    double S0 = 0, S1 = 0, S2 = 0, T0 = 0, T1 = 0;
    for (int i = 0; i < 5; ++i) {
      const double w = pos ? 1.0 / (es[i] * es[i]) : 1.0;
      S0 += w; S1 += w * mus[i]; S2 += w * mus[i] * mus[i]; T0 += w * ns[i]; T1 += w * mus[i] * ns[i];
    }
    const double det = S0 * S2 - S1 * S1;
    const double af = (S2 * T0 - S1 * T1) / det, bf = (S0 * T1 - S1 * T0) / det;
    out->mu = (n_target - af) / bf;
    out->mu_tilde = mt;
  }
  out->n_mean = n;
  out->n_stderr = err;
  out->runs = runs;
  // the system is left at the tuned mu, back at tau = 0
  rc = set_mu(h, s, out->mu, st);
  if (rc) return rc;
  return reset_sys(h, s, st);
}

int ftafqmc_system_times(ftafqmc_t h, double* h_ms) {
  if (!h) return FTAFQMC_E_ARG;
  if (!h_ms) return h->set(FTAFQMC_E_ARG, "null output");
  if (!h->times_valid) return h->set(FTAFQMC_E_STATE, "no eager ftafqmc_propagate call has been timed");
  for (size_t i = 0; i < h->sys.size(); ++i) {
    float ms = 0.0f;
    hipError_t e = hipEventSynchronize(h->sys[i].t1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, h->sys[i].t0, h->sys[i].t1);
    if (e != hipSuccess) return h->set(FTAFQMC_E_HIP, std::string("system times: ") + hipGetErrorString(e));
    h_ms[i] = ms;
  }
  return FTAFQMC_OK;
}

int ftafqmc_lowrank_ranks(ftafqmc_t h, int sys, int* d_mR, int* h_mL, void* stream) {
  int rc = check_handle(h, sys);
  if (rc) return rc;
  HostSys& s = h->sys[sys];
  if (!s.lowrank) return h->set(FTAFQMC_E_STATE, "the system was initialised without FTAFQMC_LOW_RANK");
  if (h_mL) std::memcpy(h_mL, s.lr_mL.data(), sizeof(int) * (s.n + 1));
  if (d_mR)
    HIPCHK(hipMemcpyAsync(d_mR, s.dev.lr_mR, sizeof(int) * (size_t)s.p.n_walkers * (s.n + 1), hipMemcpyDeviceToDevice,
                          (hipStream_t)stream));
  return FTAFQMC_OK;
}

int ftafqmc_kink_flags(ftafqmc_t h, int sys, double threshold, int* d_flags, void* stream) {
  int rc = check_handle(h, sys);
  if (rc) return rc;
  if (!d_flags) return h->set(FTAFQMC_E_ARG, "null flags");
  HIPCHK(launch_kink_flags(h->sys[sys].dev, threshold, d_flags, (hipStream_t)stream));
  return FTAFQMC_OK;
}

int ftafqmc_profile(ftafqmc_t h, int enable, double* h_ms, long long* h_count) {
  if (!h) return FTAFQMC_E_ARG;
  if (enable) {
    const unsigned all = (1u << FTAFQMC_PROF_CLASSES) - 1u;
    unsigned mask;
    if (enable == 1) mask = all;
    else if ((enable & ~(int)(FTAFQMC_PROFILE_ONLY | all)) == 0 && (enable & FTAFQMC_PROFILE_ONLY) && (enable & all))
      mask = (unsigned)enable & all;
    else
      return h->set(FTAFQMC_E_ARG, "profile: enable is 1 or FTAFQMC_PROFILE_ONLY with a non-empty class mask");
    h->prof = true;
    h->prof_mask = mask;
    return FTAFQMC_OK;
  }
  h->prof = false;
  if (h_ms) for (int c = 0; c < FTAFQMC_PROF_CLASSES; ++c) h_ms[c] = 0.0;
  if (h_count) for (int c = 0; c < FTAFQMC_PROF_CLASSES; ++c) h_count[c] = 0;
  int rc = FTAFQMC_OK;
  for (auto& ev : h->events) {
    float ms = 0.0f;
    hipError_t e = hipEventSynchronize(ev.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev.a, ev.b);
    if (e != hipSuccess) rc = h->set(FTAFQMC_E_HIP, std::string("profile events: ") + hipGetErrorString(e));
    if (h_ms && ev.cls >= 0 && ev.cls < FTAFQMC_PROF_CLASSES) h_ms[ev.cls] += ms;
    if (h_count && ev.cls >= 0 && ev.cls < FTAFQMC_PROF_CLASSES) h_count[ev.cls] += 1;
    (void)hipEventDestroy(ev.a);
    (void)hipEventDestroy(ev.b);
  }
  h->events.clear();
  return rc;
}

const char* ftafqmc_last_error(ftafqmc_t h) { return h ? h->err.c_str() : init_err.c_str(); }

void ftafqmc_destroy(ftafqmc_t h) {
  if (!h) return;
  static_ws_release(h);
  for (auto& ev : h->events) { (void)hipEventDestroy(ev.a); (void)hipEventDestroy(ev.b); }
  for (auto& s : h->sys) {
    if (s.t0) (void)hipEventDestroy(s.t0);
    if (s.t1) (void)hipEventDestroy(s.t1);
  }
  for (int g = 0; g + 1 < ftafqmc_ctx::MAX_LANES; ++g) {
    if (h->side[g]) { (void)hipStreamSynchronize(h->side[g]); (void)hipStreamDestroy(h->side[g]); }
    if (h->join[g]) (void)hipEventDestroy(h->join[g]);
  }
  if (h->fork) (void)hipEventDestroy(h->fork);
  if (h->bwd) { (void)hipStreamSynchronize(h->bwd); (void)hipStreamDestroy(h->bwd); }
  for (auto& e : h->bwd_ev)
    if (e) (void)hipEventDestroy(e);
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->cap) { (void)hipStreamSynchronize(h->cap); (void)hipStreamDestroy(h->cap); }
  delete h;
}

}  // extern "C"

int lib_init_error(int code, const char* msg) {
  init_err = msg ? msg : "";
  return code;
}
