"""The uniform electron gas in a plane-wave basis (oracle side; test infrastructure).

Conventions follow the paper's Sec. "Uniform Electron Gas" and "Computational
Details":
  * box length L = (4 pi N / 3)^(1/3) r_s, volume Omega = L^3;
  * Fermi temperature k_B T_F = (1/2)(9 pi / 4)^(2/3) / r_s^2 (eq. fermiT) and
    beta = 1 / (Theta T_F);
  * plane waves K = 2 pi n / L for integer n with |n|^2 <= nmax2, ordered by
    (|n|^2, then n lexicographically) -- the ordering is an interface convention;
  * kinetic energy |K|^2 / 2, scaled by the kinetic scale lambda in H_1;
  * Coulomb kernel 4 pi / (Omega |Q|^2) for Q != 0;
  * free-electron trial B_T = exp(-dtau (|K|^2/2 - mu_T)) with mu_T chosen so
    that the trial's thermal electron number is N (Sec. "Phaseless approximation"
    and the free-electron trial of Sec. "Assessing the Phaseless Constraint").

Readings of the paper taken here (each also pinned by a test):
  * Madelung: the printed constant -2.837297 (3/4pi)^(1/3) N^(2/3) / r_s is read
    with a factor 1/2, E_M = -2.837297 N / (2 L), the Hartree-unit value; with it
    the ground state at r_s = 3, N = 2, M = 7 reproduces the paper's FCI energy.
  * The sum-of-squares form of V_ee leaves a diagonal one-body remainder:
    V_ee = (1/4) sum_Q (A(Q)^2 + B(Q)^2) + sum_{K,sigma} h_K n_{K sigma} with
    h_K = -(1/2) sum_{K' != K} 4 pi / (Omega |K - K'|^2).  h_K enters the
    propagator's one-body part only.
  * The slice count is n = round(beta / dtau) and the time step is beta / n.
"""
import numpy as np
from scipy.special import expit

MADELUNG_CONSTANT = 2.837297  # Sec. "Uniform Electron Gas", Madelung energy


def plane_wave_basis(nmax2):
    """Integer vectors n with |n|^2 <= nmax2, sorted by (|n|^2, n_x, n_y, n_z)."""
    r = int(np.floor(np.sqrt(nmax2))) + 1
    pts = [(a, b, c) for a in range(-r, r + 1) for b in range(-r, r + 1)
           for c in range(-r, r + 1) if a * a + b * b + c * c <= nmax2]
    pts.sort(key=lambda v: (v[0] ** 2 + v[1] ** 2 + v[2] ** 2, v[0], v[1], v[2]))
    return np.array(pts, dtype=np.int64)


def fermi_temperature(rs):
    """k_B T_F of the unpolarised gas, eq. fermiT."""
    return 0.5 * (9.0 * np.pi / 4.0) ** (2.0 / 3.0) / rs ** 2


def box_length(n_elec, rs):
    """L = (4 pi N / 3)^(1/3) r_s (Sec. "Computational Details")."""
    return (4.0 * np.pi * n_elec / 3.0) ** (1.0 / 3.0) * rs


def thermal_hartree_fock_levels(eps, vmat, beta, n_elec, tol=1e-14, max_iter=10000):
    """Self-consistent levels of the thermal Hartree-Fock (Mermin) trial, Sec. "Results"
    (fig. thf): per spin e_K = |K|^2/2 - sum_{K' != K} v(K - K') f_K' with
    f_K = 1 / (1 + exp(beta (e_K - mu))) and 2 sum_K f_K = N (the Hartree term Q = 0 is
    removed with the neutralising background; a plane wave is a Hartree-Fock orbital of the
    uniform gas, so the trial stays diagonal).  vmat[K, K'] = v(K - K'), zero on the diagonal.
    Plain fixed-point iteration with mixing 1/2 (the map contracts for these sizes).
    Returns (e [M], mu)."""
    e = eps.copy()
    for _ in range(max_iter):
        mu = trial_chemical_potential(e, beta, n_elec)
        f = expit(-beta * (e - mu))
        e_new = eps - vmat @ f
        if np.max(np.abs(e_new - e)) <= tol * max(1.0, np.max(np.abs(e))):
            e = e_new
            break
        e = 0.5 * (e + e_new)
    else:
        raise RuntimeError("thermal Hartree-Fock iteration did not converge")
    return e, trial_chemical_potential(e, beta, n_elec)


def trial_chemical_potential(eps, beta, n_elec):
    """mu_T with 2 sum_K f(eps_K; mu_T) = N by bisection (spin factor 2)."""
    def count(mu):
        return 2.0 * np.sum(expit(-beta * (eps - mu)))
    lo, hi = eps.min() - 60.0 / beta, eps.max() + 60.0 / beta
    if not (count(lo) < n_elec < count(hi)):
        raise ValueError("electron number not reachable in this basis")
    for _ in range(400):
        mid = 0.5 * (lo + hi)
        if count(mid) < n_elec:
            lo = mid
        else:
            hi = mid
        if hi - lo <= 4e-16 * max(1.0, abs(mid)):
            break
    return 0.5 * (lo + hi)


class UEGSystem:
    """All host-side tables of one UEG system.

    Attributes (M plane waves, NQ momentum transfers):
      nvec [M,3] int, kvec [M,3], eps [M]          basis and |K|^2/2
      qvec [NQ,3] int, idx [M,M] int (-1 on the diagonal), neg [NQ]
      pairs[q] = (p_rows, p_cols): all (p, r) with K_p - K_r = Q_q
      vq [NQ] = 4 pi / (Omega |Q|^2), aq [NQ] = sqrt(pi / (Omega |Q|^2))
      hK [M] one-body remainder, mu_T, mu, kscale, beta, n_slices, dtau, E_M
    """

    def __init__(self, n_elec, rs, theta, nmax2, dtau, stab_every=1, mu=None,
                 kscale=1.0, walkers=None, trial="fe"):
        self.n_elec, self.rs, self.theta, self.nmax2 = int(n_elec), float(rs), float(theta), int(nmax2)
        self.stab_every = int(stab_every)
        self.kscale = float(kscale)
        self.L = box_length(n_elec, rs)
        self.omega = self.L ** 3
        self.T_F = fermi_temperature(rs)
        self.beta = 1.0 / (self.theta * self.T_F)
        self.n_slices = max(1, int(round(self.beta / dtau)))
        self.dtau = self.beta / self.n_slices

        self.nvec = plane_wave_basis(nmax2)
        self.M = len(self.nvec)
        self.kvec = (2.0 * np.pi / self.L) * self.nvec
        self.eps = 0.5 * np.sum(self.kvec ** 2, axis=1)

        # momentum transfers Q = K_p - K_r (p != r), sorted like the basis
        diffs = self.nvec[:, None, :] - self.nvec[None, :, :]
        keyset = {tuple(d) for d in diffs.reshape(-1, 3) if any(d)}
        qs = sorted(keyset, key=lambda v: (v[0] ** 2 + v[1] ** 2 + v[2] ** 2, v[0], v[1], v[2]))
        self.qvec = np.array(qs, dtype=np.int64)
        self.NQ = len(qs)
        where = {q: i for i, q in enumerate(qs)}
        self.idx = -np.ones((self.M, self.M), dtype=np.int64)
        for p in range(self.M):
            for r in range(self.M):
                if p != r:
                    self.idx[p, r] = where[tuple(diffs[p, r])]
        self.neg = np.array([where[(-q[0], -q[1], -q[2])] for q in qs], dtype=np.int64)
        rows, cols = np.nonzero(self.idx >= 0)
        order = np.argsort(self.idx[rows, cols], kind="stable")
        rows, cols = rows[order], cols[order]
        bounds = np.searchsorted(self.idx[rows, cols], np.arange(self.NQ + 1))
        self.pairs = [(rows[bounds[q]:bounds[q + 1]], cols[bounds[q]:bounds[q + 1]])
                      for q in range(self.NQ)]

        q2 = np.sum(((2.0 * np.pi / self.L) * self.qvec) ** 2, axis=1)
        self.vq = 4.0 * np.pi / (self.omega * q2)
        self.aq = np.sqrt(np.pi / (self.omega * q2))

        # h_K = -(1/2) sum_{K' != K} v(K - K')
        self.hK = np.array([-0.5 * np.sum(self.vq[self.idx[p][self.idx[p] >= 0]])
                            for p in range(self.M)])

        # trial levels: free-electron |K|^2/2, or thermal Hartree-Fock
        self.trial = trial
        if trial == "fe":
            self.trial_levels = self.eps.copy()
            self.mu_T = trial_chemical_potential(self.eps, self.beta, self.n_elec)
        elif trial == "thf":
            vmat = np.zeros((self.M, self.M))
            off = self.idx >= 0
            vmat[off] = self.vq[self.idx[off]]
            self.trial_levels, self.mu_T = thermal_hartree_fock_levels(self.eps, vmat, self.beta, self.n_elec)
        else:
            raise ValueError("trial is 'fe' or 'thf'")
        self.mu = self.mu_T if mu is None or (isinstance(mu, float) and np.isnan(mu)) else float(mu)
        self.E_M = -MADELUNG_CONSTANT * self.n_elec / (2.0 * self.L)
        self.walkers = walkers

    # one-body pieces ------------------------------------------------------
    def h1_diag(self):
        """Diagonal of H_1 - mu N per spin: lambda |K|^2/2 + h_K - mu."""
        return self.kscale * self.eps + self.hK - self.mu

    def log_trial_diag(self):
        """log of the diagonal of B_T = exp(-dtau (e_K - mu_T)), e_K = |K|^2/2 (free-electron
        trial) or the thermal Hartree-Fock levels."""
        return -self.dtau * (self.trial_levels - self.mu_T)

    def info(self):
        return dict(M=self.M, n_q=self.NQ, n_slices=self.n_slices, beta=self.beta,
                    dtau=self.dtau, L=self.L, omega=self.omega, mu_T=self.mu_T,
                    mu=self.mu, e_madelung=self.E_M)
