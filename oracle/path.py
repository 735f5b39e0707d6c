"""One walker's phaseless finite-temperature path (oracle side; test infrastructure).

Follows the paper's Sec. "Finite-Temperature AFQMC in the Grand Canonical
Ensemble" (the HS transform, the symmetric Trotter slice propagator eq. B, the
constrained product eq. Abrenda, the overlap ratio eq. ftoratio, the optimal force
bias, the hybrid importance function eq. import, the phaseless projection
eq. phimport/eq. theta) and Sec. "Numerical Stabilization" / "Exploiting the
stack structure" (QRCP -> QDT, stratified products, the D_b/D_s stable inverse).

Readings of the paper taken here:
  * Spin: the method is spin-restricted; every one-body matrix is one M x M block
    shared by both spins, so det(I + A) enters squared and one-body expectation
    values carry a factor 2.
  * HS operators: v_A(Q) = i A(Q)/sqrt(2), v_B(Q) = i B(Q)/sqrt(2), so that
    H_2 = -(1/2) sum v^2 = (1/4) sum (A^2 + B^2); rho(Q) = sum_K a^+_{K+Q} a_K over
    pairs inside the basis (the printed a^+ a^+ is read as a^+ a).
  * Sign: the propagator is exp(+sqrt(dtau) (x - xbar).v) with the printed bias
    xbar = -sqrt(dtau) (<v> - v0); only this pairing cancels the term linear in x
    of ln I.  The mean-field shift v0 vanishes for the diagonal free-electron trial.
  * The force bias uses P(tau) = I - G^T with G = (I + A(tau))^{-1}, A(tau) the
    constrained product of eq. Abrenda at the current slice.
  * The overlap ratio of the step that inserts B_{k+1} is
    det(I + A_{k+1})^2 / det(I + A_k)^2 with the shifted fields; theta is its
    argument; the exponential factor of eq. import enters |I| only.
  * The stable Green's function is the one of the derivation that follows the
    printed formula, G = T^{-1} (D_b Q^dagger T^{-1} + D_s)^{-1} D_b Q^dagger (the
    printed closed form is not consistent with that derivation); Q is unitary.
  * The left block B_T^{n-k} is diagonal, so only the right block needs a QDT
    stack; rows of the combined matrix are ordered by decreasing trial factor
    before the column-pivoted QR (row-sorted QRCP for a row-graded matrix).
  * A dead walker (cos theta <= 0) keeps w = 0, i.e. log w = -inf.
"""
import numpy as np
import scipy.linalg as sla


# --------------------------------------------------------------------------
# Hubbard-Stratonovich fields <-> one-body matrices
# --------------------------------------------------------------------------
def hs_rho_coefficients(sys, yA, yB):
    """Coefficients of rho(Q_q) in sqrt(dtau) * sum_alpha y_alpha v_alpha.

    Field A(Q) multiplies v_A(Q) = i a_Q (rho(Q) + rho(-Q)); field B(Q)
    multiplies v_B(Q) = -a_Q (rho(Q) - rho(-Q)), with a_Q = sqrt(pi/(Omega Q^2))
    and rho(Q)^dagger = rho(-Q) (Sec. "Uniform Electron Gas", A(Q) and B(Q)).
    """
    sdt = np.sqrt(sys.dtau)
    coef = np.zeros(sys.NQ, dtype=np.complex128)
    q = np.arange(sys.NQ)
    np.add.at(coef, q, sdt * 1j * sys.aq * yA)
    np.add.at(coef, sys.neg, sdt * 1j * sys.aq * yA)
    np.add.at(coef, q, -sdt * sys.aq * yB)
    np.add.at(coef, sys.neg, sdt * sys.aq * yB)
    return coef


def one_body_matrix(sys, coef):
    """sum_q coef_q rho(Q_q) as an M x M matrix: entry (p, r) of rho(Q) is 1 iff K_p - K_r = Q."""
    V = np.zeros((sys.M, sys.M), dtype=np.complex128)
    for q in range(sys.NQ):
        V[sys.pairs[q]] = coef[q]
    return V


def rho_expectation(sys, P):
    """<rho(Q_q)> per spin = sum over pairs (p, r) with K_p - K_r = Q_q of P_pr."""
    return np.array([P[sys.pairs[q]].sum() for q in range(sys.NQ)], dtype=np.complex128)


def force_bias(sys, P):
    """Optimal force bias xbar_alpha = -sqrt(dtau) (<v_alpha> - v0_alpha), v0 = 0.

    <v_alpha> = 2 sum_pq (v_alpha)_pq P_pq (two spins) with P = I - G^T.
    Returns (xbar_A, xbar_B), each complex [NQ].
    """
    r = rho_expectation(sys, P)
    vA = 2.0 * 1j * sys.aq * (r + r[sys.neg])
    vB = 2.0 * (-sys.aq) * (r - r[sys.neg])
    sdt = np.sqrt(sys.dtau)
    return -sdt * vA, -sdt * vB


def importance_exponent(xA, xB, xbA, xbB):
    """Exponent of the exponential factor of the importance function, eq. import.

    Sampling the shifted field x - xbar instead of x multiplies each walker's weight by
    exp(sum_alpha [x_alpha xbar_alpha - xbar_alpha^2 / 2]) (the Gaussian density ratio of
    the shift), summed over both fields A(Q) and B(Q) of every momentum transfer.  The
    shift may be complex; the sum is returned complex (its real part enters |I|).
    """
    return np.sum(xA * xbA + xB * xbB - 0.5 * (xbA ** 2 + xbB ** 2))


def slice_propagator(sys, yA, yB):
    """B = e^{-dtau/2 (H_1 - mu N)} e^{sqrt(dtau) y.v} e^{-dtau/2 (H_1 - mu N)}, eq. B."""
    V = one_body_matrix(sys, hs_rho_coefficients(sys, yA, yB))
    kh = np.exp(-0.5 * sys.dtau * sys.h1_diag())
    return kh[:, None] * sla.expm(V) * kh[None, :]


# --------------------------------------------------------------------------
# QDT factorisation and the stable Green's function
# --------------------------------------------------------------------------
def _logdet(A):
    sign, logabs = np.linalg.slogdet(A)
    return np.log(sign) + logabs


def qdt_update(C, T_prev, row_grading=None):
    """QRCP C = Q R Pi, D = diag R, T = (D^{-1} R)(Pi T_prev) (stratification step).

    With row_grading the rows are first ordered by decreasing |row_grading| and
    the order is undone in Q.
    """
    if row_grading is not None:
        order = np.argsort(-np.abs(row_grading), kind="stable")
        Qs, R, piv = sla.qr(C[order], pivoting=True)
        Q = np.empty_like(Qs)
        Q[order] = Qs
    else:
        Q, R, piv = sla.qr(C, pivoting=True)
    D = np.diagonal(R).copy()
    T = (R / D[:, None]) @ T_prev[piv, :]
    return Q, D, T


def greens_from_qdt(Q, D, T):
    """G = (I + Q D T)^{-1} and ln det(I + Q D T) via the D_b/D_s split.

    I + QDT = Q D_b^{-1} (D_b Q^dagger T^{-1} + D_s) T, hence
    G = T^{-1} (D_b Q^dagger T^{-1} + D_s)^{-1} D_b Q^dagger.
    """
    M = len(D)
    absD = np.abs(D)
    big = absD > 1.0
    Db = np.where(big, 1.0 / np.where(big, absD, 1.0), 1.0)
    Ds = np.where(big, D / np.where(big, absD, 1.0), D)
    Tinv = sla.solve(T, np.eye(M, dtype=np.complex128))
    Qh = Q.conj().T
    mid = Db[:, None] * (Qh @ Tinv) + np.diag(Ds)
    G = Tinv @ sla.solve(mid, Db[:, None] * Qh)
    lndet = _logdet(Q) - np.sum(np.log(Db)) + _logdet(mid) + _logdet(T)
    return G, lndet


class RightBlock:
    """QDT factors of the sampled product R_k = B_k ... B_1 (identity at k = 0)."""

    def __init__(self, M):
        self.Q = np.eye(M, dtype=np.complex128)
        self.D = np.ones(M, dtype=np.complex128)
        self.T = np.eye(M, dtype=np.complex128)

    def push(self, B):
        """R <- B R by C = (B Q) D -> QRCP (one stratification step)."""
        self.Q, self.D, self.T = qdt_update((B @ self.Q) * self.D[None, :], self.T)

    def product(self):
        return (self.Q * self.D[None, :]) @ self.T


def greens_at(sys, right, k, lexp=None):
    """G_k = (I + B_T^{n-k} R_k)^{-1} and ln det(I + B_T^{n-k} R_k).

    The left block is the diagonal B_T^{n-k} (B_T^lexp when lexp is given); C = B_T^{n-k} Q_R D_R
    is factorised by row-sorted QRCP and combined with T_R.
    """
    left = np.exp((sys.n_slices - k if lexp is None else lexp) * sys.log_trial_diag())
    C = left[:, None] * right.Q * right.D[None, :]
    Q, D, T = qdt_update(C, right.T, row_grading=left)
    return greens_from_qdt(Q, D, T)


def wrap_angle(x):
    """Map an angle to (-pi, pi]."""
    y = np.mod(x + np.pi, 2.0 * np.pi) - np.pi
    return np.where(y == -np.pi, np.pi, y)


# --------------------------------------------------------------------------
# One walker along the whole path
# --------------------------------------------------------------------------
ALIVE, KILLED, NUMERIC = 0, 1, 2


def shifted_one_body(sys, G, z_k):
    """The shifted one-body matrix V = sqrt(dtau) (x - xbar).v of a slice with fields z_k and
    the force bias from G, and the exponent of eq. import."""
    xbA, xbB = force_bias(sys, np.eye(sys.M) - G.T)
    xA, xB = z_k.real, z_k.imag
    V = one_body_matrix(sys, hs_rho_coefficients(sys, xA - xbA, xB - xbB))
    return V, importance_exponent(xA, xB, xbA, xbB)


def run_walker(sys, z, measure_every=None, energy_fn=None, keep_greens=False, stop_after=None,
               record_path=False, modified=False, make_walker=None):
    """Propagate one walker from tau = 0 to tau = beta with fields z[k, q].

    stop_after: end the path after that many slices (a bounded sample for timing).
    record_path: also return the sampled path, i.e. the shifted one-body matrix V_k and the
    weight exponent of every slice (out["path"]), so that replay_walker can re-run it.
    modified: the constraint of the modified overlap ratio, eq. ztfix (see Walker).
    make_walker: a factory for the walker object (default Walker(sys, modified)); the low-rank
    variant of Sec. "Exploiting the low-rank structure" plugs in here.

    z: complex [n_slices, NQ]; Re z = field of A(Q), Im z = field of B(Q).
    Measures the local energy (energy_fn(sys, G)) after slice k+1 when
    (k+1) % measure_every == 0 and at k+1 = n.
    Returns a dict with per-slice ln S and theta, per-measurement records, the
    final G, ln det(I + A) and the weight.
    """
    Vs, expos = [], []

    def shifted(k, G):
        V, expo = shifted_one_body(sys, G, z[k])
        if record_path:
            Vs.append(V)
            expos.append(expo)
        return V, expo

    out = _walk(sys, shifted, measure_every, energy_fn, keep_greens, stop_after, modified, make_walker)
    if record_path:
        out["path"] = dict(V=Vs, expo=expos)
    return out


def replay_walker(sys, frozen, measure_every=None, energy_fn=None, keep_greens=False):
    """Re-run a recorded path: the shifted one-body matrices V_k and weight exponents are
    taken from `frozen` (run_walker(..., record_path=True)["path"]) instead of the force bias,
    while the one-body factors K = exp(-dtau/2 (lambda eps + h - mu)) come from `sys`.
    Holding the path fixed makes the weight and the estimators plain functions of mu and
    lambda (the frozen-path derivatives are taken of exactly these functions)."""
    def recorded(k, G):
        return frozen["V"][k], frozen["expo"][k]
    return _walk(sys, recorded, measure_every, energy_fn, keep_greens, None)


class Walker:
    """One walker at slice k: the QDT factors of its sampled product R_k, G_k and
    ln det(I + A_k) (A_k = B_T^{n-k} R_k), ln w and its status.  step() inserts the next slice
    propagator and applies the phaseless weight update; copy() clones the walker (population
    control copies whole walkers).

    modified=True takes the constraint from the modified overlap ratio of eq. ztfix,
    S~_k = tr(B_T^n B_k ... B_1) / tr(B_T^n B_{k-1} ... B_1), i.e. A_k = B_T^n R_k at every slice:
    G, ln det, the force bias, S and theta all use it (the trial raised to the n-th power
    throughout, Sec. "The T -> 0 limit").  Estimators still use G_k = (I + B_T^{n-k} R_k)^{-1}
    (measure_greens)."""

    def __init__(self, sys, modified=False):
        self.sys = sys
        self.k = 0
        self.modified = modified
        self.right = self._new_right()
        self.G, self.ell = self._greens(0, self._lexp(0))
        self.logw, self.status = 0.0, ALIVE

    def _new_right(self):
        return RightBlock(self.sys.M)

    def _greens(self, k, lexp):
        return greens_at(self.sys, self.right, k, lexp)

    def _lexp(self, k):
        return self.sys.n_slices if self.modified else self.sys.n_slices - k

    def measure_greens(self):
        """G_k = (I + B_T^{n-k} R_k)^{-1}, the Green's function of the estimators."""
        if not self.modified:
            return self.G
        return self._greens(self.k, self.sys.n_slices - self.k)[0]

    def copy(self):
        w = Walker.__new__(Walker)
        w.sys, w.k, w.modified = self.sys, self.k, self.modified
        w.right = RightBlock(self.sys.M)
        w.right.Q, w.right.D, w.right.T = self.right.Q.copy(), self.right.D.copy(), self.right.T.copy()
        w.G, w.ell, w.logw, w.status = self.G.copy(), self.ell, self.logw, self.status
        return w

    def advance(self, z_k):
        """One slice with fields z_k (force bias from this walker's G_k)."""
        return self.step(*shifted_one_body(self.sys, self.G, z_k))

    def step(self, V, expo):
        """Slice k -> k+1 with B = K e^V K (eq. B); returns (ln S, theta, ln |I|)."""
        sys, k = self.sys, self.k
        kh = np.exp(-0.5 * sys.dtau * sys.h1_diag())
        B = kh[:, None] * sla.expm(V) * kh[None, :]          # eq. B
        self.right.push(B)
        self.G, ell_new = self._greens(k + 1, self._lexp(k + 1))
        lnS = 2.0 * (ell_new - self.ell)
        self.ell = ell_new
        theta = float(wrap_angle(lnS.imag))
        lnI = lnS.real + expo.real
        if self.status == ALIVE:
            if not (np.all(np.isfinite(self.G)) and np.isfinite(lnI)):
                self.status, self.logw = NUMERIC, -np.inf
            elif np.cos(theta) <= 0.0:
                self.status, self.logw = KILLED, -np.inf
            else:
                self.logw += lnI + np.log(np.cos(theta))
        self.k = k + 1
        return lnS, theta, lnI


def _walk(sys, shifted, measure_every, energy_fn, keep_greens, stop_after, modified=False, make_walker=None):
    n = sys.n_slices
    s = sys.stab_every if measure_every is None else measure_every
    wk = Walker(sys, modified) if make_walker is None else make_walker()
    ell0 = wk.ell
    lnS_all = np.zeros(n, dtype=np.complex128)
    theta_all = np.zeros(n)
    lnI_all = np.zeros(n)
    alive_after = np.zeros(n, dtype=bool)
    records, greens = [], []
    greens_all = [wk.G.copy()] if keep_greens == "all" else None
    for k in range(n if stop_after is None else min(n, int(stop_after))):
        V, expo = shifted(k, wk.G)
        lnS_all[k], theta_all[k], lnI_all[k] = wk.step(V, expo)
        alive_after[k] = wk.status == ALIVE
        if greens_all is not None:
            greens_all.append(wk.G.copy())
        if (k + 1) % s == 0 or k + 1 == n:
            rec = dict(slice=k + 1, logw=wk.logw, status=wk.status, lndet=wk.ell)
            if energy_fn is not None:
                rec.update(energy_fn(sys, wk.measure_greens()))
            records.append(rec)
            if keep_greens:
                greens.append(wk.measure_greens().copy())
    return dict(G=wk.measure_greens(), G_constraint=wk.G, lndet=wk.ell, lndet0=ell0, logw=wk.logw, status=wk.status, lnS=lnS_all,
                theta=theta_all, lnI=lnI_all, alive=alive_after, records=records, greens=greens,
                greens_all=greens_all, right=wk.right, walker=wk)
