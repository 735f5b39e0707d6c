"""Low-rank truncation of the stratified product (oracle side; test infrastructure).

Follows Sec. "Exploiting the low-rank structure": the threshold of eq. thresh on the diagonal
factors of the left and right blocks, the reduced-rank stratified step that combines them into
A = q d t (q: M x m_T, d: m_T x m_T, t: m_T x M), the Woodbury Green's function, the matrix
determinant lemma and the low-rank one-body density matrix; the threshold 1e-6 of
Sec. "Computational Details"; the compression percentages c_i = (1 - m_i / M) 100% of
Sec. "Efficacy of the Low-Rank Truncation".

Readings taken here:
  * Left block.  A_L = B_T^{n-k} is diagonal in the plane-wave basis, so its column-pivoted QR is
    the sort of its entries: q_L selects the plane waves in order of decreasing trial factor,
    d_L holds their factors and t_L = q_L^T.  Eq. thresh keeps the factors >= threshold
    (m_L of them).
  * Right block.  Stratified at every slice as in the full-rank path (QRCP of B q_R d_R, then
    t_R <- (D^{-1} R)(Pi t_R)); eq. thresh drops the trailing columns with |D| < threshold, so
    q_R is M x m_R, d_R is m_R x m_R, t_R is m_R x M, and the right rank never grows again.
  * Total.  c = d_L t_L q_R d_R (m_L x m_R; its rows are already ordered by decreasing trial
    factor, the row-sorted QRCP of a row-graded matrix), QRCP c = q' r' Pi' with the economic
    shapes, so m_T = min(m_L, m_R); q = q_L q', d = diag r', t = (d^{-1} r')(Pi' t_R).
  * Stable inverse.  The paper rewrites I + d t q through the inverse of t q.  Here the
    algebraically equal forms with d = d_s / d_b (the split of Sec. "Numerical Stabilization")
    are used, which need no inverse of t q:
        I + d t q = d_b^{-1} (d_b + d_s t q),
        G = I - q (d_b + d_s t q)^{-1} d_s t,
        ln det(I + q d t) = ln det(d_b + d_s t q) - sum ln d_b.
  * The one-body density matrix is P = I - G^T = t^T d_s (d_b + d_s t q)^{-T} q^T, of rank m_T.
  * m_R, m_T and the compression of a slice are those of the Green's function formed after
    that slice's propagator is inserted; the initial slice (R_0 = I) has m_R = M.
  * The two thresholds can be set apart (right_threshold): 0 keeps the whole right block and
    truncates the left block only.  That variant is the one whose result does not depend on how
    the right block is factorised (the left block is diagonal, its kept set is exact).
"""
import numpy as np
import scipy.linalg as sla

from . import path as _path

THRESHOLD = 1e-6          # eq. thresh, the value of Sec. "Computational Details"


def split_d(d):
    """d = d_s / d_b with d_b = 1/max(1, |d|) and d_s = d/max(1, |d|)."""
    a = np.abs(d)
    big = a > 1.0
    db = np.where(big, 1.0 / np.where(big, a, 1.0), 1.0)
    ds = np.where(big, d / np.where(big, a, 1.0), d)
    return db, ds


class LowRankRight:
    """Right block R_k = q_R diag(d_R) t_R with eq. thresh applied at every stratification."""

    def __init__(self, M, threshold):
        self.threshold = threshold
        self.last_D = np.ones(M)          # |D| of the last stratification before the truncation
        self.Q = np.eye(M, dtype=np.complex128)
        self.D = np.ones(M, dtype=np.complex128)
        self.T = np.eye(M, dtype=np.complex128)

    @property
    def rank(self):
        return len(self.D)

    def push(self, B):
        """R <- B R: QRCP of (B q_R) d_R, t_R <- (D^{-1} R)(Pi t_R), then drop |D| < threshold."""
        if self.rank == 0:
            return
        C = (B @ self.Q) * self.D[None, :]
        Q, R, piv = sla.qr(C, pivoting=True, mode="economic")
        D = np.diagonal(R).copy()
        T = (R / D[:, None]) @ self.T[piv, :]
        self.last_D = np.abs(D)
        keep = np.abs(D) >= self.threshold
        self.Q, self.D, self.T = Q[:, keep], D[keep], T[keep, :]

    def product(self):
        return (self.Q * self.D[None, :]) @ self.T


def left_block(sys, lexp, threshold):
    """Eq. thresh on the diagonal left block B_T^lexp: the kept plane waves in order of decreasing
    trial factor and their factors (q_L = columns of I at `S`, d_L = `dl`)."""
    left = np.exp(lexp * sys.log_trial_diag())
    order = np.argsort(-left, kind="stable")
    S = order[left[order] >= threshold]
    return S, left[S]


def lowrank_factors(sys, right, lexp, threshold):
    """A = B_T^lexp R ~ q diag(d) t by the reduced-rank step; returns (q, d, t, m_L, m_R, m_T)."""
    M = sys.M
    S, dl = left_block(sys, lexp, threshold)
    mL, mR = len(S), right.rank
    if mL == 0 or mR == 0:
        z = np.zeros((M, 0), dtype=np.complex128)
        return z, np.zeros(0, dtype=np.complex128), z.T.copy(), mL, mR, 0
    c = dl[:, None] * (right.Q[S, :] * right.D[None, :])       # d_L t_L q_R d_R
    qc, rc, piv = sla.qr(c, pivoting=True, mode="economic")
    d = np.diagonal(rc).copy()
    t = (rc / d[:, None]) @ right.T[piv, :]
    q = np.zeros((M, len(d)), dtype=np.complex128)
    q[S, :] = qc                                                 # q_L q'
    return q, d, t, mL, mR, len(d)


def lowrank_greens(sys, right, lexp, threshold):
    """G = (I + q d t)^{-1} by Woodbury and ln det(I + q d t) by the determinant lemma, both in
    m_T dimensions; returns (G, ln det, P, (m_L, m_R, m_T))."""
    M = sys.M
    q, d, t, mL, mR, mT = lowrank_factors(sys, right, lexp, threshold)
    if mT == 0:
        I = np.eye(M, dtype=np.complex128)
        return I, 0.0 + 0.0j, np.zeros((M, M), dtype=np.complex128), (mL, mR, 0)
    db, ds = split_d(d)
    core = np.diag(db) + ds[:, None] * (t @ q)                  # d_b + d_s t q
    W = np.linalg.solve(core, ds[:, None] * t)                  # (d_b + d_s t q)^{-1} d_s t
    G = np.eye(M, dtype=np.complex128) - q @ W
    sign, logabs = np.linalg.slogdet(core)
    lndet = np.log(sign) + logabs - np.sum(np.log(db))
    P = W.T @ q.T                                               # t^T d_s (d_b + d_s t q)^{-T} q^T
    return G, lndet, P, (mL, mR, mT)


def compression(m, M):
    """c_i = (1 - m_i / M) x 100 %."""
    return (1.0 - np.asarray(m, dtype=float) / M) * 100.0


class LowRankWalker(_path.Walker):
    """A walker whose Green's function and ln det come from the truncated reduced-rank product.
    `ranks` lists (m_L, m_R, m_T) of every Green's function formed (index 0: before slice 1);
    `right_D` the |D| spectrum of the right block's stratification at each (before eq. thresh)."""

    def __init__(self, sys, threshold=THRESHOLD, right_threshold=None):
        self.threshold = threshold
        self.right_threshold = threshold if right_threshold is None else right_threshold
        self.ranks = []
        self.right_D = []
        self.lowrank_P = None
        super().__init__(sys, modified=False)

    def _new_right(self):
        return LowRankRight(self.sys.M, self.right_threshold)

    def _greens(self, k, lexp):
        G, lndet, P, ranks = lowrank_greens(self.sys, self.right, lexp, self.threshold)
        self.ranks.append(ranks)
        self.right_D.append(self.right.last_D.copy())
        self.lowrank_P = P
        return G, lndet


def run_walker_lowrank(sys, z, threshold=THRESHOLD, energy_fn=None, measure_every=None, keep_greens=False,
                       right_threshold=None):
    """path.run_walker with the low-rank walker; adds out["ranks"] [n + 1][3] = (m_L, m_R, m_T)
    and out["right_D"] (the right block's |D| before truncation at every formation)."""
    out = _path.run_walker(sys, z, measure_every=measure_every, energy_fn=energy_fn, keep_greens=keep_greens,
                           make_walker=lambda: LowRankWalker(sys, threshold, right_threshold))
    out["ranks"] = np.array(out["walker"].ranks, dtype=int)
    out["right_D"] = out["walker"].right_D
    return out
