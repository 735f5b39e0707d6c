"""Population control and weighted ensemble statistics (oracle side; test infrastructure).

Sec. "Computational Details": the walker population is controlled by the comb method, and for
Theta <= 0.25 by pair branching; results are weighted means over the walkers (Sec.
"Finite-Temperature AFQMC in the Grand Canonical Ensemble": <O> = sum_w w O_w / sum_w w).
The paper cites both methods without restating them; they are written here from their
published definitions:

  comb (Booth, Thom, Alavi 2009; the CPMC-Lab program): with total weight T = sum_i w_i,
  one uniform u in [0, 1) places W teeth at (k + u) T / W, k = 0 .. W-1; walker i receives as
  many copies as teeth fall in [c_{i-1}, c_i), c_i = w_1 + ... + w_i; every copy carries T / W.

  pair branching (Wagner, Bajdich, Mitas 2009, the QWalk program): the walker of largest
  weight w_l is paired with the one of smallest weight w_s while w_l > 2 wbar or w_s < wbar / 2
  (wbar = T / W); with probability w_l / (w_l + w_s) both slots become copies of the heavy
  walker, otherwise of the light one, each with weight (w_l + w_s) / 2.  Pairs are taken in
  order: the p-th largest with the p-th smallest, p = 0, 1, ..., until a pair meets neither
  condition; pair p draws u_p.

Readings (the methods fix which walkers are copied and how often, not where copies live):
  * weights are w_i = exp(ln w_i - max_j ln w_j) for live walkers, 0 for killed and numeric
    ones; the cumulative sums run sequentially from walker 0 upwards;
  * a tooth at t belongs to the first walker with c_i > t; a tooth at or beyond c_W (rounding)
    to the last walker of nonzero weight;
  * ties in the weight order go to the lower walker index;
  * slots: a walker that keeps at least one copy keeps its own slot; further copies fill the
    slots of walkers that keep none, in ascending slot order, taken by copies in tooth order.
    Every copy therefore reads a slot that is not overwritten.
"""
import numpy as np

COMB, PAIR_BRANCH = 0, 1


def _weights(logw, status):
    live = (np.asarray(status) == 0) & np.isfinite(logw)
    if not live.any():
        return None, None
    mx = np.max(np.asarray(logw)[live])
    w = np.where(live, np.exp(np.where(live, logw, mx) - mx), 0.0)
    return w, mx


def comb(logw, status, u):
    """Returns (parent [W] int, new ln w [W]); parent[j] is the walker copied into slot j."""
    logw = np.asarray(logw, dtype=np.float64)
    W = len(logw)
    w, mx = _weights(logw, status)
    if w is None:
        return np.arange(W), logw.copy()
    c = np.cumsum(w)                        # sequential, walker 0 upwards
    total = c[-1]
    step = total / W
    last = int(np.nonzero(w > 0)[0][-1])
    counts = np.zeros(W, dtype=np.int64)
    teeth = []
    i = 0
    for k in range(W):
        t = (k + u) * step
        while i < W and not (c[i] > t):
            i += 1
        owner = i if i < W else last
        counts[owner] += 1
        teeth.append(owner)
        i = min(i, W - 1)
    parent = np.arange(W)
    free = [j for j in range(W) if counts[j] == 0]
    seen = np.zeros(W, dtype=np.int64)
    f = 0
    for owner in teeth:
        seen[owner] += 1
        if seen[owner] > 1:
            parent[free[f]] = owner
            f += 1
    assert f == len(free)
    return parent, np.full(W, np.log(step) + mx)


def pair_branch(logw, status, u, w_hi=2.0, w_lo=0.5):
    """Returns (parent [W] int, new ln w [W])."""
    logw = np.asarray(logw, dtype=np.float64)
    W = len(logw)
    w, mx = _weights(logw, status)
    if w is None:
        return np.arange(W), logw.copy()
    wbar = np.cumsum(w)[-1] / W
    idx = np.arange(W)
    desc = sorted(idx, key=lambda i: (-w[i], i))
    asc = sorted(idx, key=lambda i: (w[i], i))
    parent = np.arange(W)
    new = logw.copy()
    for p in range(W // 2):
        l, s = desc[p], asc[p]
        if not (w[l] > w_hi * wbar or w[s] < w_lo * wbar):
            break
        tot = w[l] + w[s]
        if u[p] * tot < w[l]:
            parent[s] = l
        else:
            parent[l] = s
        new[l] = new[s] = np.log(0.5 * tot) + mx
    return parent, new


def apply(parent, arrays):
    """Copy walker state: arrays are indexed by walker on axis 0; returns the new arrays."""
    return [np.asarray(a)[parent] for a in arrays]


def ensemble_stats(values, logw, status):
    """Weighted statistics of one per-walker estimator over the live walkers:
    mean = sum w O / sum w; the standard error of that ratio estimator by the delta method,
    sqrt(sum w^2 |O - mean|^2) / sum w; and the effective walker count (sum w)^2 / sum w^2."""
    w, mx = _weights(logw, status)
    if w is None:
        return dict(mean=np.nan, stderr=np.nan, n_eff=0.0, sum_w=0.0, ln_wmax=-np.inf)
    O = np.asarray(values)
    sw = np.sum(w)
    mean = np.sum(w * O) / sw
    err = np.sqrt(np.sum(w ** 2 * np.abs(O - mean) ** 2)) / sw
    return dict(mean=mean, stderr=err, n_eff=sw ** 2 / np.sum(w ** 2), sum_w=sw, ln_wmax=mx)
