"""Pins of the population-control and ensemble-statistics oracle (oracle/popctl.py).

Both methods must be unbiased: for every walker i, the expected total weight of its copies
over the method's random numbers equals its own weight w_i.  The comb's expectation over
u in [0, 1) is taken exactly (the copy counts are piecewise constant in u; every breakpoint
(c_i / step - k) is enumerated); the pair branch's over each pair's two outcomes.  These are
properties of the definitions, not of the code: a tooth placed at k u instead of k + u, an
interval taken as (c_{i-1}, c_i], a wrong split weight or a swapped keep probability breaks them.
"""
import numpy as np
import pytest

from oracle import popctl


def _weights(seed, W, spread=1.5, dead=()):
    g = np.random.default_rng(seed)
    logw = spread * g.standard_normal(W)
    status = np.zeros(W, dtype=np.int64)
    for d in dead:
        status[d] = 1
        logw[d] = -np.inf
    return logw, status


def _w(logw, status):
    live = (status == 0) & np.isfinite(logw)
    mx = logw[live].max()
    return np.where(live, np.exp(np.where(live, logw, mx) - mx), 0.0), mx


@pytest.mark.parametrize("W,dead", [(8, ()), (37, (3, 4, 20)), (64, (0, 63))])
def test_comb_is_unbiased_exactly_over_u(W, dead):
    logw, status = _weights(7 + W, W, dead=dead)
    w, mx = _w(logw, status)
    c = np.cumsum(w)
    step = c[-1] / W
    bps = {0.0, 1.0}
    for i in range(W):
        for k in range(W):
            u = c[i] / step - k
            if 0.0 < u < 1.0:
                bps.add(u)
    bps = sorted(bps)
    expect = np.zeros(W)
    for a, b in zip(bps[:-1], bps[1:]):
        if b - a < 1e-14:
            continue
        parent, neww = popctl.comb(logw, status, 0.5 * (a + b))
        wnew = np.exp(neww - mx)
        for j in range(W):
            expect[parent[j]] += (b - a) * wnew[j]
    assert np.allclose(expect, w, rtol=1e-10, atol=1e-12 * w.max())


def test_comb_slots_copies_and_weights():
    W = 50
    logw, status = _weights(3, W, spread=2.0, dead=(5, 6))
    w, mx = _w(logw, status)
    for u in (0.0, 0.3141, 0.999):
        parent, neww = popctl.comb(logw, status, u)
        counts = np.bincount(parent, minlength=W)
        step = w.sum() / W
        assert counts.sum() == W
        # every walker holds floor or ceil of w_i / step copies
        assert np.all(counts >= np.floor(w / step - 1e-12)) and np.all(counts <= np.ceil(w / step + 1e-12))
        assert counts[5] == 0 and counts[6] == 0
        kept = counts > 0
        assert np.all(parent[kept] == np.nonzero(kept)[0])          # a kept walker keeps its slot
        assert np.all(kept[parent])                                 # sources are never overwritten
        assert np.allclose(np.exp(neww - mx).sum(), w.sum(), rtol=1e-13)
        assert np.all(neww == neww[0])


@pytest.mark.parametrize("W,dead", [(16, ()), (33, (1, 2, 30)), (64, (10,))])
def test_pair_branch_is_unbiased_and_conserves_weight(W, dead):
    logw, status = _weights(11 + W, W, spread=1.2, dead=dead)
    w, mx = _w(logw, status)
    g = np.random.default_rng(5)
    u = g.random(W)
    parent, neww = popctl.pair_branch(logw, status, u)
    wn = np.where(np.isfinite(neww), np.exp(np.where(np.isfinite(neww), neww, mx) - mx), 0.0)
    assert np.isclose(wn.sum(), w.sum(), rtol=1e-13)
    # the pairs that were processed: slots whose weight changed
    changed = np.nonzero(np.abs(wn - w) > 1e-15 * w.max())[0]
    assert len(changed) % 2 == 0 and len(changed) > 0
    # exact expectation: rerun with u_p = 0 (keep the heavy walker) and u_p -> 1 (keep the light)
    expect = np.zeros(W)
    desc = sorted(range(W), key=lambda i: (-w[i], i))
    asc = sorted(range(W), key=lambda i: (w[i], i))
    npairs = len(changed) // 2
    for p in range(npairs):
        l, s = desc[p], asc[p]
        assert l in changed and s in changed
        tot = w[l] + w[s]
        expect[l] += w[l] / tot * tot          # heavy kept: both slots hold l, weight tot/2 each
        expect[s] += w[s] / tot * tot
    untouched = np.setdiff1d(np.arange(W), changed)
    expect[untouched] += w[untouched]
    assert np.allclose(expect, w, rtol=1e-12)
    # the outcome drawn: both slots of a pair hold one walker with half the pair's weight
    for p in range(npairs):
        l, s = desc[p], asc[p]
        keep = l if u[p] * (w[l] + w[s]) < w[l] else s
        assert parent[l] == keep and parent[s] == keep
        assert np.isclose(wn[l], 0.5 * (w[l] + w[s])) and np.isclose(wn[s], wn[l])
    # afterwards the first unprocessed pair meets neither condition
    wbar = w.sum() / W
    if npairs < W // 2:
        l, s = desc[npairs], asc[npairs]
        assert not (w[l] > 2 * wbar or w[s] < 0.5 * wbar)


def test_pair_branch_revives_dead_slots_and_leaves_balanced_populations():
    W = 20
    logw = np.zeros(W)
    status = np.zeros(W, dtype=np.int64)
    parent, neww = popctl.pair_branch(logw, status, np.full(W, 0.5))
    assert np.array_equal(parent, np.arange(W)) and np.array_equal(neww, logw)
    status[4] = 1
    logw[4] = -np.inf
    parent, neww = popctl.pair_branch(logw, status, np.full(W, 0.99))
    assert parent[4] != 4 and np.isfinite(neww[4])


def test_ensemble_stats_closed_forms():
    g = np.random.default_rng(2)
    O = g.standard_normal(40) + 3.0
    st = popctl.ensemble_stats(O, np.zeros(40), np.zeros(40, dtype=int))
    assert np.isclose(st["mean"], O.mean())
    assert np.isclose(st["stderr"], O.std() / np.sqrt(40))       # population std / sqrt(W)
    assert np.isclose(st["n_eff"], 40.0)
    logw = np.log(np.arange(1, 41, dtype=float))
    st = popctl.ensemble_stats(O, logw, np.zeros(40, dtype=int))
    w = np.arange(1, 41, dtype=float)
    assert np.isclose(st["mean"], np.sum(w * O) / w.sum())
    assert np.isclose(st["n_eff"], w.sum() ** 2 / np.sum(w ** 2))
