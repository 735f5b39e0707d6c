"""Pins of the oracle's low-rank truncation (oracle.lowrank; Sec. "Exploiting the low-rank
structure", eq. thresh) against what the mathematics fixes:
  * threshold 0 keeps every column and reproduces the full-rank path;
  * with zero fields every block is diagonal: the kept sets, the ranks (m_L, m_R, m_T), G and
    ln det of the truncated product have closed forms;
  * the Woodbury G, the determinant lemma and the low-rank P against 80-digit arithmetic on the
    explicit truncated product q d t;
  * the truncation at 1e-6 moves the weight and the energy of a walker by far less than the
    threshold where it is active (dynamic range ~1e30).
"""
import numpy as np
import pytest

from oracle import ueg, path, lowrank, energy
import synthinputs as si

COND30 = dict(n_elec=2, rs=0.5, theta=0.035, nmax2=1, dtau=0.05, stab_every=1)
M57_LOWT = dict(n_elec=14, rs=1.0, theta=0.0625, nmax2=5, dtau=0.05, stab_every=10)


@pytest.mark.parametrize("kw,seed", [(dict(n_elec=14, rs=1.0, theta=0.5, nmax2=2, dtau=0.05, stab_every=5), 77),
                                     (COND30, 5)])
def test_threshold_zero_is_the_full_rank_path(kw, seed):
    s = ueg.UEGSystem(**kw)
    for w in (0, 3):
        z = si.walker_fields(seed, w, s.n_slices, s.NQ)
        full = path.run_walker(s, z, energy_fn=energy.local_energy)
        lr = lowrank.run_walker_lowrank(s, z, threshold=0.0, energy_fn=energy.local_energy)
        assert lr["status"] == full["status"]
        assert abs(lr["logw"] - full["logw"]) < 1e-12 * max(1.0, abs(full["logw"]))
        assert np.abs(lr["G"] - full["G"]).max() < 1e-12
        for a, b in zip(lr["records"], full["records"]):
            for key in ("E", "N"):
                assert abs(a[key] - b[key]) < 1e-12 * max(1.0, abs(b[key]))
        assert np.all(lr["ranks"] == s.M)


@pytest.mark.parametrize("right_threshold", [None, 0.0], ids=["both", "left_only"])
@pytest.mark.parametrize("kw", [COND30, M57_LOWT])
def test_zero_fields_closed_form(kw, right_threshold):
    """Zero fields: R_k = diag(e^{-k dtau h}) and A_k = diag(B_T^{n-k} R_k).  The left block keeps
    (n-k) ln B_T >= ln thr, the right block every K with -j dtau h_K >= ln thr for all j <= k
    (a dropped column never returns), m_T = min(m_L, m_R), and G_KK = 1/(1 + A_KK) on the kept
    intersection, 1 elsewhere."""
    s = ueg.UEGSystem(**kw)
    thr = lowrank.THRESHOLD
    n, M = s.n_slices, s.M
    z = np.zeros((n, s.NQ), dtype=np.complex128)
    out = lowrank.run_walker_lowrank(s, z, keep_greens="all", right_threshold=right_threshold)
    # keep_greens="all" records G after every slice through the walker's greens
    lt, h = s.log_trial_diag(), s.h1_diag()
    lnthr = np.log(thr)
    assert out["status"] == path.ALIVE
    ranks = out["ranks"]
    truncated_somewhere = False
    wk = lowrank.LowRankWalker(s, thr, right_threshold)
    for k in range(n + 1):
        keepL = (n - k) * lt >= lnthr
        keepR = np.ones(M, dtype=bool) if k == 0 or right_threshold == 0.0 else np.all(
            [-j * s.dtau * h >= lnthr for j in range(1, k + 1)], axis=0)
        mL, mR = int(keepL.sum()), int(keepR.sum())
        assert tuple(ranks[k]) == (mL, mR, min(mL, mR)), k
        truncated_somewhere |= mL < M or mR < M
        a = np.exp((n - k) * lt - k * s.dtau * h)
        both = keepL & keepR
        gd = np.where(both, 1.0 / (1.0 + a), 1.0)
        if k > 0:
            wk.step(np.zeros((M, M), dtype=np.complex128), 0.0)
        assert np.abs(wk.G - np.diag(gd)).max() < 1e-13, k
        assert abs(wk.ell - np.sum(np.log1p(a[both]))) < 1e-12 * max(1.0, abs(wk.ell)), k
    assert truncated_somewhere


def test_woodbury_determinant_lemma_and_lowrank_P_at_80_digits():
    """At slices of the 1e30 path where the truncation is active, G, ln det(I + q d t) and P from
    the m_T-dimensional forms equal the explicit inverse and determinant of the M x M truncated
    product I + q diag(d) t evaluated with 80-digit arithmetic."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 80
    s = ueg.UEGSystem(**COND30)
    z = si.walker_fields(5, 1, s.n_slices, s.NQ)
    wk = lowrank.LowRankWalker(s)
    checked = 0
    for k in range(s.n_slices):
        wk.advance(z[k])
        if k % 13 != 12:
            continue
        lexp = s.n_slices - wk.k
        q, d, t, mL, mR, mT = lowrank.lowrank_factors(s, wk.right, lexp, lowrank.THRESHOLD)
        assert mT == min(mL, mR)
        if mT == s.M:
            continue
        G, lndet, P, _ = lowrank.lowrank_greens(s, wk.right, lexp, lowrank.THRESHOLD)
        A = mp.matrix(s.M, s.M)
        for i in range(s.M):
            for j in range(s.M):
                A[i, j] = mp.fsum(mp.mpc(q[i, a]) * mp.mpc(d[a]) * mp.mpc(t[a, j]) for a in range(mT))
        X = mp.eye(s.M) + A
        Gx = X ** -1
        Gn = np.array([[complex(Gx[i, j]) for j in range(s.M)] for i in range(s.M)])
        assert np.abs(G - Gn).max() < 1e-13 * max(1.0, np.abs(Gn).max())
        ld = mp.log(mp.det(X))
        assert abs(lndet.real - float(mp.re(ld))) < 1e-12 * max(1.0, abs(float(mp.re(ld))))
        assert abs(np.exp(1j * (lndet.imag - float(mp.im(ld)))) - 1.0) < 1e-12
        assert np.abs(P - (np.eye(s.M) - Gn.T)).max() < 1e-13
        checked += 1
    assert checked >= 2


def test_truncation_moves_results_far_below_the_threshold():
    """Eq. thresh at 1e-6 on a path with dynamic range ~1e30 (m_T down to 1): the weight, G and the
    energy of every walker stay within 1e-9 of the full-rank path."""
    s = ueg.UEGSystem(**COND30)
    active = 0
    for w in range(4):
        z = si.walker_fields(5, w, s.n_slices, s.NQ)
        full = path.run_walker(s, z, energy_fn=energy.local_energy)
        lr = lowrank.run_walker_lowrank(s, z, energy_fn=energy.local_energy)
        active += int(lr["ranks"][:, 2].min() < s.M)
        assert lr["status"] == full["status"]
        if full["status"] != path.ALIVE:
            continue
        assert abs(lr["logw"] - full["logw"]) < 1e-9
        assert np.abs(lr["G"] - full["G"]).max() < 1e-9
        assert abs(lr["records"][-1]["E"] - full["records"][-1]["E"]) < 1e-9
    assert active == 4


def test_compression_percentages():
    assert np.allclose(lowrank.compression([0, 97, 485], 485), [100.0, 80.0, 0.0])
