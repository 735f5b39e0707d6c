"""Estimator and constraint variants on the GPU against the oracle: the thermal Hartree-Fock
trial (Sec. "Results", fig. thf).  FP64 bar: 1e-10 relative for G, energies and ln w."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import ueg, path, energy  # noqa: E402
import synthinputs as si  # noqa: E402

pytestmark = pytest.mark.gpu
FP64_REL = 1e-10


def _F():
    import paper_2012_12228_amd as F
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    F.load_library()
    return F


def _check(rec, G, ref, w):
    for j, r in enumerate(ref["records"]):
        for c, key in enumerate(("E1", "E2", "E", "N")):
            assert abs(rec["trace"][j, w, c] - r[key]) < FP64_REL * abs(r[key]), (w, j, key)
        if np.isfinite(r["logw"]):
            assert abs(rec["logw"][j, w] - r["logw"]) < FP64_REL * max(1.0, abs(r["logw"])), (w, j)
    assert np.abs(G[w] - ref["G"]).max() < FP64_REL * np.abs(ref["G"]).max(), w


@pytest.mark.parametrize("case", ["m19", "m7_fig_thf"])
def test_thermal_hartree_fock_trial(case):
    F = _F()
    if case == "m19":
        sd = dict(n_elec=14, rs=1.0, theta=0.5, nmax2=2, dtau=0.05, stab_every=5, walkers=16)
    else:   # the figure's system: N = 2, M = 7, r_s = 3, beta = 40
        tf = ueg.fermi_temperature(3.0)
        sd = dict(n_elec=2, rs=3.0, theta=1.0 / (40.0 * tf), nmax2=1, dtau=0.05, stab_every=20, walkers=8)
    s = ueg.UEGSystem(sd["n_elec"], sd["rs"], sd["theta"], sd["nmax2"], sd["dtau"], stab_every=sd["stab_every"],
                      trial="thf")
    flds = si.fields(777, sd["walkers"], s.n_slices, s.NQ)
    ctx = F.Context([dict(sd, flags=F.FTAFQMC_TRIAL_THF)])
    inf = ctx.info()
    assert abs(inf["mu_T"] - s.mu_T) < 1e-12 * max(1.0, abs(s.mu_T))
    fe = ueg.UEGSystem(sd["n_elec"], sd["rs"], sd["theta"], sd["nmax2"], sd["dtau"])
    assert abs(inf["mu_T"] - fe.mu_T) > 1e-3                       # the exchange shifts the levels
    ctx.propagate([torch.from_numpy(flds).cuda()])
    rec = ctx.records()
    rec = dict(trace=rec["trace"].cpu().numpy(), logw=rec["logw"].cpu().numpy())
    G = ctx.greens().cpu().numpy()
    for w in range(sd["walkers"]):
        ref = path.run_walker(s, flds[w], energy_fn=energy.local_energy)
        _check(rec, G, ref, w)


@pytest.mark.parametrize("case", ["m19_64walkers", "m57_ragged"])
def test_density_correlation_matches_oracle(case):
    """<rho(Q) rho(-Q)> (the static structure factor times N) per walker and Q, and its weighted
    mean, against the oracle's Wick estimator on the oracle's own G at tau = beta."""
    F = _F()
    if case == "m19_64walkers":
        sd = dict(n_elec=14, rs=1.0, theta=0.5, nmax2=2, dtau=0.05, stab_every=5, walkers=64)
    else:
        sd = dict(n_elec=38, rs=1.0, theta=0.25, nmax2=5, dtau=0.05, stab_every=10, walkers=5)
    s = ueg.UEGSystem(sd["n_elec"], sd["rs"], sd["theta"], sd["nmax2"], sd["dtau"], stab_every=sd["stab_every"])
    flds = si.fields(909, sd["walkers"], s.n_slices, s.NQ)
    ctx = F.Context([sd])
    ctx.propagate([torch.from_numpy(flds).cuda()])
    assert [tuple(q) for q in s.qvec] == ctx.qvectors()
    walker, mean = ctx.density_correlation()
    walker, mean = walker.cpu().numpy(), mean.cpu().numpy()
    refs, lw = [], []
    for w in range(sd["walkers"]):
        ref = path.run_walker(s, flds[w])
        dc = energy.density_correlation(s, ref["G"])
        assert np.abs(walker[w] - dc).max() < FP64_REL * np.abs(dc).max(), w
        refs.append(dc)
        lw.append(ref["logw"])
    lw = np.array(lw)
    wts = np.exp(lw - lw.max())
    want = (wts[:, None] * np.array(refs)).sum(0) / wts.sum()
    assert np.abs(mean - want).max() < FP64_REL * np.abs(want).max()


def test_modified_overlap_constraint_matches_oracle():
    """Eq. ztfix: the constraint uses B_T^n at every slice; records and ftafqmc_energy use the
    estimators' G_k = (I + B_T^{n-k} R_k)^{-1}.  The path is propagated in two calls (7 slices,
    then the rest) so that the estimator G after a partial call is checked too."""
    F = _F()
    sd = dict(n_elec=14, rs=1.0, theta=0.5, nmax2=2, dtau=0.05, stab_every=5, walkers=16)
    s = ueg.UEGSystem(sd["n_elec"], sd["rs"], sd["theta"], sd["nmax2"], sd["dtau"], stab_every=sd["stab_every"])
    flds = si.fields(4141, sd["walkers"], s.n_slices, s.NQ)
    ctx = F.Context([dict(sd, flags=F.FTAFQMC_MODIFIED_OVERLAP)])
    f = torch.from_numpy(flds).cuda()
    ctx.propagate([f], 7)
    e7 = ctx.energy()
    G7 = ctx.greens().cpu().numpy()
    loc7, lw7 = e7["local"].cpu().numpy(), e7["logw"].cpu().numpy()
    ctx.propagate([f])
    rec = ctx.records()
    rec = dict(trace=rec["trace"].cpu().numpy(), logw=rec["logw"].cpu().numpy())
    G = ctx.greens().cpu().numpy()
    differs = 0
    for w in range(sd["walkers"]):
        wk = path.Walker(s, modified=True)
        for k in range(7):
            wk.advance(flds[w, k])
        Gm = wk.measure_greens()
        assert np.abs(G7[w] - Gm).max() < FP64_REL * np.abs(Gm).max(), w
        ref7 = energy.local_energy(s, Gm)
        for c, key in enumerate(("E1", "E2", "E", "N")):
            assert abs(loc7[w, c] - ref7[key]) < FP64_REL * abs(ref7[key]), (w, key)
        assert abs(lw7[w] - wk.logw) < FP64_REL * max(1.0, abs(wk.logw))
        ref = path.run_walker(s, flds[w], energy_fn=energy.local_energy, modified=True)
        _check(rec, G, ref, w)
        std = path.run_walker(s, flds[w])
        differs += abs(std["logw"] - ref["logw"]) > 1e-6
    assert differs == sd["walkers"]                      # the two constraints weigh walkers differently


def test_records_every_slice_and_time_slice_average():
    """FTAFQMC_MEASURE_EVERY_SLICE: a record after every slice; ftafqmc_record_stats' average is
    the mean over slices of the weighted means (the "Average" estimator of fig. averaging)."""
    F = _F()
    sd = dict(n_elec=14, rs=1.0, theta=0.5, nmax2=2, dtau=0.05, stab_every=5, walkers=16)
    s = ueg.UEGSystem(sd["n_elec"], sd["rs"], sd["theta"], sd["nmax2"], sd["dtau"], stab_every=sd["stab_every"])
    flds = si.fields(4242, sd["walkers"], s.n_slices, s.NQ)
    ctx = F.Context([dict(sd, flags=F.FTAFQMC_MEASURE_EVERY_SLICE)])
    ctx.propagate([torch.from_numpy(flds).cuda()])
    rec = ctx.records()
    assert rec["slices"] == list(range(1, s.n_slices + 1))
    assert ctx.info()["refactor_every"] >= 5
    stats, avg = ctx.record_stats()
    stats, avg = stats.cpu().numpy(), avg.cpu().numpy()
    refs = [path.run_walker(s, flds[w], energy_fn=energy.local_energy, measure_every=1) for w in range(sd["walkers"])]
    trace = rec["trace"].cpu().numpy()
    means = []
    for r in range(s.n_slices):
        lw = np.array([ref["records"][r]["logw"] for ref in refs])
        E = np.array([ref["records"][r]["E"] for ref in refs])
        for w in range(sd["walkers"]):
            assert abs(trace[r, w, 2] - E[w]) < FP64_REL * abs(E[w]), (r, w)
        wts = np.exp(lw - lw.max())
        means.append(np.sum(wts * E.real) / wts.sum())
        assert abs(stats[r, 0] - means[-1]) < FP64_REL * abs(means[-1]), r
    assert abs(avg[0] - np.mean(means)) < FP64_REL * abs(np.mean(means)) and avg[2] == s.n_slices
