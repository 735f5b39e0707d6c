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
