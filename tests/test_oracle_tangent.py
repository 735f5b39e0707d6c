"""Pins of the oracle's frozen-path derivatives in mu and the kinetic scale lambda.

Each check compares the doubled-product tangent with something it does not compute itself:
central differences of the replayed path, high-precision differences of the plain product at
cond ~1e30, the closed form of the mu direction, and the non-interacting Fermi-Dirac limit.
"""
import copy

import numpy as np
import pytest

import synthinputs as si
from oracle import energy, path, tangent, ueg

PARAMS = ("mu", "kscale")


def _shifted(s, param, h):
    s2 = copy.copy(s)
    if param == "mu":
        s2.mu = s.mu + h
    else:
        s2.kscale = s.kscale + h
    return s2


def _replay_obs(s, fwd):
    r = path.replay_walker(s, fwd["path"], energy_fn=energy.local_energy)
    rec = r["records"][-1]
    return r["logw"], rec["E"], rec["N"], r["status"]


@pytest.fixture(scope="module")
def cfg1_walkers():
    s = ueg.UEGSystem(14, 1.0, 0.5, 2, 0.05, stab_every=5)
    out = []
    for w in range(6):
        z = si.walker_fields(122281, w, s.n_slices, s.NQ)
        out.append((z,) + tangent.walker_tangents(s, z))
    return s, out


@pytest.mark.parametrize("param", PARAMS)
def test_walker_tangent_matches_central_differences(cfg1_walkers, param):
    """d ln w, dE, dN of each walker against (f(p+h) - f(p-h)) / 2h of the replayed path."""
    s, walkers = cfg1_walkers
    h = 1e-5
    for z, fwd, tans in walkers:
        plus = _replay_obs(_shifted(s, param, h), fwd)
        minus = _replay_obs(_shifted(s, param, -h), fwd)
        t = tans[param]
        fd_lw = (plus[0] - minus[0]) / (2 * h)
        fd_E = (plus[1] - minus[1]) / (2 * h)
        fd_N = (plus[2] - minus[2]) / (2 * h)
        assert t["dlogw"] == pytest.approx(fd_lw, rel=1e-8, abs=1e-8)
        assert abs(t["dE"] - fd_E) <= 1e-8 * max(1.0, abs(fd_E))
        assert abs(t["dN"] - fd_N) <= 1e-8 * max(1.0, abs(fd_N))


@pytest.mark.parametrize("param", PARAMS)
def test_ensemble_tangent_matches_central_differences(cfg1_walkers, param):
    """d<E>, d<N> of the weighted ensemble mean against central differences of the replay."""
    s, walkers = cfg1_walkers
    h = 1e-5
    means = {}
    for sgn in (+1, -1):
        obs = [_replay_obs(_shifted(s, param, sgn * h), fwd) for _, fwd, _ in walkers]
        lw = np.array([o[0] for o in obs])
        st = np.array([o[3] for o in obs])
        E = np.array([o[1] for o in obs])
        N = np.array([o[2] for o in obs])
        means[sgn] = (tangent.ensemble_tangent(E, E, lw, lw, st)[0],
                      tangent.ensemble_tangent(N, N, lw, lw, st)[0])
    lw = np.array([fwd["logw"] for _, fwd, _ in walkers])
    st = np.array([fwd["status"] for _, fwd, _ in walkers])
    dl = np.array([t[param]["dlogw"] for _, _, t in walkers])
    E = np.array([fwd["E"]["E"] for _, fwd, _ in walkers])
    dE = np.array([t[param]["dE"] for _, _, t in walkers])
    N = np.array([fwd["E"]["N"] for _, fwd, _ in walkers])
    dN = np.array([t[param]["dN"] for _, _, t in walkers])
    _, dmE = tangent.ensemble_tangent(E, dE, lw, dl, st)
    _, dmN = tangent.ensemble_tangent(N, dN, lw, dl, st)
    fdE = (means[1][0] - means[-1][0]) / (2 * h)
    fdN = (means[1][1] - means[-1][1]) / (2 * h)
    assert abs(dmE - fdE) <= 1e-7 * max(1.0, abs(fdE))
    assert abs(dmN - fdN) <= 1e-7 * max(1.0, abs(fdN))


def test_mu_direction_equals_closed_form(cfg1_walkers):
    """With the path frozen, B_k(mu) = e^{dtau mu} B_k(0): d ln det(I + A_k) = k dtau tr(I - G_k)
    and dG_n = -beta (I - G_n) G_n, from the forward Green's functions alone."""
    s, walkers = cfg1_walkers
    for z, fwd, tans in walkers:
        cf = tangent.mu_tangent_closed_form(s, path.run_walker(s, z, keep_greens="all"))
        t = tans["mu"]
        assert np.abs(cf["dlnS"] - t["dlnS"]).max() < 1e-11
        assert np.abs(cf["dG"] - t["dG"]).max() < 1e-12
        assert t["dlogw"] == pytest.approx(cf["dlogw"], rel=1e-12)
        assert abs(t["dE"] - cf["dE"]) < 1e-11 * max(1.0, abs(cf["dE"]))


def test_zero_field_fermi_dirac_derivatives():
    """z = 0: the force bias of a diagonal G vanishes, every slice is diagonal and
    G_n = 1 - f with f = 1/(1 + e^{beta (lambda eps + h - mu)}).  Then
    dN/dmu = 2 beta sum f(1-f), dN/dlambda = -2 beta sum eps f(1-f),
    d ln w/dmu = 2 beta sum f, d ln w/dlambda = -2 beta sum eps f, and the exchange energy
    E2 = -sum_{p != r} v(K_p - K_r) f_p f_r."""
    s = ueg.UEGSystem(14, 1.0, 0.5, 2, 0.05, stab_every=5)
    z = np.zeros((s.n_slices, s.NQ), dtype=np.complex128)
    fwd, tans = tangent.walker_tangents(s, z)
    b = s.beta
    x = b * (s.kscale * s.eps + s.hK - s.mu)
    f = 1.0 / (1.0 + np.exp(x))
    dfm = b * f * (1 - f)                 # df/dmu
    dfl = -b * s.eps * f * (1 - f)        # df/dlambda
    vpr = np.zeros((s.M, s.M))
    mask = s.idx >= 0
    vpr[mask] = s.vq[s.idx[mask]]
    for param, df, dlw in (("mu", dfm, 2 * b * np.sum(f)), ("kscale", dfl, -2 * b * np.sum(s.eps * f))):
        t = tans[param]
        dE1 = 2 * s.kscale * np.sum(s.eps * df) + (2 * np.sum(s.eps * f) if param == "kscale" else 0.0)
        dE2 = -2.0 * f @ vpr @ df
        assert t["dN"] == pytest.approx(2 * np.sum(df), rel=1e-11)
        assert t["dE1"] == pytest.approx(dE1, rel=1e-11)
        assert t["dE2"] == pytest.approx(dE2, rel=1e-10)
        assert t["dlogw"] == pytest.approx(dlw, rel=1e-11)


def test_energy_tangent_is_the_derivative_of_the_local_energy():
    """The estimator is at most quadratic in P, so a central difference along dG is exact up to
    rounding; checked on random complex G, dG with the kinetic scale varied too."""
    s = ueg.UEGSystem(14, 1.0, 0.5, 2, 0.05)
    g = np.random.default_rng(3)
    G = g.normal(size=(s.M, s.M)) + 1j * g.normal(size=(s.M, s.M))
    dG = g.normal(size=(s.M, s.M)) + 1j * g.normal(size=(s.M, s.M))
    h = 1e-3
    sp, sm = _shifted(s, "kscale", h), _shifted(s, "kscale", -h)
    Ep = energy.local_energy(sp, G + h * dG)
    Em = energy.local_energy(sm, G - h * dG)
    t = tangent.energy_tangent(s, G, dG, 1.0)
    for key in ("E1", "E2", "E", "N"):
        fd = (Ep[key] - Em[key]) / (2 * h)
        assert abs(t["d" + key] - fd) <= 1e-9 * max(1.0, abs(fd)), key


def test_doubled_tangent_at_cond_1e30_against_high_precision():
    """M = 7 at Theta = 0.035 (dynamic range ~1e30): the per-slice d ln S_k and dG at tau = beta
    in lambda against central differences of the plain product in 80-digit arithmetic."""
    mp = pytest.importorskip("mpmath")
    s = ueg.UEGSystem(2, 0.5, 0.035, 1, 0.05, stab_every=1)
    z = si.walker_fields(5, 1, s.n_slices, s.NQ)
    fwd, tans = tangent.walker_tangents(s, z, params=("kscale",))
    t = tans["kscale"]
    mp.mp.dps = 80
    M, n = s.M, s.n_slices
    Es = [mp.matrix(path.sla.expm(V).tolist()) for V in fwd["path"]["V"]]
    h = mp.mpf("1e-25")
    dt = mp.mpf(s.dtau)
    lt = [-dt * (mp.mpf(s.eps[i]) - mp.mpf(s.mu_T)) for i in range(M)]

    def run(lam):
        kh = [mp.exp(-dt / 2 * (lam * mp.mpf(s.eps[i]) + mp.mpf(s.hK[i]) - mp.mpf(s.mu))) for i in range(M)]
        K = mp.diag(kh)
        R = mp.eye(M)
        dets = []
        for k in range(n + 1):
            L = mp.diag([mp.exp((n - k) * lt[i]) for i in range(M)])
            dets.append(mp.det(mp.eye(M) + L * R))
            if k < n:
                R = K * Es[k] * K * R
        return dets, mp.inverse(mp.eye(M) + R)

    dp, Gp = run(mp.mpf(s.kscale) + h)
    dm, Gm = run(mp.mpf(s.kscale) - h)
    for k in range(n):
        ref = complex(2 * (mp.log(dp[k + 1] / dm[k + 1]) - mp.log(dp[k] / dm[k])) / (2 * h))
        assert abs(t["dlnS"][k] - ref) <= 1e-11 * max(1.0, abs(ref)), k
    dGref = np.array([[complex((Gp[i, j] - Gm[i, j]) / (2 * h)) for j in range(M)] for i in range(M)])
    assert np.abs(t["dG"] - dGref).max() < 1e-13
    assert np.abs(dGref).max() > 1e-2      # the derivative is not trivially small here


# ---------------------------------------------------------------- pathwise ---
def _pathwise_fd(kw, z, param, h=1e-5):
    base = dict(mu=ueg.UEGSystem(**kw).mu_T, kscale=1.0)
    out = {}
    for sg in (1, -1):
        b = dict(base)
        b[param] += sg * h
        sp = ueg.UEGSystem(mu=b["mu"], kscale=b["kscale"], **kw)
        o = path.run_walker(sp, z, energy_fn=energy.local_energy)
        out[sg] = (o["logw"], o["records"][-1]["E"], o["records"][-1]["N"])
    return [(out[1][i] - out[-1][i]) / (2 * h) for i in range(3)]


@pytest.mark.parametrize("param", ["mu", "kscale"])
@pytest.mark.parametrize("walker", [0, 3])
def test_pathwise_tangent_matches_central_differences(param, walker):
    """Raw fields held fixed, force bias recomputed: the tangent equals central differences
    (h = 1e-5) of the whole path in ln w, E and N at tau = beta (1e-7 relative: the difference
    quotient's own error is ~h^2)."""
    kw = dict(n_elec=14, rs=1.0, theta=0.5, nmax2=2, dtau=0.05, stab_every=5)
    s = ueg.UEGSystem(**kw)
    z = si.walker_fields(77, walker, s.n_slices, s.NQ)
    fwd, t = tangent.pathwise_tangent(s, z, param)
    assert tangent.kink_margin(fwd) > 1e-3
    fd = _pathwise_fd(kw, z, param)
    for got, want in ((t["dlogw"], fd[0]), (t["dE"], fd[1]), (t["dN"], fd[2])):
        assert abs(got - want) < 1e-7 * max(1.0, abs(want)), (got, want)
    # and it is not the frozen-path derivative (the force-bias feedback moves the path)
    fz = tangent.path_tangent(s, path.run_walker(s, z, record_path=True, energy_fn=energy.local_energy), param)
    assert abs(fz["dlogw"] - t["dlogw"]) > 1e-3


def test_pathwise_equals_frozen_with_zero_fields():
    """Zero fields keep G diagonal, so r_Q = 0 and dr_Q = 0 for every Q: the force bias does not
    move and the pathwise derivative is the frozen one (the mu direction in closed form)."""
    kw = dict(n_elec=14, rs=1.0, theta=0.5, nmax2=2, dtau=0.05, stab_every=5)
    s = ueg.UEGSystem(**kw)
    z = np.zeros((s.n_slices, s.NQ), dtype=np.complex128)
    fwd, t = tangent.pathwise_tangent(s, z, "mu")
    ref = path.run_walker(s, z, energy_fn=energy.local_energy, keep_greens="all")
    cf = tangent.mu_tangent_closed_form(s, ref)
    assert np.allclose(t["dlnS"], cf["dlnS"], rtol=1e-10, atol=1e-12)
    assert abs(t["dlogw"] - cf["dlogw"]) < 1e-10 * max(1.0, abs(cf["dlogw"]))
    assert np.allclose(t["dG"], cf["dG"], atol=1e-12)
    assert np.all(np.abs(t["dexpo"]) < 1e-14)


def test_pathwise_ensemble_means_match_differences():
    """d<E>/dmu and d<N>/dmu of the weighted means over 6 walkers, pathwise, against central
    differences of the means."""
    kw = dict(n_elec=14, rs=1.0, theta=0.5, nmax2=2, dtau=0.05, stab_every=5)
    s = ueg.UEGSystem(**kw)
    zs = [si.walker_fields(78, w, s.n_slices, s.NQ) for w in range(6)]
    vals, dvals, lw, dlw, st = [], [], [], [], []
    for z in zs:
        fwd, t = tangent.pathwise_tangent(s, z, "mu")
        vals.append(fwd["E"]["N"]); dvals.append(t["dN"]); lw.append(fwd["logw"]); dlw.append(t["dlogw"])
        st.append(fwd["status"])
    _, dmean = tangent.ensemble_tangent(np.array(vals), np.array(dvals), np.array(lw), np.array(dlw), np.array(st))
    h = 1e-5
    means = []
    for sg in (1, -1):
        sp = ueg.UEGSystem(mu=s.mu_T + sg * h, **kw)
        outs = [path.run_walker(sp, z, energy_fn=energy.local_energy) for z in zs]
        l = np.array([o["logw"] for o in outs])
        w = np.exp(l - l.max())
        means.append(np.sum(w * np.array([o["records"][-1]["N"] for o in outs])) / w.sum())
    fd = (means[0] - means[1]) / (2 * h)
    assert abs(dmean - fd) < 1e-7 * abs(fd)
