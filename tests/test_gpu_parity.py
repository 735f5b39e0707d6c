"""Parity of the HIP path (through the C ABI) with the FP64 oracle on identical seeded fields.

Tolerances (written here, derived in the design notes):
  FP64 path   -- relative 1e-10 for G (max-norm), E_1, E_2, E, N; ln w to 1e-10 * max(1, |ln w|);
                 status words identical.
  mixed path  -- complex64 propagator GEMMs with FP32 accumulation, FP64 everything else:
                 E_1 and E_2 relative 1e-6 each, E_1 + E_2 to 1e-6 (|E_1| + |E_2|) (the
                 condition scale of a sum: at large r_s the two nearly cancel),
                 N relative 1e-6, G relative 1e-5; ln w absolute
                 2e-7 M (1 + k/10) after k slices: ln w = 2 Re(l_k - l_0) + sum of per-slice
                 terms, where the error of l_k = ln det(I + A_k) is about M eps_fp32 (one
                 rounding-limited contribution per eigenvalue) and the per-slice terms add a
                 slowly growing part.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import ueg, path, energy  # noqa: E402
import synthinputs as si  # noqa: E402

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
FP64_REL = 1e-10
MIX_E12, MIX_N, MIX_G = 1e-6, 1e-6, 1e-5
# element-by-element G against stored oracle entries: (rtol of the entry, atol of the largest
# entry).  FP64: every entry to FP64_REL of itself (the scale-split solve keeps each entry's
# relative accuracy; 2e-12 observed at M = 123, 171, 485).  Mixed: the FP32 chain perturbs G by
# about MIX_G of its norm, so small entries move further relative to themselves (2.3e-7 of the
# largest entry observed).
G_ELEM_TOL = {False: (FP64_REL, 1e-14), True: (MIX_G, 1e-6)}


def mix_logw_tol(M, k):
    return 2e-7 * M * (1.0 + k / 10.0)


def _F():
    import paper_2012_12228_amd as F
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    F.load_library()
    return F


def oracle_system(sd):
    return ueg.UEGSystem(sd["n_elec"], sd["rs"], sd["theta"], sd["nmax2"], sd["dtau"],
                         stab_every=sd.get("stab_every", 10), mu=sd.get("mu"), kscale=sd.get("kscale", 1.0))


def gpu_run(F, systems, fields_list, n_slices=None):
    ctx = F.Context(systems)
    fds = [torch.from_numpy(np.ascontiguousarray(f)).cuda() for f in fields_list]
    ctx.propagate(fds, n_slices)
    torch.cuda.synchronize()
    return ctx, fds


def relc(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def rel_mat(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def check_mixed_energy(e1, e2, nn, r1, r2, rn, label):
    assert relc(e1, r1) < MIX_E12, label
    assert relc(e2, r2) < MIX_E12, label
    assert abs((e1 + e2) - (r1 + r2)) < MIX_E12 * (abs(r1) + abs(r2)), label
    assert relc(nn, rn) < MIX_N, label


def check_walker(rec_gpu, logw_gpu, G_gpu, ref, mixed=False, label=""):
    """rec_gpu [n_rec][4] complex, logw_gpu [n_rec]; ref: oracle output dict."""
    recs = ref["records"]
    assert len(recs) == rec_gpu.shape[0], label
    for j, r in enumerate(recs):
        e1, e2, e, nn = rec_gpu[j]
        if mixed:
            check_mixed_energy(e1, e2, nn, r["E1"], r["E2"], r["N"], (label, j))
        else:
            for got, want in ((e1, r["E1"]), (e2, r["E2"]), (e, r["E"]), (nn, r["N"])):
                assert relc(got, want) < FP64_REL, (label, j, got, want)
        if np.isfinite(r["logw"]):
            tol = mix_logw_tol(G_gpu.shape[0], r["slice"]) if mixed else FP64_REL * max(1.0, abs(r["logw"]))
            assert abs(logw_gpu[j] - r["logw"]) < tol, (label, j, logw_gpu[j], r["logw"])
        else:
            assert logw_gpu[j] == -np.inf, (label, j)
    if G_gpu is not None:
        assert rel_mat(G_gpu, ref["G"]) < (MIX_G if mixed else FP64_REL), label


# --------------------------------------------------------------- small ---
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_m19_all_walkers_full_path(precision):
    F = _F()
    wl = si.WORKLOADS["ueg_n14_m19"]
    sd = dict(wl["systems"][0], precision=precision)
    s = oracle_system(sd)
    W = sd["walkers"]
    flds = si.fields(si.system_seed("ueg_n14_m19", 0), W, s.n_slices, s.NQ)
    ctx, _ = gpu_run(F, [sd], [flds])
    inf = ctx.info()
    assert (inf["M"], inf["n_q"], inf["n_slices"]) == (s.M, s.NQ, s.n_slices)
    assert inf["mu_T"] == pytest.approx(s.mu_T, rel=1e-13)
    rec = ctx.records()
    trace = rec["trace"].cpu().numpy()
    logw = rec["logw"].cpu().numpy()
    G = ctx.greens().cpu().numpy()
    for w in range(W):
        ref = path.run_walker(s, flds[w], energy_fn=energy.local_energy)
        check_walker(trace[:, w], logw[:, w], G[w], ref, mixed=precision == 1, label="walker %d" % w)
    assert rec["slices"] == [r["slice"] for r in ref["records"]]


def test_ragged_m57_every_slice_stabilised_and_kscale_mu():
    """M=57 (ragged against 16/64 tiles), stabilisation every slice, lambda != 1, explicit mu."""
    F = _F()
    sd = dict(n_elec=38, rs=1.0, theta=0.25, nmax2=5, dtau=0.05, stab_every=1, walkers=5,
              kscale=0.85, mu=1.2)
    s = oracle_system(sd)
    flds = si.fields(77, sd["walkers"], s.n_slices, s.NQ)
    ctx, _ = gpu_run(F, [sd], [flds])
    rec = ctx.records()
    G = ctx.greens().cpu().numpy()
    for w in range(sd["walkers"]):
        ref = path.run_walker(s, flds[w], energy_fn=energy.local_energy)
        check_walker(rec["trace"].cpu().numpy()[:, w], rec["logw"].cpu().numpy()[:, w], G[w], ref, label=w)


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_m257_wide_gauss_jordan_steps(precision):
    """M = 257: above the order where the Green's function solve takes 64-column Gauss-Jordan
    steps (two 32-column panels, one K = 64 update); the last step is 32 + 1 columns."""
    F = _F()
    sd = dict(n_elec=66, rs=1.0, theta=0.5, nmax2=16, dtau=0.1, stab_every=4, walkers=2, precision=precision)
    s = oracle_system(sd)
    assert s.M == 257
    flds = si.fields(2571, sd["walkers"], s.n_slices, s.NQ)
    ctx, _ = gpu_run(F, [sd], [flds])
    rec = ctx.records()
    G = ctx.greens().cpu().numpy()
    for w in range(sd["walkers"]):
        ref = path.run_walker(s, flds[w], energy_fn=energy.local_energy)
        check_walker(rec["trace"].cpu().numpy()[:, w], rec["logw"].cpu().numpy()[:, w], G[w], ref,
                     mixed=precision == 1, label=w)


def test_profile_class_mask():
    """Profiling only the GEMM class records only GEMM launches (same count as with every class);
    values other than 1 or FTAFQMC_PROFILE_ONLY | mask are rejected."""
    F = _F()
    sd = dict(si.WORKLOADS["ueg_n14_m19"]["systems"][0], walkers=4)
    s = oracle_system(sd)
    flds = torch.from_numpy(si.fields(3, 4, s.n_slices, s.NQ)).cuda()
    ctx = F.Context(sd)
    ctx.profile(True)
    ctx.propagate(flds)
    full = ctx.profile(False)
    ctx.reset()
    ctx.profile(True, classes=["gemm"])
    ctx.propagate(flds)
    only = ctx.profile(False)
    assert only["gemm"][1] == full["gemm"][1] > 0
    assert all(v[1] == 0 for k, v in only.items() if k != "gemm")
    assert full["elim"][1] > 0
    lib = F.load_library()
    ms = (F.ctypes.c_double * len(F.PROF_CLASSES))()
    cnt = (F.ctypes.c_longlong * len(F.PROF_CLASSES))()
    for bad in (2, F.FTAFQMC_PROFILE_ONLY, F.FTAFQMC_PROFILE_ONLY | (1 << 12)):
        assert lib.ftafqmc_profile(ctx.handle, bad, ms, cnt) != 0
    ctx.close()


def test_single_walker_stabilised_only_at_the_end():
    F = _F()
    sd = dict(n_elec=14, rs=1.0, theta=0.5, nmax2=2, dtau=0.05, stab_every=1000, walkers=1)
    s = oracle_system(sd)
    flds = si.fields(5, 1, s.n_slices, s.NQ)
    ctx, _ = gpu_run(F, [sd], [flds])
    rec = ctx.records()
    assert rec["slices"] == [s.n_slices]
    ref = path.run_walker(s, flds[0], energy_fn=energy.local_energy)
    check_walker(rec["trace"].cpu().numpy()[:, 0], rec["logw"].cpu().numpy()[:, 0], ctx.greens().cpu().numpy()[0], ref)


def test_zero_fields_closed_form():
    F = _F()
    sd = dict(n_elec=14, rs=1.0, theta=0.5, nmax2=2, dtau=0.05, stab_every=5, walkers=3)
    s = oracle_system(sd)
    ctx, _ = gpu_run(F, [sd], [np.zeros((3, s.n_slices, s.NQ), complex)])
    lev = s.eps + s.hK - s.mu
    occ = 1 / (1 + np.exp(s.beta * lev))
    G = ctx.greens().cpu().numpy()
    for w in range(3):
        assert np.abs(G[w] - np.diag(1 - occ)).max() < 1e-13
    e = ctx.energy()
    ell_n = np.sum(np.log1p(np.exp(-s.beta * lev)))
    ell_0 = np.sum(np.log1p(np.exp(-s.beta * (s.eps - s.mu_T))))
    assert np.allclose(e["logw"].cpu().numpy(), 2 * (ell_n - ell_0), rtol=1e-12)
    assert e["mean"].cpu().numpy()[3].real == pytest.approx(2 * occ.sum(), rel=1e-12)


def test_slicewise_calls_clamp_and_match_one_call():
    F = _F()
    sd = dict(n_elec=14, rs=1.0, theta=0.5, nmax2=2, dtau=0.05, stab_every=5, walkers=4)
    s = oracle_system(sd)
    flds = si.fields(9, 4, s.n_slices, s.NQ)
    a, fa = gpu_run(F, [sd], [flds])
    b = F.Context([sd])
    fb = torch.from_numpy(flds).cuda()
    b.propagate([fb], 0)
    assert b.info()["slice"] == 0
    for _ in range(s.n_slices + 3):
        b.propagate([fb], 1)
    torch.cuda.synchronize()
    assert b.info()["slice"] == s.n_slices
    assert torch.equal(a.greens(), b.greens())
    b.reset()
    b.propagate([fb])
    torch.cuda.synchronize()
    assert torch.equal(a.greens(), b.greens())
    assert b.info()["n_measure"] == a.info()["n_measure"]


def test_bitwise_reproducible():
    F = _F()
    sd = dict(si.WORKLOADS["ueg_n14_m19"]["systems"][0], walkers=16)
    s = oracle_system(sd)
    flds = si.fields(3, 16, s.n_slices, s.NQ)
    a, _ = gpu_run(F, [sd], [flds])
    b, _ = gpu_run(F, [sd], [flds])
    assert torch.equal(a.greens(), b.greens())
    assert torch.equal(a.records()["trace"], b.records()["trace"])


def test_phaseless_kills_match_oracle():
    """Fields of twice the unit variance at r_s = 2 kill half the walkers (cos theta <= 0) while
    every slice's Taylor remainder bound stays below 1e-14: kills, survivors' weights and the
    final G match the oracle."""
    F = _F()
    sd = dict(n_elec=14, rs=2.0, theta=0.5, nmax2=2, dtau=0.05, stab_every=5, walkers=24)
    s = oracle_system(sd)
    flds = 2.0 * si.fields(4242, 24, s.n_slices, s.NQ)
    ctx, _ = gpu_run(F, [sd], [flds])
    e = ctx.energy()
    st = e["status"].cpu().numpy()
    refs = [path.run_walker(s, flds[w]) for w in range(24)]
    want = np.array([r["status"] for r in refs])
    assert (want == path.KILLED).sum() >= 6 and (want == path.ALIVE).sum() >= 6
    assert np.array_equal(st, want)
    lw = e["logw"].cpu().numpy()
    assert np.all(np.isinf(lw[want == path.KILLED]))
    G = ctx.greens().cpu().numpy()
    for w in range(24):
        if want[w] == path.ALIVE:
            assert abs(lw[w] - refs[w]["logw"]) < FP64_REL * max(1.0, abs(refs[w]["logw"])), w
        assert rel_mat(G[w], refs[w]["G"]) < FP64_REL, w


def test_taylor_bound_flags_oversized_fields():
    """Fields of six times the unit variance make the degree-16 Taylor polynomial of e^V
    inaccurate (remainder bound ~1e-7).  The device check must flag such walkers numeric: no
    walker may stay alive with a truncated exponential."""
    F = _F()
    sd = dict(n_elec=14, rs=1.0, theta=0.5, nmax2=2, dtau=0.05, stab_every=5, walkers=8)
    s = oracle_system(sd)
    flds = 6.0 * si.fields(4242, 8, s.n_slices, s.NQ)
    ctx, _ = gpu_run(F, [sd], [flds])
    assert ctx.info()["taylor_degree"] == 16
    e = ctx.energy()
    st = e["status"].cpu().numpy()
    assert np.all(st == path.NUMERIC), st
    assert np.all(np.isinf(e["logw"].cpu().numpy()))
    assert torch.isnan(e["mean"]).all()


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_large_dtau_raises_taylor_degree(precision):
    """dtau = 0.2 (four times the workload's step): the a-priori norm estimate of V raises the
    Taylor degree to 20 (FP64; the V^4 product's epilogue writes three of the four lower blocks
    and an elementwise pass the last) or 16 (mixed), and the path matches the oracle (expm)."""
    F = _F()
    sd = dict(n_elec=14, rs=1.0, theta=0.5, nmax2=2, dtau=0.2, stab_every=2, walkers=16, precision=precision)
    s = oracle_system(sd)
    flds = si.fields(2002, sd["walkers"], s.n_slices, s.NQ)
    ctx, _ = gpu_run(F, [sd], [flds])
    assert ctx.info()["taylor_degree"] == (20 if precision == 0 else 16)
    rec = ctx.records()
    G = ctx.greens().cpu().numpy()
    st = ctx.energy()["status"].cpu().numpy()
    for w in range(sd["walkers"]):
        ref = path.run_walker(s, flds[w], energy_fn=energy.local_energy)
        assert st[w] == ref["status"] == path.ALIVE, w
        check_walker(rec["trace"].cpu().numpy()[:, w], rec["logw"].cpu().numpy()[:, w], G[w], ref,
                     mixed=precision == 1, label=w)


@pytest.mark.parametrize("case", ["m19_theta0.0625_stab_n", "m19_theta0.5_stab_n"])
def test_stab_every_n_is_refactorised_or_flagged(case):
    """stab_every = n (one stabilisation, at the end): at Theta = 0.0625 (r_s = 0.5) the product's
    kinetic range over 43 slices is e^23, beyond one Cholesky-QR pass, so the library re-factorises
    every 10 slices on its own (records stay at slice n); at Theta = 0.5 one pass at slice 22
    suffices.  Every walker matches the oracle to 1e-10 or is flagged numeric; none is alive and
    wrong."""
    F = _F()
    if case.startswith("m19_theta0.0625"):
        sd = dict(n_elec=14, rs=0.5, theta=0.0625, nmax2=2, dtau=0.05, walkers=32)
    else:
        sd = dict(n_elec=14, rs=1.0, theta=0.5, nmax2=2, dtau=0.05, walkers=32)
    s = oracle_system(dict(sd, stab_every=1))
    sd["stab_every"] = s.n_slices
    flds = si.fields(4343, sd["walkers"], s.n_slices, s.NQ)
    ctx, _ = gpu_run(F, [sd], [flds])
    inf = ctx.info()
    assert inf["refactor_every"] == (10 if case.startswith("m19_theta0.0625") else 43)
    rec = ctx.records()
    assert rec["slices"] == [s.n_slices]
    st = ctx.energy()["status"].cpu().numpy()
    G = ctx.greens().cpu().numpy()
    s.stab_every = s.n_slices
    alive = 0
    for w in range(sd["walkers"]):
        ref = path.run_walker(s, flds[w], energy_fn=energy.local_energy)
        if st[w] == path.NUMERIC:
            continue
        assert st[w] == ref["status"], w
        check_walker(rec["trace"].cpu().numpy()[:, w], rec["logw"].cpu().numpy()[:, w], G[w], ref, label=w)
        alive += 1
    assert alive == sd["walkers"]            # the re-factorisation cap keeps every pass conditioned


def test_weighted_means_under_unequal_weights():
    """ftafqmc_energy's d_mean is sum_w w O_w / sum_w w over live walkers: checked against the
    oracle's per-walker values and weights (ln w spread over several units) at 1e-10."""
    F = _F()
    wl = si.WORKLOADS["ueg_n14_m19"]
    sd = dict(wl["systems"][0])
    s = oracle_system(sd)
    W = sd["walkers"]
    flds = si.fields(si.system_seed("ueg_n14_m19", 0), W, s.n_slices, s.NQ)
    ctx, _ = gpu_run(F, [sd], [flds])
    mean = ctx.energy()["mean"].cpu().numpy()
    refs = [path.run_walker(s, flds[w], energy_fn=energy.local_energy) for w in range(W)]
    lw = np.array([r["logw"] for r in refs])
    live = np.array([r["status"] == path.ALIVE for r in refs])
    assert live.sum() == W and lw.max() - lw.min() > 1.0       # genuinely unequal weights
    wts = np.exp(lw - lw.max())
    for c, key in enumerate(("E1", "E2", "E", "N")):
        vals = np.array([r["records"][-1][key] for r in refs])
        want = np.sum(wts * vals) / np.sum(wts)
        assert relc(mean[c], want) < FP64_REL, (key, mean[c], want)
        unweighted = vals.mean()
        assert relc(unweighted, want) > 1e3 * FP64_REL          # the weights matter at this tolerance


def test_greens_complex64_copy_and_dtype_checks():
    F = _F()
    sd = dict(n_elec=14, rs=1.0, theta=0.5, nmax2=2, dtau=0.05, stab_every=5, walkers=4)
    s = oracle_system(sd)
    flds = si.fields(31, 4, s.n_slices, s.NQ)
    ctx, _ = gpu_run(F, [sd], [flds])
    g128 = ctx.greens(dtype=torch.complex128)
    g64 = ctx.greens(dtype=torch.complex64)
    torch.cuda.synchronize()
    assert torch.equal(g64, g128.to(torch.complex64))
    for bad in (torch.empty((4, s.M, s.M), dtype=torch.float32, device="cuda"),
                torch.empty((4, s.M, s.M + 1), dtype=torch.complex128, device="cuda"),
                torch.empty((4, s.M, 2 * s.M), dtype=torch.complex128, device="cuda")[:, :, ::2]):
        with pytest.raises(ValueError):
            F.ftafqmc_greens(ctx.handle, 0, bad, ctx.device)


@pytest.mark.parametrize("nmax2,n_elec", [(2, 14), (5, 38), (9, 38)], ids=["m19", "m57", "m123"])
def test_nan_fields_flag_only_that_walker(nmax2, n_elec):
    """A NaN field marks its walker failed (status 2) and leaves the others bit-identical: with
    32-column steps (M=19) and with 64-column steps (M=57: one step narrower than the panel;
    M=123: two row slots), where the failed walker's pivot searches find no usable pivot."""
    F = _F()
    sd = dict(n_elec=n_elec, rs=1.0, theta=0.5, nmax2=nmax2, dtau=0.05, stab_every=5, walkers=4)
    s = oracle_system(sd)
    flds = si.fields(21, 4, s.n_slices, s.NQ)
    bad = flds.copy()
    bad[2, 3, 5] = np.nan
    clean, _ = gpu_run(F, [sd], [flds])
    dirty, _ = gpu_run(F, [sd], [bad])
    st = dirty.energy()["status"].cpu().numpy()
    assert list(st) == [0, 0, 2, 0]
    Gc, Gd = clean.greens(), dirty.greens()
    for w in (0, 1, 3):
        assert torch.equal(Gc[w], Gd[w])


# ---------------------------------------------------- full-size, sampled ---
def _golden(name):
    fn = os.path.join(GOLDEN, "oracle_%s.npz" % name)
    if not os.path.exists(fn):
        pytest.skip("stored oracle outputs missing: run tests/golden/make_oracle_golden.py")
    return np.load(fn)


def _check_golden(gold, key, trace, logw, G, slices, mixed=False):
    assert list(gold[key + "_slices"]) == list(slices)
    E = gold[key + "_E"]
    lw = gold[key + "_logw"]
    for j in range(len(slices)):
        if mixed:
            check_mixed_energy(trace[j, 0], trace[j, 1], trace[j, 3], E[j, 0], E[j, 1], E[j, 3], (key, j))
        else:
            for c in range(4):
                assert relc(trace[j, c], E[j, c]) < FP64_REL, (key, j, c, trace[j, c], E[j, c])
        tol = mix_logw_tol(G.shape[0], slices[j]) if mixed else FP64_REL * max(1.0, abs(lw[j]))
        assert abs(logw[j] - lw[j]) < tol, (key, j, logw[j], lw[j])
    tol = MIX_G if mixed else FP64_REL
    assert rel_mat(np.diagonal(G), gold[key + "_G_diag"]) < tol
    rows = gold[key + "_G_rows"]
    assert rel_mat(G[:rows.shape[0]], rows) < tol
    # element by element: the stored rows and the seeded entries, each within rtol of itself plus
    # atol of the matrix's largest entry
    scale = max(np.abs(rows).max(), np.abs(gold[key + "_G_diag"]).max())
    rtol, atol = G_ELEM_TOL[mixed]
    got, want = [G[:rows.shape[0]].ravel()], [rows.ravel()]
    if key + "_G_samp" in gold.files:
        got.append(G[gold[key + "_G_samp_i"], gold[key + "_G_samp_j"]])
        want.append(gold[key + "_G_samp"])
    got, want = np.concatenate(got), np.concatenate(want)
    excess = (np.abs(got - want) - rtol * np.abs(want)) / scale
    assert excess.max() <= atol, (key, float(excess.max()))


def _full_size(name, precision, flags=0):
    F = _F()
    wl = si.WORKLOADS[name]
    gold = _golden(name)
    systems = [dict(sd, precision=precision, flags=flags) for sd in wl["systems"]]
    oss = [oracle_system(sd) for sd in systems]
    flds = [si.fields(si.system_seed(name, i), sd["walkers"], s.n_slices, s.NQ)
            for i, (sd, s) in enumerate(zip(systems, oss))]
    ctx, _ = gpu_run(F, systems, flds)
    for i in range(len(systems)):
        rec = ctx.records(i)
        trace, logw = rec["trace"].cpu().numpy(), rec["logw"].cpu().numpy()
        G = ctx.greens(i).cpu().numpy()
        for key in gold.files:
            if key.startswith("s%d_w" % i) and key.endswith("_slices"):
                k = key[:-len("_slices")]
                w = int(k.split("_w")[1])
                _check_golden(gold, k, trace[:, w], logw[:, w], G[w], rec["slices"], mixed=precision == 1)
    return ctx


def test_m171_full_size_fp64():
    _full_size("ueg_n66_m171", 0)


def test_m171_full_size_mixed():
    _full_size("ueg_n66_m171", 1)


def test_m171_full_size_mixed_bf16_split():
    """The mixed path with its propagator products on the BF16 matrix cores (three-way split
    operands, FTAFQMC_BF16_SPLIT) to the same mixed-precision bars."""
    F = _F()
    _full_size("ueg_n66_m171", 1, F.FTAFQMC_BF16_SPLIT)


def test_m19_all_walkers_mixed_bf16_split():
    F = _F()
    wl = si.WORKLOADS["ueg_n14_m19"]
    sd = dict(wl["systems"][0], precision=1, flags=F.FTAFQMC_BF16_SPLIT)
    s = oracle_system(sd)
    W = sd["walkers"]
    flds = si.fields(si.system_seed("ueg_n14_m19", 0), W, s.n_slices, s.NQ)
    ctx, _ = gpu_run(F, [sd], [flds])
    rec = ctx.records()
    trace, logw = rec["trace"].cpu().numpy(), rec["logw"].cpu().numpy()
    G = ctx.greens().cpu().numpy()
    for w in range(W):
        ref = path.run_walker(s, flds[w], energy_fn=energy.local_energy)
        check_walker(trace[:, w], logw[:, w], G[w], ref, mixed=True, label="walker %d" % w)


def test_bf16_split_needs_the_mixed_precision():
    F = _F()
    sd = dict(si.WORKLOADS["ueg_n14_m19"]["systems"][0], precision=0, flags=F.FTAFQMC_BF16_SPLIT)
    with pytest.raises(RuntimeError, match="E_ARG"):
        F.ftafqmc_workspace_bytes([sd])


def test_m123_full_size_fp64():
    _full_size("ueg_n38_m123", 0)


def test_uneven_four_systems_one_handle():
    _full_size("ueg_uneven4", 1)


def test_m485_full_size_fp64():
    _full_size("ueg_n114_m485", 0)


def test_m485_full_size_mixed():
    _full_size("ueg_n114_m485", 1)


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_every_gemm_tile_shape_gives_the_same_path(precision, monkeypatch):
    """Each tile shape the autotuner may pick reproduces the default shape's result."""
    F = _F()
    sd = dict(n_elec=38, rs=1.0, theta=0.25, nmax2=5, dtau=0.05, stab_every=5, walkers=3, precision=precision)
    s = oracle_system(sd)
    flds = si.fields(31, 3, s.n_slices, s.NQ)
    ref = None
    probe = F.Context([dict(sd, walkers=1)])
    n_tiles = probe.info()["gemm_tile_shapes"]
    probe.close()
    assert n_tiles >= 9
    fp32_only = {8}                      # the 192 x 192 one-walker tile is built for FP32 MFMA only
    for tile in range(n_tiles):
        monkeypatch.setenv("FTAFQMC_GEMM_TILE", str(tile))
        ctx, _ = gpu_run(F, [sd], [flds])
        inf = ctx.info()
        chosen = (inf["gemm_tile_chain"], inf["gemm_tile_epilogue"], inf["gemm_tile_horner"], inf["gemm_tile_apply"])
        if precision == 0 and tile in fp32_only:
            assert not set(chosen) & fp32_only   # falls back to a timed choice
        else:
            assert chosen == (tile, tile, tile, tile)
        G = ctx.greens().cpu().numpy()
        E = ctx.records()["trace"].cpu().numpy()
        if ref is None:
            ref = (G, E)
        else:
            assert rel_mat(G, ref[0]) < 1e-12, tile
            assert rel_mat(E, ref[1]) < 1e-12, tile
    monkeypatch.delenv("FTAFQMC_GEMM_TILE")
    ctx, _ = gpu_run(F, [sd], [flds])
    assert 0 <= ctx.info()["gemm_tile_chain"] < n_tiles


def test_overlapped_walker_groups_give_identical_results():
    """FTAFQMC_OVERLAP (two walker groups on two streams) changes the schedule only: records,
    weights and G are bit-identical to the single-stream run, for one system and for an uneven
    pair of systems in one handle, and the path record feeds the same derivatives."""
    F = _F()
    sd = dict(n_elec=38, rs=1.0, theta=0.25, nmax2=5, dtau=0.05, stab_every=5, walkers=24)
    sd2 = dict(n_elec=14, rs=0.5, theta=0.0625, nmax2=2, dtau=0.05, stab_every=10, walkers=17)
    s1, s2 = oracle_system(sd), oracle_system(sd2)
    f1 = si.fields(91, sd["walkers"], s1.n_slices, s1.NQ)
    f2 = si.fields(92, sd2["walkers"], s2.n_slices, s2.NQ)
    out = {}
    for flags in (0, F.FTAFQMC_OVERLAP):
        ctx, _ = gpu_run(F, [dict(sd, flags=flags | F.FTAFQMC_CHECKPOINT), dict(sd2, flags=flags)], [f1, f2])
        assert ctx.info(0)["walker_groups"] == (2 if flags else 1)
        res = []
        for i in range(2):
            rec = ctx.records(i)
            res += [rec["trace"].cpu().numpy(), rec["logw"].cpu().numpy(), ctx.greens(i).cpu().numpy()]
        ctx.energy(0)
        res.append(ctx.backward(0)["walker"].cpu().numpy())
        out[flags] = res
        ctx.close()
    for a, b in zip(out[0], out[F.FTAFQMC_OVERLAP]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("overlap", [0, 1, 2], ids=["one_stream", "overlap", "lowrank_mixed_bf16"])
def test_graph_replays_match_eager_paths(overlap):
    """FTAFQMC_GRAPH: the first whole-path call is captured, later calls replay the graph.  Every
    replay, with eager work (energy, G copies, a reset) between replays and with new field values
    written into the same buffer, gives bit-identical records and G to eager propagation; also
    with the low-rank solve and the mixed split-BF16 chain (whose per-slice ranks and kernels are
    part of the captured sequence)."""
    F = _F()
    extra = {0: 0, 1: F.FTAFQMC_OVERLAP, 2: F.FTAFQMC_LOW_RANK | F.FTAFQMC_BF16_SPLIT}[overlap]
    sd = dict(n_elec=38, rs=1.0, theta=0.25, nmax2=5, dtau=0.05, stab_every=4, walkers=24)
    sd2 = dict(n_elec=14, rs=0.5, theta=0.0625, nmax2=2, dtau=0.05, stab_every=10, walkers=9)
    if overlap == 2:                                  # a low-temperature system whose solve truncates
        sd = dict(n_elec=14, rs=1.0, theta=0.0625, nmax2=5, dtau=0.05, stab_every=10, walkers=16, precision=1)
        sd2 = dict(sd2, precision=1)
    s1, s2 = oracle_system(sd), oracle_system(sd2)
    fa = [si.fields(s, sdx["walkers"], so.n_slices, so.NQ) for s, sdx, so in ((61, sd, s1), (62, sd2, s2))]
    fb = [si.fields(s, sdx["walkers"], so.n_slices, so.NQ) for s, sdx, so in ((71, sd, s1), (72, sd2, s2))]

    def snapshot(ctx):
        out = []
        for i in range(2):
            rec = ctx.records(i)
            out += [rec["trace"].cpu().numpy(), rec["logw"].cpu().numpy(), ctx.greens(i).cpu().numpy()]
        return out

    refs = []
    for fl in (fa, fb):
        ctx, _ = gpu_run(F, [dict(sd, flags=extra), dict(sd2, flags=extra)], fl)
        refs.append(snapshot(ctx))
        ctx.close()
    ctx = F.Context([dict(sd, flags=extra | F.FTAFQMC_GRAPH), dict(sd2, flags=extra)])
    bufs = [torch.from_numpy(np.ascontiguousarray(f)).cuda() for f in fa]
    for rep, which in enumerate([0, 0, 1, 0]):
        for b, f in zip(bufs, (fa, fb)[which]):
            b.copy_(torch.from_numpy(np.ascontiguousarray(f)).cuda())
        if rep:
            ctx.energy(0)
            ctx.reset()
        ctx.propagate(bufs)
        torch.cuda.synchronize()
        assert ctx.info(0)["slice"] == s1.n_slices and ctx.info(1)["slice"] == s2.n_slices
        for a, b in zip(snapshot(ctx), refs[which]):
            assert np.array_equal(a, b), (rep, which)
    ctx.close()


def test_concurrent_systems_match_serial_schedule(monkeypatch):
    """The four systems of the uneven batch run on streams of their own, enqueued longest-first;
    the same batch with FTAFQMC_SERIAL_SYSTEMS=1 (one after another) must give bit-identical
    results, and every system reports its share of the call's wall time."""
    F = _F()
    wl = si.WORKLOADS["ueg_uneven4"]
    systems = [dict(sd, walkers=8, precision=1) for sd in wl["systems"]]
    flds = []
    for i, sd in enumerate(systems):
        s = oracle_system(sd)
        flds.append(si.fields(si.system_seed("ueg_uneven4", i), sd["walkers"], s.n_slices, s.NQ))
    conc, _ = gpu_run(F, systems, flds)
    times = conc.system_times()
    assert len(times) == 4 and all(t > 0 for t in times)
    monkeypatch.setenv("FTAFQMC_SERIAL_SYSTEMS", "1")
    ser, _ = gpu_run(F, systems, flds)
    for i in range(4):
        a, b = conc.energy(i), ser.energy(i)
        assert torch.equal(a["local"], b["local"]) and torch.equal(a["logw"], b["logw"]), i
        assert torch.equal(conc.greens(i), ser.greens(i)), i


def test_rq_gather_kernel_matches_the_streamed_one(monkeypatch):
    """r_Q has two kernels: the LDS-streamed one (N_Q <= 4096, every workload here) and the per-Q
    gather for larger N_Q.  FTAFQMC_RQ_GATHER=1 runs the gather form on a ragged M=57 path and on
    M=19: the oracle's bar holds for both, and the two agree to rounding."""
    F = _F()
    for sd, seed in ((dict(n_elec=38, rs=1.0, theta=0.25, nmax2=5, dtau=0.05, stab_every=4, walkers=4), 8),
                     (dict(si.WORKLOADS["ueg_n14_m19"]["systems"][0], walkers=8), 9)):
        s = oracle_system(sd)
        flds = si.fields(seed, sd["walkers"], s.n_slices, s.NQ)
        a, _ = gpu_run(F, [sd], [flds])
        monkeypatch.setenv("FTAFQMC_RQ_GATHER", "1")
        b, _ = gpu_run(F, [sd], [flds])
        monkeypatch.delenv("FTAFQMC_RQ_GATHER")
        ta, tb = a.records()["trace"].cpu().numpy(), b.records()["trace"].cpu().numpy()
        assert rel_mat(tb, ta) < 1e-12
        Gb = b.greens().cpu().numpy()
        lw = b.records()["logw"].cpu().numpy()
        for w in range(sd["walkers"]):
            ref = path.run_walker(s, flds[w], energy_fn=energy.local_energy)
            check_walker(tb[:, w], lw[:, w], Gb[w], ref, label=("gather", w))
        a.close()
        b.close()


def _panel_case_outputs(F, systems, fields, n_slices=None, backward=False):
    ctx, fds = gpu_run(F, systems, fields, n_slices)
    out = []
    for i in range(len(systems)):
        rec = ctx.records(i)
        out += [rec["trace"].cpu().numpy(), rec["logw"].cpu().numpy(), ctx.greens(i).cpu().numpy()]
    if backward:
        ctx.energy(0)
        for mode in (F.FROZEN_PATH, F.PATHWISE):
            r = ctx.backward(0, mode=mode)
            out += [r["walker"].cpu().numpy(), r["jac"].cpu().numpy()]
    torch.cuda.synchronize()
    ctx.close()
    del fds
    return out


def test_column_split_panel_matches_row_panel(monkeypatch):
    """The Gauss-Jordan panel has two kernels with the same arithmetic and the same pivot choice:
    one row per thread (FTAFQMC_GJ_ROW_PANEL=1) and the default column-split layout.  Every panel
    shape the solves use (1 to 8 row slots, 32-column and 64-column steps, the last narrow panel,
    the doubled 2M system of both derivative modes) gives bit-identical records, weights, G and
    derivatives with either kernel."""
    F = _F()
    monkeypatch.setenv("FTAFQMC_GJ_PANEL64", "0")      # both on 32-column panels
    cases = _panel_cases(F)
    for k, (systems, n_slices, bwd) in enumerate(cases):
        fields = _panel_case_fields(k, systems)
        print("panel case", k, [oracle_system(sd).M for sd in systems], flush=True)
        split = _panel_case_outputs(F, systems, fields, n_slices, bwd)
        monkeypatch.setenv("FTAFQMC_GJ_ROW_PANEL", "1")
        row = _panel_case_outputs(F, systems, fields, n_slices, bwd)
        monkeypatch.delenv("FTAFQMC_GJ_ROW_PANEL")
        assert len(split) == len(row)
        for i, (a, b) in enumerate(zip(split, row)):
            assert np.array_equal(a, b, equal_nan=True), (k, i, np.nanmax(np.abs(a - b)))


def _panel_case_fields(k, systems):
    fields = []
    for j, sd in enumerate(systems):
        s = oracle_system(sd)
        fields.append(si.fields(700 + 10 * k + j, sd["walkers"], s.n_slices, s.NQ))
    return fields


def _panel_cases(F):
    cases = []
    # M = 19, 123, 171 in one handle (1, 2 and 3 row slots and their shrinking panels)
    sds = [dict(n_elec=14, rs=1.0, theta=0.5, nmax2=2, dtau=0.05, stab_every=5, walkers=5),
           dict(n_elec=38, rs=2.0, theta=0.25, nmax2=9, dtau=0.05, stab_every=10, walkers=4),
           dict(n_elec=66, rs=1.0, theta=0.125, nmax2=11, dtau=0.025, stab_every=10, walkers=3)]
    cases.append((sds, None, False))
    # M = 257 (6 slots, 64-column steps) and M = 485 (8 slots), the first slices
    cases.append(([dict(n_elec=66, rs=1.0, theta=0.5, nmax2=16, dtau=0.1, stab_every=4, walkers=2, precision=1)], 12, False))
    cases.append(([dict(n_elec=114, rs=0.5, theta=0.0625, nmax2=24, dtau=0.02, stab_every=8, walkers=2)], 6, False))
    # M = 123 with both derivative modes (the doubled system has 246 rows: 4 slots)
    cases.append(([dict(n_elec=38, rs=2.0, theta=0.25, nmax2=9, dtau=0.05, stab_every=10, walkers=3,
                        flags=F.FTAFQMC_CHECKPOINT)], None, True))
    # M = 57: one 64-column step narrower than the panel (57 columns)
    cases.append(([dict(n_elec=38, rs=1.0, theta=0.25, nmax2=5, dtau=0.05, stab_every=4, walkers=4)], None, False))
    return cases


def test_64_column_steps_match_32_column_steps(monkeypatch):
    """The solve takes 64-column Gauss-Jordan steps (one 64-column panel, one K = 64 update) where
    at most 256 rows are left, 32-column steps elsewhere (FTAFQMC_GJ_PANEL64=0: everywhere).  The
    two orders of the same elimination agree to rounding on every shape: M = 19/123/171 in one
    handle, M = 257 and 485 (64-column steps after two-half steps), the doubled 2M = 246 system
    of both derivative modes, and M = 57 (a single step narrower than the panel)."""
    F = _F()
    for k, (systems, n_slices, bwd) in enumerate(_panel_cases(F)):
        fields = _panel_case_fields(k, systems)
        print("64-column case", k, [oracle_system(sd).M for sd in systems], flush=True)
        wide = _panel_case_outputs(F, systems, fields, n_slices, bwd)
        monkeypatch.setenv("FTAFQMC_GJ_PANEL64", "0")
        narrow = _panel_case_outputs(F, systems, fields, n_slices, bwd)
        monkeypatch.delenv("FTAFQMC_GJ_PANEL64")
        assert len(wide) == len(narrow)
        # FP64 paths to rounding; a mixed path carries the FP64 rounding into its FP32 chain
        tol = 1e-5 if any(sd.get("precision", 0) == 1 for sd in systems) else 1e-10
        for i, (a, b) in enumerate(zip(wide, narrow)):
            fin = np.isfinite(b)
            assert np.array_equal(np.isfinite(a), fin), (k, i)
            scale = max(np.abs(b[fin]).max(), 1.0) if fin.any() else 1.0
            err = np.abs(a[fin] - b[fin]).max() / scale if fin.any() else 0.0
            assert err < tol, (k, i, err)
