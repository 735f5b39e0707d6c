"""Low-rank truncation on the GPU (FTAFQMC_LOW_RANK, through the C ABI) against the oracle's
truncated path (oracle.lowrank, Sec. "Exploiting the low-rank structure", eq. thresh) with the
threshold on the left block, on the same seeded fields, to the forward path's bars (FP64 1e-10;
mixed as in test_gpu_parity), with one change: E_1 and E_2 are compared to bar x (|E_1| + |E_2|),
the condition scale of their sum (as the mixed bar does for the sum), because at
Theta = 0.035 with N = 2 the kinetic energy is ~1e-12: a sum of occupations P_KK = 1 - G_KK of
that size, each of which carries the rounding of G_KK (~1e-16) on both sides.  The mixed path is
checked at Theta = 0.035 and at full size; at M = 57, Theta = 0.0625 its error against FP64 is
~1e-5 with or without the truncation (a property of the mixed path on that colder, longer path).

The left rank m_L is the same integer on both sides at every Green's function formation.  The
right rank is a diagnostic of two different factorisations of the same product (the oracle's QRCP
at every slice, the GPU's pre-pivoted Cholesky-QR every stab_every slices): it is compared at the
stabilisation slices, skipping those where the oracle's |D| spectrum has a value within a factor
2 of the threshold.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from threadpoolctl import threadpool_limits  # noqa: E402

from oracle import path, energy, lowrank  # noqa: E402
import synthinputs as si  # noqa: E402
from tests.test_gpu_parity import (_F, oracle_system, gpu_run, _check_golden, relc, rel_mat,  # noqa: E402
                                   mix_logw_tol, FP64_REL, MIX_E12, MIX_N, MIX_G, GOLDEN)

pytestmark = pytest.mark.gpu

COND30 = dict(n_elec=2, rs=0.5, theta=0.035, nmax2=1, dtau=0.05, stab_every=1, walkers=8)
M57_LOWT = dict(n_elec=14, rs=1.0, theta=0.0625, nmax2=5, dtau=0.05, stab_every=10, walkers=4)


def _oracle_runs(s, flds):
    out = []
    with threadpool_limits(1):
        for z in flds:
            out.append(lowrank.run_walker_lowrank(s, z, energy_fn=energy.local_energy, right_threshold=0.0))
    return out


def check_lowrank_walker(rec_gpu, logw_gpu, G_gpu, ref, mixed, label):
    bar = MIX_E12 if mixed else FP64_REL
    recs = ref["records"]
    assert len(recs) == rec_gpu.shape[0], label
    for j, r in enumerate(recs):
        e1, e2, e, nn = rec_gpu[j]
        scale = abs(r["E1"]) + abs(r["E2"])
        assert abs(e1 - r["E1"]) < bar * scale, (label, j, e1, r["E1"])
        assert abs(e2 - r["E2"]) < bar * scale, (label, j, e2, r["E2"])
        assert abs((e1 + e2) - (r["E1"] + r["E2"])) < bar * scale, (label, j)
        assert relc(nn, r["N"]) < (MIX_N if mixed else FP64_REL), (label, j, nn, r["N"])
        if np.isfinite(r["logw"]):
            tol = mix_logw_tol(G_gpu.shape[0], r["slice"]) if mixed else FP64_REL * max(1.0, abs(r["logw"]))
            assert abs(logw_gpu[j] - r["logw"]) < tol, (label, j, logw_gpu[j], r["logw"])
        else:
            assert logw_gpu[j] == -np.inf, (label, j)
    assert rel_mat(G_gpu, ref["G"]) < (MIX_G if mixed else FP64_REL), label


def _check_ranks(F, ctx, s, refs, stab_every, label):
    mL, mR = ctx.lowrank_ranks()
    mR = mR.cpu().numpy()
    n = s.n_slices
    for k in range(n + 1):
        assert mL[k] == refs[0]["ranks"][k][0], (label, k, mL[k], refs[0]["ranks"][k][0])
    compared = 0
    for w, ref in enumerate(refs):
        for k in range(0, n + 1, stab_every):
            if k == 0:
                assert mR[w, 0] == s.M
                continue
            if np.any(np.abs(np.log(ref["right_D"][k] / lowrank.THRESHOLD)) < np.log(2.0)):
                continue                                # a value near the threshold: either count is right
            want = int((ref["right_D"][k] >= lowrank.THRESHOLD).sum())
            assert mR[w, k] == want, (label, w, k, mR[w, k], want)
            compared += 1
    return compared


@pytest.mark.parametrize("cfg,precision", [("cond30", 0), ("cond30", 1), ("m57_lowT", 0)],
                         ids=["cond30-fp64", "cond30-mixed", "m57_lowT-fp64"])
def test_lowrank_matches_the_truncated_oracle(cfg, precision):
    F = _F()
    base = COND30 if cfg == "cond30" else M57_LOWT
    sd = dict(base, precision=precision, flags=F.FTAFQMC_LOW_RANK)
    s = oracle_system(sd)
    flds = si.fields(5 if cfg == "cond30" else 9, sd["walkers"], s.n_slices, s.NQ)
    ctx, _ = gpu_run(F, [sd], [flds])
    rec = ctx.records()
    trace, logw = rec["trace"].cpu().numpy(), rec["logw"].cpu().numpy()
    G = ctx.greens().cpu().numpy()
    refs = _oracle_runs(s, flds)
    truncated = 0
    for w, ref in enumerate(refs):
        check_lowrank_walker(trace[:, w], logw[:, w], G[w], ref, precision == 1, (cfg, w))
        truncated += int(ref["ranks"][:, 0].min() < s.M)
    assert truncated == len(refs)                       # the truncation is active on every walker
    if precision == 0:
        assert _check_ranks(F, ctx, s, refs, sd["stab_every"], cfg) > 0
    ctx.close()


def test_lowrank_without_active_truncation_is_the_full_rank_path():
    """M = 19 at Theta = 0.5 keeps every plane wave and every column: the flag reorders only the
    right-hand sides of the solve, so the path is bit-identical to the one without it."""
    F = _F()
    sd = dict(si.WORKLOADS["ueg_n14_m19"]["systems"][0], walkers=16)
    s = oracle_system(sd)
    flds = si.fields(21, 16, s.n_slices, s.NQ)
    a, _ = gpu_run(F, [sd], [flds])
    b, _ = gpu_run(F, [dict(sd, flags=F.FTAFQMC_LOW_RANK)], [flds])
    mL, mR = b.lowrank_ranks()
    assert min(mL) == s.M and int(mR.min()) == s.M
    assert np.array_equal(a.records()["trace"].cpu().numpy(), b.records()["trace"].cpu().numpy())
    assert np.array_equal(a.greens().cpu().numpy(), b.greens().cpu().numpy())
    a.close()
    b.close()


def test_lowrank_walker_groups_give_identical_results():
    """FTAFQMC_OVERLAP splits the walkers over two streams; the rank record follows the walkers."""
    F = _F()
    sd = dict(M57_LOWT, walkers=16, flags=F.FTAFQMC_LOW_RANK)
    s = oracle_system(sd)
    flds = si.fields(11, 16, s.n_slices, s.NQ)
    a, _ = gpu_run(F, [sd], [flds])
    b, _ = gpu_run(F, [dict(sd, flags=F.FTAFQMC_LOW_RANK | F.FTAFQMC_OVERLAP)], [flds])
    assert b.info()["walker_groups"] == 2
    assert np.array_equal(a.records()["trace"].cpu().numpy(), b.records()["trace"].cpu().numpy())
    assert np.array_equal(a.lowrank_ranks()[1].cpu().numpy(), b.lowrank_ranks()[1].cpu().numpy())
    a.close()
    b.close()


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_lowrank_m485_full_size_sampled(precision):
    """The low-temperature M = 485 workload at full size (512 walkers, the bench's launch
    configuration) with the truncation: sampled walkers against the stored truncated oracle,
    and m_L at every slice."""
    F = _F()
    name = "ueg_n114_m485"
    fn = os.path.join(GOLDEN, "oracle_lowrank_%s.npz" % name)
    if not os.path.exists(fn):
        pytest.skip("stored oracle outputs missing: run tests/golden/make_oracle_golden.py lowrank")
    gold = np.load(fn)
    sd = dict(si.WORKLOADS[name]["systems"][0], precision=precision, flags=F.FTAFQMC_LOW_RANK)
    s = oracle_system(sd)
    flds = si.fields(si.system_seed(name, 0), sd["walkers"], s.n_slices, s.NQ)
    ctx, _ = gpu_run(F, [sd], [flds])
    rec = ctx.records()
    trace, logw = rec["trace"].cpu().numpy(), rec["logw"].cpu().numpy()
    G = ctx.greens().cpu().numpy()
    mL, _ = ctx.lowrank_ranks()
    keys = sorted({k[:-len("_slices")] for k in gold.files if k.endswith("_slices")})
    assert keys
    for key in keys:
        w = int(key.split("_w")[1])
        _check_golden(gold, key, trace[:, w], logw[:, w], G[w], rec["slices"], mixed=precision == 1)
        assert list(mL) == [int(r[0]) for r in gold[key + "_ranks"]]
    assert min(mL) < s.M
    ctx.close()
