"""Write stored oracle outputs for sampled walkers of the large workloads.

Calls only oracle/ and the seeded input generator.  For each workload and each
sampled walker it runs the FP64 oracle over the whole path and keeps, at every
energy record (each stabilisation boundary and the last slice): E_1, E_2, E, N,
ln w and the status; plus the final Green's function's diagonal, first rows and 256 entries at
seeded positions (for element-by-element checks).
For the derivative workload it also keeps each sampled walker's frozen-path
derivatives (d ln w, dE, dN in mu and in lambda) from oracle.tangent, and (mode pathwise)
their pathwise derivatives with the raw fields held fixed.  Mode lowrank keeps the same
per-record values for the low-rank truncated path (oracle.lowrank) of the sampled walkers of
the large low-temperature workload, truncating the left block (the variant whose result does
not depend on how the right block is factorised), with the ranks of every slice.
Usage: python tests/golden/make_oracle_golden.py [workload ...]
       python tests/golden/make_oracle_golden.py tangent
       python tests/golden/make_oracle_golden.py pathwise
       python tests/golden/make_oracle_golden.py lowrank
"""
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ueg, path, energy, tangent, lowrank  # noqa: E402
import synthinputs as si  # noqa: E402

SAMPLES = {
    "ueg_n66_m171": {0: [0, 85, 170, 255]},
    "ueg_n38_m123": {0: [0, 42, 85, 127]},
    "ueg_uneven4": {0: [0, 170], 1: [0, 170], 2: [0, 84], 3: [0, 84]},
    "ueg_n114_m485": {0: [0, 170, 341, 511]},
}
G_ROWS = 8
G_SAMPLES = 256


def g_sample_positions(M, sidx, w):
    """Seeded entry positions (i, j) of a walker's final G, the same for the oracle and the tests."""
    rng = np.random.default_rng(1000003 * (sidx + 1) + w)
    return rng.integers(0, M, G_SAMPLES), rng.integers(0, M, G_SAMPLES)
LOWRANK_SAMPLES = {"ueg_n114_m485": {0: [0, 511]}}
TANGENT_SAMPLES = {"ueg_n38_m123": [0, 63, 127]}


def one(args):
    name, sidx, w = args[:3]
    low_rank = len(args) > 3 and args[3]
    from threadpoolctl import threadpool_limits
    wl = si.WORKLOADS[name]
    sd = wl["systems"][sidx]
    s = ueg.UEGSystem(sd["n_elec"], sd["rs"], sd["theta"], sd["nmax2"], sd["dtau"], stab_every=sd["stab_every"])
    z = si.walker_fields(si.system_seed(name, sidx), w, s.n_slices, s.NQ)
    with threadpool_limits(2):
        if low_rank:
            out = lowrank.run_walker_lowrank(s, z, energy_fn=energy.local_energy, right_threshold=0.0)
        else:
            out = path.run_walker(s, z, energy_fn=energy.local_energy)
    recs = out["records"]
    extra = dict(ranks=out["ranks"]) if low_rank else {}
    gi, gj = g_sample_positions(s.M, sidx, w)
    if not low_rank:
        extra.update(G_samp_i=gi, G_samp_j=gj, G_samp=out["G"][gi, gj].copy())
    return dict(**extra,
        system=sidx, walker=w,
        slices=np.array([r["slice"] for r in recs]),
        E=np.array([[r["E1"], r["E2"], r["E"], r["N"]] for r in recs]),
        logw=np.array([r["logw"] for r in recs]),
        status=np.array([r["status"] for r in recs]),
        G_diag=np.diagonal(out["G"]).copy(),
        G_rows=out["G"][:G_ROWS].copy(),
    )


def one_tangent(args):
    name, w, mode = args
    from threadpoolctl import threadpool_limits
    sd = si.WORKLOADS[name]["systems"][0]
    s = ueg.UEGSystem(sd["n_elec"], sd["rs"], sd["theta"], sd["nmax2"], sd["dtau"], stab_every=sd["stab_every"])
    z = si.walker_fields(si.system_seed(name, 0), w, s.n_slices, s.NQ)
    with threadpool_limits(1):
        if mode == "pathwise":
            tans = {}
            for p in ("mu", "kscale"):
                fwd, tans[p] = tangent.pathwise_tangent(s, z, p)
        else:
            fwd, tans = tangent.walker_tangents(s, z)
    out = dict(logw=fwd["logw"], status=fwd["status"], E=fwd["E"]["E"], N=fwd["E"]["N"])
    for p, t in tans.items():
        for k in ("dlogw", "dE", "dN", "dE1", "dE2"):
            out["%s_%s" % (p, k)] = t[k]
        out[p + "_dG_rows"] = t["dG"][:G_ROWS].copy()
    return out


def main_tangent(mode="tangent"):
    jobs = [(n, w, mode) for n, ws in TANGENT_SAMPLES.items() for w in ws]
    with ProcessPoolExecutor(max_workers=min(4, len(jobs))) as ex:
        results = list(ex.map(one_tangent, jobs))
    for n in TANGENT_SAMPLES:
        arrays = {}
        for (jn, w, _), r in zip(jobs, results):
            if jn == n:
                for k, v in r.items():
                    arrays["w%d_%s" % (w, k)] = np.asarray(v)
        fn = os.path.join(HERE, "oracle_%s_%s.npz" % (mode, n))
        np.savez_compressed(fn, **arrays)
        print("wrote", fn, os.path.getsize(fn), "bytes")


def main(names, low_rank=False):
    samples = LOWRANK_SAMPLES if low_rank else SAMPLES
    jobs = [(n, sidx, w, low_rank) for n in names for sidx, ws in samples[n].items() for w in ws]
    with ProcessPoolExecutor(max_workers=min(4, len(jobs))) as ex:
        results = list(ex.map(one, jobs))
    for n in names:
        arrays = {}
        for (jn, sidx, w, _), r in zip(jobs, results):
            if jn != n:
                continue
            key = "s%d_w%d" % (sidx, w)
            for k, v in r.items():
                if k not in ("system", "walker"):
                    arrays[key + "_" + k] = v
        fn = os.path.join(HERE, ("oracle_lowrank_%s.npz" if low_rank else "oracle_%s.npz") % n)
        np.savez_compressed(fn, **arrays)
        print("wrote", fn, os.path.getsize(fn), "bytes")


if __name__ == "__main__":
    if sys.argv[1:] in (["tangent"], ["pathwise"]):
        main_tangent(sys.argv[1])
    elif sys.argv[1:] == ["lowrank"]:
        main(list(LOWRANK_SAMPLES), low_rank=True)
    else:
        main(sys.argv[1:] or list(SAMPLES))
