#!/usr/bin/env python
"""Throughput of the ph-FT-AFQMC slice path on one MI355X: walker*slices per second.

One step = one whole imaginary-time path (tau = 0 .. beta, all n slices) for every
walker of the workload: per slice the force bias, the shifted propagator, the
stabilised Green's function, ln det and the phaseless weight; QR stabilisation and
the local energy at every stabilisation boundary and at slice n; then the weighted
energy means.  Inputs (fields) are resident in HBM before the timed region.  Both
precisions run on the same seeded fields; the mixed path's energy error is measured
against the FP64 path on every walker, and `value` is the mixed throughput when that
error is within 1e-6, else the FP64 throughput, under the faster of the two schedules
(one stream per system, or FTAFQMC_OVERLAP's two walker groups, whose results are
bit-identical; config.schedule names it).  The FP64 oracle is timed on the
host cores on a bounded sample of the same workload (`cpu_baseline`).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synthinputs as si  # noqa: E402

PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}


def measured_traffic(workload, precision):
    """HBM bytes per propagator-GEMM launch from the committed rocprofv3 counter summary,
    or None when no summary exists or the GEMM source changed since it was taken."""
    import hashlib
    fn = os.path.join(ROOT, "profiles", "%s_%s_gemm_traffic.txt" % (workload, precision))
    if not os.path.exists(fn):
        return None
    kv = dict(line.strip().split("=", 1) for line in open(fn) if "=" in line and not line.startswith("#"))
    src = os.path.join(ROOT, "paper_2012_12228_amd", "csrc", "gemm.hip")
    if hashlib.sha1(open(src, "rb").read()).hexdigest() != kv.get("gemm_sha1"):
        return None
    return float(kv["hbm_bytes_per_launch"])
MIXED_E_TOL = 1e-6


def _oracle_worker(args):
    name, sidx, walker, n_run = args
    from threadpoolctl import threadpool_limits
    from oracle import ueg, path, energy
    sd = si.WORKLOADS[name]["systems"][sidx]
    s = ueg.UEGSystem(sd["n_elec"], sd["rs"], sd["theta"], sd["nmax2"], sd["dtau"], stab_every=sd["stab_every"])
    z = si.walker_fields(si.system_seed(name, sidx), walker, s.n_slices, s.NQ)
    with threadpool_limits(1):
        t = time.time()
        path.run_walker(s, z, energy_fn=energy.local_energy, stop_after=n_run)
        return time.time() - t, min(n_run, s.n_slices)


def cpu_baseline(name, seconds_target=12.0):
    """Oracle throughput on the host: one walker per process, one BLAS thread each."""
    from concurrent.futures import ProcessPoolExecutor
    from oracle import ueg
    sd = si.WORKLOADS[name]["systems"][0]
    s = ueg.UEGSystem(sd["n_elec"], sd["rs"], sd["theta"], sd["nmax2"], sd["dtau"], stab_every=sd["stab_every"])
    # one process per walker over the host share of one GPU: at most 16 processes, which is the
    # CPU share a one-GPU machine gives a job whatever os.cpu_count() reports
    nproc = max(1, min(os.cpu_count() or 1, 16, sd["walkers"]))
    # calibrate the slice count so that each process works for about seconds_target
    dt1, n1 = _oracle_worker((name, 0, 0, 2))
    n_run = int(max(2, min(s.n_slices, seconds_target / max(dt1 / n1, 1e-6))))
    t = time.time()
    with ProcessPoolExecutor(max_workers=nproc) as ex:
        res = list(ex.map(_oracle_worker, [(name, 0, w, n_run) for w in range(nproc)]))
    wall = time.time() - t
    ws = sum(r[1] for r in res)
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": ws / wall, "unit": "walker*slices/s", "cores": nproc, "kind": "oracle",
            "os_cpu_count": os.cpu_count(), "cpu_model": model,
            "sample": "%d walkers x first %d of %d slices of %s (one process and one BLAS thread per walker)"
                      % (nproc, n_run, s.n_slices, name)}


def _path(ctx, fields, n_sys):
    ctx.reset()
    ctx.propagate(fields)
    for i in range(n_sys):
        ctx.energy(i)


def run_precision(F, torch, systems, fields, steps, warmup):
    """Time `steps` whole paths with no instrumentation (the throughput), then the same number
    of paths with HIP events around the propagator GEMMs only (the roofline's per-launch time),
    then one path with events around every launch (the per-class breakdown)."""
    ctx = F.Context(systems)
    n_sys = len(systems)
    infos = [ctx.info(i) for i in range(n_sys)]
    for _ in range(warmup):
        _path(ctx, fields, n_sys)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _path(ctx, fields, n_sys)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ws = sum(inf["n_walkers"] * inf["n_slices"] for inf in infos)
    out = {"seconds": t1 - t0, "walker_slices_per_s": ws * steps / (t1 - t0),
           "ms_per_step": 1e3 * (t1 - t0) / steps}
    if n_sys > 1:
        # each system's share of the last timed path (events on its own streams)
        sys_ms = ctx.system_times()
        out["system_ms"] = sys_ms
        out["system_ms_sum_over_wall"] = sum(sys_ms) / out["ms_per_step"]
    # the roofline's kernel: events on the library's stream around every propagator GEMM launch
    ctx.profile(True, classes=["gemm"])
    t2 = time.perf_counter()
    for _ in range(steps):
        _path(ctx, fields, n_sys)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    prof = ctx.profile(False)
    out["ms_per_step_gemm_events"] = 1e3 * (t3 - t2) / steps
    ctx.profile(True)
    _path(ctx, fields, n_sys)
    classes = ctx.profile(False)
    out["profile_ms_per_step"] = {k: v[0] for k, v in classes.items()}
    out["launches_per_step"] = {k: v[1] for k, v in classes.items()}
    gemm_ms, gemm_n = prof["gemm"]
    # Propagator products per slice for Taylor degree 4 nb: V^2, V^3, V^4 (with the Taylor
    # blocks), nb - 1 Horner steps and the apply.  Each walker group of a system launches them
    # for its own walkers: one complex M x M x M product per walker and launch (8 M^3
    # algorithmic flops per walker), so the total does not depend on the grouping.
    prods = [inf["taylor_degree"] // 4 + 3 for inf in infos]
    want_n = sum(pr * inf["n_slices"] * inf["walker_groups"] for pr, inf in zip(prods, infos)) * steps
    assert gemm_n == want_n, (gemm_n, want_n)
    flops = steps * sum(pr * inf["n_slices"] * 8.0 * inf["M"] ** 3 * inf["n_walkers"] for pr, inf in zip(prods, infos))
    out["taylor_degree"] = [inf["taylor_degree"] for inf in infos]
    out["sizes"] = [{"M": inf["M"], "n": inf["n_slices"], "W": inf["n_walkers"]} for inf in infos]
    out["gemm_products_per_slice"] = prods
    out["gemm_avg_ms"] = gemm_ms / max(gemm_n, 1)
    out["gemm_flops_per_launch"] = flops / max(gemm_n, 1)
    out["gemm_tflops"] = flops / (gemm_ms * 1e-3) / 1e12
    out["walker_groups"] = [inf["walker_groups"] for inf in infos]
    energies = []
    for i in range(n_sys):
        e = ctx.energy(i)
        energies.append(dict(local=e["local"].cpu().numpy(), logw=e["logw"].cpu().numpy(),
                             status=e["status"].cpu().numpy(), mean=e["mean"].cpu().numpy()))
    out["gemm_tiles"] = [(inf["gemm_tile_chain"], inf["gemm_tile_epilogue"], inf["gemm_tile_horner"],
                          inf["gemm_tile_apply"]) for inf in infos]
    return ctx, out, energies


def end_to_end(wl, r, precision):
    """End-to-end roofline of the one-stream path: the method's algorithmic FP64-equivalent flops
    per walker-slice, F = 8 M^3 g + 14.7 M^3 + 13.3 M^3 / s + 2.6 M^3 / s (g propagator products:
    the Paterson-Stockmeyer chain and the apply; one LU-class solve with its right-hand sides per
    slice; QR, Q formation and T update, and the exchange sums, every s slices), times W n, over
    the path time and the time-weighted peak (the propagator GEMMs' time at the peak of their MFMA
    type, the rest at the FP64 peak)."""
    flops = 0.0
    for sd, deg, sz in zip(wl["systems"], r["taylor_degree"], r["sizes"]):
        M = sz["M"]
        g = deg // 4 + 3
        F = 8 * M ** 3 * g + 14.7 * M ** 3 + (13.3 + 2.6) * M ** 3 / sd["stab_every"]
        flops += F * sz["W"] * sz["n"]
    t = r["ms_per_step"] * 1e-3
    t_gemm = r["profile_ms_per_step"]["gemm"] * 1e-3
    peak_gemm = PEAK_TFLOPS["f32" if precision == "mixed" else "f64"]
    peak = (min(t_gemm, t) * peak_gemm + max(t - t_gemm, 0.0) * PEAK_TFLOPS["f64"]) / t
    achieved = flops / t / 1e12
    return {"flops_per_step": flops, "achieved_tflops": achieved, "time_weighted_peak_tflops": peak,
            "frac": achieved / peak}


def mixed_vs_fp64(en64, enmx):
    """Errors of the mixed path against the FP64 path on the same fields, per system and over
    all: status mismatches; per walker alive in both, |(E1+E2)_mx - (E1+E2)_64| / |(E1+E2)_64|,
    the same over |E1| + |E2|, N and ln w; and the weighted means <E1+E2> and <N> of
    ftafqmc_energy (over each path's own live walkers and weights)."""
    per = []
    for a, b in zip(en64, enmx):
        ok = (a["status"] == 0) & (b["status"] == 0)
        la, lb = a["local"][ok], b["local"][ok]
        e12a, e12b = la[:, 0] + la[:, 1], lb[:, 0] + lb[:, 1]
        ma, mb = a["mean"], b["mean"]
        per.append({
            "status_counts_fp64": [int(np.sum(a["status"] == v)) for v in (0, 1, 2)],
            "status_counts_mixed": [int(np.sum(b["status"] == v)) for v in (0, 1, 2)],
            "status_mismatches": int(np.sum(a["status"] != b["status"])),
            "walkers_compared": int(ok.sum()),
            "max_rel_err_E1E2": float(np.max(np.abs(e12b - e12a) / np.abs(e12a))),
            "max_err_E1E2_over_abs_sum": float(np.max(np.abs(e12b - e12a) / (np.abs(la[:, 0]) + np.abs(la[:, 1])))),
            "max_rel_err_N": float(np.max(np.abs(lb[:, 3] - la[:, 3]) / np.abs(la[:, 3]))),
            "max_abs_err_logw": float(np.max(np.abs(b["logw"][ok] - a["logw"][ok]))),
            "rel_err_mean_E1E2": float(abs((mb[0] + mb[1]) - (ma[0] + ma[1])) / abs(ma[0] + ma[1])),
            "rel_err_mean_N": float(abs(mb[3] - ma[3]) / abs(ma[3])),
        })
    tot = {k: (sum(p[k] for p in per) if k in ("status_mismatches", "walkers_compared") else max(p[k] for p in per))
           for k in per[0] if not k.startswith("status_counts")}
    tot["per_system"] = per
    # the gate of the headline: every status equal, every walker's and the weighted mean's
    # E1 + E2 within MIXED_E_TOL of the FP64 path
    tot["within_tolerance"] = bool(tot["status_mismatches"] == 0 and tot["max_rel_err_E1E2"] <= MIXED_E_TOL
                                   and tot["rel_err_mean_E1E2"] <= MIXED_E_TOL)
    return tot


def load_fields(F, torch, workload):
    wl = si.WORKLOADS[workload]
    fields = []
    for i, sd in enumerate(wl["systems"]):
        probe = F.Context([dict(sd, walkers=1)])     # field shapes (n, N_Q) from the library's tables
        inf = probe.info()
        probe.close()
        f = si.fields(si.system_seed(workload, i), sd["walkers"], inf["n_slices"], inf["n_q"])
        fields.append(torch.from_numpy(f).cuda())
        del f
    torch.cuda.synchronize()
    return fields


def bench_workload(F, torch, workload, precs, steps, warmup, overlap=False):
    """Both precisions of one workload on the same fields: throughput, GEMM roofline and the
    mixed path's errors against the FP64 path."""
    wl = si.WORKLOADS[workload]
    fields = load_fields(F, torch, workload)
    results, energies = {}, {}
    for p in precs:
        systems = [dict(sd, precision=0 if p == "fp64" else 1, flags=F.FTAFQMC_OVERLAP if overlap else 0)
                   for sd in wl["systems"]]
        ctx, out, en = run_precision(F, torch, systems, fields, steps, warmup)
        print("bench: %s %s %.1f walker*slices/s" % (workload, p, out["walker_slices_per_s"]), file=sys.stderr, flush=True)
        pk = "f32" if p == "mixed" else "f64"
        out["gemm_roofline_frac"] = out["gemm_tflops"] / PEAK_TFLOPS[pk]
        results[p], energies[p] = out, en
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
    if "fp64" in energies and "mixed" in energies:
        results["mixed_vs_fp64"] = mixed_vs_fp64(energies["fp64"], energies["mixed"])
    if len(wl["systems"]) > 1 and "mixed" in results:
        # the same batch with the systems one after another on the caller's stream
        os.environ["FTAFQMC_SERIAL_SYSTEMS"] = "1"
        systems = [dict(sd, precision=1) for sd in wl["systems"]]
        ctx, ser, _ = run_precision(F, torch, systems, fields, steps, warmup)
        ctx.close()
        del os.environ["FTAFQMC_SERIAL_SYSTEMS"]
        results["mixed"]["serial_systems_walker_slices_per_s"] = ser["walker_slices_per_s"]
        results["mixed"]["serial_systems_ms"] = ser["system_ms"]
    results["energies"] = energies
    return results, fields


def time_lowrank(F, torch, workload, fields, full, precision="mixed"):
    """The low-rank truncation (FTAFQMC_LOW_RANK) on one workload beside the full-rank run `full`
    (bench_workload's record of the same precision and fields): throughput, per-class times, the
    mean compressions c_L, c_R, c_T over slices and walkers, and the truncation's effect on the
    weighted means."""
    wl = si.WORKLOADS[workload]
    systems = [dict(sd, precision=0 if precision == "fp64" else 1, flags=F.FTAFQMC_LOW_RANK) for sd in wl["systems"]]
    ctx, out, en = run_precision(F, torch, systems, fields, 1, 1)
    M = ctx.info()["M"]
    mL, mR = ctx.lowrank_ranks()
    mL = np.asarray(mL, dtype=float)
    mR = mR.cpu().numpy().astype(float)
    mT = np.minimum(mL[None, :], mR)
    ctx.close()
    torch.cuda.empty_cache()
    ma, mb = full["energies"][precision][0]["mean"], en[0]["mean"]
    base = full[precision]["profile_ms_per_step"]
    return {"workload": workload, "precision": precision,
            "walker_slices_per_s": out["walker_slices_per_s"], "ms_per_step": out["ms_per_step"],
            "full_rank_walker_slices_per_s": full[precision]["walker_slices_per_s"],
            "profile_ms_per_step": out["profile_ms_per_step"],
            "elim_ms_saved": base["elim"] - out["profile_ms_per_step"]["elim"],
            "greens_ms_saved": base["greens_transpose"] - out["profile_ms_per_step"]["greens_transpose"],
            "compression_pct_mean": {"c_L": float(100 * (1 - mL.mean() / M)), "c_R": float(100 * (1 - mR.mean() / M)),
                                     "c_T": float(100 * (1 - mT.mean() / M))},
            "m_L_min": int(mL.min()),
            "rel_diff_mean_E1E2_vs_full_rank": float(abs((mb[0] + mb[1]) - (ma[0] + ma[1])) / abs(ma[0] + ma[1])),
            "rel_diff_mean_N_vs_full_rank": float(abs(mb[3] - ma[3]) / abs(ma[3]))}


def time_graph(F, torch, systems, fields, steps):
    """Whole paths replayed from a captured HIP graph (FTAFQMC_GRAPH), timed without the
    per-launch profiling events (which keep propagation eager)."""
    ctx = F.Context([dict(sd, flags=sd.get("flags", 0) | F.FTAFQMC_GRAPH) for sd in systems])
    infos = [ctx.info(i) for i in range(len(systems))]
    for _ in range(2):                                # capture, then one replay
        ctx.reset()
        ctx.propagate(fields)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.reset()
        ctx.propagate(fields)
        for i in range(len(systems)):
            ctx.energy(i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.close()
    ws = sum(inf["n_walkers"] * inf["n_slices"] for inf in infos)
    return {"walker_slices_per_s": ws * steps / (t1 - t0), "ms_per_step": 1e3 * (t1 - t0) / steps}


def time_overlap(F, torch, systems, fields, steps):
    """Whole paths with FTAFQMC_OVERLAP (each system's walkers in two groups on two streams, one
    group's eliminations beside the other's GEMMs), eager, without profiling events.  Reported
    beside the one-stream value: its per-launch GEMM durations include the other group's
    kernels, so the roofline stays on the one-stream schedule."""
    ctx = F.Context([dict(sd, flags=sd.get("flags", 0) | F.FTAFQMC_OVERLAP) for sd in systems])
    infos = [ctx.info(i) for i in range(len(systems))]
    ctx.reset()
    ctx.propagate(fields)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.reset()
        ctx.propagate(fields)
        for i in range(len(systems)):
            ctx.energy(i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.close()
    ws = sum(inf["n_walkers"] * inf["n_slices"] for inf in infos)
    return {"walker_slices_per_s": ws * steps / (t1 - t0), "ms_per_step": 1e3 * (t1 - t0) / steps,
            "walker_groups": [inf["walker_groups"] for inf in infos]}


def time_backward(F, torch, workload="ueg_n38_m123"):
    """Wall time of one frozen-path and one pathwise derivative pass (ftafqmc_backward) on the
    derivative workload, beside the FP64 forward path they differentiate (inputs in HBM)."""
    wl = si.WORKLOADS[workload]
    sd = dict(wl["systems"][0], precision=0, flags=F.FTAFQMC_CHECKPOINT)
    ctx = F.Context(sd)
    inf = ctx.info()
    f = torch.from_numpy(si.fields(si.system_seed(workload, 0), sd["walkers"], inf["n_slices"], inf["n_q"])).cuda()
    ctx.propagate(f)
    ctx.energy()
    ctx.backward()                                   # warm-up of both passes
    torch.cuda.synchronize()
    ctx.reset()
    t0 = time.perf_counter()
    ctx.propagate(f)
    ctx.energy()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    b = ctx.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ctx.profile(True)                                # per-class breakdown from one more, untimed pass
    ctx.backward()
    prof = ctx.profile(False)
    jac = b["jac"].cpu().numpy()
    ctx.backward(mode=F.PATHWISE)                    # warm-up of the pathwise pass
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    bp = ctx.backward(mode=F.PATHWISE)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    jp = bp["jac"].cpu().numpy()
    ctx.close()
    # the same two passes with everything on the caller's stream (no second stream)
    os.environ["FTAFQMC_SERIAL_BACKWARD"] = "1"
    cs = F.Context(sd)
    del os.environ["FTAFQMC_SERIAL_BACKWARD"]
    cs.propagate(f)
    cs.energy()
    cs.backward()
    torch.cuda.synchronize()
    t5 = time.perf_counter()
    cs.backward()
    torch.cuda.synchronize()
    t6 = time.perf_counter()
    cs.backward(mode=F.PATHWISE)
    torch.cuda.synchronize()
    t7 = time.perf_counter()
    cs.close()
    ws = inf["n_walkers"] * inf["n_slices"]
    return {"workload": workload, "forward_s": t1 - t0, "backward_s": t2 - t1, "backward_over_forward": (t2 - t1) / (t1 - t0),
            "walker_slices_per_s_backward": ws / (t2 - t1),
            "profile_ms": {k: v[0] for k, v in prof.items() if v[1]},
            "d<E>/dmu": jac[0].real, "d<N>/dmu": jac[1].real, "d<E>/dlambda": jac[2].real, "d<N>/dlambda": jac[3].real,
            "pathwise_s": t4 - t3, "pathwise_over_forward": (t4 - t3) / (t1 - t0),
            "one_stream_backward_s": t6 - t5, "one_stream_pathwise_s": t7 - t6,
            "pathwise": {"d<E>/dmu": jp[0].real, "d<N>/dmu": jp[1].real, "d<E>/dlambda": jp[2].real,
                         "d<N>/dlambda": jp[3].real}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ueg_n66_m171")
    ap.add_argument("--precision", choices=["both", "fp64", "mixed"], default="both")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-backward", action="store_true", help="skip the derivative-pass timing")
    ap.add_argument("--graph", action="store_true",
                    help="also time whole paths replayed from a captured HIP graph (no profiling events)")
    ap.add_argument("--overlap", action="store_true",
                    help="propagate with FTAFQMC_OVERLAP (two walker groups on two streams)")
    ap.add_argument("--no-overlap-schedule", action="store_true",
                    help="skip the extra timing of the mixed path with FTAFQMC_OVERLAP")
    ap.add_argument("--no-extra-workloads", action="store_true",
                    help="skip the one-path timings of the uneven four-system batch and the M=485 workload")
    ap.add_argument("--profile-run", action="store_true",
                    help="one warm-up path and one path of --precision (mixed when 'both') with no HIP events and "
                         "no other measurement: the program rocprofv3 kernel-trace and counter passes run")
    ap.add_argument("--profile-flags", type=int, default=0,
                    help="with --profile-run: params flags of the profiled systems (e.g. 64 low rank, 128 split BF16)")
    ap.add_argument("--profile-backward", choices=["frozen", "pathwise"], default=None,
                    help="one warm-up and one derivative pass of that mode on the M=123 workload, nothing else "
                         "(the program of the backward kernel-trace pass)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="run one plain device copy of this many MiB first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (walkers would shard "
              "across GPUs with no per-slice communication); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2012_12228_amd as F
    F.load_library()
    if args.copy_probe > 0:
        n = args.copy_probe * (1 << 20) // 4
        src_t = torch.ones(n, dtype=torch.float32, device="cuda")
        dst_t = torch.empty_like(src_t)
        dst_t.copy_(src_t)
        torch.cuda.synchronize()
        del src_t, dst_t
    wl = si.WORKLOADS[args.workload]
    if args.profile_backward:
        name = "ueg_n38_m123"
        sd = dict(si.WORKLOADS[name]["systems"][0], precision=0, flags=F.FTAFQMC_CHECKPOINT)
        ctx = F.Context(sd)
        inf = ctx.info()
        f = torch.from_numpy(si.fields(si.system_seed(name, 0), sd["walkers"], inf["n_slices"], inf["n_q"])).cuda()
        ctx.propagate(f)
        ctx.energy()
        mode = F.PATHWISE if args.profile_backward == "pathwise" else F.FROZEN_PATH
        ctx.backward(mode=mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.backward(mode=mode)
        torch.cuda.synchronize()
        print(json.dumps({"profile_backward": args.profile_backward, "seconds": time.perf_counter() - t0}))
        ctx.close()
        return
    if args.profile_run:
        p = "mixed" if args.precision == "both" else args.precision
        fields = load_fields(F, torch, args.workload)
        ctx = F.Context([dict(sd, precision=0 if p == "fp64" else 1, flags=args.profile_flags) for sd in wl["systems"]])
        _path(ctx, fields, len(wl["systems"]))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _path(ctx, fields, len(wl["systems"]))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ws = sum(ctx.info(i)["n_walkers"] * ctx.info(i)["n_slices"] for i in range(len(wl["systems"])))
        print(json.dumps({"profile_run": args.workload, "precision": p, "walker_slices_per_s": ws / dt}))
        ctx.close()
        return
    precs = ["fp64", "mixed"] if args.precision == "both" else [args.precision]
    results, fields = bench_workload(F, torch, args.workload, precs, args.steps, args.warmup, overlap=args.overlap)
    for p in precs:
        systems = [dict(sd, precision=0 if p == "fp64" else 1, flags=F.FTAFQMC_OVERLAP if args.overlap else 0)
                   for sd in wl["systems"]]
        if args.graph:
            results[p]["graph_replay"] = time_graph(F, torch, systems, fields, args.steps)
        if p == "mixed" and not args.overlap and not args.no_overlap_schedule:
            results[p]["overlap_schedule"] = time_overlap(F, torch, systems, fields, args.steps)
    del fields
    torch.cuda.empty_cache()
    cmp = results.get("mixed_vs_fp64")
    use = "mixed" if (cmp is not None and cmp["within_tolerance"]) else precs[0]
    if args.precision == "mixed":
        use = "mixed"
    r = results[use]
    prec_key = "f32" if use == "mixed" else "f64"
    achieved = r["gemm_tflops"]
    # the schedule of the headline: one stream, or the two walker groups of FTAFQMC_OVERLAP when
    # they are faster on this workload (bit-identical results, so the same mixed-vs-FP64 gate)
    best, schedule, groups = r, "one stream per system", r["walker_groups"]
    ov = r.get("overlap_schedule")
    if ov is not None and ov["walker_slices_per_s"] > r["walker_slices_per_s"]:
        best, schedule, groups = ov, "two walker groups on two streams (FTAFQMC_OVERLAP)", ov["walker_groups"]
    line = {
        "metric": "walker*slices/s incl. stabilised G+energy, FP64 vs mixed at <=1e-6 rel error",
        "value": best["walker_slices_per_s"], "unit": "walker*slices/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": best["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64-fp32mfma+f64" if use == "mixed" else "f64",
        "data": "synthetic (seeded N(0,1) auxiliary fields, free-electron trial)",
        "config": {"workload": args.workload, "systems": [
            {k: v for k, v in sd.items()} for sd in wl["systems"]], "precision_reported": use,
            "schedule": schedule, "walker_groups": groups},
        "roofline": {"bound": "mfma", "kernel": "propagator complex GEMM (%s MFMA)" % prec_key,
                     "achieved": achieved, "peak": PEAK_TFLOPS[prec_key], "unit": "TFLOP/s",
                     "frac": achieved / PEAK_TFLOPS[prec_key],
                     "traffic": measured_traffic(args.workload, use),
                     "avg_launch_ms": r["gemm_avg_ms"]},
        "fp64": results.get("fp64"), "mixed": results.get("mixed"), "mixed_vs_fp64": cmp,
        "end_to_end": end_to_end(wl, r, use),
    }
    if not args.no_extra_workloads and args.workload == "ueg_n66_m171":
        # the mixed path with its propagator products on the BF16 matrix cores (split operands)
        fl = load_fields(F, torch, args.workload)
        systems = [dict(sd, precision=1, flags=F.FTAFQMC_BF16_SPLIT) for sd in wl["systems"]]
        ctx, rb, enb = run_precision(F, torch, systems, fl, args.steps, args.warmup)
        ctx.close()
        del fl
        torch.cuda.empty_cache()
        issued = 6 * rb["gemm_tflops"]
        line["bf16_split"] = {
            "walker_slices_per_s": rb["walker_slices_per_s"], "ms_per_step": rb["ms_per_step"],
            "gemm_ms_per_step": rb["profile_ms_per_step"]["gemm"],
            "fp32_mfma_gemm_ms_per_step": results["mixed"]["profile_ms_per_step"]["gemm"],
            "gemm_useful_tflops": rb["gemm_tflops"], "gemm_issued_bf16_tflops": issued,
            "gemm_frac_of_bf16_peak_issued": issued / 2500.0,
            "vs_fp64": mixed_vs_fp64(results["energies"]["fp64"], enb)}
        print("bench: bf16 split %.1f walker*slices/s" % rb["walker_slices_per_s"], file=sys.stderr, flush=True)
    if not args.no_extra_workloads:
        extra = {}
        for name in ("ueg_uneven4", "ueg_n114_m485"):
            if name == args.workload:
                continue
            res, flds = bench_workload(F, torch, name, ["fp64", "mixed"], 1, 1)
            if name == "ueg_n114_m485":
                line["lowrank"] = time_lowrank(F, torch, name, flds, res)
                print("bench: low-rank %s %.1f walker*slices/s" % (name, line["lowrank"]["walker_slices_per_s"]),
                      file=sys.stderr, flush=True)
            del flds
            torch.cuda.empty_cache()
            extra[name] = {
                "walker_slices_per_s": {p: res[p]["walker_slices_per_s"] for p in ("fp64", "mixed")},
                "ms_per_step": {p: res[p]["ms_per_step"] for p in ("fp64", "mixed")},
                "gemm_roofline_frac": {p: res[p]["gemm_roofline_frac"] for p in ("fp64", "mixed")},
                "gemm_avg_ms": {p: res[p]["gemm_avg_ms"] for p in ("fp64", "mixed")},
                "system_ms": {p: res[p].get("system_ms") for p in ("fp64", "mixed")},
                "system_ms_sum_over_wall": {p: res[p].get("system_ms_sum_over_wall") for p in ("fp64", "mixed")},
                "serial_systems_walker_slices_per_s": res["mixed"].get("serial_systems_walker_slices_per_s"),
                "profile_ms_per_step": {p: res[p]["profile_ms_per_step"] for p in ("fp64", "mixed")},
                "mixed_vs_fp64": res["mixed_vs_fp64"]}
            print("workload %s done" % name, file=sys.stderr, flush=True)
        line["extra_workloads"] = extra
    if not args.no_backward:
        torch.cuda.empty_cache()
        line["backward"] = time_backward(F, torch)
        print("bench: backward done", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload)
        print("bench: cpu baseline done", file=sys.stderr, flush=True)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
