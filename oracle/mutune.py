"""Tuning of the interacting chemical potential (oracle side; test infrastructure).

Sec. "Computational Details": mu is tuned so that the ensemble's electron number <N> matches
N-bar.  The paper first brackets the root with single runs (error bars ignored) until mu is
known to about 1%, mu~; then runs five poorly converged simulations on [0.975 mu~, 1.025 mu~]
and fits them by weighted least squares to obtain mu*.  The alternative here takes Newton
steps with d<N>/dmu from the frozen-path derivative (oracle.tangent).

One "run" at mu is the whole path of every walker on the same fields (common random numbers),
with <N> the weighted mean at tau = beta over live walkers and its standard error from
popctl.ensemble_stats.

Readings (the paper states the procedure in words):
  * the scale of "1%" and of the fit interval is max(|mu|, 1 / beta) (mu can be near zero);
  * bracketing starts at mu0 with steps 0.05 scale, doubled until the sign of <N> - N-bar
    changes, then bisects until the bracket is below 1% of the scale; mu~ is its midpoint;
  * the five fit points are mu~ + scale {-0.025, -0.0125, 0, 0.0125, 0.025}; the fit is a
    straight line N = a + b mu with weights 1 / sigma^2 (equal weights if any sigma is 0);
  * Newton: mu <- mu - (<N> - N-bar) / (d<N>/dmu) until |<N> - N-bar| <= tol N-bar.
"""
import numpy as np

from . import ueg, path, energy, tangent, popctl

BRACKET, NEWTON = 0, 1


def ensemble_number(sys_kwargs, fields, mu, derivative=False):
    """(<N>, standard error, d<N>/dmu or None) of one run at mu (Re parts)."""
    sysx = ueg.UEGSystem(mu=mu, **sys_kwargs)
    vals, dvals, logw, dlogw, status = [], [], [], [], []
    for z in fields:
        if derivative:
            fwd, tan = tangent.walker_tangents(sysx, z, params=("mu",))
            t = tan["mu"]
            vals.append(fwd["E"]["N"])
            dvals.append(t["dN"])
            dlogw.append(t["dlogw"])
            logw.append(fwd["logw"])
            status.append(fwd["status"])
        else:
            out = path.run_walker(sysx, z, energy_fn=energy.local_energy)
            vals.append(out["records"][-1]["N"])
            logw.append(out["logw"])
            status.append(out["status"])
    st = popctl.ensemble_stats(np.real(vals), np.array(logw), np.array(status))
    dn = None
    if derivative:
        _, dmean = tangent.ensemble_tangent(np.array(vals), np.array(dvals), np.array(logw),
                                            np.array(dlogw), np.array(status))
        dn = float(np.real(dmean))
    return float(st["mean"]), float(st["stderr"]), dn


def bracket_fit(sys_kwargs, fields, n_target, mu0, max_runs=60):
    """The paper's procedure; returns dict(mu, mu_tilde, runs, trace [(mu, N, err)])."""
    beta = ueg.UEGSystem(**sys_kwargs).beta
    trace = []

    def run(mu):
        if len(trace) >= max_runs:
            raise RuntimeError("chemical-potential tuning exceeded its run budget")
        n, e, _ = ensemble_number(sys_kwargs, fields, mu)
        trace.append((mu, n, e))
        return n

    scale0 = max(abs(mu0), 1.0 / beta)
    step = 0.05 * scale0
    if run(mu0) < n_target:
        a = mu0
        b = a + step
        while run(b) < n_target:
            a, step = b, 2.0 * step
            b = a + step
    else:
        b = mu0
        a = b - step
        while not (run(a) < n_target):
            b, step = a, 2.0 * step
            a = b - step
    while b - a > 0.01 * max(abs(0.5 * (a + b)), 1.0 / beta):
        m = 0.5 * (a + b)
        if run(m) < n_target:
            a = m
        else:
            b = m
    mu_t = 0.5 * (a + b)
    scale = max(abs(mu_t), 1.0 / beta)
    pts = []
    for off in (-0.025, -0.0125, 0.0, 0.0125, 0.025):
        mu = mu_t + off * scale
        run(mu)
        pts.append(trace[-1])
    mus, ns, errs = (np.array(x) for x in zip(*pts))
    wts = 1.0 / errs ** 2 if np.all(errs > 0) else np.ones_like(errs)
    A = np.stack([np.ones_like(mus), mus], axis=1)
    a_fit, b_fit = np.linalg.solve(A.T @ (wts[:, None] * A), A.T @ (wts * ns))
    return dict(mu=(n_target - a_fit) / b_fit, mu_tilde=mu_t, runs=len(trace), trace=trace)


def newton(sys_kwargs, fields, n_target, mu0, tol=1e-8, max_runs=30):
    """Newton steps with the frozen-path d<N>/dmu; returns dict(mu, N, runs, trace)."""
    mu, trace = mu0, []
    for _ in range(max_runs):
        n, e, dn = ensemble_number(sys_kwargs, fields, mu, derivative=True)
        trace.append((mu, n, e, dn))
        if abs(n - n_target) <= tol * n_target:
            return dict(mu=mu, N=n, runs=len(trace), trace=trace)
        mu = mu - (n - n_target) / dn
    raise RuntimeError("Newton tuning of mu did not converge")
