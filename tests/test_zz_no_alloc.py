"""The allocation-free entry point ftafqmc_init_ueg_static against ftafqmc_init_ueg.

Both handles run the same kernels on the same seeded fields; the static one takes its
workspace from the library's file-scope device array.  Two calls in a row, the second with a
smaller input (fewer walkers, another basis), must each match the workspace entry point to the
FP64 parity bar (1e-10 relative; the kernels are deterministic, so the results are in fact
identical); stale contents of the array from the first call must not leak into the second.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import ueg  # noqa: E402
import synthinputs as si  # noqa: E402

pytestmark = pytest.mark.gpu

FP64_REL = 1e-10


def _F():
    import paper_2012_12228_amd as F
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    F.load_library()
    return F


def _run(F, sd, flds, static):
    ctx = F.Context([sd], static_workspace=static)
    ctx.propagate([torch.from_numpy(flds).cuda()])
    e = ctx.energy()
    rec = ctx.records()
    out = dict(G=ctx.greens().cpu().numpy(), local=e["local"].cpu().numpy(), mean=e["mean"].cpu().numpy(),
               logw=e["logw"].cpu().numpy(), status=e["status"].cpu().numpy(),
               trace=rec["trace"].cpu().numpy(), rlogw=rec["logw"].cpu().numpy())
    ctx.close()
    torch.cuda.synchronize()
    return out


def _compare(a, b):
    assert np.array_equal(a["status"], b["status"])
    for key in ("G", "local", "mean", "trace"):
        scale = max(np.abs(b[key]).max(), 1e-300)
        assert np.abs(a[key] - b[key]).max() <= FP64_REL * scale, key
    for key in ("logw", "rlogw"):
        fin = np.isfinite(b[key])
        assert np.array_equal(fin, np.isfinite(a[key]))
        assert np.all(np.abs(a[key][fin] - b[key][fin]) <= FP64_REL * np.maximum(1.0, np.abs(b[key][fin]))), key


def test_static_workspace_matches_workspace_entry_point_twice():
    F = _F()
    first = dict(n_elec=14, rs=1.0, theta=0.5, nmax2=2, dtau=0.05, stab_every=5, walkers=64)
    second = dict(n_elec=2, rs=1.0, theta=0.5, nmax2=1, dtau=0.05, stab_every=3, walkers=8)
    for sd, seed in ((first, 101), (second, 202)):
        s = ueg.UEGSystem(sd["n_elec"], sd["rs"], sd["theta"], sd["nmax2"], sd["dtau"])
        assert F.ftafqmc_workspace_bytes([sd]) <= F.STATIC_WORKSPACE_BYTES
        flds = si.fields(seed, sd["walkers"], s.n_slices, s.NQ)
        got = _run(F, sd, flds, static=True)
        want = _run(F, sd, flds, static=False)
        _compare(got, want)


def test_static_workspace_refusals():
    F = _F()
    big = dict(n_elec=38, rs=1.0, theta=0.25, nmax2=9, dtau=0.05, stab_every=5, walkers=64)
    assert F.ftafqmc_workspace_bytes([big]) > F.STATIC_WORKSPACE_BYTES
    with pytest.raises(F.FtafqmcError) as ei:
        F.Context([big], static_workspace=True)
    assert ei.value.code == -1 and "static maximum" in str(ei.value)
    small = dict(n_elec=2, rs=1.0, theta=0.5, nmax2=1, dtau=0.05, stab_every=3, walkers=4)
    with pytest.raises(F.FtafqmcError) as ei:
        F.Context([dict(small, flags=2)], static_workspace=True)
    assert ei.value.code == -1
    holder = F.Context([small], static_workspace=True)
    with pytest.raises(F.FtafqmcError) as ei:
        F.Context([small], static_workspace=True)
    assert ei.value.code == -4
    holder.close()
    again = F.Context([small], static_workspace=True)        # released by destroy
    again.close()
