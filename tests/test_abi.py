"""The C-ABI library loads, exports every symbol the header declares, and its
host-side table code sizes workspaces and rejects invalid parameters (no GPU needed)."""
import os
import re

import pytest

torch = pytest.importorskip("torch")
import paper_2012_12228_amd as F  # noqa: E402
import synthinputs as si  # noqa: E402

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "ftafqmc.h")


def _lib():
    if not os.path.exists(F.LIB_PATH):
        pytest.skip("library not built")
    return F.load_library()


def test_header_symbols_are_exported():
    lib = _lib()
    text = open(HEADER).read()
    declared = set(re.findall(r"^\s*(?:int|void|const char\*|size_t)\s+(ftafqmc_\w+)\s*\(", text, re.M))
    assert declared == set(F.ABI_SYMBOLS)
    for name in declared:
        assert hasattr(lib, name), name


def test_workspace_sizes_of_the_workloads():
    _lib()
    for name, wl in si.WORKLOADS.items():
        b = F.ftafqmc_workspace_bytes(wl["systems"])
        assert b > 0
    one = F.ftafqmc_workspace_bytes([dict(si.WORKLOADS["ueg_n14_m19"]["systems"][0])])
    two = F.ftafqmc_workspace_bytes([dict(si.WORKLOADS["ueg_n14_m19"]["systems"][0], walkers=128)])
    assert two > one


@pytest.mark.parametrize("bad", [dict(n_elec=13), dict(n_elec=0), dict(nmax2=0), dict(walkers=0),
                                 dict(stab_every=0), dict(rs=-1.0), dict(theta=0.0), dict(dtau=0.0),
                                 dict(nmax2=30), dict(nmax2=25), dict(precision=7), dict(n_elec=200, nmax2=1)])
def test_invalid_parameters_are_rejected(bad):
    _lib()
    sysdef = dict(si.WORKLOADS["ueg_n14_m19"]["systems"][0])
    sysdef.update(bad)
    with pytest.raises(RuntimeError, match="E_ARG"):
        F.ftafqmc_workspace_bytes([sysdef])


@pytest.mark.parametrize("bad", [dict(flags=1024), dict(flags=1, precision=1), dict(flags=1, nmax2=11, n_elec=66, theta=0.125),
                                 dict(flags=64 | 1), dict(flags=64 | 16)])
def test_invalid_flags_are_rejected(bad):
    """Unknown flag bits, a path record with mixed precision, a path record whose doubled
    system would exceed the elimination's 512 rows (M = 171 is fine; M > 256 is not), and the
    low-rank truncation with the path record or the modified overlap ratio."""
    _lib()
    sysdef = dict(si.WORKLOADS["ueg_n14_m19"]["systems"][0])
    sysdef.update(bad)
    if bad.get("nmax2") == 11:
        sysdef.update(nmax2=24, n_elec=114)          # M = 485
    with pytest.raises(RuntimeError, match="E_ARG"):
        F.ftafqmc_workspace_bytes([sysdef])


def test_flag_values_match_the_header():
    text = open(HEADER).read()
    for name, val in (("FTAFQMC_CHECKPOINT", F.FTAFQMC_CHECKPOINT), ("FTAFQMC_OVERLAP", F.FTAFQMC_OVERLAP),
                      ("FTAFQMC_GRAPH", F.FTAFQMC_GRAPH), ("FTAFQMC_FROZEN_PATH", F.FROZEN_PATH),
                      ("FTAFQMC_PROFILE_ONLY", F.FTAFQMC_PROFILE_ONLY), ("FTAFQMC_TRIAL_THF", F.FTAFQMC_TRIAL_THF),
                      ("FTAFQMC_POP_COMB", F.POP_COMB), ("FTAFQMC_POP_PAIR_BRANCH", F.POP_PAIR_BRANCH),
                      ("FTAFQMC_PATHWISE", F.PATHWISE), ("FTAFQMC_LOW_RANK", F.FTAFQMC_LOW_RANK)):
        m = re.search(r"#define\s+%s\s+(\d+)" % name, text)
        assert m and int(m.group(1)) == val, name


def test_path_record_grows_the_workspace():
    _lib()
    sd = dict(si.WORKLOADS["ueg_n38_m123"]["systems"][0])
    plain = F.ftafqmc_workspace_bytes([sd])
    rec = F.ftafqmc_workspace_bytes([dict(sd, flags=F.FTAFQMC_CHECKPOINT)])
    # the record alone holds W n N_Q complex128 coefficients
    assert rec - plain > sd["walkers"] * 174 * 828 * 16


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
