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
                                 dict(nmax2=30), dict(precision=7), dict(n_elec=200, nmax2=1)])
def test_invalid_parameters_are_rejected(bad):
    _lib()
    sysdef = dict(si.WORKLOADS["ueg_n14_m19"]["systems"][0])
    sysdef.update(bad)
    with pytest.raises(RuntimeError, match="E_ARG"):
        F.ftafqmc_workspace_bytes([sysdef])
