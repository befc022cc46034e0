"""The C-ABI library loads and exports every function include/tpc_ca.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1910_12214_amd", "libtpcca.so")


def declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"^\s*(?:int|void|const char\*)\s+(tpc_\w+)\s*\(", src, flags=re.M))
    return names


def test_header_declares_the_entry_points():
    names = declared()
    for n in ("tpc_ctx_create", "tpc_track_sectors", "tpc_track_timeframe", "tpc_mlp_infer", "tpc_mlp_train"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="HIP library not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="HIP library not built")
def test_binding_matches_header():
    from paper_1910_12214_amd import tpcca

    assert set(tpcca.EXPORTS) == declared()
    # default parameters are the workload settings the oracle is checked with
    import synth

    d = tpcca.default_params()
    for k, v in synth.TRACKER_PARAMS.items():
        assert d[k] == pytest.approx(v), k


@pytest.mark.skipif(not os.path.exists(LIB), reason="HIP library not built")
def test_merge_defaults_are_the_oracle_readings():
    """tpc_merge_params_default holds the constants of the merging oracle's reading (a host call)."""
    from oracle import merge as om
    from paper_1910_12214_amd import tpcca

    mp = tpcca.Context.merge_params()
    assert (mp.rho_max, mp.centre_window, mp.chi2_max, mp.phase_sigmas, mp.phase_floor, mp.max_turns) == \
        (om.RHO_MAX, om.CENTRE_WINDOW, om.CHI2_HELIX, om.PHASE_SIGMAS, om.PHASE_FLOOR, om.MAX_TURNS)
    assert mp.sectors_per_side == 18 and mp.max_iter == 50 and mp.pair_queue == 4
