"""The C-ABI library loads on the host and exports every function that
include/mcrt.h declares (no compute calls: there is no GPU here)."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcrt.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mcrt_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("mcrt_context_create", "mcrt_grid_create_cartesian", "mcrt_grid_create_octree",
                 "mcrt_medium_create", "mcrt_source_create_point", "mcrt_source_create_expdisk",
                 "mcrt_instrument_create", "mcrt_sim_create", "mcrt_run", "mcrt_run_range",
                 "mcrt_run_into", "mcrt_result_absorption", "mcrt_result_image",
                 "mcrt_result_energy", "mcrt_result_stats", "mcrt_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1705_04702_amd import mcrt
    L = mcrt.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(mcrt.EXPORTS) == declared_functions()


def test_host_side_options_and_errors():
    from paper_1705_04702_amd import mcrt
    o = mcrt.default_options()
    assert o.precision == mcrt.FP32 and o.w_min == 1e-6 and o.event_cap == 10000
    assert o.tau_peel_max == math.inf and o.top_level == -1 and o.queue_order == mcrt.QUEUE_PAIRED
    assert o.chunk_shift == 0 and o.deposit_slots == 0
    with pytest.raises(TypeError):  # a misspelt option is an error, not a silent no-op
        mcrt.default_options(treshold=8)
    L = mcrt.lib()
    h = ctypes.c_void_p()
    # a NULL context is rejected before any device call
    box = (ctypes.c_double * 6)(0, 0, 0, 1, 1, 1)
    n = (ctypes.c_int32 * 3)(2, 2, 2)
    assert L.mcrt_grid_create_cartesian(None, box, n, ctypes.byref(h)) == mcrt.EINVAL
    assert b"NULL" in L.mcrt_last_error()
    assert L.mcrt_run_into(None, 1, 0, 1, 0, None) == mcrt.EINVAL
