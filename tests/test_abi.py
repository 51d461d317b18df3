"""The C-ABI library builds, loads and exports every entry point declared in
include/rtg.h; host-side argument checks (no GPU needed)."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from paper_2603_00839_amd import rtg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(rtg.LIB_PATH):
        from paper_2603_00839_amd import build_lib
        build_lib.build()
    return rtg.load_library()


def test_header_declares_the_four_core_calls():
    syms = rtg.header_symbols()
    for name in ["rtg_setup_operator", "rtg_sketch", "rtg_arnoldi", "rtg_solve"]:
        assert name in syms


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", rtg.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [s for s in rtg.header_symbols() if s not in exported]
    assert not missing, missing
    for s in rtg.header_symbols():
        assert getattr(lib, s) is not None


def test_library_is_gfx950(lib):
    with open(rtg.LIB_PATH, "rb") as f:
        blob = f.read()
    assert b"amdgcn-amd-amdhsa--gfx950" in blob


def test_status_strings(lib):
    assert lib.rtg_status_string(0) == b"ok"
    assert lib.rtg_status_string(-5) == b"workspace too small"


def test_setup_rejects_bad_shapes_before_touching_the_device(lib):
    h = ctypes.c_void_p()
    band = np.ones((12, 3), np.float32)
    fp = band.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    # I1 not a multiple of 8
    assert lib.rtg_setup_operator(12, 8, 3, fp, 1, fp, 1, fp, 1, ctypes.byref(h)) == -2
    # half-bandwidth beyond the supported maximum
    assert lib.rtg_setup_operator(64, 64, 3, fp, 13, fp, 1, fp, 1, ctypes.byref(h)) == -2
    # null band
    assert lib.rtg_setup_operator(16, 8, 3, None, 1, fp, 1, fp, 1, ctypes.byref(h)) == -1
    # sketch larger than the mode, or missing factor with l != I
    assert lib.rtg_setup_sketch(16, 16, 3, 32, 8, 3, fp, fp, None, ctypes.byref(h)) == -2
    assert lib.rtg_setup_sketch(16, 16, 3, 8, 8, 3, None, fp, None, ctypes.byref(h)) == -2
    assert lib.rtg_setup_sketch(16, 16, 3, 8, 8, 2, fp, fp, None, ctypes.byref(h)) == -2
    # mode 1 beyond the 32-bit offsets of the operand-order copies
    assert lib.rtg_setup_sketch(1 << 20, 16, 3, 8, 8, 3, fp, fp, None, ctypes.byref(h)) == -2
    # null handles
    assert lib.rtg_workspace_bytes(None, None, 10, 0) == 0
    assert lib.rtg_solve(None, None, None, None, None, None, 0, None, None, None) == -1
    assert lib.rtg_solve_batched(0, None, None, 0, None) == -1


def test_params_struct_layout_matches_header():
    assert ctypes.sizeof(rtg.Params) == 4 + 4 + 5 * 8 + 16     # mu_rule, method, restarts + padding
    assert rtg.Params.mu_rule.offset == 4 + 4 + 5 * 8
    assert rtg.Params.method.offset == 4 + 4 + 5 * 8 + 4
    assert rtg.Params.restarts.offset == 4 + 4 + 5 * 8 + 8
    assert ctypes.sizeof(rtg.Info) == 4 + 4 + 4 * 8
    assert rtg.Problem.params.offset == 5 * 8


def test_tune_struct_layout_matches_header():
    assert ctypes.sizeof(rtg.Tune) == 32
    for i, f in enumerate(rtg.Tune.FIELDS):
        assert getattr(rtg.Tune, f).offset == 4 * i
    assert rtg.Tune.persist.offset == 28
    t = rtg.make_tune(tile_rows=4)
    assert t.as_dict() == dict(phi_jt=-1, phi_slab=-1, phi_toeplitz=-1, tile_rows=4, step_rows=-1, step_toeplitz=-1,
                               gram_pairs=-1, persist=-1)
    with pytest.raises(rtg.RTGError):
        rtg.make_tune(rows=2)


def test_tune_calls_check_arguments_on_the_host(lib):
    t = rtg.Tune()
    ms = ctypes.c_double()
    assert lib.rtg_tune_clear() == 0
    assert lib.rtg_tune_set(0, None, ctypes.byref(t)) == -1
    assert lib.rtg_tune_get(1, None, ctypes.byref(t)) == -1
    assert lib.rtg_autotune_batched(1, None, None, 0, 1, ctypes.byref(t), ctypes.byref(ms), None) == -1
    # a problem with null handles
    arr = (rtg.Problem * 1)()
    assert lib.rtg_tune_set(1, arr, ctypes.byref(t)) == -1
    assert lib.rtg_tune_get(1, arr, None) == -1
    assert lib.rtg_autotune_batched(1, arr, None, 0, 0, ctypes.byref(t), None, None) == -1


def test_wait_limit_and_timeout_flag(lib):
    """rtg_set_wait_limit takes any count >= 0 (host state only); the flag
    that an abandoned persistent launch leaves is the header's value."""
    assert lib.rtg_set_wait_limit(-1) == -1
    assert lib.rtg_set_wait_limit(0) == 0
    assert lib.rtg_set_wait_limit(1 << 22) == 0
    with open(os.path.join(ROOT, "include", "rtg.h")) as f:
        hdr = f.read()
    assert "RTG_F_TIMEOUT = 64" in hdr and rtg.FLAG_TIMEOUT == 64
