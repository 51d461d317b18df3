"""Host logic of bench.py (no GPU): the refusal of several GPUs, the
algorithmic byte counts against their closed forms, and the conditions under
which a recorded HBM traffic figure is reported (same kernel source, variant,
batch size and launch shapes)."""
import hashlib
import json
import os
import shutil
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


@pytest.mark.parametrize("m", [1, 2, 7, 50])
def test_byte_counts_match_closed_forms(m):
    n = 786432
    for es in (2, 4):
        # fused step j = 1 .. m - 1 moves j + 1 tensors: es n (m (m + 1) / 2 - 1)
        assert bench.step_bytes(n, es, m) == es * n * (m * (m + 1) // 2 - 1)
        # tile launches: R0 sketch and V1 (8n + es n), the steps as above, the
        # assembly (X0 if given, m basis tensors, X)
        for x0 in (False, True):
            want = 8 * n + es * n + es * n * (m * (m + 1) // 2 - 1) + (4 * n if x0 else 0) + m * es * n + 4 * n
            assert bench.tile_bytes(n, es, m, x0) == want
        # operator with W in memory: m launches, each reads V_j, writes W
        assert bench.phi_bytes(n, es, m) == m * (es + 4) * n
        # Golub-Kahan: 12 n of float32 traffic (R0 twice, X) and 5 m - 2
        # basis tensors (U_1, V_1..V_m written and read back, U_2..U_m)
        assert bench.gk_tile_bytes(n, es, m) == 12 * n + es * n * (5 * m - 2)
    # one-step special cases by hand
    assert bench.step_bytes(n, 2, 2) == 2 * 2 * n     # reads V_1, writes V_2


def test_recorded_traffic_needs_the_same_source_variant_batch_and_shapes(tmp_path, monkeypatch):
    src = os.path.join(ROOT, "paper_2603_00839_amd", "csrc", "k_step.hip")
    os.makedirs(tmp_path / "paper_2603_00839_amd" / "csrc")
    os.makedirs(tmp_path / "profiles")
    shutil.copy(src, tmp_path / "paper_2603_00839_amd" / "csrc" / "k_step.hip")
    shutil.copy(os.path.join(ROOT, "paper_2603_00839_amd", "csrc", "k_tile.hip"),
                tmp_path / "paper_2603_00839_amd" / "csrc" / "k_tile.hip")
    hdr = os.path.join(ROOT, "paper_2603_00839_amd", "csrc", "rtg_internal.h")
    shutil.copy(hdr, tmp_path / "paper_2603_00839_amd" / "csrc" / "rtg_internal.h")
    # the step kernel's source followed by the one local header it includes
    # (the public header it reaches through "../../include" is absent here)
    sha = hashlib.sha256(open(src, "rb").read() + open(hdr, "rb").read()).hexdigest()
    shapes = dict(phi_jt=4, phi_slab=1, phi_toeplitz=1, tile_rows=2, step_rows=2, step_toeplitz=1)
    rec = {"k_step.hip": {"source_sha256": sha, "variant": "bf16_warm", "batch": 32, "launch_shapes": shapes,
                          "bytes_per_launch": 123.0}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    tune = {"autotuned": True, "loop_ms": 1.0, **shapes}
    assert bench.recorded_traffic("k_step.hip", "bf16_warm", tune, 32) == 123.0
    assert bench.recorded_traffic("k_step.hip", "bf16_uneven", tune, 32) is None
    assert bench.recorded_traffic("k_step.hip", "bf16_warm", tune, 16) is None
    assert bench.recorded_traffic("k_step.hip", "bf16_warm", {**tune, "step_rows": 4}, 32) is None
    assert bench.recorded_traffic("k_tile.hip", "bf16_warm", tune, 32) is None     # nothing recorded for it
    with open(tmp_path / "paper_2603_00839_amd" / "csrc" / "rtg_internal.h", "a") as f:
        f.write("\n// changed\n")
    assert bench.recorded_traffic("k_step.hip", "bf16_warm", tune, 32) is None   # a header of the kernel changed
    shutil.copy(hdr, tmp_path / "paper_2603_00839_amd" / "csrc" / "rtg_internal.h")
    assert bench.recorded_traffic("k_step.hip", "bf16_warm", tune, 32) == 123.0
    with open(tmp_path / "paper_2603_00839_amd" / "csrc" / "k_step.hip", "a") as f:
        f.write("\n// changed\n")
    assert bench.recorded_traffic("k_step.hip", "bf16_warm", tune, 32) is None
