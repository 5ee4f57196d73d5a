"""Host-side checks of the benchmark's contract and its work accounting (no
GPU): the one-GPU refusal, the per-node network work of Eq. 2's layers, the
decay-pair ceilings, the roofline's choice of bound, and that measured HBM
traffic is reported only for the kernel sources it was taken on."""
import os
import subprocess
import sys

import bench


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"], cwd=bench.ROOT,
                       capture_output=True, text=True, timeout=300)
    assert "one GPU" in r.stdout + r.stderr
    assert not any(ln.startswith("{") for ln in r.stdout.splitlines())


def test_network_work_per_node_follows_the_layer_sizes():
    # encoder 9 -> 64 -> 64 on every node of a contacted patch; decoder
    # [f; g'] -> 64 -> 3 on its passive nodes, the g' half folded into a
    # per-item constant; the global MLP 64 -> 64 -> 64 once per item
    assert bench.ENC_MAC == 9 * 64 + 64 * 64 == 4672
    assert bench.DEC_MAC == 64 * 64 + 64 * 3 == 4288
    assert bench.GLOBAL_MAC == 2 * 64 * 64
    assert bench.MFMA_PASSES == 3


def test_pair_ceilings_from_the_issue_slots():
    # 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz, one pair per PAIR_SLOTS issue slots
    slots = 256 * 4 * 16 * 2.4e9
    assert abs(bench.PAIR_CEILING - slots / bench.PAIR_SLOTS) < 1.0
    assert abs(bench.PAIR_CEILING_BWD - slots / bench.PAIR_SLOTS_BWD) < 1.0
    assert bench.PAIR_CEILING > bench.PAIR_CEILING_BWD


def test_roofline_names_the_binding_resource():
    # 1e12 FP32-equivalent flop in 1 ms: 1000 TFLOP/s against 2500, lower
    # bound 3 passes x 1e12 / 2.5e15 s = 1.2 ms, above the HBM and pair bounds
    r = bench.roofline_of("k_none", 1.0, {"mfma_flop": 1e12, "pairs": 1e6, "hbm_bytes": 1e6})
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    assert abs(r["achieved"] - 1000.0) < 1e-6 and abs(r["frac"] - 0.4) < 1e-9
    assert abs(r["lower_bound_ms"]["mfma"] - 1.2) < 1e-9
    assert r["traffic"] is None        # no profile for this kernel
    r = bench.roofline_of("k_none", 0.5, {"mfma_flop": 0.0, "pairs": 0.0, "hbm_bytes": 2e9})
    assert r["bound"] == "hbm" and abs(r["achieved"] - 4000.0) < 1e-6 and abs(r["frac"] - 0.5) < 1e-9
    r = bench.roofline_of("k_bwd_decay", 1.0, {"mfma_flop": 0.0, "pairs": 1e9, "hbm_bytes": 1e6})
    assert r["bound"] == "alu" and abs(r["peak"] - round(bench.PAIR_CEILING_BWD / 1e9, 3)) < 1e-9


def test_traffic_only_for_the_profiled_sources(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    path = tmp_path / "k_step_hand4096_hbm_traffic.txt"
    path.write_text(f"source_digest: {bench.source_digest('k_step')}\nhbm_bytes_per_launch: 123456.0\n")
    assert bench.measured_traffic("k_step", "hand") == 123456.0
    path.write_text("source_digest: 0000000000000000\nhbm_bytes_per_launch: 123456.0\n")
    assert bench.measured_traffic("k_step", "hand") is None
    assert bench.measured_traffic("k_bwd", "hand") is None        # no summary at all


def test_regressor_digest_is_separate_from_the_step():
    # the regressor's profiles stay valid across step-kernel edits and back
    assert bench.source_digest("k_regress") != bench.source_digest("k_step")
    assert bench.source_digest("k_step") == bench.source_digest("k_bwd") == bench.source_digest(None)
