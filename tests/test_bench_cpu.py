"""CPU checks of the benchmark's accounting: the algorithmic bytes per kernel
and the HBM traffic record of the dominant kernel."""
import hashlib
import json
import os

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_kernel_bytes_per_pixel():
    f = 0.785
    kb = bench.kernel_bytes(256, f)
    # y read once; phi, (kappa, theta~) and the phi output on the pupil only
    assert abs(kb["stats"] - (8 + 4 * f)) < 1e-12
    assert abs(kb["row_ifft"] - (8 + 12 * f)) < 1e-12
    assert kb["col_fused"] == 24
    assert abs(kb["row_fft"] - (8 + 20 * f)) < 1e-12
    assert abs(kb["m_step"] - (12 + 16 * f)) < 1e-12
    # the fused first row pass reads y and phi once for both jobs
    assert kb["stats_row_ifft"] == kb["row_ifft"]
    assert abs(kb["frame_worklist"] - (kb["stats"] + kb["row_ifft"] + kb["col_fused"] + kb["row_fft"])) < 1e-12
    # the eager step (fused pass, column pass, second row pass, M-step) and
    # its 56 B/px floor
    step = kb["stats_row_ifft"] + kb["col_fused"] + kb["row_fft"] + kb["m_step"]
    assert 89 < step < 91 and step > 56


def test_traffic_record_matches_the_kernel_source_or_is_refused():
    rec = json.load(open(os.path.join(ROOT, "profiles", "m_step_traffic.json")))
    src = os.path.join(ROOT, "paper_2305_03284_amd", "csrc", "ddh_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    tiles = rec["tiles"]
    traffic, note = bench.recorded_traffic("m_step", tiles)
    if rec["source_sha256_prefix"] == sha:
        assert traffic == rec["traffic_bytes"]
        assert sha in note
        # the counters' bytes: the scaled FETCH_SIZE and WRITE_SIZE (MiB)
        want = (rec["fetch_scale"] * rec["fetch_mib"] + rec["write_scale"] * rec["write_mib"]) * 2 ** 20
        assert abs(traffic - want) <= 0.01 * 2 ** 20
        # at least the kernel's algorithmic bytes at 64 x N = 256
        assert traffic >= bench.kernel_bytes(256, 0.785)["m_step"] * 64 * 256 * 256 * 0.99
    else:
        assert traffic is None and "changed" in note
    # another tiling or another kernel: no figure
    assert bench.recorded_traffic("m_step", [t + 1 for t in tiles])[0] is None
    assert bench.recorded_traffic("col_fused", tiles)[0] is None
