"""Host logic of the benchmark's `traffic` field: the committed rocprofv3
counter summary is used only when it was taken on the current stencil source,
and then for the launch shape that the autotuner kept (paired, sequential or
time-marching form)."""
import os
import re

import bench


def _summary():
    path = os.path.join(bench.ROOT, "profiles", "tsl_stencil_14x14cubed_traffic.txt")
    kv = {}
    for line in open(path):
        if ":" in line:
            a, b = line.split(":", 1)
            kv[a.strip()] = b.strip()
    return kv


def _current(kv):
    import hashlib
    src = os.path.join(bench.ROOT, "paper_1611_00195_amd", "csrc", "kernels_stencil.hip")
    return kv.get("kernels_stencil_sha256_16") == hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def test_traffic_follows_the_kept_shape():
    kv = _summary()
    fresh = _current(kv)
    cases = [
        (8, "tsl:d:1:8=map1,gpb8;", "bytes_per_launch_fp64_nrhs8_map1_gpb8"),
        (8, "tsl:d:1:8=map0,gpb1,seq;", "bytes_per_launch_fp64_nrhs8_map0_gpb1_seq"),
        (8, "op:d:1:48=map0,gpb8,rp2;tsl:d:1:8=map0,gpb2,march;", "bytes_per_launch_fp64_nrhs8_map0_gpb2_march"),
        (4, "tsl:f:1:8=map1,gpb4,march;tsl:d:1:8=map1,gpb8;", "bytes_per_launch_fp32_nrhs8_map1_gpb4_march"),
    ]
    for pb, shapes, key in cases:
        assert key in kv, key
        want = float(kv[key]) if fresh else None
        assert bench.measured_traffic(pb, 8, shapes) == want, (shapes, key)
    # no entry for this precision and batch, or a batch the summary does not cover
    # (the summary's source hash must match the stencil source for any value;
    # if the stencil changed since the counters were taken, every case is None)
    assert bench.measured_traffic(8, 8, "tsl:f:1:8=map1,gpb8;") is None
    assert bench.measured_traffic(8, 16, "tsl:d:1:16=map1,gpb8;") is None


def test_tuned_entry_picks_the_stencil_of_its_precision():
    shapes = "op:d:1:48=map0,gpb8,rp2;tsl:d:1:8=map1,gpb8;tsl:f:1:8=map0,gpb2,march;"
    assert bench.tuned_entry(shapes, 8, 8) == "tsl:d:1:8=map1,gpb8;"
    assert bench.tuned_entry(shapes, 4, 8) == "tsl:f:1:8=map0,gpb2,march;"
    assert re.search(",march;", bench.tuned_entry(shapes, 4, 8))
    assert bench.tuned_entry(shapes, 8, 32) == ""
