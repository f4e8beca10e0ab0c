"""Host-side checks of bench.py: it runs on one GPU only, its algorithmic byte counts are
the documented sums, and the committed rocprofv3 summaries it reads parse."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_byte_counts():
    import bench
    # populations read + written, u* block sum S read + written, the FP64 fold of U every
    # 16 levels (FP32/FP16) or the FP64 u* (F64); the two-level kernel moves the
    # populations and S once per two levels
    assert bench.BYTES_PER_LU == {"f32": 210.0, "f16": 114.0, "f64": 416}
    assert bench.BYTES_PER_LU_PAIR == {"f32": 212.0, "f16": 116.0, "f64": 416}
    # four levels per launch: populations and S once per launch, U folded on a quarter of them
    assert [bench.bytes_per_lu_multi(s, 4) for s in ("f32", "f16", "f64")] == [216.0, 120.0, 416]
    assert bench.bytes_per_lu_multi("f32", 2) == 212.0
    # the forward + adjoint byte model: forward, replay and adjoint in multi-level launches
    assert [bench.fwd_adj_multi_bytes("fwd", t) for t in (2, 3, 4)] == [228, 230, 232]
    # the replay's records: the F - I planes only (16 B per node and level)
    assert [bench.fwd_adj_multi_bytes("replay", t) for t in (2, 3, 4)] == [240, 256, 272]
    # the adjoint: populations 192, F - I 16 per level, mu lam 8, block sums 32, FP64 fold
    # 64 B once in 16 levels
    assert [bench.fwd_adj_multi_bytes("adj", t) for t in (2, 3, 4)] == [272, 292, 312]
    assert bench.fwd_adj_bytes_per_level("f32", 50, (4, 4, 4)) == 232 / 4 + 272 / 4 + 312 / 4 + 240 / 50
    assert bench.fwd_adj_bytes_per_level("f64", 25) == (432 + 496 + 584) / 2 + 480 / 25


def test_profile_summaries_parse():
    import bench
    for kernel, path in bench.PROFILE_PMC.items():
        assert os.path.exists(path), path
        kv = {}
        with open(path) as fh:
            for line in fh:
                if "=" in line and not line.startswith("#"):
                    k, v = line.split("=", 1)
                    kv[k.strip()] = v.strip()
        assert kv["grid"] == "8192x8192"
        ratio = float(kv["traffic_over_algorithmic"])
        assert 0.9 < ratio < 1.1, (kernel, ratio)
        t = bench.measured_traffic(8192, kernel)
        assert t is None or abs(t - float(kv["traffic_bytes_per_launch"])) < 1.0
