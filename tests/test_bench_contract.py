"""Host-side checks of the benchmark and the shipped tuning table (no GPU needed)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    """The benchmark measures one GPU: --gpus above 1 exits with status 2 and says why,
    before the GPU runtime is touched."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "--gpus 2 is not supported" in r.stderr
    assert r.stdout.strip() == ""


def test_tuning_table_uses_built_shapes():
    """Every entry of the autotuner's table names a tile shape the library builds and a
    positive row-chunk count, and the unfused switch (when present) is 0 or 1."""
    from paper_2606_01211_amd import tune

    table = json.load(open(os.path.join(ROOT, "paper_2606_01211_amd", "tuning.json")))
    assert table
    for n, t in table.items():
        assert (t["col_groups"], t["row_groups"]) in tune.SHAPES, n
        assert t["m_chunks"] >= 1, n
        assert t.get("a_source", 0) in (0, 1), n
        assert tune.lds_fits(t["col_groups"], int(n)), n


def test_lane_count_divides_the_timed_steps():
    """Every lane runs the same number of timed steps: 20 steps on at most 14 lanes use 10
    lanes of two steps, on 20 lanes (the default) one step each; 140 steps 14 or 20 lanes."""
    sys.path.insert(0, ROOT)
    import bench

    assert bench.pick_lanes(20, 14) == (10, True)
    assert bench.pick_lanes(140, 14) == (14, True)
    assert bench.pick_lanes(20, 20) == (20, True)
    assert bench.pick_lanes(140, 20) == (20, True)
    assert bench.pick_lanes(5, 14) == (5, True)
    assert bench.pick_lanes(1, 14) == (1, True)
    s, even = bench.pick_lanes(17, 14)
    assert s == 14 and not even
