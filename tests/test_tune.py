"""Host logic of the autotuner: workload classes and table lookup."""
import numpy as np


def test_workload_class_buckets():
    from paper_2002_05200_amd import tune
    c = tune.workload_class(np.array([50, 50, 100]), np.array([10000] * 3), np.array([10500] * 3))
    assert c == "x<=64/len~2^14"
    assert tune.workload_class(np.array([1000]), np.array([500000]), np.array([500000])) == \
        "x<=1024/len~2^19"
    assert tune.workload_class(np.array([5000]), np.array([10]), np.array([10])).startswith("x<=1073741824")


def test_lookup_uses_the_batch_class(tmp_path):
    from paper_2002_05200_amd import synth, tune
    bt = synth.random_cases(seed=1, n=20, len_lo=100, len_hi=200, x_choices=(10,))
    cls = tune.batch_class(bt)
    table = {cls: {"opts": {"waves_per_cu": 16, "long_job": 0, "long_tier_bias": 0,
                            "sort_jobs": 1, "sched": 0}}}
    assert tune.lookup(bt, table)["waves_per_cu"] == 16
    assert tune.lookup(bt, {}) is None


def test_shipped_table_is_well_formed():
    from paper_2002_05200_amd import tune
    t = tune.load_table()
    for cls, e in t.items():
        assert cls.startswith("x<=")
        assert set(e["opts"]) <= {"sched", "waves_per_cu", "sort_jobs", "long_job", "long_tier_bias",
                                  "multi_wave"}
        assert e["ms"] <= e["default_ms"]


def test_search_finds_grid_and_multi_wave_together():
    """A job-latency-bound workload: four wavefronts per job only pay off with
    a large persistent grid; one knob at a time would stop at two wavefronts."""
    from paper_2002_05200_amd import tune

    def timer(o):
        if o["long_tier_bias"] or o["sort_jobs"] == 0:
            return 3000.0
        return {0: {0: 2045.0}, 1: {0: 2126.0, 16: 1834.0, 24: 1850.0},
                2: {0: 2030.0}}[o["multi_wave"]].get(o["waves_per_cu"], 2100.0)

    res = tune.tune(None, None, timer=timer)
    assert res["opts"]["multi_wave"] == 1 and res["opts"]["waves_per_cu"] == 16
    assert res["ms"] == 1834.0 and res["default_ms"] == 2045.0
    assert res["opts"]["long_job"] == 0 and res["opts"]["sort_jobs"] == 1
