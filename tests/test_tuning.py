"""Host logic of the autotuner: workload signatures and the schedule it hands over."""
import synth
from paper_2607_21416_amd import tuning


def test_workload_key_separates_workloads_and_rounds_sizes():
    a = synth.anchor_scene(1, [1500, 800], 2, W=200, H=120, fx=140.0)
    b = synth.anchor_scene(2, [1500, 800], 2, W=200, H=120, fx=140.0)
    c = synth.anchor_scene(1, [1500, 800], 2, W=240, H=120, fx=140.0)
    d = synth.plain_scene(3, 2300, 200, 120)
    assert tuning.workload_key(a) == tuning.workload_key(b)  # same shape, other values
    assert tuning.workload_key(a) != tuning.workload_key(c)  # resolution differs
    assert tuning.workload_key(a) != tuning.workload_key(d)  # plain vs anchors


def test_schedule_and_defaults():
    assert tuning.DEFAULT["tile"] in tuning.TILES
    s = tuning.schedule(tuning.DEFAULT)
    assert set(s) == {"long_log2", "fwd_blocks_per_cu", "bwd_blocks_per_cu", "fwd_group_waves", "bwd_group_waves"}
    assert s["long_log2"] in tuning.LONG_LOG2
    assert (s["fwd_group_waves"], s["fwd_blocks_per_cu"]) == max(g for g in tuning.FWD_GRIDS if g[0] == 4)
    assert (s["bwd_group_waves"], s["bwd_blocks_per_cu"]) == max(g for g in tuning.BWD_GRIDS if g[0] == 4)
    # a choice stored before the group widths existed takes four waves
    old = {"tile": 16, "long_log2": 10, "fwd_blocks_per_cu": 3, "bwd_blocks_per_cu": 4}
    assert tuning.schedule(old)["fwd_group_waves"] == 4 and tuning.schedule(old)["bwd_group_waves"] == 4


def test_every_grid_candidate_is_a_valid_schedule():
    # the library accepts every (waves, workgroups per CU) the tuner tries, and the
    # built-in defaults
    from paper_2607_21416_amd import binding as B
    for gw, b in tuning.FWD_GRIDS:
        assert gw * b <= (20 if gw == 4 else 16)
    for gw, b in tuning.BWD_GRIDS:
        assert gw * b <= (24 if gw == 4 else 16)
    t = B.make_tuning(tuning.schedule(tuning.DEFAULT))
    assert (t.fwd_group_waves, t.bwd_group_waves, t.non_persistent, list(t.reserved)) == (4, 4, 0, [0, 0])


def test_stored_choices_are_valid_and_used():
    stored = tuning._load_stored()
    assert stored
    for key, c in stored.items():
        assert c["tile"] in tuning.TILES and c["long_log2"] in tuning.LONG_LOG2
        s = tuning.schedule(c)
        assert (s["fwd_group_waves"], s["fwd_blocks_per_cu"]) in tuning.FWD_GRIDS
        assert (s["bwd_group_waves"], s["bwd_blocks_per_cu"]) in tuning.BWD_GRIDS
    # the benchmark workloads have a stored choice, returned without measuring (no GPU here):
    # config 3's view 0 alone (the headline), config 3's four views, configs 4 and 5
    scenes = [synth.one_view(synth.config("C3"), 0)] + [synth.config(name) for name in ("C3", "C4", "C5")]
    for scene in scenes:
        assert tuning.workload_key(scene) in stored
        got = tuning.autotune(scene, device="cpu")
        assert got["source"] in ("stored", "cache") and got["tile"] == stored[tuning.workload_key(scene)]["tile"]
