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
    assert set(s) == {"long_log2", "fwd_blocks_per_cu", "bwd_blocks_per_cu"}
    assert s["long_log2"] in tuning.LONG_LOG2 and s["fwd_blocks_per_cu"] == max(tuning.FWD_BLOCKS)
    assert s["bwd_blocks_per_cu"] == max(tuning.BWD_BLOCKS)


def test_stored_choices_are_valid_and_used():
    stored = tuning._load_stored()
    assert stored
    for key, c in stored.items():
        assert c["tile"] in tuning.TILES and c["long_log2"] in tuning.LONG_LOG2
        assert c["fwd_blocks_per_cu"] in tuning.FWD_BLOCKS and c["bwd_blocks_per_cu"] in tuning.BWD_BLOCKS
    # the benchmark workloads have a stored choice, returned without measuring (no GPU here)
    for name in ("C3", "C4"):
        scene = synth.config(name)
        assert tuning.workload_key(scene) in stored
        got = tuning.autotune(scene, device="cpu")
        assert got["source"] in ("stored", "cache") and got["tile"] == stored[tuning.workload_key(scene)]["tile"]
