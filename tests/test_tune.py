"""Host logic of the batched autotuner (no GPU: a synthetic cost stands in
for the timed steps)."""
import pytest

from paper_2301_06984_amd.tune import coordinate_descent


def separable(cfg):
    # best at cell_factor 1.25, block 512, sort_every 5, walk_chunk 4
    return (abs(cfg["cell_factor"] - 1.25) * 10 + abs(cfg["block_size"] - 512) / 128
            + abs(cfg["sort_every"] - 5) + abs(cfg["walk_chunk"] - 4) + 1.0)


def test_finds_separable_optimum_and_caches():
    calls = []
    res = coordinate_descent(lambda c: calls.append(dict(c)) or separable(c),
                             cell_factors=(1.0, 1.25, 1.5), block_sizes=(128, 256, 512), sort_every=(1, 2, 5, 10))
    assert res.params == dict(cell_factor=1.25, block_size=512, sort_every=5, walk_chunk=4)
    assert res.ms_per_step == pytest.approx(1.0)
    keys = [(c["cell_factor"], c["block_size"], c["sort_every"], c["walk_chunk"]) for c in calls]
    assert len(keys) == len(set(keys)) == len(res.trials)   # no configuration timed twice
    assert len(calls) <= 1 + 4 + 3 + 2 + 3


def test_graph_steps_restrict_cadence():
    res = coordinate_descent(lambda c: c["sort_every"], sort_every=(1, 2, 3, 4, 5), graph_steps=10,
                             cell_factors=(1.0,), block_sizes=(256,))
    assert {c["sort_every"] for c, _ in res.trials} == {1, 5}   # 10 / k whole and even
    assert res.params["sort_every"] == 1


def test_starts_from_defaults_and_keeps_them_when_best():
    res = coordinate_descent(lambda c: 0.0 if (c["block_size"], c["sort_every"], c["cell_factor"], c["walk_chunk"])
                             == (256, 1, 1.0, 2) else 1.0)
    assert res.params == dict(cell_factor=1.0, block_size=256, sort_every=1, walk_chunk=2)
    assert res.trials[0][0] == res.params


def test_rejects_empty_candidates():
    with pytest.raises(ValueError):
        coordinate_descent(lambda c: 1.0, sort_every=(3,), graph_steps=10)
