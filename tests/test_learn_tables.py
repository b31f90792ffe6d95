"""CPU checks of the cost model's bookkeeping: the exploration tables force
every dispatch option, each timing row is labelled with the option its table
forced, and the training set marks exactly one option per row."""

import numpy as np

from paper_2006_11494_amd import aot, learn


def test_exploration_tables_cover_every_option_once():
    light, heavy = set(), set()
    for i in range(learn.N_EXPLORE):
        t = learn.exploration_table(i)
        assert len(t) == aot.AOT_NUM_BUCKETS
        tiles = {t[k] >> 8 for k in range(8)}
        arms = {t[16 + h] for h in range(16)}
        assert tiles == {learn.TILES[i]} and all(t[k] & 0xff == 0 for k in range(8))
        assert len(arms) == 1
        # the row label names what the table forced
        assert learn.TILES[learn.option_of(0, i)] == learn.TILES[i]
        assert learn.ARMS[learn.option_of(16, i) - 5] == arms.pop()
        light.add(learn.option_of(3, i))
        heavy.add(learn.option_of(20, i))
    assert light == set(range(5))
    assert heavy == set(range(5, aot.AOT_NUM_OPTIONS))


def test_plain_table_is_the_plain_rule():
    t = learn.plain_table()
    assert [t[k] >> 8 for k in range(8)] == [4, 4, 4, 8, 16, 32, 64, 64]
    assert all(t[16 + h] == 0 for h in range(16))      # bitmap for every heavy class


def test_dataset_marks_one_option_per_row():
    rng = np.random.default_rng(3)
    rows = [(rng.random(aot.AOT_NUM_FEATURES).astype(np.float32), int(rng.integers(0, 9)),
             float(rng.normal())) for _ in range(50)]
    d = learn.dataset(rows, device="cpu")
    assert d.x.shape == (50, aot.AOT_NUM_FEATURES)
    m = d.mask.numpy()
    assert np.all(m.sum(1) == 1)
    for i, (_, opt, y) in enumerate(rows):
        assert m[i, opt] == 1 and np.isclose(d.target[i, opt].item(), y)
