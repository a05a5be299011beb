"""The oracle-written golden digests of the full-size workloads agree with the
oracle where it is cheap to recompute them (no GPU): the first blocks of the
dense walk and a sample of the batched systems."""
import numpy as np
import pytest

import synth
from tests.golden import make_golden


@pytest.mark.parametrize("seed", make_golden.DENSE_SEEDS)
def test_dense_walk_file_shape(seed):
    head, data = make_golden.read_table(make_golden.dense_file(seed))
    levels = [int(x) for x in head["levels"].split()]
    assert levels == [1, 1000000, 1000000, 1000000]
    assert int(head["block_rows"]) == make_golden.BLOCK
    assert len(data) == (sum(levels) + make_golden.BLOCK - 1) // make_golden.BLOCK
    assert [int(x[0]) for x in data] == list(range(len(data)))
    assert all(len(x[1]) == make_golden.HEX and len(x[2]) == make_golden.HEX for x in data)


@pytest.mark.parametrize("seed", make_golden.DENSE_SEEDS)
def test_dense_walk_first_blocks(oracle_mod, seed):
    """Blocks 0-3 cover C0 and the first 4095 rows of level 1, which a walk
    capped at 4095 new configurations per level reproduces."""
    _, data = make_golden.read_table(make_golden.dense_file(seed))
    s = synth.config_system(3, seed)
    w = oracle_mod.bfs(s, max_depth=1, frontier_cap=4 * make_golden.BLOCK - 1, rows_cap=4 * make_golden.BLOCK)
    got = make_golden.block_digests(w.rows, w.parent, w.tindex)
    assert [list(g) for g in got] == [x[1:] for x in data[:4]]


def test_batched_file_sample(oracle_mod):
    _, data = make_golden.read_table(make_golden.BATCH_FILE)
    assert [int(x[0]) for x in data] == list(range(256))
    systems = synth.batched_systems(0, 256)
    small = sorted(range(256), key=lambda k: systems[k].m)[:4]
    for k in small:
        d = oracle_mod.deterministic(systems[k], 10000)
        fin = make_golden.sha(np.ascontiguousarray(d.final.astype("<i4")).tobytes())
        assert data[k][1:] == [str(systems[k].m), fin, str(d.halt_step), str(d.first_repeat), str(d.steps_done),
                               str(d.digest)]
