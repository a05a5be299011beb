"""Per-pass choice of form under SNP_PATH_AUTO: a level whose parents have
many canonical children runs on the int8 matrix cores, one whose parents have
few runs the sparse pull, inside one walk; results equal the oracle's and the
forced forms'."""
import numpy as np
import pytest

import synth
from paper_1104_1824_amd import snp
from tests.gpu_helpers import assert_same_bfs, gpu_bfs, note

pytestmark = pytest.mark.gpu


def ring_choice(m=100, every=10, seed=3):
    """A ring of m neurons (out-degree 1, so no one-neuron-per-lane form above
    64 neurons), one rule per neuron plus a second, different one on every
    `every`-th: C0 has 2^(number of those holding 2 or more) children, later
    configurations about 3 each."""
    rules = []
    for n in range(m):
        rules.append((n, 1, 1, 1, 1))
        if n % every == 0:
            rules.append((n, 2, 1, 2, 1))
    syn = [(n, (n + 1) % m) for n in range(m)]
    rng = np.random.default_rng(seed)
    return synth.make_system(m, rules, syn, [int(x) for x in rng.integers(0, 3, size=m)], name="ring_choice")


def test_auto_switches_form_between_levels(gpu, oracle_mod):
    s = ring_choice()
    want = oracle_mod.bfs(s, max_depth=12)
    note("ring with choices: AUTO, INT8, SPARSE against the oracle")
    g = gpu_bfs(s, max_depth=12, out_capacity=4096, path=snp.SNP_PATH_AUTO)
    assert_same_bfs(g, want)
    st = g["level_stats"][: len(want.level_sizes) - 1]
    # C0's level: no ratio known yet (dense assumed) -> int8; its 16 canonical
    # children per parent -> int8 again; then about 3.4 per parent -> sparse
    assert st[0]["int8_chunks"] == st[0]["chunks"] and st[1]["int8_chunks"] == st[1]["chunks"]
    assert all(x["int8_chunks"] == 0 and x["path_used"] == snp.SNP_PATH_SPARSE for x in st[2:])
    for path in (snp.SNP_PATH_INT8, snp.SNP_PATH_SPARSE):
        g2 = gpu_bfs(s, max_depth=12, out_capacity=4096, path=path)
        assert_same_bfs(g2, want)
        n8 = sum(x["int8_chunks"] for x in g2["level_stats"])
        assert (n8 > 0) == (path == snp.SNP_PATH_INT8)


@pytest.mark.parametrize("chunk", [16, 37, 4096])
def test_auto_chunk_invariance(gpu, oracle_mod, chunk):
    """Passes of different sizes (the form chosen per pass) give the same walk."""
    s = ring_choice(m=120, every=6, seed=9)
    want = oracle_mod.bfs(s, max_depth=10, frontier_cap=300)
    note(f"ring with choices, AUTO, chunk {chunk}")
    g = gpu_bfs(s, max_depth=10, frontier_cap=300, out_capacity=8192, chunk=chunk, path=snp.SNP_PATH_AUTO)
    assert_same_bfs(g, want)
