"""The paper's input files (Section 3.1: row-major M, C; Section 4: the rule
file) and the run trace of Section 5, on the CPU: the example's files rebuild
the example system, writing and reading a system gives it back, and the trace
of the oracle's run of the example shows the snapshots and the final allGenCk
the paper prints."""
import numpy as np
import pytest

import oracle
import synth
from paper_1104_1824_amd import paper_io
from tests.conftest import read_golden

C_TEXT = "2 1 1\n"
R_TEXT = "2 2 $ 1 $ 1 2\n"


def m_text():
    ln = [x for x in read_golden("paper_matrix.txt") if x.startswith("row-major:")][0]
    return ln.split(":", 1)[1]


def test_example_files_rebuild_the_example():
    s = paper_io.read_paper_inputs(C_TEXT, m_text(), R_TEXT)
    ex = synth.paper_example()
    assert s.m == 3 and s.c0.tolist() == [2, 1, 1]
    assert s.rule_neuron.tolist() == ex.rule_neuron.tolist()
    assert s.rule_i.tolist() == [2, 2, 1, 1, 2] == ex.rule_i.tolist()
    assert s.rule_j.tolist() == ex.rule_j.tolist() == [1] * 5
    assert s.rule_c.tolist() == ex.rule_c.tolist()
    # rules 4 and 5 belong to the output neuron, which has no synapse: M says nothing of p
    assert s.rule_p.tolist()[:3] == ex.rule_p.tolist()[:3] and s.rule_p.tolist()[3:] == [0, 0]
    assert sorted(zip(s.syn_src.tolist(), s.syn_dst.tolist())) == sorted(zip(ex.syn_src.tolist(),
                                                                              ex.syn_dst.tolist()))
    golden_M = [[int(x) for x in ln.split()] for ln in read_golden("paper_matrix.txt") if ":" not in ln]
    assert paper_io.transition_matrix(s).tolist() == golden_M == oracle.matrix_dense(ex).tolist()
    exact = paper_io.read_paper_inputs(C_TEXT, m_text(), R_TEXT, exact=True)
    assert exact.rule_j.tolist() == [0] * 5


@pytest.mark.parametrize("seed", range(8))
def test_write_then_read_round_trip(seed):
    rng = np.random.default_rng(seed)
    m = int(rng.integers(2, 9))
    rules = []
    for n in range(m):
        for _ in range(int(rng.integers(1, 4))):
            i = int(rng.integers(1, 5))
            rules.append((n, i, 1, int(rng.integers(1, i + 1)), int(rng.integers(0, 3))))
    syn = [(s, d) for s in range(m) for d in range(m) if s != d and rng.random() < 0.4]
    sysm = synth.make_system(m, rules, syn, rng.integers(0, 5, size=m).tolist())
    back = paper_io.read_paper_inputs(*paper_io.write_paper_inputs(sysm))
    assert paper_io.transition_matrix(back).tolist() == oracle.matrix_dense(sysm).tolist()
    assert back.rule_i.tolist() == sysm.rule_i.tolist() and back.rule_c.tolist() == sysm.rule_c.tolist()
    assert back.c0.tolist() == sysm.c0.tolist()
    # the walks agree: the matrix is all the dynamics needs
    a, b = oracle.bfs(sysm, max_depth=4), oracle.bfs(back, max_depth=4)
    assert a.level_sizes.tolist() == b.level_sizes.tolist() and np.array_equal(a.rows, b.rows)


@pytest.mark.parametrize("c,m,r,needle", [
    ("2 1", "-1 1 1 -2 1 1 1 -1 1 0 0 -1 0 0 -2", R_TEXT, "neurons"),
    (C_TEXT, "-1 1 1 -2 1 1 1 -1 1 0 0 -1 0 0", R_TEXT, "entries"),
    (C_TEXT, "-1 1 1 -2 1 1 1 -1 1 0 0 -1 0 0 -2", "2 x $ 1 $ 1 2", "token"),
    (C_TEXT, "-1 1 2 -2 1 1 1 -1 1 0 0 -1 0 0 -2", R_TEXT, "productions"),
    (C_TEXT, "-1 1 0 -2 1 1 1 -1 1 0 0 -1 0 0 -2", R_TEXT, "another rule"),
    (C_TEXT, "1 1 1 -2 1 1 1 -1 1 0 0 -1 0 0 -2", R_TEXT, "own neuron"),
    (C_TEXT, "-1 1 1 -2 1 1 1 -1 1 0 0 -1 0 0 -2", "2 0 $ 1 $ 1 2", "below 1"),
])
def test_malformed_inputs_are_rejected(c, m, r, needle):
    with pytest.raises(ValueError, match=needle):
        paper_io.read_paper_inputs(c, m, r)


def test_trace_of_the_example_run():
    s = paper_io.read_paper_inputs(C_TEXT, m_text(), R_TEXT)
    res = oracle.bfs(s, expand_max_count=9)
    text = paper_io.format_trace(s, res.rows, res.parent, expand_max_count=9)
    lines = text.splitlines()
    trace = {ln.split(":", 1)[0]: ln.split(":", 1)[1].strip() for ln in read_golden("paper_trace.txt") if ":" in ln}
    assert f" tmpList =  {trace['tmp2']} " in lines
    assert f" [{trace['tmp3']}] " in lines
    assert f"{trace['rules']!s}".replace(" ", "") == "2 2 $ 1 $ 1 2".replace(" ", "")
    assert "['2', '2', '$', '1', '$', '1', '2'] " in lines
    assert "Initial configuration vector: 211" in lines
    # snapshots after C0, after confVec 212 and after confVec 112, in that order
    snaps = [i for i, ln in enumerate(lines) if ln == "All generated Cks are allGenCk ="]
    assert lines[snaps[0] + 1].strip() == trace["after_211"]
    assert lines[snaps[1] - 1].strip() == "Current confVec: 212" and lines[snaps[1] + 1].strip() == trace["after_212"]
    assert lines[snaps[2] - 1].strip() == "Current confVec: 112" and lines[snaps[2] + 1].strip() == trace["after_112"]
    # the deepest expanded configuration is 1-0-9, and the final list is the printed one
    confs = [ln.split(":")[1].strip() for ln in lines if ln.startswith("Current confVec:")]
    assert confs[-1] == "109"
    final = [x for x in read_golden("paper_allgenck.txt")]
    assert lines[snaps[-1] + 1].strip() == str(final)
    assert lines[-2] == "No more Cks to use (infinite loop/s otherwise). Stop."
