"""The paper's input files run on the GPU through the command line of
paper_io: the trace printed from the GPU walk is the one built from the
oracle's walk, line for line (Section 5's run of the example, and a random
system written to files)."""
import os
import subprocess
import sys

import numpy as np
import pytest

import synth
from paper_1104_1824_amd import paper_io
from tests.gpu_helpers import note
from tests.test_paper_io import C_TEXT, R_TEXT, m_text

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_cli(tmp_path, c, m, r, *extra):
    paths = []
    for name, text in (("C", c), ("M", m), ("r", r)):
        p = tmp_path / name
        p.write_text(text)
        paths.append(str(p))
    res = subprocess.run([sys.executable, "-m", "paper_1104_1824_amd.paper_io", *paths, *extra],
                         capture_output=True, text=True, timeout=240, cwd=ROOT)
    assert res.returncode == 0, res.stderr[-2000:]
    return res.stdout


def test_example_trace_on_gpu(gpu, oracle_mod, tmp_path):
    note("paper_io command line: the example with the count filter 9")
    out = run_cli(tmp_path, C_TEXT, m_text(), R_TEXT, "--expand-max-count", "9")
    s = paper_io.read_paper_inputs(C_TEXT, m_text(), R_TEXT)
    res = oracle_mod.bfs(s, expand_max_count=9)
    assert out == paper_io.format_trace(s, res.rows, res.parent, expand_max_count=9)
    assert "Current confVec: 109 " in out.splitlines()


def test_random_system_files_on_gpu(gpu, oracle_mod, tmp_path):
    rng = np.random.default_rng(11)
    m = 6
    rules = [(n, int(rng.integers(1, 4)), 1, 1, int(rng.integers(0, 2))) for n in range(m) for _ in range(2)]
    syn = [(s, (s + 1) % m) for s in range(m)] + [(s, (s + 3) % m) for s in range(m)]
    sysm = synth.make_system(m, rules, syn, rng.integers(0, 4, size=m).tolist())
    c, mt, r = paper_io.write_paper_inputs(sysm)
    note("paper_io command line: a random system, depth 6")
    out = run_cli(tmp_path, c, mt, r, "--max-depth", "6")
    back = paper_io.read_paper_inputs(c, mt, r)
    res = oracle_mod.bfs(back, max_depth=6)
    assert res.stop_reason == 2
    assert out == paper_io.format_trace(back, res.rows, res.parent, stop_note=paper_io.stop_note(res.stop_reason))
    assert out.splitlines()[-2] == "Depth limit reached. Stop."
