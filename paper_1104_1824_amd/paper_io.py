"""The paper's simulator inputs and its run trace.

Inputs (Section 3.1, Section 4): three text files of blank-separated values,
``C`` (the initial configuration, one count per neuron), ``M`` (the spiking
transition matrix in row-major order, one row per rule) and ``r`` (one
regular-expression exponent per rule, neurons separated by ``$``).  A system
is rebuilt from them: rule ``k`` of neuron ``s`` consumes ``c = -M[k][s]`` and
sends ``p`` = the common positive entry of its row to every neuron where that
entry sits (Definition 2); the synapses of ``s`` are the neurons any of its
rules sends to (a neuron whose rules send nothing has no synapse that matters
to the matrix).  The exponent ``k`` reads as ``E = a^k a*`` ("at least k
spikes": the reading under which the printed run of Section 5 is reproduced)
or, with ``exact=True``, as ``E = a^k``.

Trace (Section 5): the lines the paper's simulator prints for a run, with
configurations as dash-joined counts ('2-1-1'), the current configuration as
concatenated digits ('212'), and after each expanded configuration the list
``allGenCk`` of every configuration produced so far, in the order produced.
``format_trace`` builds those lines from a run's rows and parents (the
breadth-first order of the library is the order of the paper's queue).

Command line: ``python -m paper_1104_1824_amd.paper_io C M r`` runs the walk
on the GPU through the C ABI and prints the trace.
"""
from __future__ import annotations

import argparse
import sys
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np


@dataclass
class PaperSystem:
    """A system in the attribute layout the binding reads (snp.snp_load)."""
    m: int
    rule_neuron: np.ndarray
    rule_i: np.ndarray
    rule_j: np.ndarray
    rule_c: np.ndarray
    rule_p: np.ndarray
    syn_src: np.ndarray
    syn_dst: np.ndarray
    c0: np.ndarray
    count_type: str = "i32"
    name: str = "paper_files"
    rule_file: List[str] = field(default_factory=list)  # the r file's tokens, '$' included
    matrix: Optional[np.ndarray] = None                 # M as read, r x m

    @property
    def count_max(self) -> int:
        return 65535 if self.count_type == "u16" else 2**31 - 1


def _ints(text: str, what: str) -> List[int]:
    try:
        return [int(x) for x in text.replace(",", " ").split()]
    except ValueError as e:
        raise ValueError(f"{what}: not a list of integers ({e})") from None


def read_paper_inputs(c_text: str, m_text: str, r_text: str, exact: bool = False) -> PaperSystem:
    """Rebuild a system from the contents of the C, M and r files."""
    c0 = _ints(c_text, "C")
    m = len(c0)
    if m < 1:
        raise ValueError("C: no neuron")
    if any(x < 0 for x in c0):
        raise ValueError("C: negative count")
    tokens = r_text.split()
    exps, owner, n = [], [], 0
    for tok in tokens:
        if tok == "$":
            n += 1
            continue
        try:
            k = int(tok)
        except ValueError:
            raise ValueError(f"r: token {tok!r} is neither an exponent nor '$'") from None
        if k < 1:
            raise ValueError(f"r: exponent {k} below 1")
        exps.append(k)
        owner.append(n)
    if n + 1 != m:
        raise ValueError(f"r: {n + 1} neurons ('$'-separated groups), C has {m}")
    r = len(exps)
    vals = _ints(m_text, "M")
    if len(vals) != r * m:
        raise ValueError(f"M: {len(vals)} entries, expected r x m = {r} x {m}")
    M = np.asarray(vals, dtype=np.int64).reshape(r, m)
    rc, rp, targets = [], [], [set() for _ in range(m)]
    for k in range(r):
        s = owner[k]
        if M[k, s] >= 0:
            raise ValueError(f"M row {k + 1}: entry of its own neuron {s + 1} is {M[k, s]}, must be -c < 0")
        others = [d for d in range(m) if d != s]
        if any(M[k, d] < 0 for d in others):
            raise ValueError(f"M row {k + 1}: negative entry outside neuron {s + 1}")
        pos = {int(M[k, d]) for d in others if M[k, d] > 0}
        if len(pos) > 1:
            raise ValueError(f"M row {k + 1}: different productions {sorted(pos)} (Definition 2 sends one p)")
        p = pos.pop() if pos else 0
        if p:
            t = {d for d in others if M[k, d] > 0}
            if targets[s] and t != targets[s]:
                raise ValueError(f"M row {k + 1}: sends to {sorted(x + 1 for x in t)}, another rule of neuron "
                                 f"{s + 1} to {sorted(x + 1 for x in targets[s])}")
            targets[s] = t
        rc.append(int(-M[k, s]))
        rp.append(int(p))
    syn = [(s, d) for s in range(m) for d in sorted(targets[s])]
    i32 = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.int32))
    return PaperSystem(
        m=m, rule_neuron=i32(owner), rule_i=i32(exps), rule_j=i32([0 if exact else 1] * r), rule_c=i32(rc),
        rule_p=i32(rp), syn_src=i32([s for s, _ in syn]), syn_dst=i32([d for _, d in syn]),
        c0=np.asarray(c0, dtype=np.int64), rule_file=tokens, matrix=M)


def read_paper_files(c_path: str, m_path: str, r_path: str, exact: bool = False) -> PaperSystem:
    with open(c_path) as fc, open(m_path) as fm, open(r_path) as fr:
        return read_paper_inputs(fc.read(), fm.read(), fr.read(), exact=exact)


def transition_matrix(system) -> np.ndarray:
    """M of Definition 2 for a system (rows = rules, columns = neurons)."""
    m, r = int(system.m), len(system.rule_neuron)
    M = np.zeros((r, m), dtype=np.int64)
    for k in range(r):
        s = int(system.rule_neuron[k])
        M[k, s] = -int(system.rule_c[k])
        for e in range(len(system.syn_src)):
            if int(system.syn_src[e]) == s:
                M[k, int(system.syn_dst[e])] = int(system.rule_p[k])
    return M


def write_paper_inputs(system) -> tuple:
    """The C, M and r file contents of a system whose rules have E = a^i (a^j)*
    with one j for all (0: exact, 1: at least); the exponents are the i."""
    js = {int(x) for x in system.rule_j}
    if not js <= {0, 1} or len(js) > 1:
        raise ValueError("the r file holds one exponent per rule: every rule needs j = 0, or every rule j = 1")
    c_text = " ".join(str(int(x)) for x in system.c0) + "\n"
    m_text = " ".join(str(int(x)) for x in transition_matrix(system).reshape(-1)) + "\n"
    groups = [[] for _ in range(int(system.m))]
    for k in range(len(system.rule_neuron)):
        groups[int(system.rule_neuron[k])].append(str(int(system.rule_i[k])))
    r_text = " $ ".join(" ".join(g) for g in groups) + "\n"
    return c_text, m_text, r_text


def conf_dashes(row: Sequence[int]) -> str:
    return "-".join(str(int(x)) for x in row)


def conf_digits(row: Sequence[int]) -> str:
    return "".join(str(int(x)) for x in row)


def _applies(n: int, i: int, j: int, c: int) -> bool:
    if n < i or n < c:
        return False
    return n == i if j == 0 else (n - i) % j == 0


def spiking_lists(system, row: Sequence[int]):
    """Per neuron, the one-hot strings of its applicable rules over its own
    rules (the neuron's choices), and their concatenations in Algorithm 2's
    order (first neuron most significant): the trace's tmpList and
    allValidSpikVec for a configuration."""
    per = [[] for _ in range(int(system.m))]
    for k in range(len(system.rule_neuron)):
        per[int(system.rule_neuron[k])].append(k)
    lists = []
    for n, ks in enumerate(per):
        if not ks:
            continue
        ok = [_applies(int(row[n]), int(system.rule_i[k]), int(system.rule_j[k]), int(system.rule_c[k])) for k in ks]
        if any(ok):
            lists.append(["".join("1" if q == a else "0" for q in range(len(ks))) for a in range(len(ks)) if ok[a]])
        else:
            lists.append(["0" * len(ks)])
    vectors = [""]
    for choices in lists:
        vectors = [v + c for v in vectors for c in choices]
    return lists, vectors


def format_trace(system, rows, parent, expand_max_count: int = -1, stop_note: Optional[str] = None) -> str:
    """The run trace of Section 5 for a walk's rows (first row C0) and the
    index of every row's parent (-1 for C0).  A configuration is listed as
    expanded ('Current confVec') unless it holds more spikes than
    expand_max_count in some neuron (the walk then records it without
    expanding it)."""
    rows = np.asarray(rows, dtype=np.int64)
    parent = np.asarray(parent, dtype=np.int64)
    n = rows.shape[0]
    out = ["****SN P system simulation run STARTS here****", "Spiking transition Matrix: "]
    M = transition_matrix(system)
    out += [" ".join(str(int(x)) for x in row) for row in M]
    tokens = list(getattr(system, "rule_file", []) or [])
    if not tokens:
        tokens = write_paper_inputs(system)[2].split()
    out += ["", "Rules of the form a^n/a^m -> a or a^n ->a loaded: ", str(tokens) + " ", ""]
    out += [f"Initial configuration vector: {conf_digits(rows[0])}", " ",
            f"Number of neurons for the SN P system is {int(system.m)} "]
    lists, vectors = spiking_lists(system, rows[0])
    out += [f" tmpList =  {lists} ", " All valid spiking vectors: allValidSpikVec =", f" [{vectors}] "]
    # rows produced while expanding row q: those whose parent is q
    last_child = np.full(n, -1, dtype=np.int64)
    for x in range(1, n):
        last_child[parent[x]] = x
    upto = 1
    listed = lambda k: [conf_dashes(rows[x]) for x in range(k)]
    upto = max(upto, int(last_child[0]) + 1)
    out += ["All generated Cks are allGenCk =", f"{listed(upto)} ", " End of C0 ", "** ", "** ", "** ",
            " initial total Ck list is", f"   {listed(upto)} "]
    for q in range(1, n):
        if expand_max_count >= 0 and int(rows[q].max()) > expand_max_count:
            continue
        upto = max(upto, int(last_child[q]) + 1)
        out += [f"Current confVec: {conf_digits(rows[q])} ", "All generated Cks are allGenCk =", f"{listed(upto)} ",
                "** ", "** ", "** "]
    out += ["", stop_note or "No more Cks to use (infinite loop/s otherwise). Stop.",
            "****SN P system simulation run ENDS here****"]
    return "\n".join(out) + "\n"


def stop_note(stop_reason: int) -> Optional[str]:
    """The trace's closing line for a run's stop reason (snp_stop): the paper's
    for an empty frontier (its second criterion), ours for the others."""
    return {1: "No rule applies anywhere. Stop.", 2: "Depth limit reached. Stop.",
            3: "Frontier cap reached. Stop.", 4: "Child budget reached. Stop."}.get(int(stop_reason))


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description="Run the paper's simulator inputs on the GPU and print the trace.")
    ap.add_argument("C")
    ap.add_argument("M")
    ap.add_argument("r")
    ap.add_argument("--exact", action="store_true", help="read an exponent k as E = a^k (default: a^k a*)")
    ap.add_argument("--expand-max-count", type=int, default=-1,
                    help="record but do not expand configurations holding more spikes than this in a neuron")
    ap.add_argument("--max-depth", type=int, default=-1)
    ap.add_argument("--max-rows", type=int, default=1 << 16)
    args = ap.parse_args(argv)
    import torch

    from paper_1104_1824_amd import snp

    s = read_paper_files(args.C, args.M, args.r, exact=args.exact)
    h = snp.snp_load(s, path=snp.SNP_PATH_SPARSE, max_rows=args.max_rows, expand_max_count=args.expand_max_count)
    try:
        c0 = torch.tensor(s.c0, dtype=torch.int32, device="cuda")
        out = torch.empty((args.max_rows, s.m), dtype=torch.int32, device="cuda")
        par = torch.empty(args.max_rows, dtype=torch.int64, device="cuda")
        res = snp.snp_run(h, c0, args.max_depth, out, args.max_rows, parent_of=par)
    finally:
        h.close()
    n = res["n_configs"]
    sys.stdout.write(format_trace(s, out[:n].cpu().numpy(), par[:n].cpu().numpy(), args.expand_max_count,
                                  stop_note(res["stop_reason"])))
    return 0


if __name__ == "__main__":
    sys.exit(main())
