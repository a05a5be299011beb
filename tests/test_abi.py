"""The C-ABI library loads and exports every entry point include/snp.h declares,
and rejects malformed systems before touching the device (no GPU needed)."""
import os
import re

import numpy as np
import pytest

import synth
from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "snp.h")


def _built_lib():
    from paper_1104_1824_amd import build, snp

    if not os.path.exists(build.library_path()):
        build.build()
    return snp


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*[A-Za-z_][\w \*]*?\b(snp_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("snp_load", "snp_free", "snp_last_error", "snp_reset", "snp_expand", "snp_run"):
        assert want in names


def test_library_exports_every_declared_symbol():
    snp = _built_lib()
    L = snp.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(snp.EXPORTED) == set(declared_functions())


def _load_status(sys_obj, **kw):
    snp = _built_lib()
    try:
        h = snp.snp_load(sys_obj, stream=0, **kw)
    except snp.SnpError as e:
        return e.status, e.message
    h.close()
    return 0, ""


def _ex(**over):
    s = synth.paper_example()
    rules = s.rules()
    syn = list(zip(s.syn_src.tolist(), s.syn_dst.tolist()))
    m = over.pop("m", s.m)
    rules = over.pop("rules", rules)
    syn = over.pop("syn", syn)
    ct = over.pop("count_type", "i32")
    return synth.make_system(m, rules, syn, [2, 1, 1][:m] + [0] * max(0, m - 3), count_type=ct)


@pytest.mark.parametrize("bad,needle", [
    (dict(syn=[(0, 1), (0, 0)]), "self-synapse"),
    (dict(syn=[(0, 1), (0, 1)]), "duplicate synapse"),
    (dict(rules=[(1, 1, 1, 1, 1), (0, 2, 1, 1, 1)]), "non-decreasing"),
    (dict(rules=[(0, 0, 1, 1, 1)]), "i must be >= 1"),
    (dict(rules=[(0, 1, -1, 1, 1)]), "j must be >= 0"),
    (dict(rules=[(0, 1, 1, 0, 1)]), "c must be >= 1"),
    (dict(rules=[(0, 1, 1, 1, -1)]), "p must be >= 0"),
    (dict(rules=[(5, 1, 1, 1, 1)]), "out of range"),
    (dict(syn=[(0, 7)]), "out of range"),
    (dict(rules=[(0, 1, 1, 1, 1)] * 17), "more than 16 rules"),
])
def test_load_rejects_malformed(bad, needle):
    st, msg = _load_status(_ex(**bad))
    assert st == 1 and needle in msg, msg


def test_load_rejects_wrong_matrix():
    import oracle

    sys_obj = synth.paper_example()
    M = oracle.matrix_dense(sys_obj).astype(np.int32)
    M[2, 0] += 1
    st, msg = _load_status(sys_obj, M=M)
    assert st == 1 and "Definition 2" in msg


def test_load_rejects_bad_options():
    st, msg = _load_status(synth.paper_example(), max_rows=0)
    assert st == 1 and "max_rows" in msg
    st, msg = _load_status(synth.paper_example(), path=7)
    assert st == 1
    st, msg = _load_status(synth.paper_example(), int8_max_k=129)
    assert st == 1 and "int8_max_k" in msg


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1104_1824_amd import snp

    monkeypatch.setattr(snp, "_lib", None)
    monkeypatch.setattr(snp, "library_path", lambda: str(tmp_path / "missing.so"))
    with pytest.raises(FileNotFoundError):
        snp.lib()


def test_stats_record_layout():
    """The binding reads level statistics through a numpy record of the same
    layout as snp_expand_stats: both views agree field by field."""
    import ctypes

    from paper_1104_1824_amd import snp

    stats = (snp.snp_expand_stats * 3)()
    for k in range(3):
        for i, (name, ct) in enumerate(snp.snp_expand_stats._fields_):
            setattr(stats[k], name, (k + 1) * 1000 + i - (7 if ct is ctypes.c_int32 else 0))
    assert snp._stats_list(stats, 3) == [stats[k].as_dict() for k in range(3)]
