"""snp_batch_run_static (the batched deterministic run that allocates nothing,
its scratch in the library's static device array) against snp_batch_run on
the same systems: every result and every final row identical, on two calls in
a row, the second with a smaller batch and fewer steps."""
import numpy as np
import pytest

import synth
from paper_1104_1824_amd import snp
from tests.gpu_helpers import from_device_rows, note

pytestmark = pytest.mark.gpu


def _c0(systems):
    import torch

    c0 = np.concatenate([np.asarray(s.c0, dtype=np.int64) for s in systems])
    if systems[0].count_type == "u16":
        return torch.from_numpy(c0.astype(np.uint16).view(np.int16)).cuda()
    return torch.from_numpy(c0.astype(np.int32)).cuda()


def _run(systems, steps, detect, static, b=None):
    import torch

    own = b is None
    if own:
        b = snp.snp_batch_load(systems)
    try:
        off = snp.snp_batch_offsets(b)
        dt = torch.int16 if systems[0].count_type == "u16" else torch.int32
        final = torch.full((int(off[-1]),), -7, dtype=dt, device="cuda")
        fn = snp.snp_batch_run_static if static else snp.snp_batch_run
        res = fn(b, _c0(systems), steps, final, detect)
        torch.cuda.synchronize()
        res["final"] = from_device_rows(systems[0], final)
        return res
    finally:
        if own:
            b.close()


def _same(a, b):
    for key in ("halt_step", "first_repeat", "steps_done", "digest", "final"):
        assert np.array_equal(a[key], b[key]), key


def test_static_matches_allocating_run(gpu):
    big = synth.batched_systems(0, 24)
    note("static scratch: 24 uneven systems x 1500 steps, after a tuned snp_batch_run")
    b = snp.snp_batch_load(big)
    try:
        want = _run(big, 1500, True, False, b)
        got = _run(big, 1500, True, True, b)
    finally:
        b.close()
    _same(got, want)
    assert (want["steps_done"] > 0).all()
    small = synth.batched_systems(40, 8)
    note("static scratch: second call, 8 systems x 700 steps, untuned batch (widest shape)")
    got2 = _run(small, 700, True, True)
    want2 = _run(small, 700, True, False)
    _same(got2, want2)
    note("static scratch: repeat detection off")
    _same(_run(small, 300, False, True), _run(small, 300, False, False))


def test_static_repeat_and_halt_cases(gpu):
    """A ring repeats at step m and a path halts at step m: the H sets in the
    static array start empty on every call."""
    rules = lambda m: [(n, 1, 1, 1, 1) for n in range(m)]
    ring = synth.make_system(20, rules(20), [(n, (n + 1) % 20) for n in range(20)], [1] + [0] * 19, name="ring20")
    path = synth.make_system(30, rules(30), [(n, n + 1) for n in range(29)], [1] + [0] * 29, name="path30")
    for k in range(2):
        note(f"static scratch: ring 20 and path 30, call {k}")
        got = _run([ring, path], 100, True, True)
        assert got["first_repeat"].tolist() == [20, -1]
        assert got["halt_step"].tolist() == [-1, 30]
        _same(got, _run([ring, path], 100, True, False))


def test_static_rejects_too_large(gpu):
    systems = synth.batched_systems(0, 256)
    note("static scratch: 256 systems x 10k steps exceed the static array")
    b = snp.snp_batch_load(systems)
    try:
        import torch

        off = snp.snp_batch_offsets(b)
        final = torch.empty(int(off[-1]), dtype=torch.int32, device="cuda")
        with pytest.raises(snp.SnpError) as e:
            snp.snp_batch_run_static(b, _c0(systems), 10000, final, True)
        assert e.value.status == snp.SNP_ERR_CAPACITY
    finally:
        b.close()
