"""The allocation-free batched count (sk_count_batch_noalloc) against
sk_count_batch, through the C ABI: two calls in a row on the library's fixed
per-device workspace, the second with fewer and smaller instances (the fixed
workspace keeps the first call's contents, which the second must clear)."""
import ctypes
import sys

import pytest

import paper_1507_00315_amd as sk

pytestmark = pytest.mark.gpu


def _run(fn, inst):
    L = sk.lib()
    arr = sk._instances(inst)
    out = (sk.U128 * len(inst))()
    st = sk.Stats()
    if fn == "noalloc":
        status = L.sk_count_batch_noalloc(arr, len(inst), None, None, ctypes.byref(st), out)
    else:
        status = L.sk_count_batch(arr, len(inst), None, None, 0, None, ctypes.byref(st), out)
    assert status == 0, (fn, status, L.sk_last_error())
    return [o.value() for o in out], st


def test_noalloc_batch_equals_batch_twice():
    first = [(16, "skolem"), (17, "skolem"), (15, "langford"), (16, "langford"), (14, "hooked", sk.ORDERED),
             (15, "hooked", sk.ORDERED), (13, "skolem"), (12, "langford", sk.NO_SHORTCUT)]
    second = [(15, "langford"), (12, "skolem")]
    for inst in (first, second):
        print("noalloc batch of", len(inst), "instances", file=sys.stderr, flush=True)
        want, _ = _run("batch", inst)
        got, st = _run("noalloc", inst)
        assert got == want
        assert st.terms > 0 and st.launches >= 1
    assert want == [39809640, 227968]


def test_noalloc_rejects_bad_input():
    L = sk.lib()
    out = (sk.U128 * 1)()
    assert L.sk_count_batch_noalloc(sk._instances([(40, "skolem")]), 1, None, None, None, out) == -1
    assert L.sk_count_batch_noalloc(None, 1, None, None, None, out) == -1
