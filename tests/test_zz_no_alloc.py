"""lcemd_topl_noalloc (the entry point for callers that cannot allocate)
against lcemd_topl, both through the C ABI on the same device inputs: the
same candidate lists bit for bit, on two calls in a row with the second one
smaller (the scratch region keeps the first call's contents), for float32 and
bfloat16 phase 1.  The calls leave the device's free memory unchanged."""
import sys

import numpy as np
import pytest

from synth import make_workload

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1812_02091_amd import lcemd

    lcemd.load_library()
    w = make_workload("text", n=3000, B=12, v=6000)
    say("[gpu] no-alloc: text-shaped workload v=6000 m=300 n=3000 B=12")
    ctx = lcemd.open_context(w.V, w.db.rowptr, w.db.col, w.db.val, precisions=("bf16",))
    return lcemd, torch, w, ctx


def _dev(torch, csr):
    d = torch.device("cuda:0")
    return (torch.from_numpy(np.ascontiguousarray(csr.rowptr)).to(d),
            torch.from_numpy(np.ascontiguousarray(csr.col)).to(d),
            torch.from_numpy(np.ascontiguousarray(csr.val)).to(d))


def _empty(torch, B, l):
    return (torch.full((B, l), -7, dtype=torch.int64, device="cuda:0"),
            torch.full((B, l), -7.0, dtype=torch.float32, device="cuda:0"))


@pytest.mark.parametrize("method,k,prec", [("act", 8, "fp32"), ("act", 8, "bf16"), ("rwmd", 1, "fp32"),
                                           ("act", 3, "bf16")])
def test_noalloc_matches_topl_on_two_calls(env, method, k, prec):
    L, torch, w, ctx = env
    calls = [(w.queries, 16), (w.queries.take(np.arange(3, 8)), 5)]
    for i, (qs, l) in enumerate(calls):
        say(f"[gpu] no-alloc call {i}: {method} k={k} {prec} B={qs.n} l={l}")
        q = _dev(torch, qs)
        ref = ctx.topl(*q, l, method=method, k=k, direction="d2q", precision=prec)
        out = _empty(torch, qs.n, l)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        ctx.topl_noalloc(*q, l, out, method=method, k=k, precision=prec)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        assert torch.equal(out[0], ref[0]), f"call {i}: indices differ"
        assert torch.equal(out[1], ref[1]), f"call {i}: distances differ"
        assert free1 == free0, f"call {i}: device free memory moved by {free0 - free1} bytes"


def test_noalloc_exclude_self(env):
    """The same with a query batch that is the database's own rows 100..107
    and exclude_self = 100 (each query leaves itself out)."""
    L, torch, w, ctx = env
    rows = w.db.take(np.arange(100, 108))
    q = _dev(torch, rows)
    ref = ctx.topl(*q, 10, method="act", k=4, direction="d2q", exclude_self=100)
    out = _empty(torch, rows.n, 10)
    ctx.topl_noalloc(*q, 10, out, method="act", k=4, exclude_self=100)
    torch.cuda.synchronize()
    assert torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1])
    assert not any(int(out[0][b].eq(100 + b).any()) for b in range(rows.n))


def test_noalloc_refuses_what_it_cannot_hold(env):
    """Limits are checked before any work: host pointers and more than 4096
    queries give clear errors, and the context stays usable."""
    L, torch, w, ctx = env
    q = _dev(torch, w.queries)
    out = _empty(torch, w.queries.n, 4)
    with pytest.raises(L.LcemdError) as e:
        ctx.topl_noalloc(w.queries.rowptr, w.queries.col, w.queries.val, 4, out)
    assert e.value.code == L.E_INVALID_ARG
    many = w.db.take(np.arange(4200) % 3000)
    qm = _dev(torch, many)
    om = _empty(torch, many.n, 4)
    with pytest.raises(L.LcemdError) as e:
        ctx.topl_noalloc(*qm, 4, om)
    assert e.value.code == L.E_CAPACITY
    # the context still answers, bit for bit as before
    ref = ctx.topl(*q, 4, method="act", k=2, direction="d2q")
    ctx.topl_noalloc(*q, 4, out, method="act", k=2)
    torch.cuda.synchronize()
    assert torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1])
