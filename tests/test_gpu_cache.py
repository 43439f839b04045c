"""Device memory cache and stream moves of the C ABI (library bookkeeping,
not part of the method).  That setups on reused blocks give the bits of
setups on fresh memory is checked with the parity tests; here: the byte
limit holds, pinned host blocks are cached under their own key, and moving
a handle to another stream waits for the work queued on the old one."""
import sys

import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2306_10025_amd as pr  # noqa: E402

DEV = torch.device("cuda:0")
KW = dict(algo="tolerance", eps=1e-8, precision="bf16x3", deterministic=True)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _solve_once(P):
    h = pr.PatchRelax(P.A, P.ptr, P.dofs, **KW)
    b = torch.as_tensor(gen.rhs(P.n, 1)).to(DEV)
    x = torch.zeros_like(b)
    h.solve(b, x, 1e-8)
    torch.cuda.synchronize()
    it = h.solve_info()["iters"]
    h.close()
    return it


def test_cache_limit_holds_and_host_blocks_are_kept():
    P = gen.q1_poisson_2d(48)
    try:
        pr.pr_release_cached_memory()
        pr.pr_set_memory_cache_limit(1 << 20)
        it_small = _solve_once(P)
        dev, host = pr.pr_memory_cache_info(0), pr.pr_memory_cache_info(-1)
        say("limit 1 MiB", dev, host)
        assert dev["idle_bytes"] <= 1 << 20
        assert host["idle_blocks"] >= 1 and host["idle_bytes"] > 0   # the pinned scalar mirror
        pr.pr_set_memory_cache_limit(1 << 34)
        it_big = _solve_once(P)
        big = pr.pr_memory_cache_info(0)
        say("limit 16 GiB", big)
        assert big["idle_bytes"] > 1 << 20 and big["idle_blocks"] > 10
        assert it_small == it_big
        pr.pr_set_memory_cache_limit(1 << 16)                         # lowering the limit trims
        assert pr.pr_memory_cache_info(0)["idle_bytes"] <= 1 << 16
        assert pr.pr_memory_cache_info(-1)["idle_bytes"] <= 1 << 16
        pr.pr_release_cached_memory()
        assert pr.pr_memory_cache_info(0)["idle_bytes"] == 0
        assert pr.pr_memory_cache_info(-1)["idle_bytes"] == 0
    finally:
        pr.pr_set_memory_cache_limit(-1)


def test_set_stream_waits_for_the_old_stream():
    P = gen.q1_poisson_2d(32)
    h = pr.PatchRelax(P.A, P.ptr, P.dofs, **KW)
    r = torch.as_tensor(np.random.default_rng(2).standard_normal(P.n)).to(DEV)
    z1 = torch.zeros_like(r)
    z2 = torch.zeros_like(r)
    torch.cuda.synchronize()
    s1 = torch.cuda.Stream()
    with torch.cuda.stream(s1):
        h.set_stream(s1)
        for _ in range(20):
            h.apply(r, z1)
    h.set_stream(torch.cuda.current_stream())    # waits for s1
    assert s1.query()
    h.apply(r, z2)
    torch.cuda.synchronize()
    assert torch.equal(z1, z2)
    h.close()
