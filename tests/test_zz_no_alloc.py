"""nn_solve_nonneg_noalloc (the solve for callers that cannot allocate):
through the C ABI, two calls in a row (the second on a smaller system) give
the results of nn_solve_nonneg and the oracle's minimiser, and no device
memory is taken through the context's allocator during either call."""
import numpy as np
import pytest

import oracle
from paper_1506_08435_amd import workloads as W

pytestmark = pytest.mark.gpu


def _hooks():
    import torch
    state = {"calls": 0, "live": {}}

    def alloc(nbytes):
        state["calls"] += 1
        p = torch.cuda.caching_allocator_alloc(nbytes, 0, torch.cuda.current_stream(0))
        state["live"][p] = nbytes
        return p

    def free(p):
        if state["live"].pop(p, None) is not None:
            torch.cuda.caching_allocator_delete(p)

    return alloc, free, state


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_matches_solve_twice_and_allocates_nothing(prec):
    import torch
    from paper_1506_08435_amd import nnqp
    precision = nnqp.NN_MIXED if prec == "mixed" else nnqp.NN_FP64
    bar = 1e-6 if prec == "mixed" else 1e-8
    alloc, free, state = _hooks()
    ctx = nnqp.Context(0, allocator=(alloc, free))
    for p in (W.cube3d(40), W.config_small()):     # the second call is the smaller system
        K, F, _ = ctx.assemble(p)
        print(f"{prec} {p.name}: n = {K.n}", flush=True)
        # the multi-block passes, which the no-allocation solve runs at every size
        c_ref, a_ref, st_ref = ctx.solve_nonneg(K, F, tol=1e-12, precision=precision, engine=1)
        c = torch.full((K.n,), 123.0, dtype=torch.float64, device=ctx.device)
        act = torch.full((K.n,), 7, dtype=torch.uint8, device=ctx.device)
        torch.cuda.synchronize()
        before = state["calls"]
        c2, a2, st2 = ctx.solve_nonneg_noalloc(K, F, c, act, tol=1e-12, precision=precision)
        torch.cuda.synchronize()
        assert state["calls"] == before, "the call took device memory through the allocator"
        assert st2["status"] == 0 and st2["kkt_rel"] <= 1e-12
        # the same kernels on the same copies of K: the result of nn_solve_nonneg
        assert torch.equal(c2, c_ref) and torch.equal(a2, a_ref)
        assert st2["outer_its"] == st_ref["outer_its"] and st2["cg_its"] == st_ref["cg_its"]
        cn = c2.cpu().numpy()
        S = oracle.assemble(p)
        ref = oracle.solve(S, tol=1e-13)
        assert ref.certified and cn.min() >= 0.0
        err = np.abs(cn - ref.c).max() / np.abs(ref.c).max()
        assert err <= bar, err
        g_ref = oracle.spmv(S, ref.c) - S.F
        fr, strict = oracle.nondegenerate_masks(ref.c, g_ref, S.F)
        assert fr.any() and strict.any()
        assert np.all(cn[fr] > 0.0) and np.all(cn[strict] == 0.0)
        print(f"  err vs oracle {err:.2e}, outer {st2['outer_its']}, cg {st2['cg_its']}")
        K.free()
    ctx.close()


def test_noalloc_limits_and_options():
    import torch
    from paper_1506_08435_amd import nnqp
    ctx = nnqp.Context(0)
    big = W.cube3d(66)                      # 65^3 = 274,625 rows > 262,144
    K, F, _ = ctx.assemble(big)
    c = torch.zeros(K.n, dtype=torch.float64, device=ctx.device)
    a = torch.empty(K.n, dtype=torch.uint8, device=ctx.device)
    with pytest.raises(nnqp.NnError) as ei:
        ctx.solve_nonneg_noalloc(K, F, c, a)
    assert ei.value.status == nnqp.NN_EINVAL and "262144" in str(ei.value)
    K.free()
    K, F, _ = ctx.assemble(W.square2d(20))
    c = torch.zeros(K.n, dtype=torch.float64, device=ctx.device)
    a = torch.empty(K.n, dtype=torch.uint8, device=ctx.device)
    for kw in ({"precision": nnqp.NN_MIXED}, {"method": nnqp.NN_BLMVM}, {"precond_degree": 3}):
        with pytest.raises(nnqp.NnError) as ei:
            ctx.solve_nonneg_noalloc(K, F, c, a, **kw)
        assert ei.value.status == nnqp.NN_EINVAL, kw
    # a plain context (hipMalloc) after the hooked ones, same device array
    c2, _, st = ctx.solve_nonneg_noalloc(K, F, c, a, tol=1e-12)
    c1, _, _ = ctx.solve_nonneg(K, F, tol=1e-12, engine=1)
    assert torch.equal(c2, c1)
    ctx.close()
