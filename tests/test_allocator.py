"""Device memory through the caller's allocator (nn_create_ex): a context
whose hooks are torch's caching allocator takes every device buffer from it
(torch's own counter sees them), gives every one back, and computes bitwise
the same results as a context on hipMalloc, for single, mixed-precision,
transient and batched solves."""
import pytest

from paper_1506_08435_amd import workloads as W


@pytest.mark.gpu
def test_torch_allocator_hooks_same_results_and_all_memory_returned():
    import torch
    from paper_1506_08435_amd import nnqp

    cube = W.cube3d(12)
    members = [W.batch_problem(i, n_range=(8, 40)) for i in range(4)]
    tr = W.config_transient3d(12, 10, 6, ell=2.0)

    def run(ctx):
        out = {}
        K, F, _ = ctx.assemble(cube)
        c, act, st = ctx.solve_nonneg(K, F, tol=1e-10)
        out["fp64"] = (c.clone(), act.clone(), st["cg_its"])
        c, act, st = ctx.solve_nonneg(K, F, tol=1e-10, precision=nnqp.NN_MIXED)
        out["mixed"] = (c.clone(), act.clone(), st["cg_its"])
        Kt, Ft, _ = ctx.assemble(tr, with_mass=True)
        ct = torch.zeros(Kt.n, dtype=torch.float64, device=ctx.device)
        for _ in range(2):
            ct, _, _ = ctx.step_transient(Kt, 1e-3, Ft, ct, tol=1e-10)
        out["transient"] = ct.clone()
        Ks, Fs = [], []
        for p in members:
            Kb, Fb, _ = ctx.assemble(p)
            Ks.append(Kb)
            Fs.append(Fb)
        cs, _, stats, _ = ctx.solve_batch(Ks, Fs, tol=1e-10)
        out["batch"] = [x.clone() for x in cs]
        for M in [K, Kt] + Ks:
            M.free()
        torch.cuda.synchronize()
        return out

    ref = run(nnqp.Context(0))
    # torch's caching allocator behind counting hooks: every pointer the
    # library takes is recorded until it comes back
    live, seen, foreign = {}, [0], []

    def alloc(nbytes):
        p = torch.cuda.caching_allocator_alloc(nbytes, 0, torch.cuda.current_stream(0))
        live[p] = nbytes
        seen[0] += 1
        return p

    def free(p):   # runs inside a library call: record, assert afterwards
        if p not in live:
            foreign.append(p)
            return
        del live[p]
        torch.cuda.caching_allocator_delete(p)

    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    ctx = nnqp.Context(0, allocator=(alloc, free))
    assert live                                           # reduction partials and scalars
    K, F, _ = ctx.assemble(cube)
    assert torch.cuda.memory_allocated() - base >= 12 * K.nnz   # the matrix lives in torch's pool
    assert sum(live.values()) >= 12 * K.nnz
    K.free()
    del F
    got = run(ctx)
    for key in ("fp64", "mixed"):
        assert torch.equal(got[key][0], ref[key][0]), key
        assert torch.equal(got[key][1], ref[key][1]), key
        assert got[key][2] == ref[key][2], key
    assert torch.equal(got["transient"], ref["transient"])
    for a, b in zip(got["batch"], ref["batch"]):
        assert torch.equal(a, b)
    assert seen[0] > 50                                   # batch arrays, copies, work vectors
    ctx.close()
    torch.cuda.synchronize()
    assert not foreign, "freed pointers the hooks did not hand out"
    assert not live, f"{len(live)} buffers not returned: {sorted(live.values())}"


@pytest.mark.gpu
def test_torch_allocator_keyword():
    """allocator="torch": the library's buffers are counted by torch."""
    import torch
    from paper_1506_08435_amd import nnqp
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    ctx = nnqp.Context(0, allocator="torch")
    K, F, _ = ctx.assemble(W.cube3d(10))
    assert torch.cuda.memory_allocated() - base >= 12 * K.nnz
    c, _, st = ctx.solve_nonneg(K, F, tol=1e-10)
    assert st["kkt_rel"] <= 1e-10


@pytest.mark.gpu
def test_allocator_failure_is_reported_and_leaks_nothing():
    """The caller's allocator refusing the k-th request (forced from the host)
    surfaces as NN_EOOM from whichever call needed the memory; every buffer
    the library did get is still given back, and nothing it did not get is
    freed."""
    import torch
    from paper_1506_08435_amd import nnqp

    cube = W.cube3d(6)
    members = [W.batch_problem(i, n_range=(8, 16)) for i in range(3)]
    outcomes = []
    for limit in list(range(0, 40, 3)) + [60, 100, 400]:
        live, foreign, count = {}, [], [0]

        def alloc(nbytes):
            count[0] += 1
            if count[0] > limit:
                return None
            p = torch.cuda.caching_allocator_alloc(nbytes, 0, torch.cuda.current_stream(0))
            live[p] = nbytes
            return p

        def free(p):
            if p not in live:
                foreign.append(p)
                return
            del live[p]
            torch.cuda.caching_allocator_delete(p)

        try:
            ctx = nnqp.Context(0, allocator=(alloc, free))
        except nnqp.NnError as e:
            assert e.status == nnqp.NN_EOOM
            outcomes.append("create")
        else:
            stage = "done"
            mats = []
            try:
                stage = "assemble"
                K, F, _ = ctx.assemble(cube)
                mats.append(K)
                stage = "solve"
                c, _, st = ctx.solve_nonneg(K, F, tol=1e-10)
                assert st["kkt_rel"] <= 1e-10
                stage = "batch"
                Ks, Fs = [], []
                for p in members:
                    Kb, Fb, _ = ctx.assemble(p)
                    mats.append(Kb)
                    Ks.append(Kb)
                    Fs.append(Fb)
                ctx.solve_batch(Ks, Fs, tol=1e-10)
                stage = "done"
            except nnqp.NnError as e:
                assert e.status == nnqp.NN_EOOM, (limit, stage, str(e))
            outcomes.append(stage)
            for M in mats:
                M.free()
            ctx.close()
        torch.cuda.synchronize()
        assert not foreign, limit
        assert not live, (limit, len(live))
    assert outcomes[0] == "create" and outcomes[-1] == "done"
    assert {"assemble", "solve", "batch"} <= set(outcomes), outcomes


@pytest.mark.gpu
def test_transient_step_after_refused_diagonal_matches_oracle():
    """A backward-Euler step whose M/dt + K diagonal allocation is refused
    (forced from the host: the first request of n float64 after arming) gives
    NN_EOOM; the next step on the same matrix, with memory available, forms
    the missing buffer and matches the oracle's step."""
    import numpy as np
    import torch
    import oracle
    from paper_1506_08435_amd import nnqp

    p = W.config_transient3d(12, 10, 6, ell=2.0)
    S = oracle.assemble(p, with_mass=True)
    arm = [False]
    live = {}

    def alloc(nbytes):
        if arm[0] and nbytes == 8 * S.n:
            arm[0] = False
            return None
        q = torch.cuda.caching_allocator_alloc(nbytes, 0, torch.cuda.current_stream(0))
        live[q] = nbytes
        return q

    def free(q):
        if live.pop(q, None) is not None:
            torch.cuda.caching_allocator_delete(q)

    ctx = nnqp.Context(0, allocator=(alloc, free))
    K, F, _ = ctx.assemble(p, with_mass=True)
    assert K.n == S.n
    c0 = torch.zeros(K.n, dtype=torch.float64, device=ctx.device)
    arm[0] = True
    with pytest.raises(nnqp.NnError) as err:
        ctx.step_transient(K, 1e-3, F, c0.clone(), tol=1e-12)
    assert err.value.status == nnqp.NN_EOOM
    assert not arm[0], "the diagonal allocation was not the one refused"
    c, _, st = ctx.step_transient(K, 1e-3, F, c0.clone(), tol=1e-12)
    ref = oracle.transient_step(S, 1e-3, np.zeros(S.n), tol=1e-13)
    assert ref.certified
    c = c.cpu().numpy()
    assert c.min() >= 0.0
    err = np.abs(c - ref.c).max() / np.abs(ref.c).max()
    assert err <= 1e-8, err
    K.free()
    ctx.close()
    torch.cuda.synchronize()
    assert not live
