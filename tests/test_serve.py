"""Continuous-batching server: served results equal the same request run
alone (bitwise: a batch member's arithmetic does not depend on the mix), match
the oracle's backward-Euler steps, and admission respects the HBM budget.
The stream generator is checked on the CPU."""
import numpy as np
import pytest

import oracle
from paper_1506_08435_amd import workloads as W


def _requests(n, steps, dof_range=(150, 2500), gap=0.002, seed=7):
    from paper_1506_08435_amd.serve import Request
    return [Request(k, W.serve_problem(k, seed=seed, dof_range=dof_range), steps, k * gap)
            for k in range(n)]


# ---------------------------------------------------------------- CPU: stream generator
def test_serve_stream_mix_and_sizes():
    dims, dofs = [], []
    for k in range(400):
        p = W.serve_problem(k, seed=3, dof_range=(1e3, 3e4))
        dims.append(p.dim)
        dofs.append(p.n_free)
        assert p.f_elem.max() == 1.0 and p.f_elem.min() == 0.0
    dims = np.array(dims)
    assert 0.4 < (dims == 2).mean() < 0.6                       # 50/50 2D / 3D
    logd = np.log(np.array(dofs))
    # log-uniform in [1e3, 3e4], up to the rounding of the grid side
    assert logd.min() > np.log(1e3) - 0.7 and logd.max() < np.log(3e4) + 0.7
    assert abs(np.median(logd) - 0.5 * (np.log(1e3) + np.log(3e4))) < 0.4


def test_serve_arrivals_poisson():
    t = W.serve_arrivals(20000, rate=500.0, seed=1)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert np.all(gaps > 0)
    assert abs(gaps.mean() - 1 / 500.0) < 0.03 / 500.0 * 3
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.05            # exponential: CV = 1


# ---------------------------------------------------------------- GPU
@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_served_result_equals_alone(prec):
    import torch
    from paper_1506_08435_amd import nnqp
    from paper_1506_08435_amd.serve import Server, solve_alone
    precision = nnqp.NN_MIXED if prec == "mixed" else nnqp.NN_FP64
    reqs = _requests(7, steps=3)
    srv = Server(precision=precision, tol=1e-10, inner_rtol=0.1, keep_states=True)
    rep = srv.run(reqs)
    assert all(r.status == 0 for r in rep.results)
    assert rep.mean_batch > 1.5, "requests should overlap on the device"
    ctx = nnqp.Context(0)
    for req, res in zip(reqs, rep.results):
        c_alone, st_alone = solve_alone(req, precision=precision, tol=1e-10, inner_rtol=0.1, ctx=ctx)
        assert torch.equal(res.c, c_alone), req.rid
        assert [s["cg_its"] for s in res.step_stats] == [s["cg_its"] for s in st_alone]
        assert all(s["kkt_rel"] <= 1e-10 for s in res.step_stats)
    print(rep.summary())


@pytest.mark.gpu
def test_lanes_tick_independently_and_equal_alone():
    """Requests routed to three size lanes (free DOF < 400, < 1200, larger)
    run on three streams at once, the top lane stepping each request with the
    single-problem solver; each result is still bitwise the request run alone
    the same way, and the HBM budget shared by the lanes holds."""
    import torch
    from paper_1506_08435_amd import nnqp
    from paper_1506_08435_amd.serve import Server, estimate_bytes, solve_alone
    reqs = _requests(12, steps=3, gap=0.0005, seed=9)
    sizes = [int((np.asarray(r.problem.dirichlet) == 0).sum()) for r in reqs]
    lanes = [sum(1 for b in (400, 1200) if n >= b) for n in sizes]
    assert sorted(set(lanes)) == [0, 1, 2], sizes
    budget = int(0.6 * sum(estimate_bytes(r.problem, nnqp.NN_FP64) for r in reqs))
    srv = Server(hbm_budget=budget, tol=1e-10, inner_rtol=0.1, keep_states=True,
                 lane_bounds=(400, 1200))
    rep = srv.run(reqs)
    assert all(r.status == 0 for r in rep.results)
    assert all(t > 0 for t in rep.lane_ticks) and len(rep.lane_ticks) == 3
    assert rep.peak_bytes <= budget
    ctx = nnqp.Context(0)
    solo = [srv.is_solo(r) for r in reqs]
    assert any(solo) and not all(solo)
    for req, res, single in zip(reqs, rep.results, solo):
        c_alone, st_alone = solve_alone(req, tol=1e-10, inner_rtol=0.1, ctx=ctx, single=single)
        assert torch.equal(res.c, c_alone), req.rid
        assert [s["cg_its"] for s in res.step_stats] == [s["cg_its"] for s in st_alone]
        assert all(s["kkt_rel"] <= 1e-10 for s in res.step_stats)
    print(rep.summary())


@pytest.mark.gpu
def test_served_steps_match_oracle():
    from paper_1506_08435_amd.serve import Server
    reqs = _requests(4, steps=3)
    srv = Server(tol=1e-12, inner_rtol=0.1, keep_states=True)
    rep = srv.run(reqs)
    for req, res in zip(reqs, rep.results):
        S = oracle.assemble(req.problem, with_mass=True)
        c_ref = np.zeros(S.n)
        for _ in range(req.steps):
            r = oracle.transient_step(S, 1e-3, c_ref, tol=1e-13)
            assert r.certified
            c_ref = r.c
        c = res.c.cpu().numpy()
        assert c.min() >= 0.0
        err = np.abs(c - c_ref).max() / np.abs(c_ref).max()
        assert err <= 1e-8, (req.rid, err)


@pytest.mark.gpu
def test_served_bounded_steps_match_oracle_and_alone():
    """Served transient steps with the bounds c_min = 0, c_max = 2e-3 of every
    step (Sec. 2.2.2, eq. Eq:non-negative; the cap is active): the oracle's
    bounded backward-Euler steps, and bitwise the request run alone."""
    import torch
    from paper_1506_08435_amd.serve import Server, solve_alone
    hi = 2e-3
    reqs = _requests(4, steps=3)
    srv = Server(tol=1e-12, inner_rtol=0.1, keep_states=True, bounds=(0.0, hi))
    rep = srv.run(reqs)
    capped = 0
    for req, res in zip(reqs, rep.results):
        assert res.status == 0
        S = oracle.assemble(req.problem, with_mass=True)
        c_ref = np.zeros(S.n)
        for _ in range(req.steps):
            r = oracle.transient_step(S, 1e-3, c_ref, tol=1e-13, hi=hi)
            assert r.certified
            c_ref = r.c
        c = res.c.cpu().numpy()
        assert c.min() >= 0.0 and c.max() <= hi
        err = np.abs(c - c_ref).max() / np.abs(c_ref).max()
        assert err <= 1e-8, (req.rid, err)
        capped += int((c == hi).sum())
        c_alone, _ = solve_alone(req, tol=1e-12, inner_rtol=0.1, bounds=(0.0, hi))
        assert torch.equal(res.c, c_alone)
    assert capped > 0


@pytest.mark.gpu
def test_admission_respects_budget():
    from paper_1506_08435_amd.serve import NN_EBUDGET, Request, Server, estimate_bytes
    from paper_1506_08435_amd import nnqp
    reqs = _requests(8, steps=2, gap=0.0)
    big = max(estimate_bytes(r.problem, nnqp.NN_FP64) for r in reqs)
    budget = int(2.2 * big)
    huge = Request(99, W.serve_problem(0, seed=11, dof_range=(2e5, 2.1e5)), 1, 0.0)
    assert estimate_bytes(huge.problem, nnqp.NN_FP64) > budget
    srv = Server(hbm_budget=budget, tol=1e-8)
    rep = srv.run(reqs + [huge])
    by = {r.rid: r for r in rep.results}
    assert by[99].status == NN_EBUDGET
    assert all(by[r.rid].status == 0 for r in reqs)
    assert rep.peak_bytes <= budget
    assert rep.deferred > 0
    print(rep.summary())


@pytest.mark.gpu
def test_admission_estimate_bounds_assembled_bytes():
    """The pre-assembly estimate used for admission is never below the
    assembled request's own figure (nn_matrix_bytes + f, c, active)."""
    from paper_1506_08435_amd import nnqp
    from paper_1506_08435_amd.serve import estimate_bytes
    ctx = nnqp.Context(0)
    for k in range(8):
        p = W.serve_problem(k, seed=21, dof_range=(500, 60000))
        K, F, _ = ctx.assemble(p, with_mass=True)
        for prec in (nnqp.NN_FP64, nnqp.NN_MIXED):
            assert estimate_bytes(p, prec) >= K.bytes(prec) + 17 * K.n, (k, prec)
        K.free()


@pytest.mark.gpu
def test_failed_request_stops_every_lane():
    """A request whose assembly fails (a non-finite source, refused on the
    host before any device work) raises from Server.run, and the other lanes
    stop rather than run on or wait for memory the failed lane holds."""
    import dataclasses
    import time
    from paper_1506_08435_amd import nnqp
    from paper_1506_08435_amd.serve import Request, Server
    reqs = _requests(6, steps=40, gap=0.0, seed=9)
    bad = W.serve_problem(0, seed=5, dof_range=(2000, 2500))
    bad = dataclasses.replace(bad, f_elem=np.full_like(bad.f_elem, np.nan))
    reqs.append(Request(99, bad, 3, 0.0))
    srv = Server(tol=1e-8, lane_bounds=(400, 1200))
    assert srv.is_solo(reqs[-1])
    t0 = time.perf_counter()
    with pytest.raises(nnqp.NnError) as err:
        srv.run(reqs)
    assert err.value.status == nnqp.NN_ENONFINITE
    assert time.perf_counter() - t0 < 60


@pytest.mark.gpu
def test_served_mixed_solo_lane_equals_alone_and_oracle():
    """Mixed precision with the upper lanes stepped by the single-problem
    solver: each served result is bitwise the request run alone the same way
    (batched or single-problem), and within 1e-6 of the oracle's float64
    backward-Euler steps; the error of every request is printed."""
    import torch
    from paper_1506_08435_amd import nnqp
    from paper_1506_08435_amd.serve import Server, solve_alone
    reqs = _requests(8, steps=3, gap=0.0005, seed=9)
    srv = Server(precision=nnqp.NN_MIXED, tol=1e-10, inner_rtol=0.1, keep_states=True,
                 lane_bounds=(400, 1200))
    solo = [srv.is_solo(r) for r in reqs]
    assert any(solo) and not all(solo)
    rep = srv.run(reqs)
    assert all(r.status == 0 for r in rep.results)
    ctx = nnqp.Context(0)
    for req, res, single in zip(reqs, rep.results, solo):
        c_alone, _ = solve_alone(req, precision=nnqp.NN_MIXED, tol=1e-10, inner_rtol=0.1,
                                 ctx=ctx, single=single)
        assert torch.equal(res.c, c_alone), req.rid
        S = oracle.assemble(req.problem, with_mass=True)
        c_ref = np.zeros(S.n)
        for _ in range(req.steps):
            r = oracle.transient_step(S, 1e-3, c_ref, tol=1e-13)
            assert r.certified
            c_ref = r.c
        c = res.c.cpu().numpy()
        assert c.min() >= 0.0
        err = np.abs(c - c_ref).max() / np.abs(c_ref).max()
        print(f"request {req.rid} n={S.n} {'single' if single else 'batched'} "
              f"mixed rel err {err:.2e}")
        assert err <= 1e-6, (req.rid, err)


def _tracking_allocator(refuse=None):
    """(alloc, free, state) over torch's caching allocator that counts live
    and peak bytes; refuse(nbytes) -> True makes an allocation fail."""
    import torch
    state = {"live": {}, "bytes": 0, "peak": 0, "refused": 0}

    def alloc(nbytes):
        if refuse is not None and refuse(nbytes):
            state["refused"] += 1
            return None
        p = torch.cuda.caching_allocator_alloc(nbytes, 0, torch.cuda.current_stream(0))
        state["live"][p] = nbytes
        state["bytes"] += nbytes
        state["peak"] = max(state["peak"], state["bytes"])
        return p

    def free(p):
        nb = state["live"].pop(p, None)
        if nb is not None:
            state["bytes"] -= nb
            torch.cuda.caching_allocator_delete(p)

    return alloc, free, state


@pytest.mark.gpu
@pytest.mark.parametrize("solo", [False, True])
def test_failed_step_call_stops_the_server(solo):
    """A step whose call fails for want of memory (the caller's allocator
    refuses every request from the lane threads after their first few, forced
    from the host) raises NN_EOOM from Server.run, for a batched lane and for
    a single-problem lane: no request is reported as stepped or finished."""
    import threading
    from paper_1506_08435_amd import nnqp
    from paper_1506_08435_amd.serve import Server
    main = threading.main_thread()
    lane_allocs = [0]

    def refuse(nbytes):
        t = threading.current_thread()
        if t is main or t.name.startswith("ThreadPoolExecutor"):
            return False              # contexts and assembly get their memory
        lane_allocs[0] += 1
        return lane_allocs[0] > 3     # the first step's call is refused part-way
    alloc, free, _ = _tracking_allocator(refuse)
    reqs = _requests(4, steps=3, gap=0.0, seed=9)
    bounds = (10, 20) if solo else (10 ** 7, 10 ** 8)
    srv = Server(tol=1e-8, lane_bounds=bounds, allocator=(alloc, free))
    assert all(srv.is_solo(r) == solo for r in reqs)
    with pytest.raises(nnqp.NnError) as err:
        srv.run(reqs)
    assert err.value.status == nnqp.NN_EOOM
    assert lane_allocs[0] > 3


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_admission_estimate_bounds_measured_step_memory(prec):
    """The admission estimate of a request covers the device memory its steps
    actually take, measured through the allocator hooks at the peak of one
    step (matrix, the copies a step adds, and the batched call's workspace or
    the single-problem solver's work vectors), plus f, c and the active set."""
    import torch
    from paper_1506_08435_amd import nnqp
    from paper_1506_08435_amd.serve import estimate_bytes
    precision = nnqp.NN_MIXED if prec == "mixed" else nnqp.NN_FP64
    for k in range(6):
        p = W.serve_problem(k, seed=21, dof_range=(500, 60000))
        for solo in (False, True):
            alloc, free, state = _tracking_allocator()
            ctx = nnqp.Context(0, allocator=(alloc, free))
            torch.cuda.synchronize()
            base = state["bytes"]
            state["peak"] = base
            K, F, _ = ctx.assemble(p, with_mass=True)
            c = torch.zeros(max(K.n, 1), dtype=torch.float64, device=ctx.device)
            torch.cuda.synchronize()
            state["peak"] = state["bytes"]   # the resident matrix, from here on
            opts = nnqp.default_opts(tol=1e-8, precision=precision)
            if solo:
                ctx.step_transient(K, 1e-3, F, c, opts=opts)
            else:
                ctx.step_transient_batch([K], 1e-3, [F], [c], opts=opts)
            torch.cuda.synchronize()
            used = state["peak"] - base + 17 * K.n
            est = estimate_bytes(p, precision, solo=solo)
            print(f"problem {k} dim {p.dim} n={K.n} solo={solo} measured {used} estimate {est}")
            assert est >= used, (k, solo, used, est)
            K.free()
            ctx.close()


@pytest.mark.gpu
def test_cancelled_requests_leave_and_the_rest_equal_alone():
    """Request 1 is cancelled before it arrives, request 2 while it is being
    stepped (it asks for 20,000 steps, seconds of work, and is cancelled 0.3 s
    after arriving), request 4 by Server.cancel from another thread: each ends
    with status CANCELLED and fewer steps than asked, the others complete
    bitwise equal to the request run alone, and every byte of budget is
    returned."""
    import threading
    import torch
    from paper_1506_08435_amd import nnqp
    from paper_1506_08435_amd.serve import CANCELLED, Server, solve_alone
    reqs = _requests(6, steps=3, gap=0.001, seed=11)
    reqs[1].cancel_at = 0.0
    reqs[2].steps = 20000
    reqs[2].cancel_at = reqs[2].arrival + 0.3
    reqs[4].steps = 20000
    srv = Server(keep_states=True, tol=1e-10, inner_rtol=0.1)
    timer = threading.Timer(0.3, srv.cancel, args=(reqs[4].rid,))
    timer.start()
    try:
        rep = srv.run(reqs)
    finally:
        timer.cancel()
    by = {r.rid: r for r in rep.results}
    for k in (1, 2, 4):
        assert by[k].status == CANCELLED, (k, by[k].status)
        assert len(by[k].step_stats) < reqs[k].steps
    assert len(by[1].step_stats) == 0
    assert rep.summary()["cancelled"] == 3
    assert rep.final_bytes == 0
    ctx = nnqp.Context(0)
    for k in (0, 3, 5):
        assert by[k].status == 0
        c_alone, _ = solve_alone(reqs[k], tol=1e-10, inner_rtol=0.1, ctx=ctx,
                                 single=srv.is_solo(reqs[k]))
        assert torch.equal(by[k].c, c_alone), k
