"""Batched launches and the continuous-batching server on the GPU (through the C ABI).

The batched kernel runs the same per-grid arithmetic as the single-grid
kernels, so every batched or served result must equal the grid's result when it
runs alone, bit for bit, and match the fp64 oracle within the mode's tolerance.
"""
import time

import numpy as np
import pytest

import paper_2506_22035_amd as sp
import stencil_inputs as si
from gpu_helpers import from_dev, rel_errors, to_dev

pytestmark = pytest.mark.gpu


def _mix(carry="f16"):
    """Four small grids of different shape and stencil."""
    out = []
    for name in ["box2d49p_10240", "star2d13p_8192", "box3d27p_512", "heat3d_256"]:
        wl = si.workload(name, small=True)
        xd, x64 = to_dev(wl["make_grid"](), carry)
        out.append((wl, xd, x64))
    out.append((dict(coeffs=si.coeffs_uniform01(2, 1, 1), shape=(200, 333), steps=7),) +
               to_dev(si.grid_uniform01((200, 333), 9), carry))
    return out


def _alone(wl, xd, steps, carry="f16", engine="sparse"):
    # batched launches run two fused steps on 2-D paired-band grids and one step on 3-D
    # grids: they equal the single-plan apply with time_block = 2 (2-D) or 1 (3-D, whose
    # own two-step kernel sums in another order) bit for bit
    import torch
    tb = 2 if len(wl["shape"]) == 2 else 1
    p = sp.Plan(wl["coeffs"], wl["shape"], carry=carry, engine=engine, time_block=tb)
    y = torch.empty_like(xd)
    p.apply(xd, y, steps)
    return from_dev(y)


@pytest.mark.parametrize("engine", ["sparse", "dense"])
def test_batch_equals_alone(oracle_mod, engine):
    import torch
    mix = _mix()
    plans = [sp.Plan(wl["coeffs"], wl["shape"], carry="f16", engine=engine) for wl, _, _ in mix]
    outs = [torch.empty_like(xd) for _, xd, _ in mix]
    steps = [wl["steps"] for wl, _, _ in mix]
    steps[1] = 3  # uneven step counts
    sp.apply_batch(plans, [xd for _, xd, _ in mix], outs, steps)
    for (wl, xd, x64), o, st in zip(mix, outs, steps):
        got = from_dev(o)
        assert np.array_equal(got, _alone(wl, xd, st, engine=engine))
        rms, mx = rel_errors(got, oracle_mod.apply(wl["coeffs"], x64, st))
        assert rms <= 2e-3 and mx <= 1e-2


def test_batch_integer_exact_aliasing_and_zero_steps(oracle_mod):
    import torch
    shapes = [(70, 300), (9, 10, 264), (33, 520)]
    plans, xs, x64s, ws = [], [], [], []
    for i, sh in enumerate(shapes):
        w = si.integer_coeffs(len(sh), 1, -1, 1, 70 + i, "box")
        xd, x64 = to_dev(si.grid_integer(sh, -1, 1, 80 + i), "f16")
        plans.append(sp.Plan(w, sh, carry="f16"))
        xs.append(xd)
        x64s.append(x64)
        ws.append(w)
    steps = [2, 1, 0]
    ins = [x.clone() for x in xs]
    outs = [ins[0], torch.empty_like(xs[1]), torch.empty_like(xs[2])]  # grid 0 in place
    sp.apply_batch(plans, ins, outs, steps)
    for i in range(3):
        assert np.array_equal(from_dev(outs[i]), oracle_mod.apply(ws[i], x64s[i], steps[i])), i


def test_batch_rejects_bad_input():
    import torch
    wl = si.workload("box2d49p_10240", small=True)
    xd, _ = to_dev(wl["make_grid"](), "f16")
    p = sp.Plan(wl["coeffs"], wl["shape"], carry="f16")
    y = torch.empty_like(xd)
    with pytest.raises(sp.SpiderError):
        sp.apply_batch([p, p], [xd, xd], [y, y], [1, 1])  # one plan twice


def test_batch_runs_unbatchable_plans_alone_and_groups_carries():
    # plans the batched kernel does not hold (the direct engine, an fp32 carry, a
    # radius above 3) run their own time loops; fp16 and bf16 plans are batched in
    # two groups: every result equals spider_apply of its plan
    import torch
    wl = si.workload("box2d49p_10240", small=True)
    cases = [(dict(carry="f32"), "f32"),                                   # direct engine
             (dict(carry="f32", engine="sparse", split=3), "f32"),          # fp32 carry
             (dict(carry="f16"), "f16"), (dict(carry="bf16"), "bf16"),
             (dict(carry="f16", band_height=16), "f16")]
    plans, xs, refs = [], [], []
    for kw, carry in cases:
        p = sp.Plan(wl["coeffs"], wl["shape"], **kw)
        xd, _ = to_dev(wl["make_grid"](), carry)
        y = torch.empty_like(xd)
        p.apply(xd, y, 5)
        plans.append(p)
        xs.append(xd)
        refs.append(from_dev(y))
    w9 = si.coeffs_uniform01(2, 4, 3)  # radius 4: 16-point bands, not batched
    p9 = sp.Plan(w9, (100, 300), carry="f16")
    x9, _ = to_dev(si.grid_uniform01((100, 300), 4), "f16")
    y9 = torch.empty_like(x9)
    p9.apply(x9, y9, 5)
    plans.append(p9)
    xs.append(x9)
    refs.append(from_dev(y9))
    outs = [torch.empty_like(x) for x in xs]
    sp.apply_batch(plans, xs, outs, [5] * len(plans))
    for o, r in zip(outs, refs):
        assert np.array_equal(from_dev(o), r)


def _wait(srv, tickets, timeout=60.0):
    t0 = time.time()
    res = {}
    while len(res) < len(tickets):
        for t in tickets:
            if t not in res:
                done, st = srv.poll(t)
                if done:
                    res[t] = st
        if time.time() - t0 > timeout:
            raise TimeoutError("server did not finish")
        time.sleep(0.001)
    return res


def test_server_results_equal_alone_in_the_mix():
    import torch
    mix = _mix()
    srv = sp.Server(hbm_budget_bytes=1 << 30, max_slots=16)
    plans, outs, tickets = [], [], []
    try:
        # several requests per plan, arriving while others are running
        for rep in range(3):
            for k, (wl, xd, _) in enumerate(mix):
                p = sp.Plan(wl["coeffs"], wl["shape"], carry="f16")
                o = torch.empty_like(xd)
                st = wl["steps"] + rep * 5
                tickets.append((srv.submit(p, xd, o, st), k, st))
                plans.append(p)
                outs.append(o)
            time.sleep(0.002)
        res = _wait(srv, [t for t, _, _ in tickets])
        assert all(v == 0 for v in res.values())
        for (t, k, st), o in zip(tickets, outs):
            wl, xd, _ = mix[k]
            assert np.array_equal(from_dev(o), _alone(wl, xd, st)), (k, st)
        stats = srv.stats()
        assert stats["completed"] == len(tickets) and stats["p99_us"] >= stats["p50_us"] > 0
    finally:
        srv.close()


def test_server_admission_by_footprint():
    import torch
    wl = si.workload("box2d49p_10240", small=True)
    xd, _ = to_dev(wl["make_grid"](), "f16")
    grid_bytes = xd.numel() * 2
    # room for exactly one request (two grid-sized buffers) at a time
    srv = sp.Server(hbm_budget_bytes=2 * grid_bytes + 100, max_slots=8, max_queue=3)
    try:
        plans = [sp.Plan(wl["coeffs"], wl["shape"], carry="f16") for _ in range(3)]
        outs = [torch.empty_like(xd) for _ in range(3)]
        ts = [srv.submit(p, xd, o, 20) for p, o in zip(plans, outs)]
        res = _wait(srv, ts)
        assert all(v == 0 for v in res.values())
        ref = _alone(wl, xd, 20)
        for o in outs:
            assert np.array_equal(from_dev(o), ref)
        big = si.workload("box2d49p_10240", small=False)
        pbig = sp.Plan(big["coeffs"], (1024, 1024), carry="f16")
        xb = torch.zeros((1024, 1024), dtype=torch.float16, device="cuda")
        with pytest.raises(sp.SpiderError) as e:
            srv.submit(pbig, xb, xb, 1)
        assert e.value.status == 3  # OOM: alone exceeds the budget
        with pytest.raises(sp.SpiderError) as e:
            srv.poll(987654321)
        assert e.value.status == 7
    finally:
        srv.close()


def test_server_queue_full_and_close():
    import torch
    wl = si.workload("box2d49p_10240", small=True)
    xd, _ = to_dev(wl["make_grid"](), "f16")
    srv = sp.Server(hbm_budget_bytes=2 * xd.numel() * 2 + 100, max_slots=1, max_queue=2)
    plans = [sp.Plan(wl["coeffs"], wl["shape"], carry="f16") for _ in range(6)]
    outs = [torch.empty_like(xd) for _ in range(6)]
    got_busy = False
    ts = []
    for p, o in zip(plans, outs):
        t = srv.try_submit(p, xd, o, 200)
        if t is None:
            got_busy = True
        else:
            ts.append(t)
    assert got_busy
    srv.close()  # admitted requests finish, queued ones fail with CLOSED
    torch.cuda.synchronize()


def test_server_zero_steps_in_place_and_threads():
    # zero-step requests copy, in-place requests (in == out) work, and submissions
    # from several host threads at once all complete with their own results
    import threading
    import torch
    mix = _mix()
    srv = sp.Server(hbm_budget_bytes=1 << 30, max_slots=8)
    try:
        jobs = []   # (mix index, steps, in_place)
        for k in range(len(mix)):
            jobs += [(k, 0, False), (k, 4, True), (k, 9, False)]
        plans = [sp.Plan(mix[k][0]["coeffs"], mix[k][0]["shape"], carry="f16") for k, _, _ in jobs]
        ins = [mix[k][1].clone() for k, _, _ in jobs]
        outs = [x if ip else torch.empty_like(x) for x, (_, _, ip) in zip(ins, jobs)]
        torch.cuda.synchronize()
        tickets = [None] * len(jobs)
        errors = []

        def submit(idx):
            try:
                for i in idx:
                    tickets[i] = srv.submit(plans[i], ins[i], outs[i], jobs[i][1])
            except Exception as e:   # reported below
                errors.append(e)

        threads = [threading.Thread(target=submit, args=(range(t, len(jobs), 4),)) for t in range(4)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        assert not errors, errors
        assert len(set(tickets)) == len(jobs)
        res = _wait(srv, tickets)
        assert all(v == 0 for v in res.values())
        for (k, st, ip), o in zip(jobs, outs):
            wl, xd, _ = mix[k]
            want = from_dev(xd) if st == 0 else _alone(wl, xd, st)
            assert np.array_equal(from_dev(o), want), (k, st, ip)
    finally:
        srv.close()


def test_server_runs_deeply_fused_grids_on_their_own(oracle_mod):
    # a 2-D grid large enough that its plan fuses three steps runs its own fused
    # launches inside the server's rounds (small grids stay batched); integer data
    # keeps every result exact over several rounds
    import torch
    shape = (2048, 4096)                       # 2^23 points: three fused steps
    shift = np.zeros((7, 7))
    shift[2, 5] = 1.0                          # one tap: values move, never grow
    taps = np.zeros((7, 7))
    taps[3, 3], taps[0, 6], taps[5, 1] = 1.0, -1.0, 1.0
    x = si.grid_integer(shape, -2, 2, 91)
    xd, x64 = to_dev(x, "f16")
    small = si.workload("box2d49p_10240", small=True)
    xs, _ = to_dev(small["make_grid"](), "f16")
    srv = sp.Server(hbm_budget_bytes=1 << 30, max_slots=8)
    try:
        jobs = [(shift, 21, False), (shift, 19, True), (taps, 6, False)]
        plans, outs, tickets = [], [], []
        for w, st, in_place in jobs:
            p = sp.Plan(w, shape, carry="f16")
            assert p.info()["time_block"] == 3
            src = xd.clone() if in_place else xd
            o = src if in_place else torch.empty_like(xd)
            tickets.append(srv.submit(p, src, o, st))
            plans.append(p)
            outs.append(o)
        ps = sp.Plan(small["coeffs"], small["shape"], carry="f16")
        os_ = torch.empty_like(xs)
        tickets.append(srv.submit(ps, xs, os_, 20))
        res = _wait(srv, tickets)
        assert all(v == 0 for v in res.values())
        for (w, st, in_place), o in zip(jobs, outs):
            assert np.array_equal(from_dev(o), oracle_mod.apply(w, x64, st)), (st, in_place)
        assert np.array_equal(from_dev(os_), _alone(small, xs, 20))
    finally:
        srv.close()


def test_server_holds_plans_and_grids_until_done():
    # the caller drops its own references to the plan and the input right after
    # submitting; the server object keeps them alive until the ticket has been
    # reported done (the library reads both until then), and the result is right
    import gc
    import weakref
    import torch
    wl, xd, _ = _mix()[0]
    want = _alone(wl, xd, 20)
    srv = sp.Server(hbm_budget_bytes=1 << 30, max_slots=4)
    try:
        p = sp.Plan(wl["coeffs"], wl["shape"], carry="f16")
        x = xd.clone()
        o = torch.empty_like(xd)
        t = srv.submit(p, x, o, 20)
        wp, wx = weakref.ref(p), weakref.ref(x)
        del p, x
        gc.collect()
        assert wp() is not None and wx() is not None   # not yet reported done
        _wait(srv, [t])
        assert np.array_equal(from_dev(o), want)
        gc.collect()
        assert wp() is None and wx() is None            # released once reported done
    finally:
        srv.close()


def test_server_releases_a_ticket_once_reported_done():
    import ctypes
    import torch
    wl, xd, _ = _mix()[1]
    srv = sp.Server(hbm_budget_bytes=1 << 30, max_slots=4)
    try:
        p = sp.Plan(wl["coeffs"], wl["shape"], carry="f16")
        o = torch.empty_like(xd)
        t = srv.submit(p, xd, o, 3)
        _wait(srv, [t])
        # the library reported it done once; a second poll of the C ABI finds no ticket
        d, r = ctypes.c_int(), ctypes.c_int()
        assert sp.lib().spider_poll(srv._h, ctypes.c_uint64(t), ctypes.byref(d), ctypes.byref(r)) == 7
        # the binding keeps the status it was told
        assert srv.poll(t) == (True, 0)
    finally:
        srv.close()


def test_batch_graph_replays_equal_direct_launches():
    # plans with use_graph capture a batch of fixed membership once and replay it; the
    # replays must equal the directly launched batch bit for bit, also after eager
    # work on the same buffers between replays, with in-place and zero-step entries,
    # and after a plan of the batch is destroyed and replaced
    import torch
    mix = _mix()
    steps = [wl["steps"] for wl, _, _ in mix]
    steps[1], steps[3] = 3, 0
    plans_d = [sp.Plan(wl["coeffs"], wl["shape"], carry="f16", use_graph=False) for wl, _, _ in mix]
    outs_d = [torch.empty_like(xd) for _, xd, _ in mix]
    ins = [xd for _, xd, _ in mix]
    sp.apply_batch(plans_d, ins, outs_d, steps)
    want = [from_dev(o) for o in outs_d]
    plans_g = [sp.Plan(wl["coeffs"], wl["shape"], carry="f16") for wl, _, _ in mix]
    outs_g = [torch.empty_like(xd) for _, xd, _ in mix]
    for rep in range(3):
        sp.apply_batch(plans_g, ins, outs_g, steps)
        torch.cuda.synchronize()
        for o, w in zip(outs_g, want):
            assert np.array_equal(from_dev(o), w), rep
        for o in outs_g:        # eager work on the outputs between replays
            o.zero_()
        plans_g[0].apply(ins[0], outs_g[0], 2)
        torch.cuda.synchronize()
    # in place: each input copied, then advanced in its own buffer
    for rep in range(2):
        bufs = [x.clone() for x in ins]
        sp.apply_batch(plans_g, bufs, bufs, steps)
        torch.cuda.synchronize()
        for b, w in zip(bufs, want):
            assert np.array_equal(from_dev(b), w), ("in place", rep)
    # a destroyed plan's graphs are dropped; its replacement computes afresh
    wl0 = mix[0][0]
    plans_g[0].close()
    plans_g[0] = sp.Plan(wl0["coeffs"], wl0["shape"], carry="f16")
    sp.apply_batch(plans_g, ins, outs_g, steps)
    torch.cuda.synchronize()
    for o, w in zip(outs_g, want):
        assert np.array_equal(from_dev(o), w)
