"""GPU parity of 1-D stencils (the paper's 1-D benchmarks: r = 1, 2 on 10 240 000 points).

The 16-point band engine applies the single kernel row to consecutive 256-point
blocks of the line, each reading its window from the same array (the halo is the
neighbouring values, zero only beyond the ends).  Integer cases are compared bit
for bit with the oracle; the workload recipes within the stated tolerances.
"""
import numpy as np
import pytest

import paper_2506_22035_amd as sp
import stencil_inputs as si
from gpu_helpers import empty_like_dev, from_dev, rel_errors, to_dev

pytestmark = pytest.mark.gpu

TOL = {"f16": (2e-3, 1e-2), "bf16": (3e-2, 6e-2), "f32": (1e-5, 1e-5), "f64": (1e-13, 1e-13)}
LENGTHS = [1, 7, 255, 256, 257, 4096, 10001, 50000, 123457]


def run(plan, x_dev, steps):
    y = empty_like_dev(x_dev)
    plan.apply(x_dev, y, steps)
    return from_dev(y)


@pytest.mark.parametrize("engine", ["sparse", "dense"])
@pytest.mark.parametrize("n", LENGTHS)
def test_integer_exact_f16(oracle_mod, engine, n):
    for r in (1, 2, 3, 5, 7):
        w = si.integer_coeffs(1, r, -4, 4, 60 + r)
        x = si.grid_integer((n,), -8, 8, 70 + n % 97)
        xd, x64 = to_dev(x, "f16")
        plan = sp.Plan(w, (n,), carry="f16", engine=engine)
        got = run(plan, xd, 1)
        ref = oracle_mod.apply(w, x64, 1)
        assert np.array_equal(got, ref), (r, np.argwhere(got != ref)[:5])


@pytest.mark.parametrize("engine", ["sparse", "dense"])
def test_integer_exact_bf16_and_multistep(oracle_mod, engine):
    n = 30001
    for r in (1, 2):
        w = si.integer_coeffs(1, r, -2, 2, 80 + r)
        xd, x64 = to_dev(si.grid_integer((n,), -2, 2, 81), "bf16")
        plan = sp.Plan(w, (n,), carry="bf16", engine=engine)
        assert np.array_equal(run(plan, xd, 1), oracle_mod.apply(w, x64, 1))
        w = si.integer_coeffs(1, r, -1, 1, 90 + r)
        xd, x64 = to_dev(si.grid_integer((n,), -2, 2, 91), "f16")
        plan = sp.Plan(w, (n,), carry="f16", engine=engine)
        for steps in (2, 3, 4):
            ref = oracle_mod.apply(w, x64, steps)
            if np.abs(ref).max() < 2048:
                assert np.array_equal(run(plan, xd, steps), ref), (r, steps)


@pytest.mark.parametrize("carry", ["f16", "bf16"])
@pytest.mark.parametrize("engine", ["sparse", "dense"])
@pytest.mark.parametrize("name", ["1d3p_10240000", "1d5p_10240000"])
def test_workload_tolerance(oracle_mod, carry, engine, name):
    wl = si.workload(name, small=True)
    xd, x64 = to_dev(wl["make_grid"](), carry)
    plan = sp.Plan(wl["coeffs"], wl["shape"], carry=carry, engine=engine)
    rms, mx = rel_errors(run(plan, xd, wl["steps"]), oracle_mod.apply(wl["coeffs"], x64, wl["steps"]))
    print("%s %s %s: rel-RMS %.3e rel-max %.3e" % (name, carry, engine, rms, mx))
    assert rms <= TOL[carry][0] and mx <= TOL[carry][1]


@pytest.mark.parametrize("carry", ["f32", "f64"])
@pytest.mark.parametrize("n", [1, 13, 4096, 50001])
def test_direct_engine(oracle_mod, carry, n):
    for r in (1, 2, 4):
        rng = np.random.default_rng(n + r)
        w = rng.uniform(-1, 1, 2 * r + 1) / (2 * r + 1)
        xd, x64 = to_dev(rng.uniform(-1, 1, n), carry)
        plan = sp.Plan(w, (n,), carry=carry)
        assert plan.info()["engine"] == "direct"
        rms, mx = rel_errors(run(plan, xd, 5), oracle_mod.apply(w, x64, 5))
        assert rms <= TOL[carry][0] and mx <= TOL[carry][1], r


def test_tile_heights_agree_and_aliasing(oracle_mod):
    import torch
    wl = si.workload("1d5p_10240000", small=True)
    xd, _ = to_dev(wl["make_grid"](), "f16")
    res = []
    for th in (0, 1, 3, 8, 9, 64, 1000):
        plan = sp.Plan(wl["coeffs"], wl["shape"], carry="f16", tile_h=th)
        res.append(run(plan, xd, 6))
    for r_ in res[1:]:
        assert np.array_equal(r_, res[0])
    plan = sp.Plan(wl["coeffs"], wl["shape"], carry="f16")
    keep = xd.clone()
    for steps in (0, 1, 2, 3):
        y = xd.clone()
        plan.apply(y, y, steps)
        assert np.array_equal(from_dev(y), run(plan, xd, steps))
    assert torch.equal(xd, keep)


def test_batch_and_server_run_1d_alone():
    # 1-D lines are not batched: batched apply and the server run them with their
    # own time loop, so the results equal spider_apply bit for bit
    import time
    import torch
    wl = si.workload("1d3p_10240000", small=True)
    x16, _ = to_dev(wl["make_grid"](), "f16")
    x32, _ = to_dev(wl["make_grid"](np.float32), "f32")
    plans = [sp.Plan(wl["coeffs"], wl["shape"], carry="f16", time_block=3),
             sp.Plan(wl["coeffs"], wl["shape"], carry="f32", engine="sparse", split=3, time_block=2)]
    xs = [x16, x32]
    refs = [run(p, x, 7) for p, x in zip(plans, xs)]
    outs = [torch.empty_like(x) for x in xs]
    sp.apply_batch(plans, xs, outs, [7, 7])
    for o, r in zip(outs, refs):
        assert np.array_equal(from_dev(o), r)
    srv = sp.Server(1 << 28)
    try:
        outs = [torch.empty_like(x) for x in xs]
        ts = [srv.submit(p, x, o, 7) for p, x, o in zip(plans, xs, outs)]
        t0 = time.time()
        while not all(srv.poll(t)[0] for t in ts):
            assert time.time() - t0 < 60
            time.sleep(0.001)
        assert all(srv.poll(t)[1] == 0 for t in ts)
        for o, r in zip(outs, refs):
            assert np.array_equal(from_dev(o), r)
    finally:
        srv.close()


# ------------------------------------------------------------------ fp32 carry on the matrix engines

@pytest.mark.parametrize("operand", ["f16", "bf16"])
@pytest.mark.parametrize("engine", ["sparse", "dense"])
@pytest.mark.parametrize("n", [1, 7, 255, 256, 257, 4099, 50000])
def test_f32_carry_integer_exact_input_split(oracle_mod, operand, engine, n):
    # all-ones taps (r = 1) on inputs in {1, 2}: the inputs of the ninth step reach ~1.3e4,
    # beyond the 16-bit significand but exact as x_hi + x_lo; outputs exact in fp32.
    # Integer taps of radius up to 7 with mixed signs over fewer steps.
    cases = [(np.ones(3), 9, (1, 2))]
    cases += [(si.integer_coeffs(1, r, -1, 1, 30 + r), 3, (-2, 2)) for r in (1, 3, 7)]
    for w, steps, (lo, hi) in cases:
        x = si.grid_integer((n,), lo, hi, 90 + n % 13)
        xd, x64 = to_dev(x, "f32")
        plan = sp.Plan(w, (n,), carry="f32", engine=engine, split=3, operand=operand)
        assert plan.info()["engine"] == engine
        ref = oracle_mod.apply(w, x64, steps)
        assert np.abs(oracle_mod.apply(w, x64, steps - 1)).max() < 65504
        got = run(plan, xd, steps)
        assert np.array_equal(got, ref), (w.shape, steps, np.argwhere(got != ref)[:5])


@pytest.mark.parametrize("operand", ["f16", "bf16"])
def test_f32_carry_without_split_equals_16bit_carry(operand):
    # without the input split the arithmetic is the 16-bit carry's: one step rounded to
    # 16 bits equals the 16-bit plan's step bit for bit
    import torch
    wl = si.workload("1d5p_10240000", small=True)
    x16, _ = to_dev(wl["make_grid"](), operand)
    x32 = x16.to(torch.float32)
    p16 = sp.Plan(wl["coeffs"], wl["shape"], carry=operand, time_block=1)
    p32 = sp.Plan(wl["coeffs"], wl["shape"], carry="f32", engine="sparse", split=2, operand=operand)
    y16, y32 = torch.empty_like(x16), torch.empty_like(x32)
    p16.apply(x16, y16, 1)
    p32.apply(x32, y32, 1)
    torch.cuda.synchronize()
    assert torch.equal(y32.to(x16.dtype), y16)


@pytest.mark.parametrize("name", ["1d3p_10240000", "1d5p_10240000"])
def test_f32_carry_workload_tolerance_tiles_and_aliasing(oracle_mod, name):
    import torch
    wl = si.workload(name, small=True)
    xd, x64 = to_dev(wl["make_grid"](np.float32), "f32")
    ref = oracle_mod.apply(wl["coeffs"], x64, wl["steps"])
    res = []
    for th in (0, 1, 3, 17, 1000):
        plan = sp.Plan(wl["coeffs"], wl["shape"], carry="f32", engine="sparse", split=3, tile_h=th)
        res.append(run(plan, xd, wl["steps"]))
    for r_ in res[1:]:
        assert np.array_equal(r_, res[0])
    rms, mx = rel_errors(res[0], ref)
    print("%s f32 carry, split 3: rel-RMS %.3e rel-max %.3e" % (name, rms, mx))
    assert rms <= 5e-5 and mx <= 5e-5
    plan = sp.Plan(wl["coeffs"], wl["shape"], carry="f32", engine="sparse", split=3)
    keep = xd.clone()
    for steps in (0, 1, 2, 3):
        y = xd.clone()
        plan.apply(y, y, steps)
        assert np.array_equal(from_dev(y), run(plan, xd, steps)), steps
    assert torch.equal(xd, keep)
