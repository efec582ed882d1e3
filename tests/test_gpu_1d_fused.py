"""GPU parity of fused time steps on 1-D lines (two to four steps per launch).

A fused launch sums every value exactly as a single step does, so it must equal
single steps bit for bit on any data, and the oracle bit for bit on integer data
whose every step stays below 2^11 (three taps of +-1, inputs in {-2..2}).  The
cases cover lines shorter than a block, ragged ends, segments of one block, step
counts that T does not divide and in-place applies.  The fp32-carry fused kernel
keeps every level as fp32 sums split into 16-bit hi (and lo) rows, exactly as a
single fp32 step splits its input, so it too equals single steps bit for bit.
"""
import numpy as np
import pytest

import paper_2506_22035_amd as sp
import stencil_inputs as si
from gpu_helpers import empty_like_dev, from_dev, to_dev

pytestmark = pytest.mark.gpu

LENGTHS = [1, 7, 255, 256, 257, 520, 4096, 10001, 50000, 123457]


def run(plan, x_dev, steps):
    y = empty_like_dev(x_dev)
    plan.apply(x_dev, y, steps)
    return from_dev(y)


def sparse_int_taps_1d(r, seed):
    rng = np.random.default_rng(seed)
    w = np.zeros(2 * r + 1)
    w[r] = 1.0
    for i in rng.choice([i for i in range(2 * r + 1) if i != r], 2, replace=False):
        w[i] = rng.choice([-1.0, 1.0])
    return w


@pytest.mark.parametrize("T", [2, 3, 4])
@pytest.mark.parametrize("engine", ["sparse", "dense"])
@pytest.mark.parametrize("n", LENGTHS)
def test_fused_integer_exact(oracle_mod, T, engine, n):
    for r in (1, 2, 3):
        w = sparse_int_taps_1d(r, 10 * r + T)
        xd, x64 = to_dev(si.grid_integer((n,), -2, 2, 3 + n % 101), "f16")
        plan = sp.Plan(w, (n,), carry="f16", engine=engine, time_block=T)
        assert plan.info()["time_block"] == T
        ref = oracle_mod.apply(w, x64, T)
        assert np.abs(ref).max() < 2048
        got = run(plan, xd, T)
        assert np.array_equal(got, ref), (r, np.argwhere(got != ref)[:5])


@pytest.mark.parametrize("T", [2, 3, 4])
@pytest.mark.parametrize("carry", ["f16", "bf16"])
def test_fused_equals_single_steps(T, carry):
    wl = si.workload("1d5p_10240000", small=True)
    xd, _ = to_dev(wl["make_grid"](), carry)
    ref = run(sp.Plan(wl["coeffs"], wl["shape"], carry=carry, time_block=1), xd, 11)
    for th in (0, 1, 2, 5, 16, 1000):
        plan = sp.Plan(wl["coeffs"], wl["shape"], carry=carry, time_block=T, tile_h=th)
        assert np.array_equal(run(plan, xd, 11), ref), th


@pytest.mark.parametrize("T", [2, 4])
def test_fused_aliasing(T):
    import torch
    wl = si.workload("1d3p_10240000", small=True)
    xd, _ = to_dev(wl["make_grid"](), "f16")
    plan = sp.Plan(wl["coeffs"], wl["shape"], carry="f16", time_block=T)
    keep = xd.clone()
    for steps in (T, T + 1, 3 * T):
        y = xd.clone()
        plan.apply(y, y, steps)
        assert np.array_equal(from_dev(y), run(plan, xd, steps))
    assert torch.equal(xd, keep)


def test_depth_limits():
    w = np.array([0.25, 0.5, 0.25])
    assert sp.Plan(w, (4096,), carry="f16", time_block=4).info()["time_block"] == 4
    w4 = np.ones(9) / 9
    assert sp.Plan(w4, (4096,), carry="f16", time_block=4).info()["time_block"] == 1  # r > 3
    assert sp.Plan(w, (4096,), carry="f32", time_block=4).info()["time_block"] == 1  # direct engine
    for eng in ("sparse", "dense"):
        assert sp.Plan(w, (4096,), carry="f32", engine=eng, split=3, time_block=4).info()["time_block"] == 4
        assert sp.Plan(w4, (4096,), carry="f32", engine=eng, split=3, time_block=4).info()["time_block"] == 1


@pytest.mark.parametrize("T", [2, 3, 4])
def test_full_size_equals_single_steps(T):
    wl = si.workload("1d3p_10240000")
    xd, _ = to_dev(wl["make_grid"](), "f16")
    a = run(sp.Plan(wl["coeffs"], wl["shape"], carry="f16", time_block=T), xd, 12)
    b = run(sp.Plan(wl["coeffs"], wl["shape"], carry="f16", time_block=1), xd, 12)
    assert np.array_equal(a, b)


# ------------------------------------------------------------------ fp32 carry

@pytest.mark.parametrize("T", [2, 3, 4])
@pytest.mark.parametrize("engine,operand,split", [("sparse", "f16", 3), ("sparse", "bf16", 3), ("dense", "f16", 3),
                                                  ("sparse", "f16", 2), ("dense", "bf16", 2)])
def test_f32_fused_equals_single_steps(T, engine, operand, split):
    wl = si.workload("1d5p_10240000", small=True)
    for n in (7, 257, 4099, wl["shape"][0]):
        x = wl["make_grid"](np.float32)[:n]
        xd, _ = to_dev(x, "f32")
        ref = run(sp.Plan(wl["coeffs"], (n,), carry="f32", engine=engine, operand=operand, split=split,
                          time_block=1), xd, 11)
        for th in (0, 1, 2, 5, 16, 1000):
            plan = sp.Plan(wl["coeffs"], (n,), carry="f32", engine=engine, operand=operand, split=split,
                           time_block=T, tile_h=th)
            assert plan.info()["time_block"] == T
            got = run(plan, xd, 11)
            assert np.array_equal(got, ref), (n, th, np.argwhere(got != ref)[:5])


@pytest.mark.parametrize("T", [2, 3, 4])
@pytest.mark.parametrize("engine", ["sparse", "dense"])
@pytest.mark.parametrize("n", LENGTHS)
def test_f32_fused_integer_exact(oracle_mod, T, engine, n):
    # all-ones taps (r = 1) on inputs in {1, 2} over nine steps: intermediate values
    # pass 2^11 (exact only as hi + lo), outputs exact in fp32; and mixed-sign
    # integer taps of radius 2 and 3
    cases = [(np.ones(3), 9, (1, 2))] + [(sparse_int_taps_1d(r, 40 + r), 5, (-2, 2)) for r in (2, 3)]
    for w, steps, (lo, hi) in cases:
        xd, x64 = to_dev(si.grid_integer((n,), lo, hi, 7 + n % 89), "f32")
        plan = sp.Plan(w, (n,), carry="f32", engine=engine, split=3, time_block=T)
        assert plan.info()["time_block"] == T
        ref = oracle_mod.apply(w, x64, steps)
        assert np.abs(oracle_mod.apply(w, x64, steps - 1)).max() < 65504
        got = run(plan, xd, steps)
        assert np.array_equal(got, ref), (w.shape, steps, np.argwhere(got != ref)[:5])


@pytest.mark.parametrize("T", [2, 4])
def test_f32_fused_aliasing(T):
    import torch
    wl = si.workload("1d3p_10240000", small=True)
    xd, _ = to_dev(wl["make_grid"](np.float32), "f32")
    plan = sp.Plan(wl["coeffs"], wl["shape"], carry="f32", engine="sparse", split=3, time_block=T)
    keep = xd.clone()
    for steps in (T, T + 1, 3 * T):
        y = xd.clone()
        plan.apply(y, y, steps)
        assert np.array_equal(from_dev(y), run(plan, xd, steps))
    assert torch.equal(xd, keep)


@pytest.mark.parametrize("T", [2, 3, 4])
def test_f32_full_size_equals_single_steps(T):
    wl = si.workload("1d3p_10240000")
    xd, _ = to_dev(wl["make_grid"](np.float32), "f32")
    a = run(sp.Plan(wl["coeffs"], wl["shape"], carry="f32", engine="sparse", split=3, time_block=T), xd, 12)
    b = run(sp.Plan(wl["coeffs"], wl["shape"], carry="f32", engine="sparse", split=3, time_block=1), xd, 12)
    assert np.array_equal(a, b)


# ----------------------------------------------------------------------------- 16-bit grid, split 3
# A 16-bit carry with split 3 on a 1-D line runs its fused launches on the
# fp32-level kernel: the 16-bit input widened exactly, the levels inside the launch
# kept as hi/lo pairs, and only the launch's output rounded to 16 bits.  So one
# launch equals the fp32-carry launch on the widened input, rounded; and the state
# is rounded once per T steps instead of once per step.

@pytest.mark.parametrize("T", [2, 3, 4])
@pytest.mark.parametrize("carry", ["f16", "bf16"])
def test_split3_16bit_launch_equals_rounded_fp32_launch(T, carry):
    import torch
    wl = si.workload("1d3p_10240000", small=True)
    xd, _ = to_dev(wl["make_grid"](np.float32), carry)
    p16 = sp.Plan(wl["coeffs"], wl["shape"], carry=carry, engine="sparse", split=3, time_block=T)
    p32 = sp.Plan(wl["coeffs"], wl["shape"], carry="f32", engine="sparse", split=3, operand=carry, time_block=T)
    assert p16.info()["time_block"] == T
    ref = xd.clone()
    for _ in range(3):
        y32 = torch.empty(ref.shape, dtype=torch.float32, device=ref.device)
        p32.apply(ref.float().contiguous(), y32, T)
        ref = y32.to(xd.dtype)
    got = torch.empty_like(xd)
    p16.apply(xd, got, 3 * T)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)


@pytest.mark.parametrize("T", [2, 3, 4])
@pytest.mark.parametrize("n", [7, 257, 10001, 123457])
def test_split3_16bit_integer_exact(oracle_mod, T, n):
    # remainders of every kind (two-step launch, single step) included
    for r in (1, 2, 3):
        w = sparse_int_taps_1d(r, 60 + r + T)
        xd, x64 = to_dev(si.grid_integer((n,), -2, 2, 11 + n % 97), "f16")
        plan = sp.Plan(w, (n,), carry="f16", engine="sparse", split=3, time_block=T)
        assert plan.info()["time_block"] == T
        for steps in (T, T + 1, 2 * T + 3):
            ref, peak = x64, 2.0
            for _ in range(steps):
                ref = oracle_mod.apply(w, ref, 1)
                peak = max(peak, float(np.abs(ref).max()))
            if peak >= 2048:
                continue
            got = run(plan, xd, steps)
            assert np.array_equal(got, ref), (r, steps, np.argwhere(got != ref)[:5])


def test_split3_16bit_aliasing():
    import torch
    wl = si.workload("1d3p_10240000", small=True)
    xd, _ = to_dev(wl["make_grid"](np.float32), "f16")
    plan = sp.Plan(wl["coeffs"], wl["shape"], carry="f16", engine="sparse", split=3, time_block=4)
    keep = xd.clone()
    for steps in (4, 5, 11):
        y = xd.clone()
        plan.apply(y, y, steps)
        assert np.array_equal(from_dev(y), run(plan, xd, steps))
    assert torch.equal(xd, keep)


def test_split3_16bit_meets_the_fp16_bound_on_1d3p(oracle_mod):
    # 1D3P at 100 steps: the 16-bit carry rounded every step misses the stated 2e-3
    # rel-RMS (2.92e-3); rounded once per fused launch of four steps it meets it
    from gpu_helpers import rel_errors
    wl = si.workload("1d3p_10240000")
    xd, x64 = to_dev(wl["make_grid"](np.float32), "f16")
    plan = sp.Plan(wl["coeffs"], wl["shape"], carry="f16", engine="sparse", split=3)
    assert plan.info()["time_block"] == 4
    got = run(plan, xd, wl["steps"])
    rms, mx = rel_errors(got, oracle_mod.apply(wl["coeffs"], x64, wl["steps"]))
    print("1D3P fp16 carry, split 3, four steps per launch: rel-RMS %.3e rel-max %.3e" % (rms, mx))
    assert rms <= 2e-3 and mx <= max(1e-2, wl["steps"] * 2.0 ** -12)
