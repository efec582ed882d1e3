"""GPU parity of the 3-D matrix engines with an fp32 carry (radius 1).

As in 2-D, every input value is split on load into 16-bit operands
x = x_hi + x_lo, and with split 3 both parts are multiplied.  Integer cases whose
values outgrow the 16-bit significand but stay exact in fp32 are reproduced bit
for bit over several steps (pinning the x_lo path); without the split the
arithmetic is the 16-bit carry's, so the fp32 result rounded to 16 bits equals
the 16-bit carry's result bit for bit; the workload recipes meet the stated
fp32-carry tolerance.
"""
import numpy as np
import pytest

import paper_2506_22035_amd as sp
import stencil_inputs as si
from gpu_helpers import empty_like_dev, from_dev, rel_errors, to_dev

pytestmark = pytest.mark.gpu

TOL3 = {"f16": (5e-5, 5e-5), "bf16": (2e-4, 2e-4)}
SHAPES_3D = [(9, 10, 300), (5, 7, 257), (1, 1, 1), (20, 9, 520), (3, 4, 8), (17, 33, 64)]


def run(plan, x_dev, steps):
    y = empty_like_dev(x_dev)
    plan.apply(x_dev, y, steps)
    return from_dev(y)


@pytest.mark.parametrize("operand", ["f16", "bf16"])
@pytest.mark.parametrize("engine", ["sparse", "dense"])
@pytest.mark.parametrize("shape", SHAPES_3D)
def test_integer_exact_input_split_3d(oracle_mod, operand, engine, shape):
    # all-ones 3x3x3 taps on inputs in {1, 2}: the inputs of the fourth step reach ~4e4,
    # beyond the 16-bit significand but exact as x_hi + x_lo; outputs are exact in fp32
    cases = [(np.ones((3, 3, 3)), 4, (1, 2))]
    cases += [(si.integer_coeffs(3, 1, -1, 1, 40 + k, kind), 3, (-2, 2)) for k, kind in enumerate(["box", "star"])]
    for w, steps, (lo, hi) in cases:
        x = si.grid_integer(shape, lo, hi, 80 + shape[2])
        xd, x64 = to_dev(x, "f32")
        plan = sp.Plan(w, shape, carry="f32", engine=engine, split=3, operand=operand)
        assert plan.info()["engine"] == engine
        ref = oracle_mod.apply(w, x64, steps)
        assert np.abs(oracle_mod.apply(w, x64, steps - 1)).max() < 65504
        got = run(plan, xd, steps)
        assert np.array_equal(got, ref), (steps, np.argwhere(got != ref)[:5])


@pytest.mark.parametrize("operand", ["f16", "bf16"])
def test_without_input_split_large_values_are_rounded_3d(oracle_mod, operand):
    shape = (12, 20, 300)
    w = np.ones((3, 3, 3))
    xd, x64 = to_dev(si.grid_integer(shape, 1, 2, 9), "f32")
    ref = oracle_mod.apply(w, x64, 4)
    got2 = run(sp.Plan(w, shape, carry="f32", engine="sparse", split=2, operand=operand), xd, 4)
    got3 = run(sp.Plan(w, shape, carry="f32", engine="sparse", split=3, operand=operand), xd, 4)
    assert np.array_equal(got3, ref)
    assert not np.array_equal(got2, ref)


@pytest.mark.parametrize("operand", ["f16", "bf16"])
@pytest.mark.parametrize("engine", ["sparse", "dense"])
@pytest.mark.parametrize("name", ["box3d27p_512", "heat3d_256"])
def test_f32_carry_rounded_equals_16bit_carry_3d(operand, engine, name):
    # one step at a time, so rounding the fp32 result of the same arithmetic to 16 bits
    # must reproduce the 16-bit carry's step exactly
    import torch
    wl = si.workload(name, small=True)
    x16, _ = to_dev(wl["make_grid"](), operand)
    x32 = x16.to(torch.float32)
    p16 = sp.Plan(wl["coeffs"], wl["shape"], carry=operand, engine=engine)
    p32 = sp.Plan(wl["coeffs"], wl["shape"], carry="f32", engine=engine, split=2, operand=operand)
    y16 = torch.empty_like(x16)
    y32 = torch.empty_like(x32)
    p16.apply(x16, y16, 1)
    p32.apply(x32, y32, 1)
    torch.cuda.synchronize()
    assert torch.equal(y32.to(x16.dtype), y16)


@pytest.mark.parametrize("operand", ["f16", "bf16"])
@pytest.mark.parametrize("engine", ["sparse", "dense"])
@pytest.mark.parametrize("name", ["box3d27p_512", "heat3d_256"])
def test_workload_tolerance_input_split_3d(oracle_mod, operand, engine, name):
    wl = si.workload(name, small=True)
    xd, x64 = to_dev(wl["make_grid"](np.float32), "f32")
    plan = sp.Plan(wl["coeffs"], wl["shape"], carry="f32", engine=engine, split=3, operand=operand)
    got = run(plan, xd, wl["steps"])
    rms, mx = rel_errors(got, oracle_mod.apply(wl["coeffs"], x64, wl["steps"]))
    print("%s f32 carry 3-D, %s operands, %s: rel-RMS %.3e rel-max %.3e" % (name, operand, engine, rms, mx))
    tr, tm = TOL3[operand]
    assert rms <= tr and mx <= tm


def test_tile_heights_and_aliasing_3d():
    import torch
    wl = si.workload("box3d27p_512", small=True)
    xd, _ = to_dev(wl["make_grid"](np.float32), "f32")
    res = []
    for th in (0, 1, 3, 8, 100):
        plan = sp.Plan(wl["coeffs"], wl["shape"], carry="f32", engine="sparse", split=3, tile_h=th)
        res.append(run(plan, xd, 4))
    for r_ in res[1:]:
        assert np.array_equal(r_, res[0])
    plan = sp.Plan(wl["coeffs"], wl["shape"], carry="f32", engine="sparse", split=3)
    keep = xd.clone()
    for steps in (0, 1, 2, 3):
        y = xd.clone()
        plan.apply(y, y, steps)
        assert np.array_equal(from_dev(y), run(plan, xd, steps)), steps
    assert torch.equal(xd, keep)
