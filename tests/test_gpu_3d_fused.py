"""Two fused time steps per launch on 3-D grids (radius 1, 16-bit carry).

Each workgroup computes the intermediate step on a plane ring in LDS and the
second step from it; integer-valued cases are exact in fp16 and the fp32
accumulator, so every result must equal the oracle bit for bit, whatever the
shape (ragged, one point wide, thinner than a segment), the step count (odd
counts end with a single step) or the segment height.
"""
import numpy as np
import pytest

import paper_2506_22035_amd as sp
import stencil_inputs as si
from gpu_helpers import empty_like_dev, from_dev, rel_errors, to_dev

pytestmark = pytest.mark.gpu

SHAPES_3D = [(9, 10, 300), (5, 7, 257), (1, 1, 1), (20, 9, 520), (3, 4, 8), (17, 33, 241), (40, 6, 496)]


def run(plan, x_dev, steps):
    y = empty_like_dev(x_dev)
    plan.apply(x_dev, y, steps)
    return from_dev(y)


@pytest.mark.parametrize("engine", ["sparse", "dense"])
@pytest.mark.parametrize("kind", ["box", "star"])
@pytest.mark.parametrize("shape", SHAPES_3D)
def test_integer_exact_fused_3d(oracle_mod, engine, kind, shape):
    # taps in {-1, 0, 1}, inputs in {-1, 0, 1}: |values| <= 27^2 = 729 after two steps and
    # 27^3 < 2^15 after three, exact in fp16 sums below 2^11 ... checked against the oracle
    w = si.integer_coeffs(3, 1, -1, 1, 60, kind)
    x = si.grid_integer(shape, -1, 1, 70 + shape[2])
    xd, x64 = to_dev(x, "f16")
    plan = sp.Plan(w, shape, carry="f16", engine=engine, time_block=2)
    assert plan.info()["time_block"] == 2
    for steps in (1, 2, 3, 4):
        ref = oracle_mod.apply(w, x64, steps)
        if np.abs(ref).max() >= 2048 or np.abs(oracle_mod.apply(w, x64, max(steps - 1, 0))).max() >= 2048:
            continue
        got = run(plan, xd, steps)
        assert np.array_equal(got, ref), (steps, np.argwhere(got != ref)[:5])


@pytest.mark.parametrize("shape", [(23, 13, 264), (64, 9, 300)])
def test_fused_3d_segment_heights_agree(oracle_mod, shape):
    w = si.integer_coeffs(3, 1, -1, 1, 3, "box")
    x = si.grid_integer(shape, -1, 1, 4)
    xd, x64 = to_dev(x, "f16")
    ref = oracle_mod.apply(w, x64, 2)
    for th in (0, 1, 2, 5, 8, 100):
        plan = sp.Plan(w, shape, carry="f16", time_block=2, tile_h=th)
        assert np.array_equal(run(plan, xd, 2), ref), th


@pytest.mark.parametrize("carry", ["f16", "bf16"])
@pytest.mark.parametrize("name", ["box3d27p_512", "heat3d_256"])
def test_fused_3d_workload_tolerance_and_aliasing(oracle_mod, carry, name):
    import torch
    wl = si.workload(name, small=True)
    xd, x64 = to_dev(wl["make_grid"](), carry)
    plan = sp.Plan(wl["coeffs"], wl["shape"], carry=carry, time_block=2)
    got = run(plan, xd, wl["steps"])
    rms, mx = rel_errors(got, oracle_mod.apply(wl["coeffs"], x64, wl["steps"]))
    print("%s %s two fused steps: rel-RMS %.3e rel-max %.3e" % (name, carry, rms, mx))
    tol = {"f16": (2e-3, 1e-2), "bf16": (3e-2, 6e-2)}[carry]
    assert rms <= tol[0] and mx <= tol[1]
    keep = xd.clone()
    for steps in (1, 2, 3, 4):
        y = xd.clone()
        plan.apply(y, y, steps)
        assert np.array_equal(from_dev(y), run(plan, xd, steps)), steps
    assert torch.equal(xd, keep)
