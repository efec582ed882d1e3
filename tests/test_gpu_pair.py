"""GPU parity of the paired-line band (band height 8, two output lines per instruction).

Same bar as the 16-point bands: integer cases bit for bit against the oracle
(every product and partial sum exact in the operand type and in fp32), workload
recipes within the stated tolerances, results independent of the segment height,
and the headline workload at full size on sampled points.
"""
import numpy as np
import pytest

import paper_2506_22035_amd as sp
import stencil_inputs as si
from gpu_helpers import empty_like_dev, from_dev, rel_errors, to_dev

pytestmark = pytest.mark.gpu

TOL = {"f16": (2e-3, 1e-2), "bf16": (3e-2, 6e-2)}
SHAPES = [(300, 520), (77, 301), (1, 1), (5, 8), (33, 256), (260, 1030), (2, 130), (41, 128)]


def run(plan, x_dev, steps):
    y = empty_like_dev(x_dev)
    plan.apply(x_dev, y, steps)
    return from_dev(y)


@pytest.mark.parametrize("engine", ["sparse", "dense"])
@pytest.mark.parametrize("shape", SHAPES)
def test_integer_exact_f16(oracle_mod, engine, shape):
    for kind, r in [("box", 1), ("box", 2), ("box", 3), ("star", 3), ("star", 1)]:
        w = si.integer_coeffs(2, r, -4, 4, 10 + r, kind)
        x = si.grid_integer(shape, -8, 8, 20 + shape[1])
        xd, x64 = to_dev(x, "f16")
        plan = sp.Plan(w, shape, carry="f16", engine=engine, band_height=8)
        info = plan.info()
        assert info["band_height"] == 8 and info["tile_h"] % 2 == 0 and info["nrows_nonzero"] == r + 1
        got = run(plan, xd, 1)
        ref = oracle_mod.apply(w, x64, 1)
        assert np.array_equal(got, ref), (kind, r, np.argwhere(got != ref)[:5])


@pytest.mark.parametrize("engine", ["sparse", "dense"])
@pytest.mark.parametrize("shape", [(300, 520), (77, 301)])
def test_integer_exact_bf16(oracle_mod, engine, shape):
    for kind, r in [("box", 1), ("box", 2), ("box", 3), ("star", 3)]:
        w = si.integer_coeffs(2, r, -2, 2, 30 + r, kind)
        x = si.grid_integer(shape, -2, 2, 40)
        xd, x64 = to_dev(x, "bf16")
        plan = sp.Plan(w, shape, carry="bf16", engine=engine, band_height=8)
        assert np.array_equal(run(plan, xd, 1), oracle_mod.apply(w, x64, 1)), (kind, r)


@pytest.mark.parametrize("steps", [2, 3, 5])
def test_integer_exact_multistep(oracle_mod, steps):
    shape = (131, 264)
    w = si.integer_coeffs(2, 1, -1, 1, 5, "box")
    x = si.grid_integer(shape, -2, 2, 6)
    xd, x64 = to_dev(x, "f16")
    ref = oracle_mod.apply(w, x64, steps)
    if np.abs(ref).max() >= 2048:
        # the values left the exact fp16 range: three taps of +-1 grow at most 3x per step
        w = np.zeros((3, 3))
        w[1, 1], w[0, 2], w[2, 0] = 1.0, -1.0, 1.0
        ref = oracle_mod.apply(w, x64, steps)
    assert np.abs(ref).max() < 2048
    plan = sp.Plan(w, shape, carry="f16", band_height=8)
    assert np.array_equal(run(plan, xd, steps), ref)


@pytest.mark.parametrize("carry", ["f16", "bf16"])
@pytest.mark.parametrize("engine", ["sparse", "dense"])
@pytest.mark.parametrize("name", ["box2d49p_10240", "star2d13p_8192"])
def test_workload_tolerance(oracle_mod, carry, engine, name):
    wl = si.workload(name, small=True)
    xd, x64 = to_dev(wl["make_grid"](), carry)
    plan = sp.Plan(wl["coeffs"], wl["shape"], carry=carry, engine=engine, band_height=8)
    got = run(plan, xd, wl["steps"])
    rms, mx = rel_errors(got, oracle_mod.apply(wl["coeffs"], x64, wl["steps"]))
    print("%s %s %s band 8: rel-RMS %.3e rel-max %.3e" % (name, carry, engine, rms, mx))
    assert rms <= TOL[carry][0] and mx <= TOL[carry][1]


@pytest.mark.parametrize("r", [1, 2])
def test_random_small_radius_tolerance(oracle_mod, r):
    rng = np.random.default_rng(100 + r)
    w = rng.uniform(0, 1, (2 * r + 1, 2 * r + 1))
    w /= w.sum()
    shape = (203, 517)
    x = rng.uniform(0, 1, shape)
    xd, x64 = to_dev(x, "f16")
    plan = sp.Plan(w, shape, carry="f16", band_height=8)
    rms, mx = rel_errors(run(plan, xd, 20), oracle_mod.apply(w, x64, 20))
    assert rms <= TOL["f16"][0] and mx <= TOL["f16"][1]


def test_tile_heights_agree_and_aliasing(oracle_mod):
    import torch
    wl = si.workload("star2d13p_8192", small=True)
    xd, _ = to_dev(wl["make_grid"](), "f16")
    res = []
    for th in (0, 1, 2, 7, 16, 50, 1000):
        plan = sp.Plan(wl["coeffs"], wl["shape"], carry="f16", band_height=8, tile_h=th)
        assert plan.info()["tile_h"] % 2 == 0
        res.append(run(plan, xd, 3))
    for r_ in res[1:]:
        assert np.array_equal(r_, res[0])
    plan = sp.Plan(wl["coeffs"], wl["shape"], carry="f16", band_height=8)
    keep = xd.clone()
    for steps in (0, 1, 2, 3):
        y = xd.clone()
        plan.apply(y, y, steps)
        assert np.array_equal(from_dev(y), run(plan, xd, steps))
    assert torch.equal(xd, keep)


def test_full_size_box2d49p_sampled(oracle_mod):
    from test_gpu_parity import _cone_samples
    wl = si.workload("box2d49p_10240")
    xd, x64 = to_dev(wl["make_grid"](), "f16")
    plan = sp.Plan(wl["coeffs"], wl["shape"], carry="f16", band_height=8)
    got = run(plan, xd, wl["steps"])
    rng = np.random.default_rng(2)
    n = wl["shape"][0]
    pts = [(0, 0), (n - 1, n - 1), (0, n - 1), (n - 1, 0), (1, 127), (2, 128), (n // 2, n // 2 + 3)]
    pts += [tuple(int(v) for v in rng.integers(0, n, 2)) for _ in range(10)]
    ref = _cone_samples(oracle_mod, wl["coeffs"], x64, wl["steps"], pts)
    rms, mx = rel_errors(np.array([got[p] for p in pts]), ref)
    print("full-size band 8 sampled rel-RMS %.3e rel-max %.3e" % (rms, mx))
    assert rms <= TOL["f16"][0] and mx <= TOL["f16"][1]


def test_batch_equals_two_step_apply():
    # batched launches run two fused steps, then one step for an odd count: equal to
    # apply with time_block = 2, bit for bit (odd and even counts, in == out too)
    import torch
    rng = np.random.default_rng(17)
    plans, ins, outs, steps, alone = [], [], [], [], []
    for r, shape, st in [(1, (130, 301), 5), (2, (77, 520), 4), (3, (203, 256), 6), (3, (9, 9), 3),
                         (3, (600, 1040), 9), (1, (64, 700), 1)]:
        w = rng.uniform(0, 1, (2 * r + 1, 2 * r + 1))
        w /= w.sum()
        xd, _ = to_dev(rng.uniform(0, 1, shape), "f16")
        plans.append(sp.Plan(w, shape, carry="f16", band_height=8))
        ins.append(xd)
        outs.append(torch.empty_like(xd))
        steps.append(st)
        alone.append(run(sp.Plan(w, shape, carry="f16", band_height=8, time_block=2), xd, st))
    sp.apply_batch(plans, ins, outs, steps)
    for o, ref in zip(outs, alone):
        assert np.array_equal(from_dev(o), ref)
    # in place (in == out), odd and even step counts
    for p, x, st, ref in zip(plans, ins, steps, alone):
        y = x.clone()
        sp.apply_batch([p], [y], [y], [st])
        assert np.array_equal(from_dev(y), ref)


# ------------------------------------------------------------------ two fused steps per launch


@pytest.mark.parametrize("engine", ["sparse", "dense"])
@pytest.mark.parametrize("shape", SHAPES)
def test_fused_integer_exact(oracle_mod, engine, shape):
    # two steps in one launch; integer data whose every step stays exact in fp16
    for kind, r, seed in [("box", 1, 3), ("box", 2, 4), ("star", 3, 5), ("box", 3, 6)]:
        w = si.integer_coeffs(2, r, -1, 1, seed, kind)
        x = si.grid_integer(shape, -2, 2, 50 + shape[0])
        xd, x64 = to_dev(x, "f16")
        ref1 = oracle_mod.apply(w, x64, 1)
        ref = oracle_mod.apply(w, x64, 2)
        if max(np.abs(ref1).max(), np.abs(ref).max()) > 2048:
            continue
        plan = sp.Plan(w, shape, carry="f16", engine=engine, band_height=8)
        assert plan.info()["time_block"] == 2 and plan.info()["tile_h2"] % 2 == 0
        got = run(plan, xd, 2)
        assert np.array_equal(got, ref), (kind, r, np.argwhere(got != ref)[:5])


@pytest.mark.parametrize("carry", ["f16", "bf16"])
def test_fused_matches_single_steps_within_rounding(oracle_mod, carry):
    wl = si.workload("box2d49p_10240", small=True)
    xd, x64 = to_dev(wl["make_grid"](), carry)
    ref = oracle_mod.apply(wl["coeffs"], x64, wl["steps"])
    outs = []
    for tb in (1, 2):
        plan = sp.Plan(wl["coeffs"], wl["shape"], carry=carry, band_height=8, time_block=tb)
        assert plan.info()["time_block"] == tb
        got = run(plan, xd, wl["steps"])
        rms, mx = rel_errors(got, ref)
        assert rms <= TOL[carry][0] and mx <= TOL[carry][1], tb
        outs.append(got)
    rms, _ = rel_errors(outs[1], outs[0])
    assert rms <= TOL[carry][0]


def test_fused_tile_heights_agree():
    wl = si.workload("box2d49p_10240", small=True)
    xd, _ = to_dev(wl["make_grid"](), "f16")
    res = []
    for th in (0, 2, 8, 31, 64, 301, 1000):
        plan = sp.Plan(wl["coeffs"], wl["shape"], carry="f16", band_height=8, tile_h=th)
        res.append(run(plan, xd, 4))
    for r_ in res[1:]:
        assert np.array_equal(r_, res[0])
