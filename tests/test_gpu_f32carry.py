"""GPU parity of the matrix engines with an fp32 carry (2-D).

With an fp32 carry every input value is split on load into 16-bit operands
x = x_hi + x_lo; with split 3 the kernel adds the products of the split
coefficients with both parts.  Integer cases whose values outgrow the 16-bit
significand (but stay exact in fp32) are therefore reproduced bit for bit over
several steps, which pins the x_lo path.  Without the input split (split 2) the
arithmetic is that of the 16-bit carry, so rounding the fp32 result to the
16-bit type must give the 16-bit carry's result bit for bit.
"""
import numpy as np
import pytest

import paper_2506_22035_amd as sp
import stencil_inputs as si
from gpu_helpers import empty_like_dev, from_dev, rel_errors, to_dev

pytestmark = pytest.mark.gpu

# stated tolerances (rel-RMS, rel-max) of the fp32 carry with split 3 versus the fp64 oracle
TOL3 = {"f16": (5e-5, 5e-5), "bf16": (2e-4, 2e-4)}

SHAPES = [(300, 520), (77, 301), (1, 1), (5, 8), (33, 256), (260, 1030)]


def run(plan, x_dev, steps):
    y = empty_like_dev(x_dev)
    plan.apply(x_dev, y, steps)
    return from_dev(y)


@pytest.mark.parametrize("band", [8, 16])
@pytest.mark.parametrize("operand", ["f16", "bf16"])
@pytest.mark.parametrize("engine", ["sparse", "dense"])
@pytest.mark.parametrize("shape", SHAPES)
def test_integer_exact_input_split(oracle_mod, operand, engine, shape, band):
    # All-ones 3x3 taps on inputs in {1, 2}: the inputs of the fifth step reach ~1e4,
    # beyond the 16-bit significand but exact as x_hi + x_lo, and the outputs (~1e5)
    # are exact in fp32.  The other cases mix signs.
    cases = [(np.ones((3, 3)), 5, (1, 2))]
    cases += [(si.integer_coeffs(2, r, -1, 1, 50 + r, kind), steps, (-2, 2))
              for kind, r, steps in [("box", 1, 4), ("star", 3, 2), ("box", 3, 2), ("box", 2, 2)]]
    for w, steps, (lo, hi) in cases:
        r = (w.shape[0] - 1) // 2
        x = si.grid_integer(shape, lo, hi, 60 + shape[1])
        xd, x64 = to_dev(x, "f32")
        plan = sp.Plan(w, shape, carry="f32", engine=engine, split=3, operand=operand, band_height=band)
        got = run(plan, xd, steps)
        ref = oracle_mod.apply(w, x64, steps)
        assert np.abs(oracle_mod.apply(w, x64, steps - 1)).max() < 65504
        assert np.array_equal(got, ref), (r, steps, np.argwhere(got != ref)[:5])


@pytest.mark.parametrize("operand", ["f16", "bf16"])
def test_without_input_split_large_values_are_rounded(oracle_mod, operand):
    # the same growing integer case without x_lo is not exact: the split is what makes it so
    shape = (64, 300)
    w = np.ones((3, 3))
    x = si.grid_integer(shape, 1, 2, 7)
    xd, x64 = to_dev(x, "f32")
    ref = oracle_mod.apply(w, x64, 5)
    got2 = run(sp.Plan(w, shape, carry="f32", engine="sparse", split=2, operand=operand), xd, 5)
    got3 = run(sp.Plan(w, shape, carry="f32", engine="sparse", split=3, operand=operand), xd, 5)
    assert np.array_equal(got3, ref)
    assert not np.array_equal(got2, ref)


@pytest.mark.parametrize("band", [16, 8])
@pytest.mark.parametrize("operand", ["f16", "bf16"])
@pytest.mark.parametrize("engine", ["sparse", "dense"])
def test_f32_carry_rounded_equals_16bit_carry(operand, engine, band):
    import torch
    wl = si.workload("box2d49p_10240", small=True)
    x16, _ = to_dev(wl["make_grid"](), operand)
    x32 = x16.to(torch.float32)
    for tb in ((1, 2, 3) if (engine == "sparse" and band == 8) else (1, 2)):
        p16 = sp.Plan(wl["coeffs"], wl["shape"], carry=operand, engine=engine, time_block=tb, band_height=band)
        y16 = torch.empty_like(x16)
        p16.apply(x16, y16, 9)
        # the fp32 16-point kernel runs one step per launch; paired bands fuse like the 16-bit plan
        p32 = sp.Plan(wl["coeffs"], wl["shape"], carry="f32", engine=engine, split=2, operand=operand,
                      band_height=band, time_block=tb if band == 8 else 1)
        y32 = torch.empty_like(x32)
        if band == 8:   # (16-point bands fuse bit-identically to single steps)
            assert p32.info()["time_block"] == p16.info()["time_block"]
        p32.apply(x32, y32, 9)
        torch.cuda.synchronize()
        assert torch.equal(y32.to(x16.dtype), y16), tb


@pytest.mark.parametrize("band", [8, 16])
@pytest.mark.parametrize("operand", ["f16", "bf16"])
@pytest.mark.parametrize("engine", ["sparse", "dense"])
@pytest.mark.parametrize("name", ["box2d49p_10240", "star2d13p_8192"])
def test_workload_tolerance_input_split(oracle_mod, operand, engine, name, band):
    wl = si.workload(name, small=True)
    xd, x64 = to_dev(wl["make_grid"](np.float32), "f32")
    plan = sp.Plan(wl["coeffs"], wl["shape"], carry="f32", engine=engine, split=3, operand=operand,
                   band_height=band)
    got = run(plan, xd, wl["steps"])
    rms, mx = rel_errors(got, oracle_mod.apply(wl["coeffs"], x64, wl["steps"]))
    print("%s f32 carry, %s operands, %s, band %d: rel-RMS %.3e rel-max %.3e" % (name, operand, engine, band, rms, mx))
    tr, tm = TOL3[operand]
    assert rms <= tr and mx <= tm


@pytest.mark.parametrize("r", [4, 5, 6, 7])
def test_large_radius_random(oracle_mod, r):
    rng = np.random.default_rng(r)
    w = rng.uniform(0, 1, (2 * r + 1, 2 * r + 1))
    w /= w.sum()
    shape = (97, 530)
    x = rng.uniform(0, 1, shape)
    xd, x64 = to_dev(x, "f32")
    for engine in ("sparse", "dense"):
        plan = sp.Plan(w, shape, carry="f32", engine=engine, split=3)
        rms, mx = rel_errors(run(plan, xd, 3), oracle_mod.apply(w, x64, 3))
        assert rms <= TOL3["f16"][0] and mx <= TOL3["f16"][1], engine


def test_tile_heights_and_aliasing(oracle_mod):
    import torch
    wl = si.workload("star2d13p_8192", small=True)
    xd, x64 = to_dev(wl["make_grid"](np.float32), "f32")
    res = []
    for th in (0, 1, 7, 16, 50, 1000):
        plan = sp.Plan(wl["coeffs"], wl["shape"], carry="f32", engine="sparse", split=3, tile_h=th)
        res.append(run(plan, xd, 5))
    for r_ in res[1:]:
        assert np.array_equal(r_, res[0])
    plan = sp.Plan(wl["coeffs"], wl["shape"], carry="f32", engine="sparse", split=3)
    keep = xd.clone()
    for steps in (0, 1, 2, 3):
        y = xd.clone()
        plan.apply(y, y, steps)
        ref = run(plan, xd, steps)
        assert np.array_equal(from_dev(y), ref)
    assert torch.equal(xd, keep)


def test_batch_and_server_accept_f32_carry(oracle_mod):
    # fp32-carry plans (2-D and 3-D) run their own time loops inside a batch and inside
    # the server's rounds: each result equals spider_apply of the same plan bit for bit,
    # also when mixed with 16-bit grids
    import time
    import torch
    cases = []
    for name in ("box2d49p_10240", "box3d27p_512"):
        wl = si.workload(name, small=True)
        xd, _ = to_dev(wl["make_grid"](np.float32), "f32")
        cases.append((sp.Plan(wl["coeffs"], wl["shape"], carry="f32", engine="sparse", split=3), xd, wl["steps"]))
    wl = si.workload("star2d13p_8192", small=True)
    x16, _ = to_dev(wl["make_grid"](), "f16")
    cases.append((sp.Plan(wl["coeffs"], wl["shape"], carry="f16"), x16, 7))
    want = [run(p, x, st) for p, x, st in cases]
    outs = [torch.empty_like(x) for _, x, _ in cases]
    sp.apply_batch([c[0] for c in cases], [c[1] for c in cases], outs, [c[2] for c in cases])
    for o, w_ in zip(outs, want):
        assert np.array_equal(from_dev(o), w_)
    srv = sp.Server(1 << 30)
    try:
        outs = [torch.empty_like(x) for _, x, _ in cases]
        tickets = [srv.submit(p, x, o, st) for (p, x, st), o in zip(cases, outs)]
        t0 = time.time()
        while not all(srv.poll(t)[0] for t in tickets):
            assert time.time() - t0 < 60
            time.sleep(0.001)
        assert all(srv.poll(t)[1] == 0 for t in tickets)
        for o, w_ in zip(outs, want):
            assert np.array_equal(from_dev(o), w_)
    finally:
        srv.close()


@pytest.mark.parametrize("operand", ["f16", "bf16"])
@pytest.mark.parametrize("shape", SHAPES + [(131, 700), (64, 233)])
def test_three_steps_integer_exact(oracle_mod, operand, shape):
    # three fused steps on the sparse engine; step counts that three does not divide
    # end with a two-step launch and a single step
    cases = [(np.ones((3, 3)), 5, (1, 2))]
    cases += [(si.integer_coeffs(2, r, -1, 1, 90 + r, kind), steps, (-2, 2))
              for kind, r, steps in [("box", 1, 4), ("star", 3, 3), ("box", 3, 3), ("box", 2, 5)]]
    for w, steps, (lo, hi) in cases:
        x = si.grid_integer(shape, lo, hi, 70 + shape[1])
        xd, x64 = to_dev(x, "f32")
        plan = sp.Plan(w, shape, carry="f32", engine="sparse", split=3, operand=operand, band_height=8,
                       time_block=3)
        assert plan.info()["time_block"] == 3
        ref = oracle_mod.apply(w, x64, steps)
        assert np.abs(oracle_mod.apply(w, x64, steps - 1)).max() < 65504
        got = run(plan, xd, steps)
        assert np.array_equal(got, ref), (w.shape, steps, np.argwhere(got != ref)[:5])


@pytest.mark.parametrize("operand", ["f16", "bf16"])
@pytest.mark.parametrize("name", ["box2d49p_10240", "star2d13p_8192"])
def test_three_steps_tolerance_tiles_and_aliasing(oracle_mod, operand, name):
    import torch
    wl = si.workload(name, small=True)
    xd, x64 = to_dev(wl["make_grid"](np.float32), "f32")
    ref = oracle_mod.apply(wl["coeffs"], x64, wl["steps"])
    res = []
    for th in (0, 2, 31, 64, 1000):
        plan = sp.Plan(wl["coeffs"], wl["shape"], carry="f32", engine="sparse", split=3, operand=operand,
                       time_block=3, tile_h=th)
        res.append(run(plan, xd, wl["steps"]))
    for r_ in res[1:]:
        assert np.array_equal(r_, res[0])
    rms, mx = rel_errors(res[0], ref)
    print("%s f32 carry, %s operands, three steps: rel-RMS %.3e rel-max %.3e" % (name, operand, rms, mx))
    tr, tm = TOL3[operand]
    assert rms <= tr and mx <= tm
    plan = sp.Plan(wl["coeffs"], wl["shape"], carry="f32", engine="sparse", split=3, operand=operand, time_block=3)
    keep = xd.clone()
    for steps in (3, 4, 5, 6):
        y = xd.clone()
        plan.apply(y, y, steps)
        assert np.array_equal(from_dev(y), run(plan, xd, steps)), steps
    assert torch.equal(xd, keep)
