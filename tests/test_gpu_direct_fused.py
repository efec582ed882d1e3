"""The direct (vector-ALU) engine with several steps per launch on 2-D grids.

Its multi-step kernel advances 32 x 32 tiles (16 x 16 on grids with fewer 32-point
tiles than CUs) with a halo of T r points T steps in LDS.  Every point sums its taps in the single-step kernel's order with the same
fused multiply-adds, so the two must agree bit for bit at any step count (fused
launches, the remainder launch, aliasing); against the fp64 oracle the results
meet the stated fp64 / fp32 tolerances, and integer data is exact."""
import time

import numpy as np
import pytest
import torch

import paper_2506_22035_amd as sp
import stencil_inputs as si
from gpu_helpers import empty_like_dev, from_dev, rel_errors, to_dev

pytestmark = pytest.mark.gpu

TOL = {"f64": (1e-13, 1e-13), "f32": (1e-5, 1e-5)}


def _coeffs(kind, r, rng):
    k = 2 * r + 1
    w = rng.uniform(-1, 1, (k, k)) / k
    if kind == "star":
        m = np.zeros((k, k), bool)
        m[r, :] = m[:, r] = True
        w = np.where(m, w, 0.0)
    elif kind == "holes":
        w[0, 0] = w[k - 1, 1] = 0.0
    return w


def _apply(plan, x, steps, alias=False):
    if alias:
        y = x.clone()
        plan.apply(y, y, steps)
    else:
        y = empty_like_dev(x)
        plan.apply(x, y, steps)
    torch.cuda.synchronize()
    return y


@pytest.mark.parametrize("carry", ["f64", "f32"])
@pytest.mark.parametrize("kind,r", [("box", 1), ("star", 1), ("holes", 2), ("box", 2), ("box", 3), ("star", 3), ("holes", 3)])
@pytest.mark.parametrize("shape", [(100, 77), (1, 1), (33, 250), (257, 64), (2, 300), (520, 530)])
def test_fused_equals_single_steps_bit_for_bit(carry, kind, r, shape):
    # grids of fewer 32-point tiles than CUs run 16-point tiles; (520, 530) runs 32
    rng = np.random.default_rng(r * 1000 + shape[0])
    w = _coeffs(kind, r, rng)
    xd, _ = to_dev(rng.uniform(-1, 1, shape), carry)
    fused = sp.Plan(w, shape, carry=carry, engine="direct")
    single = sp.Plan(w, shape, carry=carry, engine="direct", time_block=1)
    T = fused.info()["time_block"]
    assert T >= 2 and single.info()["time_block"] == 1
    for steps in sorted({1, 2, T - 1, T, T + 1, 2 * T + 3}):
        if steps < 1:
            continue
        a = _apply(fused, xd, steps)
        b = _apply(single, xd, steps)
        assert torch.equal(a, b), (carry, kind, r, shape, steps, T)
    # in == out through the fused launches and the remainder launch
    assert torch.equal(_apply(fused, xd, T + 1, alias=True), _apply(single, xd, T + 1))


@pytest.mark.parametrize("carry", ["f64", "f32"])
@pytest.mark.parametrize("r", [1, 2, 3])
def test_fused_against_the_oracle(oracle_mod, carry, r):
    rng = np.random.default_rng(40 + r)
    shape = (70, 95)
    w = _coeffs("box", r, rng)
    x = rng.uniform(0, 1, shape)
    xd, x64 = to_dev(x, carry)
    p = sp.Plan(w, shape, carry=carry, engine="direct")
    T = p.info()["time_block"]
    steps = 2 * T + 1
    got = from_dev(_apply(p, xd, steps))
    rms, mx = rel_errors(got, oracle_mod.apply(w, x64, steps))
    assert rms <= TOL[carry][0] and mx <= TOL[carry][1], (rms, mx, T)


@pytest.mark.parametrize("carry", ["f64", "f32"])
def test_fused_integer_exact(oracle_mod, carry):
    # integer taps and values: every partial sum is exact, so any summation order
    # gives the oracle's result exactly
    rng = np.random.default_rng(7)
    shape = (90, 130)
    w = rng.integers(-2, 3, (5, 5)).astype(np.float64)
    x = rng.integers(-4, 5, shape).astype(np.float64)
    xd, x64 = to_dev(x, carry)
    p = sp.Plan(w, shape, carry=carry, engine="direct")
    T = p.info()["time_block"]
    steps = 3  # |values| stay below 2^24 (fp32 exact): 4 * 50^3 < 2^24
    assert T >= steps
    got = from_dev(_apply(p, xd, steps))
    assert np.array_equal(got, oracle_mod.apply(w, x64, steps))


def test_depth_limits_and_launch_counts():
    rng = np.random.default_rng(3)
    for carry, r, want in [("f64", 1, 16), ("f64", 2, 8), ("f64", 3, 5), ("f64", 4, 1), ("f32", 1, 16),
                           ("f32", 3, 5), ("f32", 7, 1)]:
        # the tile with its halo, 32 + 2 T r points a side, stays within 64 (and its two
        # LDS copies within 64 KiB); at most 16 steps; radius 4 and up: one step
        p = sp.Plan(_coeffs("box", r, rng), (64, 64), carry=carry, engine="direct")
        assert p.info()["time_block"] == want, (carry, r)
        for steps in (0, 1, want, want + 1, 3 * want + 2):
            assert p.work(steps) == ((steps + want - 1) // want, 0)
        p.close()
    # asked-for depths are capped at the plan's maximum; 3-D grids run single steps
    p = sp.Plan(_coeffs("box", 3, rng), (64, 64), carry="f64", engine="direct", time_block=16)
    assert p.info()["time_block"] == 5
    p.close()
    w3 = rng.uniform(0, 1, (3, 3, 3))
    p = sp.Plan(w3, (8, 8, 8), carry="f64", engine="direct", time_block=4)
    assert p.info()["time_block"] == 1
    p.close()


def test_large_grids_stream_single_steps_by_default():
    w = _coeffs("box", 1, np.random.default_rng(1))
    assert sp.Plan(w, (1024, 1024), carry="f32", engine="direct").info()["time_block"] == 16
    assert sp.Plan(w, (1024, 1025), carry="f32", engine="direct").info()["time_block"] == 1


def test_box2d9p_f64_workload_in_one_launch(oracle_mod):
    # the fp64 workload (Box-2D9P, 256 x 256, 10 steps) is one launch of ten steps
    wl = si.workload("box2d9p_256_f64")
    xd, x64 = to_dev(wl["make_grid"](np.float64), "f64")
    p = sp.Plan(wl["coeffs"], wl["shape"], carry="f64")
    assert p.work(wl["steps"]) == (1, 0)
    got = from_dev(_apply(p, xd, wl["steps"]))
    rms, mx = rel_errors(got, oracle_mod.apply(wl["coeffs"], x64, wl["steps"]))
    assert rms <= 1e-13 and mx <= 1e-13


def test_batch_and_server_run_fused_direct_plans_alone():
    rng = np.random.default_rng(11)
    shapes = [(200, 150), (64, 300)]
    plans = [sp.Plan(_coeffs("box", 1 + i, rng), s, carry="f64", engine="direct") for i, s in enumerate(shapes)]
    xs = [to_dev(rng.uniform(-1, 1, s), "f64")[0] for s in shapes]
    steps = [23, 7]
    want = [_apply(p, x, n) for p, x, n in zip(plans, xs, steps)]
    outs = [empty_like_dev(x) for x in xs]
    sp.apply_batch(plans, xs, outs, steps)
    torch.cuda.synchronize()
    for o, w_ in zip(outs, want):
        assert torch.equal(o, w_)
    srv = sp.Server(1 << 30, 4)
    outs2 = [empty_like_dev(x) for x in xs]
    tickets = [srv.submit(p, x, o, n) for p, x, o, n in zip(plans, xs, outs2, steps)]
    t0 = time.time()
    pending = set(tickets)
    while pending:
        for t in list(pending):
            done, st = srv.poll(t)
            if done:
                assert st == 0
                pending.discard(t)
        assert time.time() - t0 < 60, "server did not finish"
        time.sleep(0.001)
    srv.close()
    for o, w_ in zip(outs2, want):
        assert torch.equal(o, w_)


def test_long_loops_of_fused_direct_launches():
    # more than 512 launches: cached body graphs of 256 fused launches, then the
    # remainder launch; the same bits as launches without graphs and as single steps
    rng = np.random.default_rng(5)
    w = rng.uniform(0, 1, (3, 3))
    w /= w.sum()
    shape = (40, 70)
    xd, _ = to_dev(rng.uniform(0, 1, shape), "f64")
    pg = sp.Plan(w, shape, carry="f64", engine="direct")
    pe = sp.Plan(w, shape, carry="f64", engine="direct", use_graph=False)
    p1 = sp.Plan(w, shape, carry="f64", engine="direct", time_block=1, use_graph=False)
    T = pg.info()["time_block"]
    steps = 513 * T + 5
    assert pg.work(steps)[0] == 514
    ref = _apply(p1, xd, steps)
    assert torch.equal(_apply(pe, xd, steps), ref)
    for _ in range(2):  # the second call replays the cached bodies
        assert torch.equal(_apply(pg, xd, steps), ref)
    assert torch.equal(_apply(pg, xd, steps, alias=True), ref)


def test_random_sweep_of_depths_shapes_and_taps(oracle_mod):
    # seeded: radius 1..4, ragged grids up to 400 x 400, fp32 / fp64, depth 0..16,
    # 0..39 steps, graphs on or off, in place or not; integer taps (three of +-1) and
    # inputs in {-2..2} keep every value an exact integer, so results equal the
    # oracle bit for bit (radius 4 has no fused kernel and runs single steps)
    import test_gpu_random_sweep as sweep
    rng = np.random.default_rng(2507)
    ran = 0
    for case in range(300):
        r = int(rng.integers(1, 5))
        shape = (int(rng.integers(1, 400)), int(rng.integers(1, 400)))
        carry = str(rng.choice(["f32", "f64"]))
        opts = dict(carry=carry, engine="direct", time_block=int(rng.integers(0, 17)),
                    use_graph=bool(rng.integers(0, 2)))
        steps = int(rng.integers(0, 40))
        in_place = bool(rng.integers(0, 2))
        w = sweep.int_taps(2, r, rng)
        x = si.grid_integer(shape, -2, 2, 5000 + case)
        ref, peak = x.astype(np.float64), 2.0
        for _ in range(steps):
            ref = oracle_mod.apply(w, ref, 1)
            peak = max(peak, float(np.abs(ref).max(initial=0)))
        if peak >= (2.0 ** 24 if carry == "f32" else 2.0 ** 53):
            continue
        p = sp.Plan(w, shape, **opts)
        xd = torch.from_numpy(x).to("cuda:0").to(torch.float32 if carry == "f32" else torch.float64)
        got = from_dev(_apply(p, xd, steps, alias=in_place))
        p.close()
        assert np.array_equal(got, ref), (case, r, shape, opts, steps, in_place)
        ran += 1
    assert ran >= 150
