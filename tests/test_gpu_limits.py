"""GPU parity at the size limits the planner accepts.

The longest lines (2^30 - 2 bytes of 16-bit state: 2^29 - 1 points; 2^28 - 1 for
paired-line bands and for fp32 state), grids larger than 2^32 bytes (lines
addressed past 4 GiB), tall grids one or three points wide.  The data are
integers (three taps of +-1, inputs in {-2..2}), so every value stays an exact
integer below 2^11 and the results must equal the oracle bit for bit at sampled
points (computed on their dependency cones) whatever the summation order; fused
and single-step launches must agree at every point.
"""
import numpy as np
import pytest

import paper_2506_22035_amd as sp
import stencil_inputs as si

pytestmark = pytest.mark.gpu

STEPS = 5


def int_taps(ndim, r, seed):
    """Centre tap 1 and two more taps of +-1 at random offsets."""
    rng = np.random.default_rng(seed)
    k = 2 * r + 1
    w = np.zeros((k,) * ndim)
    c = (r,) * ndim
    w[c] = 1.0
    cells = [i for i in np.ndindex(*w.shape) if i != c]
    for idx in rng.choice(len(cells), 2, replace=False):
        w[cells[idx]] = rng.choice([-1.0, 1.0])
    return w


def cone_values(oracle_mod, w, x8, steps, pts):
    """The oracle at points `pts` of S^steps(x), each from its dependency cone."""
    h = steps * ((w.shape[0] - 1) // 2)
    out = []
    for p in pts:
        lo = [max(0, c - h) for c in p]
        hi = [min(n, c + h + 1) for c, n in zip(p, x8.shape)]
        sub = x8[tuple(slice(a, b) for a, b in zip(lo, hi))].astype(np.float64)
        out.append(oracle_mod.apply(w, sub, steps)[tuple(c - a for c, a in zip(p, lo))])
    return np.array(out)


def sample_points(shape, seed, n=12):
    rng = np.random.default_rng(seed)
    corners = [tuple(0 if (k >> d) & 1 == 0 else s - 1 for d, s in enumerate(shape)) for k in range(2 ** len(shape))]
    mid = [tuple(s // 2 for s in shape), tuple(max(0, s - 3) for s in shape)]
    rand = [tuple(int(v) for v in (rng.integers(0, s) for s in shape)) for _ in range(n)]
    # the last columns of the first lines (masked lanes of a strip's ragged end sit there)
    ends = [tuple(min(i, s - 1) for s in shape[:-1]) + (max(0, shape[-1] - k),) for i in range(3) for k in (1, 2, 3)]
    return corners + mid + rand + ends


def check(oracle_mod, w, shape, carry, variants, seed):
    """Apply STEPS steps with each plan option set in `variants`; all must agree at
    every point and equal the oracle at the sampled points."""
    import torch
    x8 = si.grid_integer_int8(shape, -2, 2, seed)
    dt = torch.float16 if carry == "f16" else torch.float32
    x = torch.from_numpy(x8).to("cuda:0").to(dt)
    first = None
    for kw in variants:
        plan = sp.Plan(w, shape, carry=carry, **kw)
        want = kw.get("time_block", 1)
        got_tb = plan.info()["time_block"]
        assert got_tb == want, (kw, got_tb)
        y = torch.empty_like(x)
        plan.apply(x, y, STEPS)
        torch.cuda.synchronize()
        plan.close()
        if first is None:
            first = y
            pts = sample_points(shape, seed)
            got = np.array([float(y[p]) for p in pts])
            ref = cone_values(oracle_mod, w, x8, STEPS, pts)
            assert np.abs(ref).max() < 2048
            assert np.array_equal(got, ref), (kw, [(p, g, e) for p, g, e in zip(pts, got, ref) if g != e][:5])
        else:
            assert torch.equal(y, first), kw
            del y
    del x, first
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n", [(1 << 29) - 1, (1 << 29) - 8])
def test_longest_line_1d(oracle_mod, n):
    print("1-D line of %d points" % n, flush=True)
    check(oracle_mod, int_taps(1, 2, 3), (n,), "f16", [dict(time_block=1), dict(time_block=4)], 11)


def test_longest_line_2d_16point_bands(oracle_mod):
    shape = (3, (1 << 29) - 1)
    print("2-D", shape, flush=True)
    check(oracle_mod, int_taps(2, 3, 4), shape, "f16",
          [dict(band_height=16, time_block=1), dict(band_height=16, time_block=2)], 12)


def test_longest_line_2d_paired_bands(oracle_mod):
    shape = (5, (1 << 28) - 1)
    print("2-D", shape, flush=True)
    check(oracle_mod, int_taps(2, 3, 5), shape, "f16",
          [dict(band_height=8, time_block=1), dict(band_height=8, time_block=4)], 13)


def test_longest_line_2d_f32_split(oracle_mod):
    # two such fp32 lines span 2^31 - 8 bytes: the out-of-range offset of masked
    # lanes must lie beyond that, or their stores land in the second line's end
    shape = (3, (1 << 28) - 1)
    print("2-D fp32", shape, flush=True)
    check(oracle_mod, int_taps(2, 2, 6), shape, "f32",
          [dict(engine="sparse", split=3, time_block=1), dict(engine="sparse", split=3, time_block=2)], 14)


def test_grid_over_4gib_2d(oracle_mod):
    shape = ((1 << 15) + 100, 1 << 16)   # 2^31 + 6.5 M points, 4.3 GB of fp16
    print("2-D", shape, flush=True)
    check(oracle_mod, int_taps(2, 3, 7), shape, "f16",
          [dict(band_height=8, time_block=1), dict(band_height=8, time_block=4)], 15)


def test_grid_over_4gib_3d(oracle_mod):
    shape = (514, 2048, 2048)            # 2^31 + 8.4 M points
    print("3-D", shape, flush=True)
    check(oracle_mod, int_taps(3, 1, 8), shape, "f16", [dict(time_block=1)], 16)


@pytest.mark.parametrize("nx", [1, 3])
def test_tall_narrow_grids(oracle_mod, nx):
    shape = ((1 << 22) + 3, nx)
    print("2-D", shape, flush=True)
    check(oracle_mod, int_taps(2, 3, 9), shape, "f16",
          [dict(band_height=8, time_block=1), dict(band_height=8, time_block=4),
           dict(band_height=16, time_block=1), dict(band_height=16, time_block=2)], 17)


def test_longest_lines_direct_engine(oracle_mod):
    # fp32 1-D: 2^28 - 1 points (2^30 - 4 bytes); fp64 2-D: lines of 2^27 - 1 points
    print("1-D fp32 direct", flush=True)
    check(oracle_mod, int_taps(1, 3, 21), ((1 << 28) - 1,), "f32", [dict(engine="direct")], 31)
    import torch
    shape = (2, (1 << 27) - 1)
    print("2-D fp64 direct", shape, flush=True)
    w = int_taps(2, 2, 22)
    x8 = si.grid_integer_int8(shape, -2, 2, 32)
    x = torch.from_numpy(x8).to("cuda:0").to(torch.float64)
    y = torch.empty_like(x)
    plan = sp.Plan(w, shape, carry="f64")
    plan.apply(x, y, STEPS)
    torch.cuda.synchronize()
    plan.close()
    pts = sample_points(shape, 32)
    assert np.array_equal(np.array([float(y[p]) for p in pts]), cone_values(oracle_mod, w, x8, STEPS, pts))


def test_longest_line_3d(oracle_mod):
    shape = (3, 2, (1 << 29) - 1)
    print("3-D", shape, flush=True)
    check(oracle_mod, int_taps(3, 1, 23), shape, "f16", [dict(time_block=1)], 33)


def test_batch_at_the_limits():
    # a batched launch over the longest paired-band line, the longest 16-point line
    # and a 3-D grid: each equals its own apply with time_block = 2
    import torch
    cases = [((5, (1 << 28) - 1), int_taps(2, 3, 41), dict(band_height=8)),
             ((3, (1 << 29) - 1), int_taps(2, 2, 42), dict(band_height=16)),
             ((40, 64, 1000), int_taps(3, 1, 43), dict())]
    plans, xs, ys, refs = [], [], [], []
    for i, (shape, w, kw) in enumerate(cases):
        print("batch grid", shape, flush=True)
        x = torch.from_numpy(si.grid_integer_int8(shape, -2, 2, 50 + i)).to("cuda:0").to(torch.float16)
        p = sp.Plan(w, shape, carry="f16", **kw)
        r = torch.empty_like(x)
        sp.Plan(w, shape, carry="f16", time_block=2, **kw).apply(x, r, STEPS)
        plans.append(p)
        xs.append(x)
        ys.append(torch.empty_like(x))
        refs.append(r)
    sp.apply_batch(plans, xs, ys, [STEPS] * len(cases))
    torch.cuda.synchronize()
    for y, r, (shape, _, _) in zip(ys, refs, cases):
        assert torch.equal(y, r), shape
