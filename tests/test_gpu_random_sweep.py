"""Seeded random sweep of plan options against the oracle, bit for bit.

Each case draws a dimension, radius, carry, engine, band height, fused depth,
segment height, grid shape (ragged, often smaller than a tile), step count and
in-place flag, with integer taps (three of +-1) and integer inputs in {-2..2}:
every value then stays an exact integer (below 2^11 for fp16, 2^8 for bf16), so
the result must equal the oracle exactly whatever the summation order.  Option
sets the planner rejects as unsupported are skipped and counted.
"""
import numpy as np
import pytest

import paper_2506_22035_amd as sp
import stencil_inputs as si
from gpu_helpers import from_dev

pytestmark = pytest.mark.gpu

NCASES = 1000


def int_taps(ndim, r, rng):
    k = 2 * r + 1
    w = np.zeros((k,) * ndim)
    c = (r,) * ndim
    w[c] = 1.0
    cells = [i for i in np.ndindex(*w.shape) if i != c]
    for idx in rng.choice(len(cells), 2, replace=False):
        w[cells[idx]] = rng.choice([-1.0, 1.0])
    return w


def draw_case(rng, scale=1):
    ndim = int(rng.choice([1, 2, 2, 2, 3]))
    carry = str(rng.choice(["f16", "f16", "bf16", "f32"]))
    if ndim == 1:
        r = int(rng.integers(1, 8))
        shape = (int(rng.integers(1, 6000 * scale * scale)),)
    elif ndim == 2:
        r = int(rng.integers(1, 8))
        shape = (int(rng.integers(1, 300 * scale)), int(rng.integers(1, 700 * scale)))
    else:
        r = int(rng.integers(1, 3))
        shape = tuple(int(v) for v in rng.integers(1, 40 * (2 if scale > 1 else 1), 3))
    opts = dict(carry=carry)
    if carry == "f32":
        opts["engine"] = str(rng.choice(["sparse", "dense", "direct"]))
        if opts["engine"] != "direct":
            opts["split"] = int(rng.choice([2, 3]))
    else:
        opts["engine"] = str(rng.choice(["sparse", "dense"]))
        # split 3 with a 16-bit grid: 1-D lines (rounded once per fused launch)
        opts["split"] = int(rng.choice([1, 2, 3] if ndim == 1 else [1, 2]))
    opts["band_height"] = int(rng.choice([0, 8, 16]))
    opts["time_block"] = int(rng.integers(0, 5))
    opts["tile_h"] = int(rng.choice([0, 0, 1, 2, 7, 16, 33, 100]))
    steps = int(rng.integers(0, 8))
    in_place = bool(rng.integers(0, 2))
    return ndim, r, shape, opts, steps, in_place


@pytest.mark.parametrize("seed,ncases,scale", [(2506, NCASES, 1), (77, 150, 6)])
def test_random_sweep(oracle_mod, seed, ncases, scale):
    # scale 6: grids up to 1800 x 4200 (2-D) and 80^3 (3-D), lines up to 216 000 points
    import torch
    rng = np.random.default_rng(seed)
    ran = skipped = 0
    for case in range(ncases):
        ndim, r, shape, opts, steps, in_place = draw_case(rng, scale)
        w = int_taps(ndim, r, rng)
        x = si.grid_integer(shape, -2, 2, 1000 + case)
        # every intermediate step must stay exact in the 16-bit type, not only the last
        ref, peak = x.astype(np.float64), 2.0
        for _ in range(steps):
            ref = oracle_mod.apply(w, ref, 1)
            peak = max(peak, float(np.abs(ref).max(initial=0)))
        if peak >= (256 if opts["carry"] == "bf16" else 2048):
            continue
        print("case %d: ndim %d r %d shape %s steps %d in_place %s %s" % (case, ndim, r, shape, steps, in_place, opts),
              flush=True)
        try:
            plan = sp.Plan(w, shape, **opts)
        except sp.SpiderError as e:
            assert e.status in (1, 2), e   # an option set the library does not run
            skipped += 1
            continue
        dt = {"f16": torch.float16, "bf16": torch.bfloat16, "f32": torch.float32}[opts["carry"]]
        xd = torch.from_numpy(x).to("cuda:0").to(dt)
        if in_place:
            y = xd.clone()
            plan.apply(y, y, steps)
        else:
            y = torch.empty_like(xd)
            plan.apply(xd, y, steps)
            assert torch.equal(xd, torch.from_numpy(x).to("cuda:0").to(dt))   # input untouched
        got = from_dev(y)
        plan.close()
        assert np.array_equal(got, ref), (case, np.argwhere(got != ref)[:5])
        ran += 1
    print("ran %d cases, %d option sets rejected" % (ran, skipped))
    assert ran >= ncases // 3
