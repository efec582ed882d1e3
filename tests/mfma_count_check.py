"""Matrix-instruction counts of spider_plan_work against the hardware counter.

usage (GPU, one case per process):
    rocprofv3 --pmc SQ_INSTS_MFMA --output-format csv -d <out> -o c<i> -- python3 tests/mfma_count_check.py <i>

Runs one plan once for a fixed step count and prints plan.work(steps); the sum of
SQ_INSTS_MFMA over the dispatches of that run must equal its second element.
Not collected by pytest (the counter needs the profiler).
"""
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import numpy as np
import torch
import paper_2506_22035_amd as sp
import stencil_inputs as si
CASES = [
    ("1d3p_10240000", dict(carry="f16", engine="sparse", time_block=3), 100, False),
    ("1d3p_10240000", dict(carry="f32", engine="sparse", split=3, time_block=2), 100, False),
    ("1d5p_10240000", dict(carry="f32", engine="dense", split=3, time_block=4), 7, False),
    ("1d5p_10240000", dict(carry="f16", engine="dense", time_block=1), 3, False),
    ("box3d27p_512", dict(carry="f16", engine="sparse"), 20, False),
    ("heat3d_256", dict(carry="f16", engine="dense"), 20, False),
    ("box2d49p_10240", dict(carry="f16", engine="sparse", time_block=4), 11, True),
    ("box2d49p_10240", dict(carry="f32", engine="sparse", split=3, time_block=3), 10, True),
    ("box2d49p_10240", dict(carry="f32", engine="sparse", split=2, time_block=2), 5, True),
    ("star2d13p_8192", dict(carry="f32", engine="dense", split=3, time_block=1), 3, True),
    ("box2d49p_10240", dict(carry="f32", engine="sparse", split=3, time_block=3), 3, False),
    ("1d3p_10240000", dict(carry="f16", engine="sparse", split=3, time_block=4), 11, False),
]
i = int(sys.argv[1])
name, kw, steps, small = CASES[i]
wl = si.workload(name, small=small)
dt = {"f16": torch.float16, "f32": torch.float32}[kw["carry"]]
x = torch.from_numpy(wl["make_grid"](np.float32)).to(dt).cuda()
y = torch.empty_like(x)
p = sp.Plan(wl["coeffs"], wl["shape"], use_graph=False, **kw)
p.apply(x, y, steps)
torch.cuda.synchronize()
print(json.dumps({"case": i, "name": name, "kw": kw, "steps": steps, "info": {k: v for k, v in p.info().items() if k in ("time_block", "tile_h", "tile_h2")},
                  "work": p.work(steps)}), flush=True)
