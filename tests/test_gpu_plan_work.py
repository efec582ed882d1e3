"""spider_plan_work: the launch and matrix-instruction counts of a time loop.

The expected instruction counts are the SQ_INSTS_MFMA hardware-counter sums that
rocprofv3 recorded for the same plans applied once (profiles/
matrix_instruction_counts.md, made by tests/mfma_count_check.py), so they pin the
host-side count to what the kernels really issue.  Plans are made without
autotuning, so their segment heights come from the planner's fixed rules."""
import pytest

import paper_2506_22035_amd as sp
import stencil_inputs as si

pytestmark = pytest.mark.gpu

# (workload, small recipe, plan options, steps, launches, SQ_INSTS_MFMA sum)
COUNTED = [
    ("1d3p_10240000", False, dict(carry="f16", engine="sparse", time_block=3), 100, 34, 6004800),
    ("1d3p_10240000", False, dict(carry="f32", engine="sparse", split=3, time_block=2), 100, 50, 10000800),
    ("1d5p_10240000", False, dict(carry="f32", engine="dense", split=3, time_block=4), 7, 3, 1546688),
    ("1d5p_10240000", False, dict(carry="f16", engine="dense", time_block=1), 3, 3, 384048),
    ("box3d27p_512", False, dict(carry="f16", engine="sparse"), 20, 20, 97320960),
    ("heat3d_256", False, dict(carry="f16", engine="dense"), 20, 20, 19660800),
    ("box2d49p_10240", True, dict(carry="f16", engine="sparse", time_block=4), 11, 4, 76512),
    ("box2d49p_10240", True, dict(carry="f32", engine="sparse", split=3, time_block=3), 10, 4, 128448),
    ("box2d49p_10240", True, dict(carry="f32", engine="sparse", split=2, time_block=2), 5, 3, 27744),
    ("star2d13p_8192", True, dict(carry="f32", engine="dense", split=3, time_block=1), 3, 3, 55296),
    ("box2d49p_10240", False, dict(carry="f32", engine="sparse", split=3, time_block=3), 3, 1, 12415680),
    ("1d3p_10240000", False, dict(carry="f16", engine="sparse", split=3, time_block=4), 11, 4, 1154648),
]


def _plan(name, small, kw):
    wl = si.workload(name, small=small)
    return sp.Plan(wl["coeffs"], wl["shape"], use_graph=False, **kw)


@pytest.mark.parametrize("case", range(len(COUNTED)))
def test_counts_equal_the_hardware_counter(case):
    name, small, kw, steps, launches, instructions = COUNTED[case]
    p = _plan(name, small, kw)
    try:
        assert p.work(steps) == (launches, instructions)
    finally:
        p.close()


def test_no_steps_is_no_work():
    p = _plan("box2d49p_10240", True, dict(carry="f16", engine="sparse", time_block=4))
    try:
        assert p.work(0) == (0, 0)
    finally:
        p.close()


def test_counts_add_up_over_whole_launches():
    # a loop of whole fused launches costs that many single fused launches
    p = _plan("box2d49p_10240", True, dict(carry="f16", engine="sparse", time_block=4))
    try:
        n1, m1 = p.work(4)
        n3, m3 = p.work(12)
        assert (n1, n3) == (1, 3) and m3 == 3 * m1
    finally:
        p.close()


def test_sparse_engine_halves_the_dense_instruction_count():
    # one smfmac 16x16x64 stands for two dense mfma 16x16x32 at the same geometry
    wl = si.workload("star2d13p_8192", small=True)
    ps = sp.Plan(wl["coeffs"], wl["shape"], carry="f16", engine="sparse", time_block=1, tile_h=16, use_graph=False)
    pd = sp.Plan(wl["coeffs"], wl["shape"], carry="f16", engine="dense", time_block=1, tile_h=16, use_graph=False)
    try:
        ns, ms = ps.work(3)
        nd, md = pd.work(3)
        assert ns == nd == 3 and md == 2 * ms > 0
    finally:
        ps.close()
        pd.close()


def test_direct_engine_issues_no_matrix_instructions():
    wl = si.workload("box2d9p_256_f64")
    p1 = sp.Plan(wl["coeffs"], wl["shape"], carry="f64", engine="direct", time_block=1, use_graph=False)
    pf = sp.Plan(wl["coeffs"], wl["shape"], carry="f64", engine="direct", use_graph=False)
    try:
        assert p1.work(7) == (7, 0)
        # the small grid runs its steps in LDS tiles, sixteen per launch
        assert pf.info()["time_block"] == 16 and pf.work(7) == (1, 0) and pf.work(33) == (3, 0)
    finally:
        p1.close()
        pf.close()


def test_uncounted_plans_report_no_count_but_their_launches():
    # 3-D grids with an fp32 carry keep no instruction count
    wl = si.workload("heat3d_256", small=True)
    p = sp.Plan(wl["coeffs"], wl["shape"], carry="f32", engine="sparse", split=3, use_graph=False)
    try:
        n, m = p.work(5)
        assert n == 5 and m is None
    finally:
        p.close()
