"""Host-side checks of the offline transformation (no GPU needed).

The band matrix, strided swap, 2:4 compression and gfx950 lane packing of
SPIDER Sec. 3.1 are exposed by the library's host introspection calls; these
tests check them against the paper's worked example, against the definition of
the banded product (Sec. 3.1.1) and against the fp64 oracle.
"""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

import paper_2506_22035_amd as sp
import stencil_inputs as si

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def band(taps, L, width):
    """L x width band: row p holds the taps at columns p .. p + 2r (Sec. 3.1.1, Fig. 4)."""
    K = np.zeros((L, width))
    for p in range(L):
        K[p, p:p + len(taps)] = taps
    return K


# ------------------------------------------------------------------ the paper's rule


def test_paper_worked_example_fig5():
    # taps A..G as 1..7; the golden file lists the groups and compressed forms printed in Sec. 3.1.2
    r, L = 3, 8
    names = "ABCDEFG"
    taps = np.arange(1, 8, dtype=np.float64)
    K = band(taps, L, 2 * L)                       # 8 x 14 padded to 8 x 16 (Fig. 5 stage 1)
    perm = sp.swap_columns(L, 1)
    Ks = K[:, perm]                                 # stage 2
    vals, meta = sp.compress_24(Ks)                 # stage 3
    golden = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "fig5_r3_compression.txt")):
        if line.startswith("#") or not line.strip():
            continue
        g, v, m1, m2 = line.split()
        golden[g] = (v, int(m1, 2), int(m2, 2))

    def pattern(grp):
        return "".join("0" if x == 0 else names[int(x) - 1] for x in grp)

    found = set()
    for i in range(L):
        for g in range(L // 2):
            pat = pattern(Ks[i, 4 * g:4 * g + 4])
            if pat in golden:
                v, m1, m2 = golden[pat]
                got_v = "".join("0" if x == 0 else names[int(x) - 1] for x in vals[i, 2 * g:2 * g + 2])
                assert got_v == v and (meta[i, 2 * g], meta[i, 2 * g + 1]) == (m1, m2), (pat, got_v, meta[i])
                found.add(pat)
    assert found == set(golden), found


@pytest.mark.parametrize("r", range(0, 9))
def test_paper_swap_gives_24_for_every_radius(r):
    # L = 2r + 2 is the smallest band height with density <= 1/2 (the rule after Eq. 1)
    for L in range(2 * r + 2, 2 * r + 12, 2):
        K = band(np.arange(1, 2 * r + 2, dtype=float), L, 2 * L)
        perm = sp.swap_columns(L, 1)
        assert sorted(perm) == list(range(2 * L))
        assert np.array_equal(perm[perm], np.arange(2 * L))          # an involution
        Ks = K[:, perm]
        assert sorted(Ks.ravel()) == sorted(K.ravel())               # a pure permutation
        assert (np.count_nonzero(Ks.reshape(L, -1, 4), axis=2) <= 2).all()
        vals, meta = sp.compress_24(Ks)
        # decompress and compare bit-exactly
        D = np.zeros_like(Ks)
        for i in range(L):
            for c in range(L):
                g = c // 2
                if vals[i, c] != 0:
                    D[i, 4 * g + meta[i, c]] = vals[i, c]
        assert np.array_equal(D, Ks)


def test_too_small_band_is_not_24():
    # L = 2r fails the sparsity condition (density (2r+1)/(4r) > 1/2)
    r, L = 3, 6
    K = band(np.arange(1, 8, dtype=float), L, 2 * L)
    Ks = K[:, sp.swap_columns(L, 1)]
    assert (np.count_nonzero(Ks.reshape(L, -1, 4), axis=2) > 2).any()
    with pytest.raises(sp.SpiderError):
        sp.compress_24(Ks)


def test_swap_then_row_swap_preserves_product():
    # K' (sigma X) = K X exactly on small-integer data (Sec. 3.2, Fig. 6)
    rng = np.random.default_rng(0)
    for r in (1, 2, 3):
        L = 2 * r + 2
        K = band(rng.integers(-4, 5, 2 * r + 1).astype(float), L, 2 * L)
        X = rng.integers(-8, 9, (2 * L, 5)).astype(float)
        perm = sp.swap_columns(L, 1)
        assert np.array_equal(K[:, perm] @ X[perm], K @ X)


# ------------------------------------------------------------------ gfx950 gather order


def test_gather_positions_pair_rule():
    pos = sp.gather_positions()
    assert sorted(pos) == list(range(32))
    for g in range(8):
        grp = pos[4 * g:4 * g + 4]
        # two 32-bit column pairs, 16 columns apart
        assert grp[0] % 2 == 0 and grp[1] == grp[0] + 1 and grp[3] == grp[2] + 1
        assert grp[2] - grp[0] == 16


@pytest.mark.parametrize("r", range(1, 8))
def test_gather_band_is_24(r):
    pos = sp.gather_positions()
    # 16 outputs, window starts 8 columns before the chunk: output m uses columns 8+m-r .. 8+m+r
    K = np.zeros((16, 32))
    for m in range(16):
        K[m, 8 + m - r:8 + m + r + 1] = np.arange(1, 2 * r + 2)
    Kp = K[:, pos]
    assert (np.count_nonzero(Kp.reshape(16, 8, 4), axis=2) <= 2).all()


def _decode_smfmac_A(a_bits, idx, dtype):
    """Rebuild the dense 16 x 64 A operand from packed smfmac operands.

    Lane layout of v_smfmac_f32_16x16x64 on gfx950 (measured with one-hot probes):
    lane l holds row l % 16 and K slots 16 (l // 16) .. +15 as 4 groups of 4;
    compressed element e sits in group e // 2 at the position given by bits
    2e..2e+1 of the lane's 16-bit index field.
    """
    vals = a_bits.view(dtype).astype(np.float64) if a_bits.dtype != dtype else a_bits.astype(np.float64)
    A = np.zeros((16, 64))
    for lane in range(64):
        m, ga = lane % 16, lane // 16
        for e in range(8):
            p = (int(idx[lane]) >> (2 * e)) & 3
            k = 16 * ga + 4 * (e // 2) + p
            A[m, k] += vals[lane, e]
    return A


@pytest.mark.parametrize("operand,split", [("f16", 2), ("f16", 1), ("bf16", 2)])
@pytest.mark.parametrize("r", [1, 2, 3, 5, 7])
def test_pack_row_decodes_to_swapped_band(operand, split, r):
    rng = np.random.default_rng(r)
    row = rng.uniform(-1, 1, 2 * r + 1)
    a, idx, dense = sp.pack_row(row, r, operand, split)
    if operand == "f16":
        hi = row.astype(np.float16).astype(np.float64)
        lo = (row - hi).astype(np.float16).astype(np.float64) if split == 2 else np.zeros_like(row)
        A = _decode_smfmac_A(a, idx, np.float16)
        D = dense.view(np.float16).astype(np.float64)
    else:
        # taps exactly representable in fp32, so bf16 = round-to-nearest-even of the fp32 bits
        row = (np.round(row * 2 ** 20) / 2 ** 20).astype(np.float64)
        a, idx, dense = sp.pack_row(row, r, operand, split)

        def bf(v):
            u = np.asarray(v, dtype=np.float32).view(np.uint32).astype(np.uint64)
            u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
            return u.astype(np.uint32).view(np.float32).astype(np.float64)

        hi = bf(row)
        lo = bf(row - hi) if split == 2 else np.zeros_like(row)
        A = _decode_smfmac_A((a.astype(np.uint32) << 16).view(np.float32), idx, np.float32)
        D = (dense.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    pos = sp.gather_positions()
    Kh = np.zeros((16, 32))
    Kl = np.zeros((16, 32))
    for m in range(16):
        Kh[m, 8 + m - r:8 + m + r + 1] = hi
        Kl[m, 8 + m - r:8 + m + r + 1] = lo
    expect = np.concatenate([Kh[:, pos], Kl[:, pos]], axis=1)
    assert np.array_equal(A, expect)
    # dense operand: lane l holds row l % 16, K slots 8 (l // 16) .. +7 of K'_hi then K'_lo
    for lane in range(64):
        m, k0 = lane % 16, 8 * (lane // 16)
        assert np.array_equal(D[lane, :8], Kh[m, pos][k0:k0 + 8])
        assert np.array_equal(D[lane, 8:], Kl[m, pos][k0:k0 + 8])


def test_packed_band_product_matches_oracle(oracle_mod):
    # One kernel row applied through the packed operands (CPU emulation of the 16x16x64
    # product with the gather's B layout) equals the oracle's stencil on that line.
    r = 3
    rng = np.random.default_rng(9)
    row = rng.integers(-4, 5, 2 * r + 1).astype(np.float64)   # exact in fp16, lo part zero
    a, idx, _ = sp.pack_row(row, r, "f16", 2)
    A = _decode_smfmac_A(a, idx, np.float16)
    pos = sp.gather_positions()
    nx = 256
    x = rng.integers(-8, 9, nx).astype(np.float64)
    xp = np.concatenate([np.zeros(8), x, np.zeros(8)])
    out = np.zeros(nx)
    for n in range(16):                       # chunk n: outputs 16n .. 16n+15, window from 16n-8
        win = xp[16 * n:16 * n + 32]
        B = np.concatenate([win[pos], win[pos]])   # K slots 32..63 repeat the window for the lo part
        out[16 * n:16 * n + 16] = A @ B
    w = np.zeros((2 * r + 1, 2 * r + 1))
    w[r] = row
    ref = oracle_mod.apply(w, x[None, :].repeat(1, 0), 1)[0]
    assert np.array_equal(out, ref)


# ------------------------------------------------------------------ paired-line band (L = 8)


def test_pair_gather_positions_groups():
    pos = sp.pair_gather_positions()
    assert sorted(pos.tolist()) == list(range(16))
    for q in range(4):
        grp = pos[4 * q:4 * q + 4]
        # each 2:4 group joins a 32-bit column pair with the pair 8 columns to its right
        assert grp[1] == grp[0] + 1 and grp[3] == grp[2] + 1 and grp[2] == grp[0] + 8 and grp[0] % 2 == 0


def _pair_expected(w, r, k, hi_fn, lo_fn):
    pos = sp.pair_gather_positions()
    kw = 2 * r + 1
    A = np.zeros((16, 64))
    for phi in range(2):
        for m in range(8):
            for lam in range(2):
                row = 2 * k + lam - phi
                if not 0 <= row < kw:
                    continue
                for rho, part in enumerate((hi_fn(w[row]), lo_fn(w[row]))):
                    for s_ in range(16):
                        t = pos[s_] - 4 - m + r
                        if 0 <= t < kw:
                            A[8 * phi + m, 32 * lam + 16 * rho + s_] = part[t]
    return A


@pytest.mark.parametrize("split", [1, 2])
@pytest.mark.parametrize("r", [1, 2, 3])
def test_pack_pair_decodes_to_definition(r, split):
    rng = np.random.default_rng(40 + r)
    w = rng.uniform(-1, 1, (2 * r + 1, 2 * r + 1))

    def hi(v):
        return v.astype(np.float16).astype(np.float64)

    def lo(v):
        return (v - hi(v)).astype(np.float16).astype(np.float64) if split == 2 else np.zeros_like(v)

    for k in range(r + 1):
        a, idx, dense = sp.pack_pair(w, r, k, "f16", split)
        A = _decode_smfmac_A(a, idx, np.float16)
        E = _pair_expected(w, r, k, hi, lo)
        assert np.array_equal(A, E), k
        D = dense.view(np.float16).astype(np.float64)
        for lane in range(64):
            m, k0 = lane % 16, 8 * (lane // 16)
            assert np.array_equal(D[lane, :8], E[m, k0:k0 + 8])
            assert np.array_equal(D[lane, 8:], E[m, 32 + k0:32 + k0 + 8])


@pytest.mark.parametrize("r", [1, 2, 3])
def test_pair_band_product_matches_oracle(oracle_mod, r):
    # The whole 2-D step through the packed paired operands (CPU emulation of the
    # 16x16x64 products, B = the two windows of an input pair, each twice for hi/lo)
    # equals the oracle bit for bit on integer data.
    rng = np.random.default_rng(70 + r)
    w = rng.integers(-3, 4, (2 * r + 1, 2 * r + 1)).astype(np.float64)
    ny, nx = 14, 128
    x = rng.integers(-5, 6, (ny, nx)).astype(np.float64)
    As = [_decode_smfmac_A(*sp.pack_pair(w, r, k, "f16", 2)[:2], np.float16) for k in range(r + 1)]
    pos = sp.pair_gather_positions()
    xp = np.zeros((ny + 2 * r + 4, nx + 8))
    xp[r + 2:r + 2 + ny, 4:4 + nx] = x           # grid row y at r + 2 + y, column x at 4 + x
    out = np.zeros((ny + 1, nx))
    for i in range(0, ny, 2):                    # output pair (i, i + 1)
        acc = np.zeros((16, 16))
        for k in range(r + 1):
            j = i - r + 2 * k                    # input pair (j, j + 1)
            B = np.zeros((64, 16))
            for n in range(16):
                for lam in range(2):
                    win = xp[r + 2 + j + lam, 8 * n:8 * n + 16]    # columns 8n - 4 .. 8n + 11
                    B[32 * lam:32 * lam + 16, n] = win[pos]
                    B[32 * lam + 16:32 * lam + 32, n] = win[pos]
            acc += As[k] @ B
        for phi in range(2):
            for n in range(16):
                out[i + phi, 8 * n:8 * n + 8] = acc[8 * phi:8 * phi + 8, n]
    ref = oracle_mod.apply(w, x, 1)
    assert np.array_equal(out[:ny], ref)


# ------------------------------------------------------------------ rounding


def test_f16_split_matches_numpy_rounding():
    rng = np.random.default_rng(4)
    vals = np.concatenate([rng.uniform(-2, 2, 200), rng.uniform(-1e-5, 1e-5, 50), [65504.0, 1e-8, -3.0e-7]])
    for v in vals:
        row = np.array([0.0, v, 0.0])
        a, idx, dense = sp.pack_row(row, 1, "f16", 2)
        hi_bits = dense[0:16, :8].ravel()
        # output m = 8 - 1 + ... : find the hi tap in K'_hi of lane 0 (m = 0); tap index 1 sits at window col 8
        pos = list(sp.gather_positions())
        k = pos.index(8)
        lane = 0 + 16 * (k // 8)
        got_hi = dense[lane, k % 8].view(np.float16)
        got_lo = dense[lane, 8 + k % 8].view(np.float16)
        hi = np.float16(v)
        lo = np.float16(v - np.float64(hi))
        assert got_hi.view(np.uint16) == hi.view(np.uint16), v
        # a zero lo part is stored as +0 whatever its sign
        assert got_lo == lo and (lo == 0 or got_lo.view(np.uint16) == lo.view(np.uint16)), v


# ------------------------------------------------------------------ the C ABI


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "spider.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:spider_status|const char\*)\s+(spider_\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    names = _declared_functions()
    assert len(names) >= 17
    L = ctypes.CDLL(sp.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n


def test_invalid_arguments_rejected_without_gpu():
    L = sp.lib()
    w = np.ones((3, 3)) / 9
    shp = (ctypes.c_int64 * 2)(64, 64)
    h = ctypes.c_void_p()
    assert L.spider_plan(None, 2, shp, 1, None, ctypes.byref(h)) == 1
    assert L.spider_plan(w.ctypes.data, 4, shp, 1, None, ctypes.byref(h)) == 1
    assert L.spider_plan(w.ctypes.data, 0, shp, 1, None, ctypes.byref(h)) == 1
    long_line = (ctypes.c_int64 * 1)(1 << 29)   # 2^29 fp16 points = 2^30 bytes: too long
    assert L.spider_plan(w.ctypes.data, 1, long_line, 1, None, ctypes.byref(h)) == 2
    assert L.spider_plan(w.ctypes.data, 2, shp, 0, None, ctypes.byref(h)) == 1
    assert L.spider_plan(w.ctypes.data, 2, shp, 8, None, ctypes.byref(h)) == 1
    bad = (ctypes.c_int64 * 2)(0, 64)
    assert L.spider_plan(w.ctypes.data, 2, bad, 1, None, ctypes.byref(h)) == 1
    def opts(**kw):
        o = sp._Opts()
        L.spider_opts_default(ctypes.byref(o))
        for k, v in kw.items():
            setattr(o, k, v)
        return o

    o = opts(carry=0, engine=1)  # sparse engine with an fp64 carry
    assert L.spider_plan(w.ctypes.data, 2, shp, 1, ctypes.byref(o), ctypes.byref(h)) == 2
    assert "16-bit" in L.spider_last_error().decode()
    w3 = np.ones((3, 3, 3)) / 27
    shp3 = (ctypes.c_int64 * 3)(16, 16, 16)
    o = opts(carry=0, engine=1)  # no matrix engine takes an fp64 carry
    assert L.spider_plan(w3.ctypes.data, 3, shp3, 1, ctypes.byref(o), ctypes.byref(h)) == 2
    o = opts(carry=2, engine=1, split=3)  # with a 16-bit carry, split 3 exists on 1-D lines only
    assert L.spider_plan(w.ctypes.data, 2, shp, 1, ctypes.byref(o), ctypes.byref(h)) == 1
    assert "1-D" in L.spider_last_error().decode()
    o = opts(carry=2, engine=1, split=3)
    assert L.spider_plan(w3.ctypes.data, 3, shp3, 1, ctypes.byref(o), ctypes.byref(h)) == 1
    o = opts(carry=1, engine=1, split=4)
    assert L.spider_plan(w.ctypes.data, 2, shp, 1, ctypes.byref(o), ctypes.byref(h)) == 1
    o = opts(carry=2, engine=1, operand=3)  # operand must be the 16-bit carry type
    assert L.spider_plan(w.ctypes.data, 2, shp, 1, ctypes.byref(o), ctypes.byref(h)) == 1
    o = opts(carry=1, engine=2, operand=1)  # operands are 16-bit
    assert L.spider_plan(w.ctypes.data, 2, shp, 1, ctypes.byref(o), ctypes.byref(h)) == 1
    o = opts(band_height=12)
    assert L.spider_plan(w.ctypes.data, 2, shp, 1, ctypes.byref(o), ctypes.byref(h)) == 1
    o = opts(band_height=8)  # paired-line bands: radius <= 3
    w4 = np.ones((9, 9)) / 81
    assert L.spider_plan(w4.ctypes.data, 2, shp, 4, ctypes.byref(o), ctypes.byref(h)) == 2
    o = opts(band_height=8, carry=1, engine=3)  # and a matrix engine
    assert L.spider_plan(w.ctypes.data, 2, shp, 1, ctypes.byref(o), ctypes.byref(h)) == 2
    o = opts(row_swap=2)
    assert L.spider_plan(w.ctypes.data, 2, shp, 1, ctypes.byref(o), ctypes.byref(h)) == 1
    for tb in (-1, 17):
        o = opts(time_block=tb)
        assert L.spider_plan(w.ctypes.data, 2, shp, 1, ctypes.byref(o), ctypes.byref(h)) == 1
    # the explicit row swap: sparse engine, 16-bit carry, 2-D, band height 16, one step per launch
    for kw in (dict(engine=2), dict(band_height=8), dict(time_block=2), dict(time_block=3), dict(time_block=4), dict(carry=1, engine=1, split=3)):
        o = opts(row_swap=1, **kw)
        assert L.spider_plan(w.ctypes.data, 2, shp, 1, ctypes.byref(o), ctypes.byref(h)) == 2, kw
    o = opts(row_swap=1)
    assert L.spider_plan(w3.ctypes.data, 3, shp3, 1, ctypes.byref(o), ctypes.byref(h)) == 2
    assert L.spider_apply(None, None, None, 1, None) == 1
    assert L.spider_plan_destroy(None) == 0
    with pytest.raises(sp.SpiderError):
        sp.swap_columns(7, 1)


def test_binding_fails_loudly_without_library(tmp_path):
    # the product path has no fallback: with the library absent every call raises
    code = (
        "import numpy as np, paper_2506_22035_amd as sp\n"
        "sp.LIB_PATH = %r\n"
        "try:\n"
        "    sp.Plan(np.ones((3, 3)) / 9, (64, 64))\n"
        "except sp.SpiderError as e:\n"
        "    print('raised', e)\n"
        "else:\n"
        "    print('no error')\n" % str(tmp_path / "libspider.so"))
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.startswith("raised") and "not built" in out.stdout, out.stdout


def test_coefficient_beyond_operand_range_rejected():
    # fp16 operands hold |w| <= 65504; bf16 reaches ~3.4e38
    for v in (7e4, -1e6):
        row = np.array([0.25, v, 0.25])
        with pytest.raises(sp.SpiderError):
            sp.pack_row(row, 1, "f16", 2)
        with pytest.raises(sp.SpiderError):
            sp.pack_pair(np.full((3, 3), v), 1, 0, "f16", 2)
        sp.pack_row(row, 1, "bf16", 2)
    sp.pack_row(np.array([0.25, 65504.0, 0.25]), 1, "f16", 2)
