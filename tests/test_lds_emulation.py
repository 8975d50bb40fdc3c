"""CPU emulation of the BF16 engine's LDS indexing (no GPU): the z strips written by the forward's pair stores,
the matrix-core adjoint's operand addressing, the fold's strip reads, and the epilogue's reuse of the z buffer.

The index expressions below restate those of the fused trial kernel (paper_1404_5344_amd/csrc/kernels_trial.hpp:
ZStrips, the BF16 pair stores of mfma_forward_chunk, the adjoint's A / B operand addresses, ZLines of the fold,
gsum) and of the host table builder (adjoint_operands_bf16 in foe_lib.hip).  The emulation checks, for 32 x 32 and
32 x 16 tiles, that every LDS access stays inside the buffer the kernel declares, that every strip half the adjoint
reads was written in the chunk (or meets a zero tap), and that the lane-level 16 x 16 x 32 products reproduce the
correlation g(r, c) = sum_{a,b} ka[a][b] z3(r + a, c + b) of the adjoint bank (Sec. II-C) exactly on the
BF16-rounded operands, so that a wrong stride, offset, copy or lane mapping fails here before a GPU run.
"""
import numpy as np
import pytest

R, KS = 3, 7
SW = 22                  # strip columns
KB16_COPY = 88


def layout(TW, TH, NC=16):
    H3, W3 = TH + 2 * R, TW + 2 * R
    NS = TW // 16
    STRIP_H = H3 * SW
    FILTER_H = NS * STRIP_H
    KSTEPS = (KS * SW + 31) // 32
    NB = (TH // 16) * NS
    return dict(H3=H3, W3=W3, NS=NS, STRIP_H=STRIP_H, FILTER_H=FILTER_H, KSTEPS=KSTEPS, NB=NB,
                HALVES=NC * FILTER_H + 8, NC=NC)


def bf16(v):
    """Round to BF16 (nearest, ties to even) and back to float64."""
    a = np.atleast_1d(np.asarray(v, np.float32)).copy()
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64).reshape(np.shape(v))


def store_strips(z3, L):
    """The forward's BF16 pair stores: the lanes of columns cc (even) and cc + 1 of a row swap values and store
    one word per filter at half rr * 22 + cc of strip 0 (cc < 22) and of strip 1 (16 <= cc < W3, at cc - 16)."""
    NC, H3, W3 = z3.shape
    buf = np.full(L["HALVES"], np.nan)                 # NaN marks halves that no store wrote
    buf[NC * L["FILTER_H"]:] = 0.0                      # the zero padding the kernel writes
    for f in range(NC):
        fo = f * L["FILTER_H"]
        for rr in range(H3):
            for cc in range(0, 40, 2):                  # patches reach column 39 (padding columns)
                z0 = z3[f, rr, cc] if cc < W3 else 0.0
                z1 = z3[f, rr, cc + 1] if cc + 1 < W3 else 0.0
                zh0 = rr * SW + cc
                zh1 = zh0 + L["STRIP_H"] - 16
                for ok, base in ((cc < SW, zh0), (16 <= cc < W3, zh1)):
                    if ok:
                        o = fo + base
                        assert o % 2 == 0 and 0 <= o and o + 2 <= NC * L["FILTER_H"]
                        buf[o] = bf16(z0)
                        buf[o + 1] = bf16(z1)
    return buf


def adjoint_operands_bf16(ka):
    """The host table of one filter: 2 copies of 176 halves, copy c half x = T[x + c - 16]."""
    halves = np.zeros((2, 2 * KB16_COPY))
    for copy in range(2):
        for x in range(2 * KB16_COPY):
            k = x + copy - 16
            v = ka[(k // SW) * KS + k % SW] if 0 <= k < KS * SW and k % SW < KS else 0.0
            halves[copy, x] = bf16(v)
    return halves.reshape(-1)


def emulate_tile_adjoint(z3, ka, L):
    """Lane-level emulation of the matrix-core adjoint of one chunk: gacc per wave (filter) and block."""
    NC = z3.shape[0]
    TH = (L["H3"] - 2 * R)
    TW = (L["W3"] - 2 * R)
    buf = store_strips(z3, L)
    out = np.zeros((NC, TH, TW))
    for wv in range(NC):
        tab = adjoint_operands_bf16(ka[wv])
        for q in range(L["NB"]):
            rb, sb = divmod(q, L["NS"])
            acc = np.zeros((16, 16))
            for st in range(L["KSTEPS"]):
                A = np.zeros((16, 32)); B = np.zeros((32, 16))
                for lane in range(64):
                    ln, lkb = lane & 15, (lane >> 4) & 3
                    ia = wv * L["FILTER_H"] + ln * SW + 8 * lkb + sb * L["STRIP_H"] + 16 * rb * SW + 32 * st
                    assert ia % 2 == 0 and 0 <= ia and ia + 8 <= L["HALVES"]
                    w = (ln & 1) * KB16_COPY + ((16 - ln - (ln & 1)) >> 1) + 4 * lkb + 16 * st
                    assert 0 <= w and w + 4 <= (ln & 1) * KB16_COPY + KB16_COPY   # inside the lane's copy
                    A[ln, 8 * lkb:8 * lkb + 8] = buf[ia:ia + 8]
                    B[8 * lkb:8 * lkb + 8, ln] = tab[2 * w:2 * w + 8]
                bad = np.isnan(A)
                assert not np.any(bad & (np.abs(B).sum(axis=1)[None, :] > 0)), "unwritten z read"
                A[bad] = 0.0
                acc += A @ B
            out[wv, 16 * rb:16 * rb + 16, 16 * sb:16 * sb + 16] = acc
    return out


@pytest.mark.parametrize("TW,TH", [(32, 32), (32, 16)])
def test_matrix_core_adjoint_indexing(TW, TH):
    L = layout(TW, TH)
    rng = np.random.default_rng(TH)
    NC = 16
    z3 = rng.uniform(-0.5, 0.5, (NC, TH + 2 * R, TW + 2 * R)).astype(np.float32)
    ka = (rng.standard_normal((NC, KS * KS)) * rng.choice([1e-6, 1e-2, 0.3, 5.0], (NC, 1))).astype(np.float32)
    got = emulate_tile_adjoint(z3, ka, L)
    zb, kb = bf16(z3), bf16(ka)
    ref = np.zeros((NC, TH, TW))
    for f in range(NC):
        k = kb[f].reshape(KS, KS)
        for a in range(KS):
            for b in range(KS):
                ref[f] += k[a, b] * zb[f, a:a + TH, b:b + TW]
    # the same BF16 operands: equal up to FP64 summation order
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_planted_mistakes_are_caught():
    L = layout(32, 32)
    rng = np.random.default_rng(3)
    z3 = rng.uniform(-0.5, 0.5, (16, 38, 38)).astype(np.float32)
    ka = rng.standard_normal((16, 49)).astype(np.float32)
    good = emulate_tile_adjoint(z3, ka, L)
    global adjoint_operands_bf16
    orig = adjoint_operands_bf16
    try:
        adjoint_operands_bf16 = lambda k: np.roll(orig(k), 2)   # tap table off by one word
        bad = emulate_tile_adjoint(z3, ka, L)
    finally:
        adjoint_operands_bf16 = orig
    assert np.abs(bad - good).max() > 1e-2 * np.abs(good).max()


@pytest.mark.parametrize("TW,TH", [(32, 32), (32, 16)])
def test_lds_budget_and_gsum_reuse(TW, TH):
    L = layout(TW, TH)
    NC, NG = 16, 16
    zp_floats = max(L["HALVES"] // 2, NG * TH * TW)
    assert NG * TH * TW <= zp_floats                 # the epilogue's gsum fits in the z buffer
    W6, H6 = TW + 4 * R, TH + 4 * R
    cols = W6 + 2
    copy_w = (H6 + 1) * cols
    copy1 = copy_w + ((23 - copy_w % 64) % 64 + 64) % 64
    u16w = copy1 + copy_w
    nslot = 2 * TW + 2 * (TH + 6)
    # u6, u16 planes, z buffer, fold partials, tap words, adjoint taps, wave maxima; reductions in doubles
    total = 4 * (H6 * W6 + u16w + zp_floats + nslot * R * NC + 1024 + NC * 52 + NG) + 8 * NG * 5
    assert total <= 160 * 1024, total


@pytest.mark.parametrize("TW,TH", [(32, 32), (32, 16)])
def test_fold_lines_read_the_intended_z(TW, TH):
    """Every fold read through the strips returns BF16(z3) at the (row, column) the FP32-plane form reads."""
    L = layout(TW, TH)
    NC = 16
    rng = np.random.default_rng(5)
    z3 = rng.uniform(-0.5, 0.5, (NC, L["H3"], L["W3"])).astype(np.float32)
    buf = store_strips(z3, L)
    zb = bf16(z3)

    def zread(base, r, s, ZS, ZL):
        o = base + r * ZL + s * ZS
        assert 0 <= o < NC * L["FILTER_H"]
        return buf[o]

    FB = 2
    for j in (0, 7, 15):
        for zrow, ZL in ((R, 1), (L["H3"] - 1 - R, -1)):
            for p0 in range(0, TW, FB):
                sb = int(p0 >= 16)
                base = j * L["FILTER_H"] + sb * L["STRIP_H"] + zrow * SW + p0 - 16 * sb
                for r in range(R):
                    for s in range(FB + KS - 1):
                        assert zread(base, r, s, 1, ZL * SW) == zb[j, zrow + r * ZL, p0 + s]
        for zcol, ZL in [(R, 1)] + [(c, -1) for c in range(R, TW + R)]:
            sb = int(zcol > 21)
            for p0 in range(0, TH, FB):
                base = j * L["FILTER_H"] + sb * L["STRIP_H"] + p0 * SW + zcol - 16 * sb
                for r in range(R):
                    for s in range(FB + KS - 1):
                        assert zread(base, r, s, SW, ZL) == zb[j, p0 + s, zcol + r * ZL]
