"""CPU emulation of the FP32-plane LDS indexing of the fused trial kernel (no GPU): the z planes written by the
three forwards (direct VALU, FP32 matrix cores, split-FP16 matrix cores), the adjoint's window reads, the fold
items of the SYMMETRIC map (edge blocks and corner rows) with their partial slots, the epilogue's mirror terms,
and the epilogue's reuse of the z buffer as the group sums.

The index expressions restate those of paper_1404_5344_amd/csrc/kernels_trial.hpp (z_row_stride,
z_plane_stride, the forwards' z stores, the adjoint's zb / wrow reads, fold_block and ZLines, the fold item
decoding and slot layout, the epilogue's add(slot, d) calls, gsum) with the launch shapes of foe_lib.hip
(32 x 32 / 32 x 16 / 32 x 8 / 64 x 8 tiles, 1024 threads on the matrix-core engines and 512 on the VALU engine).  For
every tile of several images (corner, edge, ragged and interior tiles, images 4 and 5 pixels wide), the
emulation asserts that every LDS access lies inside the buffer the kernel declares, that every z value read
was written in the chunk and is not a padding column, that each fold partial has one writer per chunk, and
that the gradient it assembles equals the adjoint of the SYMMETRIC boundary extension computed directly
(Sec. II-C: grad F = sum_i K_i^T rho'(K_i u), the extension's adjoint folding the 3-wide border back onto the
image), so that a wrong stride, offset, slot or mirror index fails here before a GPU run.
"""
import numpy as np
import pytest

R, KS, KK, NC, KAP = 3, 7, 49, 16, 52
FWD_VALU, FWD_MFMA_F32, FWD_MFMA_F16X = 0, 1, 3
FB = 2


def z_row_stride(tw, fwd):
    return (tw + 2 * R + 7) // 8 * 8 if fwd == FWD_MFMA_F16X else tw + 2 * R


def z_plane_stride(tw, th, fwd):
    zw = z_row_stride(tw, fwd)
    if fwd == FWD_MFMA_F16X:
        p = (th + 2 * R) * zw
        return p + ((4 - p % 64) % 64 + 64) % 64
    return (th + 2 * R) * (tw + 2 * R)


def shape(th, fwd):
    """Launch shape of foe_lib.hip: (NT, BR, BC)."""
    br = 2 if th == 8 else 4
    if fwd == FWD_VALU:
        return 512, br, 2
    return 1024, br, (4 if th == 32 else 2)


class Lds:
    """A float LDS buffer that records writes and checks every access."""

    def __init__(self, n):
        self.v = np.full(n, np.nan)
        self.n = n

    def st(self, i, x):
        assert 0 <= i < self.n, (i, self.n)
        self.v[i] = x

    def ld(self, i):
        assert 0 <= i < self.n, (i, self.n)
        x = self.v[i]
        assert not np.isnan(x), ("read of an unwritten LDS word", i)
        return x


def forward_stores(zp, z3, fwd, TW, TH, PLANE, ZW):
    """The z stores of one chunk: every position (rr, cc) of the tile + 3 region of each plane, and the
    split forward's padding columns (its 2 x 8 patches run to column 8 NCB - 1), which must stay inside the
    padded row and are marked so that a read of them fails."""
    H3, W3 = TH + 2 * R, TW + 2 * R
    if fwd == FWD_MFMA_F16X:
        NCB = (W3 + 7) // 8
        assert 8 * NCB <= ZW
        for rr in range(H3):
            for cc in range(8 * NCB):
                for j in range(NC):
                    v = z3[j, rr, cc] if cc < W3 else np.inf   # padding: written, never to be read
                    zp.st(j * PLANE + rr * ZW + cc, v)
    elif fwd == FWD_MFMA_F32:
        PLANE3 = H3 * W3
        for g in range((PLANE3 + 15) // 16):
            for lm in range(16):
                p = g * 16 + lm
                if p >= PLANE3:
                    p = 0                                       # lanes past the plane take position 0
                r, c = divmod(p, W3)
                for j in range(NC):
                    zp.st(j * PLANE + r * ZW + c, z3[j, r, c])
    else:
        for idx in range(H3 * W3):
            r, c = divmod(idx, W3)
            for j in range(NC):
                zp.st(j * PLANE + r * ZW + c, z3[j, r, c])


def fold_block(zp, zl0, ZS, ZL, ka_s, kb0, KT, KL, fpart, out0, fpart_writes):
    Z = [[zp.ld(zl0 + r * ZL + s * ZS) for s in range(FB + KS - 1)] for r in range(R)]
    K = [[ka_s[kb0 + r * KL + t * KT] for t in range(KS)] for r in range(R)]
    for i in range(FB):
        v = [0.0, 0.0, 0.0]
        for t in range(KS):
            v[0] += K[0][t] * Z[0][i + t] + K[1][t] * Z[1][i + t] + K[2][t] * Z[2][i + t]
            v[1] += K[1][t] * Z[0][i + t] + K[2][t] * Z[1][i + t]
            v[2] += K[2][t] * Z[0][i + t]
        for d in range(R):
            o = out0 + (i * R + d) * NC
            assert 0 <= o < fpart.size
            fpart_writes.append(o)
            fpart[o] += v[d]


def emulate_tile(z_img, ka, H, W, x0, y0, TW, TH, fwd):
    """The gradient g on the tile (before the chain rule) as the kernel assembles it, for one chunk of NC
    filters; z_img: [NC, H, W] (zero off the image), ka: [NC, 49] adjoint taps."""
    NT, BR, BC = shape(TH, fwd)
    H3, W3 = TH + 2 * R, TW + 2 * R
    ZW, PLANE = z_row_stride(TW, fwd), z_plane_stride(TW, TH, fwd)
    GT = (TH // BR) * (TW // BC)
    NG = NT // GT
    FPG = NC // NG
    NPX = TH + 6
    NSLOT = 2 * TW + 2 * NPX
    # z on the tile + 3 region, zero off the image
    z3 = np.zeros((NC, H3, W3))
    for rr in range(H3):
        for cc in range(W3):
            gy, gx = y0 - R + rr, x0 - R + cc
            if 0 <= gy < H and 0 <= gx < W:
                z3[:, rr, cc] = z_img[:, gy, gx]
    zp = Lds(NC * PLANE)
    forward_stores(zp, z3, fwd, TW, TH, PLANE, ZW)
    ka_s = np.zeros(NC * KAP)
    for j in range(NC):
        ka_s[j * KAP:j * KAP + KK] = ka[j]
    # regular adjoint: group grp takes filters grp FPG .. grp FPG + FPG - 1, thread lt a BR x BC block
    acc = np.zeros((NG, TH, TW))
    for grp in range(NG):
        for lt in range(GT):
            col0 = (lt % (TW // BC)) * BC
            row0 = (lt // (TW // BC)) * BR
            for jj in range(FPG):
                j = grp * FPG + jj
                zb = j * PLANE + row0 * ZW + col0
                if ZW % 4 == 0 and BC % 4 == 0 and PLANE % 4 == 0:
                    assert zb % 4 == 0                           # float4 window reads
                else:
                    assert zb % 2 == 0                           # float2 window reads
                for q in range(BR + KS - 1):
                    wrow = [zp.ld(zb + q * ZW + s) for s in range(BC + KS - 1)]
                    assert all(np.isfinite(wrow)), "the adjoint read a padding column"
                    for ta in range(KS):
                        i = q - ta
                        if 0 <= i < BR:
                            for tb in range(KS):
                                for jx in range(BC):
                                    acc[grp, row0 + i, col0 + jx] += ka_s[j * KAP + ta * KS + tb] * wrow[jx + tb]
    # fold items
    fpart = np.zeros(NSLOT * R * NC)
    writes = []
    fold = y0 < R or y0 + TH > H - R or x0 < R or x0 + TW > W - R
    if fold:
        e_ylo, e_yhi = y0 == 0, y0 + TH >= H - (R - 1)
        e_xlo, e_xhi = x0 == 0, x0 + TW >= W - (R - 1)
        c_lo = R if y0 == 0 else 0
        c_h0, c_h1 = max(0, H - y0 - TH), min(R - 1, H - 1 - y0)
        c_hn = max(0, c_h1 - c_h0 + 1) if e_yhi else 0
        ncr = c_lo + c_hn
        f_y1 = NC * (TW // FB) if e_ylo else 0
        f_x0 = f_y1 + (NC * (TW // FB) if e_yhi else 0)
        f_x1 = f_x0 + (NC * (TH // FB) if e_xlo else 0)
        f_c0 = f_x1 + (NC * (TH // FB) if e_xhi else 0)
        f_c1 = f_c0 + (NC * ncr if e_xlo else 0)
        n_items = f_c1 + (NC * ncr if e_xhi else 0)
        for it in range(n_items):
            if it < f_x0:
                lo = it < f_y1
                loc = it - (0 if lo else f_y1)
                j, p0 = loc & (NC - 1), (loc // NC) * FB
                out0 = ((0 if lo else TW) + p0) * R * NC + j
                zrow = R if lo else H - 1 - y0 + R
                base = j * PLANE + zrow * ZW + p0
                # fold_block_y: the z lines as float2 pairs, the 24 taps from (R + 1) KS or 0 as float4 quads
                assert base % 2 == 0 and ZW % 2 == 0 and (j * KAP + ((R + 1) * KS if lo else 0)) % 4 == 0
                assert j * KAP + ((R + 1) * KS if lo else 0) + 24 <= (j + 1) * KAP
                if lo:
                    fold_block(zp, base, 1, ZW, ka_s, j * KAP + (R + 1) * KS, 1, KS, fpart, out0, writes)
                else:
                    fold_block(zp, base, 1, -ZW, ka_s, j * KAP + (R - 1) * KS, 1, -KS, fpart, out0, writes)
            elif it < f_c0:
                lo = it < f_x1
                loc = it - (f_x0 if lo else f_x1)
                j, p0 = loc & (NC - 1), (loc // NC) * FB
                out0 = (2 * TW + (0 if lo else NPX) + p0) * R * NC + j
                zcol = R if lo else W - 1 - x0 + R
                base = j * PLANE + p0 * ZW + zcol
                # fold_block_x: each three columns as a float2 pair from an even offset and a single value
                assert (j * PLANE + p0 * ZW) % 2 == 0 and ZW % 2 == 0 and (j * KAP) % 2 == 0
                if lo:
                    fold_block(zp, base, ZW, 1, ka_s, j * KAP + R + 1, KS, 1, fpart, out0, writes)
                else:
                    fold_block(zp, base, ZW, -1, ka_s, j * KAP + R - 1, KS, -1, fpart, out0, writes)
            else:
                e = 2 if it < f_c1 else 3
                loc = it - (f_c0 if e == 2 else f_c1)
                j, q = loc & (NC - 1), loc // NC
                zc0 = R if e == 2 else W - 1 - x0 + R
                zls = 1 if e == 2 else -1
                kb = j * KAP + (R + 1 if e == 2 else R - 1)
                kls = 1 if e == 2 else -1
                gy = -1 - q if q < c_lo else H + c_h0 + q - c_lo
                slot = 2 * TW + (e - 2) * NPX + (TH + q if q < c_lo else TH + R + c_h0 + q - c_lo)
                prow = gy - y0
                Z = [[0.0] * KS for _ in range(R)]
                K = [[0.0] * KS for _ in range(R)]
                for t in range(KS):
                    pr = min(max(prow + t, 0), H3 - 1)
                    for r in range(R):
                        Z[r][t] = zp.ld(j * PLANE + zc0 + pr * ZW + r * zls)
                        K[r][t] = ka_s[kb + r * kls + t * KS]
                v = [0.0, 0.0, 0.0]
                for t in range(KS):
                    v[0] += K[0][t] * Z[0][t] + K[1][t] * Z[1][t] + K[2][t] * Z[2][t]
                    v[1] += K[1][t] * Z[0][t] + K[2][t] * Z[1][t]
                    v[2] += K[2][t] * Z[0][t]
                for d in range(R):
                    o = slot * R * NC + j + d * NC
                    assert 0 <= o < fpart.size
                    writes.append(o)
                    fpart[o] += v[d]
        assert len(writes) == len(set(writes)), "a fold partial with two writers in one chunk"
    # epilogue: the group sums in the z buffer, then the mirror terms
    gsum = Lds(NC * PLANE)
    for grp in range(NG):
        for r in range(TH):
            for c in range(TW):
                gsum.st(grp * TH * TW + r * TW + c, acc[grp, r, c])
    g = np.full((TH, TW), np.nan)
    for i in range(TH):
        for jx in range(TW):
            py, px = y0 + i, x0 + jx
            if py >= H or px >= W:
                continue
            s = sum(gsum.ld(q * TH * TW + i * TW + jx) for q in range(NG))
            if fold:
                dyl, dyh, dxl, dxh = py, H - 1 - py, px, W - 1 - px
                xl, xh = 2 * TW, 2 * TW + NPX

                def add(slot, d):
                    o = (slot * R + d) * NC
                    assert 0 <= slot < NSLOT and 0 <= o and o + NC <= fpart.size
                    return fpart[o:o + NC].sum()
                if dyl < R:
                    s += add(jx, dyl)
                if dyh < R:
                    s += add(TW + jx, dyh)
                if dxl < R:
                    s += add(xl + i, dxl)
                if dxh < R:
                    s += add(xh + i, dxh)
                if dxl < R and dyl < R:
                    s += add(xl + TH + dyl, dxl)
                if dxl < R and dyh < R:
                    s += add(xl + TH + R + dyh, dxl)
                if dxh < R and dyl < R:
                    s += add(xh + TH + dyl, dxh)
                if dxh < R and dyh < R:
                    s += add(xh + TH + R + dyh, dxh)
            g[i, jx] = s
    return g


def reference_adjoint(z_img, ka, H, W):
    """sum_j of the SYMMETRIC extension's adjoint of the correlation with ka_j, from its definition: the
    correlation of the zero-padded z on the image extended by 3, each extended sample then added to the
    pixel it mirrors to (half-sample reflection, -1 - i -> i, H + i -> H - 1 - i)."""
    zpad = np.zeros((NC, H + 12, W + 12))
    zpad[:, 6:6 + H, 6:6 + W] = z_img
    g = np.zeros((H, W))
    for qy in range(-R, H + R):
        for qx in range(-R, W + R):
            win = zpad[:, qy + 3:qy + 10, qx + 3:qx + 10].reshape(NC, KK)
            v = float(np.sum(win * ka))
            my = -1 - qy if qy < 0 else (2 * H - 1 - qy if qy >= H else qy)
            mx = -1 - qx if qx < 0 else (2 * W - 1 - qx if qx >= W else qx)
            g[my, mx] += v
    return g


CASES = [  # (tile height, forward engine, image sizes)
    (32, FWD_MFMA_F16X, [(70, 75), (4, 5), (33, 34)]),
    (32, FWD_MFMA_F32, [(37, 64)]),
    (32, FWD_VALU, [(36, 40)]),
    (16, FWD_MFMA_F16X, [(35, 38), (5, 4)]),
    (8, FWD_MFMA_F16X, [(19, 35)]),
]
CASES_64 = [  # 64 x 8 tiles
    (8, FWD_MFMA_F16X, [(19, 70), (4, 5)]),
    (8, FWD_VALU, [(9, 67)]),
]


@pytest.mark.parametrize("TW,TH,fwd,sizes", [(32,) + c for c in CASES] + [(64,) + c for c in CASES_64])
def test_fp32_planes_fold_and_epilogue(TW, TH, fwd, sizes):
    rng = np.random.default_rng(TH * 10 + fwd)
    for H, W in sizes:
        z_img = rng.uniform(-0.5, 0.5, size=(NC, H, W))
        ka = rng.standard_normal((NC, KK))
        ref = reference_adjoint(z_img, ka, H, W)
        for y0 in range(0, H, TH):
            for x0 in range(0, W, TW):
                g = emulate_tile(z_img, ka, H, W, x0, y0, TW, TH, fwd)
                hh, ww = min(TH, H - y0), min(TW, W - x0)
                err = np.max(np.abs(g[:hh, :ww] - ref[y0:y0 + hh, x0:x0 + ww]))
                assert err <= 1e-10 * max(1.0, np.max(np.abs(ref))), (H, W, y0, x0, err)


def test_planted_mirror_mistake_is_caught():
    """The emulation fails when the high y edge takes its lines one row off (zrow = H - y0 + R)."""
    import inspect
    src = inspect.getsource(emulate_tile).replace("zrow = R if lo else H - 1 - y0 + R", "zrow = R if lo else H - y0 + R")
    ns = dict(globals())
    exec(src, ns)
    rng = np.random.default_rng(5)
    H, W = 20, 21
    z_img = rng.uniform(-0.5, 0.5, size=(NC, H, W))
    ka = rng.standard_normal((NC, KK))
    ref = reference_adjoint(z_img, ka, H, W)
    failed = False
    try:
        g = ns["emulate_tile"](z_img, ka, H, W, 0, 0, 32, 32, FWD_MFMA_F16X)
        failed = np.max(np.abs(g[:H, :W] - ref)) > 1e-6
    except AssertionError:
        failed = True
    assert failed
