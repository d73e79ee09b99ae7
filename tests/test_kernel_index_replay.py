"""CPU replays of the index arithmetic of the GPU kernels (host logic, no GPU).

* fp_staged_kernel and fp_staged_sp_kernel (one to four projections x 64 bins per workgroup, 16-line
  blocks staged in LDS; the groups chosen by the plan's rule, replayed here): every candidate a lane
  reads lies inside the staged segment of its line, [0, SEG) with SEG = 128 for three candidates per
  line and 224 for six, over random geometries at the edges of both pixel-size classes.  The replay
  follows the kernel's FP64 block anchor and FP32 per-line offsets (first candidate floor(v) + 1 and
  its offset a - sign(a) - a fract(v), v = u - 1/|a|), and checks both against FP64: the offset to
  2e-5, and no position outside the candidates has a hat weight above 1e-5.  Also the wavefront-to-
  line map of each group size, the closed-form hat weights and the bin-chunk-to-XCD map.
* The U-Net's direct convolutions: every staged patch and weight slot and every MFMA operand read of
  the persistent and general forms, the fused first two convolutions, the fused level-0 up-sampling,
  the weight-gradient kernel (staging, 8 x 8 transposes, operands, bias sums), the up-sampling kernels
  (operands and output coverage) and the half-wave exchange of the epilogues.
* prox_step2_kernel (two fused ROF dual steps on a 64 x 16 tile with a two-pixel halo): its loops,
  replayed with NaN-initialised LDS so that a read of an unset entry fails, equal two plain single steps
  exactly, on ragged and degenerate image shapes.
* filter4096_kernel: its index arithmetic, LDS layout and table lookups against numpy's FFT.
"""
import math

import numpy as np
import pytest

F32 = np.float32
RB = 16


def _proj(k, th, s, nx, ny, axis, shift):
    c, sn = math.cos(th), math.sin(th)
    rows = abs(c) >= abs(sn)
    a = s * c if rows else s * sn
    bb = s * sn if rows else s * c
    cx, cy = 0.5 * (nx - 1), 0.5 * (ny - 1)
    ci, cl = (cx, cy) if rows else (cy, cx)
    u_c = -(axis + shift) + a * ci + bb * cl
    return dict(k=k, rows=rows, sgn=a > 0, a=a, slope=-bb / a, rho=1.0 / abs(a), u_c=u_c, U0=u_c / a)


def staged_groups(P, nx, ny, nb, nc, cap=4):
    """The plan's staged groups: projections sorted by (walking axis, sign of a, slope); neighbours
    grouped greedily (up to cap: 4, or 2 for plans with few workgroups) while their first candidates
    span at most SEG - nc - 5 positions at every corner chunk and line block."""
    sseg = 128 if nc == 3 else 224
    v = sorted(P, key=lambda q: (not q["rows"], not q["sgn"], q["slope"]))
    nchunk = (nb + 63) // 64

    def fits(grp):
        if any(z["rows"] != grp[0]["rows"] for z in grp):
            return False
        nl = ny if grp[0]["rows"] else nx
        for jc in (0.0, 64.0 * (nchunk - 1)):
            for lc in (0.0, float(((nl - 1) // RB) * RB)):
                w = [z["U0"] + (jc + 63.0 * cj) / z["a"] + z["slope"] * (lc + (RB - 1) * cl) - z["rho"]
                     for z in grp for cj in (0, 1) for cl in (0, 1)]
                if max(w) - min(w) + nc + 5 > sseg:
                    return False
        return True
    groups, i = [], 0
    while i < len(v):
        e = i
        while e + 1 < len(v) and e + 1 - i < cap and fits(v[i:e + 2]):
            e += 1
        groups.append(tuple(v[i:e + 1]))
        i = e + 1
    return groups


def staged_columns(nx, ny, nb, angles, axis, shifts, s, cap=4):
    """(lowest, highest) LDS column read by fp_staged_kernel, the segment length and the number of
    projections that share a group with an earlier one, or None."""
    need = math.ceil(2 * math.sqrt(2) / s - 1e-9)
    nc = 3 if need <= 3 else (6 if need <= 6 else 0)
    if nc == 0:
        return None
    seg_len = 128 if nc == 3 else 224
    lo, hi = 10 ** 9, -10 ** 9
    r = np.arange(RB, dtype=F32)[:, None]
    P = [_proj(k, th, s, nx, ny, axis, shifts[k]) for k, th in enumerate(angles)]
    groups = staged_groups(P, nx, ny, nb, nc, cap)
    for grp in groups:
        n_lines = ny if grp[0]["rows"] else nx
        for j0 in range(0, nb, 64):
            for q in grp:
                q["u_first"] = (np.arange(j0, j0 + 64, dtype=np.float64) + q["u_c"]) / q["a"]
                q["blk_lo"] = (min((j0 + q["u_c"]) / q["a"], (j0 + 63 + q["u_c"]) / q["a"]) +
                               min(0.0, (RB - 1) * q["slope"]) - q["rho"])
            for b in range((n_lines + RB - 1) // RB):
                l0 = b * RB
                seg0 = math.floor(min(l0 * q["slope"] + q["blk_lo"] for q in grp)) - 2
                nl = min(RB, n_lines - l0)
                for q in grp:
                    a, rho = q["a"], q["rho"]
                    af, slopef = F32(a), F32(q["slope"])
                    c0 = F32(af - F32(math.copysign(1.0, a)))
                    ub = l0 * q["slope"] + q["u_first"]
                    ubase = np.floor(ub)
                    remv = (ub - ubase - rho).astype(F32)          # u - 1/|a| at the block's first line
                    v = (r[:nl] * slopef + remv[None]).astype(F32)
                    i0 = np.floor(v).astype(np.int64) + 1            # first candidate
                    d0 = (-af * (v - np.floor(v)) + c0).astype(F32)  # its offset t - j, a - sign(a) - a fract(v)
                    col = (ubase.astype(np.int64) - seg0)[None] + i0
                    lo, hi = min(lo, int(col.min())), max(hi, int(col.max()) + nc - 1)
                    # against FP64: the offset of the first candidate, and every position with a hat
                    # weight above 1e-5 lies among the nc candidates
                    u64 = ub[None] + r[:nl].astype(np.float64) * q["slope"]
                    d64 = a * (ubase[None] + i0 - u64)
                    assert np.max(np.abs(d0 - d64)) < 2e-5
                    for m in range(-1, nc + 1):
                        w = 1.0 - np.abs(d64 + m * a)
                        outside = (m < 0) | (m >= nc)
                        assert not np.any(outside & (w > 1e-5)), (q["k"], j0, b, m)
    return lo, hi, seg_len, sum(len(g) - 1 for g in groups)


@pytest.mark.parametrize("cap", [2, 4])
def test_fp_staging_bounds(cap):
    rng = np.random.default_rng(0)
    cases = [(256, 256, 256, np.arange(180) * math.pi / 180, 127.5, np.zeros(180), 1.0),
             (77, 53, 101, np.arange(61) * math.pi / 61 + rng.uniform(-.3, .3, 61) * math.pi / 61, 49.3,
              rng.normal(0, .5, 61), 1.0),
             (70, 70, 64, np.arange(50) * math.pi / 50, 30.8, np.zeros(50), 0.7),
             (40, 50, 100, np.arange(33) * math.pi / 33, 50.0, np.zeros(33), 1.6),
             (5, 3, 7, np.arange(4) * math.pi / 4, 3.0, np.zeros(4), 1.0),
             (1024, 1024, 1024, np.arange(128) * math.pi / 128, 511.5, np.zeros(128), 1.0)]   # TV workload
    # edges of the two classes: 3 candidates for s >= 2 sqrt 2 / 3, 6 for s >= 2 sqrt 2 / 6
    for s in (0.9429, 0.95, 1.0, 0.4715, 0.5, 0.94):
        cases.append((130, 110, 300, rng.uniform(0, 2 * math.pi, 120), 150.3, rng.normal(0, 3, 120), s))
    paired = 0
    for cs in cases:
        lo, hi, seg_len, n2 = staged_columns(*cs, cap=cap)
        assert 0 <= lo and hi < seg_len, (cs[:3], cs[6], lo, hi, seg_len)
        paired += n2
    assert paired > 100   # most cases group most of their projections


@pytest.mark.parametrize("P", [1, 2, 4])
def test_fp_wave_line_map(P):
    """Groups of one, two or four projections: wavefront w serves projection w / (4 / P) on lines
    w % (4 / P) + (4 / P) k of a block; every (projection, line) of a block is summed by exactly one
    wavefront, with accumulator k % 4, and a projection's partial sums meet in phase order."""
    wpp = 4 // P
    seen = {}
    for w in range(4):
        pw, ph = w // wpp, w % wpp
        for k in range(RB // wpp):
            line = ph + wpp * k
            assert 0 <= line < RB
            key = (pw, line)
            assert key not in seen
            seen[key] = (w, k & 3)
    assert sorted(seen) == [(p, r) for p in range(P) for r in range(RB)]


def test_fp_three_candidate_closed_form_weights():
    """The staged projector's weights for three candidates and 2/3 <= |a| <= 1, from f = fract(u - 1/|a|):
    w0 = |a| (1 - f), w1 = 1 - | |a| (2 - f) - 1 |, w2 = max(0, 2 - 3|a| + |a| f) equal the hat
    max(0, 1 - |d_n|) at the offsets d_n = |a| (1 + n - f) - 1 (in FP64, on a grid with the end points),
    and the candidates just before and after them have zero weight."""
    aa = np.concatenate([np.linspace(2.0 / 3.0, 1.0, 401), np.random.default_rng(1).uniform(2.0 / 3.0, 1.0, 4000)])
    f = np.concatenate([np.linspace(0.0, 1.0 - 2.0 ** -24, 257), np.random.default_rng(2).uniform(0.0, 1.0, 4000)])
    A, F = np.meshgrid(aa, f, indexing="ij")
    hat = lambda n: np.maximum(0.0, 1.0 - np.abs(A * (1 + n - F) - 1.0))
    np.testing.assert_allclose(A * (1.0 - F), hat(0), rtol=0, atol=1e-14)
    np.testing.assert_allclose(1.0 - np.abs(A * (2.0 - F) - 1.0), hat(1), rtol=0, atol=1e-14)
    np.testing.assert_allclose(np.clip(2.0 - 3.0 * A + A * F, 0.0, 1.0), hat(2), rtol=0, atol=1e-14)
    assert hat(-1).max() < 1e-12 and hat(3).max() < 1e-12


def _fp_chunk(i, n):
    if n % 16:
        return i
    x, k = i % 8, i // 8
    pair = x * (n // 16) + k // 2
    return n - 1 - pair if k % 2 else pair


@pytest.mark.parametrize("n", [1, 4, 8, 12, 16, 24, 32, 48, 64, 96])
def test_fp_chunk_remap(n):
    """The projector's column -> bin-chunk map is a permutation; when it remaps (n a multiple of 16),
    the columns that run on one XCD (i % 8) hold whole pairs of chunks symmetric about the centre."""
    chunks = [_fp_chunk(i, n) for i in range(n)]
    assert sorted(chunks) == list(range(n))
    if n % 16 == 0:
        for x in range(8):
            mine = {_fp_chunk(i, n) for i in range(x, n, 8)}
            assert mine == {n - 1 - c for c in mine}


# ------------------------------------------------------------------ direct 3x3 convolution (U-Net)
CT_W = 32
CT_PW = CT_W + 2


def _conv_ws(cpx):
    s = 9 * cpx
    while s % 8 != 1:
        s += 1
    return s


def _tap_row(tap):
    return (tap * 11) >> 5


def _persist_cth(cin, tn):
    """8-row tiles where the 8-row form's registers (weights, accumulators, two patches in flight, 24 more)
    stay within 240 per lane."""
    nstep = (9 * cin + 15) // 16
    wm = 4                                   # 8-row tiles: four wavefronts of two rows
    bm, bn = 8 // wm, tn // (4 // wm) // 32
    npv = (10 * CT_PW * (cin // 8) + 255) // 256
    return 8 if 4 * nstep * bn + 16 * bm * bn + 8 * npv + 24 <= 240 else 4


def _conv_tn(cin, n):
    return 128 if n >= 128 else (64 if n >= 64 else 32)


def _replay_general_chunk(X, Wt, sP, sW, b, y0, x0, n0, ch, cin, CC, CPX, CPP, WS, tn, N, H, W, seen_k):
    """One staged chunk of the general form: wavefront (wm, wn) owns output channels wn 32 .. + 31 and
    tile rows wm BM .. + BM - 1; per 16-channel slice and tap column it reads patch rows R = 0 .. BM + 1
    and the weights of the three tap rows, and output row i takes W[ty] x P[i + ty]."""
    wn_n = 4 if tn >= 128 else tn // 32
    wm_n = 4 // wn_n
    BM = 8 // wm_n
    for sl in range(CC // 16):
        for tx in range(3):
            for wave in range(4):
                wm, wn = divmod(wave, wn_n)
                gp, gw = {}, {}
                for lane in range(64):
                    col, half = lane & 31, lane >> 5
                    lp = (wm * BM * CT_PW + col) * CPP + half
                    lw = (wn * 32 + col) * WS + half
                    P = [sP[lp + (R * CT_PW + tx) * CPP + 2 * sl] for R in range(BM + 2)]
                    Wv = [sW[lw + (3 * ty + tx) * CPX + 2 * sl] for ty in range(3)]
                    for R in range(BM + 2):
                        gp.setdefault((R, lane // 8), set()).add((lp + (R * CT_PW + tx) * CPP + 2 * sl) % 8)
                    for ty in range(3):
                        gw.setdefault((ty, lane // 8), set()).add((lw + (3 * ty + tx) * CPX + 2 * sl) % 8)
                    c0 = ch * CC + 16 * sl + 8 * half
                    nn = wn * 32 + col
                    for ty in range(3):
                        k = (3 * ty + tx) * cin + c0
                        wref = Wt[n0 + nn, k:k + 8] if n0 + nn < N else np.zeros(8)
                        assert np.array_equal(Wv[ty], wref), (ch, sl, tx, ty, lane)
                        if wave == 0 and col == 0:
                            seen_k.append(k)
                        for i in range(BM):
                            yy, xx = y0 + wm * BM + i + ty - 1, x0 + col + tx - 1
                            ref = X[b, yy, xx, c0:c0 + 8] if (0 <= yy < H and 0 <= xx < W) else np.zeros(8)
                            assert np.array_equal(P[i + ty], ref), (ch, sl, tx, ty, i, lane)
                for g in list(gp.values()) + list(gw.values()):
                    assert len(g) == 8


@pytest.mark.parametrize("cin,H,W,n", [(8, 16, 16, 32), (16, 9, 40, 64), (32, 12, 33, 32), (64, 8, 64, 128),
                                       (128, 5, 31, 64), (256, 6, 20, 128), (64, 7, 35, 32), (8, 4, 8, 128),
                                       (32, 5, 70, 64), (128, 4, 32, 128), (256, 3, 9, 32)])
def test_conv3x3_patch_replay(cin, H, W, n):
    """The direct convolution's LDS staging and MFMA operand reads, replayed index by index for the form
    the library picks (persistent, CC = CIN, 8- or 4-row tiles, when TN x 9 x CIN <= 20480; else general
    with 8-row tiles, chunks of CC = min(CIN, 16 / 32 for TN = 128 / less) channels and the row-reusing
    read order of _replay_general_chunk).  Patch slot p CPP + c8 (CPP = CPX | 1) holds
    the input vector of pixel p, channels ch CC + 8 c8 (zeros outside the image); weight slot n WS + tap
    CPX + c8 holds W[n][tap CIN + ch CC + 8 c8].  Every lane of every (chunk, K step, row block, column
    block) reads, at its per-lane base plus the step's offset, the im2col value X[pixel + (ty-1, tx-1)][c]
    of its pixel and the weight of its output channel at one K index (the persistent form holds that
    weight in its register operand of the step); every K index is read once, in the
    global order with one chunk; the 8 lanes of a pass hit 8 distinct four-bank groups."""
    rng = np.random.default_rng(cin + H)
    B, N = 2, n
    X = rng.integers(1, 1000, (B, H, W, cin))
    Wt = rng.integers(1, 1000, (N, 9 * cin))
    tn = _conv_tn(cin, N)
    persist = tn * 9 * cin <= 20480
    CT_H = _persist_cth(cin, tn) if persist else 8
    CT_PIX = (CT_H + 2) * CT_PW
    cap = 16 if tn >= 128 else 32
    CC = cin if persist else min(cin, cap)
    CPX, NCH = CC // 8, cin // CC
    CPP, WS = CPX | 1, _conv_ws(CPX)
    NSTEP = (9 * CC + 15) // 16
    wm_n = 4 if (CT_H >= 8 or tn < 128) else 2   # persistent form (the general form: _replay_general_chunk)
    wn_n = 4 // wm_n
    BM, BN, WTN = CT_H // wm_n, (tn // wn_n) // 32, tn // wn_n
    tiles_x, tiles_y = -(-W // CT_W), -(-H // CT_H)
    for t in range(B * tiles_x * tiles_y):
        b, r = divmod(t, tiles_x * tiles_y)
        y0, x0 = (r // tiles_x) * CT_H, (r % tiles_x) * CT_W
        for n0 in range(0, N, tn):
            seen_k = []
            for ch in range(NCH):
                sP = np.full((CT_PIX * CPP, 8), -1, dtype=np.int64)
                for i in range(CT_PIX * CPX):
                    p, c8 = divmod(i, CPX)
                    py, px = divmod(p, CT_PW)
                    yy, xx = y0 - 1 + py, x0 - 1 + px
                    v = X[b, yy, xx, ch * CC + 8 * c8: ch * CC + 8 * c8 + 8] if (0 <= yy < H and 0 <= xx < W) \
                        else np.zeros(8, dtype=np.int64)
                    sP[p * CPP + c8] = v
                sW = np.full((tn * WS, 8), -1, dtype=np.int64)
                for j in range(tn * 9 * CPX):
                    nn, rr = divmod(j, 9 * CPX)
                    tap, c8 = divmod(rr, CPX)
                    k0 = tap * cin + ch * CC + 8 * c8
                    sW[nn * WS + tap * CPX + c8] = Wt[n0 + nn, k0:k0 + 8] if n0 + nn < N else 0
                if not persist:
                    _replay_general_chunk(X, Wt, sP, sW, b, y0, x0, n0, ch, cin, CC, CPX, CPP, WS, tn, N, H, W,
                                          seen_k)
                    continue
                for S in range(NSTEP):
                    for wave in range(4):
                        wm, wn = divmod(wave, wn_n)
                        for i in range(BM):
                            for j in range(BN):
                                ga, gw = {}, {}
                                for lane in range(64):
                                    col, half = lane & 31, lane >> 5
                                    la = ((wm * BM + i) * CT_PW + col) * CPP + (half if CC >= 16 else 0)
                                    lw = (wn * WTN + j * 32 + col) * WS + (half if CC >= 16 else 0)
                                    if CC >= 16:
                                        tap, c8b = (16 * S) // CC, ((16 * S) % CC) // 8
                                        oa = ((tap // 3) * CT_PW + tap % 3) * CPP + c8b
                                        ow = tap * CPX + c8b
                                        c8 = c8b + half
                                    else:
                                        tap = 2 * S + half
                                        if tap >= 9:
                                            continue
                                        oa, ow, c8 = (tap // 3) * CT_PW + tap % 3, tap, 0
                                    assert _tap_row(tap) == tap // 3
                                    k = tap * cin + ch * CC + 8 * c8
                                    if wave == 0 and i == 0 and j == 0 and col == 0:
                                        seen_k.append(k)
                                    yy = y0 + wm * BM + i + tap // 3 - 1
                                    xx = x0 + col + tap % 3 - 1
                                    ref = X[b, yy, xx, k - tap * cin: k - tap * cin + 8] if (
                                        0 <= yy < H and 0 <= xx < W) else np.zeros(8)
                                    assert np.array_equal(sP[la + oa], ref), (t, ch, S, lane)
                                    nn = wn * WTN + j * 32 + col
                                    wref = Wt[n0 + nn, k:k + 8] if n0 + nn < N else np.zeros(8)
                                    if persist:
                                        # register operand wr[S][j]: W[n][16 S + 8 half ..], zero past 9 CIN
                                        kr = 16 * S + 8 * half
                                        wreg = Wt[n0 + nn, kr:kr + 8] if (n0 + nn < N and kr < 9 * cin) \
                                            else np.zeros(8)
                                        assert np.array_equal(wreg, wref), (t, S, lane)
                                    else:
                                        assert np.array_equal(sW[lw + ow], wref), (t, ch, S, lane)
                                    ga.setdefault(lane // 8, set()).add((la + oa) % 8)
                                    gw.setdefault(lane // 8, set()).add((lw + ow) % 8)
                                for g in list(ga.values()) + list(gw.values()):
                                    assert len(g) == len([1 for _ in g]) and len(g) in (8,)
            assert sorted(seen_k) == list(range(0, 9 * cin, 8))
            if NCH == 1:
                assert seen_k == sorted(seen_k)


@pytest.mark.parametrize("C,H,W", [(32, 16, 64), (16, 12, 40), (8, 8, 33)])
def test_conv_pair0_patch_replay(C, H, W):
    """The fused first two convolutions: the 12 x 36 input tile staged per 8 x 32 output tile holds input
    pixel (y0 - 2 + iy, x0 - 2 + ix) (zero outside the image).  Wavefront w computes conv A for patch
    blocks pb = w, w + 4, ...: lane (col, half) is patch pixel 32 pb + col and supplies taps 8 half ..
    8 half + 7 of its B operand from input (py + t / 3, px + t % 3) of the tile, the neighbour
    (t / 3 - 1, t % 3 - 1) of activation pixel (y0 - 1 + py, x0 - 1 + px); after the half-wave exchange
    lane half h writes channel group g + h (g = 0, 2) of its pixel, so every (patch pixel, group < C / 8)
    is written exactly once and every read stays inside the tile."""
    CPX, IW, IH, PW = C // 8, CT_W + 4, 8 + 4, CT_PW
    PIX = 10 * PW
    rng = np.random.default_rng(C + H)
    X = rng.integers(1, 1000, (2, H, W))
    tiles_x, tiles_y = -(-W // CT_W), -(-H // 8)
    for t in range(2 * tiles_x * tiles_y):
        b, r = divmod(t, tiles_x * tiles_y)
        y0, x0 = (r // tiles_x) * 8, (r % tiles_x) * CT_W
        sIn = np.zeros(IH * IW, dtype=np.int64)
        for i in range(IH * IW):
            iy, ix = divmod(i, IW)
            yy, xx = y0 - 2 + iy, x0 - 2 + ix
            sIn[i] = X[b, yy, xx] if (0 <= yy < H and 0 <= xx < W) else 0
        written = np.zeros((PIX, CPX), dtype=np.int64)
        for wave in range(4):
            for pb in range(wave, -(-PIX // 32), 4):
                for lane in range(64):
                    col, half = lane & 31, lane >> 5
                    p = 32 * pb + col
                    pp = min(p, PIX - 1)
                    py, px = divmod(pp, PW)
                    ay, ax = y0 - 1 + py, x0 - 1 + px
                    for tp in range(8 * half, min(8 * half + 8, 9)):
                        k = (py + tp // 3) * IW + px + tp % 3
                        assert 0 <= k < IH * IW
                        ny, nx = ay + tp // 3 - 1, ax + tp % 3 - 1
                        ref = X[b, ny, nx] if (0 <= ny < H and 0 <= nx < W) else 0
                        if p < PIX:
                            assert sIn[k] == ref
                    for g in (0, 2):
                        grp = g + half
                        if p < PIX and grp < CPX:
                            written[p, grp] += 1
        assert (written == 1).all()


def _perm_b32(s0, s1, sel):
    """v_perm_b32: byte k of the result is byte sel[k] of the 8 bytes {s0 (bytes 4-7), s1 (bytes 0-3)}."""
    pool = [(s1 >> (8 * i)) & 255 for i in range(4)] + [(s0 >> (8 * i)) & 255 for i in range(4)]
    return sum(pool[(sel >> (8 * k)) & 255] << (8 * k) for k in range(4))


def _transpose8x8(inp):
    """The kernel's register transpose: inp[i] = 4 dwords (8 channels of pixel i, two per dword);
    out[j] = 4 dwords (8 pixels of channel j)."""
    out = []
    for j in range(8):
        sel = 0x07060302 if j & 1 else 0x05040100
        out.append([_perm_b32(inp[2 * q + 1][j >> 1], inp[2 * q][j >> 1], sel) for q in range(4)])
    return out


@pytest.mark.parametrize("cin,N,H,W", [(32, 32, 8, 32), (64, 32, 12, 40), (32, 64, 9, 33)])
def test_wgrad3x3_replay(cin, N, H, W):
    """The direct weight-gradient kernel, replayed in exact integers: the channel-major LDS staging of
    the input patch (three copies shifted by tx, from ten pixels per task) and of dZ (task d on thread
    160 + d or d - 96) through the 8 x 8 register transpose, the
    MFMA operands each wavefront reads (A = dZ[8 pixels][n], B = X[8 shifted pixels][c]), and the sums
    of the nine 32 x 32 tap blocks over the tiles of a split, against dW computed from the definition;
    the bias partials read from the staged dZ against the sums of dZ."""
    ZLD, XLD = 8 * CT_W + 8, 10 * CT_W + 8
    rng = np.random.default_rng(cin + N + H)
    B = 2
    X = rng.integers(0, 50, (B, H, W, cin))
    Z = rng.integers(0, 50, (B, H, W, N))
    # dW from the definition
    Xp = np.zeros((B, H + 2, W + 2, cin), dtype=np.int64)
    Xp[:, 1:-1, 1:-1] = X
    ref = np.zeros((N, 9, cin), dtype=np.int64)
    for t in range(9):
        ty, tx = divmod(t, 3)
        ref[:, t] = np.einsum("byxn,byxc->nc", Z, Xp[:, ty:ty + H, tx:tx + W])
    got = np.zeros_like(ref)
    bsum = np.zeros(N, dtype=np.int64)
    tiles_x, tiles_y = -(-W // CT_W), -(-H // 8)
    pack = lambda v: [int(v[2 * d]) | (int(v[2 * d + 1]) << 16) for d in range(4)]
    for t in range(B * tiles_x * tiles_y):
        b, r0 = divmod(t, tiles_x * tiles_y)
        y0, x0 = (r0 // tiles_x) * 8, (r0 % tiles_x) * CT_W
        for n0 in range(0, N, 32):
            for c0 in range(0, cin, 32):
                sX = np.full(3 * 32 * XLD, -1, dtype=np.int64)
                sZ = np.full(32 * ZLD, -1, dtype=np.int64)
                for tid in range(160):   # patch tasks: ten pixels give the three shifted copies
                    q, g, r = tid & 3, (tid >> 2) & 3, tid >> 4
                    yy = y0 - 1 + r
                    inp = []
                    for i in range(10):
                        xx = x0 - 1 + 8 * g + i
                        v = X[b, yy, xx, c0 + 8 * q:c0 + 8 * q + 8] if (0 <= yy < H and 0 <= xx < W) else [0] * 8
                        inp.append(pack(v))
                    for tx in range(3):
                        out = _transpose8x8(inp[tx:tx + 8])
                        for j in range(8):
                            base = (tx * 32 + 8 * q + j) * XLD + r * CT_W + 8 * g
                            assert (sX[base:base + 8] == -1).all()   # every slot written once
                            for d in range(4):
                                sX[base + 2 * d] = out[j][d] & 0xFFFF
                                sX[base + 2 * d + 1] = out[j][d] >> 16
                dtasks = sorted([t - 160 for t in range(160, 256)] + [96 + t for t in range(32)])
                assert dtasks == list(range(128))
                for tid in range(128):
                    g, q, y = tid & 3, (tid >> 2) & 3, tid >> 4
                    yy = y0 + y
                    inp = []
                    for i in range(8):
                        xx = x0 + 8 * g + i
                        v = Z[b, yy, xx, n0 + 8 * q:n0 + 8 * q + 8] if (yy < H and xx < W) else [0] * 8
                        inp.append(pack(v))
                    out = _transpose8x8(inp)
                    for j in range(8):
                        base = (8 * q + j) * ZLD + y * CT_W + 8 * g
                        for d in range(4):
                            sZ[base + 2 * d] = out[j][d] & 0xFFFF
                            sZ[base + 2 * d + 1] = out[j][d] >> 16
                if c0 == 0:   # bias partials: thread t sums pixels 32 (t % 8) .. + 31 of dZ row n0 + t / 8
                    for t8 in range(256):
                        seg = sZ[(t8 >> 3) * ZLD + 32 * (t8 & 7):(t8 >> 3) * ZLD + 32 * (t8 & 7) + 32]
                        assert (seg >= 0).all()
                        bsum[n0 + (t8 >> 3)] += int(seg.sum())
                for wave in range(4):
                    for kk in range(4):
                        y = 2 * wave + (kk >> 1)
                        A = np.zeros((32, 16), dtype=np.int64)
                        Bm = {t9: np.zeros((16, 32), dtype=np.int64) for t9 in range(9)}
                        for lane in range(64):
                            col, half = lane & 31, lane >> 5
                            cofs = 16 * (kk & 1) + 8 * half
                            a = sZ[col * ZLD + y * CT_W + cofs:col * ZLD + y * CT_W + cofs + 8]
                            assert (a >= 0).all()
                            A[col, 8 * half:8 * half + 8] = a
                            for ty in range(3):
                                for tx in range(3):
                                    o = (tx * 32 + col) * XLD + (y + ty) * CT_W + cofs
                                    bv = sX[o:o + 8]
                                    assert (bv >= 0).all()
                                    Bm[3 * ty + tx][8 * half:8 * half + 8, col] = bv
                        for t9 in range(9):
                            got[n0:n0 + 32, t9, c0:c0 + 32] += A @ Bm[t9]
    assert np.array_equal(got, ref)
    assert np.array_equal(bsum, Z.sum(axis=(0, 1, 2)))


def _permlane32_swap(x, y):
    """v_permlane32_swap: lanes 32..63 of the first operand trade places with lanes 0..31 of the second."""
    return x[:32] + y[:32], x[32:] + y[32:]


def _gather8(a, b):
    """The epilogues' half-wave exchange of (a, b) per lane: the first four and last four channels a lane
    stores (16 bytes), here as the first channel of each four-channel piece."""
    x, y = _permlane32_swap(a, b)
    return x, y


def test_gather8_lane_map():
    """After the exchange lane half h of pixel col holds channels 8 (g + h) .. 8 (g + h) + 7 in order, for
    every lane, given a = channels 8 g + 4 half .. + 3 and b = 8 (g + 1) + 4 half .. + 3."""
    for g in (0, 2):
        a = [(ln & 31, 8 * g + 4 * (ln >> 5)) for ln in range(64)]
        b = [(ln & 31, 8 * (g + 1) + 4 * (ln >> 5)) for ln in range(64)]
        lo, hi = _gather8(a, b)
        for ln in range(64):
            col, half = ln & 31, ln >> 5
            assert lo[ln] == (col, 8 * (g + half)) and hi[ln] == (col, 8 * (g + half) + 4)


def _up_ws(cpx):
    s = cpx
    while s % 8 != 1:
        s += 1
    return s


@pytest.mark.parametrize("cin,cout,H,W", [(64, 32, 8, 40), (128, 64, 5, 32), (32, 16, 4, 9), (16, 8, 6, 70), (128, 128, 3, 36)])
def test_up2x2_replay(cin, cout, H, W):
    """The up-sampling kernel's staging and reads, replayed: tile slot p CPP + c8 holds X[pixel p][8 c8..],
    weight slot n WS + c8 holds U[n][8 c8..]; every lane of every (K step, row block, column block) reads
    its pixel's and its output's vectors at the step's K; 8 lanes of a pass hit 8 distinct four-bank
    groups; the epilogue sends (pixel, n = d cout + co) to output pixel (2y + d / 2, 2x + d % 2), channel
    co, covering every output value exactly once."""
    rng = np.random.default_rng(cin + W)
    B, N = 2, 4 * cout
    X = rng.integers(1, 1000, (B, H, W, cin))
    U = rng.integers(1, 1000, (N, cin))
    tn = 128 if N >= 128 else (64 if N >= 64 else 32)
    CPX = cin // 8
    CPP, WS = CPX | 1, _up_ws(CPX)
    wm_n = 2 if tn >= 128 else 4
    wn_n = 4 // wm_n
    BM, BN, WTN = 4 // wm_n, (tn // wn_n) // 32, tn // wn_n
    lgc = cout.bit_length() - 1
    hit = np.zeros((B, 2 * H, 2 * W, cout), dtype=np.int64)
    tiles_x, tiles_y = -(-W // CT_W), -(-H // 4)
    for t in range(B * tiles_x * tiles_y):
        b, r = divmod(t, tiles_x * tiles_y)
        y0, x0 = (r // tiles_x) * 4, (r % tiles_x) * CT_W
        sP = np.full((4 * CT_W * CPP, 8), -1, dtype=np.int64)
        for i in range(4 * CT_W * CPX):
            p, c8 = divmod(i, CPX)
            py, px = divmod(p, CT_W)
            yy, xx = y0 + py, x0 + px
            sP[p * CPP + c8] = X[b, yy, xx, 8 * c8:8 * c8 + 8] if (yy < H and xx < W) else 0
        for n0 in range(0, N, tn):
            sW = np.full((tn * WS, 8), -1, dtype=np.int64)
            for i in range(tn * CPX):
                n, c8 = divmod(i, CPX)
                sW[n * WS + c8] = U[n0 + n, 8 * c8:8 * c8 + 8] if n0 + n < N else 0
            for S in range(cin // 16):
                for wave in range(4):
                    wm, wn = divmod(wave, wn_n)
                    for i in range(BM):
                        for j in range(BN):
                            ga, gw = {}, {}
                            for lane in range(64):
                                col, half = lane & 31, lane >> 5
                                la = ((wm * BM + i) * CT_W + col) * CPP + half
                                lw = (wn * WTN + j * 32 + col) * WS + half
                                c0 = 16 * S + 8 * half
                                yy, xx = y0 + wm * BM + i, x0 + col
                                ref = X[b, yy, xx, c0:c0 + 8] if (yy < H and xx < W) else np.zeros(8)
                                assert np.array_equal(sP[la + 2 * S], ref)
                                nn = wn * WTN + j * 32 + col
                                wref = U[n0 + nn, c0:c0 + 8] if n0 + nn < N else np.zeros(8)
                                assert np.array_equal(sW[lw + 2 * S], wref)
                                ga.setdefault(lane // 8, set()).add((la + 2 * S) % 8)
                                gw.setdefault(lane // 8, set()).add((lw + 2 * S) % 8)
                            for g in list(ga.values()) + list(gw.values()):
                                assert len(g) == 8
            # epilogue: register 4 g + q of block (j, i) = channel 8 g + 4 half + q of the block, pixel col;
            # groups g, g + 1 exchanged between the half-waves, after which lane half h stores the eight
            # channels 8 (g + h) .. + 7 of the block
            for wave in range(4):
                wm, wn = divmod(wave, wn_n)
                for i in range(BM):
                    for j in range(BN):
                        for lane in range(64):
                            col, half = lane & 31, lane >> 5
                            yy, xx = y0 + wm * BM + i, x0 + col
                            if yy >= H or xx >= W:
                                continue
                            for g in (0, 2):
                                a = [8 * g + 4 * (ln >> 5) for ln in range(64)]          # first channel held
                                bb = [8 * (g + 1) + 4 * (ln >> 5) for ln in range(64)]
                                lo, hi = _gather8(a, bb)
                                assert (lo[lane], hi[lane]) == (8 * (g + half), 8 * (g + half) + 4)
                                n = n0 + wn * WTN + j * 32 + 8 * g + 8 * half
                                if n >= N:
                                    continue
                                d, co = n >> lgc, n & (cout - 1)
                                assert (n + 7) >> lgc == d   # eight channels of one sub-pixel (cout >= 8)
                                hit[b, 2 * yy + (d >> 1), 2 * xx + (d & 1), co:co + 8] += 1
    assert (hit == 1).all()


@pytest.mark.parametrize("cin,cout,H,W", [(256, 128, 8, 64), (256, 128, 5, 40), (256, 32, 3, 33)])
def test_up2x2_wide_replay(cin, cout, H, W):
    """The up-sampling for 256 input channels: wavefront w holds tile row w, lane (col, half) loads channels
    16 S + 8 half .. + 7 of pixel (y0 + w, x0 + col) as its B operand of K step S and reads weight slot
    (32 j + col) WS + half + 2 S = U[n0 + 32 j + col][16 S + 8 half ..] for column block j; the epilogue
    sends (pixel, n = d cout + co) to output pixel (2y + d / 2, 2x + d % 2), channel co, covering every
    output value exactly once over the N / 128 workgroup columns."""
    rng = np.random.default_rng(cin + W + cout)
    B, N, TN = 2, 4 * cout, 128
    CPX = cin // 8
    WS = _up_ws(CPX)
    U = rng.integers(1, 1000, (N, cin))
    lgc = cout.bit_length() - 1
    hit = np.zeros((B, 2 * H, 2 * W, cout), dtype=np.int64)
    tiles_x, tiles_y = -(-W // CT_W), -(-H // 4)
    for n0 in range(0, N, TN):
        sW = np.full((TN * WS, 8), -1, dtype=np.int64)
        for i in range(TN * CPX):
            n, c8 = divmod(i, CPX)
            sW[n * WS + c8] = U[n0 + n, 8 * c8:8 * c8 + 8] if n0 + n < N else 0
        for lane in range(64):
            col, half = lane & 31, lane >> 5
            for j in range(TN // 32):
                lw = (j * 32 + col) * WS + half
                for S in range(cin // 16):
                    nn = n0 + j * 32 + col
                    ref = U[nn, 16 * S + 8 * half:16 * S + 8 * half + 8] if nn < N else np.zeros(8)
                    assert np.array_equal(sW[lw + 2 * S], ref)
        for t in range(B * tiles_x * tiles_y):
            b, r = divmod(t, tiles_x * tiles_y)
            y0, x0 = (r // tiles_x) * 4, (r % tiles_x) * CT_W
            for wave in range(4):
                for lane in range(64):
                    col, half = lane & 31, lane >> 5
                    yy, xx = y0 + wave, x0 + col
                    if yy >= H or xx >= W:
                        continue
                    for j in range(TN // 32):
                        for g in (0, 2):
                            n = n0 + j * 32 + 8 * g + 8 * half
                            if n >= N:
                                continue
                            d, co = n >> lgc, n & (cout - 1)
                            assert (n + 7) >> lgc == d
                            hit[b, 2 * yy + (d >> 1), 2 * xx + (d & 1), co:co + 8] += 1
    assert (hit == 1).all()


@pytest.mark.parametrize("CU,H,W", [(32, 8, 64), (32, 12, 40), (16, 8, 34), (8, 4, 70)])
def test_conv_upcat_replay(CU, H, W):
    """The decoder conv with the up-sampling inside it: per 4 x 32 output tile, staged vector i of thread
    tid (i = tid + 256 v) is skip vector i (patch pixel i / CSX, chunk i % CSX) or footprint vector
    i - NSS (low-resolution pixel ((y0 / 2) - 1 + fr, (x0 / 2) - 1 + fc)), every slot written once and
    zero outside the image.  Wavefront d = (dy, dx) sums parity pixel e = 32 blk + col (e < 51): its B
    operand at K step s is the footprint slot of the low-resolution pixel (Y / 2, X / 2) of patch pixel
    (Y, X) = (y0 - 1 + 2 (e / 17) + 1 - dy, x0 - 1 + 2 (e % 17) + 1 - dx), channels 16 s + 8 half; its
    outputs (after the half-wave exchange) fill up-channel group g + half of that patch pixel, so every
    (patch pixel, up group) is written exactly once.  With CU = 32 the conv's K step S reads its weights
    from register tap (CU / 16) + c8 / 2 (skip half) or LDS slot n WSU + tap CSX + c8 - CSX + half (up
    half), both holding W[n][16 S + 8 half ..]."""
    CL, CIN = 2 * CU, 2 * CU
    CSX, CLX, CPP, LPP = CU // 8, CL // 8, (CIN // 8) | 1, (CL // 8) | 1
    FH, FW, PC, NE = 4, 18, 17, 51
    PIX, PW = 6 * CT_PW, CT_PW
    NSS, NLS = PIX * CSX, FH * FW * CLX
    NV = -(-(NSS + NLS) // 256)
    rng = np.random.default_rng(CU + W)
    B = 2
    Hl, Wl = H // 2, W // 2
    Xs = rng.integers(1, 1000, (B, H, W, CU))
    Lo = rng.integers(1, 1000, (B, Hl, Wl, CL))
    tiles_x, tiles_y = -(-W // CT_W), -(-H // 4)
    for t in range(B * tiles_x * tiles_y):
        b, r = divmod(t, tiles_x * tiles_y)
        y0, x0 = (r // tiles_x) * 4, (r % tiles_x) * CT_W
        sP = np.full((PIX * CPP, 8), -1, dtype=np.int64)
        sL = np.full((FH * FW * LPP, 8), -1, dtype=np.int64)
        cntP = np.zeros(PIX * CPP, dtype=np.int64)
        cntL = np.zeros(FH * FW * LPP, dtype=np.int64)
        for tid in range(256):
            for v in range(NV):
                i = tid + 256 * v
                if i < NSS:
                    p, c8 = divmod(i, CSX)
                    py, px = divmod(p, PW)
                    pos, dst = (py << 16) | (px << 8) | c8, p * CPP + c8
                else:
                    k = i - NSS
                    f, c8 = divmod(k, CLX)
                    fr, fc = divmod(f, FW)
                    pos, dst = ((1 << 24) | (fr << 16) | (fc << 8) | c8) if k < NLS else -1, f * LPP + c8
                if pos < 0:
                    continue
                rr, qq, c8 = (pos >> 16) & 255, (pos >> 8) & 255, pos & 255
                if pos >> 24:
                    yy, xx = (y0 >> 1) - 1 + rr, (x0 >> 1) - 1 + qq
                    val = Lo[b, yy, xx, 8 * c8:8 * c8 + 8] if (0 <= yy < Hl and 0 <= xx < Wl) else 0
                    assert 0 <= dst < sL.shape[0]
                    sL[dst] = val
                    cntL[dst] += 1
                else:
                    yy, xx = y0 - 1 + rr, x0 - 1 + qq
                    val = Xs[b, yy, xx, 8 * c8:8 * c8 + 8] if (0 <= yy < H and 0 <= xx < W) else 0
                    assert 0 <= dst < sP.shape[0]
                    sP[dst] = val
                    cntP[dst] += 1
        for p in range(PIX):
            assert (cntP[p * CPP:p * CPP + CSX] == 1).all()
        for f in range(FH * FW):
            assert (cntL[f * LPP:f * LPP + CLX] == 1).all()
        written = np.zeros((PIX, CSX), dtype=np.int64)
        for d in range(4):
            dy, dx = d >> 1, d & 1
            for blk in range(2):
                for lane in range(64):
                    col, half = lane & 31, lane >> 5
                    e = 32 * blk + col
                    ee = min(e, NE - 1)
                    r3, c17 = divmod(ee, PC)
                    py, px = 2 * r3 + 1 - dy, 2 * c17 + 1 - dx
                    lb = ((r3 + 1 - dy) * FW + c17 + 1 - dx) * LPP + half
                    Y, X = y0 - 1 + py, x0 - 1 + px
                    live = 0 <= Y < H and 0 <= X < W
                    assert 0 <= py < 6 and 0 <= px < PW
                    if e < NE:
                        assert ((Y & 1), (X & 1)) == (dy, dx)
                    for s_ in range(CL // 16):
                        assert 0 <= lb + 2 * s_ < sL.shape[0]
                        if e < NE and live:
                            assert np.array_equal(sL[lb + 2 * s_], Lo[b, Y >> 1, X >> 1, 16 * s_ + 8 * half:16 * s_ + 8 * half + 8])
                    for g in (0, 2):
                        grp = g + half
                        if e < NE and grp < CSX:
                            written[py * PW + px, grp] += 1
        assert (written == 1).all()
    if CU == 32:
        WSU = _conv_ws(CSX)
        nr = 9 * (CU // 16)
        reg_step = [(r // (CU // 16)) * (CIN // 16) + r % (CU // 16) for r in range(nr)]
        for S in range(9 * CIN // 16):
            tap, c8 = (16 * S) // CIN, ((16 * S) % CIN) // 8
            for half in range(2):
                k = 16 * S + 8 * half
                if c8 < CSX:
                    assert reg_step[tap * (CU // 16) + c8 // 2] == S
                else:
                    slot = tap * CSX + c8 - CSX + half        # LDS slot within row n
                    stap, u8 = divmod(slot, CSX)
                    assert 0 <= slot < 9 * CSX < WSU
                    assert stap * CIN + CU + 8 * u8 == k


# ------------------------------------------------------------------ fused ROF dual steps
FTX, FTY = 64, 16
FRX, FRY = FTX + 4, FTY + 4


def _div(p1, p2):
    ny, nx = p1.shape
    a, b = np.zeros_like(p1), np.zeros_like(p1)
    if nx > 1:
        a[:, 0], a[:, 1:-1], a[:, -1] = p1[:, 0], p1[:, 1:-1] - p1[:, :-2], -p1[:, -2]
    if ny > 1:
        b[0], b[1:-1], b[-1] = p2[0], p2[1:-1] - p2[:-2], -p2[-2]
    return a + b


def _step(p1, p2, g, il, tau):
    v = _div(p1, p2) - g * il
    a, b = np.zeros_like(v), np.zeros_like(v)
    a[:, :-1], b[:-1] = v[:, 1:] - v[:, :-1], v[1:] - v[:-1]
    m = 1 + tau * np.sqrt(a * a + b * b)
    return (p1 + tau * a) / m, (p2 + tau * b) / m


def _fused(p1, p2, g, il, tau, zero):
    ny, nx = g.shape
    q1, q2 = np.full_like(g, np.nan), np.full_like(g, np.nan)

    def inside(x, y):
        return 0 <= x < nx and 0 <= y < ny
    for by in range((ny + FTY - 1) // FTY):
        for bx in range((nx + FTX - 1) // FTX):
            x0, y0 = bx * FTX - 2, by * FTY - 2
            s1 = np.full((FRY, FRX), np.nan)
            s2, sg, sv = s1.copy(), s1.copy(), s1.copy()
            for i in range(FRX * FRY):
                ry, rx = divmod(i, FRX)
                x, y = x0 + rx, y0 + ry
                inn = inside(x, y)
                s1[ry, rx] = p1[y, x] if (not zero and inn) else 0.0
                s2[ry, rx] = p2[y, x] if (not zero and inn) else 0.0
                sg[ry, rx] = g[y, x] if inn else 0.0

            def v_at(rx, ry, x, y):
                a = 0.0 if nx == 1 else (s1[ry, rx] if x == 0 else (-s1[ry, rx - 1] if x == nx - 1
                                                                      else s1[ry, rx] - s1[ry, rx - 1]))
                b = 0.0 if ny == 1 else (s2[ry, rx] if y == 0 else (-s2[ry - 1, rx] if y == ny - 1
                                                                      else s2[ry, rx] - s2[ry - 1, rx]))
                out = (a + b) - sg[ry, rx] * il
                assert np.isfinite(out)
                return out

            def q_at(rx, ry, x, y):
                v0 = sv[ry, rx]
                a = sv[ry, rx + 1] - v0 if x + 1 < nx else 0.0
                b = sv[ry + 1, rx] - v0 if y + 1 < ny else 0.0
                assert np.isfinite(v0) and np.isfinite(a) and np.isfinite(b)
                m = 1 + tau * np.sqrt(a * a + b * b)
                return (s1[ry, rx] + tau * a) / m, (s2[ry, rx] + tau * b) / m
            for i in range((FRX - 1) * (FRY - 1)):          # v on [1, FRX) x [1, FRY)
                ry, rx = 1 + i // (FRX - 1), 1 + i % (FRX - 1)
                if inside(x0 + rx, y0 + ry):
                    sv[ry, rx] = v_at(rx, ry, x0 + rx, y0 + ry)
            new = {}
            assert (FRX - 2) * (FRY - 2) <= 5 * 256             # five register slots per thread
            for i in range((FRX - 2) * (FRY - 2)):          # p' on [1, FRX - 1) x [1, FRY - 1)
                ry, rx = 1 + i // (FRX - 2), 1 + i % (FRX - 2)
                new[(ry, rx)] = q_at(rx, ry, x0 + rx, y0 + ry) if inside(x0 + rx, y0 + ry) else (0.0, 0.0)
            for (ry, rx), (n1, n2) in new.items():
                s1[ry, rx], s2[ry, rx] = n1, n2
            for i in range((FRX - 3) * (FRY - 3)):          # v' on [2, FRX - 1) x [2, FRY - 1)
                ry, rx = 2 + i // (FRX - 3), 2 + i % (FRX - 3)
                if inside(x0 + rx, y0 + ry):
                    sv[ry, rx] = v_at(rx, ry, x0 + rx, y0 + ry)
            for i in range(FTX * FTY):                      # q on the tile
                ry, rx = 2 + i // FTX, 2 + i % FTX
                x, y = x0 + rx, y0 + ry
                if inside(x, y):
                    q1[y, x], q2[y, x] = q_at(rx, ry, x, y)
    return q1, q2


@pytest.mark.parametrize("ny,nx", [(37, 70), (16, 64), (1, 50), (33, 1), (2, 2), (17, 65)])
def test_prox2_emulation(ny, nx):
    rng = np.random.default_rng(ny * 1000 + nx)
    g = rng.standard_normal((ny, nx))
    p1, p2 = 0.3 * rng.standard_normal((ny, nx)), 0.3 * rng.standard_normal((ny, nx))
    il, tau = 1 / 0.3, 0.125
    for zero in (True, False):
        a1, a2 = (np.zeros_like(g), np.zeros_like(g)) if zero else (p1, p2)
        r1, r2 = _step(*_step(a1, a2, g, il, tau), g, il, tau)
        k1, k2 = _fused(p1, p2, g, il, tau, zero)
        assert np.array_equal(k1, r1) and np.array_equal(k2, r2)


# ------------------------------------------------------------------ register FFT of the P = 4096 filter
def _rev4(k):
    return (k >> 2) | ((k & 3) << 2)


def _dft16(v, inv):
    """filter4096_kernel's 16-point DFT on v[..., 16] (input m at m, output k at rev4(k))."""
    v = v.copy()
    s = 1.0 if inv else -1.0

    def dft4(a, b, c, d):
        s02, d02, s13, d13 = a + c, a - c, b + d, b - d
        r = -1j * d13
        return (s02 + s13, d02 - r if inv else d02 + r, s02 - s13, d02 + r if inv else d02 - r)
    for q in range(4):
        v[..., q], v[..., q + 4], v[..., q + 8], v[..., q + 12] = dft4(v[..., q], v[..., q + 4], v[..., q + 8],
                                                                     v[..., q + 12])
    for q in range(1, 4):
        for r in range(1, 4):
            v[..., q + 4 * r] *= np.exp(s * 2j * np.pi * q * r / 16)
    for r in range(4):
        v[..., 4 * r], v[..., 4 * r + 1], v[..., 4 * r + 2], v[..., 4 * r + 3] = dft4(
            v[..., 4 * r], v[..., 4 * r + 1], v[..., 4 * r + 2], v[..., 4 * r + 3])
    return v


def _w4096(tw, e):
    t = tw[e & 2047]
    return np.where(e & 2048, -t, t)


def _wpow(bases, k):
    """w^k from the bases w, w^2, w^4, w^8, as the kernel forms its twiddles."""
    r = np.ones_like(bases[0])
    for i in range(4):
        if (k >> i) & 1:
            r = r * bases[i]
    return r


def test_fft4096_register_emulation():
    """The three-pass register FFT of filter4096_kernel, replayed with its LDS layout (NaN-initialised,
    so a read of an unset entry shows), its twiddles (products of eight table values per thread) and
    the bit-reversed spectrum table,
    equals ifft(fft(x) H) for a random row pair and a random real spectrum."""
    rng = np.random.default_rng(3)
    P = 4096
    x = rng.standard_normal(P) + 1j * rng.standard_normal(P)
    Hnat = rng.standard_normal(P)
    brev = np.array([int(f"{n:012b}"[::-1], 2) for n in range(P)])
    H = Hnat[brev] / P                                   # the plan's table: bit-reversed, 1/P folded
    tw = np.exp(-2j * np.pi * np.arange(P // 2) / P)     # half-circle table, Pmax = 4096
    t = np.arange(256)
    hi, lo = t >> 4, t & 15
    b1w = [_w4096(tw, t << i) for i in range(4)]          # twiddle bases, loaded once per thread
    b2w = [_w4096(tw, (16 * lo) << i) for i in range(4)]
    z = np.full(16 * 272, np.nan + 0j)
    v = x[t[:, None] + 256 * np.arange(16)[None, :]]     # thread a holds x[a + 256 m]
    v = _dft16(v, False)
    for k1 in range(16):
        z[k1 * 256 + t] = v[:, _rev4(k1)] * _wpow(b1w, k1)
    v = np.stack([z[hi * 256 + lo + 16 * d] for d in range(16)], 1)
    v = _dft16(v, False)
    z[:] = np.nan
    for b in range(16):
        z[hi * 272 + b * 17 + lo] = v[:, _rev4(b)] * _wpow(b2w, b)
    v = np.stack([z[hi * 272 + lo * 17 + c] for c in range(16)], 1)
    v = _dft16(v, False)
    X = np.empty(P, complex)
    for b2 in range(16):
        X[hi + 16 * lo + 256 * b2] = v[:, _rev4(b2)]
    np.testing.assert_allclose(X, np.fft.fft(x), rtol=0, atol=1e-9 * np.abs(X).max())
    for b2 in range(16):
        v[:, _rev4(b2)] *= H[brev[hi + 16 * lo + 256 * b2]]
    u = _dft16(np.stack([v[:, _rev4(b2)] for b2 in range(16)], 1), True)
    z[:] = np.nan
    for c in range(16):
        z[hi * 272 + lo * 17 + c] = u[:, _rev4(c)]
    v = np.stack([z[hi * 272 + b * 17 + lo] * np.conj(_wpow(b2w, b)) for b in range(16)], 1)
    v = _dft16(v, True)
    z[:] = np.nan
    for d in range(16):
        z[hi * 256 + lo + 16 * d] = v[:, _rev4(d)]
    v = np.stack([z[k1 * 256 + t] * np.conj(_wpow(b1w, k1)) for k1 in range(16)], 1)
    v = _dft16(v, True)
    y = np.empty(P, complex)
    for m in range(16):
        y[t + 256 * m] = v[:, _rev4(m)]
    ref = np.fft.ifft(np.fft.fft(x) * Hnat)
    assert not np.isnan(y).any()
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-10 * np.abs(ref).max())
