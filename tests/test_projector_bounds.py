"""Address bounds and grid decode of the direct and LDS-window projectors,
checked on the CPU.

The direct kernel (projector 2) reads image rows without clamping the tap
column: it relies on the kPadL = 96 zero columns on each side of a padded row
(csrc/ncs_internal.h) to hold every tap of a 64-ray block at every step of the
block's step range.  This test replays the
kernel's address arithmetic (the block step range with its single-precision
divisions on coefficients rounded to float; each tap column as the floor of a
double-precision anchor plus the floor of a single-precision offset) for the
workload geometries and asserts that every read stays inside the padded row:
columns -96 .. N+95.  The LDS-window kernel (projector 1) walks the same steps
with the same taps and copies, per step, the 96-element window that starts at
the block's smallest tap rounded down to 16 bytes: its first or last lane's
tap must be the smallest, the window must lie inside the padded row and hold
both taps of every lane.  Fused multiply-adds are replayed
exactly: the product of a small integer and a float is exact in double, so
one rounding of the double sum is the fused result.
"""
import math

import numpy as np
import pytest

PAD = 96
WIN = 96            # elements of the LDS window of projector 1
F32 = np.float32


def _r32(x):
    return np.asarray(x, dtype=np.float64).astype(F32)


def _fma32(a, b, c):
    """fma(a, b, c) in single precision for integer-valued a (exact product in double)."""
    return _r32(np.asarray(a, np.float64) * np.asarray(b, np.float64) + np.asarray(c, np.float64))


def _angles64(n, na, ns):
    """k1, k2, k0 per angle in double, as the host computes them."""
    hn, hs = 0.5 * (n - 1), 0.5 * (ns - 1)
    out = []
    for a in range(na):
        th = math.pi * a / na
        ct, st = math.cos(th), math.sin(th)
        if 4 * a <= na or 4 * a >= 3 * na:
            out.append((1.0 / ct, -st / ct, -hs / ct + hn * st / ct + hn))
        else:
            out.append((1.0 / st, -ct / st, -hs / st + hn * ct / st + hn))
    return out


def _angles(n, na, ns):
    """k1, k2, k0 per angle (float32), as the host computes them in double."""
    hn, hs = 0.5 * (n - 1), 0.5 * (ns - 1)
    out = []
    for a in range(na):
        th = math.pi * a / na
        ct, st = math.cos(th), math.sin(th)
        if 4 * a <= na or 4 * a >= 3 * na:
            k1, k2, k0 = 1.0 / ct, -st / ct, -hs / ct + hn * st / ct + hn
        else:
            k1, k2, k0 = 1.0 / st, -ct / st, -hs / st + hn * ct / st + hn
        out.append((F32(k1), F32(k2), F32(k0)))
    return out


def _sat(v):
    return int(min(max(float(v), -1.0e9), 1.0e9))


def _block_range(k1, k2, k0, n, d0, part, nparts):
    """The block's culled step range, split evenly into nparts."""
    bA, bB = _fma32(d0, k1, k0), _fma32(d0 + 63, k1, k0)
    blo, bhi = min(bA, bB), max(bA, bB)
    lo_x, hi_x = F32(-2), F32(n + 1)
    sb, se = 0, n
    if k2 > 0:
        sb = max(sb, _sat(np.floor(F32(lo_x - bhi) / k2)) - 1)
        se = min(se, _sat(np.ceil(F32(hi_x - blo) / k2)) + 2)
    elif k2 < 0:
        sb = max(sb, _sat(np.floor(F32(hi_x - blo) / k2)) - 1)
        se = min(se, _sat(np.ceil(F32(lo_x - bhi) / k2)) + 2)
    elif bhi < lo_x or blo > hi_x:
        se = sb
    ln = max(se - sb, 0)
    return sb + (part * ln) // nparts, sb + ((part + 1) * ln) // nparts


def _tap_columns(base64, k2d, k2, sb, se, unroll):
    """Floor of each step's coordinate as the unrolled loop forms it (rows:
    lanes, columns: steps): an anchor fma(s, k2, base) in double split into
    an integer and a fraction t0, then fma(j, k2, t0) in single precision."""
    cols = []
    s = sb
    while s < se:
        xa = s * k2d + base64
        ia = np.floor(xa)
        t0 = _r32(xa - ia)
        for j in range(unroll if s + unroll <= se else 1):
            t = t0 if j == 0 else _fma32(j, k2, t0)
            cols.append(ia + np.floor(t.astype(np.float64)))
        s += unroll if s + unroll <= se else 1
    return np.stack(cols, axis=1) if cols else np.zeros((base64.size, 0))


GEOMS = [(16, 7, 23), (64, 90, 92), (128, 179, 130), (128, 180, 185), (256, 358, 260), (256, 360, 367),
         (512, 717, 520)]


@pytest.mark.parametrize("geom", GEOMS, ids=[f"{g[0]}x{g[1]}x{g[2]}" for g in GEOMS])
def test_projector_reads_stay_in_the_padded_rows_and_windows(geom):
    n, na, ns = geom
    nb = (ns + 63) // 64
    angles = range(na) if n <= 256 else sorted(set(range(0, na, 5)) | {179, 180, 537, 538, na - 1})
    tab = _angles(n, na, ns)
    tab64 = _angles64(n, na, ns)
    lo, hi = 0, 0
    for a in angles:
        k1, k2, k0 = tab[a]
        k1d, k2d, k0d = tab64[a]
        for rb in range(nb):
            d0 = rb * 64
            lanes = np.arange(d0, d0 + 64)
            # projector 2: one ray per lane, 4 waves split the steps, anchors every 8 steps
            base64 = lanes * k1d + k0d
            for part in range(4):
                sb, se = _block_range(k1, k2, k0, n, d0, part, 4)
                if se <= sb:
                    continue
                c = _tap_columns(base64, k2d, k2, sb, se, 8)
                lo, hi = min(lo, c.min()), max(hi, c.max() + 1)
                assert c.min() >= -PAD and c.max() + 1 <= n + PAD - 1, (a, rb, part, c.min(), c.max())
                # projector 1: the window of each step (FP32: 4 elements per 16 bytes, FP64: 2)
                e = (c + PAD).astype(np.int64)
                lmin = 0 if k1 > 0 else 63
                assert np.array_equal(e[lmin], e.min(axis=0)), (a, rb, part)
                P = n + 2 * PAD
                for eq in (4, 2):
                    w = np.minimum(e[lmin] & ~(eq - 1), P - WIN)
                    assert w.min() >= 0 and w.max() + WIN <= P
                    off = e - w
                    assert off.min() >= 0 and off.max() + 1 <= WIN - 1, (a, rb, part, off.min(), off.max())
    # the margins are used, but with room to spare
    assert lo >= -PAD and hi <= n + PAD - 1


@pytest.mark.parametrize("geom", GEOMS, ids=[f"{g[0]}x{g[1]}x{g[2]}" for g in GEOMS])
def test_axis_split_grid_covers_every_block_once(geom):
    """The single-slice projection grid sends row-stepping blocks to XCDs 0-3
    and column-stepping ones to XCDs 4-7 (workgroup b on XCD b mod 8): replay
    the kernel's decode of every workgroup of the grid the host launches and
    check that each (angle, 64-ray block) pair is taken exactly once, and that
    the ray blocks go out central ones first (longest first)."""
    n, na, ns = geom
    nb = (ns + 63) // 64
    rows = [a for a in range(na) if 4 * a <= na or 4 * a >= 3 * na]
    order = rows + [a for a in range(na) if a not in set(rows)]
    nar = len(rows)
    wgs = 8 * ((max(nar, na - nar) * nb + 3) // 4)   # project_wgs_split
    seen = np.zeros((na, nb), dtype=int)
    last_dist = [0.0, 0.0]
    for local in range(wgs):
        xcd, k = local & 7, (local >> 3) * 4 + (local & 3)
        colsax = xcd >= 4
        nang = na - nar if colsax else nar
        if k >= nang * nb:
            continue
        rbi, j = divmod(k, nang)
        rb = (nb - 1) // 2 + ((rbi + 1) // 2 if rbi % 2 else -(rbi // 2))
        a = order[(nar if colsax else 0) + j]
        assert (xcd >= 4) == (a not in set(rows))
        seen[a, rb] += 1
        dist = abs(rb + 0.5 - nb / 2)    # the block's distance from the detector's centre
        assert dist >= last_dist[colsax]
        last_dist[colsax] = dist
    assert np.all(seen == 1)
