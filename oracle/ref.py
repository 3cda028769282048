"""Second, pure-Python implementation of the oracle's step for tiny grids.

TEST INFRASTRUCTURE ONLY. It is written independently of pedsim_oracle.c
(scatter from the requesters instead of gathering at the cells, big-int
Philox, numpy float32 scalars for every float operation) so that an indexing
or ordering slip in either one shows up as a disagreement. Same readings of
the paper as the C oracle (request per Sec. III / IV.b-c with eq. 1 or eq. 2,
scatter-to-gather resolve per Sec. IV.d, evaporation eq. 3 then deposit
eq. 4; mode 2 keeps a tour length per agent and deposits eq. 5's amount on
the cell an agent enters).
"""
from __future__ import annotations

import math

import numpy as np

F32 = np.float32
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32-10 (Salmon et al., SC'11) on Python ints."""
    x = [int(c) & MASK for c in ctr]
    k = [int(v) & MASK for v in key]
    for rnd in range(10):
        if rnd:
            k = [(k[0] + 0x9E3779B9) & MASK, (k[1] + 0xBB67AE85) & MASK]
        a = 0xD2511F53 * x[0]
        b = 0xCD9E8D57 * x[2]
        x = [(b >> 32) ^ x[1] ^ k[0], b & MASK, (a >> 32) ^ x[3] ^ k[1], a & MASK]
    return x


def _phi(z):
    return 0.5 * math.erfc(-z / math.sqrt(2.0))


# ceil(2^32 * Phi(j + 1/2)); double precision is ample here because none of
# the six products lies within 1e-6 of an integer.
THRESHOLDS = [int(math.ceil(4294967296.0 * _phi(j + 0.5))) for j in range(6)]

# candidate offsets (dx in units of the heading d, dy); 6..8 are the backward
# cells of the eight-neighbour set
CAND = {1: (1, 0), 2: (1, -1), 3: (1, 1), 4: (0, -1), 5: (0, 1), 6: (-1, 0), 7: (-1, -1),
        8: (-1, 1)}
# squared distance to the point two cells ahead
D2 = {2: 2, 3: 2, 4: 5, 5: 5, 6: 9, 7: 10, 8: 10}


def _weight(d2, beta):
    return F32(float(d2) ** (-0.5 * beta))


def step(code, ids, tau, *, mode, t, seed, rho, dtau, alpha, beta, tour=None, neighbours=5):
    """One step on copies; returns (code, ids, tau, req, moved), or with
    mode 2 (code, ids, tau, tour, req, moved)."""
    H, W = code.shape
    code = code.copy()
    ids = ids.copy()
    tau = None if tau is None else tau.copy()
    tour = None if tour is None else tour.copy()
    key = (seed & MASK, seed >> 32)

    def words(k):
        return philox4x32_10((k, t & MASK, t >> 32, 0), key)

    def empty(x, y):
        return 0 <= x < W and 0 <= y < H and code[y, x] == 0

    sides = (2, 3, 4, 5, 6, 7, 8) if neighbours == 8 else (2, 3, 4, 5)

    def lem(avail, r1, r2):
        order = [3, 2, 5, 4, 6, 8, 7] if (r2 & 1) else [2, 3, 4, 5, 6, 7, 8]
        ranked = [r for r in order if r in avail and avail[r]]
        if not ranked:
            return 0
        idx = sum(1 for th in THRESHOLDS[:len(sides) - 1] if r1 >= th)
        return ranked[min(idx, len(ranked) - 1)]

    req = np.zeros((H, W), dtype=np.uint8)
    for y in range(H):
        for x in range(W):
            g = int(code[y, x])
            if g not in (1, 2):
                continue
            d = 1 if g == 1 else -1
            if empty(x + d, y):
                req[y, x] = 1
                continue
            avail = {}
            for r in sides:
                ox, oy = CAND[r]
                avail[r] = empty(x + ox * d, y + oy)
            if not any(avail.values()):
                continue
            w = words(int(ids[y, x]) - 1)
            if mode == 0:
                req[y, x] = lem(avail, w[1], w[2])
                continue
            plane = tau[g - 1]
            ws = []
            for r in sides:
                if not avail[r]:
                    ws.append(F32(0.0))
                    continue
                ox, oy = CAND[r]
                tv = F32(plane[y + oy, x + ox * d])
                p = F32(1.0)
                if alpha > 0:
                    p = tv
                    for _ in range(alpha - 1):
                        p = F32(p * tv)
                ws.append(F32(p * _weight(D2[r], beta)))
            s = ws[0]
            for wv in ws[1:]:
                s = F32(s + wv)
            if s == F32(0.0):
                req[y, x] = lem(avail, w[1], w[2])
                continue
            u = F32(F32(w[1] >> 8) * F32(2.0 ** -24))
            target = F32(u * s)
            run = F32(0.0)
            pick = None
            last = None
            for i, r in enumerate(sides):
                run = F32(run + ws[i])
                if ws[i] > 0:
                    last = r
                    if target < run:
                        pick = r
                        break
            req[y, x] = pick if pick is not None else last

    # scatter: every requester registers at its target; lowest (ticket, k) kept
    best = {}
    for y in range(H):
        for x in range(W):
            r = int(req[y, x])
            if r == 0:
                continue
            g = int(code[y, x])
            d = 1 if g == 1 else -1
            ox, oy = CAND[r]
            tx, ty = x + ox * d, y + oy
            k = int(ids[y, x]) - 1
            cand = (words(k)[0], k, x, y)
            if (tx, ty) not in best or cand[:2] < best[(tx, ty)][:2]:
                best[(tx, ty)] = cand
    new_code = code.copy()
    new_ids = ids.copy()
    arrivals = {}
    for (tx, ty), (_, k, sx, sy) in best.items():
        new_code[ty, tx] = code[sy, sx]
        new_ids[ty, tx] = ids[sy, sx]
        new_code[sy, sx] = 0
        new_ids[sy, sx] = 0
        if mode == 2:
            # length of the move between cell centres: 1 straight, sqrt 2 diagonal
            length = F32(math.sqrt(2.0)) if (tx != sx and ty != sy) else F32(1.0)
            tour[k] = F32(tour[k] + length)
            arrivals[(tx, ty)] = (int(code[sy, sx]), k)
    if mode == 2:
        keep = F32(F32(1.0) - F32(rho))
        for g in (1, 2):
            plane = tau[g - 1]
            for y in range(H):
                for x in range(W):
                    v = F32(keep * plane[y, x])
                    a = arrivals.get((x, y))
                    if a is not None and a[0] == g:
                        v = F32(v + F32(F32(dtau) / tour[a[1]]))
                    plane[y, x] = v
        return new_code, new_ids, tau, tour, req, len(best)
    if mode == 1:
        keep = F32(F32(1.0) - F32(rho))
        for g in (1, 2):
            plane = tau[g - 1]
            for y in range(H):
                for x in range(W):
                    v = F32(keep * plane[y, x])
                    if new_code[y, x] == g:
                        v = F32(v + F32(dtau))
                    plane[y, x] = v
    return new_code, new_ids, tau, req, len(best)


# --- larger scanning and moving ranges (Sec. VII) -----------------------------

RAY = {1: (1, 0), 2: (1, -1), 3: (1, 1), 4: (0, -1), 5: (0, 1)}  # (forward, lateral) unit steps


def range_weight(a, f, S, M, beta):
    """eta^beta of a side ray (forward component a, free run f): the float
    nearest to (f/S)^beta * D2^(-beta/2), D2 from the landing cell to the
    point M+1 cells ahead."""
    k = min(f, M)
    d2 = (M + 1 - a * k) ** 2 + k * k
    return F32((f / S) ** beta * float(d2) ** (-0.5 * beta))


def step_range(code, ids, tau, *, mode, t, seed, rho, dtau, alpha, beta, S, M):
    """One step with scanning range S and moving range M on copies; returns
    (code, ids, tau, req, length, moved). Requesters register at their landing
    cell (scatter); the ranking sorts the open rays by the exact rational
    score f^2 / D2 (the square of C up to a common factor)."""
    from fractions import Fraction
    H, W = code.shape
    code, ids = code.copy(), ids.copy()
    tau = None if tau is None else tau.copy()
    key = (seed & MASK, seed >> 32)

    def words(k):
        return philox4x32_10((k, t & MASK, t >> 32, 0), key)

    def empty(x, y):
        return 0 <= x < W and 0 <= y < H and code[y, x] == 0

    req = np.zeros((H, W), dtype=np.uint8)
    length = np.zeros((H, W), dtype=np.uint8)
    for y in range(H):
        for x in range(W):
            g = int(code[y, x])
            if g not in (1, 2):
                continue
            d = 1 if g == 1 else -1
            run = {}
            for r, (a, b) in RAY.items():
                n = 0
                while n < S and empty(x + (n + 1) * a * d, y + (n + 1) * b):
                    n += 1
                run[r] = n
            if run[1] >= 1:
                req[y, x], length[y, x] = 1, min(run[1], M)
                continue
            open_rays = [r for r in (2, 3, 4, 5) if run[r] >= 1]
            if not open_rays:
                continue
            w = words(int(ids[y, x]) - 1)

            def d2(r):
                a, b = RAY[r]
                k = min(run[r], M)
                return (M + 1 - a * k) ** 2 + (b * k) ** 2

            def lem():
                order = [3, 2, 5, 4] if (w[2] & 1) else [2, 3, 4, 5]
                ranked = sorted([r for r in order if run[r] >= 1],
                                key=lambda r: -Fraction(run[r] ** 2, d2(r)))
                idx = sum(1 for th in THRESHOLDS[:3] if w[1] >= th)
                return ranked[min(idx, len(ranked) - 1)]

            if mode == 0:
                pick = lem()
            else:
                plane = tau[g - 1]
                ws = []
                for r in (2, 3, 4, 5):
                    if run[r] < 1:
                        ws.append(F32(0.0))
                        continue
                    a, b = RAY[r]
                    k = min(run[r], M)
                    tv = F32(plane[y + k * b, x + k * a * d])
                    p = F32(1.0)
                    if alpha > 0:
                        p = tv
                        for _ in range(alpha - 1):
                            p = F32(p * tv)
                    ws.append(F32(p * range_weight(a, run[r], S, M, beta)))
                tot = ws[0]
                for wv in ws[1:]:
                    tot = F32(tot + wv)
                if tot == F32(0.0):
                    pick = lem()
                else:
                    target = F32(F32(F32(w[1] >> 8) * F32(2.0 ** -24)) * tot)
                    acc, pick, last = F32(0.0), None, None
                    for i, r in enumerate((2, 3, 4, 5)):
                        acc = F32(acc + ws[i])
                        if ws[i] > 0:
                            last = r
                            if target < acc:
                                pick = r
                                break
                    pick = pick if pick is not None else last
            req[y, x], length[y, x] = pick, min(run[pick], M)

    best = {}
    for y in range(H):
        for x in range(W):
            r = int(req[y, x])
            if r == 0:
                continue
            d = 1 if code[y, x] == 1 else -1
            a, b = RAY[r]
            k = int(length[y, x])
            tx, ty = x + k * a * d, y + k * b
            kk = int(ids[y, x]) - 1
            cand = (words(kk)[0], kk, x, y)
            if (tx, ty) not in best or cand[:2] < best[(tx, ty)][:2]:
                best[(tx, ty)] = cand
    new_code, new_ids = code.copy(), ids.copy()
    for (tx, ty), (_, _, sx, sy) in best.items():
        new_code[ty, tx], new_ids[ty, tx] = code[sy, sx], ids[sy, sx]
        new_code[sy, sx], new_ids[sy, sx] = 0, 0
    if mode == 1:
        keep = F32(F32(1.0) - F32(rho))
        for g in (1, 2):
            plane = tau[g - 1]
            for y in range(H):
                for x in range(W):
                    v = F32(keep * plane[y, x])
                    if new_code[y, x] == g:
                        v = F32(v + F32(dtau))
                    plane[y, x] = v
    return new_code, new_ids, tau, req, length, len(best)
