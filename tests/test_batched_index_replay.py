"""Host replay of the batched kernel's thread-count-dependent index arithmetic.

k_batched<NT> (paper_2607_17978_amd/csrc/batched.hip) is offered only with
1,024 threads per workgroup: a 256-thread run once ended in a GPU fault and
512-thread runs returned NOT_CONVERGED on structures the 1,024-thread shape
solves.  This test replays, for NT = 256, 512 and 1,024 and every structure
of the 1,024-structure batch (inputs.gen.batch), the index expressions of
every loop whose trip or stride depends on NT -- the spread accumulator and
FFT staging of pass A, the line batches of passes B-D, pass E, every
compile-time FFT stage's item range and per-thread register count, the
workgroup scan, the interpolation / pair loops and the LDS carve-up -- and
asserts each index against its allocation, and that every element each loop
must cover is covered exactly as often as the 1,024-thread shape covers it.
It models the kernel's integer arithmetic (the formulas are transcribed from
the source) and runs no kernel.
"""
import math

import numpy as np
import pytest

from inputs import gen

BQ_KAX, BQ_LDS, BQ_L, MAXP, EMAX, P = 64, 64 * 128, 8, 8, 40, 6
CT_LENGTHS = (24, 32, 36, 40, 48, 60, 64)


def radices(K):
    """ct_radix_at: 5s, 3s, 8s, then a 4 or a 2."""
    out, n = [], K
    for r in (5, 3):
        while n % r == 0:
            out.append(r)
            n //= r
    while n % 8 == 0:
        out.append(8)
        n //= 8
    if n in (4, 2):
        out.append(n)
        n = 1
    assert n == 1
    return out


def nc_ks(K):
    return (64, 65) if K in CT_LENGTHS else (32, 32)


def fft_stage_indices(K, ncol, ks, nt):
    """Every LDS index a compile-time Stockham transform (fft_stage_ct) reads
    or writes for K points x ncol columns at row stride ks, and the check
    that IT = ceil(items / NT) iterations cover every item once."""
    idx, ns = [], 1
    for R in radices(K):
        per = K // R
        nitems = per * ncol
        it = -(-nitems // nt)
        items = np.arange(it * nt)
        live = items < nitems
        assert live.sum() == nitems                      # each butterfly item exactly once
        c, j = items[live] % ncol, items[live] // ncol
        kk = j % ns
        base = (j - kk) * R + kk
        for r in range(R):
            idx.append((j + r * per) * ks + c)           # reads
            idx.append((base + r * ns) * ks + c)         # writes
        # the writes are a permutation of the reads: no element lost or doubled
        w = np.concatenate([(base + r * ns) * ks + c for r in range(R)])
        rd = np.concatenate([(j + r * per) * ks + c for r in range(R)])
        assert np.array_equal(np.sort(w), np.sort(rd))
        ns *= R
    return np.concatenate(idx)


def runtime_fft_ok(K, ncol_log2, nt):
    """fft_lds: MAXIT = ceil(EMAX / R) register slots per thread must cover
    the stage's K / R x ncol items."""
    ns = 1
    for R in radices(K):
        nitems = (K // R) << ncol_log2
        if -(-EMAX // R) * nt < nitems:
            return False
        ns *= R
    return True


def structure_sizes(s, p=P, spacing=0.8, rc=12.0):
    K = list(s.grid)
    return K, s.n


@pytest.mark.parametrize("nt", [256, 512, 1024])
def test_batched_indices_stay_in_bounds(nt):
    structs = gen.batch(1024)
    nmax = max(s.n for s in structs)
    assert nmax <= 1024
    # --- LDS carve-up (dynamic): fbuf [BQ_LDS float2] | sp [nmax double] | order [nmax int]
    dyn = 8 * BQ_LDS + 8 * nmax + 4 * nmax
    static = 4 * 2 * (BQ_KAX + 1) + 8 * 3 * BQ_KAX + 4 * 3 * BQ_KAX + 4 * nt + 8 * 16 * 5 + 8 * 5 + 512
    assert dyn + static <= 160 * 1024
    seen_k = set()
    # the indices depend on the grid and the atom count only: every grid of the
    # batch, with the smallest and the largest structure that uses it
    shapes = {}
    for s in structs:
        lo, hi = shapes.get(s.grid, (s.n, s.n))
        shapes[s.grid] = (min(lo, s.n), max(hi, s.n))
    cases = sorted({(g, n) for g, ns in shapes.items() for n in ns})
    for (K1, K2, K3), n in cases:
        K3h = K3 // 2 + 1
        nhalf, npts = K1 * K2 * K3h, K1 * K2 * K3
        assert max(K1, K2, K3) <= BQ_KAX and min(K1, K2, K3) >= 2 * P
        # ---------------------------------------------- pass A (spread + R2C along axis 3)
        NC, KS = nc_ks(K3)
        D = max(1, min(2 * NC // K2, K1 - P + 1))
        RW = 2 * NC
        assert K3 * RW * 8 <= 8 * BQ_LDS                           # int64 accumulator inside fbuf
        assert D * K2 <= RW
        assert D + P - 1 <= K1                                     # candidate ranges never overlap
        rows_done = np.zeros(K1 * K2, dtype=int)
        for g1a in range(0, K1, D):
            j = np.arange(D)[:, None, None]
            g2 = np.arange(K2)[None, :, None]
            g3 = np.arange(K3)[None, None, :]
            valid = (g1a + j < K1) & np.ones_like(g2 + g3, dtype=bool)
            r = (j * K2 + g2) + 0 * g3
            acc_idx = (g3 * RW + r)[valid]
            assert acc_idx.min() >= 0 and acc_idx.max() < K3 * RW
            # conversion: e < K3 NC, buf[g3 KS + pr] (compile-time) / buf[e] (runtime)
            e = np.arange(K3 * NC)
            bidx = (e // NC) * KS + e % NC if K3 in CT_LENGTHS else e
            assert bidx.max() < BQ_LDS
            assert (2 * (e % NC) + 1).max() < RW
            # unpack: rows of this batch of planes, C[g1a K2 K3h + t]
            rows = min(D, K1 - g1a) * K2
            t = np.arange(rows * K3h)
            pr = (t // K3h) >> 1
            m = t % K3h
            assert (m * KS + pr).max() < BQ_LDS and pr.max() < NC
            cidx = g1a * K2 * K3h + t
            assert cidx.max() < nhalf
            rows_done[g1a * K2:g1a * K2 + rows] += 1
        assert np.all(rows_done == 1)                              # every (g1, g2) row once
        # ---------------------------------------------- passes B / C / D (lines along axes 2 and 1)
        for AX, K in ((1, K2), (0, K1)):
            NC, KS = nc_ks(K)
            assert nt % NC == 0
            kstep = nt // NC
            nl = K2 * K3h if AX == 0 else K1 * K3h
            kstride = K2 * K3h if AX == 0 else K3h
            tid = np.arange(nt)
            c, k0 = tid % NC, tid // NC
            hits = np.zeros((NC, K), dtype=int)
            for ci, kk0 in zip(c, k0):
                ks_ = np.arange(kk0, K, kstep)
                hits[ci, ks_] += 1
            assert np.all(hits == 1)                                # each (line, k) staged once
            assert ((K - 1) * KS + NC - 1) < BQ_LDS
            L = np.arange(0, nl, NC)[:, None] + np.arange(NC)[None, :]
            L = L[L < nl]
            base = L if AX == 0 else (L // K3h) * K2 * K3h + L % K3h
            assert (base + (K - 1) * kstride).max() < nhalf
            if K in CT_LENGTHS and (K, nt) not in seen_k:
                fi = fft_stage_indices(K, NC, KS, nt)
                assert fi.min() >= 0 and fi.max() < BQ_LDS
                seen_k.add((K, nt))
            elif K not in CT_LENGTHS:
                assert runtime_fft_ok(K, 5, nt)
        # ---------------------------------------------- pass E (C2R along axis 3 into R)
        NC, KS = nc_ks(K3)
        nrows = K1 * K2
        for r0 in range(0, nrows, 2 * NC):
            t = np.arange(NC * K3h)
            pr, m = t // K3h, t % K3h
            assert (m * KS + pr).max() < BQ_LDS and ((K3 - m[m > 0]) * KS + pr[m > 0]).max() < BQ_LDS
            rows = min(2 * NC, nrows - r0)
            tt = np.arange(rows * K3)
            rr, g3 = tt // K3, tt % K3
            assert (2 * (g3 * KS + (rr >> 1)) + (rr & 1)).max() < 2 * BQ_LDS
            assert (r0 * K3 + tt).max() < npts
        # ---------------------------------------------- scan, interpolation and pair loops
        chunk = -(-n // nt)
        lo = np.minimum(n, np.arange(nt) * chunk)
        hi = np.minimum(n, lo + chunk)
        cover = np.zeros(n, dtype=int)
        for a, b in zip(lo, hi):
            cover[a:b] += 1
        assert np.all(cover == 1)
        groups = nt // BQ_L
        atoms = np.arange(0, n, groups)[:, None] + np.arange(groups)[None, :]
        assert np.array_equal(np.sort(atoms[atoms < n]), np.arange(n))
        assert P <= BQ_L and K1 + 1 <= nt                        # interpolation lanes; hcnt zeroing
    assert seen_k
