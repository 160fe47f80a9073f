"""Pins of the weighted f-checksum oracle (Sec. 2.1 encoding on the block
product of Sec. 2.2) to facts other than itself: the unit-weight case reduces
to the plain block checksum oracle, a hand-computed Sec. 2.1 example, exact
relations on integers, brute force over every lost-block set up to f (and the
singular and too-many cases), the rounding theorem behind the threshold, and
brute-force location of every single-element error and of error pairs."""
import itertools

import numpy as np
import pytest

from oracle import weighted as wo
from paper_0806_3121_amd import synth


def int_problem(m, n, k, lo=-8, hi=8, seed=7):
    A = synth.uniform_ints(seed, synth.STREAM_A, m, k, lo, hi)
    B = synth.uniform_ints(seed, synth.STREAM_B, k, n, lo, hi)
    return A, B


def flip_bit(x: float, bit: int) -> float:
    v = np.array([x], dtype=np.float64).view(np.uint64)
    v ^= np.uint64(1) << np.uint64(bit)
    return float(v.view(np.float64)[0])


# ---------------------------------------------------------------- encoding
def test_unit_weights_reduce_to_block_checksum(orc):
    """f = 1 with unit weights is the stacked-identity checksum of Sec. 2.2."""
    m, n, k, br, bc = 12, 10, 7, 3, 2
    A = synth.uniform(3, synth.STREAM_A, m, k)
    B = synth.uniform(3, synth.STREAM_B, k, n)
    Af, Bf, Cf = wo.wproduct(A, B, np.ones((1, m // br)), np.ones((1, n // bc)), br, bc)
    Af0, Bf0, Cf0 = orc.protected_product(A, B, br, bc)
    assert np.array_equal(Af, Af0) and np.array_equal(Bf, Bf0) and np.array_equal(Cf, Cf0)


def test_section_2_1_checksums_by_hand():
    """p = 3 values (blocks of one row), f = 2: y1 = x1 + x2 + x3 and
    y2 = x1 + 2 x2 + 3 x3, written out."""
    A = np.array([[1.0, -2.0], [4.0, 0.5], [3.0, 7.0]])
    W = np.array([[1.0, 1.0, 1.0], [1.0, 2.0, 3.0]])
    Af, _ = wo.wencode(A, np.eye(2), W, np.ones((1, 2)), 1, 1)
    assert np.array_equal(Af[3], [1 + 4 + 3, -2 + 0.5 + 7])
    assert np.array_equal(Af[4], [1 + 2 * 4 + 3 * 3, -2 + 2 * 0.5 + 3 * 7])
    # B side: columns of B are the values
    B = np.array([[1.0, 2.0, 3.0, 4.0]])
    Wc = np.array([[2.0, -1.0], [0.5, 4.0]])
    _, Bf = wo.wencode(np.ones((1, 1)), B, np.ones((1, 1)), Wc, 1, 2)
    # blocks of width 2: Z_c = Wc[c,0] B[:, 0:2] + Wc[c,1] B[:, 2:4]
    assert np.array_equal(Bf[0, 4:6], [2 * 1 - 3, 2 * 2 - 4])
    assert np.array_equal(Bf[0, 6:8], [0.5 * 1 + 4 * 3, 0.5 * 2 + 4 * 4])


@pytest.mark.parametrize("fr,fc,br,bc", [(2, 2, 3, 2), (3, 1, 2, 5), (4, 3, 1, 1)])
def test_weighted_relations_exact_on_integers(orc, fr, fc, br, bc):
    """Eq. ABFT-GEMM with weighted checksum matrices: (W^T A) B = W^T (A B),
    A (B V) = (A B) V, corner both ways; exact on integer data and weights."""
    m, n, k = 12, 10, 9
    A, B = int_problem(m, n, k, seed=fr * 10 + fc)
    Wr = wo.vandermonde(fr, m // br)
    Wc = wo.vandermonde(fc, n // bc, nodes=np.arange(2, n // bc + 2))
    Af, Bf, Cf = wo.wproduct(A, B, Wr, Wc, br, bc)
    Ci = A.astype(np.int64) @ B.astype(np.int64)
    assert np.array_equal(Cf[:m, :n], Ci.astype(np.float64))
    Dc, Dr = wo.residuals(Cf, m, n, br, bc, Wr, Wc)
    assert not Dc.any() and not Dr.any()
    # the corner block: weighted sums of the carried row block equal those of the carried column block
    corner = Cf[m:, n:]
    Wi = Wr.astype(np.int64)
    Vi = Wc.astype(np.int64)
    full = np.zeros((fr * br, fc * bc), dtype=np.int64)
    for r in range(fr):
        for c in range(fc):
            for g in range(m // br):
                for h in range(n // bc):
                    full[r * br:(r + 1) * br, c * bc:(c + 1) * bc] += \
                        Wi[r, g] * Vi[c, h] * Ci[g * br:(g + 1) * br, h * bc:(h + 1) * bc]
    assert np.array_equal(corner, full.astype(np.float64))
    rep = wo.wverify(Cf, m, n, br, bc, Wr, Wc, np.zeros_like(Dc), np.zeros_like(Dr))
    assert rep["col"] == [] and rep["row"] == []


# ---------------------------------------------------------------- recovery of lost blocks
@pytest.mark.parametrize("direction", [wo.DIR_COL, wo.DIR_ROW])
def test_any_f_lost_blocks_rebuilt_exactly(orc, direction):
    """Sec. 2.1: with every f x f submatrix nonsingular, any f lost blocks
    (data or checksum) are rebuilt; brute force over every set of 1..f."""
    m, n, k, br, bc, f = 12, 12, 5, 3, 3, 2
    A, B = int_problem(m, n, k, seed=11)
    Wr = wo.vandermonde(f, m // br)
    Wc = wo.vandermonde(f, n // bc)
    Af, Bf, Cf = wo.wproduct(A, B, Wr, Wc, br, bc)
    G = m // br
    b = br
    count = 0
    for size in (1, 2):
        for lost in wo.all_lost_sets(G, f, size):
            Cx = Cf.copy()
            for g in lost:
                if direction == wo.DIR_COL:
                    Cx[g * b:(g + 1) * b, :] = np.nan
                else:
                    Cx[:, g * b:(g + 1) * b] = np.nan
            L = Cx.shape[1] if direction == wo.DIR_COL else Cx.shape[0]
            assert wo.wrecover(Cx, m, n, br, bc, Wr, Wc, direction, lost, 0, L) == 0, lost
            assert np.abs(Cx - Cf).max() < 1e-9, lost
            assert np.array_equal(np.rint(Cx), Cf), lost
            count += 1
    assert count == 6 + 15


def test_more_than_f_lost_or_singular_is_refused(orc):
    m, n, k, br, bc, f = 12, 12, 5, 3, 3, 2
    A, B = int_problem(m, n, k, seed=12)
    Wr = wo.vandermonde(f, 4)
    Wc = wo.vandermonde(f, 4)
    _, _, Cf = wo.wproduct(A, B, Wr, Wc, br, bc)
    for lost in wo.all_lost_sets(4, f, 3):
        assert wo.wrecover(Cf.copy(), m, n, br, bc, Wr, Wc, wo.DIR_COL, lost, 0, 18) == -4
    # two equal weight columns: blocks 1 and 2 cannot be told apart
    Ws = np.array([[1.0, 1.0, 1.0, 1.0], [1.0, 2.0, 2.0, 4.0]])
    _, _, Cs = wo.wproduct(A, B, Ws, Wc, br, bc)
    assert wo.wrecover(Cs.copy(), m, n, br, bc, Ws, Wc, wo.DIR_COL, [1, 2], 0, 18) == -4
    assert wo.wrecover(Cs.copy(), m, n, br, bc, Ws, Wc, wo.DIR_COL, [0, 2], 0, 18) == 0


# ---------------------------------------------------------------- thresholds
@pytest.mark.parametrize("m,n,k,br,bc,fr,fc,signed", [
    (64, 48, 200, 8, 4, 2, 2, False), (40, 60, 333, 1, 1, 3, 2, True), (96, 96, 64, 32, 32, 4, 4, False),
])
def test_det_threshold_bounds_clean_residuals(orc, m, n, k, br, bc, fr, fc, signed):
    """The rounding theorem behind wtau_det: no clean relation exceeds its
    threshold, on random binary64 data with random (and signed) weights, and
    the threshold is far below the data's scale."""
    worst = 0.0
    for seed in range(4):
        A = synth.uniform(seed, synth.STREAM_A, m, k)
        B = synth.uniform(seed, synth.STREAM_B, k, n)
        lo, hi = (-1.0, 1.0) if signed else (0.5, 1.5)
        Wr = lo + (hi - lo) * (synth.uniform(seed, synth.STREAM_X, fr, m // br) + 1) / 2
        Wc = lo + (hi - lo) * (synth.uniform(seed, synth.STREAM_PICK, fc, n // bc) + 1) / 2
        Af, Bf, Cf = wo.wproduct(A, B, Wr, Wc, br, bc)
        tc, tr = wo.wtau_det(Af, Bf, m, n, br, bc, Wr, Wc)
        Dc, Dr = wo.residuals(Cf, m, n, br, bc, Wr, Wc)
        assert np.all(np.abs(Dc) <= tc) and np.all(np.abs(Dr) <= tr)
        worst = max(worst, (np.abs(Dc) / tc).max(), (np.abs(Dr) / tr).max())
        assert tc.max() < 1e-10 * np.abs(Cf).max() and tr.max() < 1e-10 * np.abs(Cf).max()
    assert worst > 1e-4          # the bound is not vacuous


@pytest.mark.parametrize("m,n,k,br,bc,fr,fc,positive", [
    (64, 48, 200, 8, 4, 2, 2, False), (40, 60, 333, 1, 1, 3, 2, False), (96, 96, 64, 32, 32, 4, 4, False),
    (64, 32, 4096, 8, 4, 2, 2, True),
])
def test_det_threshold_binary32_bounds_binary32_residuals(orc, m, n, k, br, bc, fr, fc, positive):
    """Binary32 operands, checksum rows summed in binary64 and rounded once to
    binary32, and the product accumulated in binary32 by an independent
    routine (numpy's single-precision matrix product): no clean relation
    exceeds the binary32 threshold (u_acc = u_st = 2^-24), the largest
    residual is a sizeable part of it, and the binary64 threshold of the same
    operands is exceeded.  Positive operands at k = 4096: the accumulation
    errors of the binary32 products are many times the storage rounding of
    the checksum rows, so only the product term covers them."""
    worst, over64 = 0.0, False
    for seed in range(3):
        A = synth.uniform(seed, synth.STREAM_A, m, k, np.float32).astype(np.float64)
        B = synth.uniform(seed, synth.STREAM_B, k, n, np.float32).astype(np.float64)
        if positive:                                     # in [0.5, 1.5], rounded to binary32 operands
            A = ((A + 2.0) / 2.0).astype(np.float32).astype(np.float64)
            B = ((B + 2.0) / 2.0).astype(np.float32).astype(np.float64)
        Wr = 0.5 + (synth.uniform(seed, synth.STREAM_X, fr, m // br) + 1) / 2
        Wc = -1.0 + (synth.uniform(seed, synth.STREAM_PICK, fc, n // bc) + 1)
        Af, Bf = wo.wencode(A, B, Wr, Wc, br, bc)
        Af32, Bf32 = Af.astype(np.float32), Bf.astype(np.float32)
        Cf = (Af32 @ Bf32).astype(np.float64)
        tc, tr = wo.wtau_det(Af32, Bf32, m, n, br, bc, Wr, Wc, u_acc=wo.U32, u_st=wo.U32)
        Dc, Dr = wo.residuals(Cf, m, n, br, bc, Wr, Wc)
        assert np.all(np.abs(Dc) <= tc) and np.all(np.abs(Dr) <= tr)
        worst = max(worst, (np.abs(Dc) / tc).max(), (np.abs(Dr) / tr).max())
        t64c, t64r = wo.wtau_det(Af32, Bf32, m, n, br, bc, Wr, Wc)
        over64 |= bool(np.any(np.abs(Dc) > t64c) or np.any(np.abs(Dr) > t64r))
    assert worst > 2e-4 and over64, worst


@pytest.mark.parametrize("wlo,whi", [(0.5, 1.5), (100.0, 1000.0)])
def test_det_threshold_needs_its_summation_term(orc, wlo, whi):
    """Positive data and weights, k = 1, Gr = 2048 groups: the relation sums
    round at every partial sum, so their error is a large part of the
    threshold (beyond the product term 2 gamma_k alone) while still under it;
    large weights enter the threshold with their magnitude."""
    m, n, k = 2048, 8, 1
    A = (synth.uniform(1, synth.STREAM_A, m, k) + 1) / 2
    B = (synth.uniform(1, synth.STREAM_B, k, n) + 1) / 2
    Wr = wlo + (whi - wlo) * (synth.uniform(1, synth.STREAM_X, 2, m) + 1) / 2
    Wc = np.ones((1, n))
    Af, Bf, Cf = wo.wproduct(A, B, Wr, Wc, 1, 1)
    tc, tr = wo.wtau_det(Af, Bf, m, n, 1, 1, Wr, Wc)
    Dc, _ = wo.residuals(Cf, m, n, 1, 1, Wr, Wc)
    ratio = (np.abs(Dc) / tc).max()
    product_share = 2 * wo.gamma(k) / (2 * wo.gamma(k) + 3 * wo.gamma(m + 1))
    assert product_share < ratio <= 1.0, (ratio, product_share)


# ---------------------------------------------------------------- location and correction
def _setup_small(fr, fc, seed=5):
    m, n, k, br, bc = 8, 6, 4, 2, 3
    A, B = int_problem(m, n, k, seed=seed)
    Wr = 0.5 + (synth.uniform(seed, synth.STREAM_X, fr, m // br) + 1) / 2
    Wc = 0.5 + (synth.uniform(seed, synth.STREAM_PICK, fc, n // bc) + 1) / 2
    Af, Bf, Cf = wo.wproduct(A, B, Wr, Wc, br, bc)
    tc, tr = wo.wtau_det(Af, Bf, m, n, br, bc, Wr, Wc)
    return m, n, br, bc, Wr, Wc, Cf, tc, tr


@pytest.mark.parametrize("fr,fc", [(2, 1), (1, 2), (3, 3)])
def test_every_element_every_exponent_bit_located_and_corrected(orc, fr, fc):
    """Brute force: a flip of any exponent or high fraction bit of any element
    of C_f is located by the weight ratios of its group (the direction with
    f >= 2), classified data/checksum, and rebuilt to within rounding; a flip
    that makes the element non-finite is refused (MULTI)."""
    m, n, br, bc, Wr, Wc, Cf, tc, tr = _setup_small(fr, fc)
    M, N = Cf.shape
    scale = np.abs(Cf).max()
    for x in range(M):
        for y in range(N):
            for bit in range(44, 63):
                Cx = Cf.copy()
                Cx[x, y] = flip_bit(Cf[x, y], bit)
                if np.isfinite(Cx[x, y]) and abs(Cx[x, y] - Cf[x, y]) < 1e-6 * scale:
                    continue                  # below every threshold's reach (a flip of a zero or tiny entry)
                rep = wo.wverify(Cx, m, n, br, bc, Wr, Wc, tc, tr)
                locs = wo.wlocate(rep["col"], rep["row"], m, n, br, bc, Wr, Wc)
                if not np.isfinite(Cx[x, y]):
                    assert [l[0] for l in locs] == [wo.MULTI], (x, y, bit)
                    continue
                assert len(locs) == 1, (x, y, bit, locs)
                cls, dr, i, j = locs[0]
                if fr >= 2:
                    want = wo.DATA if x < m else wo.CHECKSUM
                else:
                    want = wo.DATA if y < n else wo.CHECKSUM
                assert (cls, i, j) == (want, x, y), (x, y, bit, locs)
                wo.wcorrect(Cx, m, n, br, bc, Wr, Wc, locs[0])
                assert abs(Cx[x, y] - Cf[x, y]) <= 1e-13 * scale, (x, y, bit)
                rep = wo.wverify(Cx, m, n, br, bc, Wr, Wc, tc, tr)
                assert rep["col"] == [] and rep["row"] == []


def test_two_errors_in_distinct_column_groups_both_located(orc):
    """With fr >= 2 each column group is located on its own: two flips in
    different groups are both found (the f = 1 intersection rule cannot)."""
    m, n, br, bc, Wr, Wc, Cf, tc, tr = _setup_small(2, 1, seed=9)
    M, N = Cf.shape
    rng = [(x, y) for x in range(M) for y in range(N)]
    for (p, q) in itertools.combinations(range(len(rng)), 2):
        (x1, y1), (x2, y2) = rng[p], rng[q]
        if y1 == y2 and x1 % br == x2 % br:
            continue                      # the same column group: two unknowns, one ratio
        Cx = Cf.copy()
        Cx[x1, y1] += 3.0
        Cx[x2, y2] -= 5.0
        rep = wo.wverify(Cx, m, n, br, bc, Wr, Wc, tc, tr)
        locs = sorted((l[2], l[3]) for l in wo.wlocate(rep["col"], rep["row"], m, n, br, bc, Wr, Wc))
        assert locs == sorted([(x1, y1), (x2, y2)]), (x1, y1, x2, y2)


def test_single_checksums_fall_back_to_intersection(orc):
    m, n, br, bc, Wr, Wc, Cf, tc, tr = _setup_small(1, 1)
    Cx = Cf.copy()
    Cx[3, 4] += 2.0
    rep = wo.wverify(Cx, m, n, br, bc, Wr, Wc, tc, tr)
    assert wo.wlocate(rep["col"], rep["row"], m, n, br, bc, Wr, Wc) == [(wo.DATA, wo.DIR_COL, 3, 4)]
    Cx[0, 0] += 2.0
    rep = wo.wverify(Cx, m, n, br, bc, Wr, Wc, tc, tr)
    assert [l[0] for l in wo.wlocate(rep["col"], rep["row"], m, n, br, bc, Wr, Wc)] == [wo.MULTI]


def test_known_erasure_skips_exactly_its_groups(orc):
    m, n, br, bc, Wr, Wc, Cf, tc, tr = _setup_small(2, 2)
    M, N = Cf.shape
    rect = (2, 1, 3, 2)                 # rows 2..4 (residues 0, 1 of br = 2), columns 1..2
    Cx = Cf.copy()
    Cx[2:5, 1:3] = np.nan
    rep = wo.wverify(Cx, m, n, br, bc, Wr, Wc, tc, tr, erasures=[rect])
    assert rep["col"] == [] and rep["row"] == []
    # brute force: a group is skipped iff one of its members lies in the rectangle
    want_c = sum(any(2 <= x < 5 and 1 <= j < 3 for x in range(i, M, br)) for i in range(br) for j in range(N))
    want_r = sum(any(2 <= x < 5 and 1 <= y < 3 for y in range(jj, N, bc)) for x in range(M) for jj in range(bc))
    assert (rep["excl_c"], rep["excl_r"]) == (want_c, want_r)
    assert wo.wrecover(Cx, m, n, br, bc, Wr, Wc, wo.DIR_COL, [1, 2], 1, 2) == 0
    assert np.abs(Cx - Cf).max() <= 1e-13 * np.abs(Cf).max()
