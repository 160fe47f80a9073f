"""FP64 CPU oracle of the weighted f-checksum encoding (Sec. 2.1) applied to
the block-encoded product of Sec. 2.2.

TEST INFRASTRUCTURE: only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module.  It never imports the
GPU package, and the GPU package never imports it.

Sec. 2.1 protects p values x_1..x_p with f checksums y_r = sum_i w_ri x_i,
r = 1..f, and recovers any f lost values when every f x f submatrix of the
f x p weight matrix is nonsingular.  Here the p values are the Gr = m/br row
blocks of A (and the Gc = n/bc column blocks of B): A_f = [A; Y] with
Y_r = sum_g Wr[r, g] A_g (fr checksum block rows), B_f = [B, Z] with
Z_c = sum_h Wc[c, h] B_h (fc checksum block columns), and C_f = A_f B_f keeps
every relation (Eq. ABFT-GEMM with weighted checksum matrices):

  column relation (r, i, j): sum_g Wr[r, g] C_f[g br + i, j] = C_f[m + r br + i, j]
  row relation (x, c, jj):   sum_h Wc[c, h] C_f[x, h bc + jj] = C_f[x, n + c bc + jj]

for every column j < n + fc bc and every row x < m + fr br (corner included).
The relations of one column j and one residue i (all r) form a column group;
those of one row x and one residue jj (all c) a row group.

Arrays are numpy float64.  B_f is the paper's k x (n + fc bc) matrix.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import oracle as _orc

U64 = 2.0 ** -53
U32 = 2.0 ** -24
COND_MAX = 1e12            # largest 1-norm condition number of a recovery system accepted
CLEAN, DATA, CHECKSUM, MULTI = 0, 1, 2, 3
DIR_COL, DIR_ROW = 0, 1


def gamma(n: float, u: float = U64) -> float:
    return n * u / (1.0 - n * u)


# ---------------------------------------------------------------- encoding (Sec. 2.1, 2.2)
def wencode(A, B, Wr, Wc, br: int, bc: int):
    """A (m x k), B (k x n), Wr (fr x m/br), Wc (fc x n/bc) -> (A_f, B_f).
    Each checksum block is the weighted sum of the data blocks, accumulated
    over the blocks in increasing order in binary64."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    Wr = np.asarray(Wr, dtype=np.float64)
    Wc = np.asarray(Wc, dtype=np.float64)
    m, k = A.shape
    n = B.shape[1]
    assert m % br == 0 and n % bc == 0
    Gr, Gc = m // br, n // bc
    fr, fc = Wr.shape[0], Wc.shape[0]
    assert Wr.shape == (fr, Gr) and Wc.shape == (fc, Gc)
    Af = np.zeros((m + fr * br, k))
    Af[:m] = A
    for r in range(fr):
        acc = np.zeros((br, k))
        for g in range(Gr):
            acc += Wr[r, g] * A[g * br:(g + 1) * br]
        Af[m + r * br:m + (r + 1) * br] = acc
    Bf = np.zeros((k, n + fc * bc))
    Bf[:, :n] = B
    for c in range(fc):
        acc = np.zeros((k, bc))
        for h in range(Gc):
            acc += Wc[c, h] * B[:, h * bc:(h + 1) * bc]
        Bf[:, n + c * bc:n + (c + 1) * bc] = acc
    return Af, Bf


def wproduct(A, B, Wr, Wc, br: int, bc: int):
    """Encode and multiply in FP64: (A_f, B_f, C_f)."""
    Af, Bf = wencode(A, B, Wr, Wc, br, bc)
    return Af, Bf, _orc.gemm(Af, Bf)


# ---------------------------------------------------------------- residuals and thresholds
def residuals(Cf, m: int, n: int, br: int, bc: int, Wr, Wc):
    """Dc (fr, br, N): column relation residuals; Dr (M, fc, bc): row relation residuals."""
    Cf = np.asarray(Cf, dtype=np.float64)
    Wr = np.asarray(Wr, dtype=np.float64)
    Wc = np.asarray(Wc, dtype=np.float64)
    fr, Gr = Wr.shape
    fc, Gc = Wc.shape
    M, N = Cf.shape
    with np.errstate(invalid="ignore", over="ignore"):
        return _residuals(Cf, m, n, br, bc, Wr, Wc, fr, Gr, fc, Gc, M, N)


def _residuals(Cf, m, n, br, bc, Wr, Wc, fr, Gr, fc, Gc, M, N):
    Dc = np.empty((fr, br, N))
    for r in range(fr):
        acc = np.zeros((br, N))
        for g in range(Gr):
            acc += Wr[r, g] * Cf[g * br:(g + 1) * br]
        Dc[r] = acc - Cf[m + r * br:m + (r + 1) * br]
    Dr = np.empty((M, fc, bc))
    for c in range(fc):
        acc = np.zeros((M, bc))
        for h in range(Gc):
            acc += Wc[c, h] * Cf[:, h * bc:(h + 1) * bc]
        Dr[:, c] = acc - Cf[:, n + c * bc:n + (c + 1) * bc]
    return Dc, Dr


def wtau_det(Af, Bf, m: int, n: int, br: int, bc: int, Wr, Wc, kappa: float = 1.0 + 2.0 ** -20,
             u_acc: float = U64, u_st: float = 0.0):
    """Rigorous thresholds (tau_c (fr, br, N), tau_r (M, fc, bc)).

    Column relation (r, i, j): every computed entry of C_f is within
    gamma_k |a_x||b_j| <= gamma_k ||a_x||_2 ||b_j||_2 of its exact value
    (gamma of the product's accumulation roundoff u_acc); the stored checksum
    row is within gamma_Gr sum_g |w_rg||a_g| of the exact weighted sum (summed
    in binary64), plus u_st sum_g |w_rg||a_g| when that sum is then rounded to
    a narrower storage format (u_st = 2^-24 for binary32 checksum rows, 0 when
    they keep the binary64 sum); the binary64 relation sum adds gamma_{Gr+1}
    times the sum of the magnitudes of its terms.  With
    S = sum_g |w_rg| ||a_{g br + i}||_2 all of them are bounded by
    (2 gamma_k + u_st + 3 gamma_{Gr+1}) S ||b_j||_2 up to products of two
    roundoffs, which kappa covers.  Rows: the same with the roles swapped.
    Binary64 operands and product: u_acc = 2^-53, u_st = 0; binary32
    operands, checksum rows and product (accumulated in binary32):
    u_acc = u_st = 2^-24."""
    Af = np.asarray(Af, dtype=np.float64)
    Bf = np.asarray(Bf, dtype=np.float64)
    Wr = np.abs(np.asarray(Wr, dtype=np.float64))
    Wc = np.abs(np.asarray(Wc, dtype=np.float64))
    k = Af.shape[1]
    fr, Gr = Wr.shape
    fc, Gc = Wc.shape
    na = np.sqrt((Af * Af).sum(axis=1))          # ||A_f[x, :]||_2, x < M
    nb = np.sqrt((Bf * Bf).sum(axis=0))          # ||B_f[:, j]||_2, j < N
    S1 = np.zeros((fr, br))
    for r in range(fr):
        for g in range(Gr):
            S1[r] += Wr[r, g] * na[g * br:(g + 1) * br]
    S2 = np.zeros((fc, bc))
    for c in range(fc):
        for h in range(Gc):
            S2[c] += Wc[c, h] * nb[h * bc:(h + 1) * bc]
    cc = kappa * (2 * gamma(k, u_acc) + u_st + 3 * gamma(Gr + 1))
    cr = kappa * (2 * gamma(k, u_acc) + u_st + 3 * gamma(Gc + 1))
    tau_c = cc * S1[:, :, None] * nb[None, None, :]
    tau_r = cr * na[:, None, None] * S2[None, :, :]
    return tau_c, tau_r


# ---------------------------------------------------------------- verify (Sec. 2.2 consistency)
def erased_groups(M, N, br, bc, erasures):
    """Masks (br x N) and (M x bc) of the column and row groups that hold an
    element of a known erased rectangle (i0, j0, h, w)."""
    ec = np.zeros((br, N), dtype=bool)
    er = np.zeros((M, bc), dtype=bool)
    for (i0, j0, h, w) in erasures or []:
        for i in range(br):
            if (i - i0) % br < h:
                ec[i, j0:j0 + w] = True
        for jj in range(bc):
            if (jj - j0) % bc < w:
                er[i0:i0 + h, jj] = True
    return ec, er


def wverify(Cf, m, n, br, bc, Wr, Wc, tau_c, tau_r, erasures=None):
    """-> dict with the residuals, the failed column groups [(i, j, d[fr], t[fr])]
    and row groups [(x, jj, d[fc], t[fc])] in increasing order, and the number
    of groups skipped because they hold an element of a known erased
    rectangle (i0, j0, h, w).  A group fails when one of its relations has
    !(|D| <= tau) (NaN fails)."""
    Dc, Dr = residuals(Cf, m, n, br, bc, Wr, Wc)
    M, N = Cf.shape
    ec, er = erased_groups(M, N, br, bc, erasures)
    fail_c = ~np.all(np.abs(Dc) <= tau_c, axis=0) & ~ec          # (br, N)
    fail_r = ~np.all(np.abs(Dr) <= tau_r, axis=1) & ~er          # (M, bc)
    gc = [(int(i), int(j), Dc[:, i, j].copy(), tau_c[:, i, j].copy()) for i, j in np.argwhere(fail_c)]
    gr = [(int(x), int(jj), Dr[x, :, jj].copy(), tau_r[x, :, jj].copy()) for x, jj in np.argwhere(fail_r)]
    return {"Dc": Dc, "Dr": Dr, "col": gc, "row": gr, "excl_c": int(ec.sum()), "excl_r": int(er.sum())}


# ---------------------------------------------------------------- locate (single error per group)
def fit_group(d, t, W):
    """One failed group with residuals d (f) and thresholds t (f); W (f x G).

    A corrupted data member g with error delta gives d = W[:, g] delta (it is
    a summand of every relation); a corrupted checksum entry r gives
    d_r = -delta and leaves the other relations of the group intact.
    Returns (DATA, g), (CHECKSUM, r) or (MULTI, -1).  With f = 1 a data member
    cannot be told from its ratio and the answer is MULTI."""
    d = np.asarray(d, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    f, G = W.shape
    if not np.all(np.isfinite(d)):
        return MULTI, -1
    failed = [r for r in range(f) if not abs(d[r]) <= t[r]]
    if len(failed) == 1 and f >= 2:
        return CHECKSUM, failed[0]
    if len(failed) < 2:
        return MULTI, -1
    eps = 4.0 * (G + 2) * U64
    cands = []
    for g in range(G):
        w = W[:, g]
        delta = float(np.dot(w, d) / np.dot(w, w))
        fit = all(abs(d[r] - w[r] * delta) <= t[r] + eps * (abs(d[r]) + abs(w[r] * delta)) for r in range(f))
        if fit:
            cands.append(g)
    return (DATA, cands[0]) if len(cands) == 1 else (MULTI, -1)


def wlocate(groups_c, groups_r, m, n, br, bc, Wr, Wc):
    """Every failed group of the direction that carries two or more checksums
    (columns when fr >= 2, else rows when fc >= 2) is located on its own, so
    errors in distinct groups are located together.  -> [(cls, dir, i, j)]."""
    Wr = np.asarray(Wr, dtype=np.float64)
    Wc = np.asarray(Wc, dtype=np.float64)
    out = []
    if Wr.shape[0] >= 2:
        for (i, j, d, t) in groups_c:
            cls, q = fit_group(d, t, Wr)
            if cls == DATA:
                out.append((DATA, DIR_COL, q * br + i, j))
            elif cls == CHECKSUM:
                out.append((CHECKSUM, DIR_COL, m + q * br + i, j))
            else:
                out.append((MULTI, DIR_COL, -1, j))
    elif Wc.shape[0] >= 2:
        for (x, jj, d, t) in groups_r:
            cls, q = fit_group(d, t, Wc)
            if cls == DATA:
                out.append((DATA, DIR_ROW, x, q * bc + jj))
            elif cls == CHECKSUM:
                out.append((CHECKSUM, DIR_ROW, x, n + q * bc + jj))
            else:
                out.append((MULTI, DIR_ROW, x, -1))
    else:
        # one checksum each way: one failed column group and one failed row group meet in one element
        if len(groups_c) == 1 and len(groups_r) == 1:
            i, j = groups_c[0][0], groups_c[0][1]
            x, jj = groups_r[0][0], groups_r[0][1]
            if x % br == i and j % bc == jj:
                out.append((DATA if (x < m and j < n) else CHECKSUM, DIR_COL, x, j))
                return out
        if groups_c or groups_r:
            out.append((MULTI, DIR_COL, -1, -1))
    return out


# ---------------------------------------------------------------- correct / recover (Sec. 2.1)
def wcorrect(Cf, m, n, br, bc, Wr, Wc, loc):
    """Rebuild one located element in place from its group (never reading it):
    a data member from the lowest-numbered checksum relation, a checksum entry
    as the weighted sum of the data members."""
    cls, dr, i, j = loc
    assert cls in (DATA, CHECKSUM)
    Wr = np.asarray(Wr, dtype=np.float64)
    Wc = np.asarray(Wc, dtype=np.float64)
    if dr == DIR_COL:
        ok = _rebuild_line(Cf[:, j], m, br, Wr, [i // br], i % br)
    else:
        ok = _rebuild_line(Cf[i, :], n, bc, Wc, [j // bc], j % bc)
    assert ok == 0


def _rebuild_line(v, m, b, W, lost, res):
    """v: a view of one column (or row) of C_f; lost: block indices along it
    (g < G data blocks, G + r checksum block r); res: the residue (offset in
    the block).  Rebuild the lost members of the group `res` in place."""
    f, G = W.shape
    U = [g for g in lost if g < G]
    Lc = [g - G for g in lost if g >= G]
    R = [r for r in range(f) if r not in Lc][:len(U)]
    if len(R) < len(U):
        return -4
    S = np.zeros(f)
    for g in range(G):
        if g not in U:
            S += W[:, g] * v[g * b + res]
    if U:
        Wsub = W[np.ix_(R, U)]
        if np.linalg.cond(Wsub, 1) > COND_MAX:
            return -4
        rhs = np.array([v[m + r * b + res] - S[r] for r in R])
        x = np.linalg.solve(Wsub, rhs)
        for p, g in enumerate(U):
            v[g * b + res] = x[p]
            S += W[:, g] * x[p]
    for r in Lc:
        v[m + r * b + res] = S[r]
    return 0


def wrecover(Cf, m, n, br, bc, Wr, Wc, direction, blocks, lo, length):
    """Sec. 2.1 recovery of lost blocks.  direction DIR_COL: `blocks` are
    block-row indices (g < Gr data, Gr + r checksum block row r) lost over the
    columns [lo, lo + length); each column group is an f x f (or smaller)
    solve with the lowest-numbered intact checksum rows, after which the lost
    checksum blocks are recomputed.  DIR_ROW: the same on block columns over
    the rows [lo, lo + length).  In place; 0, or -4 when more data blocks are
    lost than checksums survive or the system is singular (1-norm condition
    number above COND_MAX)."""
    Wr = np.asarray(Wr, dtype=np.float64)
    Wc = np.asarray(Wc, dtype=np.float64)
    blocks = sorted(set(int(g) for g in blocks))
    if direction == DIR_COL:
        W, b, base = Wr, br, m
    else:
        W, b, base = Wc, bc, n
    f, G = W.shape
    U = [g for g in blocks if g < G]
    if len(U) > f - len([g for g in blocks if g >= G]):
        return -4
    for pos in range(lo, lo + length):
        line = Cf[:, pos] if direction == DIR_COL else Cf[pos, :]
        for res in range(b):
            st = _rebuild_line(line, base, b, W, blocks, res)
            if st:
                return st
    return 0


def vandermonde(f: int, G: int, nodes=None) -> np.ndarray:
    """f x G weights w_rg = x_g^r with distinct positive nodes (default 1..G):
    every square submatrix taken on any rows and columns is nonsingular (the
    Sec. 2.1 condition)."""
    x = np.arange(1, G + 1, dtype=np.float64) if nodes is None else np.asarray(nodes, dtype=np.float64)
    return np.stack([x ** r for r in range(f)])


def all_lost_sets(G: int, f: int, size: int):
    return itertools.combinations(range(G + f), size)
