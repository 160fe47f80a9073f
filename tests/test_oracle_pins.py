"""Pins of the FP64 CPU oracle to facts other than itself.

Each test checks the oracle against something the paper or the mathematics
fixes: exact integer arithmetic, a library routine, a closed form, a theorem
(the rounding bound behind the threshold), brute force on tiny inputs, or a
published test vector.  A dropped term, a wrong sign or index or a transposed
operand in the oracle fails at least one of them.
"""
import os

import numpy as np
import pytest

from paper_0806_3121_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def int_problem(m, n, k, lo=-8, hi=8, seed=7):
    A = synth.uniform_ints(seed, synth.STREAM_A, m, k, lo, hi)
    B = synth.uniform_ints(seed, synth.STREAM_B, k, n, lo, hi)
    return A, B


# ---------------------------------------------------------------- generator
def test_splitmix64_published_vector():
    lines = [ln for ln in open(os.path.join(GOLDEN, "splitmix64.txt")) if ln.strip() and not ln.startswith("#")]
    seed = int(lines[0].split()[1])
    expect = [int(x) for x in lines[1:]]
    state, got = seed, []
    for _ in expect:
        state = (state + int(synth.GAMMA)) & synth.MASK64
        got.append(synth.mix64_int(state))
    assert got == expect
    # the counter form used for matrices is the same sequence
    key = 1234567
    z = [synth.mix64_int((key + (i + 1) * int(synth.GAMMA)) & synth.MASK64) for i in range(5)]
    assert z == expect


def test_uniform_range_and_exactness():
    x = synth.uniform(3, 0, 64, 64)
    assert x.min() >= -1.0 and x.max() < 1.0
    # every value is an integer multiple of 2^-52 (exact map)
    assert np.all((x + 1.0) * 2.0 ** 52 == np.floor((x + 1.0) * 2.0 ** 52))
    y = synth.uniform(3, 0, 64, 64, np.float32)
    assert y.dtype == np.float32 and y.min() >= -1 and y.max() < 1


# ---------------------------------------------------------------- product
def test_gemm_integer_exact(orc):
    # integer inputs: every partial sum is an integer < 2^53, so the FP64
    # product must equal the exact integer product in any order
    A, B = int_problem(37, 29, 53)
    Cm = orc.gemm(A, B)
    exact = A.astype(np.int64) @ B.astype(np.int64)
    assert np.array_equal(Cm, exact.astype(np.float64))


def test_gemm_matches_library_within_gamma_bound(orc):
    A = synth.uniform(11, 0, 40, 300)
    B = synth.uniform(11, 1, 300, 33)
    Cm = orc.gemm(A, B)
    ref = A @ B
    g = orc.lib().orc_gamma(300.0, orc.U64)
    bound = 2 * g * (np.abs(A) @ np.abs(B))
    assert np.all(np.abs(Cm - ref) <= bound)
    # and the dot entry point is the same ascending-order sum, bit for bit
    for (i, j) in [(0, 0), (5, 17), (39, 32)]:
        assert orc.dot(A[i], B[:, j]) == Cm[i, j]


def test_gemm_not_transposed(orc):
    A = np.arange(6, dtype=np.float64).reshape(2, 3)
    B = np.arange(12, dtype=np.float64).reshape(3, 4)
    assert np.array_equal(orc.gemm(A, B), np.array([[20, 23, 26, 29], [56, 68, 80, 92]], dtype=np.float64))


# ---------------------------------------------------------------- encoding
@pytest.mark.parametrize("br,bc", [(1, 1), (2, 3), (4, 1), (1, 6), (12, 6)])
def test_encoding_block_sums_exact(orc, br, bc):
    m, n, k = 24, 18, 10
    A, B = int_problem(m, n, k)
    Af, Bf = orc.encode(A, B, br, bc)
    Ai = A.astype(np.int64)
    Bi = B.astype(np.int64)
    # C_C^T A: rows of block g at residue r summed over g
    want_rows = sum(Ai[g * br:(g + 1) * br] for g in range(m // br))
    want_cols = sum(Bi[:, h * bc:(h + 1) * bc] for h in range(n // bc))
    assert np.array_equal(Af[:m], A) and np.array_equal(Bf[:, :n], B)
    assert np.array_equal(Af[m:], want_rows.astype(np.float64))
    assert np.array_equal(Bf[:, n:], want_cols.astype(np.float64))


@pytest.mark.parametrize("br,bc", [(1, 1), (3, 2), (6, 6)])
def test_eq_abft_gemm_consistency_exact(orc, br, bc):
    """Eq. ABFT-GEMM: C_C^T(AB) = (C_C^T A)B, (AB)C_R = A(BC_R), and the
    corner agrees both ways; exact for integer inputs."""
    m, n, k = 18, 12, 30
    A, B = int_problem(m, n, k, seed=3)
    Af, Bf, Cf = orc.protected_product(A, B, br, bc)
    Ci = (A.astype(np.int64) @ B.astype(np.int64))
    assert np.array_equal(Cf[:m, :n], Ci.astype(np.float64))
    col_sum = sum(Cf[g * br:(g + 1) * br] for g in range(m // br))   # C_C^T C_f over data rows
    row_sum = sum(Cf[:, h * bc:(h + 1) * bc] for h in range(n // bc))
    assert np.array_equal(col_sum, Cf[m:])          # carried row block (incl. corner)
    assert np.array_equal(row_sum, Cf[:, n:])       # carried column block (incl. corner)
    tc = np.zeros((br, n + bc))
    tr = np.zeros((m + br, bc))
    Dc, Dr, rep = orc.verify(Cf, m, n, br, bc, tc, tr)
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0
    assert not Dc.any() and not Dr.any()


# ---------------------------------------------------------------- thresholds
@pytest.mark.parametrize("br,bc", [(1, 1), (16, 16), (64, 1), (128, 128)])
def test_det_threshold_bounds_clean_residual(orc, br, bc):
    """|D| <= tau_det on clean FP64 data is a theorem (rounding-error bound)."""
    m = n = 128
    k = 200
    A = synth.uniform(5, 0, m, k)
    B = synth.uniform(5, 1, k, n)
    Af, Bf, Cf = orc.protected_product(A, B, br, bc)
    tc, tr = orc.tau_det(Af, Bf, m, n, br, bc)
    Dc, Dr, rep = orc.verify(Cf, m, n, br, bc, tc, tr)
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0
    assert rep.max_ratio_c < 1.0 and rep.max_ratio_r < 1.0
    assert np.all(np.abs(Dc) <= tc) and np.all(np.abs(Dr) <= tr)


def test_norms_bound_the_tight_sum(orc):
    """Cauchy-Schwarz: (C_C^T|A|)|B_f| <= na_abs * nb and |A_f|(|B|C_R) <= na * nb_abs,
    with the tight sums computed by the library matmul; the norms themselves
    match numpy's."""
    m, n, k, br, bc = 32, 24, 50, 8, 4
    A = synth.uniform(9, 0, m, k)
    B = synth.uniform(9, 1, k, n)
    Af, Bf = orc.encode(A, B, br, bc)
    na, na_abs, nb, nb_abs = orc.norms(Af, Bf, m, n, br, bc)
    assert np.allclose(na, np.linalg.norm(Af, axis=1), rtol=1e-14)
    assert np.allclose(nb, np.linalg.norm(Bf, axis=0), rtol=1e-14)
    cabsA = sum(np.abs(A[g * br:(g + 1) * br]) for g in range(m // br))
    absBcr = sum(np.abs(B[:, h * bc:(h + 1) * bc]) for h in range(n // bc))
    assert np.allclose(na_abs, np.linalg.norm(cabsA, axis=1), rtol=1e-14)
    assert np.allclose(nb_abs, np.linalg.norm(absBcr, axis=0), rtol=1e-14)
    tight_c = cabsA @ np.abs(Bf)
    tight_r = np.abs(Af) @ absBcr
    assert np.all(tight_c <= np.outer(na_abs, nb) * (1 + 1e-12))
    assert np.all(tight_r <= np.outer(na, nb_abs) * (1 + 1e-12))


def test_det_threshold_is_not_vacuous(orc):
    """A mantissa flip in the top 12 bits of a unit-size FP64 value must exceed
    tau_det by orders of magnitude at the paper's nb=64 scale."""
    m = n = k = 256
    A = synth.uniform(1, 0, m, k)
    B = synth.uniform(1, 1, k, n)
    Af, Bf = orc.encode(A, B, 1, 1)
    tc, tr = orc.tau_det(Af, Bf, m, n, 1, 1)
    assert tc.max() < 1e-6 and tr.max() < 1e-6
    assert 2.0 ** (40 - 52) > 1e3 * max(tc.max(), tr.max())


def test_stat_q_matches_library_gemv(orc):
    """For br = bc = 1 the stat threshold's Q is an exact GEMV:
    Q_c = v (B_f o B_f), v = colsum(A o A) + A_cs o A_cs, Q_r = (A_f o A_f) w."""
    m, n, k = 40, 30, 64
    A = synth.uniform(2, 0, m, k)
    B = synth.uniform(2, 1, k, n)
    Af, Bf = orc.encode(A, B, 1, 1)
    T, lam, u = 16.0, 10.0, orc.U32
    tc, tr = orc.tau_stat(Af, Bf, m, n, 1, 1, u_acc=u, T=T, s_store=1.0, lam=lam)
    v = (Af ** 2).sum(axis=0)                       # includes the checksum row
    w = (Bf ** 2).sum(axis=1)                       # includes the checksum column
    coef = u * u / 3 * (T / 2 + 1)
    assert np.allclose(tc[0], lam * np.sqrt(coef * (v @ Bf ** 2)), rtol=1e-12)
    assert np.allclose(tr[:, 0], lam * np.sqrt(coef * ((Af ** 2) @ w)), rtol=1e-12)


def test_stat_model_matches_simulated_fp32_accumulation(orc):
    """The stat sigma (tau/lambda) predicts the spread of D when every member
    of a relation is accumulated in binary32 with one rounding per step of
    4 products (simulated with numpy float32); rms(D/sigma) must come out
    near the model's ~0.6-1, not off by the sqrt(T/2) factor a dropped term
    would cause."""
    rng_seed = 13
    m, n, k = 64, 48, 1024
    A = synth.uniform(rng_seed, 0, m, k, np.float32).astype(np.float64)
    B = synth.uniform(rng_seed, 1, k, n, np.float32).astype(np.float64)
    Af, Bf = orc.encode(A, B, 1, 1, store_f32=True)
    step = 4
    T = k / step
    # binary32 accumulation: exact block of 4 products, one rounding per step
    prods = Af[:, None, :] * Bf.T[None, :, :]                       # (M, N, k) float64, exact
    blocks = prods.reshape(m + 1, n + 1, k // step, step).sum(axis=3)  # exact in f64 for these sizes
    acc = np.zeros((m + 1, n + 1), dtype=np.float32)
    for t in range(blocks.shape[2]):
        acc = (acc.astype(np.float64) + blocks[:, :, t]).astype(np.float32)
    Cf = acc.astype(np.float64)
    tc, tr = orc.tau_stat(Af, Bf, m, n, 1, 1, u_acc=orc.U32, T=T, s_store=1.0, lam=1.0)
    Dc, Dr, _ = orc.verify(Cf, m, n, 1, 1, tc, tr)
    z = np.concatenate([(Dc / tc).ravel(), (Dr / tr).ravel()])
    rms = np.sqrt(np.mean(z ** 2))
    assert 0.6 < rms < 1.0, rms          # T for T/2 would give ~0.53, a dropped T term ~10
    assert np.abs(z).max() < 6.0


# Hand-worked threshold values.  The sizes are chosen so that every index of
# the rigorous bound is visible: k = 2 products per entry (gamma_k = gamma_2),
# G = 2 blocks, so each relation sum adds G values and subtracts the stored
# checksum, which itself carries a (G-1)-term sum: gamma_{G+1} = gamma_3.
_A2 = np.array([[1.0, 2.0], [3.0, 4.0]])
_B2 = np.array([[5.0, -6.0], [7.0, 8.0]])
_A4 = np.array([[1.0, 2.0], [3.0, -4.0], [5.0, 6.0], [-7.0, 8.0]])
_B4 = np.array([[1.0, -2.0, 3.0, 0.0], [2.0, 1.0, -1.0, 4.0]])


def _gamma(n, u):
    return n * u / (1 - n * u)


def test_det_threshold_hand_value_b1(orc):
    """m = n = k = 2, b = 1.  By hand: A_f = [[1,2],[3,4],[4,6]],
    B_f = [[5,-6,-1],[7,8,15]]; C_C^T|A| = [4,6] (norm sqrt 52), |B| C_R =
    [11,15]^T (norm sqrt 346); column norms of B_f sqrt 74, 10, sqrt 226; row
    norms of A_f sqrt 5, 5, sqrt 52.  tau = kappa (2 gamma_2 + 2 gamma_3 +
    u_st) x (the two norms)."""
    kappa = 1 + 2.0 ** -20
    u = 2.0 ** -53
    Af, Bf = orc.encode(_A2, _B2, 1, 1)
    assert np.array_equal(Af, [[1, 2], [3, 4], [4, 6]]) and np.array_equal(Bf, [[5, -6, -1], [7, 8, 15]])
    coef = kappa * (2 * _gamma(2, u) + 2 * _gamma(3, u))
    want_c = coef * np.sqrt(52.0) * np.array([np.sqrt(74.0), 10.0, np.sqrt(226.0)])
    want_r = coef * np.array([np.sqrt(5.0), 5.0, np.sqrt(52.0)]) * np.sqrt(346.0)
    tc, tr = orc.tau_det(Af, Bf, 2, 2, 1, 1)
    assert np.allclose(tc[0], want_c, rtol=1e-13, atol=0)
    assert np.allclose(tr[:, 0], want_r, rtol=1e-13, atol=0)
    # binary32 accumulation with binary32-stored checksums: gamma_2 at 2^-24,
    # the relation sum still in binary64, plus one storage rounding u_st
    u32 = 2.0 ** -24
    coef32 = kappa * (2 * _gamma(2, u32) + 2 * _gamma(3, u) + u32)
    tc, tr = orc.tau_det(Af, Bf, 2, 2, 1, 1, u_acc=u32, u_st=u32)
    assert np.allclose(tc[0], coef32 * np.sqrt(52.0) * np.array([np.sqrt(74.0), 10.0, np.sqrt(226.0)]),
                       rtol=1e-13, atol=0)


def test_det_threshold_hand_value_b2(orc):
    """m = n = 4, k = 2, br = bc = 2 (G = 2 blocks each way).  By hand:
    C_C^T A = [[6,8],[-4,4]]; C_C^T|A| rows [6,8] and [10,12] (norms 10 and
    sqrt 244); B C_R = [[4,-2],[1,5]]; |B| C_R columns [4,3] and [2,5] (norms 5
    and sqrt 29); column norms of B_f sqrt 5, sqrt 5, sqrt 10, 4, sqrt 17,
    sqrt 29; row norms of A_f sqrt 5, 5, sqrt 61, sqrt 113, 10, sqrt 32."""
    kappa = 1 + 2.0 ** -20
    u = 2.0 ** -53
    Af, Bf = orc.encode(_A4, _B4, 2, 2)
    assert np.array_equal(Af[4:], [[6, 8], [-4, 4]]) and np.array_equal(Bf[:, 4:], [[4, -2], [1, 5]])
    coef = kappa * (2 * _gamma(2, u) + 2 * _gamma(3, u))
    nb = np.sqrt([5.0, 5.0, 10.0, 16.0, 17.0, 29.0])
    na = np.sqrt([5.0, 25.0, 61.0, 113.0, 100.0, 32.0])
    want_c = coef * np.outer([10.0, np.sqrt(244.0)], nb)
    want_r = coef * np.outer(na, [5.0, np.sqrt(29.0)])
    tc, tr = orc.tau_det(Af, Bf, 4, 4, 2, 2)
    assert np.allclose(tc, want_c, rtol=1e-13, atol=0)
    assert np.allclose(tr, want_r, rtol=1e-13, atol=0)


def test_stat_threshold_hand_value_b2(orc):
    """The b > 1 branch of the statistical threshold, by hand on the b = 2
    problem above.  v[r] sums the squares of the members of residue r,
    checksum row included: v[0] = rows 0, 2, 4 = [1+25+36, 4+36+64] = [62, 104],
    v[1] = rows 1, 3, 5 = [9+49+16, 16+64+16] = [74, 96]; likewise
    w[:, 0] = [1+9+16, 4+1+1] = [26, 6], w[:, 1] = [4+0+4, 1+16+25] = [8, 42].
    The Cauchy-Schwarz bound takes ||v_r||_2 and ||B_f[:, j]||_4^2 =
    sqrt(sum b^4): sqrt 17, sqrt 17, sqrt 82, 16, sqrt 257, sqrt 641; row
    factors ||A_f[i, :]||_4^2: sqrt 17, sqrt 337, sqrt 1921, sqrt 6497,
    sqrt 5392, sqrt 512."""
    u, T, s, lam = 2.0 ** -24, 8.0, 2.0, 10.0
    Af, Bf = orc.encode(_A4, _B4, 2, 2)
    coef = u * u / 3 * (T / 2 + s)
    nv = np.array([np.hypot(62.0, 104.0), np.hypot(74.0, 96.0)])
    nw = np.array([np.hypot(26.0, 6.0), np.hypot(8.0, 42.0)])
    b4 = np.sqrt([17.0, 17.0, 82.0, 256.0, 257.0, 641.0])
    a4 = np.sqrt([17.0, 337.0, 1921.0, 6497.0, 5392.0, 512.0])
    tc, tr = orc.tau_stat(Af, Bf, 4, 4, 2, 2, u_acc=u, T=T, s_store=s, lam=lam)
    assert np.allclose(tc, lam * np.sqrt(coef * np.outer(nv, b4)), rtol=1e-13, atol=0)
    assert np.allclose(tr, lam * np.sqrt(coef * np.outer(a4, nw)), rtol=1e-13, atol=0)
    # with C_f, each relation's stored total t adds its own binary32 rounding,
    # (u^2/3) t^2.  By hand: carried rows [6,8] and [-4,4] against the columns of
    # B_f, and the rows of A_f against the carried columns [4,1] and [-2,5].
    Cf = Af @ Bf
    t_c = np.array([[22.0, -4.0, 10.0, 32.0, 32.0, 28.0], [4.0, 12.0, -16.0, 16.0, -12.0, 28.0]])
    t_r = np.array([[6.0, 8.0], [8.0, -26.0], [26.0, 20.0], [-20.0, 54.0], [32.0, 28.0], [-12.0, 28.0]])
    assert np.array_equal(Cf[4:], t_c) and np.array_equal(Cf[:, 4:], t_r)
    tc, tr = orc.tau_stat(Af, Bf, 4, 4, 2, 2, u_acc=u, T=T, s_store=s, lam=lam, Cf=Cf)
    assert np.allclose(tc, lam * np.sqrt(coef * np.outer(nv, b4) + u * u / 3 * t_c ** 2), rtol=1e-13, atol=0)
    assert np.allclose(tr, lam * np.sqrt(coef * np.outer(a4, nw) + u * u / 3 * t_r ** 2), rtol=1e-13, atol=0)
    # stored totals that are themselves accumulated in T_c = 6 steps of the same
    # precision add (u^2/3)(T_c/3) t^2: a factor 1 + 2 = 3 on the stored-total term
    tc6, tr6 = orc.tau_stat(Af, Bf, 4, 4, 2, 2, u_acc=u, T=T, s_store=s, lam=lam, Cf=Cf, T_c=6.0)
    assert np.allclose(tc6, lam * np.sqrt(coef * np.outer(nv, b4) + 3 * u * u / 3 * t_c ** 2), rtol=1e-13, atol=0)
    assert np.allclose(tr6, lam * np.sqrt(coef * np.outer(a4, nw) + 3 * u * u / 3 * t_r ** 2), rtol=1e-13, atol=0)
    # a fault that makes a stored total infinite adds no rounding term: the
    # threshold stays that of the Q part alone, and the relation (residual -inf
    # for the column, +inf for the row through the same entry) fails
    Cx = Cf.copy()
    Cx[5, 2] = np.inf                     # column relation (1, 2); the same entry is in row 5's data
    tcx, trx = orc.tau_stat(Af, Bf, 4, 4, 2, 2, u_acc=u, T=T, s_store=s, lam=lam, Cf=Cx)
    assert np.isfinite(tcx).all() and np.isfinite(trx).all()
    assert tcx[1, 2] == pytest.approx(lam * np.sqrt(coef * nv[1] * b4[2]), rel=1e-13)
    assert np.array_equal(np.delete(tcx.ravel(), 1 * 6 + 2), np.delete(tc.ravel(), 1 * 6 + 2))
    assert np.array_equal(trx, tr)
    _, _, rep = orc.verify(Cx, 4, 4, 2, 2, tcx, trx)
    assert [(a, b) for a, b, _, _ in rep.flags_c()] == [(1, 2)]
    assert [(a, b) for a, b, _, _ in rep.flags_r()] == [(5, 0)]
    assert rep.n_nonfinite == 2


@pytest.mark.parametrize("br,bc", [(2, 3), (3, 2), (6, 1), (1, 3)])
def test_stat_bound_dominates_brute_force_q(orc, br, bc):
    """Brute force: Q of a relation is the sum over its members (checksum
    entry included) of the squares of the k products that form each member.
    The threshold is lambda sqrt(coef Q) exactly for b = 1 and, through
    Cauchy-Schwarz, never below it for b > 1."""
    m, n, k = 6, 6, 4
    u, T, s, lam = 2.0 ** -24, 2.0, 2.0, 10.0
    coef = u * u / 3 * (T / 2 + s)
    for seed in range(5):
        A, B = int_problem(m, n, k, seed=seed)
        Af, Bf = orc.encode(A, B, br, bc)
        tc, tr = orc.tau_stat(Af, Bf, m, n, br, bc, u_acc=u, T=T, s_store=s, lam=lam)
        for r in range(br):
            for j in range(n + bc):
                members = [g * br + r for g in range(m // br + 1)]
                q = sum((Af[i, l] * Bf[l, j]) ** 2 for i in members for l in range(k))
                want = lam * np.sqrt(coef * q)
                if br == 1:
                    assert tc[r, j] == pytest.approx(want, rel=1e-13)
                else:
                    assert tc[r, j] >= want * (1 - 1e-13), (seed, r, j)
        for i in range(m + br):
            for c in range(bc):
                members = [h * bc + c for h in range(n // bc + 1)]
                q = sum((Af[i, l] * Bf[l, jj]) ** 2 for jj in members for l in range(k))
                want = lam * np.sqrt(coef * q)
                if bc == 1:
                    assert tr[i, c] == pytest.approx(want, rel=1e-13)
                else:
                    assert tr[i, c] >= want * (1 - 1e-13), (seed, i, c)


@pytest.mark.parametrize("b,lo,hi", [(4, 0.45, 0.8), (32, 0.45, 0.8)])
def test_stat_model_block_checksums_simulated_fp32(orc, b, lo, hi):
    """The b > 1 statistical threshold against a simulated binary32
    accumulation (exact block of 4 products, one rounding per step, as in the
    b = 1 test): the Cauchy-Schwarz bound makes sigma somewhat larger than the
    exact-Q sigma, so rms(D/sigma) sits below the b = 1 value but well above
    what a sqrt(T/2) or norm-power slip would leave, and no |D| reaches
    lambda / 2 = 5 sigma."""
    m, n, k = 64, 64, 1024
    A = synth.uniform(21, 0, m, k, np.float32).astype(np.float64)
    B = synth.uniform(21, 1, k, n, np.float32).astype(np.float64)
    Af, Bf = orc.encode(A, B, b, b, store_f32=True)
    step = 4
    T = k / step
    prods = Af[:, None, :] * Bf.T[None, :, :]
    blocks = prods.reshape(m + b, n + b, k // step, step).sum(axis=3)
    acc = np.zeros((m + b, n + b), dtype=np.float32)
    for t in range(blocks.shape[2]):
        acc = (acc.astype(np.float64) + blocks[:, :, t]).astype(np.float32)
    Cf = acc.astype(np.float64)
    tc, tr = orc.tau_stat(Af, Bf, m, n, b, b, u_acc=orc.U32, T=T, s_store=1.0, lam=1.0)
    Dc, Dr, _ = orc.verify(Cf, m, n, b, b, tc, tr)
    z = np.concatenate([(Dc / tc).ravel(), (Dr / tr).ravel()])
    rms = np.sqrt(np.mean(z ** 2))
    assert lo < rms < hi, rms
    assert np.abs(z).max() < 5.0


# ---------------------------------------------------------------- locate / correct (brute force)
@pytest.mark.parametrize("m,n,k,br,bc", [(4, 4, 4, 1, 1), (4, 4, 6, 2, 2), (8, 8, 5, 4, 2), (3, 2, 4, 1, 1),
                                         (8, 4, 3, 2, 4)])
def test_every_element_every_bit_located_and_restored(orc, m, n, k, br, bc):
    """Brute force: integer inputs, exact mode (tau = 0).  Every element of C_f
    (data, carried checksums and corner) under every bit flip 40..62 is located
    at its exact (i, j) and rebuilt bit-exactly."""
    A, B = int_problem(m, n, k, seed=m * 100 + n)
    Af, Bf, Cf = orc.protected_product(A, B, br, bc)
    tc = np.zeros((br, n + bc))
    tr = np.zeros((m + br, bc))
    bits = Cf.view(np.uint64)
    for i in range(m + br):
        for j in range(n + bc):
            for beta in range(40, 63):
                Cx = Cf.copy()
                Cx.view(np.uint64)[i, j] = bits[i, j] ^ np.uint64(1 << beta)
                _, _, rep = orc.verify(Cx, m, n, br, bc, tc, tr)
                cls, li, lj, d = orc.classify(rep, m, n, br, bc)
                assert (li, lj) == (i, j), (i, j, beta, cls)
                assert cls == (orc.DATA if (i < m and j < n) else orc.CHECKSUM)
                v = orc.rebuild_value(Cx, m, n, br, bc, li, lj, d)
                assert v == Cf[i, j]


def test_flip_residual_equals_delta(orc):
    """The flagged residuals equal delta = value(flipped) - value with the
    sign rule (+ for a summand, - for a stored total)."""
    m, n, k, br, bc = 16, 12, 20, 4, 3
    A = synth.uniform(4, 0, m, k)
    B = synth.uniform(4, 1, k, n)
    Af, Bf, Cf = orc.protected_product(A, B, br, bc)
    tc, tr = orc.tau_det(Af, Bf, m, n, br, bc)
    for (i, j) in [(3, 5), (m + 1, 7), (9, n + 2), (m + 3, n + 1)]:
        Cx = Cf.copy()
        Cx.view(np.uint64)[i, j] ^= np.uint64(1 << 50)
        delta = Cx[i, j] - Cf[i, j]
        _, _, rep = orc.verify(Cx, m, n, br, bc, tc, tr)
        (r, jj, dc, tcq), = rep.flags_c()
        (ii, c, dr, trq), = rep.flags_r()
        assert (r, jj, ii, c) == (i % br, j, i, j % bc)
        sc = 1 if i < m else -1
        sr = 1 if j < n else -1
        assert abs(dc - sc * delta) <= tcq and abs(dr - sr * delta) <= trq


def test_nonfinite_value_fails_both_relations(orc):
    """A relation fails when !(|D| <= tau): a NaN or infinite element makes
    both of its residuals non-finite, and both relations are flagged and
    counted as non-finite, even with an infinite threshold budget elsewhere."""
    m, n, k, br, bc = 8, 6, 5, 2, 3
    A, B = int_problem(m, n, k, seed=41)
    Af, Bf, Cf = orc.protected_product(A, B, br, bc)
    tc = np.full((br, n + bc), 1e300)
    tr = np.full((m + br, bc), 1e300)
    for bad in (np.nan, np.inf, -np.inf):
        for (i, j) in [(3, 4), (m + 1, 2), (5, n + 1)]:
            Cx = Cf.copy()
            Cx[i, j] = bad
            _, _, rep = orc.verify(Cx, m, n, br, bc, tc, tr)
            assert (rep.n_flag_c, rep.n_flag_r, rep.n_nonfinite) == (1, 1, 2), (bad, i, j)
            assert rep.flags_c()[0][:2] == (i % br, j) and rep.flags_r()[0][:2] == (i, j % bc)


def _hand_report(orc, flags_c, flags_r):
    rep = orc.Report()
    rep.n_flag_c, rep.n_flag_r = len(flags_c), len(flags_r)
    for q, (a, b, d, t) in enumerate(flags_c):
        rep.fc_r[q], rep.fc_j[q], rep.fc_d[q], rep.fc_t[q] = a, b, d, t
    for q, (a, b, d, t) in enumerate(flags_r):
        rep.fr_i[q], rep.fr_c[q], rep.fr_d[q], rep.fr_t[q] = a, b, d, t
    return rep


def test_classify_rules_on_hand_made_reports(orc):
    """The single-error model on reports written by hand (m = n = 8,
    br = 2, bc = 4): one error at (i, j) fails column relation (i mod br, j)
    and row relation (i, j mod bc) with residuals +delta for a summand and
    -delta for a stored total.  Flags that do not meet in one element, or
    whose residuals disagree, are MULTI; a checksum entry is CHECKSUM."""
    m = n = 8
    br, bc = 2, 4
    cls = lambda fc, fr: orc.classify(_hand_report(orc, fc, fr), m, n, br, bc)
    assert cls([(1, 5, 3.0, 1e-3)], [(3, 1, 3.0, 1e-3)])[:3] == (orc.DATA, 3, 5)
    # row 2 is residue 0, not 1: the two relations share no element
    assert cls([(1, 5, 3.0, 1e-3)], [(2, 1, 3.0, 1e-3)])[0] == orc.MULTI
    # column 6 is residue 2 of bc = 4, not 1
    assert cls([(1, 6, 3.0, 1e-3)], [(3, 1, 3.0, 1e-3)])[0] == orc.MULTI
    # congruent but inconsistent residuals: two errors, not one
    assert cls([(1, 5, 3.0, 1e-3)], [(3, 1, 5.0, 1e-3)])[0] == orc.MULTI
    # a carried row entry (i = m + 1) is the stored total of its column
    # relation (-delta) and a summand of its row relation (+delta)
    assert cls([(1, 5, -3.0, 1e-3)], [(m + 1, 1, 3.0, 1e-3)])[:3] == (orc.CHECKSUM, m + 1, 5)
    assert cls([(1, 5, 3.0, 1e-3)], [(m + 1, 1, 3.0, 1e-3)])[0] == orc.MULTI
    assert cls([], [])[0] == orc.CLEAN
    assert cls([(1, 5, 3.0, 1e-3)], [])[0] == orc.MULTI


def test_two_errors_are_not_miscorrected(orc):
    m, n, k = 8, 8, 6
    A, B = int_problem(m, n, k)
    Af, Bf, Cf = orc.protected_product(A, B, 1, 1)
    Cx = Cf.copy()
    Cx[1, 2] += 3
    Cx[5, 6] -= 2
    _, _, rep = orc.verify(Cx, m, n, 1, 1, np.zeros((1, n + 1)), np.zeros((m + 1, 1)))
    assert orc.classify(rep, m, n, 1, 1)[0] == orc.MULTI


# ---------------------------------------------------------------- erasure recovery (Sec. 2.1)
@pytest.mark.parametrize("br,bc,bh,bw", [(4, 4, 4, 4), (2, 4, 2, 4), (4, 2, 4, 2), (8, 8, 8, 8)])
def test_every_block_position_rebuilt_exactly(orc, br, bc, bh, bw):
    m, n, k = 16, 16, 7
    A, B = int_problem(m, n, k, seed=br * 10 + bc)
    Af, Bf, Cf = orc.protected_product(A, B, br, bc)
    for use_rows in (False, True):
        if (not use_rows and bh > br) or (use_rows and bw > bc):
            continue
        for i0 in range(0, m + br - bh + 1, bh):
            for j0 in range(0, n + bc - bw + 1, bw):
                Cx = Cf.copy()
                Cx[i0:i0 + bh, j0:j0 + bw] = np.nan
                assert orc.recover(Cx, m, n, br, bc, (i0, j0, bh, bw), use_rows=use_rows) == 0
                assert np.array_equal(Cx, Cf), (i0, j0, use_rows)


@pytest.mark.parametrize("br,bc", [(1, 1), (3, 2)])
def test_outer_product_intermediates_consistent_exact(orc, br, bc):
    """Sec. 2.2 outer-product loop: every intermediate C_k is the integer
    partial product A[:, :k] B[:k, :] with its checksums, so every relation
    holds exactly after every rank-1 update; the loop ends on the product."""
    m, n, k = 12, 10, 9
    A, B = int_problem(m, n, k, seed=br + 5 * bc)
    Af, Bf = orc.encode(A, B, br, bc)
    Ai, Bi = A.astype(np.int64), B.astype(np.int64)
    Cf = np.zeros((m + br, n + bc))
    tc, tr = np.zeros((br, n + bc)), np.zeros((m + br, bc))
    for k1 in range(1, k + 1):
        orc.outer_update(Cf, Af, Bf, k1 - 1, k1)
        assert np.array_equal(Cf[:m, :n], (Ai[:, :k1] @ Bi[:k1]).astype(np.float64)), k1
        rep = orc.verify(Cf, m, n, br, bc, tc, tr)[2]
        assert rep.n_flag_c == 0 and rep.n_flag_r == 0, k1
    assert np.array_equal(Cf, orc.gemm(Af, Bf))


def test_outer_product_does_not_transpose_or_skip(orc):
    """A rank-1 update on hand-sized operands, checked entry by entry."""
    Af = np.array([[1.0, 2.0], [3.0, 4.0], [5.0, 6.0]])
    Bf = np.array([[1.0, -1.0], [10.0, 20.0]])
    Cf = np.zeros((3, 2))
    orc.outer_update(Cf, Af, Bf, 1, 2)          # only l = 1
    assert np.array_equal(Cf, [[20.0, 40.0], [40.0, 80.0], [60.0, 120.0]])
    orc.outer_update(Cf, Af, Bf, 0, 1)
    assert np.array_equal(Cf, Af @ Bf)


@pytest.mark.parametrize("br,bc,rect,use_rows", [(4, 4, (4, 8, 4, 4), False), (2, 4, (6, 16, 2, 4), False),
                                                 (4, 2, (0, 2, 4, 2), True)])
def test_mid_loop_erasure_rebuilt_then_loop_goes_on(orc, br, bc, rect, use_rows):
    """Sec. 2.2: a block lost between two updates of the outer-product loop
    is rebuilt from the consistent intermediate (exactly, on integers), and
    finishing the loop gives the product an uninterrupted loop gives."""
    m, n, k = 16, 16, 11
    A, B = int_problem(m, n, k, seed=31)
    Af, Bf = orc.encode(A, B, br, bc)
    Cf = np.zeros((m + br, n + bc))
    orc.outer_update(Cf, Af, Bf, 0, 5)
    want = Cf.copy()
    i0, j0, h, w = rect
    Cf[i0:i0 + h, j0:j0 + w] = np.nan
    assert orc.recover(Cf, m, n, br, bc, rect, use_rows=use_rows) == 0
    assert np.array_equal(Cf, want)
    orc.outer_update(Cf, Af, Bf, 5, k)
    assert np.array_equal(Cf, orc.gemm(Af, Bf))


@pytest.mark.parametrize("br,bc", [(1, 1), (4, 2)])
def test_chained_product_relations_exact_on_integers(orc, br, bc):
    """Sec. 3.2 chained calls: the carried rows of C_f are the checksum rows of
    C, so C_f[:, :n] can enter the next product as A_f without recomputing
    them; every relation of the chained product holds exactly on integers."""
    m, k1, n1, n2 = 12, 7, 10, 8
    A1, B1 = int_problem(m, n1, k1, seed=41)
    B2 = synth.uniform_ints(42, synth.STREAM_B, n1, n2, -8, 8)
    _, _, C1f = orc.protected_product(A1, B1, br, bc)
    _, B2f = orc.encode(np.zeros((m, n1)), B2, br, bc)
    Df = orc.gemm(C1f[:, :n1], B2f)
    Di = (A1.astype(np.int64) @ B1.astype(np.int64)) @ B2.astype(np.int64)
    assert np.array_equal(Df[:m, :n2], Di.astype(np.float64))
    tc, tr = np.zeros((br, n2 + bc)), np.zeros((m + br, bc))
    rep = orc.verify(Df, m, n2, br, bc, tc, tr)[2]
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0


def test_chained_threshold_binary32_bounds_single_precision_products(orc):
    """Binary32 chain: checksum rows rounded to binary32, both products
    accumulated in binary32 by an independent routine (numpy's single-precision
    matrix product); the first product verifies clean under the binary32 det
    thresholds, the chained one (the first C_f as its A_f, carried rows as they
    are) under the binary32 chained thresholds."""
    m, k1, n1, n2, b = 64, 96, 80, 48, 8
    worst = 0.0
    for seed in range(3):
        A1 = synth.uniform(seed, synth.STREAM_A, m, k1, np.float32).astype(np.float64)
        B1 = synth.uniform(seed, synth.STREAM_B, k1, n1, np.float32).astype(np.float64)
        B2 = synth.uniform(seed + 7, synth.STREAM_B, n1, n2, np.float32).astype(np.float64)
        Af1, Bf1 = orc.encode(A1, B1, b, b, store_f32=True)
        C1f = (Af1.astype(np.float32) @ Bf1.astype(np.float32)).astype(np.float64)
        tc1, tr1 = orc.tau_det(Af1, Bf1, m, n1, b, b, u_acc=orc.U32, u_st=orc.U32)
        assert orc.verify(C1f, m, n1, b, b, tc1, tr1)[2].n_flag_c == 0
        _, B2f = orc.encode(np.zeros((m, n1)), B2, b, b, store_f32=True)
        Af2 = np.ascontiguousarray(C1f[:, :n1])
        D = (Af2.astype(np.float32) @ B2f.astype(np.float32)).astype(np.float64)
        tcc, trc = orc.tau_det_chained(Af2, B2f, m, n2, b, b, tc1, u_acc=orc.U32, u_st=orc.U32)
        Dc, Dr, rep = orc.verify(D, m, n2, b, b, tcc, trc)
        assert rep.n_flag_c == 0 and rep.n_flag_r == 0
        worst = max(worst, (np.abs(Dc) / tcc).max(), (np.abs(Dr) / trc).max())
    assert worst > 1e-4, worst


def test_chained_threshold_bounds_and_needs_the_inherited_term(orc):
    """The chained det threshold bounds the residuals of D_f on random binary64
    data; and when the previous C_f's carried row is off by as much as its own
    threshold allows (a legal, verified C_f), the plain threshold of the chained
    product is exceeded while the chained one still holds."""
    m, k1, n1, n2, b = 64, 96, 80, 48, 8
    worst = 0.0
    for seed in range(3):
        A1 = synth.uniform(seed, synth.STREAM_A, m, k1)
        B1 = synth.uniform(seed, synth.STREAM_B, k1, n1)
        B2 = synth.uniform(seed + 7, synth.STREAM_B, n1, n2)
        Af1, Bf1, C1f = orc.protected_product(A1, B1, b, b)
        tc1, _ = orc.tau_det(Af1, Bf1, m, n1, b, b)
        _, B2f = orc.encode(np.zeros((m, n1)), B2, b, b)
        Af2 = np.ascontiguousarray(C1f[:, :n1])
        tcc, trc = orc.tau_det_chained(Af2, B2f, m, n2, b, b, tc1)
        Dc, Dr, rep = orc.verify(orc.gemm(Af2, B2f), m, n2, b, b, tcc, trc)
        assert rep.n_flag_c == 0 and rep.n_flag_r == 0
        worst = max(worst, (np.abs(Dc) / tcc).max())
        # the carried row shifted by 0.9 of the previous threshold (sign of B2's column sums: worst case)
        C1x = C1f.copy()
        C1x[m:m + b, :n1] += 0.9 * tc1[:, :n1] * np.sign(B2f.sum(axis=1))[None, :]
        assert orc.verify(C1x, m, n1, b, b, tc1, orc.tau_det(Af1, Bf1, m, n1, b, b)[1])[2].n_flag_c == 0
        Ax = np.ascontiguousarray(C1x[:, :n1])
        Dx = orc.gemm(Ax, B2f)
        tcp, trp = orc.tau_det(Ax, B2f, m, n2, b, b)
        assert orc.verify(Dx, m, n2, b, b, tcp, trp)[2].n_flag_c > 0          # the plain threshold is exceeded
        tcx, trx = orc.tau_det_chained(Ax, B2f, m, n2, b, b, tc1)
        assert orc.verify(Dx, m, n2, b, b, tcx, trx)[2].n_flag_c == 0        # the chained one holds
    assert worst > 1e-6


def test_recovery_formula_single_checksum(orc):
    """Sec. 2.1 with unit weights: x_i = y - sum_{k != i} x_k, on a 1-row C."""
    m, n, k = 1, 5, 1
    A = np.array([[2.0]])
    B = np.array([[1.0, -3.0, 4.0, 0.5, 7.0]])
    Af, Bf, Cf = orc.protected_product(A, B, 1, 1)
    y = Cf[0, n]
    assert y == 2 * (1 - 3 + 4 + 0.5 + 7)
    assert orc.rebuild_value(Cf, m, n, 1, 1, 0, 2, orc.DIR_ROW) == y - (2 - 6 + 1 + 14)


def test_taller_than_checksum_block_is_unrecoverable(orc):
    """A b x b hole with b > br has more unknowns than column relations
    (C1's 64x64 erasure under the (n+1) encoding)."""
    m = n = 16
    A, B = int_problem(m, n, 5)
    Af, Bf, Cf = orc.protected_product(A, B, 1, 1)
    Cx = Cf.copy()
    Cx[0:4, 0:4] = 0
    assert orc.recover(Cx, m, n, 1, 1, (0, 0, 4, 4)) == -4
    assert orc.recover(Cx, m, n, 1, 1, (0, 0, 4, 4), use_rows=True) == -4
    assert np.array_equal(Cx[0:4, 0:4], np.zeros((4, 4)))   # untouched
    _, _, rep = orc.verify(Cx, m, n, 1, 1, np.zeros((1, n + 1)), np.zeros((m + 1, 1)))
    assert rep.n_flag_c == 4 and rep.n_flag_r == 4
    assert orc.classify(rep, m, n, 1, 1)[0] == orc.MULTI


@pytest.mark.parametrize("share", ["col_band", "row_band", "neither"])
def test_flip_with_known_erasure(orc, share):
    """A flip and an erased block in one run: the erasure is passed as known,
    the flip is located and corrected first, then the block is rebuilt."""
    m = n = 32
    b = 8
    A, B = int_problem(m, n, 9, seed=21)
    Af, Bf, Cf = orc.protected_product(A, B, b, b)
    rect = (8, 16, 8, 8)
    fi, fj = {"col_band": (27, 19), "row_band": (10, 3), "neither": (30, 2)}[share]
    Cx = Cf.copy()
    Cx[fi, fj] += 5
    Cx[8:16, 16:24] = 0
    tc = np.zeros((b, n + b))
    tr = np.zeros((m + b, b))
    _, _, rep = orc.verify(Cx, m, n, b, b, tc, tr, erasures=[rect])
    cls, i, j, d = orc.classify(rep, m, n, b, b, erasures=[rect])
    assert (cls, i, j) == (orc.DATA, fi, fj)
    if share == "col_band":
        assert d == orc.DIR_ROW
    Cx[i, j] = orc.rebuild_value(Cx, m, n, b, b, i, j, d)
    assert orc.recover(Cx, m, n, b, b, rect) == 0
    assert np.array_equal(Cx, Cf)


def test_known_erasure_skips_exactly_its_relations(orc):
    """m = n = 8, br = bc = 4, erased rectangle rows 1..2, columns 2..4.  By
    hand: the column relations that hold an erased element are residues
    {1, 2} x columns {2, 3, 4} (6 relations), the row relations rows {1, 2} x
    residues {2, 3, 0} (6 relations); nothing else is skipped, and a flip
    outside them is still seen."""
    m = n = 8
    br = bc = 4
    A, B = int_problem(m, n, 5, seed=8)
    Af, Bf, Cf = orc.protected_product(A, B, br, bc)
    Cx = Cf.copy()
    Cx[1:3, 2:5] = 0.0
    tc, tr = np.zeros((br, n + bc)), np.zeros((m + br, bc))
    _, _, rep = orc.verify(Cx, m, n, br, bc, tc, tr, erasures=[(1, 2, 2, 3)])
    assert (rep.n_excl_c, rep.n_excl_r) == (6, 6)
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0
    Cx[3, 6] += 1.0                     # residue 3, column 6: neither relation holds an erased element
    _, _, rep = orc.verify(Cx, m, n, br, bc, tc, tr, erasures=[(1, 2, 2, 3)])
    assert [f[:2] for f in rep.flags_c()] == [(3, 6)] and [f[:2] for f in rep.flags_r()] == [(3, 2)]


# ---------------------------------------------------------------- residual check (Sec. 4.3)
def test_residual_check(orc):
    m, n, k = 64, 48, 80
    A = synth.uniform(6, 0, m, k)
    B = synth.uniform(6, 1, k, n)
    x = synth.uniform(6, synth.STREAM_X, 1, n)[0]
    Cm = orc.gemm(A, B)
    rho = orc.residual(A, B, Cm, x)
    assert rho < 10.0
    Cm[3, 7] += 1e-6
    assert orc.residual(A, B, Cm, x) > 1e3


# ---------------------------------------------------------------- quantizers
def _bit_patterns(count, seed=17):
    raw = synth.raw_u64(seed, 0, np.arange(count, dtype=np.uint64)).astype(np.uint64)
    u32 = (raw >> np.uint64(32)).astype(np.uint32)
    edge = np.array([0, 0x80000000, 0x3F800000, 0x3F808000, 0x3F818000, 0x3F80FFFF, 0x7F7FFFFF, 0x00000001,
                     0x007FFFFF, 0x00800000, 0x7F800000, 0xFF800000, 0x477FE000, 0x477FF000], dtype=np.uint32)
    return np.concatenate([u32, edge])


def test_bf16_rne_matches_torch(orc):
    import torch
    pats = _bit_patterns(1 << 20)
    x = pats.view(np.float32)
    x = x[~np.isnan(x)]
    ours = orc.to_bf16_bits(x)
    ref = torch.from_numpy(x.copy()).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)


def test_e4m3_decode_table_matches_torch(orc):
    import torch
    codes = np.arange(256, dtype=np.uint8)
    ref = torch.from_numpy(codes.copy()).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    ours = orc.e4m3_values(codes)
    finite = ~np.isnan(ref)
    assert np.array_equal(np.isnan(ours), ~finite)
    assert np.array_equal(ours[finite], ref[finite])
    assert ours[finite].max() == 448.0


def test_e4m3_rne_matches_torch_in_range(orc):
    import torch
    pats = _bit_patterns(1 << 20, seed=23)
    x = pats.view(np.float32)
    x = x[np.isfinite(x) & (np.abs(x) <= 464.0)]
    # add exact ties of the e4m3 grid
    grid = orc.e4m3_values(np.arange(0, 126, dtype=np.uint8))
    ties = ((grid[1:] + grid[:-1]) / 2).astype(np.float32)
    x = np.concatenate([x, ties, -ties])
    ours = orc.e4m3_values(orc.to_e4m3_codes(x))
    ref = torch.from_numpy(x.copy()).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(ours, ref)


def test_e4m3_scale_is_largest_power_of_two(orc):
    for amax in [1.0, 0.999, 3.5, 448.0, 449.0, 1e-3, 7e5]:
        x = np.array([0.25, -amax, 0.0], dtype=np.float32)
        e = orc.e4m3_scale_exp(x)
        a = max(0.25, float(np.float32(amax)))
        assert a * 2.0 ** e <= 448.0 < a * 2.0 ** (e + 1)
    assert orc.e4m3_scale_exp(np.zeros(4, dtype=np.float32)) == 0
    # the scale comes from the finite entries alone; and it reaches beyond
    # binary32's own exponent range (amax 2^-140, subnormal: e = 148)
    x = np.array([3.0, np.inf, -np.inf, np.nan, -5.0], dtype=np.float32)
    assert orc.e4m3_scale_exp(x) == 6                       # 5 * 2^6 = 320 <= 448 < 640
    assert orc.e4m3_scale_exp(np.array([np.inf, np.nan], dtype=np.float32)) == 0
    assert orc.e4m3_scale_exp(np.array([2.0 ** -140, -2.0 ** -141], dtype=np.float32)) == 148


def test_e4m3_saturation_and_nonfinite(orc):
    """The format has no infinities: magnitudes from the midpoint above 448
    (464) upward, infinities included, give +-448 (codes 0x7E / 0xFE); below
    464 they round to 448 by the ordinary rule; NaN gives 0x7F."""
    x = np.array([448.0, 463.99, 464.0, 470.0, 1e30, np.inf], dtype=np.float32)
    assert list(orc.to_e4m3_codes(x)) == [0x7E] * 6
    assert list(orc.to_e4m3_codes(-x)) == [0xFE] * 6
    assert list(orc.to_e4m3_codes(np.array([np.nan, -np.nan], dtype=np.float32))) == [0x7F, 0x7F]
    # 432 is the midpoint of 416 and 448: ties to the even fraction (448 = 1.110b 2^8)
    assert list(orc.to_e4m3_codes(np.array([432.0, 431.9], dtype=np.float32))) == [0x7E, 0x7D]


def test_exponent_bit_flip_located_on_real_data(orc):
    """An exponent-bit flip makes |delta| huge, so both residuals also carry
    the rounding of a sum that holds the bad value; the single error must
    still be located (and the element rebuilt within tau)."""
    m, n, k, br, bc = 64, 48, 96, 8, 4
    A = synth.uniform(31, 0, m, k)
    B = synth.uniform(31, 1, k, n)
    Af, Bf, Cf = orc.protected_product(A, B, br, bc)
    tc, tr = orc.tau_det(Af, Bf, m, n, br, bc)
    found = 0
    for t, (i, j) in enumerate([(5, 7), (63, 0), (m + 2, 9), (17, n + 3), (m + 7, n + 1), (30, 30)]):
        for beta in range(52, 62):
            Cx = Cf.copy()
            Cx.view(np.uint64)[i, j] ^= np.uint64(1 << beta)
            if abs(Cx[i, j] - Cf[i, j]) <= 2 * max(tc[i % br, j], tr[i, j % bc]):
                continue
            _, _, rep = orc.verify(Cx, m, n, br, bc, tc, tr)
            cls, li, lj, d = orc.classify(rep, m, n, br, bc)
            assert (li, lj) == (i, j), (i, j, beta, cls)
            if np.isfinite(Cx[i, j]):
                v = orc.rebuild_value(Cx, m, n, br, bc, i, j, d)
                assert abs(v - Cf[i, j]) <= tc[i % br, j]
            found += 1
    assert found >= 50


# ---------------------------------------------------------------- 2-D block-cyclic distribution (Sec. 4.1)
def test_block_cyclic_owner_by_hand(orc):
    """nb = 2 over P = 3: global blocks 0..5 go to processes 0,1,2,0,1,2; local
    blocks 0,0,0,1,1,1."""
    got = [orc.block_cyclic_owner(i, 2, 3) for i in range(12)]
    assert got == [(0, 0), (0, 1), (1, 0), (1, 1), (2, 0), (2, 1),
                   (0, 2), (0, 3), (1, 2), (1, 3), (2, 2), (2, 3)]


def test_block_cyclic_stack_roundtrip_and_checksum_process(orc):
    """The stacked local arrays are a permutation of the matrix; the block
    checksum of the stacked layout with br = m/P, bc = n/Q is the checksum
    process row / column of the grid: the sum over the process rows (columns)
    of the local arrays, computed here from the owner map alone."""
    nb, P, Q = 2, 3, 2
    m, n, k = nb * P * 2, nb * Q * 3, 5
    A, B = int_problem(m, n, k, seed=77)
    G = A @ B
    S = orc.block_cyclic_stack(G, nb, P, Q)
    assert np.array_equal(orc.block_cyclic_unstack(S, nb, P, Q), G)
    assert sorted(S.ravel().tolist()) == sorted(G.ravel().tolist())
    lm, ln = m // P, n // Q
    # checksum process row: for each (local row, column) the sum over p of the owners' entries
    want_row = np.zeros((lm, n))
    for i in range(m):
        p, li = orc.block_cyclic_owner(i, nb, P)
        for j in range(n):
            q, lj = orc.block_cyclic_owner(j, nb, Q)
            want_row[li, q * ln + lj] += G[i, j]
    # the product in the stacked layout: rows of A and columns of B permuted as C's
    Ar = np.empty_like(A)
    for i in range(m):
        p, li = orc.block_cyclic_owner(i, nb, P)
        Ar[p * lm + li] = A[i]
    Bc = np.empty_like(B)
    for j in range(n):
        q, lj = orc.block_cyclic_owner(j, nb, Q)
        Bc[:, q * ln + lj] = B[:, j]
    Af, Bf, Cf = orc.protected_product(Ar, Bc, lm, ln)
    assert np.array_equal(Cf[:m, :n], S)
    assert np.array_equal(Cf[m:, :n], want_row)
    want_col = np.zeros((m, ln))
    for i in range(m):
        for j in range(n):
            q, lj = orc.block_cyclic_owner(j, nb, Q)
            p, li = orc.block_cyclic_owner(i, nb, P)
            want_col[p * lm + li, lj] += G[i, j]
    assert np.array_equal(Cf[:m, n:], want_col)
