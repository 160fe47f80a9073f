"""GPU parity of the bfloat16 and FP8-E4M3 paths (binary32 inputs quantized on
the GPU, low-precision matrix cores with binary32 accumulation, binary32
checksum rows in the workspace, statistical thresholds) against the CPU oracle.

The oracle quantizes the same binary32 inputs with its own round-to-nearest-
even (FP8: after its own per-tensor power-of-two scale 2^e, the largest with
amax * 2^e <= 448), works on the quantized values exactly in binary64 (FP8 in
the scaled domain, the product scaled back by 2^-(eA+eB)), rounds its checksum
rows once to binary32 and its product to binary32.
 - quantized operands: bit-exact;
 - values: per element |C_gpu - C_oracle| <= (k u32 + w)(|A_q||B_q|)_ij + u32 |C_ij|:
   the binary32 accumulation bound (the products themselves are exact), plus for
   FP8 w = 2^-10, the matrix core's product-sum window (each group of products is
   summed to 2^-11 of its largest term, measured on gfx950); w = 0 for bfloat16;
 - decisions and indices: bit-exact outside the gray zone tau/2 < |delta| < 2 tau.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_0806_3121_amd import abft, synth  # noqa: E402

pytestmark = pytest.mark.gpu

SEED = synth.BASE_SEED + 16
LAMBDA = 10.0
U32 = 2.0 ** -24


def note(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abft.lib()
    return torch.device("cuda:0")


DTYPES = {"bf16": abft.ABFT_BF16, "fp8": abft.ABFT_FP8_E4M3}


def oracle_quantize(orc, dt, X32):
    """-> (stored codes, values in the compute domain, scale exponent)."""
    if dt == "bf16":
        q = orc.to_bf16_bits(X32)
        return q, orc.bf16_bits_to_f64(q), 0
    e = orc.e4m3_scale_exp(X32)
    q = orc.to_e4m3_codes(np.ldexp(X32.astype(np.float64), e).astype(np.float32))   # x 2^e, exact
    return q, orc.e4m3_values(q), e


def stored_codes(t, dt):
    return t.cpu().view(torch.int16).numpy().view(np.uint16) if dt == "bf16" else t.cpu().numpy()


def make(dev, orc, m, n, k, br, bc, dt="bf16"):
    A32 = synth.uniform(SEED, synth.STREAM_A, m, k, np.float32)
    B32 = synth.uniform(SEED, synth.STREAM_B, k, n, np.float32)
    P = abft.Protected(DTYPES[dt], m, n, k, br, bc, device=dev, tau_mode=abft.ABFT_TAU_STAT, lam=LAMBDA)
    abft.quantize(P.p, 0, torch.from_numpy(A32).to(dev), P.A, P.ws)
    abft.quantize(P.p, 1, torch.from_numpy(np.ascontiguousarray(B32.T)).to(dev), P.Bt, P.ws)
    torch.cuda.synchronize()
    Aq, A, eA = oracle_quantize(orc, dt, A32)
    Bq, B, eB = oracle_quantize(orc, dt, B32)
    assert np.array_equal(stored_codes(P.A, dt), Aq)
    assert np.array_equal(stored_codes(P.Bt, dt), np.ascontiguousarray(Bq.T))
    Af, Bf = orc.encode(A, B, br, bc, store_f32=True)
    sc = 2.0 ** -(eA + eB)
    C_scaled = orc.gemm(Af, Bf)
    C64 = C_scaled * sc
    # the library's statistical model: T = k/4 accumulation steps; s = 2, plus the
    # FP8 product-sum window (per-product error 2^-15, i.e. + (2^-15 / 2^-24)^2); the stored totals
    s_store = 2.0 + (2.0 ** 18 if dt == "fp8" else 0.0)
    tc, tr = orc.tau_stat(Af, Bf, m, n, br, bc, u_acc=U32, T=k / 4.0, s_store=s_store, lam=LAMBDA, Cf=C_scaled)
    P.retau = lambda Cx: tuple(t * sc for t in orc.tau_stat(Af, Bf, m, n, br, bc, u_acc=U32, T=k / 4.0,
                                                             s_store=s_store, lam=LAMBDA,
                                                             Cf=np.asarray(Cx, dtype=np.float64) / sc))
    return P, A * 2.0 ** -eA, B * 2.0 ** -eB, Af * 2.0 ** -eA, Bf * 2.0 ** -eB, C64.astype(np.float32), tc * sc, tr * sc


SHAPES = [
    (256, 256, 256, 1, 1),
    (512, 384, 1024, 1, 1),
    (200, 136, 80, 8, 4),
    (512, 512, 512, 32, 32),
    (1024, 1024, 4096, 1, 1),
    (300, 260, 528, 3, 5),
    (4096, 4096, 256, 1, 1),      # large enough for the direct-to-LDS kernel
    (4200, 4100, 384, 8, 4),      # same kernel, ragged tile edges
    (4096, 4352, 128, 1, 1),      # one FP8 slab (two bfloat16 slabs): the loop's tail alone
    (4300, 4100, 640, 1, 1),      # five FP8 slabs, ragged edges
]


@pytest.mark.parametrize("dt", ["bf16", "fp8"])
@pytest.mark.parametrize("m,n,k,br,bc", SHAPES)
def test_lowp_product_and_clean_verify(dev, orc, m, n, k, br, bc, dt):
    note(f"{dt} m={m} n={n} k={k} br={br} bc={bc}")
    P, A, B, Af, Bf, C32, tc, tr = make(dev, orc, m, n, k, br, bc, dt)
    P.encode()
    P.gemm()
    torch.cuda.synchronize()
    Cg = P.C.cpu().numpy().astype(np.float64)
    w = 2.0 ** -10 if dt == "fp8" else 0.0
    bound = (k * U32 + w) * (np.abs(Af) @ np.abs(Bf)) + U32 * np.abs(C32)
    assert np.all(np.abs(Cg - C32) <= bound * 1.01 + 1e-30)
    rep = P.verify()
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0, (rep.max_ratio_c, rep.max_ratio_r)
    note(f"  max |D|/tau {max(rep.max_ratio_c, rep.max_ratio_r):.4f}; "
         f"max rel err {np.abs(Cg - C32).max() / np.abs(C32).max():.2e}")
    # plain product = data part, bit for bit (same kernel, same k order)
    Cp = torch.zeros(m, n, dtype=torch.float32, device=dev)
    p2 = abft.problem(DTYPES[dt], m, n, k, br, bc, ldc=n, tau_mode=abft.ABFT_TAU_STAT)
    abft.gemm(p2, P.A, P.Bt, Cp, P.ws, flags=abft.ABFT_PLAIN)
    torch.cuda.synchronize()
    assert torch.equal(Cp, P.C[:m, :n])


@pytest.mark.parametrize("dt", ["bf16", "fp8"])
@pytest.mark.parametrize("m,n,k,br,bc,runs", [(256, 256, 256, 1, 1, 60), (512, 512, 512, 32, 32, 40)])
def test_lowp_flip_decisions_match_oracle(dev, orc, m, n, k, br, bc, runs, dt):
    P, A, B, Af, Bf, C32, tc, tr = make(dev, orc, m, n, k, br, bc, dt)
    P.encode()
    P.gemm()
    clean = P.C.clone()
    M, N = m + br, n + bc
    located = compared = 0
    for run in range(runs):
        i, j, bit = synth.flip_site(SEED + 9, run, M, N, 11, 30)
        note(f"{dt} flip run={run} ({i},{j}) bit {bit}")
        P.C.copy_(clean)
        abft.inject_flip(P.p, P.C, i, j, bit)
        rep = P.verify()
        loc = abft.classify(P.p, rep)
        Cx = C32.copy()
        Cx.view(np.uint32)[i, j] ^= np.uint32(1 << bit)
        delta = float(Cx[i, j]) - float(C32[i, j])
        t1, t2 = tc[i % br, j], tr[i, j % bc]
        if np.isfinite(delta) and (t1 / 2 < abs(delta) < 2 * t1 or t2 / 2 < abs(delta) < 2 * t2):
            continue
        compared += 1
        # a flip on a stored total also moves that relation's rounding term
        tcx, trx = P.retau(Cx) if (i >= m or j >= n) else (tc, tr)
        _, _, orep = orc.verify(Cx.astype(np.float64), m, n, br, bc, tcx, trx)
        ocls, oi, oj, od = orc.classify(orep, m, n, br, bc)
        assert (rep.n_flag_c, rep.n_flag_r) == (orep.n_flag_c, orep.n_flag_r), (i, j, bit, delta)
        # the GPU's statistical thresholds are the oracle's (binary32 weights in A's weighted row sums)
        for r, jj, _, tau in rep.flags_c():
            assert abs(tau - tcx[r, jj]) <= 1e-6 * tcx[r, jj]
        for ii, c, _, tau in rep.flags_r():
            assert abs(tau - trx[ii, c]) <= 1e-6 * trx[ii, c]
        assert (loc.cls, loc.i, loc.j) == (ocls, oi, oj)
        if loc.cls in (abft.ABFT_CLS_DATA, abft.ABFT_CLS_CHECKSUM):
            located += 1
            abft.correct(P.p, P.C, loc)
            rep2 = P.verify()
            assert rep2.n_flag_c == 0 and rep2.n_flag_r == 0
            assert abs(P.C[i, j].item() - clean[i, j].item()) <= min(t1, t2)
    note(f"  compared {compared}, located {located}")
    assert compared >= runs * 0.8 and located >= compared * 0.4


@pytest.mark.parametrize("dt", ["bf16", "fp8"])
def test_lowp_erasure_rebuild(dev, orc, dt):
    m = n = 512
    k, b = 256, 32
    P, A, B, Af, Bf, C32, tc, tr = make(dev, orc, m, n, k, b, b, dt)
    P.encode()
    P.gemm()
    clean = P.C.clone()
    for rect in [(64, 128, 32, 32), (512, 0, 32, 32), (5, 3, 20, 30), (64, 512, 32, 32)]:
        for use_rows in (False, True):
            note(f"{dt} erase {rect} rows={use_rows}")
            P.C.copy_(clean)
            abft.inject_erase(P.p, P.C, rect, nan_fill=True)
            rep = P.verify(known=[rect])
            assert rep.n_flag_c == 0 and rep.n_flag_r == 0
            abft.recover_block(P.p, P.C, rect, use_rows=use_rows)
            rep = P.verify()
            assert rep.n_flag_c == 0 and rep.n_flag_r == 0
            i0, j0, h, w = rect
            got = P.C[i0:i0 + h, j0:j0 + w].cpu().numpy().astype(np.float64)
            want = C32[i0:i0 + h, j0:j0 + w].astype(np.float64)
            assert np.abs(got - want).max() <= np.abs(tc).max()


@pytest.mark.parametrize("dt", ["bf16", "fp8"])
@pytest.mark.parametrize("m,n,k", [(4096, 4352, 128), (4300, 4100, 640), (300, 260, 528)])
def test_lowp_integer_products_exact(dev, m, n, k, dt):
    """Integer operands in [-4, 4] are exact in both element types (FP8 after its
    scale 2^6), and every product and partial sum of the data part is an integer
    of magnitude at most 16 k < 2^24 (times 2^12 in the FP8 domain), so the
    matrix cores must return the exact product whatever their summation order:
    the data part of C_f equals the integer product bit for bit.  This pins the
    fragment and accumulator lane layouts of each kernel (direct-to-LDS with one
    and with five FP8 slabs, padded-LDS) without any rounding tolerance."""
    note(f"{dt} integer m={m} n={n} k={k}")
    A = synth.uniform_ints(SEED + 3, synth.STREAM_A, m, k, -4, 4)
    B = synth.uniform_ints(SEED + 3, synth.STREAM_B, k, n, -4, 4)
    P = abft.Protected(DTYPES[dt], m, n, k, 1, 1, device=dev, tau_mode=abft.ABFT_TAU_STAT, lam=LAMBDA)
    abft.quantize(P.p, 0, torch.from_numpy(A.astype(np.float32)).to(dev), P.A, P.ws)
    abft.quantize(P.p, 1, torch.from_numpy(np.ascontiguousarray(B.T).astype(np.float32)).to(dev), P.Bt, P.ws)
    P.encode()
    P.gemm()
    torch.cuda.synchronize()
    want = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float32)
    got = P.C[:m, :n].cpu().numpy()
    assert np.array_equal(got, want), np.abs(got.astype(np.float64) - want).max()
    rep = P.verify()
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0


def test_fp8_every_finite_code(dev, orc):
    """A holds every finite E4M3 value (all 254 codes but the two NaN codes,
    each many times; amax 448, so the per-tensor scale is 2^0 and the stored
    codes are these values exactly).  The encode widens them with the device's
    E4M3 conversion and the matrix core with its own decode, so one code decoded
    wrongly on either side would break a relation: the product must meet the
    FP8 value bound against the oracle and verify clean."""
    m, n, k = 256, 384, 512
    codes = np.array([c for c in range(256) if c & 0x7F != 0x7F], dtype=np.uint8)
    vals = orc.e4m3_values(codes)
    idx = (np.arange(m * k) * 7) % codes.size
    A32 = vals[idx].reshape(m, k).astype(np.float32)
    B32 = synth.uniform(SEED + 5, synth.STREAM_B, k, n, np.float32)
    P = abft.Protected(abft.ABFT_FP8_E4M3, m, n, k, 1, 1, device=dev, tau_mode=abft.ABFT_TAU_STAT, lam=LAMBDA)
    abft.quantize(P.p, 0, torch.from_numpy(A32).to(dev), P.A, P.ws)
    abft.quantize(P.p, 1, torch.from_numpy(np.ascontiguousarray(B32.T)).to(dev), P.Bt, P.ws)
    torch.cuda.synchronize()
    assert np.array_equal(P.A.cpu().numpy(), codes[idx].reshape(m, k))
    Aq, A, eA = oracle_quantize(orc, "fp8", A32)
    Bq, B, eB = oracle_quantize(orc, "fp8", B32)
    assert eA == 0
    P.encode()
    P.gemm()
    torch.cuda.synchronize()
    Af, Bf = orc.encode(A, B, 1, 1, store_f32=True)
    C32 = (orc.gemm(Af, Bf) * 2.0 ** -(eA + eB)).astype(np.float32)
    Cg = P.C.cpu().numpy().astype(np.float64)
    bound = (k * U32 + 2.0 ** -10) * (np.abs(Af) @ np.abs(Bf)) * 2.0 ** -(eA + eB) + U32 * np.abs(C32)
    assert np.all(np.abs(Cg - C32) <= bound * 1.01 + 1e-30)
    rep = P.verify()
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0, (rep.max_ratio_c, rep.max_ratio_r)


# ---------------------------------------------------------------- the FP8 matrix cores' product-sum window
def _fp8_codes(orc, X):
    return orc.to_e4m3_codes(np.asarray(X, dtype=np.float32))


# (A row, B column) pairs over one k group: a large product 16 x 16 = 256 and
# small ones 2^-3 x 2^-3 = 2^-6 (exact sums 256 + 31/64 and so on); the window
# drops what lies below 2^-11 of the largest product of a group
WINDOW_PATTERNS = [
    ([16.0] + [0.125] * 31, [16.0] + [0.125] * 31),
    ([-16.0] + [0.125] * 31, [16.0] + [0.125] * 31),
    ([16.0] + [0.125] * 63, [16.0] + [0.125] * 63),
    ([0.125] * 31 + [16.0], [0.125] * 31 + [16.0]),
    ([16.0] + [0.0] * 63 + [0.125] * 31, [16.0] + [0.0] * 63 + [0.125] * 31),   # small ones in the next group
]


@pytest.mark.parametrize("m,n,k", [(64, 64, 528), (4096, 4096, 256)],
                         ids=["padded-LDS-16x16x32", "direct-LDS-32x32x64"])
def test_fp8_product_sum_window(dev, orc, m, n, k):
    """Constructed E4M3 operands (scale 2^0) through each FP8 kernel: the
    error of each product stays within 2^-11 of the largest product of its k
    group (the measured window; the value tolerance uses w = 2^-10 of
    (|A_q||B_q|)), it is a truncation (never above the exact sum, so it does
    not grow the magnitude), and a group with no large product is exact."""
    note(f"fp8 window m={m} n={n} k={k}")
    P = abft.Protected(abft.ABFT_FP8_E4M3, m, n, k, 1, 1, device=dev, tau_mode=abft.ABFT_TAU_STAT, lam=LAMBDA)
    A = np.zeros((m, k), np.float32)
    Bt = np.zeros((n, k), np.float32)
    for q, (a, b) in enumerate(WINDOW_PATTERNS):
        A[q, :len(a)] = a
        Bt[q, :len(b)] = b
    P.A.copy_(torch.from_numpy(_fp8_codes(orc, A)))
    P.Bt.copy_(torch.from_numpy(_fp8_codes(orc, Bt)))
    C = torch.zeros(m, n, dtype=torch.float32, device=dev)
    pp = abft.problem(abft.ABFT_FP8_E4M3, m, n, k, 1, 1, ldc=n)
    abft.gemm(pp, P.A, P.Bt, C, P.ws, flags=abft.ABFT_PLAIN)      # ws is zero: scale exponents 0
    torch.cuda.synchronize()
    Cg = C.cpu().numpy().astype(np.float64)
    Aq = orc.e4m3_values(_fp8_codes(orc, A))
    Bq = orc.e4m3_values(_fp8_codes(orc, Bt))
    for q in range(len(WINDOW_PATTERNS)):
        exact = float(Aq[q] @ Bq[q])
        err = Cg[q, q] - exact
        largest = float(np.abs(Aq[q] * Bq[q]).max())
        absprod = float(np.abs(Aq[q]) @ np.abs(Bq[q]))
        note(f"  pattern {q}: exact {exact} gpu {Cg[q, q]} error {err:+.6f}")
        assert abs(err) <= 2.0 ** -11 * largest, (q, err)
        assert abs(err) <= 2.0 ** -10 * absprod
        assert err <= 0.0                                        # truncated toward minus infinity
        if q == 4:
            assert err == 0.0                                    # small products alone in their group: exact
    assert Cg[0, 0] != float(Aq[0] @ Bq[0])                      # the window is there (else the model is moot)


@pytest.mark.parametrize("dt", ["fp8", "bf16"])
@pytest.mark.parametrize("k", [4096, 16384, 16400])
def test_same_sign_operands_verify_clean(dev, orc, dt, k):
    """Operands of one sign (|uniform|, the truncating FP8 window then errs in
    one direction for every product) at k = 4096 and 16384 on the
    direct-to-LDS kernel and 16400 on the padded-LDS one: the products verify
    clean under the statistical thresholds (no false positive)."""
    m = n = 4096
    note(f"same-sign {dt} m=n={m} k={k}")
    P = abft.Protected(DTYPES[dt], m, n, k, 1, 1, device=dev, tau_mode=abft.ABFT_TAU_STAT, lam=LAMBDA)
    A32 = torch.empty(m, k, dtype=torch.float32, device=dev)
    Bt32 = torch.empty(n, k, dtype=torch.float32, device=dev)
    abft.fill_uniform(abft.ABFT_F32, m, k, k, 0, SEED + 7, synth.STREAM_A, A32)
    abft.fill_uniform(abft.ABFT_F32, k, n, k, 1, SEED + 7, synth.STREAM_B, Bt32)
    A32.abs_()
    Bt32.abs_()
    abft.quantize_encode(P.p, A32, Bt32, P.A, P.Bt, P.ws)
    P.gemm()
    rep = P.verify()
    note(f"  {abft.describe_gemm(P.p)}: max |D|/tau {rep.max_ratio_c:.3f} / {rep.max_ratio_r:.3f}")
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0
    assert max(rep.max_ratio_c, rep.max_ratio_r) < 0.8


@pytest.mark.parametrize("dt", ["bf16", "fp8"])
def test_nonfinite_stored_total_fails_its_relations(dev, orc, dt):
    """A stored total made infinite (a fault in the carried row) must not lift
    its own threshold to infinity: the column relation it closes and the row
    relation it sits in both fail, with non-finite residuals, and every other
    threshold is as before (checked against the oracle on the same C)."""
    m, n, k = 256, 256, 256
    P, A, B, Af, Bf, C32, tc, tr = make(dev, orc, m, n, k, 1, 1, dt)
    P.encode()
    P.gemm()
    j = 77
    note(f"{dt} stored total C[{m}, {j}] = inf")
    P.C[m, j] = float("inf")
    rep = P.verify()
    assert [(a, b) for a, b, _, _ in rep.flags_c()] == [(0, j)]
    assert [(a, b) for a, b, _, _ in rep.flags_r()] == [(m, 0)]
    assert rep.n_nonfinite == 2
    Cx = C32.copy()
    Cx[m, j] = np.inf
    tcx, trx = P.retau(Cx)
    assert np.isfinite(tcx).all() and np.isfinite(trx).all()
    (_, _, _, tau_c), = rep.flags_c()
    (_, _, _, tau_r), = rep.flags_r()
    assert abs(tau_c - tcx[0, j]) <= 1e-6 * tcx[0, j] and abs(tau_r - trx[m, 0]) <= 1e-6 * trx[m, 0]
    _, _, orep = orc.verify(Cx.astype(np.float64), m, n, 1, 1, tcx, trx)
    assert (orep.n_flag_c, orep.n_flag_r, orep.n_nonfinite) == (1, 1, 2)
