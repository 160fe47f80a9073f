"""GPU parity of the binary32 path (binary32 inputs, binary32 matrix-core
accumulation, statistical thresholds) against the CPU oracle.

The oracle takes the same binary32 inputs exactly in binary64, keeps its
checksum rows rounded once to binary32, computes C_f in binary64 and rounds
it to binary32 (so both sides inject the same flip into the same binary32
value).  Values: max|C_gpu - C_oracle| / max|C_oracle| <= 1e-5.  Decisions
and indices: bit-exact outside the gray zone tau/2 < |delta| < 2 tau.
Flip bits 11..30 (top 12 fraction bits and every exponent bit of binary32,
no sign bit, mirroring binary64's 40..62).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_0806_3121_amd import abft, synth  # noqa: E402

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
SEED = synth.BASE_SEED + 32
LAMBDA = 10.0


def note(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abft.lib()
    return torch.device("cuda:0")


def make(dev, m, n, k, br, bc, A=None, B=None):
    if A is None:
        A = synth.uniform(SEED, synth.STREAM_A, m, k, np.float32)
        B = synth.uniform(SEED, synth.STREAM_B, k, n, np.float32)
    P = abft.Protected(abft.ABFT_F32, m, n, k, br, bc, device=dev, tau_mode=abft.ABFT_TAU_STAT, lam=LAMBDA)
    P.A[:m] = torch.from_numpy(A).to(dev)
    P.Bt[:n] = torch.from_numpy(np.ascontiguousarray(B.T)).to(dev)
    return A, B, P


def thresholds(orc, Af, Bf, m, n, br, bc, Cf):
    """The oracle's statistical thresholds; each relation's stored total is read from Cf."""
    k = Af.shape[1]
    return orc.tau_stat(Af, Bf, m, n, br, bc, u_acc=orc.U32, T=float(k), s_store=2.0, lam=LAMBDA,
                        Cf=np.asarray(Cf, dtype=np.float64))


def oracle_side(orc, A, B, br, bc):
    m, n = A.shape[0], B.shape[1]
    Af, Bf = orc.encode(A.astype(np.float64), B.astype(np.float64), br, bc, store_f32=True)
    C64 = orc.gemm(Af, Bf)
    C32 = C64.astype(np.float32)
    tc, tr = thresholds(orc, Af, Bf, m, n, br, bc, C64)
    return Af, Bf, C32, tc, tr


def residuals(Cf, m, n, br, bc):
    Dc = sum(Cf[g * br:(g + 1) * br] for g in range(m // br)) - Cf[m:m + br]
    Dr = sum(Cf[:, h * bc:(h + 1) * bc] for h in range(n // bc)) - Cf[:, n:n + bc]
    return Dc, Dr


SHAPES = [
    (256, 256, 256, 1, 1),
    (200, 136, 72, 8, 4),
    (512, 384, 1024, 64, 64),
    (384, 640, 1000, 1, 5),
    (1024, 1024, 4096, 1, 1),
]


@pytest.mark.parametrize("m,n,k,br,bc", SHAPES)
def test_f32_product_and_clean_verify(dev, orc, m, n, k, br, bc):
    note(f"f32 m={m} n={n} k={k} br={br} bc={bc}")
    A, B, P = make(dev, m, n, k, br, bc)
    P.encode()
    P.gemm()
    torch.cuda.synchronize()
    Af, Bf, C32, tc, tr = oracle_side(orc, A, B, br, bc)
    gA = P.A[m:].cpu().numpy().astype(np.float64)
    # checksum rows: binary64 sums in another order, each rounded once to binary32
    assert np.all(np.abs(gA - Af[m:]) <= 2.0 ** -23 * np.abs(Af[m:]) + 4 * m * 2.0 ** -53)
    Cg = P.C.cpu().numpy()
    err = np.abs(Cg.astype(np.float64) - C32).max() / np.abs(C32).max()
    assert err <= TOL32, err
    rep = P.verify()
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0, (rep.max_ratio_c, rep.max_ratio_r)
    # calibration read-out: the GPU residuals (summed here in binary64) against
    # the model's sigma = tau / lambda
    Dc, Dr = residuals(Cg.astype(np.float64), m, n, br, bc)
    z = np.concatenate([(Dc / (tc / LAMBDA)).ravel(), (Dr / (tr / LAMBDA)).ravel()])
    note(f"  gpu |D|/sigma: rms {np.sqrt(np.mean(z * z)):.3f} max {np.abs(z).max():.3f}; max ratio "
         f"{max(rep.max_ratio_c, rep.max_ratio_r):.4f}; C err {err:.2e}")
    assert np.abs(z).max() < LAMBDA / 2
    _, _, orep2 = orc.verify(C32.astype(np.float64), m, n, br, bc, tc, tr)
    assert orep2.n_flag_c == 0 and orep2.n_flag_r == 0


@pytest.mark.parametrize("m,n,k,br,bc,runs", [(256, 256, 256, 1, 1, 60), (512, 384, 1024, 64, 64, 40),
                                              (200, 136, 72, 8, 4, 40)])
def test_f32_flip_decisions_match_oracle(dev, orc, m, n, k, br, bc, runs):
    A, B, P = make(dev, m, n, k, br, bc)
    P.encode()
    P.gemm()
    clean = P.C.clone()
    Af, Bf, C32, tc, tr = oracle_side(orc, A, B, br, bc)
    M, N = m + br, n + bc
    located = compared = 0
    for run in range(runs):
        i, j, bit = synth.flip_site(SEED + 7, run, M, N, 11, 30)
        note(f"f32 flip run={run} ({i},{j}) bit {bit}")
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
        tcx, trx = thresholds(orc, Af, Bf, m, n, br, bc, Cx) if (i >= m or j >= n) else (tc, tr)
        _, _, orep = orc.verify(Cx.astype(np.float64), m, n, br, bc, tcx, trx)
        ocls, oi, oj, od = orc.classify(orep, m, n, br, bc)
        assert (rep.n_flag_c, rep.n_flag_r) == (orep.n_flag_c, orep.n_flag_r), (i, j, bit, delta)
        # the GPU's statistical thresholds are the oracle's (the weighted row sums of A take their weights
        # in binary32, 2^-24 relative)
        for r, jj, _, tau in rep.flags_c():
            assert abs(tau - tcx[r, jj]) <= 1e-6 * tcx[r, jj]
        for ii, c, _, tau in rep.flags_r():
            assert abs(tau - trx[ii, c]) <= 1e-6 * trx[ii, c]
        assert (loc.cls, loc.i, loc.j) == (ocls, oi, oj)
        if loc.cls in (abft.ABFT_CLS_DATA, abft.ABFT_CLS_CHECKSUM):
            located += 1
            assert (loc.i, loc.j) == (i, j)
            abft.correct(P.p, P.C, loc)
            rep2 = P.verify()
            assert rep2.n_flag_c == 0 and rep2.n_flag_r == 0
            assert abs(P.C[i, j].item() - clean[i, j].item()) <= min(t1, t2)
    note(f"  compared {compared}, located {located}")
    assert compared >= runs * 0.8 and located >= compared * 0.4


def test_f32_erasure_rebuild(dev, orc):
    m = n = 512
    k, b = 256, 64
    A, B, P = make(dev, m, n, k, b, b)
    P.encode()
    P.gemm()
    clean = P.C.clone()
    Af, Bf, C32, tc, tr = oracle_side(orc, A, B, b, b)
    for rect in [(64, 128, 64, 64), (512, 0, 64, 64), (10, 512, 50, 60)]:
        for use_rows in (False, True):
            note(f"f32 erase {rect} rows={use_rows}")
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
            assert np.abs(got - want).max() / np.abs(C32).max() <= TOL32


# Heavy-tailed inputs: N(0,1) with 1 % of the entries scaled by 1e3 (the
# second input set of the binary32 workload).  Same bars: values, clean verify
# with the statistical thresholds, flip decisions equal the oracle's.
HEAVY = [(512, 384, 2048, 1, 1), (384, 256, 1000, 8, 4)]


def heavy_inputs(m, n, k):
    A = synth.normal_with_outliers(SEED + 101, m, k)
    B = synth.normal_with_outliers(SEED + 102, k, n)
    return A, B


@pytest.mark.parametrize("m,n,k,br,bc", HEAVY)
def test_f32_heavy_tailed_product_and_clean_verify(dev, orc, m, n, k, br, bc):
    note(f"f32 heavy-tailed m={m} n={n} k={k} br={br} bc={bc}")
    A, B = heavy_inputs(m, n, k)
    A, B, P = make(dev, m, n, k, br, bc, A, B)
    P.encode()
    P.gemm()
    torch.cuda.synchronize()
    Af, Bf, C32, tc, tr = oracle_side(orc, A, B, br, bc)
    Cg = P.C.cpu().numpy()
    # per element: k binary32 accumulations of the exact products, plus the rounding of C
    bound = k * 2.0 ** -24 * (np.abs(Af) @ np.abs(Bf)) + 2.0 ** -24 * np.abs(C32)
    assert np.all(np.abs(Cg.astype(np.float64) - C32) <= bound * 1.01)
    rep = P.verify()
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0, (rep.max_ratio_c, rep.max_ratio_r)
    Dc, Dr = residuals(Cg.astype(np.float64), m, n, br, bc)
    z = np.concatenate([(Dc / (tc / LAMBDA)).ravel(), (Dr / (tr / LAMBDA)).ravel()])
    note(f"  gpu |D|/sigma: rms {np.sqrt(np.mean(z * z)):.3f} max {np.abs(z).max():.3f}; max ratio "
         f"{max(rep.max_ratio_c, rep.max_ratio_r):.4f}")
    assert np.abs(z).max() < LAMBDA / 2


def test_f32_heavy_tailed_flip_decisions_match_oracle(dev, orc):
    m, n, k, br, bc, runs = 384, 256, 1000, 8, 4, 40
    A, B = heavy_inputs(m, n, k)
    A, B, P = make(dev, m, n, k, br, bc, A, B)
    P.encode()
    P.gemm()
    clean = P.C.clone()
    Af, Bf, C32, tc, tr = oracle_side(orc, A, B, br, bc)
    M, N = m + br, n + bc
    located = compared = 0
    for run in range(runs):
        i, j, bit = synth.flip_site(SEED + 9, run, M, N, 11, 30)
        note(f"f32 heavy flip run={run} ({i},{j}) bit {bit}")
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
        tcx, trx = thresholds(orc, Af, Bf, m, n, br, bc, Cx) if (i >= m or j >= n) else (tc, tr)
        _, _, orep = orc.verify(Cx.astype(np.float64), m, n, br, bc, tcx, trx)
        ocls, oi, oj, od = orc.classify(orep, m, n, br, bc)
        assert (rep.n_flag_c, rep.n_flag_r) == (orep.n_flag_c, orep.n_flag_r), (i, j, bit, delta)
        # the GPU's statistical thresholds are the oracle's (the weighted row sums of A take their weights
        # in binary32, 2^-24 relative)
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
    note(f"  compared {compared}, located {located}")
    assert compared >= runs * 0.7 and located >= 1


def test_same_sign_long_k_rigorous_threshold_clean(dev):
    """Operands of one sign at long k (4096 x 4096 x 65536, |uniform|): the
    statistical threshold's model of zero-mean product errors no longer holds
    there (its clean residuals exceed it, measured), and the rigorous binary32
    bound (ABFT_TAU_DET: gamma_k of the products, the checksum sums and the
    storage) is the mode for such data: every relation passes, and a flip of
    an exponent bit is still located."""
    m = n = 4096
    k = 65536
    note(f"same-sign f32 m=n={m} k={k}, rigorous thresholds")
    P = abft.Protected(abft.ABFT_F32, m, n, k, 1, 1, device=dev, tau_mode=abft.ABFT_TAU_DET)
    abft.fill_uniform(abft.ABFT_F32, m, k, k, 0, SEED + 11, synth.STREAM_A, P.A)
    abft.fill_uniform(abft.ABFT_F32, k, n, k, 1, SEED + 11, synth.STREAM_B, P.Bt)
    P.A.abs_()
    P.Bt.abs_()
    P.encode()
    P.gemm()
    rep = P.verify()
    note(f"  max |D|/tau {rep.max_ratio_c:.3g} / {rep.max_ratio_r:.3g}")
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0
    abft.inject_flip(P.p, P.C, 1234, 567, 29)
    rep = P.verify()
    loc = abft.classify(P.p, rep)
    assert (loc.cls, loc.i, loc.j) == (abft.ABFT_CLS_DATA, 1234, 567)
