"""GPU tests of the fused checksum accumulation (the product kernels' epilogue
writes binary64 partial sums of each tile's columns and rows; verification
reads them instead of C) and of the in-kernel fault site (an accumulator bit
flipped before the epilogue), for every product kernel at b = 1.

 - the fused product's C equals the non-fused product's C bit for bit (same
   kernel, same k order) and the oracle's C element by element (1e-12 binary64,
   1e-5 binary32, the per-element low-precision bound);
 - clean products: the fused verification is clean, as the re-reading one;
 - an accumulator flip changes exactly that element of C; the fused
   verification fails the same relations as the re-reading one, with the
   oracle's residuals of those relations (computed on the GPU's flipped C)
   and the oracle's thresholds, so the classification locates it and the
   correction restores C;
 - a flip of C in memory after the product is seen by the re-reading
   verification only (the partials describe the product as computed).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_0806_3121_amd import abft, synth  # noqa: E402

pytestmark = pytest.mark.gpu

SEED = synth.BASE_SEED + 33
DT = {"f64": abft.ABFT_F64, "f32": abft.ABFT_F32, "bf16": abft.ABFT_BF16, "fp8": abft.ABFT_FP8_E4M3}
U32 = 2.0 ** -24
LAMBDA = 10.0


def note(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abft.lib()
    return torch.device("cuda:0")


class Case:
    """A b = 1 problem on the GPU and the oracle's view of it: the encoded
    operands in binary64 (low precision: the quantized values, scaled back),
    C_f, and the thresholds of the library's model."""

    def __init__(self, dev, orc, dt, m, n, k):
        adt = DT[dt]
        mode = abft.ABFT_TAU_DET if dt == "f64" else abft.ABFT_TAU_STAT
        self.dt, self.m, self.n, self.k = dt, m, n, k
        self.P = P = abft.Protected(adt, m, n, k, 1, 1, device=dev, tau_mode=mode, lam=LAMBDA)
        npdt = np.float64 if dt == "f64" else np.float32
        A = synth.uniform(SEED, synth.STREAM_A, m, k, npdt)
        B = synth.uniform(SEED, synth.STREAM_B, k, n, npdt)
        sc = 1.0
        if dt in ("f64", "f32"):
            P.A[:m] = torch.from_numpy(A).to(dev)
            P.Bt[:n] = torch.from_numpy(np.ascontiguousarray(B.T)).to(dev)
            Af, Bf = orc.encode(A.astype(np.float64), B.astype(np.float64), 1, 1, store_f32=(dt == "f32"))
        else:
            abft.quantize(P.p, 0, torch.from_numpy(A).to(dev), P.A, P.ws)
            abft.quantize(P.p, 1, torch.from_numpy(np.ascontiguousarray(B.T)).to(dev), P.Bt, P.ws)
            if dt == "bf16":
                Aq, Bq, eA, eB = orc.bf16_bits_to_f64(orc.to_bf16_bits(A)), orc.bf16_bits_to_f64(orc.to_bf16_bits(B)), 0, 0
            else:
                eA, eB = orc.e4m3_scale_exp(A), orc.e4m3_scale_exp(B)
                Aq = orc.e4m3_values(orc.to_e4m3_codes(A * np.float32(2.0 ** eA)))
                Bq = orc.e4m3_values(orc.to_e4m3_codes(B * np.float32(2.0 ** eB)))
            Af, Bf = orc.encode(Aq, Bq, 1, 1, store_f32=True)
            sc = 2.0 ** -(eA + eB)
        P.encode()
        C_scaled = orc.gemm(Af, Bf)
        Cf = C_scaled * sc
        self.C_orc = Cf if dt == "f64" else Cf.astype(np.float32).astype(np.float64)
        if dt == "f64":
            self.tc, self.tr = orc.tau_det(Af, Bf, m, n, 1, 1)
        else:
            T = k if dt == "f32" else k / 4.0
            s_store = 2.0 + (2.0 ** 18 if dt == "fp8" else 0.0)
            tc, tr = orc.tau_stat(Af, Bf, m, n, 1, 1, u_acc=U32, T=T, s_store=s_store, lam=LAMBDA, Cf=C_scaled)
            self.tc, self.tr = tc * sc, tr * sc
        self.absprod = (np.abs(Af) @ np.abs(Bf)) * sc if dt in ("bf16", "fp8") else None

    def value_error_ok(self, Cg):
        """C_gpu against the oracle's C, to the bar of the element type."""
        if self.dt == "f64":
            return np.abs(Cg - self.C_orc).max() / np.abs(self.C_orc).max() <= 1e-12
        if self.dt == "f32":
            return np.abs(Cg - self.C_orc).max() / np.abs(self.C_orc).max() <= 1e-5
        w = 2.0 ** -10 if self.dt == "fp8" else 0.0
        bound = (self.k * U32 + w) * self.absprod + U32 * np.abs(self.C_orc)
        return bool(np.all(np.abs(Cg - self.C_orc) <= bound * 1.01 + 1e-30))


def fused_gemm(P):
    abft.gemm(P.p, P.A, P.Bt, P.C, P.ws, flags=abft.ABFT_FUSED)


CASES = [
    ("f64", 520, 392, 256, "k_gemm_mfma2 f64 96x96"),       # direct-to-LDS, ragged edges
    ("f64", 776, 5384, 32, "k_gemm_mfma2 f64 128x96"),
    ("f64", 1032, 5384, 32, "k_gemm_mfma2 f64 128x128"),
    ("f64", 520, 392, 250, "k_gemm_mfma f64 96x96"),        # register-staged (k % 16 != 0)
    ("f32", 384, 640, 1024, "k_gemm_mfma2 f32 256x128"),
    ("f32", 384, 640, 1000, "k_gemm_mfma f32 256x128"),     # K tail
    ("bf16", 512, 384, 1024, "k_gemm_lowp bf16 128x128"),   # padded-LDS kernel
    ("bf16", 4096, 4096, 256, "k_gemm_lowp2 bf16 256x256"),  # direct-to-LDS kernel
    ("fp8", 300, 260, 528, "k_gemm_lowp fp8 128x128"),      # padded-LDS kernel, ragged
    ("fp8", 4096, 4096, 256, "k_gemm_lowp2 fp8 256x256"),    # direct-to-LDS kernel (scaled epilogue)
]
IDS = [f"{c[0]}-{c[1]}x{c[2]}x{c[3]}" for c in CASES]
BITS = {"f64": (55, 60), "f32": (26, 28), "bf16": (26, 28), "fp8": (26, 28)}


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_fused_clean_and_accumulator_flips(dev, orc, case):
    dt, m, n, k, kernel = case
    note(f"fused {case}")
    cs = Case(dev, orc, dt, m, n, k)
    P = cs.P
    assert abft.describe_gemm(P.p, abft.ABFT_FUSED).startswith(kernel + " on"), abft.describe_gemm(P.p, abft.ABFT_FUSED)
    P.gemm()                                  # the same product without the fused epilogue
    torch.cuda.synchronize()
    plain_epilogue = P.C.clone()
    fused_gemm(P)
    torch.cuda.synchronize()
    clean = P.C.clone()
    assert torch.equal(clean, plain_epilogue), "fused and non-fused epilogues store different C"
    Cg = clean.cpu().numpy().astype(np.float64)
    assert cs.value_error_ok(Cg), "fused C against the oracle"
    rf = P.verify_fused()
    rr = P.verify()
    assert rf.status == abft.ABFT_OK
    assert rf.n_flag_c == rf.n_flag_r == 0 and rr.n_flag_c == rr.n_flag_r == 0
    assert 0 < max(rf.max_ratio_c, rf.max_ratio_r) < 0.5
    note(f"  clean max |D|/tau fused {max(rf.max_ratio_c, rf.max_ratio_r):.3e} "
         f"re-read {max(rr.max_ratio_c, rr.max_ratio_r):.3e}")
    sites = [(synth.randint(SEED, synth.STREAM_FLIP, 3 * q, m), synth.randint(SEED, synth.STREAM_FLIP, 3 * q + 1, n),
              BITS[dt][q % 2]) for q in range(4)]
    sites[0] = (m - 1, n - 1, BITS[dt][0])                   # last row and column of a ragged tile
    for (i, j, bit) in sites:
        note(f"  accumulator flip ({i},{j}) bit {bit}")
        P.gemm_fault(i, j, bit, flags=abft.ABFT_FUSED)
        torch.cuda.synchronize()
        diff = (P.C != clean).nonzero().cpu().numpy()
        assert [tuple(x) for x in diff] == [(i, j)]
        rf = P.verify_fused()
        rr = P.verify()
        assert rf.status == abft.ABFT_OK
        assert [(a, b) for a, b, _, _ in rf.flags_c()] == [(a, b) for a, b, _, _ in rr.flags_c()] == [(0, j)]
        assert [(a, b) for a, b, _, _ in rf.flags_r()] == [(a, b) for a, b, _, _ in rr.flags_r()] == [(i, 0)]
        # the oracle's residuals of the two relations through (i, j), on the GPU's flipped C
        Cx = P.C.cpu().numpy().astype(np.float64)
        Dc, Dr, orep = orc.verify(Cx, m, n, 1, 1, cs.tc, cs.tr)
        assert [(r, jj) for r, jj, _, _ in orep.flags_c()] == [(0, j)]
        assert [(ii, c) for ii, c, _, _ in orep.flags_r()] == [(i, 0)]
        (_, _, dcf, tcf), = rf.flags_c()
        (_, _, drf, trf), = rf.flags_r()
        rel_tau = 1e-10 if dt == "f64" else 1e-6
        assert abs(tcf - cs.tc[0, j]) <= rel_tau * cs.tc[0, j] and abs(trf - cs.tr[i, 0]) <= rel_tau * cs.tr[i, 0]
        # residuals: the same sums in another order, each within its threshold of the other
        assert abs(dcf - Dc[0, j]) <= 1e-9 * abs(Dc[0, j]) + tcf, (dcf, Dc[0, j], tcf)
        assert abs(drf - Dr[i, 0]) <= 1e-9 * abs(Dr[i, 0]) + trf, (drf, Dr[i, 0], trf)
        for f, r in zip(rf.flags_c() + rf.flags_r(), rr.flags_c() + rr.flags_r()):
            assert abs(f[2] - r[2]) <= 1e-9 * abs(r[2]) + 2 * r[3]
        loc = abft.classify(P.p, rf)
        assert (loc.cls, loc.i, loc.j) == (abft.ABFT_CLS_DATA, i, j)
        abft.correct(P.p, P.C, loc)
        rep = P.verify()
        assert rep.n_flag_c == 0 and rep.n_flag_r == 0
        torch.cuda.synchronize()
        err = (P.C.double() - clean.double()).abs().max().item() / clean.double().abs().max().item()
        assert err <= (1e-12 if dt == "f64" else 1e-5), err
        P.C.copy_(clean)


def _mk_f64(dev, m, n, k, b=1):
    P = abft.Protected(abft.ABFT_F64, m, n, k, b, b, device=dev)
    abft.fill_uniform(abft.ABFT_F64, m, k, k, 0, SEED, synth.STREAM_A, P.A)
    abft.fill_uniform(abft.ABFT_F64, k, n, k, 1, SEED, synth.STREAM_B, P.Bt)
    P.encode()
    return P


def test_memory_flip_after_product_seen_by_reread_only(dev):
    P = _mk_f64(dev, 520, 392, 256)
    note("memory flip after a fused product")
    fused_gemm(P)
    abft.inject_flip(P.p, P.C, 100, 200, 58)
    rf = P.verify_fused()
    assert rf.status == abft.ABFT_OK
    assert rf.n_flag_c == 0 and rf.n_flag_r == 0
    rr = P.verify()
    loc = abft.classify(P.p, rr)
    assert (loc.cls, loc.i, loc.j) == (abft.ABFT_CLS_DATA, 100, 200)


def test_fused_owner_tag_and_refusals(dev):
    """The workspace records which product owns its partial sums; the fused
    verification reads them only for that product (problem and C_f), and
    reports ABFT_E_STALE, with no flags, otherwise."""
    P = _mk_f64(dev, 256, 256, 128)
    note("fused owner tag and refusals")
    P.ws.zero_()                               # a fresh workspace: no fused product recorded
    P.encode()
    rf = P.verify_fused()
    assert rf.status == abft.ABFT_E_STALE and rf.n_flag_c == rf.n_flag_r == 0
    fused_gemm(P)
    assert P.verify_fused().status == abft.ABFT_OK
    P.gemm()                                   # a product without partials makes them stale
    assert P.verify_fused().status == abft.ABFT_E_STALE
    fused_gemm(P)
    assert P.verify_fused().status == abft.ABFT_OK
    # the same partials read for another problem, or another C_f
    other = abft.problem(abft.ABFT_F64, 128, 256, 128, 1, 1, ldc=P.ldc)
    abft.verify_fused(other, P.C, P.ws, host_out=P.rep_host)
    torch.cuda.synchronize()
    assert abft.read_report(P.rep_host).status == abft.ABFT_E_STALE
    C2 = P.Cbuf.clone()
    abft.verify_fused(P.p, C2[:, :P.N], P.ws, host_out=P.rep_host)
    torch.cuda.synchronize()
    assert abft.read_report(P.rep_host).status == abft.ABFT_E_STALE
    assert P.verify_fused().status == abft.ABFT_OK   # the owner is unchanged
    with pytest.raises(abft.AbftError) as e:
        P.gemm_fault(256, 0, 3)                      # carried row: not an accumulator of the data kernel
    assert e.value.status == abft.ABFT_E_ARG
    with pytest.raises(abft.AbftError) as e:
        abft.verify_fused(P.p, P.C, P.ws[:-8])       # workspace shorter than the problem needs
    assert e.value.status == abft.ABFT_E_WORKSPACE
    Q = abft.Protected(abft.ABFT_F64, 256, 256, 128, 64, 64, device=dev)
    with pytest.raises(abft.AbftError) as e:
        abft.gemm(Q.p, Q.A, Q.Bt, Q.C, Q.ws, flags=abft.ABFT_FUSED)
    assert e.value.status == abft.ABFT_E_UNSUPPORTED
