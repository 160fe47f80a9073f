"""GPU tests of the fused checksum accumulation (the product kernels' epilogue
writes binary64 partial sums of each tile's columns and rows; verification
reads them instead of C) and of the in-kernel fault site (an accumulator bit
flipped before the epilogue), for every product kernel at b = 1.

 - clean products: the fused verification is clean, as the re-reading one;
 - an accumulator flip changes exactly that element of C, and the fused
   verification fails the same relations as the re-reading one on the same C
   (indices equal, residuals equal up to the summation order), so the oracle-
   pinned classification locates it and the correction restores C;
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


def note(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abft.lib()
    return torch.device("cuda:0")


def make(dev, dt, m, n, k):
    adt = DT[dt]
    mode = abft.ABFT_TAU_DET if dt == "f64" else abft.ABFT_TAU_STAT
    P = abft.Protected(adt, m, n, k, 1, 1, device=dev, tau_mode=mode, lam=10.0)
    if dt in ("f64", "f32"):
        abft.fill_uniform(adt, m, k, k, 0, SEED, synth.STREAM_A, P.A)
        abft.fill_uniform(adt, k, n, k, 1, SEED, synth.STREAM_B, P.Bt)
    else:
        A32 = torch.empty(m, k, dtype=torch.float32, device=dev)
        Bt32 = torch.empty(n, k, dtype=torch.float32, device=dev)
        abft.fill_uniform(abft.ABFT_F32, m, k, k, 0, SEED, synth.STREAM_A, A32)
        abft.fill_uniform(abft.ABFT_F32, k, n, k, 1, SEED, synth.STREAM_B, Bt32)
        abft.quantize(P.p, 0, A32, P.A, P.ws)
        abft.quantize(P.p, 1, Bt32, P.Bt, P.ws)
    P.encode()
    return P


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
def test_fused_clean_and_accumulator_flips(dev, case):
    dt, m, n, k, kernel = case
    note(f"fused {case}")
    P = make(dev, dt, m, n, k)
    assert abft.describe_gemm(P.p, abft.ABFT_FUSED).startswith(kernel + " on"), abft.describe_gemm(P.p, abft.ABFT_FUSED)
    fused_gemm(P)
    torch.cuda.synchronize()
    clean = P.C.clone()
    rf = P.verify_fused()
    rr = P.verify()
    assert rf.n_flag_c == rf.n_flag_r == 0 and rr.n_flag_c == rr.n_flag_r == 0
    assert 0 < max(rf.max_ratio_c, rf.max_ratio_r) < 0.5
    note(f"  clean max |D|/tau fused {max(rf.max_ratio_c, rf.max_ratio_r):.3e} "
         f"re-read {max(rr.max_ratio_c, rr.max_ratio_r):.3e}")
    sites = [(synth.randint(SEED, synth.STREAM_FLIP, 3 * q, m), synth.randint(SEED, synth.STREAM_FLIP, 3 * q + 1, n),
              BITS[dt][q % 2]) for q in range(4)]
    sites[0] = (m - 1, n - 1, BITS[dt][0])                   # last row and column of a ragged tile
    for (i, j, bit) in sites:
        note(f"  accumulator flip ({i},{j}) bit {bit}")
        abft.arm_accumulator_flip(P.p, P.ws, i, j, bit)
        fused_gemm(P)
        torch.cuda.synchronize()
        diff = (P.C != clean).nonzero().cpu().numpy()
        assert [tuple(x) for x in diff] == [(i, j)]
        rf = P.verify_fused()
        rr = P.verify()
        assert [(a, b) for a, b, _, _ in rf.flags_c()] == [(a, b) for a, b, _, _ in rr.flags_c()] == [(0, j)]
        assert [(a, b) for a, b, _, _ in rf.flags_r()] == [(a, b) for a, b, _, _ in rr.flags_r()] == [(i, 0)]
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


def test_memory_flip_after_product_seen_by_reread_only(dev):
    P = make(dev, "f64", 520, 392, 256)
    note("memory flip after a fused product")
    fused_gemm(P)
    abft.inject_flip(P.p, P.C, 100, 200, 58)
    rf = P.verify_fused()
    assert rf.n_flag_c == 0 and rf.n_flag_r == 0
    rr = P.verify()
    loc = abft.classify(P.p, rr)
    assert (loc.cls, loc.i, loc.j) == (abft.ABFT_CLS_DATA, 100, 200)


def test_fused_state_and_refusals(dev):
    P = make(dev, "f64", 256, 256, 128)
    note("fused refusals")
    with pytest.raises(abft.AbftError) as e:
        P.verify_fused()                       # no fused product on this workspace yet
    assert e.value.status == abft.ABFT_E_ARG
    fused_gemm(P)
    P.verify_fused()
    P.gemm()                                   # a product without partials makes them stale
    with pytest.raises(abft.AbftError):
        P.verify_fused()
    with pytest.raises(abft.AbftError) as e:
        abft.arm_accumulator_flip(P.p, P.ws, 256, 0, 3)    # carried row: not an accumulator of the data kernel
    assert e.value.status == abft.ABFT_E_ARG
    # partials of another problem on the same workspace are refused
    fused_gemm(P)
    other = abft.problem(abft.ABFT_F64, 128, 256, 128, 1, 1, ldc=P.ldc)
    with pytest.raises(abft.AbftError) as e:
        abft.verify_fused(other, P.C, P.ws)
    assert e.value.status == abft.ABFT_E_ARG
    P.verify_fused()
    Q = abft.Protected(abft.ABFT_F64, 256, 256, 128, 64, 64, device=dev)
    with pytest.raises(abft.AbftError) as e:
        abft.gemm(Q.p, Q.A, Q.Bt, Q.C, Q.ws, flags=abft.ABFT_FUSED)
    assert e.value.status == abft.ABFT_E_UNSUPPORTED
