"""GPU test of abft_quantize_encode: quantizing both binary32 operands and
encoding them (bfloat16 in one pass per operand) must leave A_f, B_f and the
whole workspace bitwise equal to abft_quantize (A), abft_quantize (B) and abft_encode, and
the products and verification reports that follow must be equal too.  Shapes
cover the partitioned (b = 1, 32) and direct (one group) encode passes, k with
and without the fused row statistics (k / 8 resp. k / 16 a multiple of 64),
and ragged m, n.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_0806_3121_amd import abft, synth  # noqa: E402

pytestmark = pytest.mark.gpu

SEED = synth.BASE_SEED + 91
DT = {"bf16": abft.ABFT_BF16, "fp8": abft.ABFT_FP8_E4M3}


def note(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abft.lib()
    return torch.device("cuda:0")


CASES = [
    ("bf16", 512, 384, 1024, 1),     # partitioned encode, fused row statistics
    ("bf16", 300, 260, 528, 1),      # ragged, row statistics in their own pass
    ("bf16", 512, 512, 512, 32),     # partitioned, 32 residues
    ("bf16", 256, 256, 1024, 256),   # one group: direct encode
    ("fp8", 512, 384, 1024, 1),
    ("fp8", 300, 260, 528, 1),
    ("fp8", 256, 256, 1024, 256),
]
IDS = [f"{c[0]}-{c[1]}x{c[2]}x{c[3]}-b{c[4]}" for c in CASES]


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_quantize_encode_equals_separate_calls(dev, case):
    dt, m, n, k, b = case
    note(f"quantize_encode {case}")
    A32 = torch.empty(m, k, dtype=torch.float32, device=dev)
    B32 = torch.empty(n, k, dtype=torch.float32, device=dev)
    abft.fill_uniform(abft.ABFT_F32, m, k, k, 0, SEED, synth.STREAM_A, A32)
    abft.fill_uniform(abft.ABFT_F32, k, n, k, 1, SEED, synth.STREAM_B, B32)
    mode = abft.ABFT_TAU_STAT
    P = abft.Protected(DT[dt], m, n, k, b, b, device=dev, tau_mode=mode, lam=10.0)
    Q = abft.Protected(DT[dt], m, n, k, b, b, device=dev, tau_mode=mode, lam=10.0)
    abft.quantize(P.p, 0, A32, P.A, P.ws)
    abft.quantize(P.p, 1, B32, P.Bt, P.ws)
    P.encode()
    abft.quantize_encode(Q.p, A32, B32, Q.A, Q.Bt, Q.ws)
    torch.cuda.synchronize()
    assert torch.equal(P.A, Q.A) and torch.equal(P.Bt, Q.Bt)
    assert torch.equal(P.ws, Q.ws)
    P.gemm()
    Q.gemm()
    torch.cuda.synchronize()
    assert torch.equal(P.C, Q.C)
    rp, rq = P.verify(), Q.verify()
    assert (rp.n_flag_c, rp.n_flag_r, rp.max_ratio_c, rp.max_ratio_r) == (rq.n_flag_c, rq.n_flag_r, rq.max_ratio_c,
                                                                          rq.max_ratio_r)
    assert rq.n_flag_c == 0 and rq.n_flag_r == 0
