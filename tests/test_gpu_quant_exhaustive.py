"""The device quantizers against the oracle's on every binary32 input they can
meet, bit for bit.

 - bfloat16 (round to nearest even, NaN kept quiet): all 2^32 patterns.
 - FP8 E4M3 at scale 2^0: every pattern with |x| <= 448 in both signs, both
   infinities and every NaN (about 2.3e9).  Each chunk carries one extra row
   of 448, so that its per-tensor scale is 2^0 (a finite |x| above 448 only
   ever reaches the rounding after a scale 2^e < 1 has brought it to 448 or
   below; infinities and NaN take no part in the scale).
 - FP8 at scales far from 2^0: operands with infinities and NaN, with amax
   2^-120 (scale 2^128, beyond binary32's own exponent range) and with amax
   2^120 (scale 2^-113); and a product of the first kind against the oracle.

Patterns are made on both sides from their index (no transfer of inputs);
the oracle's conversions run on host threads in slices.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_0806_3121_amd import abft, synth  # noqa: E402

pytestmark = pytest.mark.gpu

K = 8192                         # columns of a chunk matrix
ROWS = 1 << 14                   # rows of patterns per chunk: 2^27 patterns
CHUNK = ROWS * K
THREADS = 8
MAX448 = 0x43E00000              # bit pattern of 448.0
HALF8 = MAX448 + 1 + (1 << 23)   # per sign: 0 .. 448, then +inf and every NaN


def note(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abft.lib()
    return torch.device("cuda:0")


def host_patterns(kind, t0, count):
    t = np.arange(t0, t0 + count, dtype=np.int64)
    if kind == "fp8":
        h, r = t // HALF8, t % HALF8
        t = np.where(r <= MAX448, r, 0x7F800000 + (r - MAX448 - 1)) | (h << 31)
    return t.astype(np.uint32)


def device_patterns(kind, t0, count, dev):
    t = torch.arange(t0, t0 + count, dtype=torch.int64, device=dev)
    if kind == "fp8":
        h, r = t // HALF8, t % HALF8
        t = torch.where(r <= MAX448, r, 0x7F800000 + (r - MAX448 - 1)) | (h << 31)
    t = torch.where(t >= 1 << 31, t - (1 << 32), t)          # the same 32 bits as a signed word
    return t.to(torch.int32).view(torch.float32)


def oracle_codes(orc, kind, pats):
    """The oracle's conversion of the binary32 patterns pats, in slices on host threads."""
    x = pats.view(np.float32)
    conv = orc.to_bf16_bits if kind == "bf16" else orc.to_e4m3_codes
    sl = -(-x.size // THREADS)
    with ThreadPoolExecutor(THREADS) as ex:
        parts = list(ex.map(lambda q: conv(x[q * sl:(q + 1) * sl]), range(THREADS)))
    return np.concatenate(parts)


@pytest.mark.parametrize("kind", ["bf16", "fp8"])
def test_every_pattern_quantizes_as_the_oracle(dev, orc, kind):
    total = (1 << 32) if kind == "bf16" else 2 * HALF8
    rows = ROWS + (1 if kind == "fp8" else 0)
    dtype = abft.ABFT_BF16 if kind == "bf16" else abft.ABFT_FP8_E4M3
    p = abft.problem(dtype, rows, 16, K, 1, 1, tau_mode=abft.ABFT_TAU_STAT)
    ws = torch.zeros(abft.workspace_size(p), dtype=torch.uint8, device=dev)
    X = torch.zeros(rows, K, dtype=torch.float32, device=dev)
    if kind == "fp8":
        X[ROWS:] = 448.0
    dst = torch.empty(rows, K, dtype=torch.bfloat16 if kind == "bf16" else torch.uint8, device=dev)
    bad = 0
    for t0 in range(0, total, CHUNK):
        count = min(CHUNK, total - t0)
        note(f"{kind} patterns [{t0}, {t0 + count}) of {total}")
        X.view(-1)[:count] = device_patterns(kind, t0, count, dev)
        if count < CHUNK:
            X.view(-1)[count:CHUNK] = 0.0
        abft.quantize(p, 0, X, dst, ws)
        got = dst.view(-1)[:count]
        got = (got.view(torch.int16).cpu().numpy().view(np.uint16) if kind == "bf16" else got.cpu().numpy())
        want = oracle_codes(orc, kind, host_patterns(kind, t0, count))
        diff = np.nonzero(got != want)[0]
        if diff.size:
            pats = host_patterns(kind, t0, count)
            for q in diff[:8]:
                note(f"  pattern {pats[q]:#010x}: device {got[q]:#x} oracle {want[q]:#x}")
            bad += diff.size
    assert bad == 0


def test_fp8_scale_from_finite_entries_and_beyond_binary32_range(dev, orc):
    m, k = 64, 256
    base = synth.uniform(synth.BASE_SEED + 71, synth.STREAM_A, m, k, np.float32)
    cases = {"non-finite entries": base * np.float32(5.0),
             "amax 2^-120": (base.astype(np.float64) * 2.0 ** -120).astype(np.float32),
             "amax 2^120": (base.astype(np.float64) * 2.0 ** 120).astype(np.float32)}
    X0 = cases["non-finite entries"]
    X0[3, 7], X0[10, 0], X0[63, 255], X0[20, 100] = np.inf, -np.inf, np.nan, -np.nan
    p = abft.problem(abft.ABFT_FP8_E4M3, m, 16, k, 1, 1, tau_mode=abft.ABFT_TAU_STAT)
    ws = torch.zeros(abft.workspace_size(p), dtype=torch.uint8, device=dev)
    dst = torch.empty(m, k, dtype=torch.uint8, device=dev)
    for name, X in cases.items():
        e = orc.e4m3_scale_exp(X)
        note(f"fp8 quantize, {name}: oracle scale 2^{e}")
        abft.quantize(p, 0, torch.from_numpy(X).to(dev), dst, ws)
        want = orc.to_e4m3_codes(np.ldexp(X.astype(np.float64), e).astype(np.float32))
        assert np.array_equal(dst.cpu().numpy(), want), name
        if name == "non-finite entries":
            got = dst.cpu().numpy()
            assert (got[3, 7], got[10, 0], got[63, 255], got[20, 100]) == (0x7E, 0xFE, 0x7F, 0x7F)


def test_fp8_product_with_scale_beyond_binary32_range(dev, orc):
    """A (amax about 2^-120) takes the scale 2^128, whose factor binary32 cannot
    hold; the product, scaled back by 2^-(eA + eB), matches the oracle to the
    FP8 value bound and verifies clean."""
    m, n, k = 256, 192, 512
    A32 = (synth.uniform(synth.BASE_SEED + 72, synth.STREAM_A, m, k).astype(np.float64) * 2.0 ** -120).astype(
        np.float32)
    B32 = synth.uniform(synth.BASE_SEED + 72, synth.STREAM_B, k, n, np.float32)
    eA, eB = orc.e4m3_scale_exp(A32), orc.e4m3_scale_exp(B32)
    assert eA > 127
    P = abft.Protected(abft.ABFT_FP8_E4M3, m, n, k, 1, 1, device=dev, tau_mode=abft.ABFT_TAU_STAT, lam=10.0)
    abft.quantize_encode(P.p, torch.from_numpy(A32).to(dev), torch.from_numpy(np.ascontiguousarray(B32.T)).to(dev),
                         P.A, P.Bt, P.ws)
    P.gemm()
    rep = P.verify()
    note(f"fp8 eA={eA} eB={eB}: max |D|/tau {max(rep.max_ratio_c, rep.max_ratio_r):.3f}")
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0
    qa = orc.to_e4m3_codes(np.ldexp(A32.astype(np.float64), eA).astype(np.float32))
    qb = orc.to_e4m3_codes(np.ldexp(B32.astype(np.float64), eB).astype(np.float32))
    assert np.array_equal(P.A.cpu().numpy(), qa)
    assert np.array_equal(P.Bt.cpu().numpy(), np.ascontiguousarray(qb.T))
    Aq, Bq = orc.e4m3_values(qa), orc.e4m3_values(qb)
    Af, Bf = orc.encode(Aq, Bq, 1, 1, store_f32=True)
    sc = 2.0 ** -(eA + eB)
    C = (orc.gemm(Af, Bf) * sc).astype(np.float32).astype(np.float64)
    bound = (k * 2.0 ** -24 + 2.0 ** -10) * (np.abs(Af) @ np.abs(Bf)) * sc + 2.0 ** -24 * np.abs(C)
    Cg = P.C.cpu().numpy().astype(np.float64)
    assert np.all(np.isfinite(Cg))
    assert np.all(np.abs(Cg - C) <= bound * 1.01 + 1e-300)
