"""GPU parity of the bfloat16 path (binary32 inputs quantized to bfloat16 on
the GPU, bfloat16 matrix cores with binary32 accumulation, binary32 checksum
rows in the workspace, statistical thresholds) against the CPU oracle.

The oracle quantizes the same binary32 inputs with its own round-to-nearest-
even, works on the quantized values exactly in binary64, rounds its checksum
rows once to binary32 and its product to binary32.
 - quantized operands: bit-exact;
 - values: per element |C_gpu - C_oracle| <= k u32 (|A_q||B_q|)_ij + u32 |C_ij|
   (the binary32 accumulation bound; the product itself is exact);
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


def make(dev, orc, m, n, k, br, bc):
    A32 = synth.uniform(SEED, synth.STREAM_A, m, k, np.float32)
    B32 = synth.uniform(SEED, synth.STREAM_B, k, n, np.float32)
    P = abft.Protected(abft.ABFT_BF16, m, n, k, br, bc, device=dev, tau_mode=abft.ABFT_TAU_STAT, lam=LAMBDA)
    abft.quantize(P.p, 0, torch.from_numpy(A32).to(dev), P.A, P.ws)
    abft.quantize(P.p, 1, torch.from_numpy(np.ascontiguousarray(B32.T)).to(dev), P.Bt, P.ws)
    torch.cuda.synchronize()
    Aq = orc.to_bf16_bits(A32)
    Bq = orc.to_bf16_bits(B32)
    assert np.array_equal(P.A.cpu().view(torch.int16).numpy().view(np.uint16), Aq)
    assert np.array_equal(P.Bt.cpu().view(torch.int16).numpy().view(np.uint16), np.ascontiguousarray(Bq.T))
    A = orc.bf16_bits_to_f64(Aq)
    B = orc.bf16_bits_to_f64(Bq)
    Af, Bf = orc.encode(A, B, br, bc, store_f32=True)
    C64 = orc.gemm(Af, Bf)
    tc, tr = orc.tau_stat(Af, Bf, m, n, br, bc, u_acc=U32, T=float(k), s_store=2.0, lam=LAMBDA)
    return P, A, B, Af, Bf, C64.astype(np.float32), tc, tr


SHAPES = [
    (256, 256, 256, 1, 1),
    (512, 384, 1024, 1, 1),
    (200, 136, 72, 8, 4),
    (512, 512, 512, 32, 32),
    (1024, 1024, 4096, 1, 1),
    (300, 260, 520, 3, 5),
]


@pytest.mark.parametrize("m,n,k,br,bc", SHAPES)
def test_bf16_product_and_clean_verify(dev, orc, m, n, k, br, bc):
    note(f"bf16 m={m} n={n} k={k} br={br} bc={bc}")
    P, A, B, Af, Bf, C32, tc, tr = make(dev, orc, m, n, k, br, bc)
    P.encode()
    P.gemm()
    torch.cuda.synchronize()
    Cg = P.C.cpu().numpy().astype(np.float64)
    bound = k * U32 * (np.abs(Af) @ np.abs(Bf)) + U32 * np.abs(C32)
    assert np.all(np.abs(Cg - C32) <= bound * 1.01 + 1e-30)
    rep = P.verify()
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0, (rep.max_ratio_c, rep.max_ratio_r)
    note(f"  max |D|/tau {max(rep.max_ratio_c, rep.max_ratio_r):.4f}; "
         f"max rel err {np.abs(Cg - C32).max() / np.abs(C32).max():.2e}")
    # plain product = data part, bit for bit (same kernel, same k order)
    Cp = torch.zeros(m, n, dtype=torch.float32, device=dev)
    p2 = abft.problem(abft.ABFT_BF16, m, n, k, br, bc, ldc=n, tau_mode=abft.ABFT_TAU_STAT)
    abft.gemm(p2, P.A, P.Bt, Cp, flags=abft.ABFT_PLAIN)
    torch.cuda.synchronize()
    assert torch.equal(Cp, P.C[:m, :n])


@pytest.mark.parametrize("m,n,k,br,bc,runs", [(256, 256, 256, 1, 1, 60), (512, 512, 512, 32, 32, 40)])
def test_bf16_flip_decisions_match_oracle(dev, orc, m, n, k, br, bc, runs):
    P, A, B, Af, Bf, C32, tc, tr = make(dev, orc, m, n, k, br, bc)
    P.encode()
    P.gemm()
    clean = P.C.clone()
    M, N = m + br, n + bc
    located = compared = 0
    for run in range(runs):
        i, j, bit = synth.flip_site(SEED + 9, run, M, N, 11, 30)
        note(f"bf16 flip run={run} ({i},{j}) bit {bit}")
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
        _, _, orep = orc.verify(Cx.astype(np.float64), m, n, br, bc, tc, tr)
        ocls, oi, oj, od = orc.classify(orep, m, n, br, bc)
        assert (rep.n_flag_c, rep.n_flag_r) == (orep.n_flag_c, orep.n_flag_r), (i, j, bit, delta)
        assert (loc.cls, loc.i, loc.j) == (ocls, oi, oj)
        if loc.cls in (abft.ABFT_CLS_DATA, abft.ABFT_CLS_CHECKSUM):
            located += 1
            abft.correct(P.p, P.C, loc)
            rep2 = P.verify()
            assert rep2.n_flag_c == 0 and rep2.n_flag_r == 0
            assert abs(P.C[i, j].item() - clean[i, j].item()) <= min(t1, t2)
    note(f"  compared {compared}, located {located}")
    assert compared >= runs * 0.8 and located >= compared * 0.4


def test_bf16_erasure_rebuild(dev, orc):
    m = n = 512
    k, b = 256, 32
    P, A, B, Af, Bf, C32, tc, tr = make(dev, orc, m, n, k, b, b)
    P.encode()
    P.gemm()
    clean = P.C.clone()
    for rect in [(64, 128, 32, 32), (512, 0, 32, 32), (5, 3, 20, 30), (64, 512, 32, 32)]:
        for use_rows in (False, True):
            note(f"bf16 erase {rect} rows={use_rows}")
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
