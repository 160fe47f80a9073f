"""GPU parity of chained products (the previous product's C_f used as the
next A_f, its carried rows reused as checksum rows; Sec. 3.2 chained calls)
against the CPU oracle, binary64 and binary32.

 - the chained product equals the oracle's product of the GPU's C_f and the
   oracle-encoded next operand (1e-12) and verifies clean;
 - its thresholds (including the inherited term) equal the oracle's chained
   thresholds on the same operands (1e-10);
 - a flip in the chained result is located and corrected; a lost block is
   rebuilt.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_0806_3121_amd import abft, synth  # noqa: E402

pytestmark = pytest.mark.gpu

SEED = synth.BASE_SEED + 51


def note(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abft.lib()
    return torch.device("cuda:0")


def rel_err(x, ref):
    return np.abs(x - ref).max() / max(np.abs(ref).max(), 1e-300)


CASES = [
    (512, 256, 384, 320, 64, 64),    # block checksums on the matrix cores
    (400, 320, 256, 200, 1, 1),      # element checksums (streamed carried blocks), ragged tiles
    (256, 128, 256, 96, 8, 4),
]


@pytest.mark.parametrize("case", CASES, ids=["x".join(map(str, c)) for c in CASES])
def test_chained_product(dev, orc, case):
    m, k1, n1, n2, br, bc = case
    note(f"chained product {case}")
    A1 = synth.uniform(SEED, synth.STREAM_A, m, k1)
    B1 = synth.uniform(SEED, synth.STREAM_B, k1, n1)
    B2 = synth.uniform(SEED + 1, synth.STREAM_B, n1, n2)
    P1 = abft.Protected(abft.ABFT_F64, m, n1, k1, br, bc, device=dev)
    P1.A[:m] = torch.from_numpy(A1).to(dev)
    P1.Bt[:n1] = torch.from_numpy(np.ascontiguousarray(B1.T)).to(dev)
    P1.encode()
    P1.gemm()
    rep = P1.verify()
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0
    # the next product: A_f = the previous C_f (lda = its ldc), B_f = B2 with checksum columns
    N2 = n2 + bc
    ldc2 = (N2 + 1) // 2 * 2
    p2 = abft.problem(abft.ABFT_F64, m, n2, n1, br, bc, lda=P1.ldc, ldb=n1, ldc=ldc2)
    Bt2 = torch.zeros(N2, n1, dtype=torch.float64, device=dev)
    Bt2[:n2] = torch.from_numpy(np.ascontiguousarray(B2.T)).to(dev)
    ws2 = torch.zeros(abft.workspace_size(p2), dtype=torch.uint8, device=dev)
    D = torch.zeros(m + br, ldc2, dtype=torch.float64, device=dev)
    abft.encode_chained(p2, P1.Cbuf, Bt2, ws2, P1.p, P1.ws)
    abft.gemm(p2, P1.Cbuf, Bt2, D, ws2)
    host = abft.new_report_buffer()
    abft.verify(p2, D, ws2, host_out=host)
    torch.cuda.synchronize()
    rep = abft.read_report(host)
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0, (rep.max_ratio_c, rep.max_ratio_r)
    # oracle: the GPU's C_f (as the operand) times the oracle-encoded B2
    C1 = P1.C.cpu().numpy()
    Af2 = np.ascontiguousarray(C1[:, :n1])
    _, Bf2 = orc.encode(np.zeros((m, n1)), B2, br, bc)
    gB2 = Bt2.cpu().numpy().T
    H = n2 // bc
    mag = sum(np.abs(B2[:, h * bc:(h + 1) * bc]) for h in range(H))
    assert np.all(np.abs(gB2[:, n2:] - Bf2[:, n2:]) <= 2 * (H + 1) * 2.0 ** -53 * mag + 1e-300)
    Dg = D[:, :N2].cpu().numpy()
    assert rel_err(Dg, orc.gemm(Af2, gB2)) <= 1e-12
    # thresholds: the GPU's, read off flagged relations, against the oracle's chained ones
    Ap1 = P1.A.cpu().numpy()
    Bp1 = P1.Bt.cpu().numpy().T
    tc1, _ = orc.tau_det(Ap1, Bp1, m, n1, br, bc)
    tcc, trc = orc.tau_det_chained(Af2, gB2, m, n2, br, bc, tc1)
    i, j = m // 2 + 3, n2 // 3
    clean = D.clone()
    abft.inject_flip(p2, D, i, j, 57)
    abft.verify(p2, D, ws2, host_out=host)
    torch.cuda.synchronize()
    rep = abft.read_report(host)
    (r, jj, d, tau), = rep.flags_c()
    assert (r, jj) == (i % br, j)
    assert abs(tau - tcc[r, j]) <= 1e-10 * tcc[r, j]
    (ii, c, d, tau), = rep.flags_r()
    assert (ii, c) == (i, j % bc)
    assert abs(tau - trc[i, c]) <= 1e-10 * trc[i, c]
    loc = abft.classify(p2, rep)
    assert (loc.cls, loc.i, loc.j) == (abft.ABFT_CLS_DATA, i, j)
    abft.correct(p2, D, loc)
    # a lost block of the chained result
    h, w = min(br, 32), min(64, n2)
    rect = (br, 0, h, w) if br > 1 else (5, 0, 1, w)
    D[rect[0]:rect[0] + rect[2], rect[1]:rect[1] + rect[3]] = float("nan")
    abft.recover_block(p2, D, rect)
    abft.verify(p2, D, ws2, host_out=host)
    torch.cuda.synchronize()
    rep = abft.read_report(host)
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0
    assert rel_err(D[:, :N2].cpu().numpy(), clean[:, :N2].cpu().numpy()) <= 1e-12


def _raise_bit(v):
    """An exponent bit of binary32 v (26..30) whose flip multiplies |v| by 2^8 or
    more and stays finite (None for values in [1, 2))."""
    e = int(np.array([v], np.float32).view(np.uint32)[0] >> 23) & 0xFF
    for bit in (29, 28, 27, 26, 30):
        j = bit - 23
        if not (e >> j) & 1 and e + (1 << j) <= 254:
            return bit
    return None


CASES32 = [
    (512, 256, 384, 320, 64, 64),    # block checksums on the matrix cores
    (400, 320, 256, 200, 1, 1),      # element checksums (streamed carried blocks), ragged tiles
]


@pytest.mark.parametrize("case", CASES32, ids=["x".join(map(str, c)) for c in CASES32])
def test_chained_product_f32(dev, orc, case):
    """The chain in binary32 (det thresholds with the binary32 accumulation and
    storage roundoffs): the chained product within the binary32 accumulation
    bound of the oracle's product of the same operands, clean; the thresholds
    of a flipped relation equal the oracle's chained ones (1e-6); the flip is
    located and corrected; a lost block is rebuilt."""
    m, k1, n1, n2, br, bc = case
    u32 = 2.0 ** -24
    note(f"binary32 chained product {case}")
    A1 = synth.uniform(SEED, synth.STREAM_A, m, k1, np.float32)
    B1 = synth.uniform(SEED, synth.STREAM_B, k1, n1, np.float32)
    B2 = synth.uniform(SEED + 1, synth.STREAM_B, n1, n2, np.float32)
    P1 = abft.Protected(abft.ABFT_F32, m, n1, k1, br, bc, device=dev, tau_mode=abft.ABFT_TAU_DET)
    P1.A[:m] = torch.from_numpy(A1).to(dev)
    P1.Bt[:n1] = torch.from_numpy(np.ascontiguousarray(B1.T)).to(dev)
    P1.encode()
    P1.gemm()
    rep = P1.verify()
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0
    N2 = n2 + bc
    ldc2 = (N2 + 3) // 4 * 4
    p2 = abft.problem(abft.ABFT_F32, m, n2, n1, br, bc, lda=P1.ldc, ldb=n1, ldc=ldc2, tau_mode=abft.ABFT_TAU_DET)
    Bt2 = torch.zeros(N2, n1, dtype=torch.float32, device=dev)
    Bt2[:n2] = torch.from_numpy(np.ascontiguousarray(B2.T)).to(dev)
    ws2 = torch.zeros(abft.workspace_size(p2), dtype=torch.uint8, device=dev)
    D = torch.zeros(m + br, ldc2, dtype=torch.float32, device=dev)
    abft.encode_chained(p2, P1.Cbuf, Bt2, ws2, P1.p, P1.ws)
    abft.gemm(p2, P1.Cbuf, Bt2, D, ws2)
    host = abft.new_report_buffer()
    abft.verify(p2, D, ws2, host_out=host)
    torch.cuda.synchronize()
    rep = abft.read_report(host)
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0, (rep.max_ratio_c, rep.max_ratio_r)
    # oracle: the GPU's C_f (as the operand) times the oracle-encoded B2 (checksum columns rounded to binary32)
    C1 = P1.C.cpu().numpy().astype(np.float64)
    Af2 = np.ascontiguousarray(C1[:, :n1])
    _, Bf2 = orc.encode(np.zeros((m, n1)), B2.astype(np.float64), br, bc, store_f32=True)
    gB2 = Bt2.cpu().numpy().T.astype(np.float64)
    assert np.array_equal(gB2[:, :n2], B2.astype(np.float64))
    assert np.all(np.abs(gB2[:, n2:] - Bf2[:, n2:]) <= 2 * u32 * np.abs(Bf2[:, n2:]) + 1e-38)
    Dg = D[:, :N2].cpu().numpy().astype(np.float64)
    assert np.all(np.abs(Dg - orc.gemm(Af2, gB2)) <= (n1 + 2) * u32 * (np.abs(Af2) @ np.abs(gB2)))
    Ap1 = P1.A.cpu().numpy().astype(np.float64)
    Bp1 = P1.Bt.cpu().numpy().T.astype(np.float64)
    tc1, _ = orc.tau_det(Ap1, Bp1, m, n1, br, bc, u_acc=u32, u_st=u32)
    tcc, trc = orc.tau_det_chained(Af2, gB2, m, n2, br, bc, tc1, u_acc=u32, u_st=u32)
    i = m // 2 + 3
    j = next(jj for jj in range(n2 // 3, n2) if _raise_bit(Dg[i, jj]) is not None)
    clean = D.clone()
    abft.inject_flip(p2, D, i, j, _raise_bit(Dg[i, j]))
    abft.verify(p2, D, ws2, host_out=host)
    torch.cuda.synchronize()
    rep = abft.read_report(host)
    (r, jj, d, tau), = rep.flags_c()
    assert (r, jj) == (i % br, j)
    assert abs(tau - tcc[r, j]) <= 1e-6 * tcc[r, j]
    (ii, c, d, tau), = rep.flags_r()
    assert (ii, c) == (i, j % bc)
    assert abs(tau - trc[i, c]) <= 1e-6 * trc[i, c]
    loc = abft.classify(p2, rep)
    assert (loc.cls, loc.i, loc.j) == (abft.ABFT_CLS_DATA, i, j)
    abft.correct(p2, D, loc)
    h, w = min(br, 32), min(64, n2)
    rect = (br, 0, h, w) if br > 1 else (5, 0, 1, w)
    D[rect[0]:rect[0] + rect[2], rect[1]:rect[1] + rect[3]] = float("nan")
    abft.recover_block(p2, D, rect)
    abft.verify(p2, D, ws2, host_out=host)
    torch.cuda.synchronize()
    rep = abft.read_report(host)
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0
    scale = 4 * max(tcc.max(), trc.max())
    assert np.abs(D[:, :N2].cpu().numpy().astype(np.float64) - clean[:, :N2].cpu().numpy()).max() <= scale
