"""GPU parity of the weighted f-checksum path (Sec. 2.1 on the block product)
with binary32 operands and C_f, against the CPU oracle, through the C ABI.

The oracle encodes the same binary32 data in binary64 and rounds its checksum
rows once to binary32, multiplies its binary32 operands exactly (binary64),
and takes the binary32 thresholds (product accumulation and checksum-row
storage at 2^-24).  Values: data rows equal, checksum rows within one
binary32 rounding of the oracle's, C_f within the binary32 accumulation bound
(k + 2) 2^-24 |A_f||B_f|.  Decisions: on flips of high exponent bits (far
outside the gray zone) the failed groups, their thresholds (1e-6) and the
located elements equal the oracle's on its own product with the same flips;
corrections and rebuilt blocks restore C_f within the threshold scale.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import weighted as wo  # noqa: E402
from paper_0806_3121_amd import abft, synth  # noqa: E402

pytestmark = pytest.mark.gpu

SEED = synth.BASE_SEED + 50
U32 = 2.0 ** -24


def note(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abft.lib()
    return torch.device("cuda:0")


def weights(f, G, stream, lo=0.5, hi=1.5):
    return lo + (hi - lo) * (synth.uniform(SEED, stream, f, G) + 1) / 2


class Case:
    """A binary32 weighted product on the GPU and the oracle's binary32 encoding of the same data."""

    def __init__(self, dev, m, n, k, br, bc, fr, fc, A=None, B=None, Wr=None, Wc=None, tau_mode=abft.ABFT_TAU_DET):
        self.shape = (m, n, k, br, bc, fr, fc)
        if A is None:
            A = synth.uniform(SEED, synth.STREAM_A, m, k, np.float32)
            B = synth.uniform(SEED, synth.STREAM_B, k, n, np.float32)
        A, B = np.asarray(A, np.float32), np.asarray(B, np.float32)
        if Wr is None:
            Wr = weights(fr, m // br, synth.STREAM_X)
            Wc = weights(fc, n // bc, synth.STREAM_PICK)
        self.A, self.B, self.Wr, self.Wc = A, B, Wr, Wc
        P = abft.WProtected(m, n, k, br, bc, Wr, Wc, device=dev, tau_mode=tau_mode, dtype=abft.ABFT_F32)
        P.A[:m] = torch.from_numpy(A).to(dev)
        P.Bt[:n] = torch.from_numpy(np.ascontiguousarray(B.T)).to(dev)
        self.P = P
        # the oracle: binary64 weighted sums rounded once to binary32, the exact product of those operands
        Af, Bf = wo.wencode(A.astype(np.float64), B.astype(np.float64), Wr, Wc, br, bc)
        self.Af32, self.Bf32 = Af.astype(np.float32), Bf.astype(np.float32)
        self.Cref = self.Af32.astype(np.float64) @ self.Bf32.astype(np.float64)
        self.bound = (k + 2) * U32 * (np.abs(self.Af32).astype(np.float64) @ np.abs(self.Bf32).astype(np.float64))
        self.tc, self.tr = wo.wtau_det(self.Af32, self.Bf32, m, n, br, bc, Wr, Wc, u_acc=U32, u_st=U32)

    def run(self):
        self.P.encode()
        self.P.gemm()
        torch.cuda.synchronize()


SHAPES = [
    (512, 384, 256, 64, 64, 2, 2),      # MFMA-tiled checksum blocks
    (384, 256, 1000, 1, 1, 3, 2),       # element checksums: partitioned encode and verify
    (200, 136, 72, 8, 4, 4, 4),         # ragged tiles, f = ABFT_WMAX
    (256, 256, 128, 128, 128, 1, 1),    # one checksum each way, two blocks
]
IDS = ["x".join(map(str, s)) for s in SHAPES]


@pytest.mark.parametrize("shape", SHAPES, ids=IDS)
def test_f32_weighted_encode_product_and_clean_verify(dev, orc, shape):
    m, n, k, br, bc, fr, fc = shape
    note(f"binary32 weighted encode+gemm {shape}")
    c = Case(dev, *shape)
    c.run()
    gA = c.P.A.cpu().numpy()
    gB = c.P.Bt.cpu().numpy().T
    assert np.array_equal(gA[:m], c.A) and np.array_equal(gB[:, :n], c.B)
    # checksum rows: the binary64 sums may differ in their last bits (fused or separate multiply-add),
    # so the rounded values agree to one binary32 rounding
    for got, ref in ((gA[m:], c.Af32[m:]), (gB[:, n:], c.Bf32[:, n:])):
        assert np.all(np.abs(got.astype(np.float64) - ref) <= 2 * U32 * np.abs(ref) + 1e-38)
    Cg = c.P.C.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(Cg - c.Cref) <= c.bound), np.abs(Cg - c.Cref).max()
    rep = c.P.verify()
    assert rep.n_fail_c == 0 and rep.n_fail_r == 0
    assert 0 < max(rep.max_ratio_c, rep.max_ratio_r) < 0.5
    note(f"  max |D|/tau: col {rep.max_ratio_c:.2e} row {rep.max_ratio_r:.2e}")
    o = wo.wverify(c.Cref.astype(np.float32), m, n, br, bc, c.Wr, c.Wc, c.tc, c.tr)
    assert o["col"] == [] and o["row"] == []


def _flip32(x, bit):
    return (np.array([x], np.float32).view(np.uint32) ^ np.uint32(1 << bit)).view(np.float32)[0]


def _up_bit(v):
    """An exponent bit (of bits 26..30) whose flip multiplies |v| by 2^8 or more
    and stays finite: a binary32 flip must outweigh thresholds of a few 2^-24
    times the operand norms, and the location fits the residuals to a weight
    column within them."""
    e = int(np.array([v], np.float32).view(np.uint32)[0] >> 23) & 0xFF
    for bit in (29, 28, 27, 26, 30):
        j = bit - 23
        if not (e >> j) & 1 and e + (1 << j) <= 254:
            return bit
    return None                          # [1, 2): only the top exponent bit is clear, and it overflows


def _site(Co, x, y):
    """(x, y', bit): the first column y' >= y of row x whose oracle value has a raising bit."""
    for yy in range(y, Co.shape[1]):
        bit = _up_bit(Co[x, yy])
        if bit is not None:
            return x, yy, bit
    raise AssertionError(f"no raisable entry in row {x} from column {y}")


@pytest.mark.parametrize("shape", SHAPES[:3], ids=IDS[:3])
def test_f32_weighted_flips_located_corrected_with_oracle_thresholds(dev, orc, shape):
    """Flips of high exponent bits in several groups at once (data, carried
    rows, carried columns, corner): the GPU's failed groups, their thresholds
    and the located elements equal the oracle's on its own binary32 product
    with the same flips; the correction restores C_f."""
    m, n, k, br, bc, fr, fc = shape
    c = Case(dev, *shape)
    c.run()
    clean = c.P.C.cpu().numpy().copy()
    M, N = clean.shape[0], c.P.N
    Co = c.Cref.astype(np.float32)
    cells = [(3, 5), (m + 1, 7), (br + 2, n + 1), (M - 1, N - 1)]
    if br == 1:                          # distinct column groups need distinct (row residue, column) pairs
        cells = [(3, 5), (m, 7), (10, n), (M - 1, N - 1)]
    sites = [_site(Co, x, y) for (x, y) in cells]               # chosen from the oracle's values
    note(f"binary32 weighted flips {shape} at {sites}")
    for (x, y, bit) in sites:
        c.P.C[x, y] = float(_flip32(c.P.C[x, y].item(), bit))
        Co[x, y] = _flip32(Co[x, y], bit)
    rep = c.P.verify()
    orep = wo.wverify(Co.astype(np.float64), m, n, br, bc, c.Wr, c.Wc, c.tc, c.tr)
    gpu_groups = rep.groups_c(fr) if fr >= 2 else rep.groups_r(fc)
    ora_groups = orep["col"] if fr >= 2 else orep["row"]
    assert [(g[0], g[1]) for g in gpu_groups] == [(g[0], g[1]) for g in ora_groups]
    for g, o in zip(gpu_groups, ora_groups):
        assert np.allclose(g[3], o[3], rtol=1e-6, atol=0)
    st, locs = abft.wlocate(c.P.p, rep)
    want = wo.wlocate(orep["col"], orep["row"], m, n, br, bc, c.Wr, c.Wc)
    assert st == abft.ABFT_OK
    assert [(l.cls, l.i, l.j) for l in locs] == [(w[0], w[2], w[3]) for w in want]
    assert sorted((l.i, l.j) for l in locs) == sorted((x, y) for (x, y, _) in sites)
    abft.wcorrect(c.P.p, c.P.C, locs, c.P.ws)
    rep = c.P.verify()
    assert rep.n_fail_c == 0 and rep.n_fail_r == 0
    torch.cuda.synchronize()
    got = c.P.C.cpu().numpy()
    for (x, y, _) in sites:
        assert abs(float(got[x, y]) - float(clean[x, y])) <= 4 * max(c.tc.max(), c.tr.max())


ERASE = [
    (SHAPES[0], abft.ABFT_DIR_COL, [1, 6], None),          # two data block rows
    (SHAPES[0], abft.ABFT_DIR_ROW, [2, 5], None),          # two data block columns
    (SHAPES[2], abft.ABFT_DIR_COL, [3, 7, 11, 20], None),  # four of 25 block rows, f = 4
    (SHAPES[1], abft.ABFT_DIR_COL, [5, 17, 300], None),    # element checksums: three lost rows, f = 3
]


@pytest.mark.parametrize("case", ERASE, ids=[f"{'col' if e[1] == 0 else 'row'}-{e[2]}" for e in ERASE])
def test_f32_weighted_lost_blocks_rebuilt(dev, orc, case):
    """Lost blocks rebuilt by the f x f solve (binary64, stored rounded once):
    within the relations' rounding amplified by the system's condition
    number of the clean values, and the verification is clean again."""
    shape, direction, lost, rng = case
    m, n, k, br, bc, fr, fc = shape
    note(f"binary32 weighted erasure {shape} dir={direction} lost={lost}")
    c = Case(dev, *shape)
    c.run()
    clean = c.P.C.cpu().numpy().astype(np.float64).copy()
    M, N = clean.shape[0], c.P.N
    b = br if direction == abft.ABFT_DIR_COL else bc
    lines = N if direction == abft.ABFT_DIR_COL else M
    lo, length = rng if rng else (0, lines)
    for g in lost:
        if direction == abft.ABFT_DIR_COL:
            c.P.C[g * b:(g + 1) * b, lo:lo + length] = float("nan")
        else:
            c.P.C[lo:lo + length, g * b:(g + 1) * b] = float("nan")
    abft.wrecover(c.P.p, c.P.C, direction, lost, lo, length, c.P.ws)
    torch.cuda.synchronize()
    got = c.P.C.cpu().numpy().astype(np.float64)
    assert np.all(np.isfinite(got[:, :N]))
    W = c.Wr if direction == abft.ABFT_DIR_COL else c.Wc
    f, G = W.shape
    U = [g for g in lost if g < G]
    R = [r for r in range(f) if G + r not in lost][:len(U)]
    cond = np.linalg.cond(W[np.ix_(R, U)], 1) if U else 1.0
    tau = max(c.tc.max(), c.tr.max())
    note(f"  condition number {cond:.1f}, threshold scale {tau:.1e}")
    assert np.abs(got[:, :N] - clean[:, :N]).max() <= 4 * cond * tau
    rep = c.P.verify()
    assert rep.n_fail_c == 0 and rep.n_fail_r == 0


def test_f32_weighted_exact_integers(dev, orc):
    """Integer data and power-of-two Vandermonde weights small enough that
    every product and relation is exact in binary32: every relation holds
    exactly on the GPU (tau = 0), a flip is located, and two lost block rows
    are rebuilt bit for bit (the 2 x 2 inverse is exact)."""
    m, n, k, br, bc, fr, fc = 128, 128, 64, 32, 32, 2, 2
    A = synth.uniform_ints(SEED, synth.STREAM_A, m, k, -8, 8)
    B = synth.uniform_ints(SEED, synth.STREAM_B, k, n, -8, 8)
    Wr = wo.vandermonde(fr, m // br, nodes=2.0 ** np.arange(m // br))
    Wc = wo.vandermonde(fc, n // bc, nodes=2.0 ** np.arange(n // bc))
    note("binary32 weighted exact integers")
    c = Case(dev, m, n, k, br, bc, fr, fc, A=A, B=B, Wr=Wr, Wc=Wc, tau_mode=abft.ABFT_TAU_EXACT)
    c.run()
    assert np.abs(c.Cref).max() < 2.0 ** 24                      # every entry exact in binary32
    assert np.array_equal(c.P.C.cpu().numpy().astype(np.float64), c.Cref)
    rep = c.P.verify()
    assert rep.n_fail_c == 0 and rep.n_fail_r == 0
    c.P.C[40, 50] += 1.0
    st, locs = abft.wlocate(c.P.p, c.P.verify())
    assert st == abft.ABFT_OK and [(l.cls, l.i, l.j) for l in locs] == [(abft.ABFT_CLS_DATA, 40, 50)]
    abft.wcorrect(c.P.p, c.P.C, locs, c.P.ws)
    c.P.C[64:128, :] = float("nan")
    abft.wrecover(c.P.p, c.P.C, abft.ABFT_DIR_COL, [2, 3], 0, c.P.N, c.P.ws)
    torch.cuda.synchronize()
    assert np.array_equal(c.P.C.cpu().numpy()[:, :c.P.N].astype(np.float64), c.Cref)


def test_f32_weighted_matrix_vector_product(dev, orc):
    """The binary32 protected matrix-vector product (n = 1, bc = 1, fc = 1) on
    the streaming kernel (binary64 accumulation): within the bound of the
    oracle's, clean, and a flip of y located and corrected."""
    m, n, k, br, bc, fr, fc = 4096, 1, 2048, 64, 1, 2, 1
    note("binary32 weighted matrix-vector product")
    c = Case(dev, m, n, k, br, bc, fr, fc)
    c.run()
    Cg = c.P.C.cpu().numpy()[:, :c.P.N].astype(np.float64)
    assert np.all(np.abs(Cg - c.Cref) <= c.bound)
    rep = c.P.verify()
    assert rep.n_fail_c == 0 and rep.n_fail_r == 0
    clean = Cg.copy()
    x = next(i for i in range(5, m) if _up_bit(np.float32(c.Cref[i, 0])) is not None)
    c.P.C[x, 0] = float(_flip32(c.P.C[x, 0].item(), _up_bit(np.float32(c.Cref[x, 0]))))
    st, locs = abft.wlocate(c.P.p, c.P.verify())
    assert st == abft.ABFT_OK and [(l.cls, l.i, l.j) for l in locs] == [(abft.ABFT_CLS_DATA, x, 0)]
    abft.wcorrect(c.P.p, c.P.C, locs, c.P.ws)
    torch.cuda.synchronize()
    assert abs(c.P.C[x, 0].item() - clean[x, 0]) <= 4 * max(c.tc.max(), c.tr.max())
