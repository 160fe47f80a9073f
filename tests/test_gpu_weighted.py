"""GPU parity of the weighted f-checksum path (Sec. 2.1 on the block product)
against the CPU oracle, through the C ABI.

Values: checksum rows/columns within the rounding of their weighted sums;
C_f within 1e-12 of the oracle's (relative to its largest entry); thresholds
within 1e-10 of the oracle's.  Decisions: every injected error located at the
oracle's element with the oracle's class; rebuilt blocks equal to the
oracle's rebuild of the same damaged C_f within the rounding of the relation
sums times the condition number of the solved system (1e-12 at least).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import weighted as wo  # noqa: E402
from paper_0806_3121_amd import abft, synth  # noqa: E402

pytestmark = pytest.mark.gpu

SEED = synth.BASE_SEED
TOL = 1e-12


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


def make(dev, m, n, k, br, bc, fr, fc, A=None, B=None, Wr=None, Wc=None, tau_mode=abft.ABFT_TAU_DET):
    if A is None:
        A = synth.uniform(SEED, synth.STREAM_A, m, k)
        B = synth.uniform(SEED, synth.STREAM_B, k, n)
    if Wr is None:
        Wr = weights(fr, m // br, synth.STREAM_X)
        Wc = weights(fc, n // bc, synth.STREAM_PICK)
    P = abft.WProtected(m, n, k, br, bc, Wr, Wc, device=dev, tau_mode=tau_mode)
    P.A[:m] = torch.from_numpy(A).to(dev)
    P.Bt[:n] = torch.from_numpy(np.ascontiguousarray(B.T)).to(dev)
    return A, B, Wr, Wc, P


def rel_err(x, ref):
    return np.abs(x - ref).max() / max(np.abs(ref).max(), 1e-300)


def flip(P, x, y, bit):
    v = P.C[x, y].clone().view(torch.int64) ^ (1 << bit)
    P.C[x, y] = v.view(torch.float64)


SHAPES = [
    (512, 384, 256, 64, 64, 2, 2),      # MFMA-tiled checksum blocks
    (384, 256, 1000, 1, 1, 3, 2),       # element checksums: partitioned encode and verify, K tail
    (200, 136, 72, 8, 4, 4, 4),         # ragged tiles, f = ABFT_WMAX
    (256, 256, 128, 128, 128, 1, 1),    # one checksum each way, two blocks
]
IDS = ["x".join(map(str, s)) for s in SHAPES]


@pytest.mark.parametrize("shape", SHAPES, ids=IDS)
def test_weighted_encode_product_and_clean_verify(dev, orc, shape):
    m, n, k, br, bc, fr, fc = shape
    note(f"weighted encode+gemm {shape}")
    A, B, Wr, Wc, P = make(dev, *shape)
    P.encode()
    P.gemm()
    torch.cuda.synchronize()
    Af, Bf, Cf = wo.wproduct(A, B, Wr, Wc, br, bc)
    gA = P.A.cpu().numpy()
    gB = P.Bt.cpu().numpy().T
    G = m // br
    for r in range(fr):
        mag = sum(abs(Wr[r, g]) * np.abs(A[g * br:(g + 1) * br]) for g in range(G))
        assert np.all(np.abs(gA[m + r * br:m + (r + 1) * br] - Af[m + r * br:m + (r + 1) * br])
                      <= 2 * (G + 1) * 2.0 ** -53 * mag + 1e-300)
    H = n // bc
    for c in range(fc):
        mag = sum(abs(Wc[c, h]) * np.abs(B[:, h * bc:(h + 1) * bc]) for h in range(H))
        assert np.all(np.abs(gB[:, n + c * bc:n + (c + 1) * bc] - Bf[:, n + c * bc:n + (c + 1) * bc])
                      <= 2 * (H + 1) * 2.0 ** -53 * mag + 1e-300)
    assert np.array_equal(gA[:m], A) and np.array_equal(gB[:, :n], B)
    Cg = P.C.cpu().numpy()
    assert rel_err(Cg, Cf) <= TOL
    rep = P.verify()
    assert rep.n_fail_c == 0 and rep.n_fail_r == 0
    assert 0 < max(rep.max_ratio_c, rep.max_ratio_r) < 0.5
    note(f"  max |D|/tau: col {rep.max_ratio_c:.2e} row {rep.max_ratio_r:.2e}")
    # the oracle on its own product, and on the GPU's, is clean too
    tc, tr = wo.wtau_det(Af, Bf, m, n, br, bc, Wr, Wc)
    for C in (Cf, Cg):
        o = wo.wverify(C, m, n, br, bc, Wr, Wc, tc, tr)
        assert o["col"] == [] and o["row"] == []


@pytest.mark.parametrize("shape", SHAPES[:3], ids=IDS[:3])
def test_weighted_flips_located_corrected_with_oracle_thresholds(dev, orc, shape):
    """One flip per group in several groups at once (data, carried rows,
    carried columns, corner): located from the weight ratios, the GPU group
    residuals and thresholds equal the oracle's on the same damaged C_f, and
    the correction restores C_f."""
    m, n, k, br, bc, fr, fc = shape
    A, B, Wr, Wc, P = make(dev, *shape)
    P.encode()
    P.gemm()
    torch.cuda.synchronize()
    clean = P.C.cpu().numpy().copy()
    M, N = clean.shape
    Af, Bf = P.A.cpu().numpy(), P.Bt.cpu().numpy().T
    tc, tr = wo.wtau_det(Af, Bf, m, n, br, bc, Wr, Wc)
    sites = [(3, 5, 55), (m + 1, 7, 52), (br + 2, n + 1, 60), (M - 1, N - 1, 50)]
    if br == 1:                          # distinct column groups need distinct (row residue, column) pairs
        sites = [(3, 5, 55), (m, 7, 52), (10, n, 60), (M - 1, N - 1, 50)]
    note(f"weighted flips {shape} at {sites}")
    for (x, y, bit) in sites:
        flip(P, x, y, bit)
    rep = P.verify()
    Cx = P.C.cpu().numpy()
    orep = wo.wverify(Cx, m, n, br, bc, Wr, Wc, tc, tr)
    # same failed groups, residuals and thresholds as the oracle on the same damaged C_f
    gpu_groups = rep.groups_c(fr) if fr >= 2 else rep.groups_r(fc)
    ora_groups = orep["col"] if fr >= 2 else orep["row"]
    assert [(g[0], g[1]) for g in gpu_groups] == [(g[0], g[1]) for g in ora_groups]
    for g, o in zip(gpu_groups, ora_groups):
        # failed relations: the same residual; clean relations of a failed group: both within tau
        assert np.allclose(g[2], o[2], rtol=1e-10, atol=2 * max(o[3]))
        assert np.allclose(g[3], o[3], rtol=1e-10, atol=0)
    st, locs = abft.wlocate(P.p, rep)
    want = wo.wlocate(orep["col"], orep["row"], m, n, br, bc, Wr, Wc)
    assert st == abft.ABFT_OK
    assert [(l.cls, l.i, l.j) for l in locs] == [(w[0], w[2], w[3]) for w in want]
    assert sorted((l.i, l.j) for l in locs) == sorted((x, y) for (x, y, _) in sites)
    abft.wcorrect(P.p, P.C, locs, P.ws)
    rep = P.verify()
    assert rep.n_fail_c == 0 and rep.n_fail_r == 0
    torch.cuda.synchronize()
    assert rel_err(P.C.cpu().numpy(), clean) <= TOL


def test_weighted_single_checksums_intersection(dev, orc):
    shape = SHAPES[3]
    m, n, k, br, bc, fr, fc = shape
    A, B, Wr, Wc, P = make(dev, *shape)
    P.encode()
    P.gemm()
    torch.cuda.synchronize()
    clean = P.C.cpu().numpy().copy()
    note("weighted f = 1 intersection")
    flip(P, 77, 201, 54)
    rep = P.verify()
    st, locs = abft.wlocate(P.p, rep)
    assert st == abft.ABFT_OK and [(l.cls, l.i, l.j) for l in locs] == [(abft.ABFT_CLS_DATA, 77, 201)]
    abft.wcorrect(P.p, P.C, locs, P.ws)
    torch.cuda.synchronize()
    assert rel_err(P.C.cpu().numpy(), clean) <= TOL
    flip(P, 1, 2, 56)
    flip(P, 3, 4, 56)
    st, locs = abft.wlocate(P.p, P.verify())
    assert st == abft.ABFT_E_UNCORRECTABLE
    with pytest.raises(abft.AbftError):
        abft.wcorrect(P.p, P.C, locs, P.ws)


ERASE = [
    # shape, direction, lost blocks, line range (lo, len) or None for all
    (SHAPES[0], abft.ABFT_DIR_COL, [1, 6], None),          # two data block rows (the paper's f failures)
    (SHAPES[0], abft.ABFT_DIR_COL, [0, 8], (64, 128)),     # a data block row and checksum block row 0
    (SHAPES[0], abft.ABFT_DIR_ROW, [2, 5], None),          # two data block columns
    (SHAPES[2], abft.ABFT_DIR_COL, [3, 7, 11, 20], None),  # four of 25 block rows, f = 4
    (SHAPES[2], abft.ABFT_DIR_ROW, [0, 33, 34, 36], (10, 50)),
    (SHAPES[1], abft.ABFT_DIR_COL, [5, 17, 300], None),    # element checksums: three lost rows, f = 3
]


@pytest.mark.parametrize("case", ERASE, ids=[f"{'col' if c[1] == 0 else 'row'}-{c[2]}" for c in ERASE])
def test_weighted_lost_blocks_rebuilt(dev, orc, case):
    shape, direction, lost, rng = case
    m, n, k, br, bc, fr, fc = shape
    note(f"weighted erasure {shape} dir={direction} lost={lost} lines={rng}")
    A, B, Wr, Wc, P = make(dev, *shape)
    P.encode()
    P.gemm()
    torch.cuda.synchronize()
    clean = P.C.cpu().numpy().copy()
    M, N = clean.shape
    b = br if direction == abft.ABFT_DIR_COL else bc
    lines = N if direction == abft.ABFT_DIR_COL else M
    lo, length = rng if rng else (0, lines)
    rects = []
    for g in lost:
        if direction == abft.ABFT_DIR_COL:
            rects.append((g * b, lo, b, length))
        else:
            rects.append((lo, g * b, length, b))
    for (i0, j0, h, w) in rects:
        P.C[i0:i0 + h, j0:j0 + w] = float("nan")
    if len(rects) <= 4:
        rep = P.verify(known=rects)
        assert rep.n_fail_c == 0 and rep.n_fail_r == 0
        ec, er = wo.erased_groups(M, N, br, bc, rects)
        assert (rep.n_excl_c, rep.n_excl_r) == (int(ec.sum()), int(er.sum()))
    damaged = P.C.cpu().numpy().copy()
    abft.wrecover(P.p, P.C, direction, lost, lo, length, P.ws)
    torch.cuda.synchronize()
    got = P.C.cpu().numpy()
    Co = damaged.copy()
    assert wo.wrecover(Co, m, n, br, bc, Wr, Wc, direction, lost, lo, length) == 0
    # rounding amplified by the 1-norm condition number of the solved system
    W = Wr if direction == abft.ABFT_DIR_COL else Wc
    f, G = W.shape
    U = [g for g in lost if g < G]
    R = [r for r in range(f) if G + r not in lost][:len(U)]
    cond = np.linalg.cond(W[np.ix_(R, U)], 1) if U else 1.0
    tol = max(1e-12, 4 * (G + 2) * 2.0 ** -53 * cond * np.abs(W).max() / np.abs(W).min())
    note(f"  condition number {cond:.1f}, tolerance {tol:.1e}")
    scale = np.abs(clean).max()
    assert np.abs(got - Co).max() / scale <= tol
    assert np.abs(got - clean).max() / scale <= tol
    rep = P.verify()
    assert rep.n_fail_c == 0 and rep.n_fail_r == 0


def test_weighted_too_many_lost_refused(dev):
    A, B, Wr, Wc, P = make(dev, *SHAPES[0])
    note("weighted refusal")
    with pytest.raises(abft.AbftError) as e:
        abft.wrecover(P.p, P.C, abft.ABFT_DIR_COL, [0, 1, 2], 0, 10, P.ws)
    assert e.value.status == abft.ABFT_E_UNRECOVERABLE


def test_weighted_exact_integers(dev, orc):
    """Integer data and integer (Vandermonde) weights: every relation holds
    exactly on the GPU (tau = 0), any flip is located, two lost block rows are
    rebuilt bit for bit."""
    m, n, k, br, bc, fr, fc = 256, 192, 64, 32, 32, 2, 2
    A = synth.uniform_ints(SEED, synth.STREAM_A, m, k, -8, 8)
    B = synth.uniform_ints(SEED, synth.STREAM_B, k, n, -8, 8)
    # power-of-two nodes: the host's inverse of every 2 x 2 system is exact
    Wr = wo.vandermonde(fr, m // br, nodes=2.0 ** np.arange(m // br))
    Wc = wo.vandermonde(fc, n // bc, nodes=2.0 ** np.arange(n // bc))
    note("weighted exact integers")
    _, _, _, _, P = make(dev, m, n, k, br, bc, fr, fc, A=A, B=B, Wr=Wr, Wc=Wc, tau_mode=abft.ABFT_TAU_EXACT)
    P.encode()
    P.gemm()
    torch.cuda.synchronize()
    Af, Bf, Cf = wo.wproduct(A, B, Wr, Wc, br, bc)
    assert np.array_equal(P.C.cpu().numpy(), Cf)
    rep = P.verify()
    assert rep.n_fail_c == 0 and rep.n_fail_r == 0
    P.C[40, 50] += 1.0
    st, locs = abft.wlocate(P.p, P.verify())
    assert st == abft.ABFT_OK and [(l.cls, l.i, l.j) for l in locs] == [(abft.ABFT_CLS_DATA, 40, 50)]
    abft.wcorrect(P.p, P.C, locs, P.ws)
    P.C[64:128, :] = float("nan")
    abft.wrecover(P.p, P.C, abft.ABFT_DIR_COL, [2, 3], 0, P.N, P.ws)
    torch.cuda.synchronize()
    assert np.array_equal(P.C.cpu().numpy(), Cf)


def test_weighted_deterministic(dev):
    A, B, Wr, Wc, P = make(dev, *SHAPES[1])
    note("weighted determinism")
    out = []
    for _ in range(2):
        P.encode()
        P.gemm()
        rep = P.verify()
        out.append((P.A.cpu().numpy().tobytes(), P.C.cpu().numpy().tobytes(), rep.max_ratio_c, rep.max_ratio_r))
    assert out[0] == out[1]


def test_weighted_matrix_vector_product_many_rows(dev, orc):
    """The matrix-vector product at the bench's row count (16384 data rows, two
    weighted checksum block rows of 512): equal to the oracle's encoded
    product; clean verification; one flip located and corrected."""
    m, n, k, br, bc, fr, fc = 16384, 1, 1024, 512, 1, 2, 1
    note("weighted matrix-vector product, 16384 rows")
    A, B, Wr, Wc, P = make(dev, m, n, k, br, bc, fr, fc)
    P.encode()
    P.gemm()
    torch.cuda.synchronize()
    Af, Bf, Cf = wo.wproduct(A, B, Wr, Wc, br, bc)
    clean = P.C.cpu().numpy().copy()
    assert clean.shape == (m + fr * br, 2)
    assert rel_err(clean, Cf) <= TOL
    rep = P.verify()
    assert rep.n_fail_c == 0 and rep.n_fail_r == 0
    flip(P, 12345, 0, 57)
    rep = P.verify()
    st, locs = abft.wlocate(P.p, rep)
    assert st == abft.ABFT_OK
    assert [(l.cls, l.i, l.j) for l in locs] == [(abft.ABFT_CLS_DATA, 12345, 0)]
    abft.wcorrect(P.p, P.C, locs, P.ws)
    rep = P.verify()
    assert rep.n_fail_c == 0 and rep.n_fail_r == 0
    torch.cuda.synchronize()
    assert rel_err(P.C.cpu().numpy(), clean) <= 1e-11


def test_weighted_matrix_vector_product(dev, orc):
    """The protected matrix-vector product (n = 1, bc = 1, fc = 1): y_f = A_f x
    on the streaming kernel, equal to the oracle's encoded product; two flips of
    y in distinct row residues located by the weight ratios and corrected; two
    lost blocks of y rebuilt."""
    m, n, k, br, bc, fr, fc = 4096, 1, 2048, 64, 1, 2, 1
    note("weighted matrix-vector product")
    A, B, Wr, Wc, P = make(dev, m, n, k, br, bc, fr, fc)
    P.encode()
    P.gemm()
    torch.cuda.synchronize()
    Af, Bf, Cf = wo.wproduct(A, B, Wr, Wc, br, bc)
    clean = P.C.cpu().numpy().copy()
    assert clean.shape == (m + fr * br, 2)
    assert rel_err(clean, Cf) <= TOL
    rep = P.verify()
    assert rep.n_fail_c == 0 and rep.n_fail_r == 0
    for (x, bit) in [(5, 57), (3 * br + 17, 54)]:
        flip(P, x, 0, bit)
    rep = P.verify()
    st, locs = abft.wlocate(P.p, rep)
    assert st == abft.ABFT_OK
    assert sorted((l.cls, l.i, l.j) for l in locs) == [(abft.ABFT_CLS_DATA, 5, 0), (abft.ABFT_CLS_DATA, 3 * br + 17, 0)]
    abft.wcorrect(P.p, P.C, locs, P.ws)
    P.C[7 * br:8 * br, :] = float("nan")
    P.C[40 * br:41 * br, :] = float("nan")
    abft.wrecover(P.p, P.C, abft.ABFT_DIR_COL, [7, 40], 0, P.N, P.ws)
    rep = P.verify()
    assert rep.n_fail_c == 0 and rep.n_fail_r == 0
    torch.cuda.synchronize()
    assert rel_err(P.C.cpu().numpy(), clean) <= 1e-11
