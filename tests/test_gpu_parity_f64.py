"""GPU parity of the binary64 path against the CPU oracle, through the C ABI.

Values: max|C_gpu - C_oracle| / max|C_oracle| <= 1e-12 (binary64).
Decisions and indices: bit-exact, except where the oracle's |delta| lies in
the gray zone tau/2 < |delta| < 2 tau (reported, not compared).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_0806_3121_amd import abft, synth  # noqa: E402

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
SEED = synth.BASE_SEED


def note(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abft.lib()
    return torch.device("cuda:0")


def make(dev, m, n, k, br, bc, seed=SEED, tau_mode=None):
    A = synth.uniform(seed, synth.STREAM_A, m, k)
    B = synth.uniform(seed, synth.STREAM_B, k, n)
    P = abft.Protected(abft.ABFT_F64, m, n, k, br, bc, device=dev, tau_mode=tau_mode)
    P.A[:m] = torch.from_numpy(A).to(dev)
    P.Bt[:n] = torch.from_numpy(np.ascontiguousarray(B.T)).to(dev)
    return A, B, P


def rel_err(x, ref):
    return np.abs(x - ref).max() / max(np.abs(ref).max(), 1e-300)


SHAPES = [
    (256, 256, 256, 1, 1),      # C1 flip encoding
    (256, 256, 256, 64, 64),    # C1 erasure encoding (paper's block size 64)
    (200, 136, 72, 8, 4),       # ragged: no dimension a multiple of the tile; partial K slab
    (1024, 512, 384, 128, 1),   # asymmetric blocks
    (64, 64, 16, 64, 64),       # one group (G = 1)
    (384, 640, 1000, 3, 5),     # odd block sizes, K tail
    (130, 34, 2, 2, 2),         # tiny K
    (1536, 1024, 64, 512, 512), # wide blocks, few groups: one-pass verify of both directions
]


@pytest.mark.parametrize("m,n,k,br,bc", SHAPES)
def test_encode_and_product_match_oracle(dev, orc, m, n, k, br, bc):
    note(f"encode+gemm f64 m={m} n={n} k={k} br={br} bc={bc}")
    A, B, P = make(dev, m, n, k, br, bc)
    P.encode()
    P.gemm()
    torch.cuda.synchronize()
    Af, Bf, Cf = orc.protected_product(A, B, br, bc)
    gA = P.A.cpu().numpy()
    gB = P.Bt.cpu().numpy().T
    # checksum rows/columns: sums in another order, within gamma_G * sum|.|
    G = m // br
    absA = sum(np.abs(A[g * br:(g + 1) * br]) for g in range(G))
    assert np.all(np.abs(gA[m:] - Af[m:]) <= 2 * G * 2.0 ** -53 * absA + 1e-300)
    absB = sum(np.abs(B[:, h * bc:(h + 1) * bc]) for h in range(n // bc))
    assert np.all(np.abs(gB[:, n:] - Bf[:, n:]) <= 2 * (n // bc) * 2.0 ** -53 * absB + 1e-300)
    assert np.array_equal(gA[:m], A) and np.array_equal(gB[:, :n], B)
    Cg = P.C.cpu().numpy()
    assert rel_err(Cg, Cf) <= TOL64
    rep = P.verify()
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0
    assert rep.max_ratio_c < 0.5 and rep.max_ratio_r < 0.5
    # the oracle, on its own product, is clean too
    tc, tr = orc.tau_det(Af, Bf, m, n, br, bc)
    _, _, orep = orc.verify(Cf, m, n, br, bc, tc, tr)
    assert orep.n_flag_c == 0 and orep.n_flag_r == 0


def test_plain_product_is_data_part_bitwise(dev):
    note("plain vs protected data part")
    m, n, k = 300, 260, 520
    A, B, P = make(dev, m, n, k, 4, 4)
    P.encode()
    P.gemm()
    Cp = torch.zeros(m, n, dtype=torch.float64, device=dev)
    p2 = abft.problem(abft.ABFT_F64, m, n, k, 4, 4, ldc=n)
    abft.gemm(p2, P.A, P.Bt, Cp, flags=abft.ABFT_PLAIN)
    torch.cuda.synchronize()
    assert torch.equal(Cp, P.C[:m, :n])


def test_deterministic(dev):
    note("determinism")
    A, B, P = make(dev, 512, 384, 256, 1, 1)
    P.encode()
    P.gemm()
    c1 = P.C.clone()
    r1 = P.verify()
    P.encode()
    P.gemm()
    r2 = P.verify()
    assert torch.equal(c1, P.C)
    assert (r1.max_ratio_c, r1.max_ratio_r) == (r2.max_ratio_c, r2.max_ratio_r)


@pytest.mark.parametrize("dtype,transpose", [(abft.ABFT_F64, 0), (abft.ABFT_F64, 1), (abft.ABFT_F32, 0)])
def test_fill_uniform_matches_host_generator(dev, dtype, transpose):
    note(f"fill dtype={dtype} transpose={transpose}")
    rows, cols = 123, 77
    tdt = torch.float64 if dtype == abft.ABFT_F64 else torch.float32
    ndt = np.float64 if dtype == abft.ABFT_F64 else np.float32
    ld = 80 if not transpose else 128
    buf = torch.zeros((cols, ld) if transpose else (rows, ld), dtype=tdt, device=dev)
    abft.fill_uniform(dtype, rows, cols, ld, transpose, 99, 1, buf)
    torch.cuda.synchronize()
    host = synth.uniform(99, 1, rows, cols, ndt)
    got = buf.cpu().numpy()
    got = got[:, :rows].T if transpose else got[:, :cols]
    assert np.array_equal(got, host)


def _oracle_decision(orc, Cf, m, n, br, bc, tc, tr, i, j, bit, known=None):
    Cx = Cf.copy()
    Cx.view(np.uint64)[i, j] ^= np.uint64(1 << bit)
    delta = Cx[i, j] - Cf[i, j]
    _, _, orep = orc.verify(Cx, m, n, br, bc, tc, tr, erasures=known)
    cls = orc.classify(orep, m, n, br, bc, erasures=known)
    gray = np.isfinite(delta) and any(t / 2 < abs(delta) < 2 * t for t in (tc[i % br, j], tr[i, j % bc]))
    return cls, orep, gray


@pytest.mark.parametrize("m,n,k,br,bc,runs", [(256, 256, 256, 1, 1, 48), (256, 256, 256, 64, 64, 24),
                                              (200, 136, 72, 8, 4, 24), (1024, 512, 384, 128, 1, 16),
                                              (1536, 1024, 64, 512, 512, 24)])
def test_flip_detect_locate_correct(dev, orc, m, n, k, br, bc, runs):
    """Seeded single bit flips (bits 40..62) anywhere in C_f, data and
    checksums: the GPU flags, location and class equal the oracle's; the
    corrected value is within tau of the clean value; re-verify is clean."""
    A, B, P = make(dev, m, n, k, br, bc)
    P.encode()
    P.gemm()
    clean = P.C.clone()
    Af, Bf, Cf = orc.protected_product(A, B, br, bc)
    tc, tr = orc.tau_det(Af, Bf, m, n, br, bc)
    M, N = m + br, n + bc
    compared = gray_count = 0
    for run in range(runs):
        i, j, bit = synth.flip_site(SEED + 1, run, M, N, 40, 62)
        note(f"flip m={m} br={br} run={run} at ({i},{j}) bit {bit}")
        P.C.copy_(clean)
        abft.inject_flip(P.p, P.C, i, j, bit)
        rep = P.verify()
        loc = abft.classify(P.p, rep)
        (ocls, oi, oj, od), orep, gray = _oracle_decision(orc, Cf, m, n, br, bc, tc, tr, i, j, bit)
        if gray:
            gray_count += 1
            continue
        compared += 1
        assert (rep.n_flag_c, rep.n_flag_r) == (orep.n_flag_c, orep.n_flag_r)
        assert [f[:2] for f in rep.flags_c()] == [f[:2] for f in orep.flags_c()]
        assert [f[:2] for f in rep.flags_r()] == [f[:2] for f in orep.flags_r()]
        # the GPU's thresholds (statistics from the encode pass or from their own pass) are the oracle's
        for r, jj, _, tau in rep.flags_c():
            assert abs(tau - tc[r, jj]) <= 1e-10 * tc[r, jj]
        for ii, c, _, tau in rep.flags_r():
            assert abs(tau - tr[ii, c]) <= 1e-10 * tr[ii, c]
        assert (loc.cls, loc.i, loc.j, loc.dir) == (ocls, oi, oj, od)
        if loc.cls in (abft.ABFT_CLS_DATA, abft.ABFT_CLS_CHECKSUM):
            assert (loc.i, loc.j) == (i, j)
            abft.correct(P.p, P.C, loc)
            rep2 = P.verify()
            assert rep2.n_flag_c == 0 and rep2.n_flag_r == 0
            fixed = P.C[i, j].item()
            want = Cf[i, j]
            assert abs(fixed - want) <= min(tc[i % br, j], tr[i, j % bc]) + TOL64 * np.abs(Cf).max()
            assert abs(fixed - orc.rebuild_value(Cf, m, n, br, bc, i, j, loc.dir)) <= TOL64 * np.abs(Cf).max()
    assert compared >= runs - 2, (compared, gray_count)


@pytest.mark.parametrize("m,n,k,b,rects", [
    (256, 256, 256, 64, [(64, 128, 64, 64), (0, 0, 64, 64), (256, 192, 64, 64), (192, 256, 64, 64), (256, 256, 64, 64)]),
    (1024, 1024, 128, 128, [(384, 512, 128, 128), (1024, 0, 128, 128), (17, 33, 100, 90)]),
    (1024, 1024, 64, 512, [(512, 0, 512, 512), (1024, 512, 512, 512), (100, 700, 300, 200)]),  # one-pass verify
])
def test_erase_and_rebuild_block(dev, orc, m, n, k, b, rects):
    """Zeroed or NaN-filled blocks (data, carried row block, carried column
    block, corner) are skipped by verify when known, rebuilt from the
    column relations (and, cross-checked, the row relations), and the
    rebuilt C_f matches the oracle's."""
    A, B, P = make(dev, m, n, k, b, b)
    P.encode()
    P.gemm()
    clean = P.C.clone()
    Af, Bf, Cf = orc.protected_product(A, B, b, b)
    for q, rect in enumerate(rects):
        for use_rows in (False, True):
            note(f"erase {rect} use_rows={use_rows}")
            P.C.copy_(clean)
            abft.inject_erase(P.p, P.C, rect, nan_fill=bool(q % 2))
            rep = P.verify(known=[rect])
            assert rep.n_flag_c == 0 and rep.n_flag_r == 0 and rep.n_excl_c > 0 and rep.n_excl_r > 0
            abft.recover_block(P.p, P.C, rect, use_rows=use_rows)
            rep = P.verify()
            assert rep.n_flag_c == 0 and rep.n_flag_r == 0
            Cg = P.C.cpu().numpy()
            assert rel_err(Cg, Cf) <= TOL64
            Co = Cf.copy()
            i0, j0, h, w = rect
            Co[i0:i0 + h, j0:j0 + w] = 0
            assert orc.recover(Co, m, n, b, b, rect, use_rows=use_rows) == 0
            assert rel_err(Cg[i0:i0 + h, j0:j0 + w], Co[i0:i0 + h, j0:j0 + w]) <= TOL64


def test_unrecoverable_hole_is_refused(dev):
    note("unrecoverable")
    A, B, P = make(dev, 256, 256, 256, 1, 1)
    with pytest.raises(abft.AbftError) as e:
        abft.recover_block(P.p, P.C, (0, 0, 64, 64))
    assert e.value.status == abft.ABFT_E_UNRECOVERABLE


@pytest.mark.parametrize("where", ["col_band", "row_band", "elsewhere"])
def test_flip_and_erasure_in_one_run(dev, orc, where):
    """A flip plus an erased block: verify with the erasure known, locate and
    correct the flip (by the row relation when it shares the block's column
    band), then rebuild the block; the result matches the clean product."""
    m = n = 1024
    k, b = 256, 128
    A, B, P = make(dev, m, n, k, b, b)
    P.encode()
    P.gemm()
    clean = P.C.cpu().numpy()
    Af, Bf, Cf = orc.protected_product(A, B, b, b)
    rect = (256, 512, 128, 128)
    site = {"col_band": (900, 600), "row_band": (300, 40), "elsewhere": (1000, 1000)}[where]
    note(f"flip+erase {where}")
    abft.inject_flip(P.p, P.C, site[0], site[1], 52)
    abft.inject_erase(P.p, P.C, rect)
    rep = P.verify(known=[rect])
    loc = abft.classify(P.p, rep, known=[rect])
    assert (loc.cls, loc.i, loc.j) == (abft.ABFT_CLS_DATA, site[0], site[1])
    assert loc.dir == (abft.ABFT_DIR_ROW if where == "col_band" else abft.ABFT_DIR_COL)
    abft.correct(P.p, P.C, loc)
    abft.recover_block(P.p, P.C, rect)
    rep = P.verify()
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0
    Cg = P.C.cpu().numpy()
    assert rel_err(Cg, Cf) <= TOL64 and rel_err(Cg, clean) <= TOL64


def test_odd_k_by_zero_padding(dev, orc):
    """k = 255 is refused (rows of A_f and columns of B_f must be whole 16-byte
    chunks); padded with one zero column of A and zero row of B it gives the
    unpadded product (the oracle's C_f of the 255-deep problem), verifies
    clean, and locates a flip."""
    m, n, k, b = 512, 384, 255, 64
    A = synth.uniform(SEED + 5, synth.STREAM_A, m, k)
    B = synth.uniform(SEED + 5, synth.STREAM_B, k, n)
    p_odd = abft.problem(abft.ABFT_F64, m, n, k, b, b)
    ws = torch.zeros(abft.workspace_size(p_odd), dtype=torch.uint8, device=dev)
    with pytest.raises(abft.AbftError):
        abft.encode(p_odd, torch.zeros(m + b, k, dtype=torch.float64, device=dev),
                    torch.zeros(n + b, k, dtype=torch.float64, device=dev), ws)
    P = abft.Protected(abft.ABFT_F64, m, n, k + 1, b, b, device=dev)
    P.A[:m, :k] = torch.from_numpy(A).to(dev)
    P.Bt[:n, :k] = torch.from_numpy(np.ascontiguousarray(B.T)).to(dev)
    P.encode()
    P.gemm()
    torch.cuda.synchronize()
    _, _, Cf = orc.protected_product(A, B, b, b)
    assert rel_err(P.C.cpu().numpy(), Cf) <= TOL64
    rep = P.verify()
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0
    abft.inject_flip(P.p, P.C, 300, 200, 55)
    loc = abft.classify(P.p, P.verify())
    assert (loc.cls, loc.i, loc.j) == (abft.ABFT_CLS_DATA, 300, 200)
