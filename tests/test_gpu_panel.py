"""GPU parity of the panel-update entry point (outer-product form of the
product, Sec. 2.2; rank-nb updates, Sec. 3.2) against the CPU oracle.

After each panel C_f must match the oracle's encoded partial product
A_f[:, :k1] B_f[:k1, :] (binary64: 1e-12, binary32: 1e-5 relative to its
largest entry) and verify clean; a block lost or a bit flipped between two
panels is rebuilt or corrected from the intermediate and the loop goes on to
the product an uninterrupted loop gives.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_0806_3121_amd import abft, synth  # noqa: E402

pytestmark = pytest.mark.gpu

SEED = synth.BASE_SEED
LAMBDA = 10.0
TOL = {abft.ABFT_F64: 1e-12, abft.ABFT_F32: 1e-5}


def note(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abft.lib()
    return torch.device("cuda:0")


def make(dev, dtype, m, n, k, br, bc):
    npdt = np.float64 if dtype == abft.ABFT_F64 else np.float32
    A = synth.uniform(SEED, synth.STREAM_A, m, k, npdt)
    B = synth.uniform(SEED, synth.STREAM_B, k, n, npdt)
    mode = abft.ABFT_TAU_DET if dtype == abft.ABFT_F64 else abft.ABFT_TAU_STAT
    P = abft.Protected(dtype, m, n, k, br, bc, device=dev, tau_mode=mode, lam=LAMBDA)
    P.A[:m] = torch.from_numpy(A).to(dev)
    P.Bt[:n] = torch.from_numpy(np.ascontiguousarray(B.T)).to(dev)
    return A, B, P


def oracle_encoded(orc, dtype, A, B, br, bc):
    return orc.encode(A.astype(np.float64), B.astype(np.float64), br, bc, store_f32=dtype == abft.ABFT_F32)


def rel_err(x, ref):
    return np.abs(x.astype(np.float64) - ref).max() / max(np.abs(ref).max(), 1e-300)


def run_panel(P, k0, k1, accumulate=True):
    abft.gemm_panel(P.p, P.A, P.Bt, P.C, k0, k1, abft.ABFT_ACCUMULATE if accumulate else 0)


DTYPES = [abft.ABFT_F64, abft.ABFT_F32]
CASES = [
    # m, n, k, br, bc, panel edges
    (512, 512, 768, 64, 64, [0, 256, 512, 768]),     # checksum blocks on the matrix cores
    (384, 256, 1000, 1, 1, [0, 336, 672, 1000]),     # thin checksum blocks (streaming kernel), K tail
    (200, 136, 72, 8, 4, [0, 16, 72]),               # ragged tiles, one short panel
    (256, 128, 64, 2, 2, [0, 64]),                   # one panel = the whole product
]


def ids(c):
    return "x".join(map(str, c[:5])) + "-p" + str(len(c[5]) - 1)


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
@pytest.mark.parametrize("case", CASES, ids=[ids(c) for c in CASES])
def test_panels_match_partial_products_and_verify_clean(dev, orc, dtype, case):
    m, n, k, br, bc, edges = case
    note(f"panels dtype={dtype} m={m} n={n} k={k} br={br} bc={bc} edges={edges}")
    A, B, P = make(dev, dtype, m, n, k, br, bc)
    P.encode()
    P.C.fill_(float("nan"))            # the first panel overwrites
    Af, Bf = oracle_encoded(orc, dtype, A, B, br, bc)
    for q in range(len(edges) - 1):
        run_panel(P, edges[q], edges[q + 1], accumulate=q > 0)
        torch.cuda.synchronize()
        want = orc.gemm(Af[:, :edges[q + 1]], Bf[:edges[q + 1], :])
        err = rel_err(P.C.cpu().numpy(), want)
        assert err <= TOL[dtype], (q, err)
        rep = P.verify()
        assert rep.n_flag_c == 0 and rep.n_flag_r == 0, (q, rep.max_ratio_c, rep.max_ratio_r)
    # the panel loop ends on the one-call product
    final = P.C.cpu().numpy().copy()
    P.gemm()
    torch.cuda.synchronize()
    assert rel_err(final, P.C.cpu().numpy().astype(np.float64)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_plain_panels_touch_only_the_data_block(dev, orc, dtype):
    m, n, k, br, bc = 256, 192, 320, 4, 4
    note(f"plain panels dtype={dtype}")
    A, B, P = make(dev, dtype, m, n, k, br, bc)
    P.encode()
    P.C.fill_(float("nan"))
    abft.gemm_panel(P.p, P.A, P.Bt, P.C, 0, 160, abft.ABFT_PLAIN)
    abft.gemm_panel(P.p, P.A, P.Bt, P.C, 160, 320, abft.ABFT_PLAIN | abft.ABFT_ACCUMULATE)
    torch.cuda.synchronize()
    Cg = P.C.cpu().numpy()
    want = A.astype(np.float64) @ B.astype(np.float64)
    assert rel_err(Cg[:m, :n], want) <= TOL[dtype]
    assert np.isnan(Cg[m:]).all() and np.isnan(Cg[:, n:]).all()


ERASE = [
    # m, n, k, br, bc, edges, lost block (i0, j0, h, w), rebuild along rows
    (512, 512, 768, 64, 64, [0, 256, 512, 768], (128, 320, 64, 64), False),
    (512, 512, 768, 64, 64, [0, 256, 512, 768], (512, 64, 64, 64), False),    # in the carried row block
    (384, 256, 1000, 1, 1, [0, 336, 672, 1000], (0, 17, 1, 100), False),
    (384, 256, 1000, 1, 1, [0, 336, 672, 1000], (40, 0, 200, 1), True),
]


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
@pytest.mark.parametrize("case", ERASE, ids=[f"{c[0]}x{c[3]}-{c[6]}-{'row' if c[7] else 'col'}" for c in ERASE])
def test_block_lost_between_panels_is_rebuilt_and_loop_goes_on(dev, orc, dtype, case):
    m, n, k, br, bc, edges, rect, use_rows = case
    note(f"mid-loop erasure dtype={dtype} m={m} br={br} rect={rect} rows={use_rows}")
    A, B, P = make(dev, dtype, m, n, k, br, bc)
    P.encode()
    Af, Bf = oracle_encoded(orc, dtype, A, B, br, bc)
    run_panel(P, edges[0], edges[1], accumulate=False)
    run_panel(P, edges[1], edges[2])
    abft.inject_erase(P.p, P.C, rect)
    rep = P.verify(known=[rect])
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0
    abft.recover_block(P.p, P.C, rect, use_rows=use_rows)
    torch.cuda.synchronize()
    partial = orc.gemm(Af[:, :edges[2]], Bf[:edges[2], :])
    # the oracle rebuilds the same block of its own intermediate
    Co = partial.copy()
    i0, j0, h, w = rect
    Co[i0:i0 + h, j0:j0 + w] = np.nan
    assert orc.recover(Co, m, n, br, bc, rect, use_rows=use_rows,
                       round_f32=dtype == abft.ABFT_F32) == 0
    Cg = P.C.cpu().numpy()
    blk = (slice(i0, i0 + h), slice(j0, j0 + w))
    scale = np.abs(partial).max()
    assert np.abs(Cg[blk].astype(np.float64) - Co[blk]).max() / scale <= TOL[dtype]
    assert rel_err(Cg, partial) <= TOL[dtype]
    for q in range(2, len(edges) - 1):
        run_panel(P, edges[q], edges[q + 1])
    rep = P.verify()
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0
    torch.cuda.synchronize()
    assert rel_err(P.C.cpu().numpy(), orc.gemm(Af, Bf)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_flip_between_panels_located_corrected_and_loop_goes_on(dev, orc, dtype):
    m, n, k, br, bc = 384, 256, 1000, 1, 1
    edges = [0, 336, 672, 1000]
    i, j = 201, 77
    bit = 58 if dtype == abft.ABFT_F64 else 28     # an exponent bit: a large, finite error
    note(f"mid-loop flip dtype={dtype} at ({i},{j}) bit {bit}")
    A, B, P = make(dev, dtype, m, n, k, br, bc)
    P.encode()
    Af, Bf = oracle_encoded(orc, dtype, A, B, br, bc)
    run_panel(P, edges[0], edges[1], accumulate=False)
    abft.inject_flip(P.p, P.C, i, j, bit)
    rep = P.verify()
    loc = abft.classify(P.p, rep)
    assert (loc.cls, loc.i, loc.j) == (abft.ABFT_CLS_DATA, i, j)
    abft.correct(P.p, P.C, loc)
    for q in range(1, len(edges) - 1):
        run_panel(P, edges[q], edges[q + 1])
    rep = P.verify()
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0
    torch.cuda.synchronize()
    assert rel_err(P.C.cpu().numpy(), orc.gemm(Af, Bf)) <= TOL[dtype]
