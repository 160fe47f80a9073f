"""Full-size binary64 parity at the benchmark workload, in its launch
configuration: n = 8192 with an 8 x 8 grid of 1024 x 1024 blocks (one checksum
block row and column), and the same inputs with the classic b = 1 encoding.

The oracle cannot afford the whole product here, so it computes sampled rows
and columns of C_f one by one, every checksum row and column of the encoded
operands, and the residuals of the relations the GPU flags; the rest is
checked through properties that hold at any size (clean verify before the
faults, exact location of the injected flip, clean verify after repair,
repaired C_f equal to the clean one within the binary64 tolerance).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_0806_3121_amd import abft, synth  # noqa: E402

pytestmark = pytest.mark.gpu

SEED = synth.BASE_SEED
TOL64 = 1e-12


def note(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def inputs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    n = 8192
    note("generating 8192^2 inputs on the host")
    A = synth.uniform(SEED, synth.STREAM_A, n, n)
    B = synth.uniform(SEED, synth.STREAM_B, n, n)
    return A, B


def oracle_relation_residual(orc, Af, Bf, m, n, br, bc, i, j, flip_bit, direction):
    """Oracle residual of the relation through (i, j) of C_f after the flip,
    each member computed as an ascending-order dot product."""
    M, N = Af.shape[0], Bf.shape[1]
    k = Af.shape[1]

    def elem(a, b):
        v = orc.dot(Af[a], np.ascontiguousarray(Bf[:, b]))
        if (a, b) == (i, j):
            v = np.array([v]).view(np.uint64)
            v ^= np.uint64(1 << flip_bit)
            v = float(v.view(np.float64)[0])
        return v

    if direction == "col":
        r = i % br
        s = sum(elem(g * br + r, j) for g in range(m // br))
        return s - elem(m + r, j)
    c = j % bc
    s = sum(elem(i, h * bc + c) for h in range(n // bc))
    return s - elem(i, n + c)


@pytest.mark.parametrize("b", [1024, 1])
def test_fullsize_pipeline(inputs, orc, b):
    A, B = inputs
    n = m = k = 8192
    dev = torch.device("cuda:0")
    note(f"full size n=8192 b={b}: upload, encode, gemm")
    P = abft.Protected(abft.ABFT_F64, m, n, k, b, b, device=dev)
    P.A[:m] = torch.from_numpy(A).to(dev)
    P.Bt[:n] = torch.from_numpy(np.ascontiguousarray(B.T)).to(dev)
    P.encode()
    P.gemm()
    torch.cuda.synchronize()
    note("clean verify")
    rep = P.verify()
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0
    assert rep.max_ratio_c < 1e-2 and rep.max_ratio_r < 1e-2

    note("oracle encode + sampled rows/columns")
    Af, Bf = orc.encode(A, B, b, b)
    gA = P.A[m:].cpu().numpy()
    gB = P.Bt[n:].cpu().numpy().T
    G = m // b
    assert np.abs(gA - Af[m:]).max() <= 2 * G * 2.0 ** -53 * 8192
    assert np.abs(gB - Bf[:, n:]).max() <= 2 * G * 2.0 ** -53 * 8192
    rows = [0, 1, 4097, m - 1, m, m + b - 1]
    cols = [0, 5000, n - 1, n, n + b - 1]
    Cg_rows = P.C[rows].cpu().numpy()
    Co_rows = orc.gemm(Af[rows], Bf)
    cmax = np.abs(Co_rows).max()
    assert np.abs(Cg_rows - Co_rows).max() / cmax <= TOL64
    Cg_cols = P.C[:, cols].cpu().numpy()
    Co_cols = orc.gemm(Af, np.ascontiguousarray(Bf[:, cols]))
    assert np.abs(Cg_cols - Co_cols).max() / max(cmax, np.abs(Co_cols).max()) <= TOL64

    # one flip (bits 40..62) and, for the block encoding, one erased 1024^2 block
    clean = P.C.clone()
    rect = None
    if b > 1:
        I, J = synth.erase_block(SEED, 0, m // b, n // b)
        rect = (I * b, J * b, b, b)
    i, j, bit = synth.flip_site(SEED, 0, m, n, 40, 62, avoid=rect)
    note(f"flip ({i},{j}) bit {bit}, erase {rect}")
    abft.inject_flip(P.p, P.C, i, j, bit)
    known = [rect] if rect else None
    if rect:
        abft.inject_erase(P.p, P.C, rect)
    rep = P.verify(known=known)
    loc = abft.classify(P.p, rep, known=known)
    # the oracle's own residuals for the relations through the flipped element
    tc, tr = orc.tau_det(Af, Bf, m, n, b, b)
    col_erased = rect is not None and rect[1] <= j < rect[1] + rect[3]
    row_erased = rect is not None and rect[0] <= i < rect[0] + rect[2]
    d_row = oracle_relation_residual(orc, Af, Bf, m, n, b, b, i, j, bit, "row")
    d_col = None if col_erased else oracle_relation_residual(orc, Af, Bf, m, n, b, b, i, j, bit, "col")
    t_row, t_col = tr[i, j % b], tc[i % b, j]
    assert not (abs(d_row) <= t_row)
    if d_col is not None:
        assert not (abs(d_col) <= t_col)
    gpu_rows = [f[:2] for f in rep.flags_r()]
    gpu_cols = [f[:2] for f in rep.flags_c()]
    # the GPU's thresholds of these relations (row statistics from the encode pass) are the oracle's
    for f in rep.flags_r():
        assert abs(f[3] - tr[f[0], f[1]]) <= 1e-10 * tr[f[0], f[1]]
    for f in rep.flags_c():
        assert abs(f[3] - tc[f[0], f[1]]) <= 1e-10 * tc[f[0], f[1]]
    assert gpu_rows == [(i, j % b)]
    assert gpu_cols == ([] if col_erased else [(i % b, j)])
    assert (loc.cls, loc.i, loc.j) == (abft.ABFT_CLS_DATA, i, j)
    assert loc.dir == (abft.ABFT_DIR_ROW if col_erased else abft.ABFT_DIR_COL)
    assert not row_erased
    abft.correct(P.p, P.C, loc)
    if rect:
        abft.recover_block(P.p, P.C, rect)
    note("re-verify")
    rep = P.verify()
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0
    diff = (P.C - clean).abs().max().item()
    assert diff / clean.abs().max().item() <= TOL64
    assert abs(P.C[i, j].item() - Af[i] @ Bf[:, j]) <= max(t_row, t_col)
    # the paper's residual check (Sec. 4.3) on the repaired product, in the infinity norm with the unit
    # roundoff of the accumulation: rho = ||C x - A (B x)|| / (k u ||C|| ||x||), small (<= 10)
    x = synth.uniform(SEED, synth.STREAM_X, n, 1)[:, 0]
    C = P.C[:m, :n].cpu().numpy()
    rho = np.abs(C @ x - A @ (B @ x)).max() / (k * 2.0 ** -53 * np.abs(C).sum(axis=1).max() * np.abs(x).max())
    note(f"residual rho {rho:.3e}")
    assert rho <= 10.0
