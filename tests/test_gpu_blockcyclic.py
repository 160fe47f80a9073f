"""GPU tests of the 2-D block-cyclic layout (Sec. 4.1) against the CPU
oracle's owner map: the stacked local arrays of a P x Q grid bit for bit for
every element size, and the protected product in that layout — its block
checksums are the grid's checksum process row and column, and a lost
process's local array is rebuilt."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_0806_3121_amd import abft, synth  # noqa: E402

pytestmark = pytest.mark.gpu

SEED = synth.BASE_SEED + 71


def note(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abft.lib()
    return torch.device("cuda:0")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.int16, torch.uint8])
@pytest.mark.parametrize("rows,cols,nb,P,Q", [(384, 256, 32, 3, 2), (256, 448, 64, 1, 7), (128, 96, 16, 4, 1)])
def test_stack_unstack_match_owner_map(dev, orc, dtype, rows, cols, nb, P, Q):
    note(f"block-cyclic stack {dtype} {rows}x{cols} nb={nb} grid {P}x{Q}")
    vals = synth.uniform_ints(SEED, synth.STREAM_A, rows, cols, 0, 100)
    G = torch.from_numpy(vals.astype(np.float64)).to(dtype).to(dev)
    S = torch.full((rows, cols + 3), 7, dtype=dtype, device=dev)[:, :cols]      # padded leading dimension
    abft.block_cyclic_stack(G, rows, cols, nb, P, Q, S)
    back = torch.zeros_like(G)
    abft.block_cyclic_unstack(S, rows, cols, nb, P, Q, back)
    torch.cuda.synchronize()
    want = orc.block_cyclic_stack(vals.astype(np.float64), nb, P, Q)
    assert np.array_equal(S.cpu().double().numpy(), want)
    assert torch.equal(back, G)


def test_block_cyclic_product_checksum_processes_and_lost_process(dev, orc):
    m, n, k, nb, P, Q = 1024, 768, 512, 64, 4, 3
    br, bc = m // P, n // Q
    note(f"block-cyclic product {m}x{n}x{k} nb={nb} grid {P}x{Q}")
    A = synth.uniform(SEED, synth.STREAM_A, m, k)
    B = synth.uniform(SEED, synth.STREAM_B, k, n)
    Ag = torch.from_numpy(A).to(dev)
    Btg = torch.from_numpy(np.ascontiguousarray(B.T)).to(dev)
    Pr = abft.Protected(abft.ABFT_F64, m, n, k, br, bc, device=dev)
    abft.block_cyclic_stack(Ag, m, k, nb, P, 1, Pr.A[:m])        # A's rows over the process rows
    abft.block_cyclic_stack(Btg, n, k, nb, Q, 1, Pr.Bt[:n])      # B's columns (B^T's rows) over the process columns
    Pr.encode()
    Pr.gemm()
    rep = Pr.verify()
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0
    Cf = Pr.C.cpu().numpy()
    G = orc.gemm(A, B)
    scale = np.abs(G).max()
    assert np.abs(Cf[:m, :n] - orc.block_cyclic_stack(G, nb, P, Q)).max() <= 1e-12 * scale
    # the checksum process row and column: sums of the local arrays over the grid's rows / columns
    want_row = np.zeros((br, n))
    want_col = np.zeros((m, bc))
    S = orc.block_cyclic_stack(G, nb, P, Q)
    for p in range(P):
        want_row += S[p * br:(p + 1) * br]
    for q in range(Q):
        want_col += S[:, q * bc:(q + 1) * bc]
    assert np.abs(Cf[m:, :n] - want_row).max() <= 1e-12 * np.abs(want_row).max()
    assert np.abs(Cf[:m, n:] - want_col).max() <= 1e-12 * np.abs(want_col).max()
    # process (2, 1) fails: its whole local array is lost, then rebuilt
    clean = Pr.C.clone()
    rect = (2 * br, 1 * bc, br, bc)
    Pr.C[rect[0]:rect[0] + br, rect[1]:rect[1] + bc] = float("nan")
    rep = Pr.verify(known=[rect])
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0
    abft.recover_block(Pr.p, Pr.C, rect)
    rep = Pr.verify()
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0
    torch.cuda.synchronize()
    assert (Pr.C - clean).abs().max().item() <= 1e-12 * scale
    # back to the global layout
    Cg = torch.zeros(m, n, dtype=torch.float64, device=dev)
    abft.block_cyclic_unstack(Pr.C[:m, :n], m, n, nb, P, Q, Cg)
    torch.cuda.synchronize()
    assert np.abs(Cg.cpu().numpy() - G).max() <= 1e-12 * scale
