"""GPU parity of every binary64 / binary32 product tile against the CPU oracle.

The product dispatch picks a kernel (direct-to-LDS when k is a multiple of
the 128-byte slab, register-staged otherwise) and a block tile per shape.
Each case below names the kernel and tile that abft_describe_gemm must report
for its shape, so a change of the tile tables that leaves a tile untested
fails here, and checks the whole protected product (b = 1: data part on that
tile, carried row and column by the streaming kernel) against the oracle:
max|C_gpu - C_oracle| / max|C_oracle| <= 1e-12 (binary64) or 1e-5
(binary32, oracle in binary64 rounded once), then a clean verification.
Shapes are ragged in both m and n (no multiple of 32) so every tile has
partial edge tiles.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_0806_3121_amd import abft, synth  # noqa: E402

pytestmark = pytest.mark.gpu

SEED = synth.BASE_SEED + 77
DT = {"f64": abft.ABFT_F64, "f32": abft.ABFT_F32}

CASES = [
    # direct-to-LDS binary64 (k % 16 == 0)
    ("f64", 72, 72, 32, "k_gemm_mfma2 f64 96x96"),
    ("f64", 776, 5384, 32, "k_gemm_mfma2 f64 128x96"),
    ("f64", 1032, 5384, 32, "k_gemm_mfma2 f64 128x128"),
    # register-staged binary64 (k % 16 != 0)
    ("f64", 72, 72, 40, "k_gemm_mfma f64 96x96"),
    ("f64", 776, 5384, 40, "k_gemm_mfma f64 128x96"),
    ("f64", 1288, 5384, 40, "k_gemm_mfma f64 128x128"),
    ("f64", 1032, 5384, 40, "k_gemm_mfma f64 256x128"),
    # binary32: direct (k % 32 == 0) and register-staged
    ("f32", 72, 72, 64, "k_gemm_mfma2 f32 256x128"),
    ("f32", 1288, 5384, 64, "k_gemm_mfma2 f32 128x128"),
    ("f32", 72, 72, 40, "k_gemm_mfma f32 256x128"),
    ("f32", 1288, 5384, 40, "k_gemm_mfma f32 128x128"),
]
IDS = [f"{c[0]}-{c[1]}x{c[2]}x{c[3]}" for c in CASES]


def note(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abft.lib()
    return torch.device("cuda:0")


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_tile_matches_oracle(dev, orc, case):
    dt, m, n, k, kernel = case
    note(f"tile {case}")
    npdt = np.float64 if dt == "f64" else np.float32
    A = synth.uniform(SEED, synth.STREAM_A, m, k, npdt)
    B = synth.uniform(SEED, synth.STREAM_B, k, n, npdt)
    mode = abft.ABFT_TAU_DET if dt == "f64" else abft.ABFT_TAU_STAT
    P = abft.Protected(DT[dt], m, n, k, 1, 1, device=dev, tau_mode=mode, lam=10.0)
    desc = abft.describe_gemm(P.p)
    assert desc.startswith(kernel + f" on {m}x{n} k={k}"), desc
    P.A[:m] = torch.from_numpy(A).to(dev)
    P.Bt[:n] = torch.from_numpy(np.ascontiguousarray(B.T)).to(dev)
    P.encode()
    P.gemm()
    torch.cuda.synchronize()
    Af, Bf = orc.encode(A.astype(np.float64), B.astype(np.float64), 1, 1, store_f32=(dt == "f32"))
    Cref = orc.gemm(Af, Bf)
    if dt == "f32":
        Cref = Cref.astype(np.float32).astype(np.float64)
    Cg = P.C.cpu().numpy().astype(np.float64)
    err = np.abs(Cg - Cref).max() / np.abs(Cref).max()
    assert err <= (1e-12 if dt == "f64" else 1e-5), err
    rep = P.verify()
    assert rep.n_flag_c == 0 and rep.n_flag_r == 0
    assert max(rep.max_ratio_c, rep.max_ratio_r) < 0.5


def test_every_table_tile_is_covered():
    """The cases above name each tile of both kernels once per element type."""
    names = {c[4] for c in CASES}
    assert len(names) == len(CASES)
    for dt, tiles in (("f64", ("96x96", "128x96", "128x128")), ("f32", ("256x128", "128x128"))):
        for t in tiles:
            assert f"k_gemm_mfma2 {dt} {t}" in names
    for dt, tiles in (("f64", ("96x96", "128x96", "128x128", "256x128")), ("f32", ("256x128", "128x128"))):
        for t in tiles:
            assert f"k_gemm_mfma {dt} {t}" in names
