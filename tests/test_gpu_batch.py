"""GPU parity of the batched bfloat16 path (many independent protected
products of uneven shapes, flattened descriptors, persistent product kernel)
against the CPU oracle, and of its hipGraph replay against eager launches.

Per problem the oracle does what the single-problem bfloat16 test does: its
own round-to-nearest-even of the binary32 inputs (bit-exact vs the device
quantizer), binary32 checksum rows, the exact product in binary64 rounded to
binary32, the statistical thresholds with T = k/4, s = 2 (Sec. 3 reading).
 - values: |C_gpu - C_oracle| <= k u32 (|A_q||B_q|)_ij + u32 |C_ij|;
 - both tile shapes give the same C bit for bit (same k order per element);
 - flip decisions and locations equal the oracle's outside the gray zone;
 - a graph replay equals the eager pass bit for bit, replay after replay.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_0806_3121_amd import abft, synth  # noqa: E402

pytestmark = pytest.mark.gpu

SEED = synth.BASE_SEED + 40
LAMBDA = 20.0
U32 = 2.0 ** -24


def note(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abft.lib()
    return torch.device("cuda:0")


def batch_shapes():
    # edge shapes (one group, minimal k, ragged tiles, one large problem) then seeded draws
    shapes = [(32, 32, 8, 32, 1), (64, 40, 24, 32, 8), (96, 200, 72, 32, 1), (2048, 1056, 1024, 32, 32),
              (128, 132, 64, 32, 2), (192, 1060, 128, 32, 4),
              # small br (several partitions of A's groups), br = 1 (B's rows weighted by A's sums of
              # squares, taken after A's pass), rows in one and in several 128-column strips
              (64, 96, 256, 1, 1), (96, 64, 200, 4, 1), (40, 48, 136, 8, 2), (33, 70, 520, 1, 2),
              (48, 50, 1032, 1, 1)]
    for q, (m, n, k) in enumerate(synth.batched_shapes(SEED, 20, lo=64, hi=640, step=32)):
        shapes.append((m, n, k, 32, 1 if q % 2 == 0 else 32))
    return shapes


class Case:
    def __init__(self, dev, orc):
        self.shapes = batch_shapes()
        self.B = abft.Batch(self.shapes, device=dev, tau_mode=abft.ABFT_TAU_STAT, lam=LAMBDA)
        self.ref = []
        for q, (m, n, k, br, bc) in enumerate(self.shapes):
            A32 = synth.uniform(SEED + q, synth.STREAM_A, m, k, np.float32)
            B32 = synth.uniform(SEED + q, synth.STREAM_B, k, n, np.float32)
            self.B.A32[q].copy_(torch.from_numpy(A32))
            self.B.Bt32[q].copy_(torch.from_numpy(np.ascontiguousarray(B32.T)))
            Aq = orc.to_bf16_bits(A32)
            Bq = orc.to_bf16_bits(B32)
            A = orc.bf16_bits_to_f64(Aq)
            Bm = orc.bf16_bits_to_f64(Bq)
            Af, Bf = orc.encode(A, Bm, br, bc, store_f32=True)
            C64 = orc.gemm(Af, Bf)
            C32 = C64.astype(np.float32)
            # the carried totals are accumulated on the matrix cores: T_c = k / 4 steps
            tc, tr = orc.tau_stat(Af, Bf, m, n, br, bc, u_acc=U32, T=k / 4.0, s_store=2.0, lam=LAMBDA, Cf=C64,
                                  T_c=k / 4.0)
            retau = (lambda Af, Bf, m, n, k, br, bc: lambda Cx: orc.tau_stat(
                Af, Bf, m, n, br, bc, u_acc=U32, T=k / 4.0, s_store=2.0, lam=LAMBDA,
                Cf=np.asarray(Cx, dtype=np.float64), T_c=k / 4.0))(Af, Bf, m, n, k, br, bc)
            bound = k * U32 * (np.abs(Af) @ np.abs(Bf)) + U32 * np.abs(C32)
            self.ref.append(dict(Aq=Aq, Bq=Bq, C32=C32, tc=tc, tr=tr, bound=bound, retau=retau))
        torch.cuda.synchronize()

    def run(self, tile):
        abft.batch_quantize(self.B.plan)
        abft.batch_encode(self.B.plan)
        abft.batch_gemm(self.B.plan, tile)
        abft.batch_verify(self.B.plan)
        return self.B.reports()


@pytest.fixture(scope="module")
def case(dev, orc):
    note(f"batch of {len(batch_shapes())} problems")
    return Case(dev, orc)


def test_batch_quantize_bit_exact(case):
    abft.batch_quantize(case.B.plan)
    torch.cuda.synchronize()
    for q, r in enumerate(case.ref):
        note(f"quantize problem {q} {case.shapes[q]}")
        a = case.B.A[q].cpu().view(torch.int16).numpy().view(np.uint16)
        b = case.B.Bt[q].cpu().view(torch.int16).numpy().view(np.uint16)
        assert np.array_equal(a, r["Aq"])
        assert np.array_equal(b, np.ascontiguousarray(r["Bq"].T))


@pytest.mark.parametrize("tile", range(abft.ABFT_BATCH_TILES))
def test_batch_product_and_clean_verify(case, tile):
    note(f"batch pass tile={tile}")
    reps = case.run(tile)
    for q, r in enumerate(case.ref):
        Cg = case.B.C[q].cpu().numpy().astype(np.float64)
        err = np.abs(Cg - r["C32"])
        assert np.all(err <= r["bound"] * 1.01 + 1e-30), (q, case.shapes[q], err.max())
        assert reps[q].n_flag_c == 0 and reps[q].n_flag_r == 0, (q, reps[q].max_ratio_c, reps[q].max_ratio_r)
    note(f"  max |D|/tau {max(max(x.max_ratio_c, x.max_ratio_r) for x in reps):.4f}")


def test_batch_thresholds_match_oracle(case):
    """The thresholds the verification uses (the encode's threshold statistics,
    the product's stored totals) against the oracle's for every relation of
    every problem, after the encode of stored bfloat16 operands; the fused
    quantize + encode gives the same thresholds bit for bit.  Tolerance: the
    stored totals are binary32 sums on the matrix cores (the oracle's are
    exact), which moves a threshold by far less than 1e-4 of itself."""
    case.run(0)
    torch.cuda.synchronize()

    def thresholds():
        out = []
        for q, (m, n, k, br, bc) in enumerate(case.shapes):
            tc = torch.empty(br, n + bc, dtype=torch.float64, device=case.B.C[q].device)
            tr = torch.empty(m + br, bc, dtype=torch.float64, device=case.B.C[q].device)
            abft.batch_thresholds(case.B.plan, q, tc, tr)
            out.append((tc, tr))
        torch.cuda.synchronize()
        return [(tc.cpu().numpy(), tr.cpu().numpy()) for tc, tr in out]

    enc = thresholds()
    for q, ((tc, tr), r) in enumerate(zip(enc, case.ref)):
        note(f"thresholds problem {q} {case.shapes[q]}")
        assert np.all(np.isfinite(tc)) and np.all(tc > 0) and np.all(np.isfinite(tr)) and np.all(tr > 0)
        np.testing.assert_allclose(tc, r["tc"], rtol=1e-4, atol=0)
        np.testing.assert_allclose(tr, r["tr"], rtol=1e-4, atol=0)
    abft.batch_quantize_encode(case.B.plan)
    fused = thresholds()
    for q, (a, b) in enumerate(zip(enc, fused)):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), q


def test_batch_tiles_agree_and_tune(case, tmp_path):
    """Every tile shape, and each problem with its own (the model's, then
    the tuner's), gives the same C bit for bit; the tuner measures every
    problem under every shape; its costs round-trip through the cache file."""
    case.run(0)
    C0 = [c.clone() for c in case.B.C]
    for tile in list(range(1, abft.ABFT_BATCH_TILES)) + [abft.ABFT_BATCH_MIXED]:
        note(f"tile {tile} vs tile 0")
        case.run(tile)
        torch.cuda.synchronize()
        for q in range(len(C0)):
            assert torch.equal(C0[q], case.B.C[q]), (tile, q)
    costs, tiles = abft.batch_tune(case.B.plan)
    assert len(tiles) == len(case.shapes) and all(0 <= t < abft.ABFT_BATCH_TILES for t in tiles)
    assert all(c > 0 for row in costs for c in row)
    assert all(row[t] == min(row) for row, t in zip(costs, tiles))
    note(f"  tuned shapes {tiles}")
    case.B.set_tiles(tiles)
    reps = case.run(abft.ABFT_BATCH_MIXED)
    torch.cuda.synchronize()
    for q in range(len(C0)):
        assert torch.equal(C0[q], case.B.C[q]), ("tuned", q)
        assert reps[q].n_flag_c == 0 and reps[q].n_flag_r == 0
    ms, choice = abft.batch_choose(case.B.plan, reps=2)
    note(f"  launch choice ms {[round(x, 3) for x in ms]} -> {choice}")
    assert len(ms) == abft.ABFT_BATCH_TILES + 1 and all(x > 0 for x in ms)
    assert ms[choice] == min(ms)
    case.run(choice)
    torch.cuda.synchronize()
    for q in range(len(C0)):
        assert torch.equal(C0[q], case.B.C[q]), ("chosen", q)
    path = str(tmp_path / "batch_tiles.txt")
    abft.batch_cache_store(path, case.B.probs, costs, arch="gfx950")
    found, cached = abft.batch_cache_lookup(path, case.B.probs, arch="gfx950")
    assert found == len(case.shapes) and all(0 <= t < abft.ABFT_BATCH_TILES for t in cached)


def test_batch_fused_quantize_encode_matches_separate_steps(case):
    reps0 = case.run(0)
    torch.cuda.synchronize()
    C0 = [c.clone() for c in case.B.C]
    for a, b in zip(case.B.A, case.B.Bt):
        a.zero_()
        b.zero_()
    abft.batch_quantize_encode(case.B.plan)
    abft.batch_gemm(case.B.plan, 0)
    abft.batch_verify(case.B.plan)
    reps = case.B.reports()
    for q, r in enumerate(case.ref):
        note(f"fused quantize+encode problem {q}")
        a = case.B.A[q].cpu().view(torch.int16).numpy().view(np.uint16)
        assert np.array_equal(a, r["Aq"])
        assert torch.equal(case.B.C[q], C0[q]), q
        assert reps[q].max_ratio_c == reps0[q].max_ratio_c and reps[q].max_ratio_r == reps0[q].max_ratio_r


def test_batch_plain_product_is_data_block(case):
    case.run(0)
    torch.cuda.synchronize()
    C0 = [c[:m, :n].clone() for c, (m, n, k, br, bc) in zip(case.B.C, case.shapes)]
    for c in case.B.Cbuf:
        c.fill_(float("nan"))
    abft.batch_gemm(case.B.plan, 3, abft.ABFT_PLAIN)
    torch.cuda.synchronize()
    for q, (m, n, k, br, bc) in enumerate(case.shapes):
        assert torch.equal(case.B.C[q][:m, :n], C0[q]), q
        assert torch.isnan(case.B.C[q][m:, :]).all() and torch.isnan(case.B.C[q][:, n:]).all()


def test_batch_flips_match_oracle(case, orc):
    case.run(0)
    torch.cuda.synchronize()
    clean = [c.clone() for c in case.B.C]
    targets = synth.pick_distinct(SEED + 1, 6, len(case.shapes))
    compared = located = 0
    for run, q in enumerate(targets):
        m, n, k, br, bc = case.shapes[q]
        r = case.ref[q]
        p = case.B.probs[q]
        i, j, bit = synth.flip_site(SEED + 2, run, m + br, n + bc, 11, 30)
        note(f"flip problem {q} {case.shapes[q]} at ({i},{j}) bit {bit}")
        case.B.C[q].copy_(clean[q])
        abft.inject_flip(p, case.B.C[q], i, j, bit)
        abft.batch_verify(case.B.plan)
        reps = case.B.reports()
        for q2, rep in enumerate(reps):
            if q2 != q:
                assert rep.n_flag_c == 0 and rep.n_flag_r == 0, q2
        rep = reps[q]
        Cx = r["C32"].copy()
        Cx.view(np.uint32)[i, j] ^= np.uint32(1 << bit)
        delta = float(Cx[i, j]) - float(r["C32"][i, j])
        t1, t2 = r["tc"][i % br, j], r["tr"][i, j % bc]
        if np.isfinite(delta) and (t1 / 2 < abs(delta) < 2 * t1 or t2 / 2 < abs(delta) < 2 * t2):
            case.B.C[q].copy_(clean[q])
            continue
        compared += 1
        # a flip on a stored total also moves that relation's rounding term
        tcx, trx = r["retau"](Cx) if (i >= m or j >= n) else (r["tc"], r["tr"])
        _, _, orep = orc.verify(Cx.astype(np.float64), m, n, br, bc, tcx, trx)
        ocls, oi, oj, _ = orc.classify(orep, m, n, br, bc)
        assert (rep.n_flag_c, rep.n_flag_r) == (orep.n_flag_c, orep.n_flag_r)
        loc = abft.classify(p, rep)
        assert (loc.cls, loc.i, loc.j) == (ocls, oi, oj)
        if loc.cls in (abft.ABFT_CLS_DATA, abft.ABFT_CLS_CHECKSUM):
            located += 1
            abft.correct(p, case.B.C[q], loc)
            abft.batch_verify(case.B.plan)
            rep2 = case.B.reports()[q]
            assert rep2.n_flag_c == 0 and rep2.n_flag_r == 0
            assert abs(case.B.C[q][i, j].item() - clean[q][i, j].item()) <= min(t1, t2)
        case.B.C[q].copy_(clean[q])
    note(f"  compared {compared}, located {located}")
    assert compared >= 4 and located >= 2


def test_batch_erasure_rebuild(case):
    case.run(0)
    torch.cuda.synchronize()
    clean = [c.clone() for c in case.B.C]
    for q in synth.pick_distinct(SEED + 3, 4, len(case.shapes)):
        m, n, k, br, bc = case.shapes[q]
        gi = synth.randint(SEED + 4, synth.STREAM_PICK, 2 * q, m // 32 + 1)
        gj = synth.randint(SEED + 4, synth.STREAM_PICK, 2 * q + 1, n // 32)
        rect = (gi * 32, gj * 32, 32, 32)
        note(f"erase problem {q} {case.shapes[q]} rect {rect}")
        p = case.B.probs[q]
        abft.inject_erase(p, case.B.C[q], rect, nan_fill=True)
        abft.recover_block(p, case.B.C[q], rect, use_rows=False)
        abft.batch_verify(case.B.plan)
        rep = case.B.reports()[q]
        assert rep.n_flag_c == 0 and rep.n_flag_r == 0
        i0, j0, h, w = rect
        got = case.B.C[q][i0:i0 + h, j0:j0 + w].cpu().numpy().astype(np.float64)
        want = case.ref[q]["C32"][i0:i0 + h, j0:j0 + w].astype(np.float64)
        assert np.abs(got - want).max() <= np.abs(case.ref[q]["tc"]).max()
        case.B.C[q].copy_(clean[q])


def test_batch_graph_replay_matches_eager(case):
    reps_eager = case.run(0)
    torch.cuda.synchronize()
    C_eager = [c.clone() for c in case.B.C]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            abft.batch_quantize(case.B.plan)
            abft.batch_encode(case.B.plan)
            abft.batch_gemm(case.B.plan, 0)
            abft.batch_verify(case.B.plan)
    torch.cuda.current_stream().wait_stream(s)
    for rep_no in range(4):
        note(f"graph replay {rep_no}")
        # eager work between replays: wipe C and plant a flip the replay must overwrite
        for c in case.B.C:
            c.zero_()
        abft.inject_flip(case.B.probs[0], case.B.C[0], 0, 0, 30)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        reps = case.B.reports()
        for q in range(len(C_eager)):
            assert torch.equal(case.B.C[q], C_eager[q]), (rep_no, q)
            assert reps[q].n_flag_c == 0 and reps[q].n_flag_r == 0
            assert reps[q].max_ratio_c == reps_eager[q].max_ratio_c
            assert reps[q].max_ratio_r == reps_eager[q].max_ratio_r
    del g


def test_batch_unpadded_rows_match_padded(dev):
    """C rows not 16-byte aligned (ldc = n + bc, not a multiple of 4) take the
    element-wise store and verification; they must give the padded batch's C
    bit for bit, a clean verification, and the same failed relations and
    classification for the same flips (bc = 1 and 2, one and two strips)."""
    shapes = [(256, 200, 96, 32, 1), (128, 132, 64, 32, 2), (96, 1064, 80, 32, 2), (64, 2000, 296, 32, 1)]
    pads = [abft.Batch(shapes, device=dev, tau_mode=abft.ABFT_TAU_STAT, lam=LAMBDA, ldc_align=a) for a in (4, 1)]
    assert all((n + bc) % 4 != 0 for (_, n, _, _, bc) in shapes)
    for B in pads:
        for q, (m, n, k, br, bc) in enumerate(shapes):
            abft.fill_uniform(abft.ABFT_F32, m, k, k, 0, SEED + 50 + q, synth.STREAM_A, B.A32[q])
            abft.fill_uniform(abft.ABFT_F32, k, n, k, 1, SEED + 50 + q, synth.STREAM_B, B.Bt32[q])
    for tile in (0, 3):
        note(f"unpadded vs padded rows, tile {tile}")
        reps = []
        for B in pads:
            abft.batch_quantize_encode(B.plan)
            abft.batch_gemm(B.plan, tile)
            abft.batch_verify(B.plan)
            reps.append(B.reports())
        for q in range(len(shapes)):
            assert torch.equal(pads[0].C[q], pads[1].C[q]), (tile, q)
            for rp in reps:
                assert rp[q].n_flag_c == 0 and rp[q].n_flag_r == 0, (tile, q)
    clean = [[c.clone() for c in B.C] for B in pads]
    for run, q in enumerate([0, 1, 2, 3, 2]):
        m, n, k, br, bc = shapes[q]
        i, j, bit = synth.flip_site(SEED + 51, run, m + br, n + bc, 24, 30)
        note(f"flip problem {q} ({i},{j}) bit {bit}")
        got = []
        for B, cl in zip(pads, clean):
            B.C[q].copy_(cl[q])
            abft.inject_flip(B.probs[q], B.C[q], i, j, bit)
            abft.batch_verify(B.plan)
            rep = B.reports()[q]
            loc = abft.classify(B.probs[q], rep)
            got.append((sorted((a, b) for a, b, _, _ in rep.flags_c()), sorted((a, b) for a, b, _, _ in rep.flags_r()),
                        (loc.cls, loc.i, loc.j)))
            B.C[q].copy_(cl[q])
        assert got[0] == got[1], (q, i, j, bit, got)


def test_batch_same_sign_operands_verify_clean(dev):
    """Operands of one sign (|uniform|) over the batch's shape range up to k =
    2048: the carried checksum rows run on the matrix cores (hi + mid + lo),
    so their accumulation errors have one sign too; every relation passes."""
    shapes = [(2048, 2048, 2048, 32, 1), (1024, 2048, 2048, 32, 32), (512, 640, 1536, 32, 1), (96, 200, 2048, 32, 8)]
    B = abft.Batch(shapes, device=dev, tau_mode=abft.ABFT_TAU_STAT, lam=LAMBDA)
    for q, (m, n, k, br, bc) in enumerate(shapes):
        abft.fill_uniform(abft.ABFT_F32, m, k, k, 0, SEED + 60 + q, synth.STREAM_A, B.A32[q])
        abft.fill_uniform(abft.ABFT_F32, k, n, k, 1, SEED + 60 + q, synth.STREAM_B, B.Bt32[q])
        B.A32[q].abs_()
        B.Bt32[q].abs_()
    abft.batch_quantize_encode(B.plan)
    for tile in (0, 3):
        abft.batch_gemm(B.plan, tile)
        abft.batch_verify(B.plan)
        reps = B.reports()
        note(f"same-sign batch, tile {tile}: max |D|/tau " +
             " ".join(f"{max(r.max_ratio_c, r.max_ratio_r):.3f}" for r in reps))
        for q, r in enumerate(reps):
            assert r.n_flag_c == 0 and r.n_flag_r == 0, (tile, q, r.max_ratio_c, r.max_ratio_r)


def test_batch_padded_operand_rows(dev, orc):
    """Operand rows padded to 64 elements (lda = ldb > k, every bfloat16 row on
    a 128-byte line): the quantized rows are bit-exact and nothing is written
    past k; C equals the unpadded batch's bit for bit (the same products in
    the same k order) and lies within the oracle's bound; verification is
    clean for the uniform and the per-problem launches."""
    shapes = [(64, 96, 72, 32, 1), (96, 64, 200, 4, 1), (40, 48, 136, 8, 2), (128, 132, 520, 32, 2),
              (66, 70, 1032, 1, 2), (256, 320, 64, 32, 1)]
    note(f"padded batch of {len(shapes)} problems")
    Bp = abft.Batch(shapes, device=dev, tau_mode=abft.ABFT_TAU_STAT, lam=LAMBDA, ld_align=64)
    Bu = abft.Batch(shapes, device=dev, tau_mode=abft.ABFT_TAU_STAT, lam=LAMBDA)
    refs = []
    for q, (m, n, k, br, bc) in enumerate(shapes):
        assert Bp.lda[q] % 64 == 0 and Bp.lda[q] >= k and Bp.A[q].stride(0) == Bp.lda[q]
        A32 = synth.uniform(SEED + 50 + q, synth.STREAM_A, m, k, np.float32)
        B32 = synth.uniform(SEED + 50 + q, synth.STREAM_B, k, n, np.float32)
        for Bx in (Bp, Bu):
            Bx.A32[q].copy_(torch.from_numpy(A32))
            Bx.Bt32[q].copy_(torch.from_numpy(np.ascontiguousarray(B32.T)))
        Aq, Bq = orc.to_bf16_bits(A32), orc.to_bf16_bits(B32)
        Af, Bf = orc.encode(orc.bf16_bits_to_f64(Aq), orc.bf16_bits_to_f64(Bq), br, bc, store_f32=True)
        C32 = orc.gemm(Af, Bf).astype(np.float32)
        bound = k * U32 * (np.abs(Af) @ np.abs(Bf)) + U32 * np.abs(C32)
        refs.append((Aq, Bq, C32, bound))
    for tile in (0, abft.ABFT_BATCH_MIXED):
        for Bx in (Bp, Bu):
            abft.batch_quantize_encode(Bx.plan)
            abft.batch_gemm(Bx.plan, tile)
            abft.batch_verify(Bx.plan)
        reps = Bp.reports()
        for q, (m, n, k, br, bc) in enumerate(shapes):
            note(f"padded problem {q} {shapes[q]} lda {Bp.lda[q]} tile {tile}")
            Aq, Bq, C32, bound = refs[q]
            a = Bp.A[q].cpu().view(torch.int16).numpy().view(np.uint16)
            b = Bp.Bt[q].cpu().view(torch.int16).numpy().view(np.uint16)
            assert np.array_equal(a, Aq) and np.array_equal(b, np.ascontiguousarray(Bq.T))
            ld = Bp.lda[q]
            for t, rows in ((Bp.A[q], m), (Bp.Bt[q], n)):
                full = t.as_strided((rows, ld), (ld, 1))
                assert not full[:, k:].view(torch.int16).any(), "written past k"
            assert torch.equal(Bp.C[q], Bu.C[q]), q
            err = np.abs(Bp.C[q].cpu().numpy().astype(np.float64) - C32)
            assert np.all(err <= bound * 1.01 + 1e-30), (q, err.max())
            assert reps[q].n_flag_c == 0 and reps[q].n_flag_r == 0, (q, reps[q].max_ratio_c, reps[q].max_ratio_r)
