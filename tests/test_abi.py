"""CPU tests of the C-ABI library: it loads without a GPU, exports every
symbol include/abft.h declares, rejects bad arguments before any launch, and
its host-side classification takes the oracle's decisions on the same reports."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_0806_3121_amd import abft, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NULL_STREAM = None


def header_functions():
    src = open(os.path.join(ROOT, "include", "abft.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(abft_\w+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = abft.lib()
    names = header_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(L, name), name


def test_struct_sizes_match_header_layout():
    assert C.sizeof(abft.abft_problem) == 4 + 4 + 8 * 8 + 8 * 2
    assert C.sizeof(abft.abft_flag) == 32
    assert C.sizeof(abft.abft_report) == 8 * 6 + 8 * 2 + 2 * 64 * 32
    assert C.sizeof(abft.abft_location) == 24
    assert C.sizeof(abft.abft_fault) == 24


def _call(name, *args):
    return getattr(abft.lib(), name)(*args)


@pytest.mark.parametrize("field,value", [("m", 0), ("br", 3), ("bc", 7), ("k", -1), ("dtype", 9), ("tau_mode", 5),
                                         ("br", 512)])
def test_bad_problem_rejected_before_launch(field, value):
    p = abft.problem(abft.ABFT_F64, 256, 256, 256, 1, 1)
    setattr(p, field, value)
    fake = C.c_void_p(256)     # never dereferenced: the checks fail first
    assert abft.workspace_size(p) == 0
    assert _call("abft_gemm", C.byref(p), fake, fake, fake, None, 0, 0, NULL_STREAM) == abft.ABFT_E_ARG


BIG = 1 << 40      # a workspace size no problem here exceeds (the pointers are never dereferenced)


def test_layout_and_alignment_rejected():
    fake = C.c_void_p(256)
    p = abft.problem(abft.ABFT_F64, 256, 256, 256, 1, 1, lda=255)
    assert _call("abft_encode", C.byref(p), fake, fake, fake, BIG, NULL_STREAM) == abft.ABFT_E_ARG
    p = abft.problem(abft.ABFT_F64, 256, 256, 256, 1, 1, ldc=256)          # < n + bc
    assert _call("abft_gemm", C.byref(p), fake, fake, fake, None, 0, 0, NULL_STREAM) == abft.ABFT_E_ARG
    p = abft.problem(abft.ABFT_F64, 256, 256, 256, 1, 1)
    assert _call("abft_gemm", C.byref(p), C.c_void_p(8), fake, fake, None, 0, 0, NULL_STREAM) == abft.ABFT_E_ARG
    assert _call("abft_gemm", C.byref(p), fake, fake, fake, None, 0, 8, NULL_STREAM) == abft.ABFT_E_ARG  # unknown flag
    assert _call("abft_encode", C.byref(p), fake, fake, None, BIG, NULL_STREAM) == abft.ABFT_E_WORKSPACE
    p = abft.problem(abft.ABFT_F64, 256, 256, 251, 1, 1, lda=252, ldb=252)  # k*8 not a multiple of 16
    assert _call("abft_encode", C.byref(p), fake, fake, fake, BIG, NULL_STREAM) == abft.ABFT_E_ARG


@pytest.mark.parametrize("dt,b", [(abft.ABFT_F64, 1), (abft.ABFT_F64, 64), (abft.ABFT_F32, 1), (abft.ABFT_BF16, 1),
                                  (abft.ABFT_FP8_E4M3, 4)])
def test_short_workspace_rejected_before_launch(dt, b):
    """Every call that takes a workspace refuses one smaller than
    abft_workspace_size (or none) before anything is queued."""
    fake = C.c_void_p(256)
    p = abft.problem(dt, 256, 256, 256, b, b)
    need = abft.workspace_size(p)
    assert need > 0
    rect = abft.abft_rect(0, 0, 1, 1)
    for short in (need - 1, 0):
        ws = None if short == 0 else fake
        calls = {
            "encode": lambda: _call("abft_encode", C.byref(p), fake, fake, ws, short, NULL_STREAM),
            "gemm": lambda: _call("abft_gemm", C.byref(p), fake, fake, fake, ws, short, 0, NULL_STREAM),
            "verify": lambda: _call("abft_verify", C.byref(p), fake, C.byref(rect), 0, ws, short, None, NULL_STREAM),
        }
        if b == 1:
            calls["gemm_fused"] = lambda: _call("abft_gemm", C.byref(p), fake, fake, fake, ws, short, abft.ABFT_FUSED,
                                                NULL_STREAM)
            calls["verify_fused"] = lambda: _call("abft_verify_fused", C.byref(p), fake, ws, short, None, NULL_STREAM)
        if dt in (abft.ABFT_BF16, abft.ABFT_FP8_E4M3):
            calls["quantize"] = lambda: _call("abft_quantize", C.byref(p), 0, fake, 256, fake, ws, short, NULL_STREAM)
            calls["quantize_encode"] = lambda: _call("abft_quantize_encode", C.byref(p), fake, 256, fake, 256, fake,
                                                     fake, ws, short, NULL_STREAM)
        for name, call in calls.items():
            if dt in (abft.ABFT_F64, abft.ABFT_F32) and name == "gemm" and ws is None:
                continue                                          # optional for these types: nothing to refuse
            assert call() == abft.ABFT_E_WORKSPACE, (name, short)
    if dt == abft.ABFT_F64:
        prev = abft.problem(abft.ABFT_F64, 256, 256, 256, b, b, ldc=320)      # the next A_f is this C_f
        q = abft.problem(abft.ABFT_F64, 256, 128, 256, b, b, lda=320)
        chained = lambda wb, pb: _call("abft_encode_chained", C.byref(q), fake, fake, fake, wb, C.byref(prev), fake,
                                       pb, NULL_STREAM)
        assert chained(abft.workspace_size(q) - 1, BIG) == abft.ABFT_E_WORKSPACE
        assert chained(BIG, abft.workspace_size(prev) - 1) == abft.ABFT_E_WORKSPACE


def test_panel_range_and_dtype_rejected():
    fake = C.c_void_p(256)
    p = abft.problem(abft.ABFT_F64, 256, 256, 256, 1, 1)
    panel = lambda k0, k1, flags=0: _call("abft_gemm_panel", C.byref(p), fake, fake, fake, k0, k1, flags, NULL_STREAM)
    assert panel(0, 0) == abft.ABFT_E_ARG            # empty panel
    assert panel(128, 64) == abft.ABFT_E_ARG         # k1 < k0
    assert panel(0, 257) == abft.ABFT_E_ARG          # beyond k
    assert panel(-2, 64) == abft.ABFT_E_ARG
    assert panel(1, 64) == abft.ABFT_E_ARG           # panel start not on a 16-byte boundary
    assert panel(0, 63) == abft.ABFT_E_ARG           # panel end not on a 16-byte boundary
    assert panel(0, 64, 4) == abft.ABFT_E_ARG        # unknown flag
    p = abft.problem(abft.ABFT_BF16, 256, 256, 256, 1, 1)
    assert panel(0, 64) == abft.ABFT_E_UNSUPPORTED


def test_fused_flags_and_fault_hook_rejected():
    fake = C.c_void_p(256)
    p = abft.problem(abft.ABFT_F64, 256, 256, 256, 1, 1)
    gemm = lambda q, flags, ws=fake: _call("abft_gemm", C.byref(q), fake, fake, fake, ws, BIG, flags, NULL_STREAM)
    assert gemm(p, abft.ABFT_FUSED | abft.ABFT_PLAIN) == abft.ABFT_E_ARG
    assert gemm(p, abft.ABFT_FUSED, None) == abft.ABFT_E_WORKSPACE
    q = abft.problem(abft.ABFT_F64, 256, 256, 256, 64, 64)
    assert gemm(q, abft.ABFT_FUSED) == abft.ABFT_E_UNSUPPORTED
    q = abft.problem(abft.ABFT_F64, 256, 256, 256, 64, 64)
    assert _call("abft_verify_fused", C.byref(q), fake, fake, BIG, None, NULL_STREAM) == abft.ABFT_E_UNSUPPORTED

    def fault(prob, i, j, bit):
        f = abft.abft_fault(i, j, bit)
        return _call("abft_gemm_fault", C.byref(prob), fake, fake, fake, fake, BIG, 0, C.byref(f), NULL_STREAM)
    assert fault(p, 256, 0, 3) == abft.ABFT_E_ARG          # rows of C only (the carried row is not the kernel's)
    assert fault(p, 0, -1, 3) == abft.ABFT_E_ARG
    assert fault(p, 0, 0, 64) == abft.ABFT_E_ARG
    p32 = abft.problem(abft.ABFT_F32, 256, 256, 256, 1, 1)
    assert fault(p32, 0, 0, 32) == abft.ABFT_E_ARG


def test_describe_gemm_names_kernels_and_tiles():
    """Host-only: the kernel and tile the product dispatch picks, per dtype and shape."""
    d = lambda dt, m, n, k, b, flags=0: abft.describe_gemm(abft.problem(dt, m, n, k, b, b), flags)
    assert d(abft.ABFT_F64, 8192, 8192, 8192, 1024) == "k_gemm_mfma2 f64 96x96 on 9216x9216 k=8192"
    assert d(abft.ABFT_F64, 8192, 8192, 8192, 1) == ("k_gemm_mfma2 f64 128x128 on 8192x8192 k=8192"
                                                     " + k_sliver carried rows + k_sliver carried columns")
    assert d(abft.ABFT_F64, 8192, 8192, 8192, 1, abft.ABFT_PLAIN) == "k_gemm_mfma2 f64 128x128 on 8192x8192 k=8192"
    assert d(abft.ABFT_F64, 256, 256, 250, 64) == "k_gemm_mfma f64 96x96 on 320x320 k=250"
    # one checksum row over 16384 or more operand rows: the multi-row carried-block kernel
    assert d(abft.ABFT_F32, 16384, 8192, 32768, 1) == ("k_gemm_mfma2 f32 256x128 on 16384x8192 k=32768"
                                                       " + k_sliver carried rows + k_sliver1 carried columns")
    assert d(abft.ABFT_BF16, 16384, 16384, 16384, 1) == (
        "k_gemm_lowp2 bf16 256x256 on 16384x16384 k=16384"
        " + k_sliver1 carried rows + k_sliver corner + k_sliver1 carried columns")
    assert d(abft.ABFT_FP8_E4M3, 300, 260, 528, 1, abft.ABFT_PLAIN) == "k_gemm_lowp fp8 128x128 on 300x260 k=528"
    p = abft.problem(abft.ABFT_F64, 256, 256, 256, 1, 1)
    buf = C.create_string_buffer(16)
    assert _call("abft_describe_gemm", C.byref(p), 0, buf, 16) == abft.ABFT_E_ARG      # too short
    assert buf.value == b"k_gemm_mfma2 f6"                                             # truncated, terminated
    assert _call("abft_describe_gemm", C.byref(p), 8, buf, 16) == abft.ABFT_E_ARG      # unknown flag
    assert _call("abft_describe_gemm", C.byref(p), 0, None, 16) == abft.ABFT_E_ARG
    bad = abft.problem(abft.ABFT_F64, 256, 256, 256, 3, 1)                              # br does not divide m
    assert _call("abft_describe_gemm", C.byref(bad), 0, C.create_string_buffer(256), 256) == abft.ABFT_E_ARG


def test_quantize_encode_rejected():
    fake = C.c_void_p(256)
    qe = lambda q, a32=fake, lda=256, b32=fake, ldb=256, ws=fake: _call(
        "abft_quantize_encode", C.byref(q), a32, lda, b32, ldb, fake, fake, ws, BIG, NULL_STREAM)
    p = abft.problem(abft.ABFT_BF16, 256, 256, 256, 1, 1)
    assert qe(abft.problem(abft.ABFT_F64, 256, 256, 256, 1, 1)) == abft.ABFT_E_UNSUPPORTED
    assert qe(p, a32=C.c_void_p(260)) == abft.ABFT_E_ARG        # binary32 rows not 16-byte aligned
    assert qe(p, b32=None) == abft.ABFT_E_ARG
    assert qe(p, lda=255) == abft.ABFT_E_ARG                    # shorter than k
    assert qe(p, ldb=258) == abft.ABFT_E_ARG                    # not a multiple of 4
    assert qe(p, ws=None) == abft.ABFT_E_WORKSPACE


def test_block_cyclic_arguments_rejected():
    fake = C.c_void_p(256)
    call = lambda rows, cols, es, nb, P, Q, ld=4096: _call("abft_block_cyclic_stack", fake, ld, rows, cols, es, nb,
                                                           P, Q, fake, ld, NULL_STREAM)
    assert call(512, 512, 3, 64, 2, 2) == abft.ABFT_E_ARG          # element size
    assert call(500, 512, 8, 64, 2, 2) == abft.ABFT_E_ARG          # rows not whole blocks per process
    assert call(512, 500, 8, 64, 2, 2) == abft.ABFT_E_ARG
    assert call(512, 512, 8, 64, 0, 2) == abft.ABFT_E_ARG
    assert call(512, 512, 8, 64, 2, 2, ld=500) == abft.ABFT_E_ARG  # leading dimension below cols
    assert _call("abft_block_cyclic_unstack", fake, 512, 512, 512, 8, 64, 2, 2, None, 512,
                 NULL_STREAM) == abft.ABFT_E_ARG


def test_unrecoverable_and_bad_rects_rejected():
    fake = C.c_void_p(256)
    p = abft.problem(abft.ABFT_F64, 256, 256, 256, 1, 1)
    r = abft.abft_rect(0, 0, 64, 64)
    assert _call("abft_recover_block", C.byref(p), fake, r, 0, NULL_STREAM) == abft.ABFT_E_UNRECOVERABLE
    assert _call("abft_recover_block", C.byref(p), fake, r, 1, NULL_STREAM) == abft.ABFT_E_UNRECOVERABLE
    p = abft.problem(abft.ABFT_F64, 256, 256, 256, 64, 64)
    assert _call("abft_recover_block", C.byref(p), fake, abft.abft_rect(300, 0, 64, 64), 0, NULL_STREAM) == abft.ABFT_E_ARG
    assert _call("abft_inject_flip", C.byref(p), fake, 0, 0, 64, NULL_STREAM) == abft.ABFT_E_ARG
    assert _call("abft_inject_flip", C.byref(p), fake, 320, 0, 3, NULL_STREAM) == abft.ABFT_E_ARG


def test_correct_refuses_multi_and_ignores_clean():
    fake = C.c_void_p(256)
    p = abft.problem(abft.ABFT_F64, 256, 256, 256, 1, 1)
    loc = abft.abft_location(abft.ABFT_CLS_MULTI, 0, 0, 0)
    assert _call("abft_correct", C.byref(p), fake, C.byref(loc), NULL_STREAM) == abft.ABFT_E_UNCORRECTABLE
    loc = abft.abft_location(abft.ABFT_CLS_CLEAN, 0, -1, -1)
    assert _call("abft_correct", C.byref(p), fake, C.byref(loc), NULL_STREAM) == abft.ABFT_OK


# ---------------------------------------------------------------- classification vs the oracle
def _to_lib_report(orep):
    rep = abft.abft_report()
    rep.n_flag_c, rep.n_flag_r = orep.n_flag_c, orep.n_flag_r
    fc, fr = orep.flags_c(), orep.flags_r()
    # the device writes flags in arbitrary order: feed them reversed
    for q, (a, b, d, t) in enumerate(reversed(fc)):
        rep.flag_c[q] = abft.abft_flag(a, b, d, t)
    for q, (a, b, d, t) in enumerate(reversed(fr)):
        rep.flag_r[q] = abft.abft_flag(a, b, d, t)
    return rep


@pytest.mark.parametrize("m,n,br,bc", [(8, 8, 1, 1), (8, 12, 2, 3), (16, 16, 4, 4)])
def test_classification_matches_oracle(orc, m, n, br, bc):
    k = 5
    A = synth.uniform_ints(1, 0, m, k, -4, 4)
    B = synth.uniform_ints(1, 1, k, n, -4, 4)
    Af, Bf, Cf = orc.protected_product(A, B, br, bc)
    p = abft.problem(abft.ABFT_F64, m, n, k, br, bc, tau_mode=abft.ABFT_TAU_EXACT)
    tc = np.zeros((br, n + bc))
    tr = np.zeros((m + br, bc))
    cases = []
    for i in range(m + br):
        for j in range(n + bc):
            cases.append(([(i, j, 3.0)], None))
    cases.append(([(0, 0, 1.0), (1, 1, 1.0)], None))
    cases.append(([(0, 0, 1.0), (0, 1, 2.0)], None))
    rect = (0, 0, br, bc)
    cases.append(([(br, bc, 1.0)], [rect]))
    cases.append(([(m - 1, 0, 1.0)], [rect]))
    cases.append(([(0, n - 1, 1.0)], [rect]))
    for errs, known in cases:
        Cx = Cf.copy()
        for (i, j, d) in errs:
            Cx[i, j] += d
        if known:
            i0, j0, h, w = known[0]
            Cx[i0:i0 + h, j0:j0 + w] = 0
        _, _, orep = orc.verify(Cx, m, n, br, bc, tc, tr, erasures=known)
        ocls, oi, oj, od = orc.classify(orep, m, n, br, bc, erasures=known)
        loc = abft.classify(p, _to_lib_report(orep), known=known)
        assert (loc.cls, loc.i, loc.j, loc.dir) == (ocls, oi, oj, od), (errs, known)


def test_batch_setup_rejects_before_any_copy():
    good = abft.problem(abft.ABFT_BF16, 64, 32, 16, 32, 1, ldc=36, tau_mode=abft.ABFT_TAU_STAT)
    assert abft.batch_workspace_size([good]) > 0
    bad = [
        abft.problem(abft.ABFT_F64, 64, 32, 16, 32, 1, ldc=33),                                # dtype
        abft.problem(abft.ABFT_BF16, 64, 32, 16, 32, 1, ldc=36, tau_mode=abft.ABFT_TAU_DET),   # tau mode
        abft.problem(abft.ABFT_BF16, 64, 30, 16, 32, 3, ldc=36, tau_mode=abft.ABFT_TAU_STAT),  # bc does not divide 256
        abft.problem(abft.ABFT_BF16, 64, 32, 12, 32, 1, ldc=36, tau_mode=abft.ABFT_TAU_STAT),  # k % 8
        abft.problem(abft.ABFT_BF16, 64, 32, 16, 32, 1, ldc=32, tau_mode=abft.ABFT_TAU_STAT),  # ldc < n + bc
    ]
    for p in bad:
        assert abft.batch_workspace_size([good, p]) == 0
    # fake, never dereferenced device addresses: each call must fail on the host
    fake = abft.abft_batch_item(None, None, 0x10000, 0x20000, 0x30000)
    L = abft.lib()
    plan = abft.abft_batch_plan()
    probs = (abft.abft_problem * 1)(good)
    items = (abft.abft_batch_item * 1)(fake)
    need = abft.batch_workspace_size([good])
    assert L.abft_batch_setup(probs, items, 1, C.c_void_p(0x40000), need - 1, C.byref(plan)) == abft.ABFT_E_WORKSPACE
    assert L.abft_batch_setup(probs, items, 0, C.c_void_p(0x40000), need, C.byref(plan)) == abft.ABFT_E_ARG
    misaligned = (abft.abft_batch_item * 1)(abft.abft_batch_item(None, None, 0x10008, 0x20000, 0x30000))
    assert L.abft_batch_setup(probs, misaligned, 1, C.c_void_p(0x40000), need, C.byref(plan)) == abft.ABFT_E_ARG
    assert L.abft_batch_gemm(None, 0, 0, None) == abft.ABFT_E_ARG
    assert L.abft_batch_verify(None, None) == abft.ABFT_E_ARG


def test_batch_tile_cache_round_trip(tmp_path):
    """Host only: costs stored per bucket (m, n by 128, k by powers of two,
    br, bc, arch) and looked up again; a bucket's shape is the least summed
    cost of its problems; other architectures and unseen buckets are absent."""
    P = lambda m, n, k: abft.problem(abft.ABFT_BF16, m, n, k, 32, 1, ldc=n + 4, tau_mode=abft.ABFT_TAU_STAT)
    probs = [P(64, 96, 100), P(96, 128, 128), P(1024, 2048, 1024), P(640, 64, 300)]
    costs = [[4.0, 3.0, 2.0, 1.0], [1.0, 9.0, 9.0, 9.0], [1.0, 2.0, 3.0, 4.0], [5.0, 1.0, 5.0, 5.0]]
    path = str(tmp_path / "tiles.txt")
    abft.batch_cache_store(path, probs, costs, arch="gfx950")
    found, tiles = abft.batch_cache_lookup(path, probs, arch="gfx950")
    # problems 0 and 1 share a bucket (m, n <= 128, k in (64, 128]): summed costs [5, 12, 11, 10] -> shape 0
    assert found == 4 and tiles == [0, 0, 0, 1]
    found, tiles = abft.batch_cache_lookup(path, probs, arch="gfx942")
    assert found == 0 and tiles == [-1] * 4
    found, tiles = abft.batch_cache_lookup(path, [P(2048, 2048, 2048)], arch="gfx950")
    assert found == 0 and tiles == [-1]
    # a new measurement of a bucket replaces the old one, other buckets stay
    abft.batch_cache_store(path, [P(1024, 2048, 1024)], [[9.0, 9.0, 9.0, 1.0]], arch="gfx950")
    found, tiles = abft.batch_cache_lookup(path, probs, arch="gfx950")
    assert found == 4 and tiles == [0, 0, 3, 1]


# ---------------------------------------------------------------- weighted f-checksums
def test_weighted_struct_sizes():
    assert C.sizeof(abft.abft_wproblem) == C.sizeof(abft.abft_problem) + 4 + 4 + 8 + 8
    assert C.sizeof(abft.abft_wgroup) == 16 + 2 * 8 * abft.ABFT_WMAX
    assert C.sizeof(abft.abft_wreport) == 8 * 6 + 2 * 64 * C.sizeof(abft.abft_wgroup)


def _wp(**kw):
    args = dict(m=256, n=192, k=128, br=64, bc=64, wr=np.ones((2, 4)), wc=np.ones((2, 3)))
    args.update(kw)
    return abft.wproblem(**args)


def test_weighted_bad_problems_rejected_before_launch():
    fake = C.c_void_p(256)
    assert abft.wworkspace_size(_wp()) > 0
    assert abft.wworkspace_size(_wp(dtype=abft.ABFT_F32)) > 0
    bad = [
        (_wp(wr=np.ones((5, 4))), abft.ABFT_E_ARG),                   # fr > ABFT_WMAX
        (_wp(dtype=abft.ABFT_F32, k=126), abft.ABFT_E_ARG),          # binary32 rows: k a multiple of 4
        (_wp(wr=np.array([[1.0, np.nan, 1.0, 1.0]])), abft.ABFT_E_ARG),  # weights must be finite
        (_wp(k=127), abft.ABFT_E_ARG),                               # k odd: rows not 16-byte multiples
        (_wp(ldc=200), abft.ABFT_E_ARG),                             # ldc < n + fc*bc
        (_wp(tau_mode=abft.ABFT_TAU_STAT), abft.ABFT_E_UNSUPPORTED),
    ]
    for wp, want in bad:
        assert abft.wworkspace_size(wp) == 0
        assert _call("abft_wencode", C.byref(wp), fake, fake, fake, BIG, NULL_STREAM) == want
    wp = _wp()
    wp.p.dtype = abft.ABFT_BF16
    assert _call("abft_wgemm", C.byref(wp), fake, fake, fake, NULL_STREAM) == abft.ABFT_E_UNSUPPORTED
    wp = _wp()
    assert _call("abft_wencode", C.byref(wp), C.c_void_p(8), fake, fake, BIG, NULL_STREAM) == abft.ABFT_E_ARG
    assert _call("abft_wencode", C.byref(wp), fake, fake, None, BIG, NULL_STREAM) == abft.ABFT_E_WORKSPACE
    need = abft.wworkspace_size(wp)
    assert _call("abft_wencode", C.byref(wp), fake, fake, fake, need - 1, NULL_STREAM) == abft.ABFT_E_WORKSPACE
    assert _call("abft_wsetup", C.byref(wp), fake, need - 1) == abft.ABFT_E_WORKSPACE
    assert _call("abft_wverify", C.byref(wp), fake, None, 0, fake, need - 1, None, NULL_STREAM) == abft.ABFT_E_WORKSPACE
    one = (abft.abft_location * 1)(abft.abft_location(abft.ABFT_CLS_DATA, 0, 0, 0))
    assert _call("abft_wcorrect", C.byref(wp), fake, one, 1, fake, need - 1, NULL_STREAM) == abft.ABFT_E_WORKSPACE
    blocks = (C.c_int32 * 3)(0, 1, 2)
    # three data blocks lost with two checksums: refused on the host
    assert _call("abft_wrecover", C.byref(wp), fake, abft.ABFT_DIR_COL, blocks, 3, 0, 10, fake, BIG,
                 NULL_STREAM) == abft.ABFT_E_UNRECOVERABLE
    assert _call("abft_wrecover", C.byref(wp), fake, abft.ABFT_DIR_COL, blocks, 3, 0, 10, fake, need - 1,
                 NULL_STREAM) == abft.ABFT_E_WORKSPACE
    # a singular system: two equal weight columns
    ws = _wp(wr=np.array([[1.0, 1.0, 1.0, 1.0], [1.0, 2.0, 2.0, 3.0]]))
    two = (C.c_int32 * 2)(1, 2)
    assert _call("abft_wrecover", C.byref(ws), fake, abft.ABFT_DIR_COL, two, 2, 0, 10, fake, BIG,
                 NULL_STREAM) == abft.ABFT_E_UNRECOVERABLE
    assert _call("abft_wrecover", C.byref(wp), fake, abft.ABFT_DIR_COL, two, 2, 0, 1000, fake, BIG,
                 NULL_STREAM) == abft.ABFT_E_ARG                      # beyond the columns of C_f


def _to_wreport(orep, fr, fc):
    rep = abft.abft_wreport()
    rep.n_fail_c, rep.n_fail_r = len(orep["col"]), len(orep["row"])
    # the device writes groups in arbitrary order: feed them reversed
    for q, (a, b, d, t) in enumerate(reversed(orep["col"][:64])):
        rep.col[q].a, rep.col[q].b = a, b
        for r in range(fr):
            rep.col[q].d[r], rep.col[q].tau[r] = d[r], t[r]
    for q, (a, b, d, t) in enumerate(reversed(orep["row"][:64])):
        rep.row[q].a, rep.row[q].b = a, b
        for c in range(fc):
            rep.row[q].d[c], rep.row[q].tau[c] = d[c], t[c]
    return rep


@pytest.mark.parametrize("fr,fc", [(2, 2), (1, 3), (3, 1), (1, 1)])
def test_weighted_location_matches_oracle(orc, fr, fc):
    """abft_wlocate (host C++) takes the oracle's decisions on the oracle's own
    reports: every element of a small C_f, several exponent bits, and pairs."""
    from oracle import weighted as wo
    m, n, k, br, bc = 8, 6, 4, 2, 3
    A = synth.uniform_ints(4, synth.STREAM_A, m, k, -8, 8)
    B = synth.uniform_ints(4, synth.STREAM_B, k, n, -8, 8)
    Wr = 0.5 + (synth.uniform(4, synth.STREAM_X, fr, m // br) + 1) / 2
    Wc = 0.5 + (synth.uniform(4, synth.STREAM_PICK, fc, n // bc) + 1) / 2
    Af, Bf, Cf = wo.wproduct(A, B, Wr, Wc, br, bc)
    tc, tr = wo.wtau_det(Af, Bf, m, n, br, bc, Wr, Wc)
    wp = abft.wproblem(m, n, k, br, bc, Wr, Wc)
    M, N = Cf.shape
    cases = [[(x, y, bit)] for x in range(M) for y in range(N) for bit in (45, 52, 61)]
    cases += [[(0, 0, 60), (M - 1, N - 1, 58)], [(1, 2, 55), (3, 2, 55)], [(2, 1, 57), (2, 4, 57)]]
    checked = 0
    for case in cases:
        Cx = Cf.copy()
        for (x, y, bit) in case:
            v = np.array([Cx[x, y]]).view(np.uint64) ^ np.uint64(1 << bit)
            Cx[x, y] = v.view(np.float64)[0]
        orep = wo.wverify(Cx, m, n, br, bc, Wr, Wc, tc, tr)
        want = wo.wlocate(orep["col"], orep["row"], m, n, br, bc, Wr, Wc)
        st, got = abft.wlocate(wp, _to_wreport(orep, fr, fc))
        got = [(l.cls, l.dir, l.i, l.j) if l.cls != abft.ABFT_CLS_MULTI else (l.cls, l.dir) for l in got]
        want = [w if w[0] != wo.MULTI else (w[0], w[1]) for w in want]
        assert got == want, (case, got, want)
        assert (st == abft.ABFT_E_UNCORRECTABLE) == any(w[0] == wo.MULTI for w in want)
        checked += 1
    assert checked == len(cases)
