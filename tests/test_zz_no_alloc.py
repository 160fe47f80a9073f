"""GPU test of abft_verify_noalloc, the verification entry point that
allocates nothing (its scratch is a static device array of the library):
through the C ABI, its report equals abft_verify's on the same C_f -- counts,
flagged relations with their residuals and thresholds, and the largest
ratios -- on consecutive calls, each later one on a smaller problem than the
one before, so stale contents of the shared array from a larger call cannot
go unnoticed.  Clean products and products with one flipped element."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_0806_3121_amd import abft, synth  # noqa: E402

pytestmark = pytest.mark.gpu

SEED = synth.BASE_SEED + 77


def note(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    abft.lib()
    return torch.device("cuda:0")


def product(dev, dt, m, n, k, b):
    mode = abft.ABFT_TAU_DET if dt == abft.ABFT_F64 else abft.ABFT_TAU_STAT
    P = abft.Protected(dt, m, n, k, b, b, device=dev, tau_mode=mode, lam=10.0)
    abft.fill_uniform(dt, m, k, k, 0, SEED, synth.STREAM_A, P.A)
    abft.fill_uniform(dt, k, n, k, 1, SEED, synth.STREAM_B, P.Bt)
    P.encode()
    P.gemm()
    return P


def same_report(a, b):
    assert (a.n_flag_c, a.n_flag_r, a.n_excl_c, a.n_excl_r, a.n_nonfinite, a.status) == \
        (b.n_flag_c, b.n_flag_r, b.n_excl_c, b.n_excl_r, b.n_nonfinite, b.status)
    assert a.max_ratio_c == b.max_ratio_c and a.max_ratio_r == b.max_ratio_r
    assert a.flags_c() == b.flags_c() and a.flags_r() == b.flags_r()


# largest first: each call's scratch is smaller than the one before (one path each:
# the one-pass block check, the b = 1 tile partials, the two-level partial sums)
CASES = [
    (abft.ABFT_F64, 4096, 4096, 256, 512),
    (abft.ABFT_F32, 2048, 1536, 512, 1),
    (abft.ABFT_F64, 1024, 768, 128, 1),
    (abft.ABFT_F64, 512, 512, 96, 64),
    (abft.ABFT_F64, 256, 192, 64, 16),
]


def test_noalloc_verify_equals_verify(dev):
    host = abft.new_report_buffer()
    for (dt, m, n, k, b) in CASES:
        note(f"noalloc verify dtype={dt} m={m} n={n} k={k} b={b}")
        P = product(dev, dt, m, n, k, b)
        for flip in (None, (m // 3, n // 2 + 1, 60 if dt == abft.ABFT_F64 else 28)):
            if flip:
                abft.inject_flip(P.p, P.C, *flip)
            want = P.verify()
            abft.verify_noalloc(P.p, P.C, P.ws, host_out=host)
            torch.cuda.synchronize()
            got = abft.read_report(host)
            same_report(got, want)
            if flip:
                assert got.n_flag_c == 1 and got.n_flag_r == 1
                loc = abft.classify(P.p, got)
                assert (loc.cls, loc.i, loc.j) == (abft.ABFT_CLS_DATA, flip[0], flip[1])
            else:
                assert got.n_flag_c == 0 and got.n_flag_r == 0
        # with a known erasure: the same relations skipped
        rect = (0, 0, b, b)
        abft.inject_erase(P.p, P.C, rect)
        want = P.verify(known=[rect])
        abft.verify_noalloc(P.p, P.C, P.ws, known=[rect], host_out=host)
        torch.cuda.synchronize()
        same_report(abft.read_report(host), want)


def test_noalloc_refusals(dev):
    P = product(dev, abft.ABFT_F64, 256, 256, 64, 1)
    L = abft.lib()
    p = P.p
    args = lambda ws_bytes, out: (C.byref(p), C.c_void_p(P.C.data_ptr()), None, 0, C.c_void_p(P.ws.data_ptr()),
                                  ws_bytes, out, None)
    host = abft.new_report_buffer()
    assert L.abft_verify_noalloc(*args(P.ws.numel() - 1, C.c_void_p(host.data_ptr()))) == abft.ABFT_E_WORKSPACE
    assert L.abft_verify_noalloc(*args(P.ws.numel(), None)) == abft.ABFT_E_ARG
    # a b = 1 problem whose tile partials exceed the static array
    big = abft.problem(abft.ABFT_F32, 32768, 32768, 16, 1, 1, ldc=32772)
    assert abft.workspace_size(big) > 0
    fake = C.c_void_p(1 << 20)
    assert L.abft_verify_noalloc(C.byref(big), fake, None, 0, fake, 1 << 40, C.c_void_p(host.data_ptr()),
                                 None) == abft.ABFT_E_WORKSPACE
