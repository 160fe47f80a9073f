"""Thin ctypes binding of libabft (include/abft.h): same names, argument
marshalling only.  Device buffers are torch tensors on a ROCm device; every
computation runs in the library's HIP kernels.  There is no CPU fallback: if
the library is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libabft.so")

ABFT_F64, ABFT_F32, ABFT_BF16, ABFT_FP8_E4M3 = 0, 1, 2, 3
ABFT_OK, ABFT_FAULT_DETECTED = 0, 1
ABFT_E_ARG, ABFT_E_HIP, ABFT_E_UNCORRECTABLE, ABFT_E_UNRECOVERABLE, ABFT_E_WORKSPACE, ABFT_E_UNSUPPORTED = \
    -1, -2, -3, -4, -5, -6
ABFT_E_STALE = -7
ABFT_TAU_DET, ABFT_TAU_STAT, ABFT_TAU_EXACT = 0, 1, 2
ABFT_PLAIN = 1
ABFT_ACCUMULATE = 2
ABFT_FUSED = 4
ABFT_CLS_CLEAN, ABFT_CLS_DATA, ABFT_CLS_CHECKSUM, ABFT_CLS_MULTI = 0, 1, 2, 3
ABFT_DIR_COL, ABFT_DIR_ROW = 0, 1
ABFT_MAX_FLAGS = 64


class AbftError(RuntimeError):
    def __init__(self, fn, status, msg):
        super().__init__(f"{fn}: {msg} (status {status})")
        self.status = status


class abft_problem(C.Structure):
    _fields_ = [("dtype", C.c_int32), ("tau_mode", C.c_int32),
                ("m", C.c_int64), ("n", C.c_int64), ("k", C.c_int64),
                ("br", C.c_int64), ("bc", C.c_int64),
                ("lda", C.c_int64), ("ldb", C.c_int64), ("ldc", C.c_int64),
                ("lambda_", C.c_double), ("kappa", C.c_double)]


class abft_rect(C.Structure):
    _fields_ = [("i0", C.c_int64), ("j0", C.c_int64), ("h", C.c_int64), ("w", C.c_int64)]


class abft_flag(C.Structure):
    _fields_ = [("a", C.c_int64), ("b", C.c_int64), ("d", C.c_double), ("tau", C.c_double)]


class abft_report(C.Structure):
    _fields_ = [("n_flag_c", C.c_int64), ("n_flag_r", C.c_int64),
                ("n_excl_c", C.c_int64), ("n_excl_r", C.c_int64),
                ("n_nonfinite", C.c_int64), ("status", C.c_int64),
                ("max_ratio_c", C.c_double), ("max_ratio_r", C.c_double),
                ("flag_c", abft_flag * ABFT_MAX_FLAGS), ("flag_r", abft_flag * ABFT_MAX_FLAGS)]

    def flags_c(self):
        return sorted((f.a, f.b, f.d, f.tau) for f in self.flag_c[:min(self.n_flag_c, ABFT_MAX_FLAGS)])

    def flags_r(self):
        return sorted((f.a, f.b, f.d, f.tau) for f in self.flag_r[:min(self.n_flag_r, ABFT_MAX_FLAGS)])


class abft_location(C.Structure):
    _fields_ = [("cls", C.c_int32), ("dir", C.c_int32), ("i", C.c_int64), ("j", C.c_int64)]


class abft_fault(C.Structure):
    _fields_ = [("i", C.c_int64), ("j", C.c_int64), ("bit", C.c_int32)]


class abft_batch_item(C.Structure):
    _fields_ = [("A32", C.c_void_p), ("Bt32", C.c_void_p), ("A_f", C.c_void_p), ("B_f", C.c_void_p),
                ("C_f", C.c_void_p)]


ABFT_BATCH_TILES = 4      # product tile shapes: 256x256, 256x128, 128x256, 128x128
ABFT_BATCH_MIXED = ABFT_BATCH_TILES   # every problem with its own shape
BATCH_TILE_SHAPES = [(256, 256), (256, 128), (128, 256), (128, 128)]


class abft_batch_plan(C.Structure):
    _fields_ = [("bws", C.c_void_p), ("count", C.c_int32), ("dtype", C.c_int32),
                ("n_tiles", (C.c_int64 * 2) * (ABFT_BATCH_TILES + 1)),
                ("n_work", C.c_int64 * 12),
                ("bytes", C.c_size_t), ("ttime_off", C.c_size_t), ("n_shape", C.c_int32 * ABFT_BATCH_TILES)]


ABFT_WMAX = 4


class abft_wproblem(C.Structure):
    _fields_ = [("p", abft_problem), ("fr", C.c_int32), ("fc", C.c_int32),
                ("wr", C.POINTER(C.c_double)), ("wc", C.POINTER(C.c_double))]


class abft_wgroup(C.Structure):
    _fields_ = [("a", C.c_int64), ("b", C.c_int64), ("d", C.c_double * ABFT_WMAX), ("tau", C.c_double * ABFT_WMAX)]


class abft_wreport(C.Structure):
    _fields_ = [("n_fail_c", C.c_int64), ("n_fail_r", C.c_int64),
                ("n_excl_c", C.c_int64), ("n_excl_r", C.c_int64),
                ("max_ratio_c", C.c_double), ("max_ratio_r", C.c_double),
                ("col", abft_wgroup * ABFT_MAX_FLAGS), ("row", abft_wgroup * ABFT_MAX_FLAGS)]

    def groups_c(self, f):
        g = self.col[:min(self.n_fail_c, ABFT_MAX_FLAGS)]
        return sorted((x.a, x.b, list(x.d[:f]), list(x.tau[:f])) for x in g)

    def groups_r(self, f):
        g = self.row[:min(self.n_fail_r, ABFT_MAX_FLAGS)]
        return sorted((x.a, x.b, list(x.d[:f]), list(x.tau[:f])) for x in g)


_lib = None
_V = C.c_void_p
_Z = C.c_size_t
_P = C.POINTER


def lib():
    """Load libabft.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_0806_3121_amd.build`")
        L = C.CDLL(LIB_PATH)
        sig = {
            "abft_workspace_size": (C.c_size_t, [_P(abft_problem)]),
            "abft_encode": (C.c_int, [_P(abft_problem), _V, _V, _V, _Z, _V]),
            "abft_encode_chained": (C.c_int, [_P(abft_problem), _V, _V, _V, _Z, _P(abft_problem), _V, _Z, _V]),
            "abft_gemm": (C.c_int, [_P(abft_problem), _V, _V, _V, _V, _Z, C.c_uint32, _V]),
            "abft_gemm_fault": (C.c_int, [_P(abft_problem), _V, _V, _V, _V, _Z, C.c_uint32, _P(abft_fault), _V]),
            "abft_gemm_panel": (C.c_int, [_P(abft_problem), _V, _V, _V, C.c_int64, C.c_int64, C.c_uint32, _V]),
            "abft_describe_gemm": (C.c_int, [_P(abft_problem), C.c_uint32, C.c_char_p, C.c_size_t]),
            "abft_quantize_encode": (C.c_int, [_P(abft_problem), _V, C.c_int64, _V, C.c_int64, _V, _V, _V, _Z, _V]),
            "abft_quantize": (C.c_int, [_P(abft_problem), C.c_int, _V, C.c_int64, _V, _V, _Z, _V]),
            "abft_verify": (C.c_int, [_P(abft_problem), _V, _P(abft_rect), C.c_int, _V, _Z, _V, _V]),
            "abft_verify_fused": (C.c_int, [_P(abft_problem), _V, _V, _Z, _V, _V]),
            "abft_verify_noalloc": (C.c_int, [_P(abft_problem), _V, _P(abft_rect), C.c_int, _V, _Z, _V, _V]),
            "abft_classify": (C.c_int, [_P(abft_problem), _P(abft_report), _P(abft_rect), C.c_int,
                                        _P(abft_location)]),
            "abft_correct": (C.c_int, [_P(abft_problem), _V, _P(abft_location), _V]),
            "abft_recover_block": (C.c_int, [_P(abft_problem), _V, abft_rect, C.c_int, _V]),
            "abft_inject_flip": (C.c_int, [_P(abft_problem), _V, C.c_int64, C.c_int64, C.c_int, _V]),
            "abft_inject_erase": (C.c_int, [_P(abft_problem), _V, abft_rect, C.c_int, _V]),
            "abft_fill_uniform": (C.c_int, [C.c_int32, C.c_int64, C.c_int64, C.c_int64, C.c_int, C.c_uint64,
                                            C.c_int32, _V, _V]),
            "abft_batch_workspace_size": (C.c_size_t, [_P(abft_problem), C.c_int]),
            "abft_batch_setup": (C.c_int, [_P(abft_problem), _P(abft_batch_item), C.c_int, _V, C.c_size_t,
                                           _P(abft_batch_plan)]),
            "abft_batch_quantize": (C.c_int, [_P(abft_batch_plan), _V]),
            "abft_batch_encode": (C.c_int, [_P(abft_batch_plan), _V]),
            "abft_batch_quantize_encode": (C.c_int, [_P(abft_batch_plan), _V]),
            "abft_batch_gemm": (C.c_int, [_P(abft_batch_plan), C.c_int, C.c_uint32, _V]),
            "abft_batch_setup_tiles": (C.c_int, [_P(abft_problem), _P(abft_batch_item), C.c_int, _P(C.c_int32), _V,
                                                 C.c_size_t, _P(abft_batch_plan)]),
            "abft_batch_tune": (C.c_int, [_P(abft_batch_plan), _P(C.c_double), _P(C.c_int32), _V]),
            "abft_batch_choose": (C.c_int, [_P(abft_batch_plan), C.c_int, _P(C.c_double), _P(C.c_int32), _V]),
            "abft_batch_cache_lookup": (C.c_int, [C.c_char_p, C.c_char_p, _P(abft_problem), C.c_int, _P(C.c_int32)]),
            "abft_batch_cache_store": (C.c_int, [C.c_char_p, C.c_char_p, _P(abft_problem), C.c_int,
                                                 _P(C.c_double)]),
            "abft_batch_verify": (C.c_int, [_P(abft_batch_plan), _V]),
            "abft_batch_reports": (C.c_int, [_P(abft_batch_plan), _V, _V]),
            "abft_batch_thresholds": (C.c_int, [_P(abft_batch_plan), C.c_int, _V, _V, _V]),
            "abft_wworkspace_size": (C.c_size_t, [_P(abft_wproblem)]),
            "abft_wsetup": (C.c_int, [_P(abft_wproblem), _V, _Z]),
            "abft_wencode": (C.c_int, [_P(abft_wproblem), _V, _V, _V, _Z, _V]),
            "abft_wgemm": (C.c_int, [_P(abft_wproblem), _V, _V, _V, _V]),
            "abft_wverify": (C.c_int, [_P(abft_wproblem), _V, _P(abft_rect), C.c_int, _V, _Z, _V, _V]),
            "abft_wlocate": (C.c_int, [_P(abft_wproblem), _P(abft_wreport), _P(abft_location), C.c_int,
                                       _P(C.c_int)]),
            "abft_wcorrect": (C.c_int, [_P(abft_wproblem), _V, _P(abft_location), C.c_int, _V, _Z, _V]),
            "abft_wrecover": (C.c_int, [_P(abft_wproblem), _V, C.c_int, _P(C.c_int32), C.c_int, C.c_int64,
                                        C.c_int64, _V, _Z, _V]),
            "abft_block_cyclic_stack": (C.c_int, [_V, C.c_int64, C.c_int64, C.c_int64, C.c_int32, C.c_int64,
                                                  C.c_int32, C.c_int32, _V, C.c_int64, _V]),
            "abft_block_cyclic_unstack": (C.c_int, [_V, C.c_int64, C.c_int64, C.c_int64, C.c_int32, C.c_int64,
                                                    C.c_int32, C.c_int32, _V, C.c_int64, _V]),
            "abft_fill_normal": (C.c_int, [C.c_int64, C.c_int64, C.c_int64, C.c_int, C.c_uint64, C.c_double,
                                           C.c_float, _V, _V]),
            "abft_probe_mfma": (C.c_int, [C.c_int32, C.c_int64, _V, C.c_int64, _P(C.c_double), _V]),
            "abft_probe_stream": (C.c_int, [_V, _Z, _V, C.c_int64, _V]),
            "abft_last_hip_error": (C.c_int, []),
            "abft_status_string": (C.c_char_p, [C.c_int]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(fn, st, ok=(ABFT_OK,)):
    if st not in ok:
        msg = lib().abft_status_string(st).decode()
        if st == ABFT_E_HIP:
            msg += f" (hipError {lib().abft_last_hip_error()})"
        raise AbftError(fn, st, msg)
    return st


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    return C.c_void_p(t.data_ptr())


def _nbytes(t) -> int:
    """Size in bytes of a workspace tensor (0 for None)."""
    return 0 if t is None else t.numel() * t.element_size()


def problem(dtype, m, n, k, br, bc, lda=None, ldb=None, ldc=None, tau_mode=None, lam=0.0, kappa=0.0):
    if tau_mode is None:
        tau_mode = ABFT_TAU_DET if dtype == ABFT_F64 else ABFT_TAU_STAT
    return abft_problem(dtype, tau_mode, m, n, k, br, bc,
                        lda if lda is not None else k, ldb if ldb is not None else k,
                        ldc if ldc is not None else n + bc, lam, kappa)


def workspace_size(p: abft_problem) -> int:
    return lib().abft_workspace_size(C.byref(p))


def encode(p, A_f, B_f, ws, stream=None):
    return _check("abft_encode", lib().abft_encode(C.byref(p), _ptr(A_f), _ptr(B_f), _ptr(ws), _nbytes(ws),
                                                   _stream(stream)))


def encode_chained(p, A_f, B_f, ws, prev, ws_prev, stream=None):
    """A_f: the previous product's C_f (lda = prev.ldc); B_f: the new operand."""
    return _check("abft_encode_chained", lib().abft_encode_chained(C.byref(p), _ptr(A_f), _ptr(B_f), _ptr(ws),
                                                                   _nbytes(ws), C.byref(prev), _ptr(ws_prev),
                                                                   _nbytes(ws_prev), _stream(stream)))


def gemm(p, A_f, B_f, C_f, ws=None, flags=0, stream=None):
    return _check("abft_gemm", lib().abft_gemm(C.byref(p), _ptr(A_f), _ptr(B_f), _ptr(C_f), _ptr(ws), _nbytes(ws),
                                               flags, _stream(stream)))


def gemm_fault(p, A_f, B_f, C_f, ws, i, j, bit, flags=0, stream=None):
    """Test hook: abft_gemm with bit `bit` of the accumulator of C[i, j] flipped inside the product kernel."""
    f = abft_fault(i, j, bit)
    return _check("abft_gemm_fault", lib().abft_gemm_fault(C.byref(p), _ptr(A_f), _ptr(B_f), _ptr(C_f), _ptr(ws),
                                                           _nbytes(ws), flags, C.byref(f), _stream(stream)))


def describe_gemm(p, flags=0) -> str:
    """The kernels and block tile abft_gemm launches for p and flags."""
    buf = C.create_string_buffer(256)
    _check("abft_describe_gemm", lib().abft_describe_gemm(C.byref(p), C.c_uint32(flags), buf, C.c_size_t(256)))
    return buf.value.decode()


def gemm_panel(p, A_f, B_f, C_f, k0, k1, flags=0, stream=None):
    """C_f (+)= A_f[:, k0:k1) B_f[k0:k1, :) (ABFT_ACCUMULATE in flags adds)."""
    return _check("abft_gemm_panel", lib().abft_gemm_panel(C.byref(p), _ptr(A_f), _ptr(B_f), _ptr(C_f), k0, k1,
                                                           flags, _stream(stream)))


def quantize(p, which, X, dst, ws, stream=None):
    """X: float32 device tensor (A: m x k, or B^T: n x k); dst: the A_f / Bt tensor."""
    return _check("abft_quantize", lib().abft_quantize(C.byref(p), which, _ptr(X), X.stride(0), _ptr(dst), _ptr(ws),
                                                       _nbytes(ws), _stream(stream)))


def quantize_encode(p, A32, B32, A_f, B_f, ws, stream=None):
    """Quantize A32 (m x k) and B32 (B^T, n x k) binary32 tensors into A_f, B_f and encode, in one pass."""
    return _check("abft_quantize_encode",
                  lib().abft_quantize_encode(C.byref(p), _ptr(A32), A32.stride(0), _ptr(B32), B32.stride(0),
                                             _ptr(A_f), _ptr(B_f), _ptr(ws), _nbytes(ws), _stream(stream)))


def _rects(known):
    known = list(known or [])
    arr = (abft_rect * max(1, len(known)))(*[abft_rect(*r) for r in known])
    return arr, len(known)


def verify(p, C_f, ws, known=None, host_out=None, stream=None):
    """host_out: a pinned uint8 CPU tensor of sizeof(abft_report) bytes, or None."""
    arr, nk = _rects(known)
    hp = C.c_void_p(host_out.data_ptr()) if host_out is not None else None
    return _check("abft_verify", lib().abft_verify(C.byref(p), _ptr(C_f), arr, nk, _ptr(ws), _nbytes(ws), hp,
                                                   _stream(stream)))


def verify_noalloc(p, C_f, ws, known=None, host_out=None, stream=None):
    """abft_verify with the library's static scratch (allocates nothing); ws is
    read only; host_out (a pinned buffer from new_report_buffer) is required."""
    arr, nk = _rects(known)
    hp = C.c_void_p(host_out.data_ptr()) if host_out is not None else None
    return _check("abft_verify_noalloc", lib().abft_verify_noalloc(C.byref(p), _ptr(C_f), arr, nk, _ptr(ws),
                                                                   _nbytes(ws), hp, _stream(stream)))


def verify_fused(p, C_f, ws, host_out=None, stream=None):
    """The report's status is ABFT_E_STALE when ws holds no fused partial sums of this problem and C_f."""
    hp = C.c_void_p(host_out.data_ptr()) if host_out is not None else None
    return _check("abft_verify_fused", lib().abft_verify_fused(C.byref(p), _ptr(C_f), _ptr(ws), _nbytes(ws), hp,
                                                               _stream(stream)))


def new_report_buffer():
    import torch
    return torch.empty(C.sizeof(abft_report), dtype=torch.uint8, pin_memory=True)


def read_report(host_buf) -> abft_report:
    """Copy the report out of a pinned buffer (synchronise the stream first)."""
    return abft_report.from_buffer_copy(host_buf.numpy().tobytes())


def classify(p, rep: abft_report, known=None) -> abft_location:
    arr, nk = _rects(known)
    loc = abft_location()
    _check("abft_classify", lib().abft_classify(C.byref(p), C.byref(rep), arr, nk, C.byref(loc)))
    return loc


def correct(p, C_f, loc: abft_location, stream=None):
    return _check("abft_correct", lib().abft_correct(C.byref(p), _ptr(C_f), C.byref(loc), _stream(stream)))


def recover_block(p, C_f, rect, use_rows=False, stream=None):
    return _check("abft_recover_block",
                  lib().abft_recover_block(C.byref(p), _ptr(C_f), abft_rect(*rect), int(use_rows), _stream(stream)))


def inject_flip(p, C_f, i, j, bit, stream=None):
    return _check("abft_inject_flip", lib().abft_inject_flip(C.byref(p), _ptr(C_f), i, j, bit, _stream(stream)))


def inject_erase(p, C_f, rect, nan_fill=False, stream=None):
    return _check("abft_inject_erase",
                  lib().abft_inject_erase(C.byref(p), _ptr(C_f), abft_rect(*rect), int(nan_fill), _stream(stream)))


def fill_uniform(dtype, rows, cols, ld, transpose, seed, stream_id, dst, stream=None):
    return _check("abft_fill_uniform", lib().abft_fill_uniform(dtype, rows, cols, ld, int(transpose), seed, stream_id,
                                                               _ptr(dst), _stream(stream)))


def fill_normal(rows, cols, ld, transpose, seed, dst, frac=0.01, scale=1e3, stream=None):
    """Heavy-tailed binary32 inputs on the device (N(0,1), a fraction frac scaled by scale)."""
    return _check("abft_fill_normal", lib().abft_fill_normal(rows, cols, ld, int(transpose), seed, frac, scale,
                                                             _ptr(dst), _stream(stream)))


def batch_workspace_size(probs) -> int:
    arr = (abft_problem * len(probs))(*probs)
    return lib().abft_batch_workspace_size(arr, len(probs))


def batch_setup(probs, items, bws, tiles=None) -> abft_batch_plan:
    """probs: abft_problem list; items: abft_batch_item list; bws: device uint8 tensor;
    tiles: per-problem product tile shapes for ABFT_BATCH_MIXED (None or -1 entries: the library's model)."""
    pa = (abft_problem * len(probs))(*probs)
    ia = (abft_batch_item * len(items))(*items)
    plan = abft_batch_plan()
    if tiles is None:
        _check("abft_batch_setup", lib().abft_batch_setup(pa, ia, len(probs), _ptr(bws), bws.numel(), C.byref(plan)))
    else:
        ta = (C.c_int32 * len(probs))(*[int(t) for t in tiles])
        _check("abft_batch_setup_tiles", lib().abft_batch_setup_tiles(pa, ia, len(probs), ta, _ptr(bws), bws.numel(),
                                                                       C.byref(plan)))
    return plan


def batch_quantize(plan, stream=None):
    return _check("abft_batch_quantize", lib().abft_batch_quantize(C.byref(plan), _stream(stream)))


def batch_encode(plan, stream=None):
    return _check("abft_batch_encode", lib().abft_batch_encode(C.byref(plan), _stream(stream)))


def batch_quantize_encode(plan, stream=None):
    return _check("abft_batch_quantize_encode", lib().abft_batch_quantize_encode(C.byref(plan), _stream(stream)))


def batch_gemm(plan, tile=0, flags=0, stream=None):
    return _check("abft_batch_gemm", lib().abft_batch_gemm(C.byref(plan), tile, flags, _stream(stream)))


def batch_tune(plan, stream=None):
    """-> (per-problem costs: count x ABFT_BATCH_TILES list of lists, per-problem best shapes)."""
    n = plan.count
    costs = (C.c_double * (n * ABFT_BATCH_TILES))()
    tiles = (C.c_int32 * n)()
    _check("abft_batch_tune", lib().abft_batch_tune(C.byref(plan), costs, tiles, _stream(stream)))
    return ([list(costs[p * ABFT_BATCH_TILES:(p + 1) * ABFT_BATCH_TILES]) for p in range(n)],
            [int(t) for t in tiles])


def batch_choose(plan, reps=3, stream=None):
    """-> (median ms of the protected product per choice: uniform shapes, then per-problem; fastest choice)."""
    ms = (C.c_double * (ABFT_BATCH_TILES + 1))()
    choice = C.c_int32(-1)
    _check("abft_batch_choose", lib().abft_batch_choose(C.byref(plan), reps, ms, C.byref(choice), _stream(stream)))
    return list(ms), int(choice.value)


def batch_cache_lookup(path, probs, arch=None):
    """-> (found, per-problem tile shapes or -1) from the tuning cache file."""
    pa = (abft_problem * len(probs))(*probs)
    tiles = (C.c_int32 * len(probs))()
    found = lib().abft_batch_cache_lookup(path.encode(), arch.encode() if arch else None, pa, len(probs), tiles)
    if found < 0:
        _check("abft_batch_cache_lookup", found)
    return found, [int(t) for t in tiles]


def batch_cache_store(path, probs, costs, arch=None):
    pa = (abft_problem * len(probs))(*probs)
    flat = (C.c_double * (len(probs) * ABFT_BATCH_TILES))(*[c for row in costs for c in row])
    return _check("abft_batch_cache_store",
                  lib().abft_batch_cache_store(path.encode(), arch.encode() if arch else None, pa, len(probs), flat))


def batch_verify(plan, stream=None):
    return _check("abft_batch_verify", lib().abft_batch_verify(C.byref(plan), _stream(stream)))


def batch_thresholds(plan, problem, tau_c, tau_r, stream=None):
    """tau_c: float64 device tensor (br, n + bc); tau_r: (m + br, bc)."""
    return _check("abft_batch_thresholds", lib().abft_batch_thresholds(C.byref(plan), problem, _ptr(tau_c),
                                                                       _ptr(tau_r), _stream(stream)))


def batch_reports(plan, host_out, stream=None):
    """host_out: pinned uint8 CPU tensor of count * sizeof(abft_report) bytes."""
    return _check("abft_batch_reports",
                  lib().abft_batch_reports(C.byref(plan), C.c_void_p(host_out.data_ptr()), _stream(stream)))


def probe_mfma(dtype, iters, sink, stream=None) -> float:
    """Launch the matrix-core peak probe (sink: float64 device tensor of >= 512
    entries); returns the flops it executes."""
    flops = C.c_double(0.0)
    _check("abft_probe_mfma", lib().abft_probe_mfma(dtype, iters, _ptr(sink), sink.numel(), C.byref(flops),
                                                    _stream(stream)))
    return flops.value


def probe_stream(buf, sink, stream=None):
    """Launch the HBM read probe over the device tensor buf (sink: float64
    device tensor of >= 1 entry)."""
    return _check("abft_probe_stream", lib().abft_probe_stream(_ptr(buf), _nbytes(buf), _ptr(sink), sink.numel(),
                                                               _stream(stream)))


# ---------------------------------------------------------------- conveniences
class Protected:
    """Device buffers of one protected product (A_f, B_f, C_f, workspace),
    allocated with torch.  B_f is stored column-major: the tensor Bt is
    B_f^T, (n + bc) x k row-major."""

    def __init__(self, dtype, m, n, k, br, bc, device="cuda", tau_mode=None, lam=0.0):
        import torch
        tdt = {ABFT_F64: torch.float64, ABFT_F32: torch.float32, ABFT_BF16: torch.bfloat16,
               ABFT_FP8_E4M3: torch.uint8}[dtype]
        cdt = torch.float64 if dtype == ABFT_F64 else torch.float32
        self.M, self.N = m + br, n + bc
        # rows of C_f padded to 16 bytes so the verification passes use 16-byte loads
        vec = 16 // (8 if dtype == ABFT_F64 else 4)
        self.ldc = (self.N + vec - 1) // vec * vec
        self.p = problem(dtype, m, n, k, br, bc, ldc=self.ldc, tau_mode=tau_mode, lam=lam)
        lowp = dtype in (ABFT_BF16, ABFT_FP8_E4M3)      # checksum rows kept in the workspace
        self.A = torch.zeros(m if lowp else self.M, k, dtype=tdt, device=device)
        self.Bt = torch.zeros(n if lowp else self.N, k, dtype=tdt, device=device)
        self.Cbuf = torch.zeros(self.M, self.ldc, dtype=cdt, device=device)
        self.C = self.Cbuf[:, :self.N]          # view; the library sees ldc = self.ldc
        self.ws = torch.zeros(workspace_size(self.p), dtype=torch.uint8, device=device)
        self.rep_host = new_report_buffer()

    def encode(self):
        encode(self.p, self.A, self.Bt, self.ws)

    def gemm(self, flags=0):
        gemm(self.p, self.A, self.Bt, self.C, self.ws, flags)

    def gemm_fault(self, i, j, bit, flags=0):
        gemm_fault(self.p, self.A, self.Bt, self.C, self.ws, i, j, bit, flags)

    def verify(self, known=None) -> abft_report:
        import torch
        verify(self.p, self.C, self.ws, known=known, host_out=self.rep_host)
        torch.cuda.current_stream().synchronize()
        return read_report(self.rep_host)

    def verify_fused(self) -> abft_report:
        import torch
        verify_fused(self.p, self.C, self.ws, host_out=self.rep_host)
        torch.cuda.current_stream().synchronize()
        return read_report(self.rep_host)


class Batch:
    """Device buffers of a batch of bfloat16 protected products: per problem
    binary32 inputs A32 (m x k) and Bt32 (n x k), their bfloat16 copies A and
    Bt, and C_f with rows padded to 16 bytes; one batch workspace and a pinned
    buffer for the reports.  shapes: list of (m, n, k, br, bc).  A32, Bt32, A
    and Bt are (m, k) / (n, k) views of buffers with rows of lda = ldb
    elements (lda[q]; k unless ld_align pads them)."""

    def __init__(self, shapes, device="cuda", tau_mode=ABFT_TAU_STAT, lam=0.0, tiles=None, ldc_align=4,
                 ld_align=1):
        """ldc_align: rows of C_f padded to a multiple of this many elements (4: 16-byte rows, the
        vector forms of the product's store and of the verification; 1: no padding).  ld_align: rows
        of the operands padded to a multiple of this many elements (a multiple of 8; 64: every
        bfloat16 row starts on a 128-byte line, so the quantizing pass writes whole lines)."""
        import torch
        if ld_align < 1 or (ld_align > 1 and ld_align % 8):
            raise ValueError("ld_align: 1 or a multiple of 8")
        self.shapes = list(shapes)
        self.probs, self.items, self.lda = [], [], []
        self.A32, self.Bt32, self.A, self.Bt, self.Cbuf, self.C = [], [], [], [], [], []
        for (m, n, k, br, bc) in self.shapes:
            N = n + bc
            ldc = (N + ldc_align - 1) // ldc_align * ldc_align
            ld = (k + ld_align - 1) // ld_align * ld_align
            p = problem(ABFT_BF16, m, n, k, br, bc, lda=ld, ldb=ld, ldc=ldc, tau_mode=tau_mode, lam=lam)
            a32 = torch.zeros(m, ld, dtype=torch.float32, device=device)[:, :k]
            b32 = torch.zeros(n, ld, dtype=torch.float32, device=device)[:, :k]
            a = torch.zeros(m, ld, dtype=torch.bfloat16, device=device)[:, :k]
            b = torch.zeros(n, ld, dtype=torch.bfloat16, device=device)[:, :k]
            cb = torch.zeros(m + br, ldc, dtype=torch.float32, device=device)
            self.probs.append(p)
            self.lda.append(ld)
            self.items.append(abft_batch_item(a32.data_ptr(), b32.data_ptr(), a.data_ptr(), b.data_ptr(),
                                              cb.data_ptr()))
            self.A32.append(a32); self.Bt32.append(b32); self.A.append(a); self.Bt.append(b)
            self.Cbuf.append(cb); self.C.append(cb[:, :N])
        nbytes = batch_workspace_size(self.probs)
        if nbytes == 0:
            raise AbftError("abft_batch_workspace_size", ABFT_E_ARG, "invalid batch")
        self.bws = torch.zeros(nbytes, dtype=torch.uint8, device=device)
        self.plan = batch_setup(self.probs, self.items, self.bws, tiles)
        self.rep_host = torch.empty(len(self.probs) * C.sizeof(abft_report), dtype=torch.uint8, pin_memory=True)

    def set_tiles(self, tiles):
        """Rebuild the plan with per-problem tile shapes for ABFT_BATCH_MIXED (synchronous)."""
        self.plan = batch_setup(self.probs, self.items, self.bws, tiles)

    def fetch_reports(self, stream=None):
        """Copy every report into the pinned buffer (synchronises the stream);
        returns the indices of the problems with a failed relation."""
        import numpy as np
        import torch
        batch_reports(self.plan, self.rep_host, stream)
        (stream or torch.cuda.current_stream()).synchronize()
        w = self.rep_host.numpy().view(np.int64).reshape(len(self.probs), C.sizeof(abft_report) // 8)
        return [int(q) for q in np.nonzero(w[:, 0] + w[:, 1])[0]]

    def report(self, q) -> abft_report:
        """Problem q's report from the last fetch_reports."""
        sz = C.sizeof(abft_report)
        return abft_report.from_buffer_copy(self.rep_host.numpy()[q * sz:(q + 1) * sz].tobytes())

    def reports(self, stream=None):
        """Copy every report out (synchronises the current stream)."""
        import torch
        batch_reports(self.plan, self.rep_host, stream)
        (stream or torch.cuda.current_stream()).synchronize()
        raw = self.rep_host.numpy().tobytes()
        sz = C.sizeof(abft_report)
        return [abft_report.from_buffer_copy(raw[q * sz:(q + 1) * sz]) for q in range(len(self.probs))]


# ---------------------------------------------------------------- weighted f-checksums (Sec. 2.1)
def wproblem(m, n, k, br, bc, wr, wc, lda=None, ldb=None, ldc=None, tau_mode=ABFT_TAU_DET, kappa=0.0,
             dtype=None):
    """wr (fr x m/br), wc (fc x n/bc): float64 numpy arrays kept alive by the
    returned structure's `_keep` attribute (the library reads them on the host).
    dtype: ABFT_F64 (default) or ABFT_F32."""
    import numpy as np
    wr = np.ascontiguousarray(wr, dtype=np.float64)
    wc = np.ascontiguousarray(wc, dtype=np.float64)
    fr, fc = wr.shape[0], wc.shape[0]
    base = problem(ABFT_F64 if dtype is None else dtype, m, n, k, br, bc, lda, ldb,
                   ldc if ldc is not None else n + fc * bc, tau_mode=tau_mode, kappa=kappa)
    wp = abft_wproblem(base, fr, fc, wr.ctypes.data_as(C.POINTER(C.c_double)),
                       wc.ctypes.data_as(C.POINTER(C.c_double)))
    wp._keep = (wr, wc)
    return wp


def wworkspace_size(wp) -> int:
    return lib().abft_wworkspace_size(C.byref(wp))


def wsetup(wp, ws):
    return _check("abft_wsetup", lib().abft_wsetup(C.byref(wp), _ptr(ws), _nbytes(ws)))


def wencode(wp, A_f, B_f, ws, stream=None):
    return _check("abft_wencode", lib().abft_wencode(C.byref(wp), _ptr(A_f), _ptr(B_f), _ptr(ws), _nbytes(ws),
                                                     _stream(stream)))


def wgemm(wp, A_f, B_f, C_f, stream=None):
    return _check("abft_wgemm", lib().abft_wgemm(C.byref(wp), _ptr(A_f), _ptr(B_f), _ptr(C_f), _stream(stream)))


def wverify(wp, C_f, ws, known=None, host_out=None, stream=None):
    arr, nk = _rects(known)
    hp = C.c_void_p(host_out.data_ptr()) if host_out is not None else None
    return _check("abft_wverify", lib().abft_wverify(C.byref(wp), _ptr(C_f), arr, nk, _ptr(ws), _nbytes(ws), hp,
                                                     _stream(stream)))


def new_wreport_buffer():
    import torch
    return torch.empty(C.sizeof(abft_wreport), dtype=torch.uint8, pin_memory=True)


def read_wreport(host_buf) -> abft_wreport:
    return abft_wreport.from_buffer_copy(host_buf.numpy().tobytes())


def wlocate(wp, rep: abft_wreport, max_out=ABFT_MAX_FLAGS):
    """-> (status, [abft_location]); status ABFT_OK or ABFT_E_UNCORRECTABLE."""
    out = (abft_location * max(1, max_out))()
    n = C.c_int(0)
    st = _check("abft_wlocate", lib().abft_wlocate(C.byref(wp), C.byref(rep), out, max_out, C.byref(n)),
                ok=(ABFT_OK, ABFT_E_UNCORRECTABLE))
    return st, [out[q] for q in range(min(n.value, max_out))]


def wcorrect(wp, C_f, locs, ws, stream=None):
    arr = (abft_location * max(1, len(locs)))(*locs)
    return _check("abft_wcorrect", lib().abft_wcorrect(C.byref(wp), _ptr(C_f), arr, len(locs), _ptr(ws),
                                                       _nbytes(ws), _stream(stream)))


def wrecover(wp, C_f, direction, blocks, lo, length, ws, stream=None):
    blocks = list(blocks)
    arr = (C.c_int32 * max(1, len(blocks)))(*blocks)
    return _check("abft_wrecover", lib().abft_wrecover(C.byref(wp), _ptr(C_f), direction, arr, len(blocks), lo,
                                                       length, _ptr(ws), _nbytes(ws), _stream(stream)))


class WProtected:
    """Device buffers of one weighted-checksum product (binary64, or binary32
    with dtype=ABFT_F32): A_f ((m + fr br) x k), B_f^T ((n + fc bc) x k), C_f
    with rows padded to 16 bytes, the workspace (weights copied in) and a
    pinned report buffer."""

    def __init__(self, m, n, k, br, bc, wr, wc, device="cuda", tau_mode=ABFT_TAU_DET, dtype=None):
        import torch
        dtype = ABFT_F64 if dtype is None else dtype
        tdt = torch.float64 if dtype == ABFT_F64 else torch.float32
        per16 = 2 if dtype == ABFT_F64 else 4
        fr, fc = len(wr), len(wc)
        self.M, self.N = m + fr * br, n + fc * bc
        self.ldc = (self.N + per16 - 1) // per16 * per16
        self.p = wproblem(m, n, k, br, bc, wr, wc, ldc=self.ldc, tau_mode=tau_mode, dtype=dtype)
        self.A = torch.zeros(self.M, k, dtype=tdt, device=device)
        self.Bt = torch.zeros(self.N, k, dtype=tdt, device=device)
        self.Cbuf = torch.zeros(self.M, self.ldc, dtype=tdt, device=device)
        self.C = self.Cbuf[:, :self.N]
        self.ws = torch.zeros(wworkspace_size(self.p), dtype=torch.uint8, device=device)
        wsetup(self.p, self.ws)
        self.rep_host = new_wreport_buffer()

    def encode(self):
        wencode(self.p, self.A, self.Bt, self.ws)

    def gemm(self):
        wgemm(self.p, self.A, self.Bt, self.C)

    def verify(self, known=None) -> abft_wreport:
        import torch
        wverify(self.p, self.C, self.ws, known=known, host_out=self.rep_host)
        torch.cuda.current_stream().synchronize()
        return read_wreport(self.rep_host)


# ---------------------------------------------------------------- 2-D block-cyclic layout (Sec. 4.1)
def block_cyclic_stack(G, rows, cols, nb, P, Q, S, stream=None):
    """G, S: 2-D device tensors (row-major, any element size); the leading
    dimensions are their row strides."""
    return _check("abft_block_cyclic_stack",
                  lib().abft_block_cyclic_stack(_ptr(G), G.stride(0), rows, cols, G.element_size(), nb, P, Q,
                                                _ptr(S), S.stride(0), _stream(stream)))


def block_cyclic_unstack(S, rows, cols, nb, P, Q, G, stream=None):
    return _check("abft_block_cyclic_unstack",
                  lib().abft_block_cyclic_unstack(_ptr(S), S.stride(0), rows, cols, S.element_size(), nb, P, Q,
                                                  _ptr(G), G.stride(0), _stream(stream)))
