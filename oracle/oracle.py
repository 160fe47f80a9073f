"""ctypes front end of the FP64 CPU oracle (``abft_oracle.c``).

TEST INFRASTRUCTURE: only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module.  It never imports the
GPU package, and the GPU package never imports it.

All arrays are numpy float64, row-major.  B_f is the paper's k x (n+bc)
matrix (Sec. 2.2, Eq. ABFT-GEMM); callers holding a column-major copy pass
its transpose.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "abft_oracle.c")
LIB_PATH = os.path.join(_HERE, "liboracle.so")

MAXFLAG = 64
CLEAN, DATA, CHECKSUM, MULTI = 0, 1, 2, 3
DIR_COL, DIR_ROW = 0, 1
U64 = 2.0 ** -53
U32 = 2.0 ** -24


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (binary64, no contraction, no fast-math)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(_SRC):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Report(C.Structure):
    _fields_ = [("n_flag_c", C.c_int64), ("n_flag_r", C.c_int64),
                ("n_excl_c", C.c_int64), ("n_excl_r", C.c_int64),
                ("n_nonfinite", C.c_int64),
                ("max_ratio_c", C.c_double), ("max_ratio_r", C.c_double),
                ("fc_r", C.c_int64 * MAXFLAG), ("fc_j", C.c_int64 * MAXFLAG),
                ("fc_d", C.c_double * MAXFLAG), ("fc_t", C.c_double * MAXFLAG),
                ("fr_i", C.c_int64 * MAXFLAG), ("fr_c", C.c_int64 * MAXFLAG),
                ("fr_d", C.c_double * MAXFLAG), ("fr_t", C.c_double * MAXFLAG)]

    def flags_c(self):
        k = min(self.n_flag_c, MAXFLAG)
        return [(self.fc_r[q], self.fc_j[q], self.fc_d[q], self.fc_t[q]) for q in range(k)]

    def flags_r(self):
        k = min(self.n_flag_r, MAXFLAG)
        return [(self.fr_i[q], self.fr_c[q], self.fr_d[q], self.fr_t[q]) for q in range(k)]


_lib = None
_P = C.c_void_p
_I = C.c_int64
_D = C.c_double


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        sig = {
            "orc_encode_rows": (None, [_I, _I, _I, _P, _I, C.c_int]),
            "orc_encode_cols": (None, [_I, _I, _I, _P, _I, C.c_int]),
            "orc_gemm": (None, [_I, _I, _I, _P, _I, _P, _I, _P, _I]),
            "orc_dot": (_D, [_I, _P, _I, _P, _I]),
            "orc_row_norms": (None, [_I, _I, _P, _I, _P]),
            "orc_group_abs_row_norms": (None, [_I, _I, _I, _P, _I, _P]),
            "orc_col_norms": (None, [_I, _I, _P, _I, _P]),
            "orc_group_abs_col_norms": (None, [_I, _I, _I, _P, _I, _P]),
            "orc_gamma": (_D, [_D, _D]),
            "orc_tau_det": (None, [_I, _I, _I, _I, _I, _P, _P, _P, _P, _D, _D, _D, _P, _P]),
            "orc_tau_stat": (None, [_I, _I, _I, _I, _I, _P, _I, _P, _I, _D, _D, _D, _D, _P, _I, _D, _P, _P]),
            "orc_report_size": (_I, []),
            "orc_verify": (None, [_I, _I, _I, _I, _P, _I, _P, _P, _P, C.c_int, _P, _P, _P]),
            "orc_classify": (C.c_int, [_I, _I, _I, _I, _P, _P, C.c_int, _P, _P, _P]),
            "orc_rebuild_value": (_D, [_I, _I, _I, _I, _P, _I, _I, _I, C.c_int]),
            "orc_recover": (C.c_int, [_I, _I, _I, _I, _P, _I, _I, _I, _I, _I, C.c_int, C.c_int]),
            "orc_residual": (_D, [_I, _I, _I, _P, _I, _P, _I, _P, _I, _P, _D]),
            "orc_to_bf16": (None, [_I, _P, _P]),
            "orc_e4m3_value": (_D, [C.c_uint8]),
            "orc_to_e4m3": (None, [_I, _P, _P]),
            "orc_e4m3_scale_exp": (C.c_int, [_I, _P]),
            "orc_num_threads": (C.c_int, []),
            "orc_set_num_threads": (None, [C.c_int]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        assert L.orc_report_size() == C.sizeof(Report), "oracle report layout mismatch"
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- encoding
def encode(A: np.ndarray, B: np.ndarray, br: int, bc: int, store_f32: bool = False):
    """A (m x k), B (k x n) -> A_f ((m+br) x k), B_f (k x (n+bc)) per Eq. ABFT-GEMM."""
    m, k = A.shape
    k2, n = B.shape
    assert k == k2 and m % br == 0 and n % bc == 0
    Af = np.zeros((m + br, k))
    Af[:m] = A
    Bf = np.zeros((k, n + bc))
    Bf[:, :n] = B
    lib().orc_encode_rows(m, k, br, _p(Af), k, int(store_f32))
    lib().orc_encode_cols(k, n, bc, _p(Bf), n + bc, int(store_f32))
    return Af, Bf


def encode_rows_inplace(Af: np.ndarray, m: int, br: int, store_f32: bool = False):
    assert Af.flags.c_contiguous and Af.dtype == np.float64
    lib().orc_encode_rows(m, Af.shape[1], br, _p(Af), Af.shape[1], int(store_f32))


def gemm(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    A = _f64(A)
    B = _f64(B)
    M, K = A.shape
    K2, N = B.shape
    assert K == K2
    Cm = np.empty((M, N))
    lib().orc_gemm(M, N, K, _p(A), K, _p(B), N, _p(Cm), N)
    return Cm


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))


def dot(a: np.ndarray, b: np.ndarray) -> float:
    a = _f64(a)
    b = _f64(b)
    return lib().orc_dot(a.shape[0], _p(a), 1, _p(b), 1)


# ---------------------------------------------------------------- thresholds
def norms(Af: np.ndarray, Bf: np.ndarray, m: int, n: int, br: int, bc: int):
    """(na, na_abs, nb, nb_abs) of the det threshold."""
    Af = _f64(Af)
    Bf = _f64(Bf)
    M, k = Af.shape
    N = Bf.shape[1]
    na = np.empty(M)
    na_abs = np.empty(br)
    nb = np.empty(N)
    nb_abs = np.empty(bc)
    L = lib()
    L.orc_row_norms(M, k, _p(Af), k, _p(na))
    L.orc_group_abs_row_norms(m, k, br, _p(Af), k, _p(na_abs))
    L.orc_col_norms(k, N, _p(Bf), N, _p(nb))
    L.orc_group_abs_col_norms(k, n, bc, _p(Bf), N, _p(nb_abs))
    return na, na_abs, nb, nb_abs


def tau_det(Af, Bf, m, n, br, bc, u_acc=U64, u_st=0.0, kappa=1.0 + 2.0 ** -20):
    k = Af.shape[1]
    na, na_abs, nb, nb_abs = norms(Af, Bf, m, n, br, bc)
    tc = np.empty((br, n + bc))
    tr = np.empty((m + br, bc))
    lib().orc_tau_det(m, n, k, br, bc, _p(na), _p(na_abs), _p(nb), _p(nb_abs), u_acc, u_st, kappa, _p(tc), _p(tr))
    return tc, tr


def tau_det_chained(Af, Bf, m, n, br, bc, tau_c_prev, kappa=1.0 + 2.0 ** -20, u_acc=U64, u_st=0.0):
    """Thresholds of a chained product D_f = A_f B_f whose A_f is a previous
    product's C_f (its data columns), the carried rows used as A's checksum
    rows without recomputation (Sec. 3.2, chained calls).  Every previous
    column relation (r, l) holds up to its residual, at most tau_c_prev[r, l];
    through the product these add sum_l tau_c_prev[r, l] |B_f[l, j]| to the
    column relation (r, j) of D_f.  Row relations are those of a plain product
    (u_acc, u_st: its roundoffs, as for tau_det)."""
    Bf = _f64(Bf)
    k = Bf.shape[0]
    tc, tr = tau_det(Af, Bf, m, n, br, bc, u_acc=u_acc, u_st=u_st, kappa=kappa)
    return tc + _f64(tau_c_prev)[:, :k] @ np.abs(Bf), tr


def tau_stat(Af, Bf, m, n, br, bc, u_acc=U32, T=None, s_store=1.0, lam=10.0, Cf=None, T_c=0.0):
    """Statistical thresholds; Cf (the encoded product, same domain as A_f B_f)
    adds the binary32 rounding of each relation's stored total, and T_c the
    accumulation steps of the stored totals when they are themselves summed in
    that precision (0: binary64)."""
    Af = _f64(Af)
    Bf = _f64(Bf)
    k = Af.shape[1]
    if T is None:
        T = k / 4.0
    tc = np.empty((br, n + bc))
    tr = np.empty((m + br, bc))
    if Cf is not None:
        Cf = _f64(Cf)
        assert Cf.shape[0] >= m + br and Cf.shape[1] >= n + bc
    lib().orc_tau_stat(m, n, k, br, bc, _p(Af), k, _p(Bf), n + bc, u_acc, float(T), s_store, lam,
                       _p(Cf) if Cf is not None else None, Cf.shape[1] if Cf is not None else 0, float(T_c),
                       _p(tc), _p(tr))
    return tc, tr


# ---------------------------------------------------------------- verify / locate / fix
def _erasure_array(erasures):
    er = np.zeros((max(1, len(erasures or [])), 4), dtype=np.int64)
    for q, e in enumerate(erasures or []):
        er[q] = e
    return er


def verify(Cf: np.ndarray, m: int, n: int, br: int, bc: int, tau_c, tau_r, erasures=None):
    """-> (Dc, Dr, Report)."""
    Cf = _f64(Cf)
    tc = _f64(tau_c)
    tr = _f64(tau_r)
    er = _erasure_array(erasures)
    Dc = np.empty((br, n + bc))
    Dr = np.empty((m + br, bc))
    rep = Report()
    lib().orc_verify(m, n, br, bc, _p(Cf), Cf.shape[1], _p(tc), _p(tr), _p(er), len(erasures or []),
                     _p(Dc), _p(Dr), C.byref(rep))
    return Dc, Dr, rep


def classify(rep: Report, m, n, br, bc, erasures=None):
    """-> (cls, i, j, direction)."""
    er = _erasure_array(erasures)
    oi, oj, od = C.c_int64(), C.c_int64(), C.c_int()
    cls = lib().orc_classify(m, n, br, bc, C.byref(rep), _p(er), len(erasures or []),
                             C.byref(oi), C.byref(oj), C.byref(od))
    return cls, oi.value, oj.value, od.value


def rebuild_value(Cf, m, n, br, bc, i, j, direction=DIR_COL) -> float:
    Cf = _f64(Cf)
    return lib().orc_rebuild_value(m, n, br, bc, _p(Cf), Cf.shape[1], i, j, direction)


def recover(Cf: np.ndarray, m, n, br, bc, rect, use_rows=False, round_f32=False) -> int:
    """In place on a float64 C_f; rect = (i0, j0, h, w).  0, -1 (bad args) or -4."""
    assert Cf.flags.c_contiguous and Cf.dtype == np.float64
    i0, j0, h, w = rect
    return lib().orc_recover(m, n, br, bc, _p(Cf), Cf.shape[1], i0, j0, h, w, int(use_rows), int(round_f32))


def residual(A, B, Cm, x, u=U64) -> float:
    A = _f64(A)
    B = _f64(B)
    Cm = _f64(Cm)
    x = _f64(x)
    m, k = A.shape
    n = B.shape[1]
    return lib().orc_residual(m, n, k, _p(A), k, _p(B), n, _p(Cm), Cm.shape[1], _p(x), u)


# ---------------------------------------------------------------- quantizers
def to_bf16_bits(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.empty(x.shape, dtype=np.uint16)
    lib().orc_to_bf16(x.size, _p(x), _p(out))
    return out


def bf16_bits_to_f64(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)


def to_e4m3_codes(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.empty(x.shape, dtype=np.uint8)
    lib().orc_to_e4m3(x.size, _p(x), _p(out))
    return out


def e4m3_values(codes: np.ndarray) -> np.ndarray:
    table = np.array([lib().orc_e4m3_value(c) for c in range(256)])
    return table[np.asarray(codes, dtype=np.uint8)]


def e4m3_scale_exp(x: np.ndarray) -> int:
    x = np.ascontiguousarray(x, dtype=np.float32)
    return lib().orc_e4m3_scale_exp(x.size, _p(x))


# ---------------------------------------------------------------- whole pipeline
def outer_update(Cf: np.ndarray, Af: np.ndarray, Bf: np.ndarray, k0: int, k1: int) -> np.ndarray:
    """Outer-product form of the product (Sec. 2.2; the rank-nb updates of
    Sec. 3.2): C_f += A_f[:, l] B_f[l, :] for l = k0 .. k1-1, one rank-1
    update at a time, in place on a float64 C_f.  After the updates over
    [0, k1) C_f is the encoded product of A[:, :k1] and B[:k1, :], so it is
    consistent at every step of the loop."""
    assert Cf.dtype == np.float64 and Cf.shape == (Af.shape[0], Bf.shape[1])
    Af = _f64(Af)
    Bf = _f64(Bf)
    for l in range(k0, k1):
        Cf += np.outer(Af[:, l], Bf[l, :])
    return Cf


def protected_product(A: np.ndarray, B: np.ndarray, br: int, bc: int):
    """Encode and multiply in FP64: returns (A_f, B_f, C_f)."""
    Af, Bf = encode(A, B, br, bc)
    return Af, Bf, gemm(Af, Bf)


# ---------------------------------------------------------------- 2-D block-cyclic distribution (Sec. 4.1)
def block_cyclic_owner(i: int, nb: int, P: int):
    """Global index i of a dimension distributed block-cyclically with blocks
    of nb over P processes: (process p, local index li).  Global block I = i div nb
    belongs to process I mod P and is that process's local block I div P."""
    I, ii = divmod(i, nb)
    return I % P, (I // P) * nb + ii


def block_cyclic_stack(G: np.ndarray, nb: int, P: int, Q: int) -> np.ndarray:
    """The local arrays of a P x Q process grid, stacked: process (p, q)'s
    local array occupies rows [p*m/P, (p+1)*m/P) and columns [q*n/Q, (q+1)*n/Q).
    Written element by element from the owner map (m % (nb*P) == 0,
    n % (nb*Q) == 0, so every local array has the same shape)."""
    G = _f64(G)
    m, n = G.shape
    assert m % (nb * P) == 0 and n % (nb * Q) == 0
    lm, ln = m // P, n // Q
    rows = np.empty(m, dtype=np.int64)
    cols = np.empty(n, dtype=np.int64)
    for i in range(m):
        p, li = block_cyclic_owner(i, nb, P)
        rows[i] = p * lm + li
    for j in range(n):
        q, lj = block_cyclic_owner(j, nb, Q)
        cols[j] = q * ln + lj
    S = np.empty_like(G)
    S[np.ix_(rows, cols)] = G
    return S


def block_cyclic_unstack(S: np.ndarray, nb: int, P: int, Q: int) -> np.ndarray:
    """Inverse of block_cyclic_stack."""
    S = _f64(S)
    m, n = S.shape
    lm, ln = m // P, n // Q
    G = np.empty_like(S)
    for i in range(m):
        p, li = block_cyclic_owner(i, nb, P)
        for j in range(n):
            q, lj = block_cyclic_owner(j, nb, Q)
            G[i, j] = S[p * lm + li, q * ln + lj]
    return G
