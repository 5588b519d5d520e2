"""Python binding of libqmm (include/qmm.h): argument marshalling only.

Every call goes to the HIP library; torch supplies device memory and the current
stream.  There is no CPU fallback: if libqmm.so is missing the import of this
module's functions raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqmm.so")

# qmm_status
OK, EINVAL, EBOUND, EVALUE, ENOSPACE, EDEVICE, EUNSUPPORTED = range(7)
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "EBOUND", 3: "EVALUE", 4: "ENOSPACE", 5: "EDEVICE", 6: "EUNSUPPORTED"}
# qmm_path
(PATH_AUTO, PATH_FP64_QADIC, PATH_FP64_REDQ, PATH_FP32_QADIC, PATH_FP32_REDQ, PATH_INT8, PATH_FP4,
 PATH_FP64_LEFT, PATH_FP32_LEFT, PATH_FP64_FULL, PATH_FP32_FULL) = range(11)
PATH_NAMES = {0: "auto", 1: "fp64_qadic", 2: "fp64_redq", 3: "fp32_qadic", 4: "fp32_redq", 5: "int8", 6: "fp4",
              7: "fp64_left", 8: "fp32_left", 9: "fp64_full", 10: "fp32_full"}
# qmm_regime
REGIME_EXACT, REGIME_OFFSET, REGIME_PAPER, REGIME_INT = range(4)
REGIME_NAMES = {0: "exact", 1: "offset", 2: "paper", 3: "int"}
# flags
BOUND_PROVEN, BOUND_PAPER, PLAN_UNBLOCKED, BOUND_G4, BOUND_EQ4, PLAN_ANY_COMPRESSION = 0, 1, 2, 4, 8, 16
BATCH_FORCE_FP64 = 1
BATCH_INT8_ONLY = 2
BATCH_SHAPE_64x64, BATCH_SHAPE_32x128, BATCH_SHAPE_128x32, BATCH_SHAPE_128x128 = 0x100, 0x200, 0x300, 0x400
BATCH_MEASURE = 0x1000
BATCH_RAW = 0x2000
NOALLOC_SCRATCH_BYTES = 64 << 20  # QMM_NOALLOC_SCRATCH_BYTES
N_BATCH_COSTS = 8  # (fixed, per_stage) for each of the four INT8 tile shapes
# unpack selectors
ROWS_REV, COLS_FWD, ROWS_FWD = 0, 1, 2

EXPORTS = [
    "qmm_choose_Qd", "qmm_validate_plan", "qmm_pack_rows_rev", "qmm_pack_cols_fwd", "qmm_pack_rows_fwd",
    "qmm_unpack", "qmm_extract", "qmm_redq", "qmm_gemm_workspace_size", "qmm_gemm_mod_p", "qmm_gemm_packed",
    "qmm_batched_create", "qmm_gemm_mod_p_batched", "qmm_batched_plan", "qmm_batched_destroy",
    "qmm_last_error", "qmm_version", "qmm_pack_centred_cols", "qmm_gemm_centred",
    "qmm_gemm_right_packed", "qmm_batched_tune", "qmm_batched_set_costs", "qmm_count_nonresidues",
    "qmm_pack_fp4_rows", "qmm_pack_fp4_cols", "qmm_gemm_fp4", "qmm_pack_fp4",
    "qmm_gemm_packed_compress", "qmm_pack_left", "qmm_pack_full_right", "qmm_gemm_left_packed",
    "qmm_gemm_full_packed", "qmm_operand_ld", "qmm_gemm_mod_p_noalloc", "qmm_batched_tune_workspace_size",
    "qmm_tune_cache_put", "qmm_tune_cache_get", "qmm_tune_cache_load", "qmm_tune_cache_save", "qmm_tune_cache_clear",
]


class Plan(ctypes.Structure):
    _fields_ = [("p", ctypes.c_uint32), ("t", ctypes.c_uint32), ("d", ctypes.c_uint32),
                ("beta", ctypes.c_uint32), ("k_block", ctypes.c_int64), ("path", ctypes.c_uint32),
                ("regime", ctypes.c_uint32), ("g", ctypes.c_uint32), ("tile", ctypes.c_uint32),
                ("d2", ctypes.c_uint32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}

    def __repr__(self):
        return (f"Plan(p={self.p}, t={self.t}, d={self.d}, beta={self.beta}, k_block={self.k_block}, "
                f"path={PATH_NAMES.get(self.path, self.path)}, regime={REGIME_NAMES.get(self.regime, self.regime)}, "
                f"g={self.g}, tile={self.tile}, d2={self.d2})")


class Problem(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int64), ("p", ctypes.c_uint32),
                ("A", ctypes.c_void_p), ("lda", ctypes.c_int64), ("B", ctypes.c_void_p), ("ldb", ctypes.c_int64),
                ("C", ctypes.c_void_p), ("ldc", ctypes.c_int64)]


class QmmError(RuntimeError):
    def __init__(self, status, where, detail=None):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {detail if detail else last_error()}")


_lib = None


def lib():
    """The loaded libqmm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_0803_1975_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        i64, u32, vp, sz = ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_size_t
        P = ctypes.POINTER(Plan)
        sig = {
            "qmm_choose_Qd": [u32, i64, i64, i64, u32, ctypes.c_int, u32, P],
            "qmm_validate_plan": [P, i64, i64, i64],
            "qmm_pack_rows_rev": [P, i64, i64, vp, i64, vp, i64, vp],
            "qmm_pack_cols_fwd": [P, i64, i64, vp, i64, vp, i64, vp],
            "qmm_pack_rows_fwd": [P, i64, i64, vp, i64, vp, i64, vp],
            "qmm_unpack": [P, ctypes.c_int, i64, i64, vp, i64, vp, i64, vp],
            "qmm_extract": [P, i64, i64, vp, i64, vp, i64, vp],
            "qmm_redq": [P, i64, i64, vp, i64, vp, i64, vp],
            "qmm_gemm_workspace_size": [P, i64, i64, i64, ctypes.POINTER(sz)],
            "qmm_gemm_mod_p": [P, i64, i64, i64, u32, vp, i64, vp, i64, vp, i64, vp, sz, vp],
            "qmm_gemm_packed": [P, i64, i64, i64, vp, i64, vp, i64, vp, i64, vp],
            "qmm_gemm_right_packed": [P, i64, i64, i64, vp, i64, vp, i64, vp, i64, vp],
            "qmm_pack_centred_cols": [P, i64, i64, vp, i64, vp, i64, vp],
            "qmm_gemm_centred": [P, i64, i64, i64, vp, i64, vp, i64, vp, i64, vp],
            "qmm_batched_create": [i64, ctypes.POINTER(Problem), u32, ctypes.POINTER(vp)],
            "qmm_gemm_mod_p_batched": [vp, vp],
            "qmm_batched_plan": [vp, i64, P],
            "qmm_batched_destroy": [vp],
            "qmm_batched_tune": [u32, i64, i64, vp, sz, vp, ctypes.POINTER(ctypes.c_double)],
            "qmm_batched_tune_workspace_size": [i64, i64, ctypes.POINTER(sz)],
            "qmm_tune_cache_put": [ctypes.c_char_p, u32, i64, i64, ctypes.POINTER(ctypes.c_double)],
            "qmm_tune_cache_get": [ctypes.c_char_p, u32, i64, i64, ctypes.POINTER(ctypes.c_double)],
            "qmm_tune_cache_load": [ctypes.c_char_p],
            "qmm_tune_cache_save": [ctypes.c_char_p],
            "qmm_tune_cache_clear": [],
            "qmm_batched_set_costs": [ctypes.POINTER(ctypes.c_double)],
            "qmm_count_nonresidues": [u32, i64, i64, vp, i64, vp, vp],
            "qmm_pack_fp4_rows": [P, i64, i64, vp, i64, vp, i64, vp],
            "qmm_pack_fp4_cols": [P, i64, i64, vp, i64, vp, i64, vp],
            "qmm_gemm_fp4": [P, i64, i64, i64, vp, i64, vp, i64, vp, i64, vp],
            "qmm_pack_fp4": [P, i64, i64, i64, vp, i64, vp, i64, vp, i64, vp, i64, vp],
            "qmm_gemm_packed_compress": [P, i64, i64, i64, vp, i64, vp, i64, vp, i64, vp],
            "qmm_pack_left": [P, i64, i64, vp, i64, vp, i64, vp],
            "qmm_pack_full_right": [P, i64, i64, vp, i64, vp, i64, vp],
            "qmm_gemm_left_packed": [P, i64, i64, i64, vp, i64, vp, i64, vp, i64, vp],
            "qmm_gemm_full_packed": [P, i64, i64, i64, vp, i64, vp, i64, vp, i64, vp],
            "qmm_operand_ld": [P, i64, ctypes.POINTER(i64)],
            "qmm_gemm_mod_p_noalloc": [P, i64, i64, i64, u32, vp, i64, vp, i64, vp, i64, vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.qmm_last_error.restype = ctypes.c_char_p
        L.qmm_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def last_error() -> str:
    return lib().qmm_last_error().decode()


def version() -> str:
    return lib().qmm_version().decode()


def _check(st, where):
    if st != OK:
        raise QmmError(st, where)


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream if isinstance(stream, int) else stream.cuda_stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _side(stream):
    """The torch stream of a `stream` argument that is not torch's current stream, else None."""
    if stream is None:
        return None
    import torch
    cur = torch.cuda.current_stream().cuda_stream
    handle = stream if isinstance(stream, int) else stream.cuda_stream
    if handle == cur:
        return None
    return torch.cuda.ExternalStream(stream) if isinstance(stream, int) else stream


def _new(t, stream):
    """A tensor this binding allocated for work on `stream`.  torch's caching allocator
    orders a block's uses on torch's current stream only: when `stream` is another one,
    it first waits for the current stream (earlier users of the block are done), and the
    block is recorded on it, so that freeing the tensor does not hand its memory to other
    work before the kernels on `stream` are done with it."""
    s = _side(stream)
    if s is not None:
        import torch
        s.wait_stream(torch.cuda.current_stream())
        t.record_stream(s)
    return t


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _ld(t):
    """Leading dimension of a 2-D tensor with unit column stride."""
    if t.dim() != 2:
        raise ValueError("2-D tensors are required")
    if t.numel() == 0:
        return max(t.shape[1], 1)
    if t.shape[1] > 1 and t.stride(1) != 1:
        raise ValueError("2-D tensors with contiguous rows are required")
    return t.stride(0) if t.shape[0] > 1 else max(t.shape[1], 1)


def _u8(t, name):
    import torch
    if t.dtype != torch.uint8 or not t.is_cuda:
        raise TypeError(f"{name} must be a uint8 CUDA tensor")


def word_dtype(plan):
    import torch
    return torch.float32 if plan.beta == 24 else torch.float64


# ---------------------------------------------------------------------------
def choose_Qd(p, m, n, k, beta=0, path=PATH_AUTO, flags=0) -> Plan:
    pl = Plan()
    _check(lib().qmm_choose_Qd(p, m, n, k, beta, path, flags, ctypes.byref(pl)), "qmm_choose_Qd")
    return pl


def try_choose_Qd(p, m, n, k, beta=0, path=PATH_AUTO, flags=0):
    """(status, plan) without raising."""
    pl = Plan()
    st = lib().qmm_choose_Qd(p, m, n, k, beta, path, flags, ctypes.byref(pl))
    return st, pl


def validate_plan(plan, m, n, k) -> int:
    return lib().qmm_validate_plan(ctypes.byref(plan), m, n, k)


def pack_rows_rev(plan, A, CA=None, stream=None):
    import torch
    _u8(A, "A")
    m, k = A.shape
    if CA is None:
        CA = _new(torch.empty((m, -(-k // (plan.d + 1))), dtype=word_dtype(plan), device=A.device), stream)
    _check(lib().qmm_pack_rows_rev(ctypes.byref(plan), m, k, _ptr(A), _ld(A), _ptr(CA), _ld(CA), _stream(stream)),
           "qmm_pack_rows_rev")
    return CA


def pack_cols_fwd(plan, B, CB=None, stream=None):
    import torch
    _u8(B, "B")
    k, n = B.shape
    if CB is None:
        CB = _new(torch.empty((-(-k // (plan.d + 1)), n), dtype=word_dtype(plan), device=B.device), stream)
    _check(lib().qmm_pack_cols_fwd(ctypes.byref(plan), k, n, _ptr(B), _ld(B), _ptr(CB), _ld(CB), _stream(stream)),
           "qmm_pack_cols_fwd")
    return CB


def pack_rows_fwd(plan, B, CBr=None, stream=None):
    import torch
    _u8(B, "B")
    k, n = B.shape
    if CBr is None:
        CBr = _new(torch.empty((k, -(-n // (plan.d + 1))), dtype=word_dtype(plan), device=B.device), stream)
    _check(lib().qmm_pack_rows_fwd(ctypes.byref(plan), k, n, _ptr(B), _ld(B), _ptr(CBr), _ld(CBr), _stream(stream)),
           "qmm_pack_rows_fwd")
    return CBr


def unpack(plan, which, rows, cols, packed, out=None, stream=None):
    import torch
    if out is None:
        out = _new(torch.empty((rows, cols), dtype=torch.uint8, device=packed.device), stream)
    _check(lib().qmm_unpack(ctypes.byref(plan), which, rows, cols, _ptr(packed), _ld(packed), _ptr(out), _ld(out),
                            _stream(stream)), "qmm_unpack")
    return out


def extract(plan, T, C=None, stream=None):
    import torch
    m, n = T.shape
    if C is None:
        C = _new(torch.empty((m, n), dtype=torch.uint8, device=T.device), stream)
    _check(lib().qmm_extract(ctypes.byref(plan), m, n, _ptr(T), _ld(T), _ptr(C), _ld(C), _stream(stream)),
           "qmm_extract")
    return C


def redq(plan, CC, n, C=None, stream=None):
    import torch
    m = CC.shape[0]
    if C is None:
        C = _new(torch.empty((m, n), dtype=torch.uint8, device=CC.device), stream)
    _check(lib().qmm_redq(ctypes.byref(plan), m, n, _ptr(CC), _ld(CC), _ptr(C), _ld(C), _stream(stream)), "qmm_redq")
    return C


def gemm_workspace_size(plan, m, n, k) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().qmm_gemm_workspace_size(ctypes.byref(plan), m, n, k, ctypes.byref(out)), "qmm_gemm_workspace_size")
    return out.value


def workspace(plan, m, n, k, device="cuda"):
    """A device workspace tensor large enough for gemm_mod_p(plan, ...)."""
    import torch
    return torch.empty(max(gemm_workspace_size(plan, m, n, k), 1), dtype=torch.uint8, device=device)


def count_nonresidues(p, X, count=None, stream=None):
    """Device int32 tensor of one entry: the number of entries x >= p of the uint8
    matrix X (asynchronous; read it after the stream's work is done)."""
    import torch
    _u8(X, "X")
    if count is None:
        count = _new(torch.empty(1, dtype=torch.int32, device=X.device), stream)
    rows, cols = X.shape
    _check(lib().qmm_count_nonresidues(p, rows, cols, _ptr(X), _ld(X), _ptr(count), _stream(stream)),
           "qmm_count_nonresidues")
    return count


def gemm_mod_p(A, B, p, plan=None, C=None, ws=None, stream=None, validate=False):
    """C = A x B mod p (uint8 device tensors).  validate=True first counts the
    entries of A and B that are not residues mod p, synchronises, and raises
    QmmError(EVALUE) if there are any (the product itself leaves them undefined)."""
    import torch
    _u8(A, "A")
    _u8(B, "B")
    m, k = A.shape
    k2, n = B.shape
    if k2 != k:
        raise ValueError("inner dimensions differ")
    if validate:
        counts = [count_nonresidues(p, X, stream=stream) for X in (A, B)]
        side = _side(stream)
        if side is not None:
            side.synchronize()  # .item() below waits for torch's current stream only
        bad = [int(c.item()) for c in counts]
        if any(bad):
            raise QmmError(EVALUE, "gemm_mod_p", f"{bad[0]} entries of A and {bad[1]} of B are not residues mod {p}")
    if plan is None:
        plan = choose_Qd(p, m, n, k)
    if C is None:
        C = _new(torch.empty((m, n), dtype=torch.uint8, device=A.device), stream)
    if ws is None:
        ws = _new(workspace(plan, m, n, k, A.device), stream)
    _check(lib().qmm_gemm_mod_p(ctypes.byref(plan), m, n, k, p, _ptr(A), _ld(A), _ptr(B), _ld(B), _ptr(C), _ld(C),
                                _ptr(ws), ws.numel(), _stream(stream)), "qmm_gemm_mod_p")
    return C


def gemm_mod_p_noalloc(A, B, p, plan=None, C=None, stream=None):
    """C = A x B mod p through qmm_gemm_mod_p_noalloc: no workspace argument, the
    library's per-GPU scratch instead (products whose workspace exceeds
    NOALLOC_SCRATCH_BYTES raise QmmError(ENOSPACE)).  plan=None passes NULL, so the
    library chooses the plan, as qmm_gemm_mod_p does."""
    import torch
    _u8(A, "A")
    _u8(B, "B")
    m, k = A.shape
    k2, n = B.shape
    if k2 != k:
        raise ValueError("inner dimensions differ")
    if C is None:
        C = _new(torch.empty((m, n), dtype=torch.uint8, device=A.device), stream)
    _check(lib().qmm_gemm_mod_p_noalloc(ctypes.byref(plan) if plan is not None else None, m, n, k, p, _ptr(A), _ld(A),
                                        _ptr(B), _ld(B), _ptr(C), _ld(C), _stream(stream)), "qmm_gemm_mod_p_noalloc")
    return C


def gemm_packed(plan, k, CA, CB, C=None, stream=None):
    """Procedure (1): C = digit d of CA x CB, mod p."""
    import torch
    m, n = CA.shape[0], CB.shape[1]
    if C is None:
        C = _new(torch.empty((m, n), dtype=torch.uint8, device=CA.device), stream)
    _check(lib().qmm_gemm_packed(ctypes.byref(plan), m, n, k, _ptr(CA), _ld(CA), _ptr(CB), _ld(CB), _ptr(C), _ld(C),
                                 _stream(stream)), "qmm_gemm_packed")
    return C


def gemm_packed_compress(plan, k, CA, CB, CC=None, stream=None):
    """Procedure (1) with ReduceAndCompress: CC = CompressRows(digit d of CA x CB mod p),
    m x ceil(n/(d+1)) words, usable as the CA of a next product with k = n."""
    import torch
    m, n = CA.shape[0], CB.shape[1]
    if CC is None:
        CC = _new(torch.empty((m, -(-n // (plan.d + 1))), dtype=word_dtype(plan), device=CA.device), stream)
    _check(lib().qmm_gemm_packed_compress(ctypes.byref(plan), m, n, k, _ptr(CA), _ld(CA), _ptr(CB), _ld(CB),
                                          _ptr(CC), _ld(CC), _stream(stream)), "qmm_gemm_packed_compress")
    return CC


def pack_left(plan, A, CAl=None, stream=None):
    """Left operand packed along m: CAl[I][l] = sum_i A[I(d+1)+i][l] Q^i (LEFT and FULL plans)."""
    import torch
    _u8(A, "A")
    m, k = A.shape
    if CAl is None:
        CAl = _new(torch.empty((-(-m // (plan.d + 1)), k), dtype=word_dtype(plan), device=A.device), stream)
    _check(lib().qmm_pack_left(ctypes.byref(plan), m, k, _ptr(A), _ld(A), _ptr(CAl), _ld(CAl), _stream(stream)),
           "qmm_pack_left")
    return CAl


def pack_full_right(plan, B, CBt=None, stream=None):
    """Right operand of full compression, packed along n in Theta = Q^(d+1) (FULL plans)."""
    import torch
    _u8(B, "B")
    k, n = B.shape
    if CBt is None:
        CBt = _new(torch.empty((k, -(-n // (plan.d2 + 1))), dtype=word_dtype(plan), device=B.device), stream)
    _check(lib().qmm_pack_full_right(ctypes.byref(plan), k, n, _ptr(B), _ld(B), _ptr(CBt), _ld(CBt),
                                     _stream(stream)), "qmm_pack_full_right")
    return CBt


def gemm_left_packed(plan, CAl, B, m, C=None, stream=None):
    """Left compression: C = REDQ(CAl x B), d+1 rows of C per word."""
    import torch
    _u8(B, "B")
    k, n = B.shape
    if C is None:
        C = _new(torch.empty((m, n), dtype=torch.uint8, device=B.device), stream)
    _check(lib().qmm_gemm_left_packed(ctypes.byref(plan), m, n, k, _ptr(CAl), _ld(CAl), _ptr(B), _ld(B), _ptr(C),
                                      _ld(C), _stream(stream)), "qmm_gemm_left_packed")
    return C


def gemm_full_packed(plan, CAl, CBt, m, n, C=None, stream=None):
    """Full compression: C = two-variable REDQ of CAl x CBt."""
    import torch
    k = CAl.shape[1]
    if C is None:
        C = _new(torch.empty((m, n), dtype=torch.uint8, device=CAl.device), stream)
    _check(lib().qmm_gemm_full_packed(ctypes.byref(plan), m, n, k, _ptr(CAl), _ld(CAl), _ptr(CBt), _ld(CBt),
                                      _ptr(C), _ld(C), _stream(stream)), "qmm_gemm_full_packed")
    return C


def gemm_right_packed(plan, A, CBr, n, C=None, stream=None):
    """Procedure (5) with B already row-compressed: C = REDQ(A x CBr)."""
    import torch
    _u8(A, "A")
    m, k = A.shape
    if C is None:
        C = _new(torch.empty((m, n), dtype=torch.uint8, device=A.device), stream)
    _check(lib().qmm_gemm_right_packed(ctypes.byref(plan), m, n, k, _ptr(A), _ld(A), _ptr(CBr), _ld(CBr), _ptr(C),
                                       _ld(C), _stream(stream)), "qmm_gemm_right_packed")
    return C


def operand_ld(path, k) -> int:
    """Row stride (bytes) of the packed INT8 (Bt) or FP4 (A4, Bt4) operands for inner
    dimension k: the library's own choice (qmm_operand_ld)."""
    pl = Plan(path=path)
    out = ctypes.c_int64(0)
    _check(lib().qmm_operand_ld(ctypes.byref(pl), k, ctypes.byref(out)), "qmm_operand_ld")
    return out.value


def centred_ld(k) -> int:
    """Leading dimension of the centred, transposed right operand of the INT8 path."""
    return operand_ld(PATH_INT8, k)


def pack_centred_cols(plan, B, Bt=None, stream=None):
    """INT8 conversion step: Bt = centred(B)^T (n x centred_ld(k), int8)."""
    import torch
    _u8(B, "B")
    k, n = B.shape
    if Bt is None:
        Bt = _new(torch.empty((n, centred_ld(k)), dtype=torch.int8, device=B.device), stream)
    _check(lib().qmm_pack_centred_cols(ctypes.byref(plan), k, n, _ptr(B), _ld(B), _ptr(Bt), _ld(Bt), _stream(stream)),
           "qmm_pack_centred_cols")
    return Bt


def gemm_centred(plan, A, Bt, n, C=None, stream=None):
    """INT8 product step: C = centred(A) x Bt^T mod p."""
    import torch
    _u8(A, "A")
    m, k = A.shape
    if C is None:
        C = _new(torch.empty((m, n), dtype=torch.uint8, device=A.device), stream)
    _check(lib().qmm_gemm_centred(ctypes.byref(plan), m, n, k, _ptr(A), _ld(A), _ptr(Bt), _ld(Bt), _ptr(C), _ld(C),
                                  _stream(stream)), "qmm_gemm_centred")
    return C


@dataclass
class Batch:
    handle: ctypes.c_void_p
    count: int
    keep: list

    def run(self, stream=None):
        _check(lib().qmm_gemm_mod_p_batched(self.handle, _stream(stream)), "qmm_gemm_mod_p_batched")

    def plan(self, i) -> Plan:
        pl = Plan()
        _check(lib().qmm_batched_plan(self.handle, i, ctypes.byref(pl)), "qmm_batched_plan")
        return pl

    def destroy(self):
        if self.handle:
            lib().qmm_batched_destroy(self.handle)
            self.handle = ctypes.c_void_p(0)


def batched_create(problems, flags=0) -> Batch:
    """problems: list of (A, B, C, p) uint8 device tensors; C is written by run()."""
    arr = (Problem * len(problems))()
    for i, (A, B, C, p) in enumerate(problems):
        m, k = A.shape
        n = B.shape[1]
        arr[i] = Problem(m, n, k, p, A.data_ptr(), _ld(A), B.data_ptr(), _ld(B), C.data_ptr(), _ld(C))
    h = ctypes.c_void_p(0)
    _check(lib().qmm_batched_create(len(problems), arr, flags, ctypes.byref(h)), "qmm_batched_create")
    return Batch(h, len(problems), [problems])


def batched_tune_workspace_size(m=256, n=256) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().qmm_batched_tune_workspace_size(m, n, ctypes.byref(out)), "qmm_batched_tune_workspace_size")
    return out.value


def batched_tune(p=7, m=256, n=256, ws=None, stream=None, device="cuda"):
    """Calibrate the batched autotuner on this GPU with m x n products at prime p;
    returns the 8 fitted costs.  ws: a device uint8 tensor of at least
    batched_tune_workspace_size(m, n) bytes (allocated here when None)."""
    import torch
    if ws is None:
        ws = _new(torch.empty(batched_tune_workspace_size(m, n), dtype=torch.uint8, device=device), stream)
    out = (ctypes.c_double * N_BATCH_COSTS)()
    _check(lib().qmm_batched_tune(p, m, n, _ptr(ws), ws.numel(), _stream(stream), out), "qmm_batched_tune")
    return list(out)


def tune_cache_put(arch, p, m, n, costs):
    if len(costs) != N_BATCH_COSTS:
        raise ValueError(f"expected {N_BATCH_COSTS} costs, got {len(costs)}")
    arr = (ctypes.c_double * N_BATCH_COSTS)(*costs)
    _check(lib().qmm_tune_cache_put(arch.encode(), p, m, n, arr), "qmm_tune_cache_put")


def tune_cache_get(arch, p, m, n):
    """The cached costs for (arch, encoding of p, nearest shape bucket), or None."""
    arr = (ctypes.c_double * N_BATCH_COSTS)()
    st = lib().qmm_tune_cache_get(arch.encode(), p, m, n, arr)
    if st == EVALUE:
        return None
    _check(st, "qmm_tune_cache_get")
    return list(arr)


def tune_cache_load(path):
    _check(lib().qmm_tune_cache_load(os.fsencode(path)), "qmm_tune_cache_load")


def tune_cache_save(path):
    _check(lib().qmm_tune_cache_save(os.fsencode(path)), "qmm_tune_cache_save")


def tune_cache_clear():
    _check(lib().qmm_tune_cache_clear(), "qmm_tune_cache_clear")


def batched_set_costs(costs):
    if len(costs) != N_BATCH_COSTS:
        raise ValueError(f"expected {N_BATCH_COSTS} costs, got {len(costs)}")
    arr = (ctypes.c_double * N_BATCH_COSTS)(*costs)
    _check(lib().qmm_batched_set_costs(arr), "qmm_batched_set_costs")


def fp4_ld(k) -> int:
    """Row stride (bytes) of packed FP4 operands."""
    return operand_ld(PATH_FP4, k)


def pack_fp4_rows(plan, A, A4=None, stream=None):
    """FP4 conversion of the left operand: A4 = codes of centred(A) (m x fp4_ld(k) bytes)."""
    import torch
    _u8(A, "A")
    m, k = A.shape
    if A4 is None:
        A4 = _new(torch.empty((m, fp4_ld(k)), dtype=torch.uint8, device=A.device), stream)
    _check(lib().qmm_pack_fp4_rows(ctypes.byref(plan), m, k, _ptr(A), _ld(A), _ptr(A4), _ld(A4), _stream(stream)),
           "qmm_pack_fp4_rows")
    return A4


def pack_fp4_cols(plan, B, Bt4=None, stream=None):
    """FP4 conversion of the right operand: Bt4 = codes of centred(B)^T (n x fp4_ld(k) bytes)."""
    import torch
    _u8(B, "B")
    k, n = B.shape
    if Bt4 is None:
        Bt4 = _new(torch.empty((n, fp4_ld(k)), dtype=torch.uint8, device=B.device), stream)
    _check(lib().qmm_pack_fp4_cols(ctypes.byref(plan), k, n, _ptr(B), _ld(B), _ptr(Bt4), _ld(Bt4), _stream(stream)),
           "qmm_pack_fp4_cols")
    return Bt4


def gemm_fp4(plan, A4, Bt4, k, C=None, stream=None):
    """FP4 product step: C = (A4 x Bt4^T) mod p from the packed operands."""
    import torch
    m, n = A4.shape[0], Bt4.shape[0]
    if C is None:
        C = _new(torch.empty((m, n), dtype=torch.uint8, device=A4.device), stream)
    _check(lib().qmm_gemm_fp4(ctypes.byref(plan), m, n, k, _ptr(A4), _ld(A4), _ptr(Bt4), _ld(Bt4), _ptr(C), _ld(C),
                              _stream(stream)), "qmm_gemm_fp4")
    return C


def pack_fp4(plan, A, B, A4=None, Bt4=None, stream=None):
    """Both FP4 conversions in one launch: (A4, Bt4) as pack_fp4_rows / pack_fp4_cols."""
    import torch
    _u8(A, "A")
    _u8(B, "B")
    m, k = A.shape
    n = B.shape[1]
    if A4 is None:
        A4 = _new(torch.empty((m, fp4_ld(k)), dtype=torch.uint8, device=A.device), stream)
    if Bt4 is None:
        Bt4 = _new(torch.empty((n, fp4_ld(k)), dtype=torch.uint8, device=B.device), stream)
    _check(lib().qmm_pack_fp4(ctypes.byref(plan), m, n, k, _ptr(A), _ld(A), _ptr(B), _ld(B), _ptr(A4), _ld(A4),
                              _ptr(Bt4), _ld(Bt4), _stream(stream)), "qmm_pack_fp4")
    return A4, Bt4
