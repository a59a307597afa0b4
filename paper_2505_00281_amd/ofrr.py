"""Thin Python binding of the C ABI in include/ofrr.h (ctypes).

Argument marshalling only: torch tensors supply device memory and the
current HIP stream; every step of the method runs in the HIP library
libofrr.so.  There is no fallback: if the library is missing or no GPU is
visible, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libofrr.so")

# ofrr_status
OK, NOT_CONVERGED = 0, 1
ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_NO_DEVICE, ERR_OOM, ERR_HIP, ERR_NUMERIC = -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", -1: "INVALID_ARG", -2: "UNSUPPORTED",
                -3: "NO_DEVICE", -4: "OOM", -5: "HIP", -6: "NUMERIC"}
# enums
DENSE, CSR = 0, 1
F64, F32, BF16, F16, F8E4M3 = 0, 1, 2, 3, 4
ACC_F32, ACC_F32_COMPENSATED, ACC_F64 = 0, 1, 2
LARGEST, SMALLEST = 0, 1
POWER, CHEBYSHEV = 0, 1

_DTYPES = {"f64": F64, "f32": F32, "bf16": BF16, "f16": F16, "f8e4m3": F8E4M3}
_ACCUM = {"f32": ACC_F32, "f32c": ACC_F32_COMPENSATED, "f64": ACC_F64}
_WHICH = {"largest": LARGEST, "smallest": SMALLEST}
_FILTER = {"power": POWER, "chebyshev": CHEBYSHEV}
_TAIL = {"f64": 0, "i8": 1}

EXPORTED = ["ofrr_plan_default", "ofrr_create", "ofrr_destroy", "ofrr_last_error",
            "ofrr_kernel_stats", "ofrr_kernel_stats_reset", "ofrr_set_profile", "ofrr_eig_partial",
            "ofrr_svd_partial", "ofrr_eig_partial_batched", "ofrr_batched_last_config", "ofrr_krylov_eig",
            "ofrr_quantize",
            "ofrr_quantize_fp8_blocks", "ofrr_block_product", "ofrr_block_product_sliced",
            "ofrr_block_product_fp8", "ofrr_hessenberg", "ofrr_hessenberg_noalloc", "ofrr_basis_generate",
            "ofrr_project", "ofrr_pencil_eig", "ofrr_svd_pencil", "ofrr_eig_general",
            "ofrr_pencil_eig_general"]


class OfrrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Matrix(ctypes.Structure):
    _fields_ = [("format", ctypes.c_int), ("dtype", ctypes.c_int), ("rows", ctypes.c_int64),
                ("cols", ctypes.c_int64), ("ld", ctypes.c_int64), ("values", ctypes.c_void_p),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("nnz", ctypes.c_int64)]


class Plan(ctypes.Structure):
    _fields_ = [("basis_dtype", ctypes.c_int), ("gram_accum", ctypes.c_int),
                ("refine", ctypes.c_int32), ("filter", ctypes.c_int), ("degree", ctypes.c_int32),
                ("lo", ctypes.c_double), ("hi", ctypes.c_double), ("drop_tol", ctypes.c_double),
                ("tol", ctypes.c_double), ("anorm", ctypes.c_double),
                ("max_iters", ctypes.c_int32), ("stall_iters", ctypes.c_int32),
                ("switch_resid", ctypes.c_double), ("b_split", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("tail_product", ctypes.c_int32),
                ("gram_switch_t", ctypes.c_double), ("svd_form", ctypes.c_int32),
                ("stab", ctypes.c_int32), ("projection", ctypes.c_int32),
                ("qr_dtype", ctypes.c_int32), ("matvec_round", ctypes.c_int32),
                ("tail_digits", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("iters_low", ctypes.c_int32),
                ("n_converged", ctypes.c_int32), ("basis_eff", ctypes.c_int32),
                ("products", ctypes.c_int32), ("max_resid", ctypes.c_double),
                ("seconds", ctypes.c_double), ("gram_t_max", ctypes.c_double),
                ("grams_f64", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libofrr.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OfrrError(ERR_UNSUPPORTED, f"HIP library not built: {path} is missing "
                                         "(run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    lib.ofrr_plan_default.argtypes = [P(Plan)]
    lib.ofrr_plan_default.restype = None
    lib.ofrr_create.argtypes = [P(vp), ctypes.c_int, vp]
    lib.ofrr_destroy.argtypes = [vp]
    lib.ofrr_last_error.argtypes = [vp]
    lib.ofrr_last_error.restype = ctypes.c_char_p
    lib.ofrr_kernel_stats.argtypes = [vp, ctypes.c_char_p, P(i64), P(dbl)]
    lib.ofrr_kernel_stats_reset.argtypes = [vp]
    lib.ofrr_set_profile.argtypes = [vp, i32]
    lib.ofrr_eig_partial.argtypes = [vp, P(Matrix), i32, i32, ctypes.c_int, P(Plan), vp, vp, vp,
                                     vp, P(Info)]
    lib.ofrr_svd_partial.argtypes = [vp, P(Matrix), i32, i32, P(Plan), vp, vp, vp, vp, vp, P(Info)]
    lib.ofrr_eig_partial_batched.argtypes = [vp, i32, P(Matrix), i32, i32, ctypes.c_int, P(Plan),
                                             P(vp), P(vp), P(vp), P(vp), P(Info)]
    lib.ofrr_krylov_eig.argtypes = [vp, P(Matrix), i32, i32, i32, ctypes.c_int, vp, dbl, vp, vp, vp, P(Info)]
    lib.ofrr_batched_last_config.argtypes = [vp, P(i32), P(i32), P(i32), P(i32), P(dbl)]
    lib.ofrr_quantize.argtypes = [vp, ctypes.c_int, i64, vp, vp]
    lib.ofrr_quantize_fp8_blocks.argtypes = [vp, i64, i64, vp, i64, vp, vp]
    lib.ofrr_block_product.argtypes = [vp, P(Matrix), i32, i32, ctypes.c_int, vp, vp]
    lib.ofrr_block_product_sliced.argtypes = [vp, P(Matrix), i32, i32, i32, vp, vp]
    lib.ofrr_block_product_fp8.argtypes = [vp, i64, i64, vp, vp, i32, i32, vp, vp]
    lib.ofrr_hessenberg.argtypes = [vp, ctypes.c_int, i64, i32, vp, i64, dbl, vp, vp, P(i32)]
    lib.ofrr_hessenberg_noalloc.argtypes = [vp, ctypes.c_int, i64, i32, vp, i64, dbl, vp, vp, P(i32)]
    lib.ofrr_basis_generate.argtypes = [vp, ctypes.c_int, ctypes.c_int, i64, i32, vp, i64, dbl, vp, vp, vp,
                                        P(i32), P(dbl)]
    lib.ofrr_project.argtypes = [vp, i64, i32, ctypes.c_int, vp, ctypes.c_int, vp, ctypes.c_int,
                                 vp, vp]
    lib.ofrr_pencil_eig.argtypes = [vp, i32, vp, vp, ctypes.c_int, vp, vp, P(i32)]
    lib.ofrr_svd_pencil.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, vp]
    lib.ofrr_eig_general.argtypes = [vp, P(Matrix), i32, i32, P(Plan), vp, vp, vp, vp, vp, vp, P(Info)]
    lib.ofrr_pencil_eig_general.argtypes = [vp, i32, vp, vp, vp, vp, vp]
    for name in EXPORTED:
        if name not in ("ofrr_plan_default", "ofrr_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def make_plan(basis_dtype="f64", gram_accum="f64", refine=False, filter="power", degree=1,
              lo=0.0, hi=0.0, drop_tol=0.0, tol=0.0, anorm=0.0, max_iters=20, stall_iters=3,
              switch_resid=0.0, b_split=1, profile=False, tail="f64", gram_switch_t=0.0,
              svd_form="augmented", stab="hessenberg", projection="ofrr", qr_dtype=None,
              matvec_round=None, tail_digits=0) -> Plan:
    p = Plan()
    load_library().ofrr_plan_default(ctypes.byref(p))
    p.basis_dtype = _DTYPES[basis_dtype] if isinstance(basis_dtype, str) else basis_dtype
    p.gram_accum = _ACCUM[gram_accum] if isinstance(gram_accum, str) else gram_accum
    p.refine = int(refine)  # False/True/0/1/2
    p.filter = _FILTER[filter] if isinstance(filter, str) else filter
    p.degree = degree
    p.lo, p.hi = float(lo), float(hi)
    p.drop_tol, p.tol, p.anorm = float(drop_tol), float(tol), float(anorm)
    p.max_iters, p.stall_iters = max_iters, stall_iters
    p.switch_resid = float(switch_resid)
    p.b_split = b_split
    p.profile = int(bool(profile))
    p.tail_product = _TAIL[tail] if isinstance(tail, str) else int(tail)
    p.gram_switch_t = float(gram_switch_t)
    p.svd_form = {"augmented": 0, "normal": 1}[svd_form] if isinstance(svd_form, str) else int(svd_form)
    p.stab = {"hessenberg": 0, "qr": 1}[stab] if isinstance(stab, str) else int(stab)
    p.projection = {"ofrr": 0, "classical": 1}[projection] if isinstance(projection, str) else int(projection)
    # QR arithmetic of stab="qr" (None: the phase's storage type)
    p.qr_dtype = -1 if qr_dtype is None else (_DTYPES[qr_dtype] if isinstance(qr_dtype, str) else int(qr_dtype))
    # storage type every reduced-phase product is rounded to (None: none)
    p.matvec_round = -1 if matvec_round is None else (
        _DTYPES[matvec_round] if isinstance(matvec_round, str) else int(matvec_round))
    p.tail_digits = int(tail_digits)
    return p


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def dense_matrix(A: torch.Tensor, symmetric: bool = False) -> Matrix:
    """Descriptor of a dense device matrix.  Column-major tensors (stride
    (1, ld)) are passed as they are; a row-major contiguous tensor is the
    column-major storage of its transpose, which is accepted for symmetric
    matrices only."""
    m = Matrix()
    m.format = DENSE
    dt = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16, torch.float16: F16}
    if A.dtype not in dt:
        raise OfrrError(ERR_INVALID_ARG, f"unsupported dtype {A.dtype}")
    m.dtype = dt[A.dtype]
    rows, cols = A.shape
    if A.stride(0) == 1 and (cols == 1 or A.stride(1) >= rows):
        ld = A.stride(1) if cols > 1 else rows
    elif symmetric and rows == cols and A.is_contiguous():
        ld = cols
    else:
        raise OfrrError(ERR_INVALID_ARG, "dense A must be column-major (stride (1, ld))")
    m.rows, m.cols, m.ld = rows, cols, ld
    m.values = A.data_ptr()
    m._keep = (A,)  # the descriptor holds raw pointers: keep the tensor alive with it
    return m


def csr_matrix(row_ptr: torch.Tensor, col_idx: torch.Tensor, values: torch.Tensor,
               n_cols: int | None = None) -> Matrix:
    m = Matrix()
    m.format = CSR
    m.dtype = F64 if values.dtype == torch.float64 else F32
    m.rows = row_ptr.numel() - 1
    m.cols = m.rows if n_cols is None else n_cols
    m.ld = 0
    m.values = values.data_ptr()
    m.row_ptr = row_ptr.data_ptr()
    m.col_idx = col_idx.data_ptr()
    m.nnz = col_idx.numel()
    if row_ptr.dtype != torch.int32 or col_idx.dtype != torch.int32:
        raise OfrrError(ERR_INVALID_ARG, "CSR row_ptr and col_idx must be int32")
    m._keep = (row_ptr, col_idx, values)  # keep the arrays alive with the descriptor
    return m


def _colmajor_f64(X, rows, cols, device):
    if X is None:
        return None
    X = X.to(device=device, dtype=torch.float64)
    if tuple(X.shape) != (rows, cols):
        raise OfrrError(ERR_INVALID_ARG, f"start block must be {rows} x {cols}")
    return X.t().contiguous().t()


def _empty_colmajor(rows, cols, device):
    return torch.empty((cols, rows), dtype=torch.float64, device=device).t()


@dataclass
class EigResult:
    evals: torch.Tensor
    evecs: torch.Tensor
    resid: torch.Tensor
    info: dict
    status: int


@dataclass
class GeneralResult:
    evals: torch.Tensor  # complex128, k
    evecs: torch.Tensor  # complex128, n x k
    resid: torch.Tensor
    info: dict
    status: int


@dataclass
class SvdResult:
    sigma: torch.Tensor
    U: torch.Tensor
    V: torch.Tensor
    resid: torch.Tensor
    info: dict
    status: int


class Context:
    """An ofrr context on one device, bound to torch's current stream of
    that device at creation."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise OfrrError(ERR_NO_DEVICE, "no GPU visible to torch")
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        st = self.lib.ofrr_create(ctypes.byref(h), device, ctypes.c_void_p(self.stream.cuda_stream))
        if st != OK:
            raise OfrrError(st, self.lib.ofrr_last_error(None).decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.ofrr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------- validation
    # Every pointer handed to the library must be device memory of this
    # context's device, and every block must have the rows the operation
    # reads: a host pointer or a short block would otherwise reach a kernel.
    def _on_device(self, *tensors):
        for t in tensors:
            if t is None:
                continue
            if not (t.is_cuda and t.device == self.device):
                raise OfrrError(ERR_INVALID_ARG,
                                f"tensor on {t.device}; this context needs {self.device}")

    def _mat(self, A, symmetric=False) -> Matrix:
        mat = A if isinstance(A, Matrix) else dense_matrix(A, symmetric=symmetric)
        self._on_device(*getattr(mat, "_keep", ()))
        return mat

    @staticmethod
    def _rows(t, rows, what):
        if t.dim() != 2 or t.shape[0] != rows:
            raise OfrrError(ERR_INVALID_ARG, f"{what} must have {rows} rows, got shape {tuple(t.shape)}")

    @staticmethod
    def _dtype(t, allowed, what):
        if t.dtype not in allowed:
            raise OfrrError(ERR_INVALID_ARG, f"{what} has dtype {t.dtype}; expected one of "
                                             f"{[str(d) for d in allowed]}")

    def _check(self, st, allow_warning=False):
        if st < 0 or (st > 0 and not allow_warning):
            raise OfrrError(st, self.lib.ofrr_last_error(self.h).decode())
        return st

    # ---------------------------------------------------------- whole method
    def eig_partial(self, A, k: int, basis: int, which: str = "largest", plan: Plan | None = None,
                    X0=None) -> EigResult:
        mat = self._mat(A, symmetric=True)
        n = mat.rows
        plan = plan or make_plan()
        X0c = _colmajor_f64(X0, n, basis, self.device)
        evals = torch.empty(k, dtype=torch.float64, device=self.device)
        evecs = _empty_colmajor(n, k, self.device)
        resid = torch.empty(k, dtype=torch.float64, device=self.device)
        info = Info()
        st = self.lib.ofrr_eig_partial(self.h, ctypes.byref(mat), k, basis, _WHICH[which],
                                       ctypes.byref(plan), _ptr(X0c), _ptr(evals), _ptr(evecs),
                                       _ptr(resid), ctypes.byref(info))
        self._check(st, allow_warning=True)
        return EigResult(evals, evecs, resid, info.as_dict(), st)

    def eig_general(self, A, k: int, basis: int, plan: Plan | None = None, X0=None) -> GeneralResult:
        """k eigenpairs of largest modulus of a real non-symmetric A (dense
        column-major or CSR); complex values and vectors."""
        mat = self._mat(A)
        n = mat.rows
        plan = plan or make_plan()
        X0c = _colmajor_f64(X0, n, basis, self.device)
        ere = torch.empty(k, dtype=torch.float64, device=self.device)
        eim = torch.empty(k, dtype=torch.float64, device=self.device)
        vre = _empty_colmajor(n, k, self.device)
        vim = _empty_colmajor(n, k, self.device)
        resid = torch.empty(k, dtype=torch.float64, device=self.device)
        info = Info()
        st = self.lib.ofrr_eig_general(self.h, ctypes.byref(mat), k, basis, ctypes.byref(plan), _ptr(X0c),
                                       _ptr(ere), _ptr(eim), _ptr(vre), _ptr(vim), _ptr(resid),
                                       ctypes.byref(info))
        self._check(st, allow_warning=True)
        return GeneralResult(torch.complex(ere, eim), torch.complex(vre, vim), resid, info.as_dict(), st)

    def svd_partial(self, A, k: int, basis: int, plan: Plan | None = None, V0=None) -> SvdResult:
        mat = self._mat(A)
        m, n = mat.rows, mat.cols
        plan = plan or make_plan()
        V0c = _colmajor_f64(V0, n, basis, self.device)
        sigma = torch.empty(k, dtype=torch.float64, device=self.device)
        U = _empty_colmajor(m, k, self.device)
        V = _empty_colmajor(n, k, self.device)
        resid = torch.empty(k, dtype=torch.float64, device=self.device)
        info = Info()
        st = self.lib.ofrr_svd_partial(self.h, ctypes.byref(mat), k, basis, ctypes.byref(plan),
                                       _ptr(V0c), _ptr(sigma), _ptr(U), _ptr(V), _ptr(resid),
                                       ctypes.byref(info))
        self._check(st, allow_warning=True)
        return SvdResult(sigma, U, V, resid, info.as_dict(), st)

    def krylov_eig(self, A, k: int, nev: int, restarts: int = 0, basis_dtype: str = "f64", v0=None,
                   tol: float = 0.0) -> EigResult:
        """Restarted Krylov-Hessenberg + OFRR (ofrr_krylov_eig); A dense or
        a csr_matrix descriptor, symmetric."""
        mat = self._mat(A, symmetric=True)
        n = mat.rows
        if v0 is not None:
            v0 = torch.as_tensor(v0, dtype=torch.float64).reshape(-1).to(self.device).contiguous()
            if v0.numel() != n:
                raise OfrrError(ERR_INVALID_ARG, f"v0 has {v0.numel()} entries, A has {n} rows")
        evals = torch.empty(nev, dtype=torch.float64, device=self.device)
        evecs = _empty_colmajor(n, nev, self.device)
        resid = torch.empty(nev, dtype=torch.float64, device=self.device)
        info = Info()
        st = self.lib.ofrr_krylov_eig(self.h, ctypes.byref(mat), k, nev, restarts, _DTYPES[basis_dtype],
                                      _ptr(v0), float(tol), _ptr(evals), _ptr(evecs), _ptr(resid),
                                      ctypes.byref(info))
        self._check(st, allow_warning=True)
        return EigResult(evals, evecs, resid, info.as_dict(), st)

    def eig_partial_batched(self, As, k: int, basis: int, which: str = "largest",
                            plan: Plan | None = None, X0s=None):
        nprob = len(As)
        # the descriptors (and the tensors they keep alive) live until the call returns
        descs = [self._mat(a, symmetric=True) for a in As]
        mats = (Matrix * nprob)(*descs)
        plan = plan or make_plan()
        X0c = [(_colmajor_f64(X0s[p], mats[p].rows, basis, self.device) if X0s else None)
               for p in range(nprob)]
        outs = []
        for p in range(nprob):
            n = mats[p].rows
            outs.append((torch.empty(k, dtype=torch.float64, device=self.device),
                         _empty_colmajor(n, k, self.device),
                         torch.empty(k, dtype=torch.float64, device=self.device)))
        arr = lambda ts: (ctypes.c_void_p * nprob)(*[t.data_ptr() if t is not None else None for t in ts])
        infos = (Info * nprob)()
        st = self.lib.ofrr_eig_partial_batched(
            self.h, nprob, mats, k, basis, _WHICH[which], ctypes.byref(plan),
            arr(X0c) if X0s else None, arr([o[0] for o in outs]), arr([o[1] for o in outs]),
            arr([o[2] for o in outs]), infos)
        self._check(st, allow_warning=True)
        return [EigResult(o[0], o[1], o[2], infos[p].as_dict(), st) for p, o in enumerate(outs)]

    def set_profile(self, on: bool):
        """Kernel timing for the step calls (see kernel_stats)."""
        self._check(self.lib.ofrr_set_profile(self.h, 1 if on else 0))

    def batched_last_config(self) -> dict:
        """What the last eig_partial_batched call ran: grouped path or not,
        the autotuned row-tile heights of its grouped products, and the
        number of iteration-graph replays."""
        g, rr, rf, rp = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        fm = ctypes.c_double()
        self._check(self.lib.ofrr_batched_last_config(self.h, ctypes.byref(g), ctypes.byref(rr), ctypes.byref(rf),
                                                      ctypes.byref(rp), ctypes.byref(fm)))
        return {"grouped": bool(g.value), "rows_red": rr.value, "rows_f64": rf.value, "replays": rp.value,
                "first_product_ms": fm.value}

    # ----------------------------------------------------------------- steps
    def quantize(self, src: torch.Tensor, dtype: str = "bf16") -> torch.Tensor:
        self._on_device(src)
        self._dtype(src, (torch.float32,), "src")
        src = src.contiguous()
        out = torch.empty(src.shape, dtype=torch.int16, device=self.device)
        self._check(self.lib.ofrr_quantize(self.h, _DTYPES[dtype], src.numel(), _ptr(src), _ptr(out)))
        return out

    def quantize_fp8_blocks(self, A: torch.Tensor):
        mat = self._mat(A)
        if mat.dtype != F32:
            raise OfrrError(ERR_INVALID_ARG, "quantize_fp8_blocks: A must be float32")
        rows, cols = mat.rows, mat.cols
        codes = torch.empty((cols, rows), dtype=torch.uint8, device=self.device).t()
        br, bc = (rows + 31) // 32, (cols + 31) // 32
        scales = torch.empty((bc, br), dtype=torch.float32, device=self.device).t()
        self._check(self.lib.ofrr_quantize_fp8_blocks(self.h, rows, cols, ctypes.c_void_p(mat.values),
                                                      mat.ld, _ptr(codes), _ptr(scales)))
        return codes, scales

    def block_product(self, A, V: torch.Tensor, trans: bool = False, v_dtype: str | None = None):
        """W = op(A) V with V a row-major (rows x b) device block."""
        mat = A if isinstance(A, Matrix) else dense_matrix(A)
        self._rows(V, mat.rows if trans else mat.cols, "V")
        b = V.shape[1]
        rows = mat.cols if trans else mat.rows
        if v_dtype is None:
            v_dtype = {torch.float64: "f64", torch.float32: "f32", torch.float16: "f16",
                       torch.bfloat16: "bf16"}.get(V.dtype)
            if v_dtype is None:
                raise OfrrError(ERR_INVALID_ARG, f"V has dtype {V.dtype}")
        if V.element_size() != {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}.get(v_dtype, 0):
            raise OfrrError(ERR_INVALID_ARG, f"V dtype {V.dtype} does not hold {v_dtype} elements")
        if mat.format == DENSE:
            want = {F64: ("f64",), F32: ("f64",), BF16: ("bf16",), F16: ("f16",)}[mat.dtype]
            if v_dtype not in want:
                raise OfrrError(ERR_INVALID_ARG, f"dense A of this dtype takes V as {want[0]}")
        elif trans:
            raise OfrrError(ERR_INVALID_ARG, "CSR products take trans = 0")
        self._mat(mat)
        self._on_device(V)
        V = V.contiguous()
        if mat.format == DENSE and mat.dtype in (BF16, F16):
            wdt = torch.float32
        elif mat.format == CSR and v_dtype != "f64":
            wdt = torch.float32
        else:
            wdt = torch.float64
        W = torch.empty((rows, b), dtype=wdt, device=self.device)
        self._check(self.lib.ofrr_block_product(self.h, ctypes.byref(mat), int(trans), b,
                                                _DTYPES[v_dtype], _ptr(V), _ptr(W)))
        return W

    def block_product_sliced(self, A, V: torch.Tensor, trans: bool = False, digits: int = 6):
        """W = op(A) V (FP64, row-major) from exact INT8 digit-plane products
        with `digits` (4, 5 or 6) signed 7-bit digits per side; A dense
        F32/F64."""
        mat = A if isinstance(A, Matrix) else dense_matrix(A)
        self._rows(V, mat.rows if trans else mat.cols, "V")
        self._mat(mat)
        self._on_device(V)
        V = V.to(torch.float64).contiguous()
        b = V.shape[1]
        rows = mat.cols if trans else mat.rows
        W = torch.empty((rows, b), dtype=torch.float64, device=self.device)
        self._check(self.lib.ofrr_block_product_sliced(self.h, ctypes.byref(mat), int(trans), b, int(digits),
                                                       _ptr(V), _ptr(W)))
        return W

    def block_product_fp8(self, codes: torch.Tensor, scales: torch.Tensor, V: torch.Tensor,
                          trans: bool = False):
        """W = op(A) V for FP8 block-quantised A (codes, scales from
        quantize_fp8_blocks, column-major) and an FP32 row-major V."""
        self._on_device(codes, scales, V)
        self._dtype(codes, (torch.uint8,), "codes")
        self._dtype(scales, (torch.float32,), "scales")
        rows, cols = codes.shape
        if not (codes.stride(0) == 1 and codes.stride(1) == rows and scales.stride(0) == 1
                and tuple(scales.shape) == ((rows + 31) // 32, (cols + 31) // 32)
                and scales.stride(1) == scales.shape[0]):
            raise OfrrError(ERR_INVALID_ARG, "codes and scales must be the column-major arrays of "
                                             "quantize_fp8_blocks")
        self._rows(V, rows if trans else cols, "V")
        V = V.to(torch.float32).contiguous()
        b = V.shape[1]
        W = torch.empty((cols if trans else rows, b), dtype=torch.float32, device=self.device)
        self._check(self.lib.ofrr_block_product_fp8(self.h, rows, cols, _ptr(codes), _ptr(scales),
                                                    int(trans), b, _ptr(V), _ptr(W)))
        return W

    def hessenberg(self, Y: torch.Tensor, tol: float):
        """In-place Hessenberg process on a row-major (n x b) FP64/FP32 block.
        Returns (piv, keep, kept)."""
        self._on_device(Y)
        self._dtype(Y, (torch.float64, torch.float32), "Y")
        if Y.dim() != 2 or not Y.is_contiguous():
            raise OfrrError(ERR_INVALID_ARG, "Y must be a contiguous (row-major) n x b block")
        n, b = Y.shape
        piv = torch.empty(b, dtype=torch.int32, device=self.device)
        keep = torch.empty(b, dtype=torch.int32, device=self.device)
        kept = ctypes.c_int32()
        dt = F64 if Y.dtype == torch.float64 else F32
        self._check(self.lib.ofrr_hessenberg(self.h, dt, n, b, _ptr(Y), b, float(tol), _ptr(piv),
                                             _ptr(keep), ctypes.byref(kept)))
        return piv, keep, kept.value

    def hessenberg_noalloc(self, Y: torch.Tensor, tol: float, piv: torch.Tensor, keep: torch.Tensor):
        """The allocation-free sweep (ofrr_hessenberg_noalloc) on a row-major
        (n x b) FP64/FP32 block, in place; piv and keep are caller-given
        int32 device vectors of length >= b.  Returns the kept count."""
        self._on_device(Y, piv, keep)
        self._dtype(Y, (torch.float64, torch.float32), "Y")
        self._dtype(piv, (torch.int32,), "piv")
        self._dtype(keep, (torch.int32,), "keep")
        if Y.dim() != 2 or not Y.is_contiguous():
            raise OfrrError(ERR_INVALID_ARG, "Y must be a contiguous (row-major) n x b block")
        n, b = Y.shape
        if piv.numel() < b or keep.numel() < b:
            raise OfrrError(ERR_INVALID_ARG, "piv and keep need b entries")
        kept = ctypes.c_int32()
        dt = F64 if Y.dtype == torch.float64 else F32
        self._check(self.lib.ofrr_hessenberg_noalloc(self.h, dt, n, b, _ptr(Y), b, float(tol), _ptr(piv),
                                                     _ptr(keep), ctypes.byref(kept)))
        return kept.value

    BASIS_METHODS = {"mgs_l": 0, "mgs_r": 1, "cgs": 2, "cgs2": 3, "hess_l": 4, "hess_r": 5, "mgs2": 6}

    def basis_generate(self, A: torch.Tensor, method: str, tol: float = 0.0, want_r: bool = False):
        """ofrr_basis_generate in place on a column-major m x n block (a
        transposed view of a contiguous n x m tensor): float64, float32, or
        float16 (binary16 storage, FP32 arithmetic).  Returns (R or None,
        piv, keep, kept, kernel_ms)."""
        self._on_device(A)
        self._dtype(A, (torch.float64, torch.float32, torch.float16), "A")
        if A.dim() != 2 or A.stride(0) != 1:
            raise OfrrError(ERR_INVALID_ARG, "A must be column-major (a transposed contiguous tensor)")
        m, n = A.shape
        lda = A.stride(1)
        st = {torch.float64: F64, torch.float32: F32, torch.float16: F16}[A.dtype]
        R = torch.zeros((n, n), dtype=torch.float64, device=self.device) if want_r else None
        piv = torch.empty(n, dtype=torch.int32, device=self.device)
        keep = torch.empty(n, dtype=torch.int32, device=self.device)
        kept = ctypes.c_int32()
        ms = ctypes.c_double()
        self._check(self.lib.ofrr_basis_generate(self.h, self.BASIS_METHODS[method], st, m, n, _ptr(A), lda,
                                                 float(tol), _ptr(R) if want_r else None, _ptr(piv), _ptr(keep),
                                                 ctypes.byref(kept), ctypes.byref(ms)))
        # R is column-major: the tensor holds R^T
        return (R.t().contiguous() if want_r else None), piv, keep, kept.value, ms.value

    def project(self, V: torch.Tensor, W: torch.Tensor, accum: str = "f64", v_dtype: str | None = None):
        """G = V^T V, H = V^T W for row-major (n x b) blocks; FP64 b x b
        outputs (column-major; symmetric G)."""
        self._on_device(V, W)
        self._dtype(W, (torch.float64, torch.float32), "W")
        if V.dim() != 2 or tuple(W.shape) != tuple(V.shape):
            raise OfrrError(ERR_INVALID_ARG, f"V {tuple(V.shape)} and W {tuple(W.shape)} must both be n x b")
        V = V.contiguous()
        W = W.contiguous()
        n, b = V.shape
        vdt = v_dtype or {torch.float64: "f64", torch.float32: "f32", torch.float16: "f16",
                          torch.bfloat16: "bf16", torch.int16: "bf16"}.get(V.dtype)
        if vdt is None or V.element_size() != {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}[vdt]:
            raise OfrrError(ERR_INVALID_ARG, f"V dtype {V.dtype} does not hold {vdt} elements")
        wdt = {torch.float64: "f64", torch.float32: "f32"}[W.dtype]
        G = _empty_colmajor(b, b, self.device)
        H = _empty_colmajor(b, b, self.device)
        self._check(self.lib.ofrr_project(self.h, n, b, _DTYPES[vdt], _ptr(V), _DTYPES[wdt], _ptr(W),
                                          _ACCUM[accum], _ptr(G), _ptr(H)))
        return G, H

    def pencil_eig(self, H: torch.Tensor, G: torch.Tensor, which: str = "largest"):
        self._on_device(H, G)
        b = H.shape[0]
        if tuple(H.shape) != (b, b) or tuple(G.shape) != (b, b):
            raise OfrrError(ERR_INVALID_ARG, "H and G must be square and of the same size")
        Hc = H.to(torch.float64).t().contiguous().t()
        Gc = G.to(torch.float64).t().contiguous().t()
        theta = torch.empty(b, dtype=torch.float64, device=self.device)
        Y = _empty_colmajor(b, b, self.device)
        rank = ctypes.c_int32()
        self._check(self.lib.ofrr_pencil_eig(self.h, b, _ptr(Hc), _ptr(Gc), _WHICH[which],
                                             _ptr(theta), _ptr(Y), ctypes.byref(rank)))
        return theta, Y, rank.value

    def pencil_eig_general(self, H: torch.Tensor, G: torch.Tensor):
        """Non-symmetric pencil: (theta_re, theta_im, Y packed real)."""
        self._on_device(H, G)
        b = H.shape[0]
        if tuple(H.shape) != (b, b) or tuple(G.shape) != (b, b):
            raise OfrrError(ERR_INVALID_ARG, "H and G must be square and of the same size")
        Hc = H.to(torch.float64).t().contiguous().t()
        Gc = G.to(torch.float64).t().contiguous().t()
        tre = torch.empty(b, dtype=torch.float64, device=self.device)
        tim = torch.empty(b, dtype=torch.float64, device=self.device)
        Y = _empty_colmajor(b, b, self.device)
        self._check(self.lib.ofrr_pencil_eig_general(self.h, b, _ptr(Hc), _ptr(Gc), _ptr(tre), _ptr(tim), _ptr(Y)))
        return tre, tim, Y

    def svd_pencil(self, B: torch.Tensor, MU: torch.Tensor, MV: torch.Tensor):
        self._on_device(B, MU, MV)
        k1, k2 = B.shape
        if tuple(MU.shape) != (k1, k1) or tuple(MV.shape) != (k2, k2):
            raise OfrrError(ERR_INVALID_ARG, "MU must be k1 x k1 and MV k2 x k2 for a k1 x k2 B")
        r = min(k1, k2)
        cm = lambda t: t.to(torch.float64).t().contiguous().t()
        Bc, MUc, MVc = cm(B), cm(MU), cm(MV)
        sigma = torch.empty(r, dtype=torch.float64, device=self.device)
        Y = _empty_colmajor(k1, r, self.device)
        Z = _empty_colmajor(k2, r, self.device)
        self._check(self.lib.ofrr_svd_pencil(self.h, k1, k2, _ptr(Bc), _ptr(MUc), _ptr(MVc),
                                             _ptr(sigma), _ptr(Y), _ptr(Z)))
        return sigma, Y, Z

    # ---------------------------------------------------------------- timing
    def kernel_stats(self, family: str):
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        self._check(self.lib.ofrr_kernel_stats(self.h, family.encode(), ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    def kernel_stats_reset(self):
        self._check(self.lib.ofrr_kernel_stats_reset(self.h))
