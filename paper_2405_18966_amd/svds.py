"""Thin Python binding of the C ABI (include/svds.h, include/svds_ops.h).

Argument marshalling only: the functions below take torch tensors that live
on the GPU (device memory and streams come from PyTorch), build the C structs
and call libsvds.so, whose HIP kernels do all the work.  Names follow the C
entry points.  The library is loaded from this package directory; if it is
missing the import fails with an explicit error -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsvds.so")

SVDS_OK, SVDS_NOT_CONVERGED = 0, 1
SVDS_EINVAL, SVDS_ENOMEM, SVDS_EDEVICE, SVDS_EUNSUPPORTED = -1, -2, -3, -4
SVDS_F64, SVDS_F32, SVDS_BF16 = 0, 1, 2
SVDS_CGS2_NOALLOC_MAX_VECTOR_BYTES = 16 << 20  # svds_op_cgs2_noalloc: L * element size
SVDS_PREC_FP64, SVDS_PREC_MIXED = 0, 1
SVDS_FLAG_TIMING, SVDS_FLAG_NO_RESIDUALS, SVDS_FLAG_NO_SIGNFIX, SVDS_FLAG_GRAPH, SVDS_FLAG_AUTOTUNE = 1, 2, 4, 8, 16
SVDS_FLAG_ITEMS_1K, SVDS_FLAG_UNSORTED, SVDS_FLAG_NO_PANELS, SVDS_FLAG_SMALLEST = 32, 64, 128, 256
SVDS_FLAG_SELECTIVE_REORTH = 512
SVDS_FLAG_PARTIAL_REORTH = 1024
SVDS_FLAG_EARLY_STOP = 2048
SVDS_FLAG_HARMONIC = 4096
SVDS_FLAG_EXPECT_BREAKDOWNS = 8192
KERNEL_CLASSES = ["spmv", "spmvT", "cgs_proj", "cgs_updproj", "cgs_updnorm", "cgs_reduce", "smallsvd",
                  "rotate", "other"]
KC_COUNT = len(KERNEL_CLASSES)


class svds_csr(C.Structure):
    _fields_ = [("m", C.c_int64), ("n", C.c_int64), ("nnz", C.c_int64),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("val", C.c_void_p),
                ("dtype", C.c_int32)]


class svds_dense(C.Structure):
    _fields_ = [("m", C.c_int64), ("n", C.c_int64), ("ld", C.c_int64),
                ("a", C.c_void_p), ("dtype", C.c_int32)]


class svds_opts(C.Structure):
    _fields_ = [("k", C.c_int32), ("p", C.c_int32), ("tol", C.c_double), ("maxit", C.c_int32),
                ("precision", C.c_int32), ("seed", C.c_uint64), ("v0", C.c_void_p),
                ("stream", C.c_void_p), ("flags", C.c_int32)]


class svds_tuning(C.Structure):
    _fields_ = [("tuned", C.c_int32), ("fwd_nnz_cap", C.c_int32), ("fwd_sorted", C.c_int32),
                ("bwd_nnz_cap", C.c_int32), ("bwd_sorted", C.c_int32), ("bwd_panels", C.c_int32),
                ("cgs_slab_shift", C.c_int32), ("cgs_cpw", C.c_int32),
                ("fwd_us", C.c_double), ("fwd_default_us", C.c_double), ("bwd_us", C.c_double),
                ("bwd_default_us", C.c_double), ("cgs_us", C.c_double), ("cgs_default_us", C.c_double),
                ("ms_tune", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class svds_info(C.Structure):
    _fields_ = [("nconv", C.c_int32), ("cycles", C.c_int32), ("cycles_fp32", C.c_int32),
                ("cycles_fp64", C.c_int32), ("breakdowns", C.c_int32), ("converged", C.c_int32),
                ("n_spmv", C.c_int64), ("n_spmvT", C.c_int64),
                ("max_res_est", C.c_double), ("max_res_true", C.c_double), ("max_res_av", C.c_double),
                ("ms_total", C.c_double), ("bytes_alg", C.c_double),
                ("kc_ms", C.c_double * KC_COUNT), ("kc_bytes", C.c_double * KC_COUNT),
                ("kc_flops", C.c_double * KC_COUNT), ("kc_launches", C.c_int64 * KC_COUNT),
                ("kc_sampled_launches", C.c_int64 * KC_COUNT), ("kc_sampled_bytes", C.c_double * KC_COUNT),
                ("workspace_bytes", C.c_int64), ("graph_captures", C.c_int32),
                ("graph_replays", C.c_int32), ("tuning", svds_tuning), ("reorth_tests", C.c_int32),
                ("reorth_second_passes", C.c_int32), ("partial_steps", C.c_int64),
                ("partial_columns", C.c_int64), ("partial_possible", C.c_int64),
                ("early_checks", C.c_int32), ("lanczos_dim_last", C.c_int32)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if not f.startswith("kc_") and f != "tuning"}
        d["tuning"] = self.tuning.as_dict()
        for f in ("kc_ms", "kc_bytes", "kc_flops", "kc_launches", "kc_sampled_launches", "kc_sampled_bytes"):
            d[f] = dict(zip(KERNEL_CLASSES, list(getattr(self, f))))
        return d


def _load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"native library {LIB_PATH} not built: run "
                           "`python -c 'import __graft_entry__ as g; g.build()'` first")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, d, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_uint64
    P = C.POINTER
    sig = {
        "svds_plan_create_csr": (i32, [P(svds_csr), P(svds_opts), P(vp)]),
        "svds_plan_create_dense": (i32, [P(svds_dense), P(svds_opts), P(vp)]),
        "svds_plan_execute": (i32, [vp, vp, vp, vp, P(svds_info)]),
        "svds_plan_destroy": (None, [vp]),
        "svds_csr_solve": (i32, [P(svds_csr), P(svds_opts), vp, vp, vp, P(svds_info)]),
        "svds_dense_solve": (i32, [P(svds_dense), P(svds_opts), vp, vp, vp, P(svds_info)]),
        "svds_csr_solve_batched": (i32, [i32, P(svds_csr), P(svds_opts), P(vp), P(vp), P(vp),
                                         P(svds_info)]),
        "svds_residuals_csr": (i32, [P(svds_csr), i32, vp, vp, vp, vp, vp, vp]),
        "svds_residuals_dense": (i32, [P(svds_dense), i32, vp, vp, vp, vp, vp, vp]),
        "svds_strerror": (C.c_char_p, [i32]),
        "svds_version": (C.c_char_p, []),
        "svds_op_spmv_csr": (i32, [P(svds_csr), vp, vp, vp, vp, vp, i32, vp]),
        "svds_op_dense_matvec": (i32, [P(svds_dense), i32, vp, vp, vp, vp, vp, i32, vp]),
        "svds_op_csr_matvec": (i32, [P(svds_csr), i32, vp, vp, vp, vp, vp, i32, P(i32), vp]),
        "svds_op_csc_build": (i32, [P(svds_csr), vp, vp, vp, vp]),
        "svds_op_cgs2": (i32, [i64, i32, vp, i64, vp, vp, P(d), i32, vp]),
        "svds_op_cgs2_noalloc": (i32, [i64, i32, vp, i64, vp, vp, P(d), i32, vp]),
        "svds_op_small_svd": (i32, [i32, i32, d, vp, vp, vp, vp, vp, vp, P(i32), vp]),
        "svds_op_harmonic_basis": (i32, [i32, i32, vp, vp, vp, vp, vp]),
        "svds_op_gather_copy": (i32, [i64, vp, vp, vp, i32, vp, i32, P(d), vp]),
        "svds_op_rotate": (i32, [i64, i32, i32, vp, i64, i32, vp, i64, vp, i64, vp]),
        "svds_op_philox_normal": (i32, [i64, u64, C.c_uint32, vp, vp]),
        "svds_op_copy_f64": (i32, [i64, vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


class SvdsError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {lib.svds_strerror(code).decode()} (code {code})")
        self.code = code


def _check(rc: int, where: str) -> int:
    if rc < 0:
        raise SvdsError(rc, where)
    return rc


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


_VT = {torch.float64: SVDS_F64, torch.float32: SVDS_F32, torch.uint16: SVDS_BF16,
       torch.bfloat16: SVDS_BF16}


def make_csr(row_ptr: torch.Tensor, col_idx: torch.Tensor, val: torch.Tensor, m: int, n: int) -> svds_csr:
    """C struct for a device CSR (int32 row_ptr/col_idx, FP64/FP32 values);
    it holds references to the three tensors (see make_dense)."""
    assert row_ptr.dtype == torch.int32 and col_idx.dtype == torch.int32
    assert row_ptr.is_cuda and col_idx.is_cuda and val.is_cuda
    assert row_ptr.numel() == m + 1
    c = svds_csr(m, n, col_idx.numel(), row_ptr.data_ptr(), col_idx.data_ptr(), val.data_ptr(),
                 _VT[val.dtype])
    c._keep = (row_ptr, col_idx, val)
    return c


def make_dense(a: torch.Tensor, m: int, n: int) -> svds_dense:
    """C struct for a column-major device matrix given as a 1-D tensor of
    m*n (ld = m) FP64/FP32 values or BF16 bit patterns (uint16/bfloat16).
    The struct holds a reference to `a`, so the memory stays allocated while
    the struct lives (a tensor made inline would otherwise go back to
    torch's caching allocator at once and be handed to the next tensor)."""
    assert a.is_cuda and a.numel() == m * n
    d = svds_dense(m, n, m, a.data_ptr(), _VT[a.dtype])
    d._keep = a
    return d


def make_opts(k, p=0, tol=0.0, maxit=0, precision=SVDS_PREC_FP64, seed=0, v0=None, flags=0,
              stream=None) -> svds_opts:
    """Solver options; the struct holds a reference to the device tensor v0
    (see make_dense)."""
    o = svds_opts(k, p, tol, maxit, precision, seed, None if v0 is None else v0.data_ptr(),
                  _stream(stream), flags)
    o._keep = v0
    return o


def _outputs(m, n, k, device):
    U = torch.empty((k, m), dtype=torch.float64, device=device)  # column j = U[j]
    S = torch.empty(k, dtype=torch.float64, device=device)
    V = torch.empty((k, n), dtype=torch.float64, device=device)
    return U, S, V


@dataclass
class Result:
    U: torch.Tensor   # m x k (a transposed view of column-major storage)
    S: torch.Tensor   # k
    V: torch.Tensor   # n x k
    info: dict
    status: int


def svds_csr_solve(A: svds_csr, opts: svds_opts) -> Result:
    """k largest singular triplets of a device CSR matrix (create + execute +
    destroy of a plan)."""
    dev = torch.device("cuda", torch.cuda.current_device())
    U, S, V = _outputs(A.m, A.n, opts.k, dev)
    info = svds_info()
    rc = _check(lib.svds_csr_solve(C.byref(A), C.byref(opts), _ptr(U), _ptr(S), _ptr(V),
                                   C.byref(info)), "svds_csr_solve")
    return Result(U.T, S, V.T, info.as_dict(), rc)


def svds_dense_solve(A: svds_dense, opts: svds_opts) -> Result:
    dev = torch.device("cuda", torch.cuda.current_device())
    U, S, V = _outputs(A.m, A.n, opts.k, dev)
    info = svds_info()
    rc = _check(lib.svds_dense_solve(C.byref(A), C.byref(opts), _ptr(U), _ptr(S), _ptr(V),
                                     C.byref(info)), "svds_dense_solve")
    return Result(U.T, S, V.T, info.as_dict(), rc)


class Plan:
    """svds_plan_create_* / svds_plan_execute / svds_plan_destroy."""

    def __init__(self, A, opts: svds_opts):
        self._A = A      # keep the struct (and the tensors it holds) alive
        self._opts = opts
        self.m, self.n, self.k = A.m, A.n, opts.k
        h = C.c_void_p()
        if isinstance(A, svds_csr):
            _check(lib.svds_plan_create_csr(C.byref(A), C.byref(opts), C.byref(h)), "svds_plan_create_csr")
        else:
            _check(lib.svds_plan_create_dense(C.byref(A), C.byref(opts), C.byref(h)), "svds_plan_create_dense")
        self._h = h

    def execute(self, out=None) -> Result:
        dev = torch.device("cuda", torch.cuda.current_device())
        U, S, V = out if out is not None else _outputs(self.m, self.n, self.k, dev)
        info = svds_info()
        rc = _check(lib.svds_plan_execute(self._h, _ptr(U), _ptr(S), _ptr(V), C.byref(info)),
                    "svds_plan_execute")
        return Result(U.T, S, V.T, info.as_dict(), rc)

    def destroy(self):
        if self._h:
            lib.svds_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


svds_plan_create_csr = Plan
svds_plan_create_dense = Plan


def svds_csr_solve_batched(As, opts: svds_opts):
    dev = torch.device("cuda", torch.cuda.current_device())
    outs = [_outputs(A.m, A.n, opts.k, dev) for A in As]
    arr = (svds_csr * len(As))(*As)
    Up = (C.c_void_p * len(As))(*[o[0].data_ptr() for o in outs])
    Sp = (C.c_void_p * len(As))(*[o[1].data_ptr() for o in outs])
    Vp = (C.c_void_p * len(As))(*[o[2].data_ptr() for o in outs])
    infos = (svds_info * len(As))()
    rc = _check(lib.svds_csr_solve_batched(len(As), arr, C.byref(opts), Up, Sp, Vp, infos),
                "svds_csr_solve_batched")
    return [Result(o[0].T, o[1], o[2].T, infos[i].as_dict(), rc) for i, o in enumerate(outs)], rc


def svds_residuals_csr(A: svds_csr, U: torch.Tensor, S: torch.Tensor, V: torch.Tensor, stream=None):
    """(|A v_j - s_j u_j|, |A^T u_j - s_j v_j|) for column-major U (m x k), V (n x k)."""
    k = S.numel()
    Uc = U.T.contiguous()
    Vc = V.T.contiguous()
    r1 = torch.empty(k, dtype=torch.float64, device=S.device)
    r2 = torch.empty(k, dtype=torch.float64, device=S.device)
    _check(lib.svds_residuals_csr(C.byref(A), k, _ptr(Uc), _ptr(S), _ptr(Vc), _ptr(r1), _ptr(r2),
                                  _stream(stream)), "svds_residuals_csr")
    return r1, r2


def svds_residuals_dense(A: svds_dense, U: torch.Tensor, S: torch.Tensor, V: torch.Tensor, stream=None):
    """(|A v_j - s_j u_j|, |A^T u_j - s_j v_j|) for a dense A and column-major U (m x k), V (n x k)."""
    k = S.numel()
    Uc = U.T.contiguous()
    Vc = V.T.contiguous()
    r1 = torch.empty(k, dtype=torch.float64, device=S.device)
    r2 = torch.empty(k, dtype=torch.float64, device=S.device)
    _check(lib.svds_residuals_dense(C.byref(A), k, _ptr(Uc), _ptr(S), _ptr(Vc), _ptr(r1), _ptr(r2),
                                    _stream(stream)), "svds_residuals_dense")
    return r1, r2


# --- single steps -------------------------------------------------------------

def svds_op_spmv_csr(A: svds_csr, x, x_scale=None, coef=None, yprev=None, y=None, stream=None):
    dt = SVDS_F64 if x.dtype == torch.float64 else SVDS_F32
    if y is None:
        y = torch.empty(A.m, dtype=x.dtype, device=x.device)
    _check(lib.svds_op_spmv_csr(C.byref(A), _ptr(x), _ptr(x_scale), _ptr(coef), _ptr(yprev), _ptr(y), dt,
                                _stream(stream)), "svds_op_spmv_csr")
    return y


def svds_op_csr_matvec(A: svds_csr, transpose: bool, x, x_scale=None, coef=None, yprev=None, y=None,
                       stream=None):
    """Returns (y, panels): panels = column panels the transposed product used."""
    dt = SVDS_F64 if x.dtype == torch.float64 else SVDS_F32
    if y is None:
        y = torch.empty(A.n if transpose else A.m, dtype=x.dtype, device=x.device)
    np_ = C.c_int32(0)
    _check(lib.svds_op_csr_matvec(C.byref(A), int(transpose), _ptr(x), _ptr(x_scale), _ptr(coef), _ptr(yprev),
                                  _ptr(y), dt, C.byref(np_), _stream(stream)), "svds_op_csr_matvec")
    return y, np_.value


def svds_op_dense_matvec(A: svds_dense, transpose: bool, x, x_scale=None, coef=None, yprev=None,
                         y=None, stream=None):
    dt = SVDS_F64 if x.dtype == torch.float64 else SVDS_F32
    if y is None:
        y = torch.empty(A.n if transpose else A.m, dtype=x.dtype, device=x.device)
    _check(lib.svds_op_dense_matvec(C.byref(A), int(transpose), _ptr(x), _ptr(x_scale), _ptr(coef),
                                    _ptr(yprev), _ptr(y), dt, _stream(stream)), "svds_op_dense_matvec")
    return y


def svds_op_csc_build(A: svds_csr, val_dtype=torch.float64, stream=None):
    dev = torch.device("cuda", torch.cuda.current_device())
    trp = torch.empty(A.n + 1, dtype=torch.int32, device=dev)
    tci = torch.empty(max(A.nnz, 1), dtype=torch.int32, device=dev)
    tv = torch.empty(max(A.nnz, 1), dtype=val_dtype, device=dev)
    _check(lib.svds_op_csc_build(C.byref(A), _ptr(trp), _ptr(tci), _ptr(tv), _stream(stream)),
           "svds_op_csc_build")
    return trp, tci[:A.nnz], tv[:A.nnz]


def svds_op_cgs2(Q: torch.Tensor, j: int, w: torch.Tensor, ldq: int | None = None, stream=None):
    """Q: column-major basis given as a (cols, ldq) tensor (column c = Q[c])."""
    dt = SVDS_F64 if w.dtype == torch.float64 else SVDS_F32
    L = w.numel()
    out = torch.empty_like(w)
    nrm = C.c_double()
    _check(lib.svds_op_cgs2(L, j, _ptr(Q) if j > 0 else None, ldq or (Q.shape[1] if j > 0 else L), _ptr(w),
                            _ptr(out), C.byref(nrm), dt, _stream(stream)), "svds_op_cgs2")
    return out, nrm.value


def svds_op_cgs2_noalloc(Q: torch.Tensor, j: int, w: torch.Tensor, out: torch.Tensor,
                         ldq: int | None = None, stream=None) -> float:
    """svds_op_cgs2 into a caller-given `out` through the entry point that
    allocates no device memory; returns the norm."""
    dt = SVDS_F64 if w.dtype == torch.float64 else SVDS_F32
    nrm = C.c_double()
    _check(lib.svds_op_cgs2_noalloc(w.numel(), j, _ptr(Q) if j > 0 else None,
                                    ldq or (Q.shape[1] if j > 0 else w.numel()), _ptr(w), _ptr(out),
                                    C.byref(nrm), dt, _stream(stream)), "svds_op_cgs2_noalloc")
    return nrm.value


def svds_op_small_svd(T: torch.Tensor, p: int, k: int, tol: float, stream=None):
    """T: (p+1) x (p+1) row-major FP64 device tensor (overwritten by the
    restarted matrix).  Returns Uk (k x p: row j = left vector j), Vext
    ((k+1) x (p+1)), sig, res, rho, flags."""
    dev = T.device
    Uk = torch.empty((k, p), dtype=torch.float64, device=dev)
    Vext = torch.empty((k + 1, p + 1), dtype=torch.float64, device=dev)
    sig = torch.empty(k, dtype=torch.float64, device=dev)
    res = torch.empty(k, dtype=torch.float64, device=dev)
    rho = torch.empty(k, dtype=torch.float64, device=dev)
    flags = (C.c_int32 * 3)()
    _check(lib.svds_op_small_svd(p, k, tol, _ptr(T), _ptr(Uk), _ptr(Vext), _ptr(sig), _ptr(res), _ptr(rho),
                                 flags, _stream(stream)), "svds_op_small_svd")
    return Uk, Vext, sig, res, rho, list(flags)


def svds_op_harmonic_basis(T: torch.Tensor, p: int, k: int, stream=None):
    """T: (p+1) x (p+1) row-major FP64 device tensor (only read).  Returns
    QC ((k+1) x (p+1): row j = column j of Q_C), QM (k x p: row j = column j
    of Q_M) and R (k x k)."""
    dev = T.device
    QC = torch.empty((k + 1, p + 1), dtype=torch.float64, device=dev)
    QM = torch.empty((k, p), dtype=torch.float64, device=dev)
    R = torch.empty((k, k), dtype=torch.float64, device=dev)
    _check(lib.svds_op_harmonic_basis(p, k, _ptr(T), _ptr(QC), _ptr(QM), _ptr(R), _stream(stream)),
           "svds_op_harmonic_basis")
    return QC, QM, R


def svds_op_gather_copy(idx: torch.Tensor, x: torch.Tensor, nseg: int = 1, seg=None, out=None, reps: int = 1,
                        stream=None):
    """out[i] = x[idx[i]]; seg: host sequence of nseg + 1 offsets (or None).
    Returns (out, average ms per launch over `reps` back-to-back launches)."""
    assert idx.dtype == torch.int32 and x.dtype == torch.float64
    if out is None:
        out = torch.empty(idx.numel(), dtype=torch.float64, device=x.device)
    sp = None if seg is None else (C.c_int64 * (nseg + 1))(*[int(v) for v in seg])
    ms = C.c_double()
    _check(lib.svds_op_gather_copy(idx.numel(), _ptr(idx), _ptr(x), _ptr(out), nseg, sp, reps, C.byref(ms),
                                   _stream(stream)), "svds_op_gather_copy")
    return out, ms.value


SVDS_ROTATE_VECTOR = 256


def svds_op_rotate(B: torch.Tensor, pc: int, Y: torch.Tensor, kc: int, stream=None, vector: bool = False):
    """B: (pc, L) tensor (column-major L x pc), Y: (kc, pc) FP64 (column-major
    pc x kc).  Returns out as (kc, L).  ``vector``: the vector-FMA kernel
    instead of the matrix-core one."""
    L = B.shape[1]
    out = torch.empty((kc, L), dtype=torch.float64, device=B.device)
    bt = (SVDS_F64 if B.dtype == torch.float64 else SVDS_F32) | (SVDS_ROTATE_VECTOR if vector else 0)
    _check(lib.svds_op_rotate(L, pc, kc, _ptr(B), L, bt, _ptr(Y), Y.shape[1], _ptr(out), L, _stream(stream)),
           "svds_op_rotate")
    return out


def svds_op_philox_normal(L: int, seed: int, stream_id: int, stream=None):
    dev = torch.device("cuda", torch.cuda.current_device())
    out = torch.empty(L, dtype=torch.float64, device=dev)
    _check(lib.svds_op_philox_normal(L, seed, stream_id, _ptr(out), _stream(stream)), "svds_op_philox_normal")
    return out


def svds_op_copy_f64(src: torch.Tensor, dst: torch.Tensor, stream=None):
    _check(lib.svds_op_copy_f64(src.numel(), _ptr(src), _ptr(dst), _stream(stream)), "svds_op_copy_f64")
    return dst


# --- conveniences ---------------------------------------------------------------

def csr_to_device(A, dtype=None, device="cuda"):
    """Upload an ``inputs.CSR`` to the device; returns (struct, tensors)."""
    val = torch.from_numpy(A.val)
    if dtype is not None:
        val = val.to(dtype)
    t = (torch.from_numpy(A.row_ptr).to(device), torch.from_numpy(A.col_idx).to(device), val.to(device))
    return make_csr(t[0], t[1], t[2], A.m, A.n), t
