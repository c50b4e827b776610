"""ctypes binding of libsko (include/sko.h): argument marshalling only.

Every computation runs in the HIP library.  Device arrays are torch tensors on a
ROCm device (torch supplies memory and streams, nothing else); tall matrices are
column-major, i.e. 2-D tensors with stride (1, ld).  Importing this module loads
libsko.so and raises if it has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsko.so")

SKO_OK, SKO_EINVAL, SKO_EDEVICE, SKO_ENOMEM, SKO_EBREAKDOWN, SKO_ENOCONV, SKO_EUNSUPPORTED, SKO_ESCRATCH = range(8)
SKO_NOALLOC_SCRATCH_BYTES = 32 << 20
SKO_F64, SKO_MIXED_F32 = 0, 1
SKO_SKETCH_GAUSSIAN, SKO_SKETCH_SPARSE_SIGN, SKO_SKETCH_COUNT_GAUSS = 0, 1, 2
SKO_INTRA_CHOLQR2, SKO_INTRA_RANDCHOLQR, SKO_INTRA_CHOLQR2_RECURSIVE = 0, 1, 2
SKO_PREPROC_RANDBCGS2, SKO_PREPROC_PIP = 0, 1
SKO_BASIS_MONOMIAL, SKO_BASIS_NEWTON = 0, 1

EXPORTED = ["sko_create", "sko_destroy", "sko_set_stream", "sko_strerror", "sko_orth_block",
            "sko_orth_block_noalloc", "sko_orth_blocks", "sko_sketch_apply", "sko_gmres", "sko_gmres_batched", "sko_autotune_orth",
            "sko_profile_enable", "sko_profile_read"]


class sko_sketch(C.Structure):
    _fields_ = [("kind", C.c_int32), ("k", C.c_int32), ("zeta", C.c_int32), ("k_count", C.c_int32),
                ("seed", C.c_uint64), ("theta", C.c_void_p), ("ld_theta", C.c_int64)]


class sko_orth_opts(C.Structure):
    _fields_ = [("intra", C.c_int32), ("two_stage", C.c_int32), ("panels_per_big", C.c_int32),
                ("reorth", C.c_int32), ("precision", C.c_int32), ("preproc", C.c_int32),
                ("sketch", sko_sketch)]


class sko_csr(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("rowptr", C.c_void_p), ("colind", C.c_void_p),
                ("val", C.c_void_p)]


class sko_gmres_opts(C.Structure):
    _fields_ = [("s", C.c_int32), ("shat", C.c_int32), ("m", C.c_int32), ("two_stage", C.c_int32),
                ("precond", C.c_int32), ("intra", C.c_int32), ("precision", C.c_int32),
                ("phase_timing", C.c_int32), ("sketch", sko_sketch), ("tol", C.c_double),
                ("maxiter", C.c_int64), ("basis", C.c_int32), ("eager", C.c_int32)]


class sko_gmres_info(C.Structure):
    _fields_ = [("converged", C.c_int32), ("breakdown_col", C.c_int32), ("iters", C.c_int64),
                ("restarts", C.c_int64), ("relres", C.c_double), ("relres_implicit", C.c_double),
                ("t_total", C.c_double), ("t_spmv", C.c_double), ("t_orth", C.c_double), ("t_small", C.c_double)]


class sko_kernel_stat(C.Structure):
    _fields_ = [("name", C.c_char * 96), ("launches", C.c_int64), ("total_ms", C.c_double),
                ("bytes", C.c_double)]


def load_library(path: str = _LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise RuntimeError(f"libsko.so not built (expected at {path}); run paper_2503_16717_amd.build")
    lib = C.CDLL(path)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    lib.sko_create.argtypes = [C.c_int, vp, C.POINTER(vp)]
    lib.sko_destroy.argtypes = [vp]
    lib.sko_set_stream.argtypes = [vp, vp]
    lib.sko_strerror.argtypes = [C.c_int]
    lib.sko_strerror.restype = C.c_char_p
    lib.sko_orth_block.argtypes = [vp, i64, i32, i32, vp, i64, vp, i64, vp, i64, dp, dp,
                                   C.POINTER(sko_orth_opts), C.POINTER(i32)]
    lib.sko_orth_block_noalloc.argtypes = lib.sko_orth_block.argtypes
    lib.sko_orth_blocks.argtypes = [vp, i64, i32, i32, vp, i64, vp, i64, dp, i64,
                                    C.POINTER(sko_orth_opts), C.POINTER(i32)]
    lib.sko_sketch_apply.argtypes = [vp, i64, i32, vp, i64, i32, C.POINTER(sko_sketch), dp, i64]
    lib.sko_gmres.argtypes = [vp, C.POINTER(sko_csr), vp, vp, C.POINTER(sko_gmres_opts),
                              C.POINTER(sko_gmres_info)]
    lib.sko_gmres_batched.argtypes = [vp, i32, C.POINTER(sko_csr), C.POINTER(vp), C.POINTER(vp),
                                      C.POINTER(sko_gmres_opts), C.POINTER(sko_gmres_info)]
    lib.sko_autotune_orth.argtypes = [vp, i64, i32, i32, C.POINTER(sko_orth_opts)]
    lib.sko_profile_enable.argtypes = [vp, C.c_int]
    lib.sko_profile_read.argtypes = [vp, C.POINTER(sko_kernel_stat), i32]
    for name in EXPORTED:
        if name != "sko_strerror":
            getattr(lib, name).restype = C.c_int
    return lib


_lib = load_library()


class SkoError(RuntimeError):
    def __init__(self, status: int, where: str, col: int = 0):
        msg = _lib.sko_strerror(status).decode()
        super().__init__(f"{where}: {msg} (status {status}{', column %d' % col if col else ''})")
        self.status, self.col = status, col


def strerror(status: int) -> str:
    return _lib.sko_strerror(status).decode()


_PRECISIONS = {"f64": SKO_F64, "mixed": SKO_MIXED_F32}
_INTRAS = {"randcholqr": SKO_INTRA_RANDCHOLQR, "cholqr2": SKO_INTRA_CHOLQR2,
           "cholqr2_recursive": SKO_INTRA_CHOLQR2_RECURSIVE}


def _precision_code(precision: str) -> int:
    if precision not in _PRECISIONS:
        raise ValueError(f"precision must be one of {sorted(_PRECISIONS)}, not {precision!r}")
    return _PRECISIONS[precision]


def _intra_code(intra: str) -> int:
    if intra not in _INTRAS:
        raise ValueError(f"intra must be one of {sorted(_INTRAS)}, not {intra!r}")
    return _INTRAS[intra]


def _storage_dtype(precision: str):
    import torch
    return torch.float32 if _precision_code(precision) == SKO_MIXED_F32 else torch.float64


def _check_tensor(t, name, dtype, device_index=None):
    """The library reads element sizes from the precision option, not from the tensor: a
    tensor of another dtype, or on another device, would be read out of bounds."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, not {t.dtype}")
    if t.device.type != "cuda" or (device_index is not None and t.device.index != device_index):
        raise ValueError(f"{name} must be on cuda:{device_index}, not {t.device}")


def _colmajor(t, name, dtype=None, device_index=None):
    if dtype is not None:
        _check_tensor(t, name, dtype, device_index)
    if t.dim() != 2 or t.stride(0) != 1:
        raise ValueError(f"{name} must be a column-major 2-D tensor (stride(0) == 1)")
    return t.data_ptr(), max(t.stride(1), t.shape[0])


def make_sketch(kind: str = "sparse_sign", k: int = 64, zeta: int = 8, seed: int = 0, theta=None) -> sko_sketch:
    """theta: column-major float64 device tensor, (n x k) for the Gaussian sketch, (k_count x k)
    (the Gaussian factor) for the Count-Gauss composite, whose Count part has k_count =
    theta.shape[0] rows, zeta nonzeros per row and stream seed `seed` (k is then theta.shape[1]).
    The caller keeps theta alive while the sketch is in use."""
    sk = sko_sketch()
    if kind == "sparse_sign":
        sk.kind, sk.k, sk.zeta, sk.seed = SKO_SKETCH_SPARSE_SIGN, k, zeta, seed
    elif kind == "gaussian":
        import torch
        ptr, ld = _colmajor(theta, "theta", torch.float64)
        sk.kind, sk.k, sk.zeta, sk.seed, sk.theta, sk.ld_theta = SKO_SKETCH_GAUSSIAN, theta.shape[1], 0, 0, ptr, ld
    elif kind == "count_gauss":
        import torch
        ptr, ld = _colmajor(theta, "theta", torch.float64)
        sk.kind, sk.k, sk.k_count, sk.zeta, sk.seed = SKO_SKETCH_COUNT_GAUSS, theta.shape[1], theta.shape[0], zeta, seed
        sk.theta, sk.ld_theta = ptr, ld
    else:
        raise ValueError(kind)
    return sk


def orth_opts(intra="randcholqr", two_stage=False, panels_per_big=1, reorth=True, precision="f64",
              sketch: sko_sketch | None = None, preproc: str = "randbcgs2") -> sko_orth_opts:
    o = sko_orth_opts()
    o.intra = _intra_code(intra)
    o.two_stage = int(bool(two_stage))
    codes = {"randbcgs2": SKO_PREPROC_RANDBCGS2, "pip": SKO_PREPROC_PIP}
    if preproc not in codes:
        raise ValueError(f"unknown pre-processing {preproc!r}")
    o.preproc = codes[preproc]
    o.panels_per_big = int(panels_per_big)
    o.reorth = int(bool(reorth))
    o.precision = _precision_code(precision)
    o.sketch = sketch if sketch is not None else make_sketch()
    return o


def gmres_opts(s=5, m=30, shat=0, two_stage=False, precond=0, intra="randcholqr", precision="f64",
               sketch: sko_sketch | None = None, tol=1e-10, maxiter=0, phase_timing=False,
               basis: str = "monomial", eager: bool = False) -> sko_gmres_opts:
    o = sko_gmres_opts()
    o.phase_timing = int(bool(phase_timing))
    o.eager = int(bool(eager))
    bases = {"monomial": SKO_BASIS_MONOMIAL, "newton": SKO_BASIS_NEWTON}
    if basis not in bases:
        raise ValueError(f"unknown basis {basis!r}")
    o.basis = bases[basis]
    o.s, o.m, o.shat, o.two_stage = int(s), int(m), int(shat), int(bool(two_stage))
    o.precond = int(precond)
    o.intra = _intra_code(intra)
    o.precision = _precision_code(precision)
    o.sketch = sketch if sketch is not None else make_sketch()
    o.tol = float(tol)
    o.maxiter = int(maxiter)
    return o


def info_dict(inf: sko_gmres_info) -> dict:
    return {f: getattr(inf, f) for f, _ in sko_gmres_info._fields_}


class Context:
    """Owns an sko_ctx bound to a device and a HIP stream (default: torch's current stream)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = C.c_void_p()
        st = _lib.sko_create(device, C.c_void_p(stream.cuda_stream), C.byref(h))
        if st != SKO_OK:
            raise SkoError(st, "sko_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            _lib.sko_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- raw entry points with the C names --------------------------------------------------
    def sko_orth_blocks(self, n, nb, w, V_ptr, ldv, Q_ptr, ldq, R: np.ndarray | None, ldr, opts):
        col = C.c_int32(0)
        rp = R.ctypes.data_as(C.POINTER(C.c_double)) if R is not None else None
        st = _lib.sko_orth_blocks(self.h, n, nb, w, V_ptr, ldv, Q_ptr, ldq, rp, ldr, C.byref(opts), C.byref(col))
        return st, col.value

    def sko_orth_block(self, n, p, w, Q_ptr, ldq, V_ptr, ldv, Qo_ptr, ldqo, Rp, Rd, opts):
        col = C.c_int32(0)
        rpp = Rp.ctypes.data_as(C.POINTER(C.c_double)) if Rp is not None else None
        rdp = Rd.ctypes.data_as(C.POINTER(C.c_double)) if Rd is not None else None
        st = _lib.sko_orth_block(self.h, n, p, w, Q_ptr, ldq, V_ptr, ldv, Qo_ptr, ldqo, rpp, rdp,
                                 C.byref(opts), C.byref(col))
        return st, col.value

    def sko_orth_block_noalloc(self, n, p, w, Q_ptr, ldq, V_ptr, ldv, Qo_ptr, ldqo, Rp, Rd, opts):
        col = C.c_int32(0)
        rpp = Rp.ctypes.data_as(C.POINTER(C.c_double)) if Rp is not None else None
        rdp = Rd.ctypes.data_as(C.POINTER(C.c_double)) if Rd is not None else None
        st = _lib.sko_orth_block_noalloc(self.h, n, p, w, Q_ptr, ldq, V_ptr, ldv, Qo_ptr, ldqo, rpp, rdp,
                                         C.byref(opts), C.byref(col))
        return st, col.value

    def sko_gmres(self, A: sko_csr, b_ptr, x_ptr, opts: sko_gmres_opts):
        info = sko_gmres_info()
        st = _lib.sko_gmres(self.h, C.byref(A), b_ptr, x_ptr, C.byref(opts), C.byref(info))
        return st, info

    def sko_gmres_batched(self, As, b_ptrs, x_ptrs, opts: sko_gmres_opts):
        ns = len(As)
        Aarr = (sko_csr * ns)(*As)
        barr = (C.c_void_p * ns)(*b_ptrs)
        xarr = (C.c_void_p * ns)(*x_ptrs)
        infos = (sko_gmres_info * ns)()
        st = _lib.sko_gmres_batched(self.h, ns, Aarr, barr, xarr, C.byref(opts), infos)
        return st, list(infos)

    def sko_autotune_orth(self, n, nb, w, opts: sko_orth_opts):
        return _lib.sko_autotune_orth(self.h, n, nb, w, C.byref(opts))

    def autotune_orth(self, n: int, nb: int, w: int, **opt_kw):
        """Tune the launch shapes of sko_orth_blocks(n, nb, w, opts(**opt_kw)) on this context."""
        st = self.sko_autotune_orth(n, nb, w, orth_opts(**opt_kw))
        if st != SKO_OK:
            raise SkoError(st, "sko_autotune_orth")

    def sko_profile_enable(self, enable: bool):
        st = _lib.sko_profile_enable(self.h, int(bool(enable)))
        if st != SKO_OK:
            raise SkoError(st, "sko_profile_enable")

    def sko_profile_read(self):
        """List of dicts (name, launches, total_ms, bytes), largest total time first."""
        cnt = _lib.sko_profile_read(self.h, None, 0)
        if cnt < 0:
            raise SkoError(-cnt, "sko_profile_read")
        arr = (sko_kernel_stat * max(cnt, 1))()
        _lib.sko_profile_read(self.h, arr, cnt)
        return [dict(name=a.name.decode(), launches=a.launches, total_ms=a.total_ms, bytes=a.bytes)
                for a in arr[:cnt]]

    # -- tensor conveniences --------------------------------------------------------------
    def orth_blocks(self, V, w: int, Q=None, R: bool = True, raise_on_error: bool = True, **opt_kw):
        """Orthogonalise the column-major tensor V (n x nb*w).  Returns (Q, R, status, col)."""
        import torch
        dt = _storage_dtype(opt_kw.get("precision", "f64"))
        n, N = V.shape
        if N % w:
            raise ValueError("columns must be a multiple of w")
        if Q is None:
            Q = torch.empty((N, n), dtype=dt, device=V.device).t()
        vp, ldv = _colmajor(V, "V", dt, self.device)
        qp, ldq = _colmajor(Q, "Q", dt, self.device)
        Rh = np.zeros((N, N), order="F") if R else None
        opts = orth_opts(**opt_kw)
        st, col = self.sko_orth_blocks(n, N // w, w, vp, ldv, qp, ldq, Rh, N, opts)
        if raise_on_error and st not in (SKO_OK, SKO_EBREAKDOWN):
            raise SkoError(st, "sko_orth_blocks", col)
        return Q, Rh, st, col

    def orth_block(self, Qprev, V, Qout=None, raise_on_error: bool = True, noalloc: bool = False, **opt_kw):
        """One BCGS2 block step (noalloc: through sko_orth_block_noalloc; Qout must then be
        given, since the binding would otherwise allocate it).  Returns (Qout, R_proj, R_diag,
        status, col)."""
        import torch
        dt = _storage_dtype(opt_kw.get("precision", "f64"))
        n, w = V.shape
        p = 0 if Qprev is None else Qprev.shape[1]
        if Qout is None:
            if noalloc:
                raise ValueError("orth_block(noalloc=True) needs Qout")
            Qout = torch.empty((w, n), dtype=dt, device=V.device).t()
        vp, ldv = _colmajor(V, "V", dt, self.device)
        op, ldo = _colmajor(Qout, "Qout", dt, self.device)
        if p > 0:
            qp, ldq = _colmajor(Qprev, "Q", dt, self.device)
        else:
            qp, ldq = None, n
        Rp = np.zeros((p, w), order="F") if p > 0 else None
        Rd = np.zeros((w, w), order="F")
        opts = orth_opts(**opt_kw)
        call = self.sko_orth_block_noalloc if noalloc else self.sko_orth_block
        st, col = call(n, p, w, qp, ldq, vp, ldv, op, ldo, Rp, Rd, opts)
        if raise_on_error and st not in (SKO_OK, SKO_EBREAKDOWN):
            raise SkoError(st, "sko_orth_block_noalloc" if noalloc else "sko_orth_block", col)
        return Qout, Rp, Rd, st, col

    def sko_sketch_apply(self, n, w, X_ptr, ldx, precision: int, sketch: sko_sketch, Y: np.ndarray, ldy):
        yp = Y.ctypes.data_as(C.POINTER(C.c_double))
        return _lib.sko_sketch_apply(self.h, n, w, X_ptr, ldx, precision, C.byref(sketch), yp, ldy)

    def sketch_apply(self, X, sketch: sko_sketch, precision: str = "f64"):
        """Y = Theta^T X for the column-major device tensor X (n x w).  Returns Y (k x w)."""
        n, w = X.shape
        xp, ldx = _colmajor(X, "X", _storage_dtype(precision), self.device)
        Y = np.zeros((sketch.k, w), order="F")
        st = self.sko_sketch_apply(n, w, xp, ldx, _precision_code(precision), sketch, Y, sketch.k)
        if st != SKO_OK:
            raise SkoError(st, "sko_sketch_apply")
        return Y


def _gmres_method(self, A, b, x0=None, raise_on_error=False, **opt_kw):
    """Solve A x = b (A: workloads.CSR or (sko_csr, keep-alive) from csr_to_device; b: host
    array or device float64 tensor).  Returns (x device tensor, info dict, status)."""
    import torch
    if isinstance(A, tuple):
        Ad, keep = A
    else:
        Ad, keep = csr_to_device(A, "cuda:%d" % self.device)
    bt = b if isinstance(b, torch.Tensor) else torch.from_numpy(np.asarray(b, dtype=np.float64)).to(
        "cuda:%d" % self.device)
    if x0 is None:
        x = torch.zeros_like(bt)
    else:
        x = (x0 if isinstance(x0, torch.Tensor) else torch.from_numpy(np.asarray(x0, dtype=np.float64)).to(
            bt.device)).clone()
    _check_tensor(bt, "b", torch.float64, self.device)
    _check_tensor(x, "x", torch.float64, self.device)
    if bt.dim() != 1 or bt.shape[0] != Ad.n or not bt.is_contiguous() or x.shape != bt.shape or not x.is_contiguous():
        raise ValueError("b and x must be contiguous vectors of length A.n")
    opts = gmres_opts(**opt_kw)
    st, inf = self.sko_gmres(Ad, bt.data_ptr(), x.data_ptr(), opts)
    if raise_on_error and st not in (SKO_OK, SKO_ENOCONV):
        raise SkoError(st, "sko_gmres", inf.breakdown_col)
    del keep
    return x, info_dict(inf), st


Context.gmres = _gmres_method


def colmajor_from_numpy(a: np.ndarray, device="cuda", dtype=None):
    """Upload a host (n x m) array as a column-major device tensor."""
    import torch
    a = np.asarray(a)
    t = torch.from_numpy(np.ascontiguousarray(a.T)).to(device)
    if dtype is not None:
        t = t.to(dtype)
    return t.t()


def csr_to_device(A, device="cuda"):
    """Upload a workloads.CSR; returns (sko_csr struct, tensors kept alive)."""
    import torch
    if A.rowptr.dtype != np.int32 or A.colind.dtype != np.int32 or A.val.dtype != np.float64:
        raise TypeError("CSR indices must be int32 and values float64")
    if A.rowptr.shape != (A.n + 1,) or A.colind.shape != (A.nnz,) or A.val.shape != (A.nnz,):
        raise ValueError("CSR arrays have inconsistent lengths")
    rp = torch.from_numpy(A.rowptr).to(device)
    ci = torch.from_numpy(A.colind).to(device)
    va = torch.from_numpy(A.val).to(device)
    s = sko_csr()
    s.n, s.nnz, s.rowptr, s.colind, s.val = A.n, A.nnz, rp.data_ptr(), ci.data_ptr(), va.data_ptr()
    return s, (rp, ci, va)
