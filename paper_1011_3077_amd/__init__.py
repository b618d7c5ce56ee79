"""Python binding of libsdc (include/sdc.h): the inverse-free spectral split
step on MI355X (gfx950).

Argument marshalling only: every step of the computation runs in the HIP
library.  Matrices are torch float64 tensors on a HIP device; the library is
column-major, so a tensor is handed over as the memory of its transpose and
outputs are returned as transposed views of column-major buffers.

If the compiled library is missing this module raises ImportError; there is
no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsdc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} not built; run `python -m paper_1011_3077_amd.build`")
# torch first: torch carries its own HIP runtime under the same soname as the
# system's, and the first one loaded serves the whole process.  Loading
# torch's before the library keeps one runtime, the one torch was built for,
# whatever order the caller imports the two modules in (with the system's
# loaded first and torch initializing the device first, creating a handle
# failed with SDC_ERR_DEVICE).
import torch  # noqa: E402,F401

lib = C.CDLL(LIB_PATH)

SDC_OK, SDC_NOT_CONVERGED, SDC_NO_SPLIT, SDC_RANK_AMBIGUOUS = 0, 1, 2, 3
SDC_ERR_INVALID, SDC_ERR_NOMEM, SDC_ERR_DEVICE, SDC_ERR_NONFINITE = -1, -2, -3, -4
SDC_FP64, SDC_FP32_REFINE = 0, 1
SDC_UNIT_DISK, SDC_DISK, SDC_HALFPLANE = 0, 1, 2

EXPORTED = ["sdc_opts_default", "sdc_create", "sdc_destroy", "sdc_status_string", "sdc_irs",
            "sdc_split_sym", "sdc_split_sym_noalloc", "sdc_split_nonsym", "sdc_split_pencil", "sdc_split_sym_batched", "sdc_split_svd",
            "sdc_eig_dc",
            "sdc_block_eigvals", "sdc_trevc",
            "sdc_gaussian", "sdc_tune_set", "sdc_tune_get", "sdc_autotune", "sdc_tune_save", "sdc_tune_load",
            "sdc_graphs_enable",
            "sdc_tree_overlap_enable", "sdc_lookahead_set",
            "sdc_profile_enable", "sdc_profile_read", "sdc_server_create", "sdc_server_submit",
            "sdc_server_poll", "sdc_server_wait", "sdc_server_stats", "sdc_server_destroy"]
SDC_REQ_SYM, SDC_REQ_PENCIL = 0, 1


class Region(C.Structure):
    _fields_ = [("kind", C.c_int), ("center", C.c_double), ("radius", C.c_double),
                ("shift", C.c_double), ("scale", C.c_double)]


class Opts(C.Structure):
    _fields_ = [("prec", C.c_int), ("tau", C.c_double), ("maxit", C.c_int), ("seed", C.c_uint64),
                ("max_retries", C.c_int), ("split_tol", C.c_double), ("G", C.c_void_p),
                ("diagnostics", C.c_int), ("panel_width", C.c_int)]


class Info(C.Structure):
    _fields_ = [("n", C.c_int), ("k_lead", C.c_int), ("n_inside", C.c_int), ("iters_right", C.c_int),
                ("iters_left", C.c_int), ("attempts", C.c_int), ("refine_rounds", C.c_int),
                ("k_rho", C.c_int), ("rconv_last", C.c_double), ("e21_rel", C.c_double),
                ("orth_err", C.c_double), ("rank_gap", C.c_double), ("ms", C.c_double),
                ("fp64_fallback", C.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class DcInfo(C.Structure):
    _fields_ = [("n", C.c_int), ("nblocks", C.c_int), ("splits", C.c_int), ("accepted", C.c_int),
                ("extra_splits", C.c_int), ("levels", C.c_int), ("unsplit", C.c_int), ("near_singular", C.c_int),
                ("iters_total", C.c_int),
                ("nominal_flops", C.c_double), ("ms", C.c_double), ("e21_max", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class BlockBound(C.Structure):
    _fields_ = [("re_lo", C.c_double), ("re_hi", C.c_double), ("radius", C.c_double), ("inverted", C.c_int),
                ("unsplit", C.c_int)]


class KernelStats(C.Structure):
    _fields_ = [("launches", C.c_longlong), ("ms", C.c_double), ("flops", C.c_double), ("bytes", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


KERNEL_UPDATE, KERNEL_PANEL, KERNEL_GEMM, KERNEL_LA = 0, 1, 2, 3
SDC_PANEL64_NEVER = -1


class TuneResult(C.Structure):
    _fields_ = [("n", C.c_int), ("prec", C.c_int), ("ms_nb32", C.c_double), ("ms_nb64", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Request(C.Structure):
    _fields_ = [("kind", C.c_int), ("n", C.c_int), ("A", C.c_void_p), ("lda", C.c_int), ("B", C.c_void_p),
                ("ldb", C.c_int), ("region", Region), ("opts", Opts), ("Q", C.c_void_p), ("ldq", C.c_int),
                ("QL", C.c_void_p), ("ldql", C.c_int), ("Ahat", C.c_void_p), ("ldah", C.c_int),
                ("Bhat", C.c_void_p), ("ldbh", C.c_int)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_longlong), ("completed", C.c_longlong), ("failed", C.c_longlong),
                ("active", C.c_int), ("pending", C.c_int), ("peak_active", C.c_int), ("ticks", C.c_longlong),
                ("p50_ms", C.c_double), ("p99_ms", C.c_double), ("mean_ms", C.c_double), ("max_ms", C.c_double),
                ("wall_ms", C.c_double), ("nominal_flops", C.c_double), ("peak_bytes", C.c_size_t),
                ("budget_bytes", C.c_size_t)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}

_P = C.c_void_p
_I = C.c_int
lib.sdc_opts_default.argtypes = [C.POINTER(Opts)]
lib.sdc_opts_default.restype = None
lib.sdc_create.argtypes = [C.POINTER(_P), _I, C.c_size_t, _P]
lib.sdc_create.restype = _I
lib.sdc_destroy.argtypes = [_P]
lib.sdc_destroy.restype = _I
lib.sdc_status_string.argtypes = [_I]
lib.sdc_status_string.restype = C.c_char_p
lib.sdc_irs.argtypes = [_P, _I, _P, _I, _P, _I, _I, Region, C.POINTER(Opts), _P, _P, _P, _I,
                        C.POINTER(_I), C.POINTER(C.c_double)]
lib.sdc_irs.restype = _I
lib.sdc_split_sym.argtypes = [_P, _I, _P, _I, Region, C.POINTER(Opts), _P, _I, _P, _I, C.POINTER(Info)]
lib.sdc_split_sym.restype = _I
lib.sdc_split_pencil.argtypes = [_P, _I, _P, _I, _P, _I, Region, C.POINTER(Opts), _P, _I, _P, _I,
                                 _P, _I, _P, _I, C.POINTER(Info)]
lib.sdc_split_pencil.restype = _I
lib.sdc_split_sym_batched.argtypes = [_P, _I, C.POINTER(_I), C.POINTER(_P), C.POINTER(_I),
                                      C.POINTER(Region), C.POINTER(Opts), C.POINTER(_P), C.POINTER(_I),
                                      C.POINTER(_P), C.POINTER(_I), C.POINTER(Info), C.POINTER(_I)]
lib.sdc_split_sym_batched.restype = _I
lib.sdc_eig_dc.argtypes = [_P, _I, _P, _I, _P, _I, _I, _I, C.POINTER(Opts), _P, _I, _P, _I, _P, _I, _P, _I,
                           C.POINTER(_I), C.POINTER(_I), C.POINTER(BlockBound), C.POINTER(DcInfo)]
lib.sdc_eig_dc.restype = _I
lib.sdc_split_sym_noalloc.argtypes = [_P, _I, _P, _I, Region, C.POINTER(Opts), _P, _I, _P, _I, C.POINTER(Info)]
lib.sdc_split_sym_noalloc.restype = _I
NOALLOC_MAX_N = 1024
lib.sdc_split_nonsym.argtypes = [_P, _I, _P, _I, Region, C.POINTER(Opts), _P, _I, _P, _I, C.POINTER(Info)]
lib.sdc_split_nonsym.restype = _I
lib.sdc_split_svd.argtypes = [_P, _I, _I, _P, _I, Region, C.POINTER(Opts), _P, _I, _P, _I, _P, _I, C.POINTER(Info)]
lib.sdc_split_svd.restype = _I
lib.sdc_block_eigvals.argtypes = [_P, _I, _P, _I, _P, _I, _I, C.POINTER(_I), _I, _P, _P, _P, _I]
lib.sdc_block_eigvals.restype = _I
lib.sdc_trevc.argtypes = [_P, _I, _P, _I, _P, _I, _P, _I]
lib.sdc_trevc.restype = _I
lib.sdc_profile_enable.argtypes = [_P, _I]
lib.sdc_profile_enable.restype = _I
lib.sdc_profile_read.argtypes = [_P, _I, C.POINTER(KernelStats)]
lib.sdc_profile_read.restype = _I
lib.sdc_gaussian.argtypes = [_P, _I, C.c_uint64, _I, _P, _I]
lib.sdc_gaussian.restype = _I
lib.sdc_graphs_enable.argtypes = [_P, _I]
lib.sdc_graphs_enable.restype = _I
lib.sdc_tree_overlap_enable.argtypes = [_P, _I]
lib.sdc_tree_overlap_enable.restype = _I
lib.sdc_lookahead_set.argtypes = [_P, _I]
lib.sdc_lookahead_set.restype = _I
lib.sdc_tune_set.argtypes = [_P, _I, _I]
lib.sdc_tune_set.restype = _I
lib.sdc_tune_get.argtypes = [_P, C.POINTER(_I), C.POINTER(_I)]
lib.sdc_tune_get.restype = _I
lib.sdc_autotune.argtypes = [_P, C.POINTER(_I), _I, _I, C.POINTER(TuneResult)]
lib.sdc_autotune.restype = _I
lib.sdc_tune_save.argtypes = [_P, C.c_char_p]
lib.sdc_tune_save.restype = _I
lib.sdc_tune_load.argtypes = [_P, C.c_char_p]
lib.sdc_tune_load.restype = _I
lib.sdc_server_create.argtypes = [C.POINTER(_P), _I, C.c_size_t, _I]
lib.sdc_server_create.restype = _I
lib.sdc_server_submit.argtypes = [_P, C.POINTER(Request), C.POINTER(C.c_longlong)]
lib.sdc_server_submit.restype = _I
lib.sdc_server_poll.argtypes = [_P, C.c_longlong, C.POINTER(_I), C.POINTER(_I), C.POINTER(Info)]
lib.sdc_server_poll.restype = _I
lib.sdc_server_wait.argtypes = [_P, C.c_longlong, C.POINTER(_I), C.POINTER(Info)]
lib.sdc_server_wait.restype = _I
lib.sdc_server_stats.argtypes = [_P, C.POINTER(ServerStats)]
lib.sdc_server_stats.restype = _I
lib.sdc_server_destroy.argtypes = [_P]
lib.sdc_server_destroy.restype = _I


def status_string(s: int) -> str:
    return lib.sdc_status_string(int(s)).decode()


class SdcError(RuntimeError):
    pass


def _check(st: int) -> int:
    if st < 0:
        raise SdcError(status_string(st))
    return st


def region(kind: str = "unit_disk", center: float = 0.0, radius: float = 1.0, shift: float = 0.0,
           scale: float = 1.0) -> Region:
    k = {"unit_disk": SDC_UNIT_DISK, "disk": SDC_DISK, "halfplane": SDC_HALFPLANE}[kind]
    return Region(k, center, radius, shift, scale)


def opts(prec: int = SDC_FP64, tau: float = 0.0, maxit: int = 60, seed: int = 0, max_retries: int = 2,
         split_tol: float = 1e-10, G=None, diagnostics: int = 0, panel_width: int = 0) -> Opts:
    o = Opts()
    lib.sdc_opts_default(C.byref(o))
    o.prec, o.tau, o.maxit, o.seed = prec, tau, maxit, seed
    o.max_retries, o.split_tol, o.diagnostics = max_retries, split_tol, diagnostics
    o.panel_width = panel_width
    o.G = None if G is None else G.data_ptr()
    return o


def _cm(t):
    """Column-major device buffer of matrix t (n x n float64 torch tensor)."""
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.dim() == 2):
        raise TypeError("expected a 2-D float64 tensor on a HIP device")
    return t.t().contiguous()


def _cm_sym(t):
    """Column-major buffer of a symmetric matrix: its own memory when it is
    contiguous (a symmetric matrix equals its transpose), else a copy."""
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.dim() == 2):
        raise TypeError("expected a 2-D float64 tensor on a HIP device")
    return t if t.is_contiguous() else t.t().contiguous()


def _out(n, like):
    import torch
    return torch.empty((n, n), dtype=torch.float64, device=like.device)


@dataclass
class SplitResult:
    status: int
    info: dict
    Q: object          # Q (symmetric) / Q_R (pencil), n x n torch tensor
    QL: object
    Ahat: object
    Bhat: object


class Handle:
    """Owns an sdc handle bound to a device and (optionally) a torch stream."""

    def __init__(self, device: int = 0, budget_bytes: int = 0, stream=None):
        import torch
        self.device = device
        s = stream.cuda_stream if stream is not None else torch.cuda.current_stream(device).cuda_stream
        h = C.c_void_p()
        _check(lib.sdc_create(C.byref(h), device, budget_bytes, C.c_void_p(s)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib.sdc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- entry points (same names as the C ABI without the prefix) ---------
    def irs(self, A, B=None, reg: Region | None = None, o: Opts | None = None, transpose: bool = False):
        n = A.shape[0]
        a = _cm(A)
        b = _cm(B) if B is not None else None
        ap, bp, r = _out(n, A), _out(n, A), _out(n, A)
        p = C.c_int()
        rc = C.c_double()
        st = _check(lib.sdc_irs(self._h, n, a.data_ptr(), n, None if b is None else b.data_ptr(), n,
                                int(transpose), reg or region(), C.byref(o or opts()), ap.data_ptr(),
                                bp.data_ptr(), r.data_ptr(), n, C.byref(p), C.byref(rc)))
        return st, ap.t(), bp.t(), r.t(), p.value, rc.value

    def split_sym(self, A, reg: Region | None = None, o: Opts | None = None) -> SplitResult:
        n = A.shape[0]
        a = _cm_sym(A)
        q, ah = _out(n, A), _out(n, A)
        info = Info()
        st = _check(lib.sdc_split_sym(self._h, n, a.data_ptr(), n, reg or region(), C.byref(o or opts()),
                                      q.data_ptr(), n, ah.data_ptr(), n, C.byref(info)))
        return SplitResult(st, info.as_dict(), q.t(), None, ah.t(), None)

    def split_sym_noalloc(self, A_cm, Q_cm, Ahat_cm, reg: Region | None = None, o: Opts | None = None):
        """sdc_split_sym_noalloc on caller-owned column-major buffers (float64
        device tensors of shape (n, n) holding the transposes, e.g. made once
        with torch.empty and reused): nothing is allocated here or in the
        library.  Returns (status, info)."""
        n = A_cm.shape[0]
        for t in (A_cm, Q_cm, Ahat_cm):
            if not (t.is_cuda and t.is_contiguous() and tuple(t.shape) == (n, n)):
                raise TypeError("expected contiguous (n, n) device tensors")
        info = Info()
        st = _check(lib.sdc_split_sym_noalloc(self._h, n, A_cm.data_ptr(), n, reg or region(), C.byref(o or opts()),
                                              Q_cm.data_ptr(), n, Ahat_cm.data_ptr(), n, C.byref(info)))
        return st, info.as_dict()

    def split_nonsym(self, A, reg: Region | None = None, o: Opts | None = None) -> SplitResult:
        n = A.shape[0]
        a = _cm(A)
        q, ah = _out(n, A), _out(n, A)
        info = Info()
        st = _check(lib.sdc_split_nonsym(self._h, n, a.data_ptr(), n, reg or region(), C.byref(o or opts()),
                                         q.data_ptr(), n, ah.data_ptr(), n, C.byref(info)))
        return SplitResult(st, info.as_dict(), q.t(), None, ah.t(), None)

    def split_pencil(self, A, B, reg: Region | None = None, o: Opts | None = None) -> SplitResult:
        n = A.shape[0]
        a, b = _cm(A), _cm(B)
        ql, qr, ah, bh = _out(n, A), _out(n, A), _out(n, A), _out(n, A)
        info = Info()
        st = _check(lib.sdc_split_pencil(self._h, n, a.data_ptr(), n, b.data_ptr(), n, reg or region(),
                                         C.byref(o or opts()), ql.data_ptr(), n, qr.data_ptr(), n,
                                         ah.data_ptr(), n, bh.data_ptr(), n, C.byref(info)))
        return SplitResult(st, info.as_dict(), qr.t(), ql.t(), ah.t(), bh.t())

    def split_sym_batched(self, As, regs, o: Opts | None = None):
        cnt = len(As)
        cms = [_cm_sym(a) for a in As]
        outs_q = [_out(a.shape[0], a) for a in As]
        outs_a = [_out(a.shape[0], a) for a in As]
        ns = (_I * cnt)(*[a.shape[0] for a in As])
        ptr_a = (_P * cnt)(*[c.data_ptr() for c in cms])
        ptr_q = (_P * cnt)(*[q.data_ptr() for q in outs_q])
        ptr_h = (_P * cnt)(*[q.data_ptr() for q in outs_a])
        rg = (Region * cnt)(*regs)
        infos = (Info * cnt)()
        sts = (_I * cnt)()
        _check(lib.sdc_split_sym_batched(self._h, cnt, ns, ptr_a, ns, rg, C.byref(o or opts()), ptr_q, ns,
                                         ptr_h, ns, infos, sts))
        return [SplitResult(sts[i], infos[i].as_dict(), outs_q[i].t(), None, outs_a[i].t(), None)
                for i in range(cnt)]

    def eig_dc(self, A, B=None, leaf_max: int = 64, o: Opts | None = None, symmetric: bool = False,
               factors: bool = True):
        """Divide and conquer to blocks <= leaf_max.  Returns
        (status, T, S, QL, QR, block_starts, info); S/QL are None for symmetric.
        info["bounds"] holds one (re_lo, re_hi, radius, inverted, unsplit)
        tuple per block (sdc_block_bound_t)."""
        n = A.shape[0]
        a = _cm(A)
        b = _cm(B) if (B is not None and not symmetric) else None
        t = _out(n, A)
        s = _out(n, A) if b is not None else None
        ql = _out(n, A) if (factors and b is not None) else None
        qr = _out(n, A) if factors else None
        nb = C.c_int()
        starts = (_I * (n + 1))()
        info = DcInfo()
        bounds = (BlockBound * max(n, 1))()
        ptr = lambda x: None if x is None else x.data_ptr()
        st = _check(lib.sdc_eig_dc(self._h, n, a.data_ptr(), n, ptr(b), n, int(symmetric), leaf_max,
                                   C.byref(o or opts()), t.data_ptr(), n, ptr(s), n, ptr(ql), n, ptr(qr), n,
                                   C.byref(nb), starts, bounds, C.byref(info)))
        tr = lambda x: None if x is None else x.t()
        d = info.as_dict()
        d["bounds"] = [(x.re_lo, x.re_hi, x.radius, x.inverted, x.unsplit) for x in bounds[:nb.value]]
        return st, tr(t), tr(s), tr(ql), tr(qr), [starts[i] for i in range(nb.value + 1)], d

    def split_svd(self, A, reg: Region | None = None, o: Opts | None = None):
        """RSVD split of the m x n A at the half plane reg (see sdc_split_svd):
        returns (status, info, U, V, S11) with U m x r, V n x r, S11 r x r
        (r = min(m, n)), of which the first info["k_lead"] columns are valid."""
        import torch
        if not (A.is_cuda and A.dtype == torch.float64 and A.dim() == 2):
            raise TypeError("expected a 2-D float64 tensor on a HIP device")
        m, n = A.shape
        r = min(m, n)
        a = A.t().contiguous()
        u = torch.empty((r, m), dtype=torch.float64, device=A.device)
        v = torch.empty((r, n), dtype=torch.float64, device=A.device)
        s11 = torch.empty((r, r), dtype=torch.float64, device=A.device)
        info = Info()
        st = _check(lib.sdc_split_svd(self._h, m, n, a.data_ptr(), m, reg or region("halfplane"), C.byref(o or opts()),
                                      u.data_ptr(), m, v.data_ptr(), n, s11.data_ptr(), r, C.byref(info)))
        return st, info.as_dict(), u.t(), v.t(), s11.t()

    def block_eigvals(self, T, S, starts, symmetric: bool = False, vectors: bool = False):
        """Eigenvalues of the diagonal blocks of eig_dc's T (and S): returns
        (wr, wi), two length-n float64 device tensors, and with vectors=True
        (symmetric only) also V, n x n block diagonal, the blocks'
        eigenvectors (see sdc_block_eigvals)."""
        import torch
        n = T.shape[0]
        t = _cm(T)
        s = _cm(S) if (S is not None and not symmetric) else None
        nb = len(starts) - 1
        st = (_I * (nb + 1))(*starts)
        wr = torch.empty(n, dtype=torch.float64, device=T.device)
        wi = torch.empty(n, dtype=torch.float64, device=T.device)
        v = torch.zeros((n, n), dtype=torch.float64, device=T.device) if vectors else None
        _check(lib.sdc_block_eigvals(self._h, n, t.data_ptr(), n, None if s is None else s.data_ptr(), n, nb, st,
                                     int(symmetric), wr.data_ptr(), wi.data_ptr(),
                                     None if v is None else v.data_ptr(), n))
        return (wr, wi) if v is None else (wr, wi, v.t())

    def trevc(self, T, S=None):
        """Eigenvectors of the upper-triangular T (pencil (T, S)): X upper
        triangular with unit diagonal, T X = S X diag(T_jj / S_jj)."""
        n = T.shape[0]
        t = _cm(T)
        s = _cm(S) if S is not None else None
        x = _out(n, T)
        _check(lib.sdc_trevc(self._h, n, t.data_ptr(), n, None if s is None else s.data_ptr(), n, x.data_ptr(), n))
        return x.t()

    def profile_enable(self, on: bool = True):
        _check(lib.sdc_profile_enable(self._h, int(on)))

    def profile_read(self, kernel: int) -> dict:
        ks = KernelStats()
        _check(lib.sdc_profile_read(self._h, kernel, C.byref(ks)))
        return ks.as_dict()

    def gaussian(self, n: int, seed: int, tag: int):
        import torch
        g = torch.empty((n, n), dtype=torch.float64, device=f"cuda:{self.device}")
        _check(lib.sdc_gaussian(self._h, n, seed, tag, g.data_ptr(), n))
        return g.t()

    def graphs_enable(self, on: bool = True):
        _check(lib.sdc_graphs_enable(self._h, 1 if on else 0))

    def tree_overlap_enable(self, on: bool = True):
        """Factor a QR panel's tree above its leaves beside the leaves'
        trailing update (on, the default) or before it; bitwise the same."""
        _check(lib.sdc_tree_overlap_enable(self._h, 1 if on else 0))

    def lookahead_set(self, min_cols: int):
        """Problems of at least min_cols factored columns take the two-stream
        look-ahead QR schedule; min_cols <= 0 (the default): none."""
        _check(lib.sdc_lookahead_set(self._h, int(min_cols)))

    def tune_set(self, nb64_min_fp64: int, nb64_min_fp32: int):
        _check(lib.sdc_tune_set(self._h, nb64_min_fp64, nb64_min_fp32))

    def tune_get(self):
        a, b = _I(), _I()
        _check(lib.sdc_tune_get(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def autotune(self, orders, reps: int = 2, cache: str | None = None):
        """sdc_autotune over `orders`; returns the timings (FP64 rows first)
        and, with `cache`, writes the resulting table there as JSON."""
        arr = (_I * len(orders))(*orders)
        res = (TuneResult * (2 * len(orders)))()
        _check(lib.sdc_autotune(self._h, arr, len(orders), reps, res))
        if cache is not None:
            _check(lib.sdc_tune_save(self._h, cache.encode()))
        return [r.as_dict() for r in res]

    def tune_save(self, path: str):
        _check(lib.sdc_tune_save(self._h, path.encode()))

    def tune_load(self, path: str):
        _check(lib.sdc_tune_load(self._h, path.encode()))


class Server:
    """Served form (sdc_server_*): requests are queued and run with continuous
    batching on the library's own worker thread and stream.  submit() keeps
    the column-major inputs and the outputs alive until the request is done."""

    def __init__(self, device: int = 0, budget_bytes: int = 0, max_active: int = 0):
        self.device = device
        s = C.c_void_p()
        _check(lib.sdc_server_create(C.byref(s), device, budget_bytes, max_active))
        self._s = s
        self._live = {}

    def close(self):
        if getattr(self, "_s", None):
            lib.sdc_server_destroy(self._s)
            self._s = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, A, B=None, reg: Region | None = None, o: Opts | None = None) -> int:
        """Queue a split of symmetric A (B is None) or of the pencil (A, B)."""
        import torch
        n = A.shape[0]
        a = _cm(A)
        b = _cm(B) if B is not None else None
        q, ah = _out(n, A), _out(n, A)
        ql = _out(n, A) if b is not None else None
        bh = _out(n, A) if b is not None else None
        torch.cuda.current_stream(A.device).synchronize()  # the input copies complete before the worker reads them
        r = Request()
        r.kind = SDC_REQ_PENCIL if b is not None else SDC_REQ_SYM
        r.n = n
        r.A, r.lda = a.data_ptr(), n
        r.B, r.ldb = (b.data_ptr() if b is not None else None), n
        r.region = reg or region()
        r.opts = o or opts()
        r.Q, r.ldq = q.data_ptr(), n
        r.QL, r.ldql = (ql.data_ptr() if ql is not None else None), n
        r.Ahat, r.ldah = ah.data_ptr(), n
        r.Bhat, r.ldbh = (bh.data_ptr() if bh is not None else None), n
        t = C.c_longlong()
        _check(lib.sdc_server_submit(self._s, C.byref(r), C.byref(t)))
        self._live[t.value] = (a, b, q, ql, ah, bh)
        return t.value

    def _result(self, ticket, st, info) -> SplitResult:
        a, b, q, ql, ah, bh = self._live.pop(ticket)
        tr = lambda x: None if x is None else x.t()
        return SplitResult(st, info.as_dict(), tr(q), tr(ql), tr(ah), tr(bh))

    def poll(self, ticket: int):
        """None while running, else the SplitResult."""
        done, st, info = C.c_int(), C.c_int(), Info()
        _check(lib.sdc_server_poll(self._s, ticket, C.byref(done), C.byref(st), C.byref(info)))
        return self._result(ticket, st.value, info) if done.value else None

    def wait(self, ticket: int) -> SplitResult:
        st, info = C.c_int(), Info()
        _check(lib.sdc_server_wait(self._s, ticket, C.byref(st), C.byref(info)))
        return self._result(ticket, st.value, info)

    def stats(self) -> dict:
        s = ServerStats()
        _check(lib.sdc_server_stats(self._s, C.byref(s)))
        return s.as_dict()
