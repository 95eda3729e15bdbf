"""ctypes binding of libgwas (include/gwas.h): argument marshalling only.

Every step of the computation runs in the library's HIP kernels. PyTorch is
used for device memory (tensors) and streams. Loading fails loudly when the
library has not been built; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgwas.so")

OK, EINVAL, ENOMEM, EHIP, EBUSY, ESTATE = 0, 1, 2, 3, 4, 5
DT_F64, DT_F32, DT_U8 = 0, 1, 2
FORM_F64, FORM_F32, FORM_BF16X3, FORM_BF16X6 = 0, 1, 2, 3
FORMS = {"f64": FORM_F64, "f32": FORM_F32, "bf16x3": FORM_BF16X3, "bf16x6": FORM_BF16X6}

_lib = None


class GwasError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("libgwas status %d: %s" % (status, msg))
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("m_capacity", ctypes.c_int64), ("forms", ctypes.c_uint32),
                ("device", ctypes.c_int32), ("max_traits", ctypes.c_int32),
                ("slab_snps", ctypes.c_int32), ("f32_flush", ctypes.c_int32),
                ("timing", ctypes.c_int32), ("ring_slots", ctypes.c_int32),
                ("host_threads", ctypes.c_int32), ("geno_chunk_snps", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 5)]


class Slab(ctypes.Structure):
    _fields_ = [("index", ctypes.c_int64), ("i0", ctypes.c_int64), ("count", ctypes.c_int64),
                ("j0", ctypes.c_int32), ("tb", ctypes.c_int32), ("p", ctypes.c_int32),
                ("form", ctypes.c_int32), ("b", ctypes.c_void_p), ("bytes", ctypes.c_int64),
                ("checksum", ctypes.c_uint64)]


SLAB_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.POINTER(Slab))


class ServerOptions(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_int64), ("max_slots", ctypes.c_int32), ("form", ctypes.c_int32),
                ("item_problems", ctypes.c_int32), ("max_traits", ctypes.c_int32),
                ("ring_slots", ctypes.c_int32), ("host_threads", ctypes.c_int32),
                ("skip_checksum", ctypes.c_int32), ("grid_wgs", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 4)]


class ServerStats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int64), ("items", ctypes.c_int64), ("ring_stalls", ctypes.c_int64),
                ("stage_stalls", ctypes.c_int64), ("bytes_d2h", ctypes.c_int64),
                ("checksum_s", ctypes.c_double), ("busy_s", ctypes.c_double),
                ("issue_s", ctypes.c_double), ("kernel_s", ctypes.c_double),
                ("reserved", ctypes.c_int64 * 6)]


class Request(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int32), ("p", ctypes.c_int32), ("Y", ctypes.c_void_p),
                ("h2", ctypes.c_void_p), ("i0", ctypes.c_int64), ("m", ctypes.c_int64),
                ("b", ctypes.c_void_p), ("fn", ctypes.c_void_p), ("user", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("error", ctypes.c_int32), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double), ("problems", ctypes.c_int64),
                ("slabs", ctypes.c_int64), ("checksum", ctypes.c_uint64), ("reserved", ctypes.c_int64 * 4)]


REQ_STATES = {0: "queued", 1: "running", 2: "done", 3: "cancelled", 4: "failed"}


class Stats(ctypes.Structure):
    _fields_ = [("non_spd", ctypes.c_int64), ("snps_rotated", ctypes.c_int64),
                ("problems", ctypes.c_int64), ("bytes_h2d", ctypes.c_int64),
                ("bytes_d2h", ctypes.c_int64), ("resident_bytes", ctypes.c_int64),
                ("fused_launches", ctypes.c_int64), ("fused_ms", ctypes.c_double),
                ("rotate_launches", ctypes.c_int64), ("rotate_ms", ctypes.c_double),
                ("dot_launches", ctypes.c_int64), ("reserved", ctypes.c_int64 * 5)]


def load():
    """Load libgwas.so (raises if it is missing: build it with paper_1210_7683_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libgwas.so is not built (%s); run python -m paper_1210_7683_amd.build"
                          % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.gwas_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.gwas_default_options.restype = None
    lib.gwas_eigh.argtypes = [i32, vp, vp, vp, i32, vp]
    lib.gwas_eigh.restype = i32
    lib.gwas_setup.argtypes = [ctypes.POINTER(vp), i32, i32, vp, vp, vp, ctypes.POINTER(Options)]
    lib.gwas_setup.restype = i32
    lib.gwas_rotate.argtypes = [vp, i64, i64, vp, i32, i32, vp]
    lib.gwas_rotate.restype = i32
    lib.gwas_solve.argtypes = [vp, i64, i64, i32, vp, i32, vp, i32, vp, i32, vp]
    lib.gwas_solve.restype = i32
    lib.gwas_solve_noalloc.argtypes = [vp, i64, i64, i32, vp, i32, vp, i32, vp, vp]
    lib.gwas_solve_noalloc.restype = i32
    lib.gwas_solve_stream.argtypes = [vp, i64, i64, i32, vp, i32, vp, i32, SLAB_FN, vp,
                                      ctypes.POINTER(ctypes.c_uint64), i64, ctypes.POINTER(i64), vp]
    lib.gwas_solve_stream.restype = i32
    lib.gwas_solve_snp_stream.argtypes = [vp, vp, i32, i64, i32, vp, i32, vp, i32, SLAB_FN, vp,
                                          ctypes.POINTER(ctypes.c_uint64), i64, ctypes.POINTER(i64), vp]
    lib.gwas_solve_snp_stream.restype = i32
    lib.gwas_checksum.argtypes = [vp, i64]
    lib.gwas_checksum.restype = ctypes.c_uint64
    lib.gwas_clock.argtypes = []
    lib.gwas_clock.restype = ctypes.c_double
    lib.gwas_server_create.argtypes = [vp, ctypes.POINTER(ServerOptions), ctypes.POINTER(vp)]
    lib.gwas_server_create.restype = i32
    lib.gwas_server_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    lib.gwas_server_submit.restype = i32
    lib.gwas_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(Result)]
    lib.gwas_server_poll.restype = i32
    lib.gwas_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(Result)]
    lib.gwas_server_wait.restype = i32
    lib.gwas_server_cancel.argtypes = [vp, ctypes.c_uint64]
    lib.gwas_server_cancel.restype = i32
    lib.gwas_server_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    lib.gwas_server_stats.restype = i32
    lib.gwas_server_destroy.argtypes = [vp]
    lib.gwas_server_destroy.restype = i32
    lib.gwas_copy_rotated.argtypes = [vp, i64, i64, i32, vp, i32, vp]
    lib.gwas_copy_rotated.restype = i32
    lib.gwas_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    lib.gwas_stats.restype = i32
    lib.gwas_reset_stats.argtypes = [vp]
    lib.gwas_reset_stats.restype = i32
    lib.gwas_debug_size.argtypes = [vp, i32, i32]
    lib.gwas_debug_size.restype = i64
    lib.gwas_debug_copy.argtypes = [vp, i32, i32, vp, i64]
    lib.gwas_debug_copy.restype = i32
    lib.gwas_destroy.argtypes = [vp]
    lib.gwas_destroy.restype = None
    lib.gwas_last_error.argtypes = []
    lib.gwas_last_error.restype = ctypes.c_char_p
    lib.gwas_version.argtypes = []
    lib.gwas_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(st: int):
    if st != OK:
        raise GwasError(st, load().gwas_last_error().decode())


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _is_device(x) -> bool:
    try:
        import torch
        return isinstance(x, torch.Tensor) and x.is_cuda
    except ImportError:
        return False


def _ptr(x):
    """(pointer, on_device, keepalive) of a numpy array or torch tensor."""
    import torch
    if isinstance(x, torch.Tensor):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return ctypes.c_void_p(x.data_ptr()), int(x.is_cuda), x
    a = np.ascontiguousarray(x)
    return ctypes.c_void_p(a.ctypes.data), 0, a


_DT = {np.dtype(np.float64): DT_F64, np.dtype(np.float32): DT_F32, np.dtype(np.uint8): DT_U8}


def _dtype_code(x) -> int:
    import torch
    if isinstance(x, torch.Tensor):
        m = {torch.float64: DT_F64, torch.float32: DT_F32, torch.uint8: DT_U8}
        if x.dtype not in m:
            raise ValueError("unsupported dtype %s" % x.dtype)
        return m[x.dtype]
    d = np.asarray(x).dtype
    if d not in _DT:
        raise ValueError("unsupported dtype %s" % d)
    return _DT[d]


class Cohort:
    """A resident cohort on one GPU: Z, w, rotated X_L and rotated SNPs.

    Z [n][n] array whose column k is eigenvector k of Phi (numpy.linalg.eigh
    output), w [n] eigenvalues, xl [(p-1)][n] covariate columns.
    """

    def __init__(self, Z, w, xl, m_capacity: int, forms=("f64", "f32", "bf16x3"),
                 max_traits: int = 1024, device: int = 0, slab_snps: int = 0,
                 f32_flush: int | None = None, timing: bool = False, ring_slots: int = 0,
                 host_threads: int = 0, geno_chunk_snps: int = 0):
        lib = load()
        Z = np.asarray(Z, dtype=np.float64)
        n = Z.shape[0]
        # column-major n x n: column k contiguous
        zc = np.ascontiguousarray(Z.T)
        w = np.ascontiguousarray(w, dtype=np.float64)
        xl = np.ascontiguousarray(np.atleast_2d(xl), dtype=np.float64)
        if Z.shape != (n, n) or w.shape != (n,) or xl.shape[1] != n:
            raise ValueError("inconsistent shapes")
        opt = Options()
        lib.gwas_default_options(ctypes.byref(opt))
        opt.m_capacity = int(m_capacity)
        opt.forms = sum(1 << FORMS[f] for f in forms)
        opt.device = int(device)
        opt.max_traits = int(max_traits)
        opt.slab_snps = int(slab_snps)
        if f32_flush is not None:
            opt.f32_flush = int(f32_flush)
        opt.timing = int(bool(timing))
        opt.ring_slots = int(ring_slots)
        opt.host_threads = int(host_threads)
        opt.geno_chunk_snps = int(geno_chunk_snps)
        h = ctypes.c_void_p()
        _check(lib.gwas_setup(ctypes.byref(h), n, xl.shape[0] + 1, zc.ctypes.data, w.ctypes.data,
                              xl.ctypes.data, ctypes.byref(opt)))
        self._h = h
        self.n, self.p, self.m_capacity = n, xl.shape[0] + 1, int(m_capacity)
        self.forms = tuple(forms)
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            load().gwas_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def rotate(self, m0: int, xr, stream=None):
        """Rotate SNP columns xr [mb][n] (uint8, float32 or float64; numpy or torch) into [m0, m0+mb)."""
        ptr, dev, keep = _ptr(xr)
        mb = int(xr.shape[0]) if len(xr.shape) == 2 else 0
        if mb and int(xr.shape[1]) != self.n:
            raise ValueError("SNP block must be [mb][n]")
        _check(load().gwas_rotate(self._h, int(m0), mb, ptr, _dtype_code(xr), dev, _stream_ptr(stream)))
        if not dev:
            self._sync(stream)
        return keep

    def solve(self, y, h2, form: str = "f32", i0: int = 0, m: int | None = None, out=None,
              stream=None):
        """b [m][t][p] for SNPs [i0, i0+m) and traits y [t][n] with heritabilities h2 [t].

        out: a preallocated torch tensor (device or pinned host) or None (a new
        device tensor). Enqueued on `stream` (default: torch's current stream).
        """
        import torch
        lib = load()
        f = FORMS[form]
        m = self.m_capacity - i0 if m is None else int(m)
        t = int(y.shape[0])
        h2 = np.ascontiguousarray(h2, dtype=np.float64)
        if h2.shape != (t,):
            raise ValueError("h2 needs one value per trait")
        yp, ydev, ykeep = _ptr(y if _is_device(y) else np.ascontiguousarray(y, dtype=np.float64))
        if _is_device(y) and y.dtype != torch.float64:
            raise ValueError("device traits must be float64")
        dt = torch.float64 if f == FORM_F64 else torch.float32
        if out is None:
            out = torch.empty((m, t, self.p), dtype=dt, device="cuda:%d" % self.device)
        if out.dtype != dt or tuple(out.shape) != (m, t, self.p) or not out.is_contiguous():
            raise ValueError("out must be a contiguous %s tensor of shape %s" % (dt, (m, t, self.p)))
        _check(lib.gwas_solve(self._h, int(i0), m, t, yp, ydev, h2.ctypes.data, f,
                              ctypes.c_void_p(out.data_ptr()), int(out.is_cuda), _stream_ptr(stream)))
        self._keep = (ykeep, h2)
        return out

    def solve_noalloc(self, y, h2, out, form: str = "f32", i0: int = 0, stream=None):
        """gwas_solve_noalloc: b for SNPs [i0, i0 + out.shape[0]) and traits y [t][n]
        into `out`, a preallocated contiguous device tensor [m][t][p]; the library
        allocates nothing (its per-call buffers live in a fixed device array)."""
        import torch
        f = FORMS[form]
        m, t = int(out.shape[0]), int(y.shape[0])
        h2 = np.ascontiguousarray(h2, dtype=np.float64)
        if h2.shape != (t,):
            raise ValueError("h2 needs one value per trait")
        if _is_device(y) and y.dtype != torch.float64:
            raise ValueError("device traits must be float64")
        yp, ydev, ykeep = _ptr(y if _is_device(y) else np.ascontiguousarray(y, dtype=np.float64))
        dt = torch.float64 if f == FORM_F64 else torch.float32
        if not out.is_cuda or out.dtype != dt or tuple(out.shape) != (m, t, self.p) or not out.is_contiguous():
            raise ValueError("out must be a contiguous device %s tensor of shape %s" % (dt, (m, t, self.p)))
        _check(load().gwas_solve_noalloc(self._h, int(i0), m, t, yp, ydev, h2.ctypes.data, f,
                                         ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        self._keep = (ykeep, h2)
        return out

    def _slab_callback(self, form, on_slab, errors):
        dt = np.float64 if FORMS[form] == FORM_F64 else np.float32

        def cb(_user, sp):
            if on_slab is None:
                return
            try:
                s = sp.contents
                n_el = s.bytes // np.dtype(dt).itemsize
                buf = (ctypes.c_char * s.bytes).from_address(s.b)
                arr = np.frombuffer(buf, dtype=dt, count=n_el).reshape(s.count, s.tb, s.p)
                on_slab({"index": s.index, "i0": s.i0, "count": s.count, "j0": s.j0, "tb": s.tb,
                         "checksum": s.checksum}, arr)
            except Exception as e:       # never propagate through the C frame
                errors.append(e)

        return SLAB_FN(cb)

    def _traits(self, y, h2):
        t = int(y.shape[0])
        h2 = np.ascontiguousarray(h2, dtype=np.float64)
        if h2.shape != (t,):
            raise ValueError("h2 needs one value per trait")
        yp, ydev, ykeep = _ptr(y if _is_device(y) else np.ascontiguousarray(y, dtype=np.float64))
        return t, h2, yp, ydev, ykeep

    def solve_stream(self, y, h2, form: str = "f32", i0: int = 0, m: int | None = None,
                     on_slab=None, stream=None, max_slabs: int = 1 << 20):
        """Streamed solve: b arrives slab by slab in pinned host memory.

        on_slab(slab_info: dict, b: numpy view) is called for each slab on the
        calling thread; the view is valid only during the call. Returns the
        list of slab checksums (see gwas_checksum).
        """
        lib = load()
        f = FORMS[form]
        m = self.m_capacity - i0 if m is None else int(m)
        t, h2, yp, ydev, ykeep = self._traits(y, h2)
        errors = []
        fn = self._slab_callback(form, on_slab, errors)
        sums = (ctypes.c_uint64 * max_slabs)()
        n = ctypes.c_int64(0)
        _check(lib.gwas_solve_stream(self._h, int(i0), m, t, yp, ydev, h2.ctypes.data, f, fn, None,
                                     sums, max_slabs, ctypes.byref(n), _stream_ptr(stream)))
        if errors:
            raise errors[0]
        del ykeep
        return [int(sums[k]) for k in range(min(n.value, max_slabs))]

    def solve_snp_stream(self, xr, y, h2, form: str = "f32", on_slab=None, stream=None,
                         max_slabs: int = 1 << 20):
        """Genotype stream: SNP columns xr [m][n] (uint8, float32 or float64; numpy, or a
        pinned or device torch tensor) are copied, rotated and solved block by block
        through the resident store (m may exceed m_capacity); b arrives as in
        solve_stream, slab i0 being the SNP's row in xr. Returns the slab checksums."""
        lib = load()
        f = FORMS[form]
        xp, _xdev, xkeep = _ptr(xr)
        m = int(xr.shape[0])
        if m and int(xr.shape[1]) != self.n:
            raise ValueError("SNP columns must be [m][n]")
        t, h2, yp, ydev, ykeep = self._traits(y, h2)
        errors = []
        fn = self._slab_callback(form, on_slab, errors)
        sums = (ctypes.c_uint64 * max_slabs)()
        n = ctypes.c_int64(0)
        _check(lib.gwas_solve_snp_stream(self._h, xp, _dtype_code(xr), m, t, yp, ydev, h2.ctypes.data, f, fn,
                                         None, sums, max_slabs, ctypes.byref(n), _stream_ptr(stream)))
        if errors:
            raise errors[0]
        del ykeep, xkeep
        return [int(sums[k]) for k in range(min(n.value, max_slabs))]

    def copy_rotated(self, i0: int, m: int, form: str = "f64"):
        """Rotated SNP columns [i0, i0+m) from the resident store (numpy, [m][n])."""
        f = FORMS[form]
        out = np.empty((m, self.n), dtype=np.float64 if f == FORM_F64 else np.float32)
        _check(load().gwas_copy_rotated(self._h, int(i0), int(m), f, out.ctypes.data, 0,
                                        _stream_ptr(None)))
        return out

    def stats(self) -> dict:
        s = Stats()
        _check(load().gwas_stats(self._h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in Stats._fields_ if k != "reserved"}

    def debug_copy(self, what: str, form: str = "f64"):
        """An internal buffer as a flat numpy array (see gwas_debug_copy)."""
        code = {"xl": 0, "yt": 1, "fac": 2, "panels": 3}[what]
        f = FORMS[form]
        size = load().gwas_debug_size(self._h, code, f)
        if size < 0:
            raise ValueError("no such buffer")
        dt = np.uint16 if (what == "panels" and f in (FORM_BF16X3, FORM_BF16X6)) else \
            (np.float32 if (what == "panels" and f == FORM_F32) else np.float64)
        out = np.empty(size // np.dtype(dt).itemsize, dtype=dt)
        _check(load().gwas_debug_copy(self._h, code, f, out.ctypes.data, size))
        return out

    def reset_stats(self):
        _check(load().gwas_reset_stats(self._h))

    def _sync(self, stream):
        import torch
        (stream or torch.cuda.current_stream()).synchronize()


class Server:
    """Continuous-batching server over a resident Cohort (gwas_server_* in gwas.h).

    submit() copies the traits and returns a ticket at once; requests that
    arrive while others are on the GPU are admitted as slots and the HBM budget
    free up, and each scheduling round runs one slab of every admitted request
    in a single launch.
    """

    def __init__(self, cohort: "Cohort", form: str = "f32", hbm_budget: int = 0, max_slots: int = 0,
                 item_problems: int = 0, max_traits: int = 0, ring_slots: int = 0, host_threads: int = 0,
                 skip_checksum: bool = False, grid_wgs: int = 0):
        lib = load()
        opt = ServerOptions()
        opt.hbm_budget = int(hbm_budget)
        opt.max_slots = int(max_slots)
        opt.form = FORMS[form]
        opt.item_problems = int(item_problems)
        opt.max_traits = int(max_traits)
        opt.ring_slots = int(ring_slots)
        opt.host_threads = int(host_threads)
        opt.skip_checksum = int(bool(skip_checksum))
        opt.grid_wgs = int(grid_wgs)
        h = ctypes.c_void_p()
        _check(lib.gwas_server_create(cohort._h, ctypes.byref(opt), ctypes.byref(h)))
        self._h = h
        self.cohort = cohort
        self.form = form
        self._outs = {}

    def submit(self, y, h2, p: int, out=None, i0: int = 0, m: int = 0) -> int:
        """Queue a request: traits y [t][n], h2 [t], design width p (intercept-first
        covariate prefix). out: host array/tensor [m][t][p] kept until completion,
        or None (b streams through the pinned ring and is checksummed)."""
        y = np.ascontiguousarray(y, dtype=np.float64)
        h2 = np.ascontiguousarray(h2, dtype=np.float64)
        r = Request()
        r.t = int(y.shape[0])
        r.p = int(p)
        r.Y = y.ctypes.data
        r.h2 = h2.ctypes.data
        r.i0 = int(i0)
        r.m = int(m)
        keep = None
        if out is not None:
            bp, dev, keep = _ptr(out)
            if dev:
                raise ValueError("a request's output must be host memory")
            r.b = bp.value
        tk = ctypes.c_uint64()
        _check(load().gwas_server_submit(self._h, ctypes.byref(r), ctypes.byref(tk)))
        if keep is not None:
            self._outs[tk.value] = keep
        return tk.value

    @staticmethod
    def _res(res: Result) -> dict:
        return {"state": REQ_STATES[res.state], "error": res.error, "t_submit": res.t_submit,
                "t_admit": res.t_admit, "t_done": res.t_done, "problems": res.problems,
                "slabs": res.slabs, "checksum": int(res.checksum)}

    def poll(self, ticket: int) -> dict:
        res = Result()
        _check(load().gwas_server_poll(self._h, int(ticket), ctypes.byref(res)))
        return self._res(res)

    def wait(self, ticket: int, timeout: float | None = None) -> dict:
        res = Result()
        _check(load().gwas_server_wait(self._h, int(ticket), -1.0 if timeout is None else float(timeout),
                                       ctypes.byref(res)))
        self._outs.pop(int(ticket), None)
        return self._res(res)

    def cancel(self, ticket: int):
        _check(load().gwas_server_cancel(self._h, int(ticket)))

    def stats(self) -> dict:
        st = ServerStats()
        _check(load().gwas_server_stats(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_ if k != "reserved"}

    def close(self):
        if getattr(self, "_h", None):
            _check(load().gwas_server_destroy(self._h))
            self._h = None
            self._outs.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def eigh(phi, stream=None):
    """Eigendecomposition of the symmetric kinship matrix on the GPU (gwas_eigh),
    in numpy.linalg.eigh's convention: (w ascending, Z with column k the unit
    eigenvector k). A torch CUDA tensor gives CUDA tensors back (FP64); anything
    else is taken as a host array and numpy arrays come back."""
    if _is_device(phi):
        import torch
        a = phi.to(torch.float64).contiguous()
        n = a.shape[0]
        if a.shape != (n, n):
            raise ValueError("Phi must be square")
        z = torch.empty_like(a)
        w = torch.empty(n, dtype=torch.float64, device=a.device)
        # column-major Phi is Phi itself (symmetric); column-major Z is Z^T row-major
        _check(load().gwas_eigh(n, a.data_ptr(), z.data_ptr(), w.data_ptr(), 1, _stream_ptr(stream)))
        return w, z.T.contiguous()
    a = np.ascontiguousarray(phi, dtype=np.float64)
    n = a.shape[0]
    if a.shape != (n, n):
        raise ValueError("Phi must be square")
    zc = np.empty((n, n), dtype=np.float64)
    w = np.empty(n, dtype=np.float64)
    st = load().gwas_eigh(n, a.ctypes.data, zc.ctypes.data, w.ctypes.data, 0, None)
    _check(st)
    return w, np.ascontiguousarray(zc.T)


def clock() -> float:
    """The library's steady clock (seconds), the time base of request timestamps."""
    return float(load().gwas_clock())


def checksum(arr) -> int:
    """The slab checksum of gwas_solve_stream, computed by the library on host memory."""
    a = np.ascontiguousarray(arr)
    return int(load().gwas_checksum(a.ctypes.data, a.nbytes))


def version() -> str:
    return load().gwas_version().decode()
