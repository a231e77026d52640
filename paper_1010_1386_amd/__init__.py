"""Python binding of librsl (resultants of bivariate integer polynomials on MI355X).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``librsl.so``; this module converts Python integers to and from
the limb arrays of the C-ABI (``include/rsl.h``) and uses PyTorch solely for
the device workspace tensor and the HIP stream.  If the native library is
missing, importing this package raises -- there is no CPU fallback.

Polynomials are 2-D arrays ``F[j][i]`` = coefficient of x^i y^j (lists of
Python ints or numpy integer arrays).  Results are lists of Python ints,
lowest power first, ``[]`` for the zero polynomial.
"""

from __future__ import annotations

import ctypes
import os
import threading
import weakref

import numpy as np

# torch must be imported before librsl.so is loaded: torch ships its own HIP
# runtime (SONAME libamdhip64.so.7); loading torch first makes librsl bind to
# that same runtime, so device pointers and streams are shared.  Loading the
# system runtime first would put two HIP runtimes into one process.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "librsl.so")

if not os.path.exists(_LIBPATH):
    raise ImportError(f"librsl.so not built ({_LIBPATH}); run `python paper_1010_1386_amd/build.py`")

_lib = ctypes.CDLL(_LIBPATH)

RSL_OK, RSL_EINVAL, RSL_ERANGE, RSL_ENOMEM, RSL_EPRIMES, RSL_EDEVICE, RSL_EAGAIN, RSL_ETIMEDOUT = (
    0, -1, -2, -3, -4, -5, -6, -7)
RSL_Y, RSL_X = 0, 1
RSL_PLAIN, RSL_BATCHED, RSL_STAGED, RSL_AUTO = 0, 1, 2, 3
RSL_GRAPH = 0x100
RSL_POINTS_REPLACE, RSL_POINTS_FORMAL = 0, 1


class rsl_poly(ctypes.Structure):
    _fields_ = [("dx", ctypes.c_int32), ("dy", ctypes.c_int32), ("limbs", ctypes.c_int32),
                ("coeff", ctypes.POINTER(ctypes.c_uint32))]


class rsl_result(ctypes.Structure):
    _fields_ = [("cap_deg", ctypes.c_int32), ("limbs", ctypes.c_int32),
                ("coeff", ctypes.POINTER(ctypes.c_uint32)), ("deg", ctypes.c_int32),
                ("needed_limbs", ctypes.c_int32)]


class rsl_info(ctypes.Structure):
    _fields_ = [("D", ctypes.c_int32), ("bound_bits", ctypes.c_int32), ("n_primes", ctypes.c_int32),
                ("n_points", ctypes.c_int32), ("out_limbs", ctypes.c_int32), ("my", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("bad_primes", ctypes.c_int32), ("footprint_bytes", ctypes.c_size_t),
                ("table_bytes", ctypes.c_size_t), ("origin", ctypes.c_int32)]


class rsl_opts(ctypes.Structure):
    _fields_ = [("points", ctypes.c_int32), ("prime_start", ctypes.c_int32), ("extra_primes", ctypes.c_int32),
                ("point_origin", ctypes.c_int32), ("extra_points", ctypes.c_int32),
                ("prime_limit", ctypes.c_int32), ("eval_lanes", ctypes.c_int32), ("eval_regs", ctypes.c_int32),
                ("eval_schur", ctypes.c_int32), ("interp_mm", ctypes.c_int32),
                ("interp_newton", ctypes.c_int32)]


class rsl_counters(ctypes.Structure):
    _fields_ = [("problems", ctypes.c_int64), ("pairs", ctypes.c_int64), ("bad_pairs", ctypes.c_int64),
                ("bad_primes", ctypes.c_int64), ("slow_primes", ctypes.c_int64),
                ("ms_device", ctypes.c_double), ("ms_total", ctypes.c_double), ("ms_build", ctypes.c_double),
                ("ms_bind", ctypes.c_double), ("ms_transfer", ctypes.c_double), ("ms_decode", ctypes.c_double)]


class rsl_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("in_flight", ctypes.c_int64), ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("mean_ms", ctypes.c_double), ("throughput", ctypes.c_double),
                ("admitted_bytes_peak", ctypes.c_int64), ("launches", ctypes.c_int64),
                ("max_batch", ctypes.c_int64)]


class rsl_job_info(ctypes.Structure):
    _fields_ = [("n_problems", ctypes.c_int32), ("n_live", ctypes.c_int32), ("pairs", ctypes.c_int64),
                ("mulmods", ctypes.c_int64), ("device_bytes", ctypes.c_size_t), ("upload_bytes", ctypes.c_size_t),
                ("download_bytes", ctypes.c_size_t), ("layout_mode", ctypes.c_int32),
                ("chunk_target", ctypes.c_int32), ("grid_mult", ctypes.c_int32), ("eval_lanes", ctypes.c_int32),
                ("eval_mfma", ctypes.c_int32), ("mulmods_sums_mfma", ctypes.c_int64), ("mulmods_valu", ctypes.c_int64),
                ("mfma_int8_macs", ctypes.c_int64), ("interp_mulmods", ctypes.c_int64)]


class rsl_upoly(ctypes.Structure):
    _fields_ = [("deg", ctypes.c_int32), ("limbs", ctypes.c_int32), ("coeff", ctypes.POINTER(ctypes.c_uint32))]


class rsl_tune_result(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("chunk_target", ctypes.c_int32), ("grid_mult", ctypes.c_int32),
                ("evk", ctypes.c_int32), ("conv_whole", ctypes.c_int32), ("schur", ctypes.c_int32),
                ("interp_mm", ctypes.c_int32),
                ("candidates", ctypes.c_int32),
                ("ms", ctypes.c_double),
                ("ms_worst", ctypes.c_double)]


STAGES = ("reduce", "eval_ures", "interp_conv", "interp_stir", "interp_newton", "crt")

_P = ctypes.POINTER
_vp = ctypes.c_void_p
_SIGS = {
    "rsl_ctx_create": (ctypes.c_int, [ctypes.c_int, _vp, ctypes.c_size_t, _vp, ctypes.c_size_t, _vp, _P(_vp)]),
    "rsl_ctx_destroy": (ctypes.c_int, [_vp]),
    "rsl_query": (ctypes.c_int, [_P(rsl_poly), _P(rsl_poly), ctypes.c_int, _P(rsl_info)]),
    "rsl_res": (ctypes.c_int, [_vp, _P(rsl_poly), _P(rsl_poly), ctypes.c_int, _P(rsl_opts), _P(rsl_result)]),
    "rsl_res_static": (ctypes.c_int, [_vp, _P(rsl_poly), _P(rsl_poly), ctypes.c_int, _P(rsl_opts), _P(rsl_result)]),
    "rsl_res_y": (ctypes.c_int, [_vp, _P(rsl_poly), _P(rsl_poly), _P(rsl_result)]),
    "rsl_res_x": (ctypes.c_int, [_vp, _P(rsl_poly), _P(rsl_poly), _P(rsl_result)]),
    "rsl_res_xy": (ctypes.c_int, [_vp, _P(rsl_poly), _P(rsl_poly), _P(rsl_opts), _P(rsl_result), _P(rsl_result)]),
    "rsl_gcd": (ctypes.c_int, [_vp, _P(rsl_upoly), _P(rsl_upoly), _P(rsl_result), _P(rsl_result), _P(rsl_result)]),
    "rsl_sqfree_part": (ctypes.c_int, [_vp, _P(rsl_upoly), _P(rsl_result), _P(rsl_result)]),
    "rsl_sqfree_factor": (ctypes.c_int, [_vp, _P(rsl_upoly), ctypes.c_int, _P(rsl_result), _P(ctypes.c_int)]),
    "rsl_batch": (ctypes.c_int, [_vp, ctypes.c_int, _P(rsl_poly), _P(rsl_poly), _P(ctypes.c_int),
                                 _P(rsl_result), _P(ctypes.c_int), ctypes.c_int]),
    "rsl_last_counters": (ctypes.c_int, [_vp, _P(rsl_counters)]),
    "rsl_server_create": (ctypes.c_int, [_vp, ctypes.c_size_t, ctypes.c_int, ctypes.c_int, _P(_vp)]),
    "rsl_server_submit": (ctypes.c_int, [_vp, _P(rsl_poly), _P(rsl_poly), ctypes.c_int, _P(rsl_result),
                                         _P(ctypes.c_uint64)]),
    "rsl_server_plan": (ctypes.c_int, [_vp, _P(rsl_poly), _P(rsl_poly), ctypes.c_int, _P(rsl_info),
                                       _P(ctypes.c_uint64)]),
    "rsl_server_enqueue": (ctypes.c_int, [_vp, ctypes.c_uint64, _P(rsl_result), _P(ctypes.c_uint64)]),
    "rsl_server_poll": (ctypes.c_int, [_vp, ctypes.c_uint64, _P(ctypes.c_int)]),
    "rsl_server_wait": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.c_int]),
    "rsl_server_stats": (ctypes.c_int, [_vp, _P(rsl_stats)]),
    "rsl_server_destroy": (ctypes.c_int, [_vp]),
    "rsl_job_create": (ctypes.c_int, [_vp, ctypes.c_int, _P(rsl_poly), _P(rsl_poly), _P(ctypes.c_int),
                                      _P(rsl_opts), _P(ctypes.c_int), _P(_vp)]),
    "rsl_job_bind": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_size_t]),
    "rsl_job_run": (ctypes.c_int, [_vp, _vp, ctypes.c_int]),
    "rsl_job_results": (ctypes.c_int, [_vp, _vp, _P(rsl_result), _P(ctypes.c_int)]),
    "rsl_job_info_get": (ctypes.c_int, [_vp, _P(rsl_job_info)]),
    "rsl_job_destroy": (ctypes.c_int, [_vp]),
    "rsl_job_tune": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _P(rsl_tune_result)]),
    "rsl_tune_save": (ctypes.c_int, [_vp, ctypes.c_char_p]),
    "rsl_tune_load": (ctypes.c_int, [_vp, ctypes.c_char_p]),
    "rsl_profile_enable": (ctypes.c_int, [_vp, ctypes.c_int]),
    "rsl_profile_take": (ctypes.c_int, [_vp, _P(ctypes.c_double), _P(ctypes.c_int)]),
    "rsl_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "rsl_last_error": (ctypes.c_char_p, [_vp]),
    "rsl_version": (ctypes.c_char_p, []),
}
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


class RSLError(RuntimeError):
    def __init__(self, code, msg=""):
        self.code = code
        super().__init__(f"{_lib.rsl_strerror(code).decode()} ({code}){': ' + msg if msg else ''}")


def library_path():
    return _LIBPATH


def version():
    return _lib.rsl_version().decode()


# ------------------------------------------------------------------ marshalling


class Poly:
    """A bivariate polynomial packed as C-ABI limbs (keeps the buffer alive)."""

    def __init__(self, F):
        arr = F if isinstance(F, np.ndarray) else None
        if arr is not None and arr.dtype != object and np.issubdtype(arr.dtype, np.integer):
            a = np.ascontiguousarray(arr, dtype=np.int64)
            if a.ndim != 2 or a.size == 0:
                raise ValueError("polynomial must be a non-empty 2-D array")
            self.dy, self.dx = a.shape[0] - 1, a.shape[1] - 1
            self.limbs = 2
            self.buf = np.ascontiguousarray(a.view(np.uint32))
        else:
            rows = [list(r) for r in F]
            if not rows:
                rows = [[0]]
            width = max(1, max(len(r) for r in rows))
            self.dy, self.dx = len(rows) - 1, width - 1
            flat = [int(v) for r in rows for v in (list(r) + [0] * (width - len(r)))]
            bits = max((v.bit_length() + 1 for v in flat), default=1)
            if bits <= 64:
                self.limbs = 2
                self.buf = np.ascontiguousarray(np.array(flat, dtype=np.int64).view(np.uint32))
            else:
                self.limbs = (bits + 31) // 32
                nb = 4 * self.limbs
                raw = b"".join(v.to_bytes(nb, "little", signed=True) for v in flat)
                self.buf = np.frombuffer(raw, dtype=np.uint32).copy()
        self.c = rsl_poly(self.dx, self.dy, self.limbs,
                          self.buf.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))


class UPoly:
    """A univariate integer polynomial (list, lowest power first) packed as C-ABI limbs."""

    def __init__(self, a):
        vals = [int(v) for v in a]
        bits = max((v.bit_length() + 1 for v in vals), default=1)
        self.limbs = max(1, (bits + 31) // 32)
        nb = 4 * self.limbs
        raw = b"".join(v.to_bytes(nb, "little", signed=True) for v in vals) or bytes(nb)
        self.buf = np.frombuffer(raw, dtype=np.uint32).copy()
        self.deg = len(vals) - 1
        self.c = rsl_upoly(self.deg, self.limbs, self.buf.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
        # size of any factor's coefficients (Mignotte): deg + log2 ||a||_2 bits
        norm2 = sum(v * v for v in vals)
        self.factor_bits = max(self.deg, 0) + (norm2.bit_length() + 2) // 2 + 2


def _as_poly(F):
    return F if isinstance(F, Poly) else Poly(F)


def _var_code(var):
    if var in ("y", RSL_Y):
        return RSL_Y
    if var in ("x", RSL_X):
        return RSL_X
    raise ValueError("var must be 'y' or 'x'")


class _Result:
    def __init__(self, cap_deg, limbs):
        self.buf = np.zeros(max(1, (cap_deg + 1) * limbs), dtype=np.uint32)
        self.c = rsl_result(cap_deg, limbs, self.buf.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), 0, 0)

    def raw(self):
        """(degree, limbs, the used limb words as bytes): the result without conversion."""
        deg, L = self.c.deg, self.c.limbs
        return deg, L, self.buf[:max(deg + 1, 0) * L].tobytes()

    def value(self):
        deg, L = self.c.deg, self.c.limbs
        if deg < 0:
            return []
        w = self.buf[:(deg + 1) * L]
        if L == 2:
            return [int(v) for v in w.view(np.int64)]
        raw = w.tobytes()
        nb = 4 * L
        return [int.from_bytes(raw[k * nb:(k + 1) * nb], "little", signed=True) for k in range(deg + 1)]


def query(f, g, var="y"):
    """Sizing of res(f, g, var) without device work (dict of rsl_info fields)."""
    pf, pg = _as_poly(f), _as_poly(g)
    info = rsl_info()
    rc = _lib.rsl_query(ctypes.byref(pf.c), ctypes.byref(pg.c), _var_code(var), ctypes.byref(info))
    if rc:
        raise RSLError(rc)
    return {name: getattr(info, name) for name, _ in rsl_info._fields_}


def _opts(points="replace", prime_start=0, extra_primes=0, point_origin=0, extra_points=0, prime_limit=0,
          eval_lanes=0, eval_regs=True, eval_schur=False, interp_mm=False, interp_newton=False):
    if eval_lanes not in (0, 1, 2, 4):
        raise ValueError("eval_lanes must be 0, 1, 2 or 4")
    o = rsl_opts()
    o.eval_lanes = eval_lanes
    o.eval_regs = 0 if eval_regs else -1
    o.eval_schur = 1 if eval_schur else 0
    o.interp_newton = 1 if interp_newton else 0
    o.interp_mm = 1 if interp_mm else 0
    o.points = RSL_POINTS_FORMAL if points in ("formal", RSL_POINTS_FORMAL) else RSL_POINTS_REPLACE
    o.prime_start, o.extra_primes = prime_start, extra_primes
    o.point_origin, o.extra_points, o.prime_limit = point_origin, extra_points, prime_limit
    return o


# ------------------------------------------------------------------ context


class Context:
    """A device context: torch uint8 tensors on ``cuda:device`` for the per-call
    workspace and the constant tables, plus a HIP stream.  The library allocates
    no device memory of its own (rsl_res_static's fixed array aside)."""

    def __init__(self, device=0, workspace_bytes=256 << 20, stream=None, table_bytes=256 << 20,
                 tables_in_workspace=False):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: librsl runs only on the device")
        self.device = device
        self.workspace = torch.empty(workspace_bytes, dtype=torch.uint8, device=f"cuda:{device}")
        # tables_in_workspace: the top table_bytes of the workspace hold the tables
        self.tables = None if tables_in_workspace else torch.empty(table_bytes, dtype=torch.uint8,
                                                                    device=f"cuda:{device}")
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        h = _vp()
        tab = ctypes.c_void_p(self.tables.data_ptr()) if self.tables is not None else None
        rc = _lib.rsl_ctx_create(device, ctypes.c_void_p(self.workspace.data_ptr()), workspace_bytes,
                                 tab, table_bytes, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc:
            raise RSLError(rc, "rsl_ctx_create")
        self.h = h
        self.lock = threading.RLock()
        self._owned = weakref.WeakSet()  # jobs and servers made on this context: closed before it

    def close(self):
        if getattr(self, "h", None):
            for o in list(getattr(self, "_owned", ())):
                o.close()  # their destruction synchronizes on the context's stream
            _lib.rsl_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self):
        return _lib.rsl_last_error(self.h).decode()

    def counters(self):
        c = rsl_counters()
        _lib.rsl_last_counters(self.h, ctypes.byref(c))
        return {name: getattr(c, name) for name, _ in rsl_counters._fields_}

    def _check(self, rc, what):
        if rc:
            raise RSLError(rc, f"{what}: {self.last_error()}")

    def res(self, f, g, var="y", **opts):
        """res(f, g, var) as a list of Python ints (lowest power first)."""
        pf, pg = _as_poly(f), _as_poly(g)
        v = _var_code(var)
        info = rsl_info()
        rc = _lib.rsl_query(ctypes.byref(pf.c), ctypes.byref(pg.c), v, ctypes.byref(info))
        self._check(rc, "rsl_query")
        o = _opts(**opts)
        lim = info.out_limbs + (1 if o.extra_primes else 0) + o.extra_primes
        out = _Result(max(info.D, 0), max(1, lim))
        with self.lock:
            rc = _lib.rsl_res(self.h, ctypes.byref(pf.c), ctypes.byref(pg.c), v, ctypes.byref(o),
                              ctypes.byref(out.c))
        self._check(rc, "rsl_res")
        return out.value()

    def res_static(self, f, g, var="y", **opts):
        """res(f, g, var) through rsl_res_static: no device memory is allocated (the job
        lives in the library's fixed device array; the context's tables must cover it)."""
        pf, pg = _as_poly(f), _as_poly(g)
        v = _var_code(var)
        info = rsl_info()
        self._check(_lib.rsl_query(ctypes.byref(pf.c), ctypes.byref(pg.c), v, ctypes.byref(info)), "rsl_query")
        o = _opts(**opts)
        lim = info.out_limbs + (1 if o.extra_primes else 0) + o.extra_primes
        out = _Result(max(info.D, 0), max(1, lim))
        with self.lock:
            rc = _lib.rsl_res_static(self.h, ctypes.byref(pf.c), ctypes.byref(pg.c), v, ctypes.byref(o),
                                     ctypes.byref(out.c))
        self._check(rc, "rsl_res_static")
        return out.value()

    def res_y(self, f, g):
        return self.res(f, g, "y")

    def res_x(self, f, g):
        return self.res(f, g, "x")

    def res_xy(self, f, g, **opts):
        """(res(f, g, y), res(f, g, x)) computed as one job."""
        pf, pg = _as_poly(f), _as_poly(g)
        o = _opts(**opts)
        outs = []
        for v in (RSL_Y, RSL_X):
            info = rsl_info()
            self._check(_lib.rsl_query(ctypes.byref(pf.c), ctypes.byref(pg.c), v, ctypes.byref(info)), "rsl_query")
            lim = info.out_limbs + (1 if o.extra_primes else 0) + o.extra_primes
            outs.append(_Result(max(info.D, 0), max(1, lim)))
        with self.lock:
            rc = _lib.rsl_res_xy(self.h, ctypes.byref(pf.c), ctypes.byref(pg.c), ctypes.byref(o),
                                 ctypes.byref(outs[0].c), ctypes.byref(outs[1].c))
        self._check(rc, "rsl_res_xy")
        return outs[0].value(), outs[1].value()

    def gcd(self, u, v):
        """(G, u / G, v / G): G = gcd(pp(u), pp(v)) in Z[x], primitive with positive
        leading coefficient; polynomials as lists of ints, lowest power first."""
        pu, pv = UPoly(u), UPoly(v)
        bits = max(pu.factor_bits, pv.factor_bits)
        limbs = bits // 32 + 2
        outs = [_Result(max(pu.deg, pv.deg, 0), limbs) for _ in range(3)]
        with self.lock:
            rc = _lib.rsl_gcd(self.h, ctypes.byref(pu.c), ctypes.byref(pv.c), ctypes.byref(outs[0].c),
                              ctypes.byref(outs[1].c), ctypes.byref(outs[2].c))
        self._check(rc, "rsl_gcd")
        return tuple(o.value() for o in outs)

    def sqfree_part(self, r):
        """(q, g): g = gcd(pp(r), pp(r)'), q = r / g (pp(q) is the square-free part)."""
        pr = UPoly(r)
        limbs = pr.factor_bits // 32 + 2
        outs = [_Result(max(pr.deg, 0), limbs) for _ in range(2)]
        with self.lock:
            rc = _lib.rsl_sqfree_part(self.h, ctypes.byref(pr.c), ctypes.byref(outs[0].c), ctypes.byref(outs[1].c))
        self._check(rc, "rsl_sqfree_part")
        return tuple(o.value() for o in outs)

    def sqfree_factor(self, r):
        """[r_1, r_2, ...] with pp(r) = prod r_i^i (Yun's algorithm on the device gcd)."""
        pr = UPoly(r)
        n = max(pr.deg, 1)
        limbs = pr.factor_bits // 32 + 2
        # r_i^i divides pp(r): the i-th factor has degree at most deg r / i
        outs = [_Result(max(pr.deg, 0) // (i + 1), limbs) for i in range(n)]
        arr = (rsl_result * n)(*[o.c for o in outs])
        cnt = ctypes.c_int(0)
        with self.lock:
            rc = _lib.rsl_sqfree_factor(self.h, ctypes.byref(pr.c), n, arr, ctypes.byref(cnt))
        self._check(rc, "rsl_sqfree_factor")
        res = []
        for i in range(cnt.value):
            outs[i].c = arr[i]
            res.append(outs[i].value())
        return res

    def batch(self, problems, mode="batched"):
        """problems: list of (f, g, var); returns a list of results (lists of ints)."""
        pb = PreparedBatch(problems)
        pb.run(self, mode)
        return pb.results()

    def profile_enable(self, on=True):
        self._check(_lib.rsl_profile_enable(self.h, 1 if on else 0), "rsl_profile_enable")

    def profile_take(self):
        """(per-stage device ms summed over the profiled launches, number of launches)."""
        ms = (ctypes.c_double * len(STAGES))()
        runs = ctypes.c_int()
        self._check(_lib.rsl_profile_take(self.h, ms, ctypes.byref(runs)), "rsl_profile_take")
        return dict(zip(STAGES, list(ms))), runs.value

    def tune_save(self, path):
        with self.lock:
            self._check(_lib.rsl_tune_save(self.h, os.fsencode(path)), "rsl_tune_save")

    def tune_load(self, path):
        with self.lock:
            self._check(_lib.rsl_tune_load(self.h, os.fsencode(path)), "rsl_tune_load")

    def job(self, problems, **opts):
        return Job(self, problems, **opts)


class PreparedBatch:
    """The C-ABI arguments of one batch, packed once: input limbs, variables and result
    buffers sized by rsl_query.  run() is then a single rsl_batch call (host limbs in,
    host limbs out: planning, upload, device pipeline, download and decoding into the
    result buffers all happen inside it); results() converts the limbs to Python ints."""

    def __init__(self, problems):
        n = len(problems)
        self.n = n
        self._polys, self._outs = [], []
        self.fa = (rsl_poly * max(n, 1))()
        self.ga = (rsl_poly * max(n, 1))()
        self.va = (ctypes.c_int * max(n, 1))()
        self.ra = (rsl_result * max(n, 1))()
        self.st = (ctypes.c_int * max(n, 1))()
        self.infos = []
        for k, (f, g, var) in enumerate(problems):
            pf, pg = _as_poly(f), _as_poly(g)
            v = _var_code(var)
            info = rsl_info()
            rc = _lib.rsl_query(ctypes.byref(pf.c), ctypes.byref(pg.c), v, ctypes.byref(info))
            if rc:
                raise RSLError(rc, f"rsl_query (problem {k})")
            r = _Result(max(info.D, 0), info.out_limbs)
            self._polys.append((pf, pg))
            self._outs.append(r)
            self.infos.append(info)
            self.fa[k], self.ga[k], self.va[k], self.ra[k] = pf.c, pg.c, v, r.c

    def run(self, ctx, mode="auto"):
        code = _modecode(mode)
        with ctx.lock:
            rc = _lib.rsl_batch(ctx.h, self.n, self.fa, self.ga, self.va, self.ra, self.st, code)
        ctx._check(rc, "rsl_batch")

    def statuses(self):
        return [self.st[k] for k in range(self.n)]

    def results(self):
        res = []
        for k in range(self.n):
            self._outs[k].c = self.ra[k]
            res.append(self._outs[k].value())
        return res


def _modecode(mode):
    codes = {"plain": RSL_PLAIN, "batched": RSL_BATCHED, "staged": RSL_STAGED, "auto": RSL_AUTO,
             RSL_PLAIN: RSL_PLAIN, RSL_BATCHED: RSL_BATCHED, RSL_STAGED: RSL_STAGED, RSL_AUTO: RSL_AUTO}
    if mode not in codes:
        raise ValueError("mode must be 'plain', 'batched', 'staged' or 'auto'")
    return codes[mode]


class Job:
    """Problems planned once with inputs resident on the device; run() repeats the device pipeline.

    The job's device memory is a torch uint8 tensor of ``device_bytes`` (default:
    the planned layout's size plus ``headroom``, so that the autotuner can try
    layouts that need a little more)."""

    def __init__(self, ctx, problems, device_bytes=None, headroom=0.5, **opts):
        self.ctx = ctx
        ctx._owned.add(self)
        n = len(problems)
        self.n = n
        self._polys = []
        self._outs = []
        self.fa = (rsl_poly * max(n, 1))()
        self.ga = (rsl_poly * max(n, 1))()
        self.va = (ctypes.c_int * max(n, 1))()
        self.ra = (rsl_result * max(n, 1))()
        for k, (f, g, var) in enumerate(problems):
            pf, pg = _as_poly(f), _as_poly(g)
            v = _var_code(var)
            info = rsl_info()
            ctx._check(_lib.rsl_query(ctypes.byref(pf.c), ctypes.byref(pg.c), v, ctypes.byref(info)), "rsl_query")
            r = _Result(max(info.D, 0), info.out_limbs)
            self._polys.append((pf, pg))
            self._outs.append(r)
            self.fa[k], self.ga[k], self.va[k], self.ra[k] = pf.c, pg.c, v, r.c
        o = _opts(**opts)
        st = (ctypes.c_int * max(n, 1))()
        h = _vp()
        with ctx.lock:
            rc = _lib.rsl_job_create(ctx.h, n, self.fa, self.ga, self.va, ctypes.byref(o), st, ctypes.byref(h))
        ctx._check(rc, "rsl_job_create")
        self.h = h
        if device_bytes is None:
            need = self.info()["device_bytes"]
            device_bytes = max(int(need * (1.0 + headroom)), 1 << 20)
        self.bind(device_bytes)

    def bind(self, device_bytes):
        """Give the job a fresh device buffer of ``device_bytes`` and upload its inputs."""
        import torch

        mem = torch.empty(int(device_bytes), dtype=torch.uint8, device=f"cuda:{self.ctx.device}")
        with self.ctx.lock:
            rc = _lib.rsl_job_bind(self.ctx.h, self.h, ctypes.c_void_p(mem.data_ptr()), int(device_bytes))
        self.ctx._check(rc, "rsl_job_bind")
        self.mem = mem  # released after the job (close() drops it last)

    def run(self, mode="batched", graph=False):
        """One device run of the whole pipeline; graph=True replays it as a captured HIP graph."""
        code = _modecode(mode) | (RSL_GRAPH if graph else 0)
        with self.ctx.lock:
            rc = _lib.rsl_job_run(self.ctx.h, self.h, code)
        self.ctx._check(rc, "rsl_job_run")

    def results(self):
        st = (ctypes.c_int * max(self.n, 1))()
        with self.ctx.lock:
            rc = _lib.rsl_job_results(self.ctx.h, self.h, self.ra, st)
        self.ctx._check(rc, "rsl_job_results")
        out = []
        for k in range(self.n):
            self._outs[k].c = self.ra[k]
            out.append(self._outs[k].value())
        return out

    def tune(self, reps=5):
        """Time the candidate schedules on this job, keep the fastest (the job is laid
        out again with it) and remember it for jobs of the same shape bucket."""
        r = rsl_tune_result()
        with self.ctx.lock:
            rc = _lib.rsl_job_tune(self.ctx.h, self.h, int(reps), ctypes.byref(r))
        self.ctx._check(rc, "rsl_job_tune")
        names = {RSL_STAGED: "staged", RSL_BATCHED: "batched"}
        return {"mode": names.get(r.mode, r.mode), "chunk_target": r.chunk_target, "grid_mult": r.grid_mult,
                "lanes_per_pair": r.evk, "conv_whole": r.conv_whole, "schur": r.schur, "interp_mm": r.interp_mm,
                "candidates": r.candidates, "ms": r.ms,
                "ms_worst": r.ms_worst}

    def info(self):
        i = rsl_job_info()
        _lib.rsl_job_info_get(self.h, ctypes.byref(i))
        return {name: getattr(i, name) for name, _ in rsl_job_info._fields_}

    def close(self):
        if getattr(self, "h", None):
            _lib.rsl_job_destroy(self.h)  # waits for the job's work on the context stream
            self.h = None
        self.mem = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default = None
_default_lock = threading.Lock()


def default_context():
    global _default
    with _default_lock:
        if _default is None:
            _default = Context()
        return _default


def res(f, g, var="y", **opts):
    return default_context().res(f, g, var, **opts)


def res_y(f, g):
    return res(f, g, "y")


def res_x(f, g):
    return res(f, g, "x")


def res_xy(f, g, **opts):
    return default_context().res_xy(f, g, **opts)


def batch(problems, mode="batched"):
    return default_context().batch(problems, mode)


from .server import Server  # noqa: E402,F401
