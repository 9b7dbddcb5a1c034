"""ctypes binding of libps.so (include/ps.h, include/ps_host.h).

Argument marshalling only: every step of the setup and solve runs in the native
library.  Device vectors are passed as torch tensors (or raw integer addresses),
streams as torch streams (or raw hipStream_t addresses).  There is no fallback:
if the library is not built, loading raises.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libps.so")

PS_OK, PS_PENDING = 0, 1
PS_EINVAL, PS_ENOMEM, PS_EDEVICE, PS_ENOTSETUP, PS_ESINGULAR = -1, -2, -3, -4, -5
PS_EMAXIT, PS_EPRECISION, PS_EBUSY, PS_EBREAKDOWN = -6, -7, -8, -9
PS_FP64, PS_FP32_PREC = 0, 1
PS_CHEB2, PS_L1JAC = 0, 1
PS_FGMRES, PS_RICHARDSON = 0, 1
PS_QUASI_IMPES, PS_TRUE_IMPES = 0, 1
PS_FS_GIVEN, PS_FS_RSL = 0, 1
PS_CGS2, PS_DCGS2 = 0, 1
PS_BILU0, PS_BJACOBI, PS_MCGS = 0, 1, 2
PS_H_SDC, PS_H_PRES = 0, 1
PS_KT_ALL = -1

_i32p = C.POINTER(C.c_int32)
_f64p = C.POINTER(C.c_double)


class ps_bsr(C.Structure):
    _fields_ = [("nbrows", C.c_int32), ("nbcols", C.c_int32), ("br", C.c_int32), ("bc", C.c_int32),
                ("nblocks", C.c_int32), ("rowptr", _i32p), ("colind", _i32p), ("vals", _f64p)]


class ps_system(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_cells", C.c_int32), ("nf", C.c_int32), ("p_index", C.c_int32),
                ("Auu", ps_bsr), ("Auf", ps_bsr), ("Afu", ps_bsr), ("Aff", ps_bsr),
                ("d_sp", _f64p), ("d_pp", _f64p), ("mech_key", C.c_uint64), ("ml_part", _i32p)]


class ps_options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("restart", C.c_int32), ("maxit", C.c_int32),
                ("smoother", C.c_int32), ("ml_kind", C.c_int32), ("ml_sweeps", C.c_int32),
                ("coarse_max", C.c_int32), ("max_levels", C.c_int32), ("fp32_fallback", C.c_int32),
                ("theta", C.c_double), ("method", C.c_int32), ("reduction", C.c_int32),
                ("fixed_stress", C.c_int32), ("fs_iters", C.c_int32), ("orth", C.c_int32)]


class ps_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("restarts", C.c_int32),
                ("rel_residual", C.c_double), ("setup_s", C.c_double), ("solve_s", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_SIGS = {
    "ps_default_options": (None, [C.POINTER(ps_options)]),
    "ps_ctx_create": (C.c_int, [C.c_int, C.c_size_t, C.POINTER(C.c_void_p)]),
    "ps_ctx_destroy": (None, [C.c_void_p]),
    "ps_create": (C.c_int, [C.c_void_p, C.POINTER(ps_system), C.POINTER(ps_options), C.POINTER(C.c_void_p)]),
    "ps_update_flow": (C.c_int, [C.c_void_p, _f64p, _f64p, _f64p, _f64p, _f64p]),
    "ps_setup": (C.c_int, [C.c_void_p]),
    "ps_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.POINTER(ps_result)]),
    "ps_solve_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p,
                                   C.POINTER(ps_result)]),
    "ps_apply_precond": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ps_spmv": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ps_submit": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.POINTER(C.c_uint64)]),
    "ps_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(ps_result)]),
    "ps_wait": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(ps_result)]),
    "ps_ctx_batches": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    "ps_footprint": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "ps_kernel_timing": (C.c_int, [C.c_int]),
    "ps_kernel_stats": (C.c_int, [C.c_int, C.c_char_p, C.c_size_t, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                  C.POINTER(C.c_double)]),
    "ps_pressure_level": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_double), C.POINTER(C.c_int8)]),
    "ps_destroy": (None, [C.c_void_p]),
    "ps_strerror": (C.c_char_p, [C.c_int]),
    "ps_last_error": (C.c_char_p, []),
    "ps_host_setup_create": (C.c_int, [C.POINTER(ps_system), C.POINTER(ps_options), C.POINTER(C.c_void_p)]),
    "ps_host_setup_destroy": (None, [C.c_void_p]),
    "ps_host_levels": (C.c_int, [C.c_void_p, C.c_int, _i32p]),
    "ps_host_level": (C.c_int, [C.c_void_p, C.c_int, C.c_int, _i32p, _i32p, _i32p, _i32p, _f64p,
                                C.POINTER(C.c_int8), _i32p, _i32p, _i32p, _i32p, _f64p]),
    "ps_host_level_lambda": (C.c_int, [C.c_void_p, C.c_int, C.c_int, _f64p]),
    "ps_host_spp": (C.c_int, [C.c_void_p, _f64p]),
    "ps_host_bilu": (C.c_int, [C.c_void_p, _f64p]),
    "ps_host_bilu_levels": (C.c_int, [C.c_void_p, _i32p, _i32p]),
}

_lib = None


def load(path=LIB_PATH):
    """Load libps.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise OSError("libps.so is not built; run paper_1812_05540_amd/build.py (%s)" % path)
        lib = C.CDLL(path)
        for name, (res, args) in _SIGS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def exported_symbols():
    return list(_SIGS)


class PsError(RuntimeError):
    def __init__(self, code, where):
        lib = load()
        msg = lib.ps_last_error().decode() or lib.ps_strerror(code).decode()
        super().__init__("%s: %s (%d)" % (where, msg, code))
        self.code = code


def _check(code, where):
    if code != PS_OK:
        raise PsError(code, where)


def _ptr(t):
    """Device address of a torch tensor, or an int passed through."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(s):
    if s is None:
        try:
            import torch
            return torch.cuda.current_stream().cuda_stream
        except Exception:
            return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


# ---------------------------------------------------------------------------- marshalling
def _bsr(b, keep):
    rp = np.ascontiguousarray(b.rowptr, dtype=np.int32)
    ci = np.ascontiguousarray(b.colind, dtype=np.int32)
    v = np.ascontiguousarray(b.vals, dtype=np.float64)
    keep += [rp, ci, v]
    nb, br, bc = v.shape if v.ndim == 3 else (ci.shape[0], b.br, b.bc)
    return ps_bsr(rp.shape[0] - 1, int(b.nbcols), int(br), int(bc), int(ci.shape[0]),
                  rp.ctypes.data_as(_i32p), ci.ctypes.data_as(_i32p), v.ctypes.data_as(_f64p))


def make_system(sysobj, mech_key=0):
    """ps_system from an object with Auu/Auf/Afu/Aff (rowptr, colind, vals, nbcols),
    d_sp, d_pp, n_nodes, n_cells, nf, p_index.  Returns (struct, keepalive)."""
    keep = []
    d_sp = np.ascontiguousarray(sysobj.d_sp, dtype=np.float64)
    d_pp = np.ascontiguousarray(sysobj.d_pp, dtype=np.float64)
    keep += [d_sp, d_pp]
    part = getattr(sysobj, "ml_part", None)
    part_ptr = None
    if part is not None:
        part = np.ascontiguousarray(part, dtype=np.int32)
        keep.append(part)
        part_ptr = part.ctypes.data_as(_i32p)
    s = ps_system(int(sysobj.n_nodes), int(sysobj.n_cells), int(sysobj.nf), int(sysobj.p_index),
                  _bsr(sysobj.Auu, keep), _bsr(sysobj.Auf, keep), _bsr(sysobj.Afu, keep), _bsr(sysobj.Aff, keep),
                  d_sp.ctypes.data_as(_f64p), d_pp.ctypes.data_as(_f64p), int(mech_key), part_ptr)
    return s, keep


def options(**kw):
    o = ps_options()
    load().ps_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


# ---------------------------------------------------------------------------- C-named calls
def ps_default_options():
    return options()


def ps_ctx_create(device=0, hbm_budget_bytes=0):
    out = C.c_void_p()
    _check(load().ps_ctx_create(device, hbm_budget_bytes, C.byref(out)), "ps_ctx_create")
    return out.value


def ps_ctx_destroy(ctx):
    load().ps_ctx_destroy(ctx)


def ps_create(ctx, sysobj, opts=None, mech_key=0):
    s, keep = make_system(sysobj, mech_key)
    out = C.c_void_p()
    _check(load().ps_create(ctx, C.byref(s), C.byref(opts) if opts is not None else None, C.byref(out)),
           "ps_create")
    return out.value


def ps_update_flow(h, afu_vals=None, aff_vals=None, d_sp=None, d_pp=None, auf_vals=None):
    arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64)
            for a in (afu_vals, aff_vals, d_sp, d_pp, auf_vals)]
    ptrs = [None if a is None else a.ctypes.data_as(_f64p) for a in arrs]
    _check(load().ps_update_flow(h, *ptrs), "ps_update_flow")


def ps_setup(h):
    _check(load().ps_setup(h), "ps_setup")


def ps_solve(h, rhs, x, rtol, stream=None, raise_on_error=False):
    """Returns the ps_result as a dict (status included)."""
    r = ps_result()
    code = load().ps_solve(h, _ptr(rhs), _ptr(x), float(rtol), _stream(stream), C.byref(r))
    if raise_on_error and code != PS_OK:
        raise PsError(code, "ps_solve")
    d = r.as_dict()
    d["status"] = code
    return d


def ps_solve_noalloc(h, rhs, x, rtol, stream=None):
    """ps_solve with the FGMRES workspace in the library's static device scratch (no
    allocation); returns the ps_result as a dict (status included)."""
    r = ps_result()
    code = load().ps_solve_noalloc(h, _ptr(rhs), _ptr(x), float(rtol), _stream(stream), C.byref(r))
    d = r.as_dict()
    d["status"] = code
    return d


def ps_apply_precond(h, v, z, stream=None):
    _check(load().ps_apply_precond(h, _ptr(v), _ptr(z), _stream(stream)), "ps_apply_precond")


def ps_spmv(h, x, y, stream=None):
    _check(load().ps_spmv(h, _ptr(x), _ptr(y), _stream(stream)), "ps_spmv")


def ps_submit(h, rhs, x, rtol, stream=None):
    t = C.c_uint64()
    _check(load().ps_submit(h, _ptr(rhs), _ptr(x), float(rtol), _stream(stream), C.byref(t)), "ps_submit")
    return t.value


def ps_poll(ctx, ticket):
    r = ps_result()
    code = load().ps_poll(ctx, ticket, C.byref(r))
    d = r.as_dict()
    d["status"] = code
    return d


def ps_wait(ctx, ticket):
    r = ps_result()
    code = load().ps_wait(ctx, ticket, C.byref(r))
    d = r.as_dict()
    d["status"] = code
    return d


def ps_ctx_batches(ctx):
    """(batched step-1 launch sequences, requests they covered) since ps_ctx_create."""
    a, b = C.c_uint64(), C.c_uint64()
    _check(load().ps_ctx_batches(ctx, C.byref(a), C.byref(b)), "ps_ctx_batches")
    return a.value, b.value


def ps_kernel_timing(enable):
    """True: bracket every instrumented kernel; False: stop; an int: ps.h's bit mask."""
    mask = PS_KT_ALL if enable is True else 0 if enable is False else int(enable)
    _check(load().ps_kernel_timing(mask), "ps_kernel_timing")


def kernel_index(name):
    """Index of an instrumented kernel by name (its bit in ps_kernel_timing's mask)."""
    return list(ps_kernel_stats()).index(name)


def ps_kernel_stats():
    """Instrumented kernel totals: {name: dict(launches, seconds, bytes)}."""
    lib = load()
    out = {}
    idx = 0
    while True:
        name = C.create_string_buffer(64)
        n, sec, b = C.c_int64(), C.c_double(), C.c_double()
        code = lib.ps_kernel_stats(idx, name, 64, C.byref(n), C.byref(sec), C.byref(b))
        if code == PS_EINVAL:
            return out
        _check(code, "ps_kernel_stats")
        out[name.value.decode()] = dict(launches=n.value, seconds=sec.value, bytes=b.value)
        idx += 1


def ps_pressure_level(h, lvl):
    """Level lvl of the handle's pressure hierarchy: dict(nlevels, n, rowptr, colind, vals, cf)."""
    lib = load()
    nl, n, nnz = C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib.ps_pressure_level(h, lvl, C.byref(nl), C.byref(n), C.byref(nnz), None, None, None, None),
           "ps_pressure_level")
    rp = np.zeros(n.value + 1, np.int32)
    ci = np.zeros(nnz.value, np.int32)
    v = np.zeros(nnz.value, np.float64)
    cf = np.zeros(n.value, np.int8)
    _check(lib.ps_pressure_level(h, lvl, None, None, None, rp.ctypes.data_as(_i32p), ci.ctypes.data_as(_i32p),
                                 v.ctypes.data_as(_f64p), cf.ctypes.data_as(C.POINTER(C.c_int8))),
           "ps_pressure_level")
    return dict(nlevels=nl.value, n=n.value, rowptr=rp, colind=ci, vals=v, cf=cf)


def ps_footprint(h):
    b = C.c_size_t()
    _check(load().ps_footprint(h, C.byref(b)), "ps_footprint")
    return b.value


def ps_destroy(h):
    load().ps_destroy(h)


def ps_strerror(code):
    return load().ps_strerror(code).decode()


def ps_last_error():
    return load().ps_last_error().decode()


# ---------------------------------------------------------------------------- host setup
class HostSetup:
    """Host-side setup phase (ps_host.h): callable without a GPU."""

    h = None

    def __init__(self, sysobj, opts=None):
        s, keep = make_system(sysobj)
        out = C.c_void_p()
        _check(load().ps_host_setup_create(C.byref(s), C.byref(opts) if opts is not None else None, C.byref(out)),
               "ps_host_setup_create")
        self.h = out.value
        self.nblocks_ff = int(np.asarray(sysobj.Aff.colind).shape[0])
        self.nf = int(sysobj.nf)

    def close(self):
        if self.h:
            load().ps_host_setup_destroy(self.h)
            self.h = None

    __del__ = close

    def levels(self, which):
        n = C.c_int32()
        _check(load().ps_host_levels(self.h, which, C.byref(n)), "ps_host_levels")
        return n.value

    def level(self, which, lvl):
        lib = load()
        n, nnz, nc, pnnz = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib.ps_host_level(self.h, which, lvl, C.byref(n), C.byref(nnz), None, None, None, None,
                                 C.byref(nc), C.byref(pnnz), None, None, None), "ps_host_level")
        rp = np.zeros(n.value + 1, np.int32)
        ci = np.zeros(nnz.value, np.int32)
        v = np.zeros(nnz.value, np.float64)
        cf = np.zeros(n.value, np.int8)
        has_p = pnnz.value > 0
        prp = np.zeros(n.value + 1, np.int32)
        pci = np.zeros(pnnz.value, np.int32)
        pv = np.zeros(pnnz.value, np.float64)
        _check(lib.ps_host_level(self.h, which, lvl, None, None, rp.ctypes.data_as(_i32p), ci.ctypes.data_as(_i32p),
                                 v.ctypes.data_as(_f64p), cf.ctypes.data_as(C.POINTER(C.c_int8)), None, None,
                                 prp.ctypes.data_as(_i32p), pci.ctypes.data_as(_i32p), pv.ctypes.data_as(_f64p)),
               "ps_host_level")
        out = dict(n=n.value, rowptr=rp, colind=ci, vals=v, cf=cf)
        if has_p:
            out.update(nc=nc.value, p_rowptr=prp, p_colind=pci, p_vals=pv)
        return out

    def lam(self, which, lvl):
        x = C.c_double()
        _check(load().ps_host_level_lambda(self.h, which, lvl, C.byref(x)), "ps_host_level_lambda")
        return x.value

    def spp(self):
        v = np.zeros(self.nblocks_ff, np.float64)
        _check(load().ps_host_spp(self.h, v.ctypes.data_as(_f64p)), "ps_host_spp")
        return v

    def bilu(self):
        v = np.zeros((self.nblocks_ff, self.nf, self.nf), np.float64)
        _check(load().ps_host_bilu(self.h, v.ctypes.data_as(_f64p)), "ps_host_bilu")
        return v

    def bilu_levels(self):
        f, b = C.c_int32(), C.c_int32()
        _check(load().ps_host_bilu_levels(self.h, C.byref(f), C.byref(b)), "ps_host_bilu_levels")
        return f.value, b.value


# ---------------------------------------------------------------------------- convenience
class Solver:
    """One handle: a system, its setup and its solves."""

    def __init__(self, ctx, sysobj, mech_key=0, **opts):
        self.ctx = ctx
        self.opts = options(**opts)
        self.h = ps_create(ctx, sysobj, self.opts, mech_key=mech_key)
        self.N = 3 * int(sysobj.n_nodes) + int(sysobj.nf) * int(sysobj.n_cells)

    def setup(self):
        ps_setup(self.h)

    def solve(self, rhs, x, rtol=1e-8, stream=None):
        return ps_solve(self.h, rhs, x, rtol, stream)

    def apply_precond(self, v, z, stream=None):
        ps_apply_precond(self.h, v, z, stream)

    def spmv(self, x, y, stream=None):
        ps_spmv(self.h, x, y, stream)

    def submit(self, rhs, x, rtol=1e-8, stream=None):
        return ps_submit(self.h, rhs, x, rtol, stream)

    def footprint(self):
        return ps_footprint(self.h)

    def pressure_level(self, lvl):
        return ps_pressure_level(self.h, lvl)

    def close(self):
        if self.h:
            ps_destroy(self.h)
            self.h = None
