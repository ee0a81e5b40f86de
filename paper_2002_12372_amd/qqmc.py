"""Python binding of libqqmc (argument marshalling only).

Every function wraps the C entry point of the same name in ``include/qqmc.h``;
all arithmetic runs in the library's HIP kernels.  PyTorch supplies device
buffers (``tensor.data_ptr()``) and streams (``torch.cuda.current_stream()``)
and nothing else.  Importing this module does not build anything: if
``libqqmc.so`` is missing the first call raises, it never falls back to
other code.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqqmc.so")

OK, PENDING = 0, 1
EINVAL, ENOMEM, EDEVICE, EADMIT, ENOTICKET = -1, -2, -3, -4, -5
MODE_CHARGE, MODE_MODEL, MODE_CONSTANT, MODE_CURRENT = 0, 1, 2, 3
OBS_CHARGE, OBS_CURRENT = 0, 1
METHOD_TREE, METHOD_DIRECT = 0, 1
MAX_ORDER = 14


class QQMCError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("qqmc status %d: %s" % (status, msg))
        self.status = status


class qqmc_dot(ctypes.Structure):
    _fields_ = [("eps_d", ctypes.c_double), ("gamma", ctypes.c_double),
                ("beta", ctypes.c_double), ("bias_v", ctypes.c_double),
                ("t_half", ctypes.c_double), ("n_grid", ctypes.c_int32),
                ("half_bandwidth", ctypes.c_double), ("lead", ctypes.c_int32)]


class qqmc_order(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("log2_n", ctypes.c_int32),
                ("lattice_a", ctypes.c_uint64), ("n_shifts", ctypes.c_int32),
                ("shifts", ctypes.POINTER(ctypes.c_double)),
                ("model_tau", ctypes.c_double), ("t_meas", ctypes.c_double),
                ("mode", ctypes.c_int32), ("model", ctypes.c_void_p),
                ("alpha", ctypes.c_double),
                ("sobol_v", ctypes.POINTER(ctypes.c_uint32)),
                ("sobol_shifts", ctypes.POINTER(ctypes.c_uint32))]


class qqmc_learn_params(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("log2_m", ctypes.c_int32),
                ("lattice_a", ctypes.c_uint64), ("shift", ctypes.POINTER(ctypes.c_double)),
                ("model_tau", ctypes.c_double), ("t_meas", ctypes.c_double),
                ("n_bins", ctypes.c_int32), ("lam", ctypes.c_double),
                ("floor_eps", ctypes.c_double), ("alpha", ctypes.c_double),
                ("sobol_v", ctypes.POINTER(ctypes.c_uint32)),
                ("sobol_shift", ctypes.POINTER(ctypes.c_uint32))]


class qqmc_batch_item(ctypes.Structure):
    _fields_ = [("tables", ctypes.c_void_p), ("order", qqmc_order)]


_lib = None

# (name, restype, argtypes) of every exported symbol of include/qqmc.h
_P = ctypes.POINTER
_d, _i32, _i64, _u64, _vp = (ctypes.c_double, ctypes.c_int32, ctypes.c_int64,
                             ctypes.c_uint64, ctypes.c_void_p)
_PD = _P(ctypes.c_double)
SIGNATURES = [
    ("qqmc_make_tables", _i32, [_P(qqmc_dot), _vp, _P(_vp)]),
    ("qqmc_tables_compute_host", _i32, [_P(qqmc_dot), _PD, _PD, _PD]),
    ("qqmc_tables_from_host", _i32, [_PD, _PD, _i32, _d, _d, _vp, _P(_vp)]),
    ("qqmc_tables_export", _i32, [_vp, _PD, _PD, _PD]),
    ("qqmc_tables_info", _i32, [_vp, _P(_i32), _PD]),
    ("qqmc_free_tables", None, [_vp]),
    ("qqmc_eval_order", _i32, [_vp, _P(qqmc_order), _vp, _PD, _PD, _PD]),
    ("qqmc_eval_order_async", _i32, [_vp, _P(qqmc_order), _i32, _vp, _vp, _vp, _P(_i64)]),
    ("qqmc_eval_order_noalloc", _i32, [_vp, _P(qqmc_order), _i32, _vp, _vp, _P(_i64)]),
    ("qqmc_eval_points", _i32, [_vp, _i32, _d, _d, _i32, _vp, _i64, _i32, _vp, _vp, _vp]),
    ("qqmc_lead_tables_compute_host", _i32, [_P(qqmc_dot), _PD, _PD]),
    ("qqmc_tables_lead_from_host", _i32, [_vp, _PD, _PD]),
    ("qqmc_plan_create", _i32, [_P(qqmc_batch_item), _i32, _i32, _i32, _vp, _P(_vp)]),
    ("qqmc_plan_run", _i32, [_vp, _vp]),
    ("qqmc_plan_results", _i32, [_vp, _vp, _PD]),
    ("qqmc_plan_info", _i32, [_vp, _P(_i64), _P(_i64), _P(_i32), _P(_i32), _P(_i32), _P(_i32)]),
    ("qqmc_plan_set_geometry", _i32, [_vp, _i32, _i32, _i32]),
    ("qqmc_plan_destroy", None, [_vp]),
    ("qqmc_server_create", _i32, [ctypes.c_size_t, _i32, _i32, _P(_vp)]),
    ("qqmc_submit", _i32, [_vp, _P(qqmc_dot), _P(qqmc_order), _P(_u64)]),
    ("qqmc_poll", _i32, [_vp, _u64, _PD, _PD, _PD, _PD, _PD]),
    ("qqmc_server_now", _d, [_vp]),
    ("qqmc_server_drain", _i32, [_vp]),
    ("qqmc_server_destroy", None, [_vp]),
    ("qqmc_learn_model", _i32, [_vp, _P(qqmc_learn_params), _vp, _P(_vp)]),
    ("qqmc_model_from_host", _i32, [_i32, _i32, _PD, _vp, _P(_vp)]),
    ("qqmc_model_export", _i32, [_vp, _P(_i32), _P(_i32), _PD, _PD]),
    ("qqmc_free_model", None, [_vp]),
    ("qqmc_last_error", ctypes.c_char_p, []),
]


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libqqmc.so is not built (run __graft_entry__.build())")
        l = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(l, name)
            f.restype = res
            f.argtypes = args
        _lib = l
    return _lib


def last_error():
    return lib().qqmc_last_error().decode()


def _check(st):
    if st < 0:
        raise QQMCError(st, last_error())
    return st


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _pd(a):
    return a.ctypes.data_as(_PD)


class Tables:
    """Owning wrapper of a qqmc_tables handle."""

    def __init__(self, handle, n_grid, t_half):
        self.handle = ctypes.c_void_p(handle)
        self.n_grid, self.t_half = n_grid, t_half

    def __del__(self):
        if getattr(self, "handle", None) and self.handle.value and _lib is not None:
            _lib.qqmc_free_tables(self.handle)
            self.handle = None


def make_dot(d):
    return qqmc_dot(d.eps_d, d.gamma, d.beta, d.bias_v, d.t_half, d.n_grid,
                    getattr(d, "half_bandwidth", 0.0), getattr(d, "lead", 0))


def make_tables(dot, stream=None):
    """dot: qqmc_inputs.Dot (or anything with the same fields)."""
    h = ctypes.c_void_p()
    cd = make_dot(dot)
    _check(lib().qqmc_make_tables(ctypes.byref(cd), _stream(stream), ctypes.byref(h)))
    return Tables(h.value, dot.n_grid, dot.t_half)


def lead_tables_compute_host(dot):
    """(cl, cg): the lead's gamma g^<_{0i}, gamma g^>_{0i} on the dot's grid
    (dot.lead = 1 or 2, finite band), computed on the host."""
    cd = make_dot(dot)
    cl = np.zeros(2 * dot.n_grid)
    cg = np.zeros(2 * dot.n_grid)
    _check(lib().qqmc_lead_tables_compute_host(ctypes.byref(cd), _pd(cl), _pd(cg)))
    return cl, cg


def tables_lead_from_host(tables, cl, cg):
    cl = np.ascontiguousarray(cl, dtype=np.float64)
    cg = np.ascontiguousarray(cg, dtype=np.float64)
    _check(lib().qqmc_tables_lead_from_host(tables.handle, _pd(cl), _pd(cg)))


def tables_compute_host(dot):
    """(gl, gg, n_sigma) computed on the host, no GPU involved."""
    gl = np.zeros(2 * dot.n_grid)
    gg = np.zeros(2 * dot.n_grid)
    ns = ctypes.c_double()
    cd = make_dot(dot)
    _check(lib().qqmc_tables_compute_host(ctypes.byref(cd), _pd(gl), _pd(gg), ctypes.byref(ns)))
    return gl, gg, ns.value


def tables_from_host(gl, gg, n_grid, t_half, n_sigma, stream=None):
    gl = np.ascontiguousarray(gl, dtype=np.float64)
    gg = np.ascontiguousarray(gg, dtype=np.float64)
    h = ctypes.c_void_p()
    _check(lib().qqmc_tables_from_host(_pd(gl), _pd(gg), int(n_grid), float(t_half),
                                       float(n_sigma), _stream(stream), ctypes.byref(h)))
    return Tables(h.value, n_grid, t_half)


def tables_export(tables):
    gl = np.zeros(2 * tables.n_grid)
    gg = np.zeros(2 * tables.n_grid)
    ns = ctypes.c_double()
    _check(lib().qqmc_tables_export(tables.handle, _pd(gl), _pd(gg), ctypes.byref(ns)))
    return gl, gg, ns.value


def make_order(job, t_meas, model=None):
    """job: qqmc_inputs.OrderJob; model: a Model of the same order or None.
    The returned struct keeps the shift array alive through ``_keep``."""
    sh = np.ascontiguousarray(job.shifts, dtype=np.float64)
    sv = getattr(job, "sobol_v", None)
    pv = ps = ss = None
    if sv is not None:
        sv = np.ascontiguousarray(sv, dtype=np.uint32)
        ss = np.ascontiguousarray(job.sobol_shifts, dtype=np.uint32)
        pv = sv.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
        ps = ss.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
    o = qqmc_order(job.order, job.log2_n, job.lattice_a, sh.shape[0], _pd(sh),
                   job.model_tau, t_meas, job.mode,
                   model.handle if model is not None else None, job.alpha, pv, ps)
    o._keep = (sh, model, sv, None if sv is None else ss)
    return o


class Model:
    """Learned second warp (App. I): per-coordinate CDFs at the bin edges."""

    def __init__(self, handle):
        self.handle = ctypes.c_void_p(handle)

    def export(self):
        """(cdf, hist) numpy arrays, shapes (order, n_bins + 1), (order, n_bins)."""
        n, nb = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().qqmc_model_export(self.handle, ctypes.byref(n), ctypes.byref(nb), None, None))
        cdf = np.zeros((n.value, nb.value + 1))
        hist = np.zeros((n.value, nb.value))
        _check(lib().qqmc_model_export(self.handle, None, None, _pd(cdf), _pd(hist)))
        return cdf, hist

    def close(self):
        if self.handle:
            lib().qqmc_free_model(self.handle)
            self.handle = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def learn_model(tables, order, log2_m, lattice_a, shift, model_tau, t_meas, n_bins=100,
                lam=0.05, floor_eps=1e-3, stream=None, alpha=0.0, sobol_v=None,
                sobol_shift=None):
    """Learning pass over one shifted lattice (lattice_a, shift), or over
    Sobol' points (sobol_v: order x 32 direction numbers, sobol_shift: order
    words; lattice_a and shift are then ignored)."""
    sh = np.ascontiguousarray(np.asarray(shift if shift is not None else np.zeros(order),
                                         dtype=np.float64).reshape(order))
    pv = ps = None
    if sobol_v is not None:
        sobol_v = np.ascontiguousarray(sobol_v, dtype=np.uint32).reshape(order, 32)
        sobol_shift = np.ascontiguousarray(sobol_shift, dtype=np.uint32).reshape(order)
        pv = sobol_v.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
        ps = sobol_shift.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
    p = qqmc_learn_params(order, log2_m, lattice_a, _pd(sh), model_tau, t_meas, n_bins,
                          lam, floor_eps, alpha, pv, ps)
    h = ctypes.c_void_p()
    _check(lib().qqmc_learn_model(tables.handle, ctypes.byref(p), _stream(stream),
                                  ctypes.byref(h)))
    return Model(h.value)


def model_from_host(cdf, stream=None):
    cdf = np.ascontiguousarray(cdf, dtype=np.float64)
    h = ctypes.c_void_p()
    _check(lib().qqmc_model_from_host(cdf.shape[0], cdf.shape[1] - 1, _pd(cdf),
                                      _stream(stream), ctypes.byref(h)))
    return Model(h.value)


def eval_order(tables, job, t_meas, stream=None, model=None):
    """(q_shift complex[K], q_mean complex, q_stderr float)."""
    o = make_order(job, t_meas, model)
    K = o.n_shifts
    q = np.zeros(2 * K)
    m = np.zeros(2)
    se = ctypes.c_double()
    _check(lib().qqmc_eval_order(tables.handle, ctypes.byref(o), _stream(stream), _pd(q),
                                 _pd(m), ctypes.byref(se)))
    return q[0::2] + 1j * q[1::2], m[0] + 1j * m[1], se.value


def eval_order_async(tables, job, t_meas, shift_sums, tile_sums=None, tile_len=0, stream=None,
                     model=None):
    """shift_sums / tile_sums: float64 CUDA tensors (2*K, 2*n_tiles)."""
    o = make_order(job, t_meas, model)
    nt = ctypes.c_int64()
    _check(lib().qqmc_eval_order_async(
        tables.handle, ctypes.byref(o), int(tile_len), _stream(stream),
        ctypes.c_void_p(tile_sums.data_ptr() if tile_sums is not None else 0),
        ctypes.c_void_p(shift_sums.data_ptr()), ctypes.byref(nt)))
    return nt.value


def eval_order_noalloc(tables, job, t_meas, shift_sums, tile_len=0, stream=None, model=None):
    """qqmc_eval_order_noalloc: the per-shift sums of eval_order_async into
    shift_sums (float64 CUDA tensor, 2*K), with no device allocation (the
    library's static per-device scratch).  Returns the number of tiles."""
    o = make_order(job, t_meas, model)
    nt = ctypes.c_int64()
    _check(lib().qqmc_eval_order_noalloc(
        tables.handle, ctypes.byref(o), int(tile_len), _stream(stream),
        ctypes.c_void_p(shift_sums.data_ptr()), ctypes.byref(nt)))
    return nt.value


def n_tiles(job, tile_len):
    return job.shifts.shape[0] * ((1 << job.log2_n) // tile_len)


def eval_points(tables, order, t_meas, u, f, method=METHOD_TREE, stream=None, alpha=0.0,
                current=False, mass=None):
    """u: (P, order) float64 CUDA tensor; f: (P, 2) float64 CUDA tensor;
    mass: (P,) float64 CUDA tensor or None (direct method only)."""
    P = u.shape[0]
    assert u.dtype.is_floating_point and u.is_contiguous() and f.is_contiguous()
    assert f.numel() >= 2 * P and u.numel() == P * order
    if mass is not None:
        assert mass.is_contiguous() and mass.numel() >= P
    _check(lib().qqmc_eval_points(tables.handle, int(order), float(t_meas), float(alpha),
                                  OBS_CURRENT if current else OBS_CHARGE,
                                  ctypes.c_void_p(u.data_ptr()), P, int(method),
                                  ctypes.c_void_p(f.data_ptr()),
                                  ctypes.c_void_p(mass.data_ptr() if mass is not None else 0),
                                  _stream(stream)))


class Plan:
    def __init__(self, handle, items, n_shifts):
        self.handle = ctypes.c_void_p(handle)
        self._items = items
        self.n_shifts = n_shifts

    def __del__(self):
        if getattr(self, "handle", None) and self.handle.value and _lib is not None:
            _lib.qqmc_plan_destroy(self.handle)
            self.handle = None


def plan_create(entries, t_meas, tile_len=0, grid_blocks=0, stream=None):
    """entries: list of (Tables, OrderJob) or (Tables, OrderJob, Model)."""
    arr = (qqmc_batch_item * len(entries))()
    keep = []
    for k, entry in enumerate(entries):
        tb, job = entry[0], entry[1]
        o = make_order(job, t_meas, entry[2] if len(entry) > 2 else None)
        keep.append((tb, o))
        arr[k].tables = tb.handle
        arr[k].order = o
    h = ctypes.c_void_p()
    _check(lib().qqmc_plan_create(arr, len(entries), int(tile_len), int(grid_blocks),
                                  _stream(stream), ctypes.byref(h)))
    return Plan(h.value, keep, [e[1].shifts.shape[0] for e in entries])


def plan_run(plan, stream=None):
    _check(lib().qqmc_plan_run(plan.handle, _stream(stream)))


def plan_results(plan, stream=None):
    tot = sum(plan.n_shifts)
    q = np.zeros(2 * tot)
    _check(lib().qqmc_plan_results(plan.handle, _stream(stream), _pd(q)))
    qc = q[0::2] + 1j * q[1::2]
    out, b = [], 0
    for k in plan.n_shifts:
        out.append(qc[b:b + k])
        b += k
    return out


def plan_info(plan):
    """Tile count, points, tile length, workgroups and, per order n present,
    the lane mapping geometry[n] = (lanes per item, cooperative top levels)."""
    nt, npnt, tl, gb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
    lanes = (ctypes.c_int32 * MAX_ORDER)()
    top = (ctypes.c_int32 * MAX_ORDER)()
    _check(lib().qqmc_plan_info(plan.handle, ctypes.byref(nt), ctypes.byref(npnt),
                                ctypes.byref(tl), ctypes.byref(gb), lanes, top))
    return dict(n_tiles=nt.value, n_points=npnt.value, tile_len=tl.value, grid_blocks=gb.value,
                geometry={n + 1: (lanes[n], top[n]) for n in range(MAX_ORDER) if lanes[n]})


def plan_set_geometry(plan, order, lanes_per_item, top_levels):
    """Selects the lane mapping (lanes per item, cooperative top levels) of
    the plan's scalar-tree charge group of this order."""
    _check(lib().qqmc_plan_set_geometry(plan.handle, int(order), int(lanes_per_item),
                                        int(top_levels)))


class Server:
    def __init__(self, hbm_budget_bytes, max_slots, batch_tiles=0):
        h = ctypes.c_void_p()
        _check(lib().qqmc_server_create(int(hbm_budget_bytes), int(max_slots), int(batch_tiles),
                                        ctypes.byref(h)))
        self.handle = h
        self._n_shifts = {}

    def submit(self, dot, job, t_meas, model=None):
        """model (optional) is kept alive here until the request is polled done."""
        cd = make_dot(dot)
        o = make_order(job, t_meas, model)
        t = ctypes.c_uint64()
        _check(lib().qqmc_submit(self.handle, ctypes.byref(cd), ctypes.byref(o), ctypes.byref(t)))
        self._n_shifts[t.value] = (o.n_shifts, model)
        return t.value

    def poll(self, ticket):
        """None while pending; else dict(q_shift, q_mean, q_stderr, t_submit, t_done)."""
        K = self._n_shifts.get(ticket, (1, None))[0]
        q = np.zeros(2 * K)
        m = np.zeros(2)
        se, ts, td = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        st = lib().qqmc_poll(self.handle, ctypes.c_uint64(ticket), _pd(q), _pd(m),
                             ctypes.byref(se), ctypes.byref(ts), ctypes.byref(td))
        if st == PENDING:
            return None
        _check(st)
        self._n_shifts.pop(ticket, None)
        return dict(q_shift=q[0::2] + 1j * q[1::2], q_mean=m[0] + 1j * m[1],
                    q_stderr=se.value, t_submit=ts.value, t_done=td.value)

    def now(self):
        return lib().qqmc_server_now(self.handle)

    def drain(self):
        _check(lib().qqmc_server_drain(self.handle))

    def close(self):
        if self.handle and self.handle.value:
            lib().qqmc_server_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
