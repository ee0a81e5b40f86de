"""CPU FP64 oracle for the QQMC charge integrand (arXiv:2002.12372).

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, by ``__graft_entry__.smoke``
and by the ``cpu_baseline`` leg of ``bench.py``; the product package never
imports it.  The arithmetic lives in ``qqmc_oracle.c`` (plain C, one LU per
determinant, all 2^n Keldysh index vectors enumerated); this module only
marshals numpy arrays through ctypes.

Every entry point mirrors a function of ``qqmc_oracle.h``; see that header for
the passages of the paper each one writes out.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(verbose=False):
    """Compile ``liboracle.so`` with gcc (C11, OpenMP, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-fno-fast-math", "-ffp-contract=off", "-Wall", "-Wextra",
           os.path.join(_HERE, "qqmc_oracle.c"), "-o", LIB_PATH + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    lib = ctypes.CDLL(LIB_PATH)
    d, i, i64, u64 = ctypes.c_double, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64
    P = ctypes.POINTER(ctypes.c_double)
    PI = ctypes.POINTER(ctypes.c_int)
    lib.oracle_tables.argtypes = [d, d, d, d, i, d, P, P, P]
    lib.oracle_tables.restype = i
    lib.oracle_n_sigma.argtypes = [d, d, d, d]
    lib.oracle_n_sigma.restype = d
    lib.oracle_gf_direct.argtypes = [d, d, d, d, d, P]
    lib.oracle_n_sigma_band.argtypes = [d, d, d, d, d]
    lib.oracle_n_sigma_band.restype = d
    lib.oracle_gf_band.argtypes = [d, d, d, d, d, d, P]
    lib.oracle_tables_band.argtypes = [d, d, d, d, d, i, d, P, P, P]
    lib.oracle_tables_band.restype = i
    lib.oracle_gf_lead.argtypes = [d, d, d, d, d, i, d, P]
    lib.oracle_lead_tables.argtypes = [d, d, d, d, d, i, i, d, P, P]
    lib.oracle_lead_tables.restype = i
    lib.oracle_keldysh_sum_lead.argtypes = [P, P, P, P, i, d, d, d, d, i, P, P, P]
    lib.oracle_eval_sums_lead.argtypes = [P, P, P, P, i, d, d, d, d, i, i, u64, i, P, d,
                                          i64, i64, i, P, P]
    lib.oracle_eval_sums_lead.restype = i
    PU = ctypes.POINTER(ctypes.c_uint32)
    lib.oracle_sobol_point.argtypes = [u64, i, PU, PU, P]
    lib.oracle_eval_sums_sobol.argtypes = [P, P, i, d, d, d, d, i, PU, i, PU, d, P, i, i,
                                           i64, i64, i, P]
    lib.oracle_eval_sums_sobol.restype = i
    lib.oracle_interp.argtypes = [P, i, d, d, P]
    lib.oracle_det.argtypes = [i, P, P]
    lib.oracle_wick_matrix.argtypes = [P, P, i, d, d, d, d, i, P, PI, P]
    lib.oracle_keldysh_sum.argtypes = [P, P, i, d, d, d, d, i, P, P, P]
    lib.oracle_lattice_point.argtypes = [u64, i, i, u64, P, P]
    lib.oracle_warp.argtypes = [i, P, d, d, P, P]
    lib.oracle_warp.restype = i
    lib.oracle_eval_sums.argtypes = [P, P, i, d, d, d, d, i, i, u64, i, P, d, i,
                                     i64, i64, i, P]
    lib.oracle_eval_sums.restype = i
    lib.oracle_eval_mass.argtypes = [P, P, i, d, d, d, d, i, i, u64, i, P, d, i64, i64, i, P]
    lib.oracle_eval_mass.restype = i
    lib.oracle_max_threads.restype = i
    lib.oracle_eval_sums_model.argtypes = [P, P, i, d, d, d, d, i, i, u64, i, P, d, P, i, i,
                                           i64, i64, i, P]
    lib.oracle_eval_sums_model.restype = i
    lib.oracle_learn_model.argtypes = [P, P, i, d, d, d, d, i, i, u64, P, d, i, d, d, i, P, P]
    lib.oracle_learn_model.restype = i
    lib.oracle_learn_model_sobol.argtypes = [P, P, i, d, d, d, d, i, i, PU, PU, d, i, d, d, i,
                                             P, P]
    lib.oracle_learn_model_sobol.restype = i
    lib.oracle_model_from_hist.argtypes = [i, i, P, d, d, P]
    lib.oracle_model_from_hist.restype = i
    lib.oracle_model_inverse.argtypes = [P, i, d, P]
    lib.oracle_model_inverse.restype = d
    _lib = lib
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Tables:
    """g^<, g^> on the uniform grid plus the exact n_sigma (App. E); wide
    band, or semicircular leads of half-bandwidth D when D > 0."""

    def __init__(self, eps_d, gamma, beta, bias_v, n_grid=8192, t_half=10.0,
                 half_bandwidth=0.0, lead=0):
        lib = _load()
        self.eps_d, self.gamma, self.beta, self.bias_v = eps_d, gamma, beta, bias_v
        self.half_bandwidth = float(half_bandwidth)
        self.n_grid, self.t_half = int(n_grid), float(t_half)
        self.gl = np.zeros(2 * self.n_grid)
        self.gg = np.zeros(2 * self.n_grid)
        ns = ctypes.c_double()
        if self.half_bandwidth > 0.0:
            rc = lib.oracle_tables_band(eps_d, gamma, beta, bias_v, self.half_bandwidth,
                                        self.n_grid, self.t_half, _p(self.gl), _p(self.gg),
                                        ctypes.byref(ns))
        else:
            rc = lib.oracle_tables(eps_d, gamma, beta, bias_v, self.n_grid,
                                   self.t_half, _p(self.gl), _p(self.gg),
                                   ctypes.byref(ns))
        if rc != 0:
            raise ValueError("oracle_tables: bad arguments")
        self.n_sigma = ns.value
        # current into lead 1 (mu = -V/2) or 2 (mu = +V/2): the lead's
        # gamma g^<_{0i}, gamma g^>_{0i} on the same grid (finite band only)
        self.lead = int(lead)
        self.cl = self.cg = None
        if self.lead:
            self.cl = np.zeros(2 * self.n_grid)
            self.cg = np.zeros(2 * self.n_grid)
            rc = lib.oracle_lead_tables(eps_d, gamma, beta, bias_v, self.half_bandwidth,
                                        self.lead, self.n_grid, self.t_half, _p(self.cl),
                                        _p(self.cg))
            if rc != 0:
                raise ValueError("oracle_lead_tables: bad arguments (finite band, lead 1 or 2)")

    @property
    def grid(self):
        h = 2.0 * self.t_half / (self.n_grid - 1)
        return -self.t_half + np.arange(self.n_grid) * h

    def gl_c(self):
        return self.gl[0::2] + 1j * self.gl[1::2]

    def gg_c(self):
        return self.gg[0::2] + 1j * self.gg[1::2]

    def interp(self, which, tau):
        tab = self.gl if which == "<" else self.gg
        out = np.zeros(2)
        _load().oracle_interp(_p(tab), self.n_grid, self.t_half, float(tau), _p(out))
        return out[0] + 1j * out[1]

    def _args(self, alpha=0.0):
        """Table arguments of the C functions; alpha shifts every vertex
        diagonal by -i alpha (App. E)."""
        return (_p(self.gl), _p(self.gg), self.n_grid, self.t_half, self.n_sigma, float(alpha))


def n_sigma(eps_d, gamma, beta, bias_v):
    return _load().oracle_n_sigma(eps_d, gamma, beta, bias_v)


def gf_band(eps_d, gamma, beta, bias_v, D, tau):
    """(g^<(tau), g^>(tau)) with semicircular leads of half-bandwidth D."""
    out = np.zeros(4)
    _load().oracle_gf_band(eps_d, gamma, beta, bias_v, D, tau, _p(out))
    return out[0] + 1j * out[1], out[2] + 1j * out[3]


def gf_lead(eps_d, gamma, beta, bias_v, D, lead, tau):
    """(gamma g^<_{0i}(tau), gamma g^>_{0i}(tau)) for lead i (finite band)."""
    out = np.zeros(4)
    _load().oracle_gf_lead(eps_d, gamma, beta, bias_v, D, int(lead), float(tau), _p(out))
    return out[0] + 1j * out[1], out[2] + 1j * out[3]


def current_integrand(tables, t_meas, u, alpha=0.0):
    """f^I_n(u) = -4 i^n S(u) with the measurement column from the lead's
    tables (Re: the order-n integrand of the particle current into the
    lead), and 4 M(u)."""
    u = _f64(u)
    n = u.shape[0]
    S = np.zeros(2)
    M = ctypes.c_double()
    gl, gg, ng, th, ns, a = tables._args(alpha)
    _load().oracle_keldysh_sum_lead(gl, gg, _p(tables.cl), _p(tables.cg), ng, th, ns, a,
                                    t_meas, n, _p(u), _p(S), ctypes.byref(M))
    return -4.0 * (1j ** n) * (S[0] + 1j * S[1]), 4.0 * M.value


def eval_current(tables, t_meas, n, log2_n, lattice_a, shifts, model_tau, i_begin=0,
                 i_end=None, n_threads=0, alpha=0.0):
    """Per-shift sums of f^I W over lattice indices [i_begin, i_end) and the
    per-shift term masses."""
    shifts = _f64(shifts)
    K = shifts.shape[0]
    if i_end is None:
        i_end = 1 << log2_n
    sums = np.zeros(2 * K)
    mass = np.zeros(K)
    gl, gg, ng, th, ns, a = tables._args(alpha)
    rc = _load().oracle_eval_sums_lead(gl, gg, _p(tables.cl), _p(tables.cg), ng, th, ns, a,
                                       t_meas, n, log2_n, int(lattice_a), K, _p(shifts),
                                       model_tau, int(i_begin), int(i_end), n_threads,
                                       _p(sums), _p(mass))
    if rc != 0:
        raise ValueError("oracle_eval_sums_lead: bad arguments")
    return sums[0::2] + 1j * sums[1::2], mass


def eval_order_current(tables, t_meas, n, log2_n, lattice_a, shifts, model_tau, alpha=0.0):
    """I^{(s)} per shift (complex; the real part is the current coefficient),
    their mean, the standard error of the real parts, and the mean term mass
    per lattice point."""
    N = 1 << log2_n
    sums, mass = eval_current(tables, t_meas, n, log2_n, lattice_a, shifts, model_tau,
                              alpha=alpha)
    q = sums / N
    K = q.shape[0]
    se = float(np.std(q.real, ddof=1) / np.sqrt(K)) if K > 1 else float("nan")
    return q, q.mean(), se, mass / N


def _pu(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def sobol_point(i, V, dshift=None):
    """Sobol' point i (App. B) from direction numbers V (n x 32 uint32) and
    an optional digital shift (n uint32)."""
    V = np.ascontiguousarray(V, dtype=np.uint32)
    n = V.shape[0]
    x = np.zeros(n)
    ds = None if dshift is None else np.ascontiguousarray(dshift, dtype=np.uint32)
    _load().oracle_sobol_point(int(i), n, _pu(V), _pu(ds) if ds is not None else None, _p(x))
    return x


def _cdf_arg(cdf, n):
    if cdf is None:
        return None, 0
    cdf = _f64(cdf)
    assert cdf.ndim == 2 and cdf.shape[0] == n
    return cdf, cdf.shape[1] - 1


def eval_sums_sobol(tables, t_meas, n, V, dshifts, model_tau, i_begin, i_end, mode=0,
                    alpha=0.0, n_threads=0, cdf=None):
    """Per-shift sums of fbar W over Sobol' indices [i_begin, i_end)
    (cdf: the learned second warp, (n, n_bins + 1), or None)."""
    V = np.ascontiguousarray(V, dtype=np.uint32)
    dshifts = np.ascontiguousarray(dshifts, dtype=np.uint32)
    K = dshifts.shape[0]
    sums = np.zeros(2 * K)
    cdf, nb = _cdf_arg(cdf, n)
    rc = _load().oracle_eval_sums_sobol(*tables._args(alpha), t_meas, n, _pu(V), K,
                                        _pu(dshifts), model_tau,
                                        _p(cdf) if cdf is not None else None, nb, mode,
                                        int(i_begin), int(i_end), n_threads, _p(sums))
    if rc != 0:
        raise ValueError("oracle_eval_sums_sobol: bad arguments")
    return sums[0::2] + 1j * sums[1::2]


def eval_order_sobol(tables, t_meas, n, log2_n, V, dshifts, model_tau, mode=0, alpha=0.0,
                     n_threads=0, cdf=None):
    """Q^{(s)} over the first 2^log2_n Sobol' points, one digital shift per
    row of dshifts; their mean and standard error (cdf as in
    eval_sums_sobol)."""
    V = np.ascontiguousarray(V, dtype=np.uint32)
    dshifts = np.ascontiguousarray(dshifts, dtype=np.uint32)
    K = dshifts.shape[0]
    assert V.shape == (n, 32) and dshifts.shape == (K, n)
    sums = np.zeros(2 * K)
    N = 1 << log2_n
    cdf, nb = _cdf_arg(cdf, n)
    rc = _load().oracle_eval_sums_sobol(*tables._args(alpha), t_meas, n, _pu(V), K,
                                        _pu(dshifts), model_tau,
                                        _p(cdf) if cdf is not None else None, nb, mode, 0, N,
                                        n_threads, _p(sums))
    if rc != 0:
        raise ValueError("oracle_eval_sums_sobol: bad arguments")
    q = (sums[0::2] + 1j * sums[1::2]) / N
    se = float(np.std(q.real, ddof=1) / np.sqrt(K)) if K > 1 else float("nan")
    return q, q.mean(), se


def n_sigma_band(eps_d, gamma, beta, bias_v, D):
    return _load().oracle_n_sigma_band(eps_d, gamma, beta, bias_v, D)


def gf_direct(eps_d, gamma, beta, bias_v, tau):
    out = np.zeros(4)
    _load().oracle_gf_direct(eps_d, gamma, beta, bias_v, float(tau), _p(out))
    return out[0] + 1j * out[1], out[2] + 1j * out[3]


def det(mat):
    mat = np.asarray(mat, dtype=np.complex128)
    m = mat.shape[0]
    a = _f64(np.stack([mat.real, mat.imag], axis=-1).reshape(-1))
    out = np.zeros(2)
    _load().oracle_det(m, _p(a), _p(out))
    return out[0] + 1j * out[1]


def wick_matrix(tables, t_meas, u, a, alpha=0.0):
    u = _f64(u)
    n = u.shape[0]
    av = np.ascontiguousarray(a, dtype=np.int32)
    out = np.zeros(2 * (n + 1) ** 2)
    _load().oracle_wick_matrix(*tables._args(alpha), t_meas, n, _p(u),
                               av.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                               _p(out))
    c = out[0::2] + 1j * out[1::2]
    return c.reshape(n + 1, n + 1)


def keldysh_sum(tables, t_meas, u, alpha=0.0):
    """S(u) and the term mass M(u) for one point u = (u_1..u_n)."""
    u = _f64(u)
    S = np.zeros(2)
    M = ctypes.c_double()
    _load().oracle_keldysh_sum(*tables._args(alpha), t_meas, u.shape[0], _p(u),
                               _p(S), ctypes.byref(M))
    return S[0] + 1j * S[1], M.value


def integrand(tables, t_meas, u, alpha=0.0):
    """f_n(u) = -2 i^{n+1} S(u): integrand of Q_n over the ordered simplex."""
    S, M = keldysh_sum(tables, t_meas, u, alpha)
    n = len(u)
    return -2.0 * (1j ** (n + 1)) * S, 2.0 * M


def lattice_point(i, n, log2_n, lattice_a, shift):
    x = np.zeros(n)
    sh = _f64(shift)
    _load().oracle_lattice_point(int(i), n, log2_n, int(lattice_a), _p(sh), _p(x))
    return x


def warp(x, model_tau, t_meas):
    x = _f64(x)
    u = np.zeros(x.shape[0])
    W = ctypes.c_double()
    inside = _load().oracle_warp(x.shape[0], _p(x), model_tau, t_meas, _p(u),
                                 ctypes.byref(W))
    return u, W.value, bool(inside)


def eval_sums(tables, t_meas, n, log2_n, lattice_a, shifts, model_tau, mode=0,
              i_begin=0, i_end=None, n_threads=0, cdf=None, alpha=0.0):
    """Per-shift sums of fbar over lattice indices [i_begin, i_end); cdf: a
    learned second warp (n x (n_bins+1)) or None."""
    shifts = _f64(shifts)
    K = shifts.shape[0]
    assert shifts.shape == (K, n)
    if i_end is None:
        i_end = 1 << log2_n
    sums = np.zeros(2 * K)
    if cdf is None:
        cp, nb = None, 0
    else:
        cdf = _f64(cdf)
        assert cdf.ndim == 2 and cdf.shape[0] == n
        cp, nb = _p(cdf), cdf.shape[1] - 1
    rc = _load().oracle_eval_sums_model(*tables._args(alpha), t_meas, n, log2_n,
                                        int(lattice_a), K, _p(shifts), model_tau,
                                        cp, nb, mode, int(i_begin), int(i_end), n_threads,
                                        _p(sums))
    if rc != 0:
        raise ValueError("oracle_eval_sums_model: bad arguments")
    return sums[0::2] + 1j * sums[1::2]


def eval_mass(tables, t_meas, n, log2_n, lattice_a, shifts, model_tau, i_begin=0,
              i_end=None, n_threads=0, alpha=0.0):
    """Per-shift term mass sum_i 2 W |terms| of the charge estimate over
    lattice indices [i_begin, i_end): the scale of rounding in the sums."""
    shifts = _f64(shifts)
    K = shifts.shape[0]
    if i_end is None:
        i_end = 1 << log2_n
    mass = np.zeros(K)
    rc = _load().oracle_eval_mass(*tables._args(alpha), t_meas, n, log2_n, int(lattice_a), K,
                                  _p(shifts), model_tau, int(i_begin), int(i_end), n_threads,
                                  _p(mass))
    if rc != 0:
        raise ValueError("oracle_eval_mass: bad arguments")
    return mass


def eval_order(tables, t_meas, n, log2_n, lattice_a, shifts, model_tau, mode=0,
               n_threads=0, cdf=None, alpha=0.0):
    """Q^{(s)} for every shift, their mean and standard error (App. G)."""
    N = 1 << log2_n
    q = eval_sums(tables, t_meas, n, log2_n, lattice_a, shifts, model_tau,
                  mode, 0, N, n_threads, cdf, alpha) / N
    K = q.shape[0]
    mean = q.mean()
    stderr = float(np.std(q.real, ddof=1) / np.sqrt(K)) if K > 1 else float("nan")
    return q, mean, stderr


def learn_model(tables, t_meas, n, log2_m, lattice_a, shift, model_tau, n_bins,
                lam, floor_eps, n_threads=0, alpha=0.0):
    """Learned second warp (App. I): returns (hist, cdf), shapes
    (n, n_bins) and (n, n_bins + 1)."""
    shift = _f64(shift).reshape(n)
    hist = np.zeros((n, n_bins))
    cdf = np.zeros((n, n_bins + 1))
    rc = _load().oracle_learn_model(*tables._args(alpha), t_meas, n, log2_m, int(lattice_a),
                                    _p(shift), model_tau, n_bins, lam, floor_eps,
                                    n_threads, _p(hist), _p(cdf))
    assert rc == 0
    return hist, cdf


def learn_model_sobol(tables, t_meas, n, log2_m, V, dshift, model_tau, n_bins, lam,
                      floor_eps, n_threads=0, alpha=0.0):
    """learn_model over the Sobol' points i < 2^log2_m with one digital
    shift (dshift: n words)."""
    V = np.ascontiguousarray(V, dtype=np.uint32)
    dshift = np.ascontiguousarray(dshift, dtype=np.uint32).reshape(n)
    assert V.shape == (n, 32)
    hist = np.zeros((n, n_bins))
    cdf = np.zeros((n, n_bins + 1))
    rc = _load().oracle_learn_model_sobol(*tables._args(alpha), t_meas, n, log2_m, _pu(V),
                                          _pu(dshift), model_tau, n_bins, lam, floor_eps,
                                          n_threads, _p(hist), _p(cdf))
    assert rc == 0
    return hist, cdf


def model_from_hist(hist, lam, floor_eps):
    hist = _f64(hist)
    n, nb = hist.shape
    cdf = np.zeros((n, nb + 1))
    assert _load().oracle_model_from_hist(n, nb, _p(hist), lam, floor_eps, _p(cdf)) == 0
    return cdf


def model_inverse(cdf_row, x):
    """(w, q(w)) for one coordinate's CDF row."""
    cdf_row = _f64(cdf_row)
    w = np.zeros(1)
    q = _load().oracle_model_inverse(_p(cdf_row), cdf_row.shape[0] - 1, float(x), _p(w))
    return float(w[0]), float(q)


def max_threads():
    return _load().oracle_max_threads()
