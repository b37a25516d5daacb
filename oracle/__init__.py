"""FP64 CPU oracle for the ReLCP time-step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU
library (``paper_2506_14097_amd``) and never imports it; the GPU library never
imports this package.

The arithmetic lives in ``relcp_oracle.c`` (plain C, FP64, built with
``-ffp-contract=off``) and in ``mlp.py`` (numpy FP64); this module is argument
marshalling over ctypes.  Each wrapped function cites the passage of the paper
(Palmer, Aktulga, Gao, arXiv 2506.14097) that it follows in the C source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "relcp_oracle.c")
_LIB = os.path.join(_HERE, "_liboracle.so")

MAXREC = 64

OK, E_INVALID, E_OOM, E_DEVICE, E_LCP_MAXITER, E_RECURSION_CAP, E_SKIN, E_NAN, E_CAPACITY = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (no FMA contraction; OpenMP shares
    independent pairs among threads, OMP_NUM_THREADS sets how many)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC,
                               "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [("dynamics", C.c_int), ("planar", C.c_int), ("max_recursions", C.c_int),
                ("lcp_mode", C.c_int), ("lcp_max_iters", C.c_int), ("form", C.c_int),
                ("dt", C.c_double), ("eps", C.c_double), ("tol", C.c_double), ("skin", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("status", C.c_int), ("recursions", C.c_int), ("n_pairs", C.c_int), ("n_rows", C.c_int),
                ("n_contacts", C.c_int * (MAXREC + 1)), ("n_new", C.c_int * (MAXREC + 1)),
                ("lcp_iters", C.c_int * (MAXREC + 1)), ("W", C.c_double * (MAXREC + 1)),
                ("margin", C.c_double * (MAXREC + 1)), ("residual", C.c_double),
                ("max_overlap", C.c_double), ("max_disp", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        assert L.orc_stats_size() == C.sizeof(Stats), "oracle stats layout mismatch"
        assert L.orc_params_size() == C.sizeof(Params), "oracle params layout mismatch"
        L.orc_broadphase.restype = C.c_int64
        L.orc_broadphase_cells.restype = C.c_int64
        _lib = L
    return _lib


def threads(n=0):
    """Set the OpenMP threads of the per-pair loops (n > 0); returns the
    number in use."""
    return int(lib().orc_threads(C.c_int(n)))


def _d(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None:
        assert a.size == n, (a.size, n)
    return a


def _i(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.c_void_p)


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------
def quat_to_R(q):
    R = np.zeros(9)
    lib().orc_quat_to_R(_p(_d(q, 4)), _p(R))
    return R.reshape(3, 3)


def integrate_body(x, q, v, dt):
    xo, qo = np.zeros(3), np.zeros(4)
    lib().orc_integrate_body(_p(_d(x, 3)), _p(_d(q, 4)), _p(_d(v, 6)), C.c_double(dt), _p(xo), _p(qo))
    return xo, qo


def snsd_ellipsoid(d, qa, ea, qb, eb, nsamp=2000):
    """Ellipsoid SNSD: returns (Phi, n, r_a, r_b) with n from a to b."""
    out = np.zeros(10)
    lib().orc_snsd_ellipsoid(_p(_d(d, 3)), _p(_d(qa, 4)), _p(_d(ea, 3)), _p(_d(qb, 4)), _p(_d(eb, 3)),
                             C.c_int(nsamp), _p(out))
    return out[0], out[1:4].copy(), out[4:7].copy(), out[7:10].copy()


def snsd_spherocyl(d, ta, la, ra, tb, lb, rb, planar=0):
    """Spherocylinder SNSD (axis segments of length l, cap radius r)."""
    out = np.zeros(10)
    lib().orc_snsd_spherocyl(_p(_d(d, 3)), _p(_d(ta, 3)), C.c_double(la), C.c_double(ra), _p(_d(tb, 3)),
                             C.c_double(lb), C.c_double(rb), C.c_int(planar), _p(out))
    return out[0], out[1:4].copy(), out[4:7].copy(), out[7:10].copy()


def snsd_torus(d, ea, Ra, ra, eb, Rb, rb):
    """Torus SNSD (Sec. 6, rings): centre-circle distance minus the minor
    radii.  Returns (Phi, n, r_a, r_b, margin) with margin the centre-circle
    distance of the best other local minimum (inf if none)."""
    out = np.zeros(10)
    sec = C.c_double(0.0)
    lib().orc_snsd_torus(_p(_d(d, 3)), _p(_d(ea, 3)), C.c_double(Ra), C.c_double(ra), _p(_d(eb, 3)),
                         C.c_double(Rb), C.c_double(rb), _p(out), C.byref(sec))
    return out[0], out[1:4].copy(), out[4:7].copy(), out[7:10].copy(), sec.value


def snsd_pairs(pa, pb, x, q, kind, shape, box, planar=0):
    """SNSD of every listed pair at configuration (x, q): array (m, 10) of
    [Phi, n(3), r_a(3), r_b(3)]."""
    pa, pb = _i(pa), _i(pb)
    m = pa.size
    out = np.zeros((max(m, 1), 10))
    lib().orc_snsd_pairs(C.c_int(m), _p(pa), _p(pb), _p(_d(x)), _p(_d(q)), _p(_i(kind)), _p(_d(shape)),
                         _p(_d(box, 3)), C.c_int(planar), _p(out))
    return out[:m]


def broadphase(x, kind, shape, box, skin, cells=False):
    """All pairs a < b with bounding-sphere gap <= skin, sorted by (a, b):
    by brute force over all pairs, or (cells=True) through a cell grid, the
    search the oracle step uses for large n."""
    x = _d(x)
    n = x.size // 3
    kind, shape, box = _i(kind), _d(shape), _d(box, 3)
    L = lib()
    f = L.orc_broadphase_cells if cells else L.orc_broadphase
    m = f(C.c_int(n), _p(x), _p(kind), _p(shape), _p(box), C.c_double(skin), C.c_int64(0), None, None)
    pa = np.zeros(max(m, 1), np.int32)
    pb = np.zeros(max(m, 1), np.int32)
    f(C.c_int(n), _p(x), _p(kind), _p(shape), _p(box), C.c_double(skin), C.c_int64(m), _p(pa), _p(pb))
    return pa[:m], pb[:m]


# --------------------------------------------------------------------------
# dynamics and LCP
# --------------------------------------------------------------------------
def body_K(dynamics, planar, dt, kind, shape, q, rho_xi):
    kind = _i(kind)
    n = kind.size
    kt, Kr = np.zeros(3 * n), np.zeros(9 * n)
    rc = lib().orc_body_K(C.c_int(n), C.c_int(dynamics), C.c_int(planar), C.c_double(dt), _p(kind),
                          _p(_d(shape)), _p(_d(q)), _p(_d(rho_xi)), _p(kt), _p(Kr))
    if rc != 0:
        raise ValueError("invalid body for the chosen law of motion")
    return kt.reshape(n, 3), Kr.reshape(n, 3, 3)


def dense_A(n, ia, ib, nrm, ta, tb, kt, Kr, dt):
    """A = dt D^T K D as a dense matrix (rows given SoA)."""
    ia, ib = _i(ia), _i(ib)
    m = ia.size
    A = np.zeros((max(m, 1), max(m, 1)))
    lib().orc_dense_A(C.c_int(n), C.c_int(m), _p(ia), _p(ib), _p(_d(nrm)), _p(_d(ta)), _p(_d(tb)), _p(_d(kt)),
                      _p(_d(Kr)), C.c_double(dt), _p(A))
    return A[:m, :m]


def lcp_enumerate(A, qv):
    """Exact LCP 0 <= A g + qv _|_ g >= 0 by enumerating active sets (m <= 16)."""
    A = _d(A)
    qv = _d(qv)
    m = qv.size
    g = np.zeros(max(m, 1))
    rc = lib().orc_lcp_enumerate(C.c_int(m), _p(A), _p(qv), _p(g))
    if rc != 0:
        raise RuntimeError("no complementary solution found")
    return g[:m]


def lcp_bbpgd_rows(n, ia, ib, nrm, ta, tb, kt, Kr, dt, qv, gamma0=None, tol=1e-12, max_iter=1000000):
    """Jacobi-scaled BB projected gradient on rows; returns (gamma, iters, residual)."""
    ia, ib = _i(ia), _i(ib)
    m = ia.size
    g = np.zeros(max(m, 1)) if gamma0 is None else _d(gamma0).copy()
    res = C.c_double(0.0)
    it = lib().orc_lcp_bbpgd_rows(C.c_int(n), C.c_int(m), _p(ia), _p(ib), _p(_d(nrm)), _p(_d(ta)), _p(_d(tb)),
                                  _p(_d(kt)), _p(_d(Kr)), C.c_double(dt), _p(_d(qv)), _p(g), C.c_double(tol),
                                  C.c_int(max_iter), C.byref(res))
    return g[:m], it, res.value


def relcp_step(x, q, kind, shape, rho_xi, box, *, dt, eps, tol, skin, u=None, fext=None, dynamics=0, planar=0,
               max_recursions=64, lcp_mode=0, lcp_max_iters=1000000, form=0, prev=None, row_cap=None):
    """One ReLCP step (Alg. 1 / Eq. relcp; inertial Eq. relcp_inertial).

    prev = (a, b, lam) arrays sorted by (a, b): previous-step multipliers
    per pair, used as the warm start of the iteration-0 rows.
    Returns a dict with the status, accepted state, velocity V_n, rows and
    the per-recursion statistics."""
    x, q = _d(x).copy(), _d(q).copy()
    n = x.size // 3
    kind, shape, rho_xi, box = _i(kind), _d(shape), _d(rho_xi), _d(box, 3)
    uu = None if u is None else _d(u, 6 * n)
    ff = None if fext is None else _d(fext, 6 * n)
    if prev is None:
        pa_, pb_, pl_ = np.zeros(1, np.int32), np.zeros(1, np.int32), np.zeros(1)
        npv = 0
    else:
        pa_, pb_, pl_ = _i(prev[0]), _i(prev[1]), _d(prev[2])
        npv = pa_.size
    P = Params(dynamics, planar, max_recursions, lcp_mode, lcp_max_iters, form, dt, eps, tol, skin)
    if row_cap is None:
        row_cap = max(64, 40 * n)
    xo, qo, Uo = np.zeros(3 * n), np.zeros(4 * n), np.zeros(6 * n)
    r_ia = np.zeros(row_cap, np.int32)
    r_ib = np.zeros(row_cap, np.int32)
    r_rec = np.zeros(row_cap, np.int32)
    r_pair = np.zeros(row_cap, np.int32)
    r_gam = np.zeros(row_cap)
    r_phi = np.zeros(row_cap)
    r_n = np.zeros(3 * row_cap)
    r_ta = np.zeros(3 * row_cap)
    r_tb = np.zeros(3 * row_cap)
    st = Stats()
    rc = lib().orc_relcp_step(
        C.c_int(n), _p(x), _p(q), _p(uu), _p(kind), _p(shape), _p(rho_xi), _p(box), _p(ff), C.c_int(npv), _p(pa_),
        _p(pb_), _p(pl_), C.byref(P), _p(xo), _p(qo), _p(Uo), C.c_int(row_cap), _p(r_ia), _p(r_ib), _p(r_rec),
        _p(r_pair), _p(r_gam), _p(r_phi), _p(r_n), _p(r_ta), _p(r_tb), C.byref(st))
    m = st.n_rows
    R = st.recursions
    return dict(
        status=rc, x=xo.reshape(n, 3), q=qo.reshape(n, 4), U=Uo.reshape(n, 6),
        ia=r_ia[:m].copy(), ib=r_ib[:m].copy(), rec=r_rec[:m].copy(), pair=r_pair[:m].copy(),
        gamma=r_gam[:m].copy(), phi=r_phi[:m].copy(), n=r_n[:3 * m].reshape(m, 3).copy(),
        ta=r_ta[:3 * m].reshape(m, 3).copy(), tb=r_tb[:3 * m].reshape(m, 3).copy(),
        recursions=R, n_pairs=st.n_pairs, n_rows=m,
        n_contacts=np.array(st.n_contacts[:R + 1]), n_new=np.array(st.n_new[:R + 1]),
        lcp_iters=np.array(st.lcp_iters[:R + 1]), W=np.array(st.W[:R + 1]), margin=np.array(st.margin[:R + 1]),
        residual=st.residual, max_overlap=st.max_overlap, max_disp=st.max_disp)


def pair_lambda(res):
    """Per-pair multiplier sums of a step result (the next step's warm start),
    sorted by (a, b)."""
    if res["n_rows"] == 0:
        return np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0)
    key = res["ia"].astype(np.int64) * (1 << 31) + res["ib"]
    uk, inv = np.unique(key, return_inverse=True)
    lam = np.zeros(uk.size)
    np.add.at(lam, inv, res["gamma"])
    return (uk // (1 << 31)).astype(np.int32), (uk % (1 << 31)).astype(np.int32), lam
