"""Thin ctypes binding of librelcp.so (the C ABI in include/relcp.h).

Argument marshalling only: every step of the time-step runs in the HIP
kernels of librelcp.so.  There is no fallback: if the library is missing the
import of this module's functions raises.

Host arrays are numpy (array-of-structs per body, FP64); the ``*_device``
helpers take torch tensors on the GPU and pass their data pointers.
"""
from __future__ import annotations

import ctypes as C
import os
from collections.abc import Mapping

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "librelcp.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "relcp.h")

OK = 0
E_INVALID, E_OOM, E_DEVICE, E_LCP_MAXITER, E_RECURSION_CAP, E_SKIN, E_NAN, E_CAPACITY = (-1, -2, -3, -4, -5, -6,
                                                                                       -7, -8)
ELLIPSOID, SPHEROCYLINDER, TORUS = 0, 1, 2
OVERDAMPED, INERTIAL = 0, 1
WS_COLD, WS_PREV, WS_LEARNED = 0, 1, 2
MAX_RECORDED = 65

STATUS_NAMES = {0: "ok", -1: "invalid", -2: "out of memory", -3: "device error", -4: "LCP iteration cap",
                -5: "recursion cap", -6: "skin exceeded", -7: "non-finite value", -8: "capacity"}


class RelcpError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__("relcp status %d (%s): %s" % (status, STATUS_NAMES.get(status, "?"), msg))
        self.status = status


class Bodies(C.Structure):
    _fields_ = [("n", C.c_int32), ("x", C.c_void_p), ("q", C.c_void_p), ("u", C.c_void_p), ("w", C.c_void_p),
                ("n_batch", C.c_int32), ("batch_off", C.c_void_p), ("box", C.c_void_p)]


class Shapes(C.Structure):
    _fields_ = [("kind", C.c_void_p), ("p", C.c_void_p), ("rho_or_xi", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("dynamics", C.c_int32), ("precision", C.c_int32), ("warm_start", C.c_int32), ("planar", C.c_int32),
                ("max_recursions", C.c_int32), ("lcp_max_iters", C.c_int32), ("lcp_fixed_iters", C.c_int32),
                ("skin", C.c_double), ("stream", C.c_void_p)]


class StepStats(C.Structure):
    _fields_ = [("recursions", C.c_int32), ("lcp_iters_total", C.c_int32), ("n_pairs", C.c_int32),
                ("n_contacts_final", C.c_int32), ("n_contacts", C.c_int32 * MAX_RECORDED),
                ("lcp_iters", C.c_int32 * MAX_RECORDED), ("lcp_iters64", C.c_int32 * MAX_RECORDED),
                ("W", C.c_double * MAX_RECORDED),
                ("margin", C.c_double * MAX_RECORDED), ("residual_fp64", C.c_double),
                ("residual_lowp", C.c_double), ("max_overlap", C.c_double), ("max_disp", C.c_double),
                ("t_narrow", C.c_double), ("t_lcp", C.c_double), ("t_other", C.c_double),
                ("rowgraph_entries", C.c_int32 * MAX_RECORDED), ("pairs_rebuilt", C.c_int32),
                ("n_waits", C.c_int32), ("t_wait", C.c_double), ("rowgraph_restarts", C.c_int32)]

    def as_dict(self):
        R = self.recursions
        k = min(R + 1, MAX_RECORDED)
        return dict(recursions=R, lcp_iters_total=self.lcp_iters_total, n_pairs=self.n_pairs,
                    n_contacts_final=self.n_contacts_final, n_contacts=np.array(self.n_contacts[:k]),
                    lcp_iters=np.array(self.lcp_iters[:k]), lcp_iters64=np.array(self.lcp_iters64[:k]),
                    W=np.array(self.W[:k]), margin=np.array(self.margin[:k]),
                    residual_fp64=self.residual_fp64, residual_lowp=self.residual_lowp,
                    max_overlap=self.max_overlap, max_disp=self.max_disp, t_narrow=self.t_narrow, t_lcp=self.t_lcp,
                    t_other=self.t_other, rowgraph_entries=np.array(self.rowgraph_entries[:k]),
                    pairs_rebuilt=self.pairs_rebuilt, n_waits=self.n_waits, t_wait=self.t_wait,
                    rowgraph_restarts=self.rowgraph_restarts)


class StepResult(Mapping):
    """The statistics of one step, read-only: the keys of StepStats.as_dict()
    and "status".  The C struct is converted on the first access to a key
    other than "status", so that a caller that reads none of them (or reads
    them later) spends no host time on it between steps."""
    __slots__ = ("_st", "_rc", "_d")

    def __init__(self, st, rc):
        self._st, self._rc, self._d = st, rc, None

    def _dict(self):
        if self._d is None:
            d = self._st.as_dict()
            d["status"] = self._rc
            self._d, self._st = d, None
        return self._d

    def __getitem__(self, key):
        if key == "status":
            return self._rc
        return self._dict()[key]

    def __iter__(self):
        return iter(self._dict())

    def __len__(self):
        return len(self._dict())

    def __repr__(self):
        return repr(self._dict())


_lib = None

# every entry point of include/relcp.h with its ctypes signature
_SIGS = {
    "relcp_create": (C.c_int, [C.POINTER(Bodies), C.POINTER(Shapes), C.POINTER(Params), C.POINTER(C.c_void_p)]),
    "relcp_destroy": (None, [C.c_void_p]),
    "relcp_last_error": (C.c_char_p, [C.c_void_p]),
    "relcp_set_external": (C.c_int, [C.c_void_p, C.c_void_p]),
    "relcp_step": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_double, C.POINTER(StepStats)]),
    "relcp_get_state": (C.c_int, [C.c_void_p] + [C.c_void_p] * 4),
    "relcp_get_state_device": (C.c_int, [C.c_void_p] + [C.c_void_p] * 4),
    "relcp_set_state": (C.c_int, [C.c_void_p, C.POINTER(Bodies), C.POINTER(Shapes)]),
    "relcp_affine_rescale": (C.c_int, [C.c_void_p, C.c_double]),
    "relcp_affine_rescale_packings": (C.c_int, [C.c_void_p, C.c_void_p]),
    "relcp_get_contacts": (C.c_int, [C.c_void_p] + [C.c_void_p] * 6),
    "relcp_grow": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_void_p]),
    "relcp_divide": (C.c_int, [C.c_void_p, C.c_double, C.c_void_p, C.c_int32, C.c_void_p]),
    "relcp_set_lcp_config": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32]),
    "relcp_autotune": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_int32, C.c_void_p, C.c_void_p]),
    "relcp_set_timing": (C.c_int, [C.c_void_p, C.c_int32]),
    "relcp_get_timing": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    "relcp_set_warm_start": (C.c_int, [C.c_void_p, C.c_int32]),
    "relcp_set_warmstart_model": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "relcp_enable_contact_log": (C.c_int, [C.c_void_p, C.c_int32]),
    "relcp_log_contacts": (C.c_int, [C.c_void_p] + [C.c_void_p] * 4 + [C.c_int32, C.POINTER(C.c_int32)]),
    "relcp_mlp_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p]),
    "relcp_mlp_workspace_bytes": (C.c_size_t, [C.c_int32]),
    "relcp_mlp_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32] + [C.c_void_p] * 6 + [C.c_size_t, C.c_void_p]),
    "relcp_mlp_adam": (C.c_int, [C.c_void_p] * 4 + [C.c_int32, C.c_float, C.c_void_p]),
    "relcp_snsd_device": (C.c_int, [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "relcp_broadphase_device": (C.c_int, [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                          C.c_int32, C.c_void_p, C.c_void_p, C.POINTER(C.c_int32), C.c_void_p]),
    "relcp_lcp_solve_device": (C.c_int, [C.c_int32, C.c_int32] + [C.c_void_p] * 8 + [C.c_double, C.c_int32, C.c_int32,
                                         C.c_int32, C.c_double, C.c_int32, C.c_void_p, C.POINTER(C.c_int32),
                                         C.POINTER(C.c_double), C.c_void_p]),
    "relcp_exclusive_scan_device": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "relcp_exclusive_scan_device_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "relcp_compact_flags_device": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
}


def lib():
    """Load librelcp.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise ImportError("librelcp.so is not built: run `python -m paper_2506_14097_amd.build`")
        L = C.CDLL(LIBPATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _d(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError("expected %d values, got %d" % (n, a.size))
    return a


def _i(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a):
    return None if a is None else a.ctypes.data


def _tptr(t):
    """Device pointer of a torch tensor (or None)."""
    return None if t is None else t.data_ptr()


class Simulation:
    """A ReLCP context: one or several independent packings on one GPU."""

    def __init__(self, x, q, kind, shape, rho_xi, box, u=None, w=None, batch_off=None, *, dynamics=OVERDAMPED,
                 precision=64, warm_start=WS_PREV, planar=False, max_recursions=64, lcp_max_iters=0,
                 lcp_fixed_iters=0, skin=0.05, stream=None):
        L = lib()
        self._keep = []
        self.ctx = C.c_void_p()
        B, S = self._structs(x, q, kind, shape, rho_xi, box, u, w, batch_off)
        P = Params(dynamics, precision, warm_start, 1 if planar else 0, max_recursions, lcp_max_iters,
                   lcp_fixed_iters, skin, stream)
        rc = L.relcp_create(C.byref(B), C.byref(S), C.byref(P), C.byref(self.ctx))
        self._keep = []
        if rc != OK:
            self.ctx = None
            raise RelcpError(rc, "relcp_create")

    def _structs(self, x, q, kind, shape, rho_xi, box, u, w, batch_off):
        x = _d(x)
        n = x.size // 3
        q = _d(q, 4 * n)
        kind = _i(kind)
        shape = _d(shape, 3 * n)
        rho_xi = _d(rho_xi, n)
        box = _d(box)
        nb = box.size // 3
        boff = None if batch_off is None else _i(batch_off)
        uu = None if u is None else _d(u, 3 * n)
        ww = None if w is None else _d(w, 3 * n)
        self._keep = [x, q, kind, shape, rho_xi, box, boff, uu, ww]
        self.n = n
        self.n_batch = nb
        B = Bodies(n, _ptr(x), _ptr(q), _ptr(uu), _ptr(ww), nb, _ptr(boff), _ptr(box))
        S = Shapes(_ptr(kind), _ptr(shape), _ptr(rho_xi))
        return B, S

    def close(self):
        ctx, self.ctx = getattr(self, "ctx", None), None
        if ctx and _lib is not None:
            _lib.relcp_destroy(ctx)

    __del__ = close

    def _err(self):
        return lib().relcp_last_error(self.ctx).decode()

    def set_external(self, f):
        f = None if f is None else _d(f, 6 * self.n)
        rc = lib().relcp_set_external(self.ctx, _ptr(f))
        if rc != OK:
            raise RelcpError(rc, self._err())

    def step(self, dt, overlap_tol, lcp_tol, raise_on_error=True):
        st = StepStats()
        rc = lib().relcp_step(self.ctx, dt, overlap_tol, lcp_tol, C.byref(st))
        if rc != OK and raise_on_error:
            raise RelcpError(rc, self._err())
        return StepResult(st, rc)

    def get_state(self):
        n = self.n
        x, q, u, w = np.zeros(3 * n), np.zeros(4 * n), np.zeros(3 * n), np.zeros(3 * n)
        rc = lib().relcp_get_state(self.ctx, _ptr(x), _ptr(q), _ptr(u), _ptr(w))
        if rc != OK:
            raise RelcpError(rc, self._err())
        return x.reshape(n, 3), q.reshape(n, 4), np.concatenate([u.reshape(n, 3), w.reshape(n, 3)], 1)

    def get_state_device(self, x, q, u, w):
        rc = lib().relcp_get_state_device(self.ctx, _tptr(x), _tptr(q), _tptr(u), _tptr(w))
        if rc != OK:
            raise RelcpError(rc, self._err())

    def set_state(self, x, q, kind, shape, rho_xi, box, u=None, w=None, batch_off=None):
        B, S = self._structs(x, q, kind, shape, rho_xi, box, u, w, batch_off)
        rc = lib().relcp_set_state(self.ctx, C.byref(B), C.byref(S))
        self._keep = []
        if rc != OK:
            raise RelcpError(rc, self._err())

    def affine_rescale(self, s):
        rc = lib().relcp_affine_rescale(self.ctx, s)
        if rc != OK:
            raise RelcpError(rc, self._err())

    def grow(self, dl, l_div=float("inf"), count=False):
        """Cylinder lengths of all spherocylinders += dl (device side);
        with count=True returns how many reached l_div (one wait)."""
        n = C.c_int32(0)
        rc = lib().relcp_grow(self.ctx, float(dl), float(l_div), C.byref(n) if count else None)
        if rc != OK:
            raise RelcpError(rc, self._err())
        return n.value if count else None

    def divide(self, l_div, jitter):
        """Split every spherocylinder with l >= l_div into its two halves,
        each turned about z by its angle in jitter (two per dividing cell,
        in the order of the parents' indices); returns the number divided."""
        jit = np.ascontiguousarray(jitter, dtype=np.float64)
        n = C.c_int32(0)
        rc = lib().relcp_divide(self.ctx, float(l_div), _ptr(jit) if jit.size else None, int(jit.size), C.byref(n))
        if rc != OK:
            raise RelcpError(rc, self._err())
        self.n += n.value
        return n.value

    TIMING_CLASSES = ("lcp_scatter", "lcp_gather", "snsd", "pairs", "trial", "lcp_resident", "warm_start",
                      "lcp_rowgraph", "rowgraph_build", "lcp_rowgraph_idle", "lcp_rowgraph64",
                      "lcp_rowgraph_start")
    LCP_CONFIGS = ("grid", "resident-256", "resident-256-lds", "resident-512", "resident-512-lds",
                   "resident-1024", "resident-1024-lds", "rowgraph", "rowgraph-perpass")

    def set_lcp_config(self, mode, block=256, lds=True):
        """mode: 0 automatic, 1 grid, 2 resident (one workgroup per packing),
        3 row graph (A assembled over rows, one pass per iteration, passes
        replayed from an instantiated HIP graph), 4 row graph with a launch
        per pass."""
        rc = lib().relcp_set_lcp_config(self.ctx, mode, block, 1 if lds else 0)
        if rc != OK:
            raise RelcpError(rc, self._err())

    def autotune(self, dt, lcp_tol, reps=3):
        cfg = np.zeros(3, np.int32)
        ms = np.zeros(len(self.LCP_CONFIGS))
        rc = lib().relcp_autotune(self.ctx, dt, lcp_tol, reps, _ptr(cfg), _ptr(ms))
        if rc != OK:
            raise RelcpError(rc, self._err())
        return dict(mode=int(cfg[0]), block=int(cfg[1]), lds=bool(cfg[2]),
                    ms={k: float(v) for k, v in zip(self.LCP_CONFIGS, ms)})

    def set_timing(self, on):
        rc = lib().relcp_set_timing(self.ctx, 1 if on else 0)
        if rc != OK:
            raise RelcpError(rc, self._err())

    def get_timing(self, reset=True):
        cnt = np.zeros(len(self.TIMING_CLASSES), np.int32)
        ms = np.zeros(len(self.TIMING_CLASSES))
        rc = lib().relcp_get_timing(self.ctx, _ptr(cnt), _ptr(ms), 1 if reset else 0)
        if rc != OK:
            raise RelcpError(rc, self._err())
        return {k: (int(c), float(t)) for k, c, t in zip(self.TIMING_CLASSES, cnt, ms)}

    def affine_rescale_packings(self, s):
        s = _d(s, self.n_batch)
        rc = lib().relcp_affine_rescale_packings(self.ctx, _ptr(s))
        if rc != OK:
            raise RelcpError(rc, self._err())

    def get_contacts(self, m):
        ia, ib, rec = np.zeros(m, np.int32), np.zeros(m, np.int32), np.zeros(m, np.int32)
        gam, phi, nrm = np.zeros(m), np.zeros(m), np.zeros(3 * m)
        rc = lib().relcp_get_contacts(self.ctx, _ptr(ia), _ptr(ib), _ptr(rec), _ptr(gam), _ptr(phi), _ptr(nrm))
        if rc != OK:
            raise RelcpError(rc, self._err())
        return dict(ia=ia, ib=ib, rec=rec, gamma=gam, phi=phi, n=nrm.reshape(m, 3))


    # ---- learned warm start ----
    def set_warm_start(self, mode):
        rc = lib().relcp_set_warm_start(self.ctx, int(mode))
        if rc != OK:
            raise RelcpError(rc, self._err())

    def set_warmstart_model(self, params, norm):
        params = np.ascontiguousarray(params, dtype=np.float32)
        norm = np.ascontiguousarray(norm, dtype=np.float32)
        if params.size != MLP_NPARAM or norm.size != MLP_NORM:
            raise ValueError("model needs %d weights and %d normalisation values" % (MLP_NPARAM, MLP_NORM))
        rc = lib().relcp_set_warmstart_model(self.ctx, _ptr(params), _ptr(norm))
        if rc != OK:
            raise RelcpError(rc, self._err())

    def enable_contact_log(self, on=True):
        rc = lib().relcp_enable_contact_log(self.ctx, 1 if on else 0)
        if rc != OK:
            raise RelcpError(rc, self._err())

    def log_contacts(self, device="cuda:0"):
        """Rows of A_0 of the last accepted step: (feat (m, 8) float32,
        gamma (m,) float32, ia (m,), ib (m,) int32), torch tensors on the GPU."""
        import torch
        cnt = C.c_int32(0)
        rc = lib().relcp_log_contacts(self.ctx, None, None, None, None, 0, C.byref(cnt))
        if rc not in (OK, E_CAPACITY):
            raise RelcpError(rc, self._err())
        m = cnt.value
        feat = torch.empty((max(m, 1), MLP_NFEAT), dtype=torch.float32, device=device)
        gam = torch.empty(max(m, 1), dtype=torch.float32, device=device)
        ia = torch.empty(max(m, 1), dtype=torch.int32, device=device)
        ib = torch.empty(max(m, 1), dtype=torch.int32, device=device)
        if m > 0:
            rc = lib().relcp_log_contacts(self.ctx, _tptr(feat), _tptr(gam), _tptr(ia), _tptr(ib), m, C.byref(cnt))
            if rc != OK:
                raise RelcpError(rc, self._err())
        return feat[:m], gam[:m], ia[:m], ib[:m]


# --------------------------------------------------------------------------
# learned warm start: device training and inference kernels
# --------------------------------------------------------------------------
MLP_NPARAM = 17793
MLP_NORM = 17
MLP_NFEAT = 8


def mlp_forward(params, norm, feat, idx=None, out=None, stream=None):
    """Warm start max(0, f_2 + scale z) (length units) for the rows of feat
    (n, 8) (or feat[idx]);
    params: float32 cuda tensor of MLP_NPARAM values; norm: 17 host floats."""
    import torch
    n = feat.shape[0] if idx is None else idx.numel()
    if out is None:
        out = torch.empty(max(feat.shape[0], 1), dtype=torch.float32, device=feat.device)
    nh = np.ascontiguousarray(norm, dtype=np.float32)
    rc = lib().relcp_mlp_forward(_tptr(params), _ptr(nh), n, _tptr(feat), _tptr(idx), _tptr(out), stream)
    if rc != OK:
        raise RelcpError(rc, "relcp_mlp_forward")
    return out


def mlp_workspace(n, device):
    import torch
    nbytes = int(lib().relcp_mlp_workspace_bytes(int(n)))
    return torch.empty(max(nbytes // 4, 1), dtype=torch.float32, device=device)


def mlp_grad(params, norm, feat, target, idx=None, grad=None, loss=None, work=None, stream=None):
    """Gradient of mean (z - (target - f_2) / scale)^2 over the batch.
    Returns (grad, loss) as cuda tensors."""
    import torch
    n = feat.shape[0] if idx is None else idx.numel()
    dev = params.device
    if grad is None:
        grad = torch.empty(MLP_NPARAM, dtype=torch.float32, device=dev)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=dev)
    if work is None:
        work = mlp_workspace(n, dev)
    nh = np.ascontiguousarray(norm, dtype=np.float32)
    rc = lib().relcp_mlp_grad(_tptr(params), _ptr(nh), n, _tptr(feat), _tptr(target), _tptr(idx), _tptr(grad),
                              _tptr(loss), _tptr(work), work.numel() * 4, stream)
    if rc != OK:
        raise RelcpError(rc, "relcp_mlp_grad")
    return grad, loss


def mlp_adam(params, grad, m, v, t, lr, stream=None):
    rc = lib().relcp_mlp_adam(_tptr(params), _tptr(grad), _tptr(m), _tptr(v), int(t), float(lr), stream)
    if rc != OK:
        raise RelcpError(rc, "relcp_mlp_adam")


# --------------------------------------------------------------------------
# stand-alone device operations (torch tensors in, torch tensors out)
# --------------------------------------------------------------------------
def snsd_device(x_soa, q_soa, kind, p_soa, pa, pb, box, planar=False, out=None, stream=None):
    """SNSD of pairs on the GPU: x_soa (3, nb), q_soa (4, nb), p_soa (3, nb)
    float64 cuda tensors; kind, pa, pb int32 cuda tensors.  Returns out (10, m)."""
    import torch
    nb = x_soa.shape[1]
    m = pa.numel()
    if out is None:
        out = torch.empty((10, max(m, 1)), dtype=torch.float64, device=x_soa.device)
    boxh = _d(box, 3)
    rc = lib().relcp_snsd_device(nb, _tptr(x_soa), _tptr(q_soa), _tptr(kind), _tptr(p_soa), m, _tptr(pa), _tptr(pb),
                                 boxh.ctypes.data, 1 if planar else 0, _tptr(out), stream)
    if rc != OK:
        raise RelcpError(rc, "relcp_snsd_device")
    return out[:, :m]


def broadphase_device(x_soa, kind, p_soa, box, skin, cap=None, stream=None):
    import torch
    nb = x_soa.shape[1]
    if cap is None:
        cap = 64 * nb
    pa = torch.empty(max(cap, 1), dtype=torch.int32, device=x_soa.device)
    pb = torch.empty(max(cap, 1), dtype=torch.int32, device=x_soa.device)
    m = C.c_int32(0)
    boxh = _d(box, 3)
    rc = lib().relcp_broadphase_device(nb, _tptr(x_soa), _tptr(kind), _tptr(p_soa), boxh.ctypes.data, skin, cap,
                                       _tptr(pa), _tptr(pb), C.byref(m), stream)
    if rc != OK:
        raise RelcpError(rc, "relcp_broadphase_device")
    k = min(m.value, cap)
    return pa[:k], pb[:k], m.value


def lcp_solve_device(nb, ia, ib, n_soa, ta_soa, tb_soa, qv, kt, Kr_soa, dt, gamma, *, planar=False, precision=64,
                     mode=0, tol=1e-12, max_iters=0, stream=None):
    """Solve 0 <= qv + dt D^T K D gamma _|_ gamma >= 0 on the GPU (gamma
    in/out).  Returns (iterations, FP64 residual, status)."""
    m = ia.numel()
    it = C.c_int32(0)
    res = C.c_double(0.0)
    rc = lib().relcp_lcp_solve_device(nb, m, _tptr(ia), _tptr(ib), _tptr(n_soa), _tptr(ta_soa), _tptr(tb_soa),
                                      _tptr(qv), _tptr(kt), _tptr(Kr_soa), dt, 1 if planar else 0, precision, mode,
                                      tol, max_iters, _tptr(gamma), C.byref(it), C.byref(res), stream)
    return it.value, res.value, rc


def exclusive_scan_device(x, out=None, stream=None):
    """Exclusive prefix sum of an int32 device tensor; returns (out, total)."""
    import torch
    out = torch.empty_like(x) if out is None else out
    tot = torch.zeros(1, dtype=torch.int32, device=x.device)
    rc = lib().relcp_exclusive_scan_device(_tptr(x), _tptr(out), x.numel(), _tptr(tot), stream)
    if rc != OK:
        raise RelcpError(rc, "exclusive scan failed")
    return out, int(tot.item())


NOALLOC_SCAN_MAX = 8388608


def exclusive_scan_device_noalloc(x, out, total, stream=None):
    """The same prefix sum through the entry point that allocates nothing
    (scratch in the library's static device array; asynchronous on the
    stream).  Returns the status."""
    return lib().relcp_exclusive_scan_device_noalloc(_tptr(x), _tptr(out), x.numel(), _tptr(total), stream)


def compact_flags_device(flags, stream=None):
    """Indices of the nonzero entries of an int32 device tensor (increasing)."""
    import torch
    out = torch.empty(max(flags.numel(), 1), dtype=torch.int32, device=flags.device)
    cnt = torch.zeros(1, dtype=torch.int32, device=flags.device)
    rc = lib().relcp_compact_flags_device(_tptr(flags), flags.numel(), _tptr(out), _tptr(cnt), stream)
    if rc != OK:
        raise RelcpError(rc, "compaction failed")
    return out[:int(cnt.item())]


def header_symbols():
    """Names of the functions declared in include/relcp.h."""
    import re
    with open(HEADER) as f:
        txt = f.read()
    return sorted(set(re.findall(r"RELCP_API\s+[\w\s\*]*?\b(relcp_\w+)\s*\(", txt)))
