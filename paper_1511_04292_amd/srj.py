"""Thin ctypes binding of libsrj (include/srj.h): argument marshalling only.

Every step of the solver runs in the HIP library; PyTorch supplies device memory (float64
CUDA tensors, dense, ring included) and the current stream.  The library must have been
built (``__graft_entry__.build()`` or ``python paper_1511_04292_amd/build.py``); importing
this module without it raises -- there is no fallback path.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libsrj.so")

SRJ_F64, SRJ_F32, SRJ_BF16 = 0, 1, 2
DTYPES = {"f64": SRJ_F64, "f32": SRJ_F32, "bf16": SRJ_BF16}
MAX_LEVELS = 16
STATUS = {0: "ok", 1: "einval", 2: "enomem", 3: "ehip", 4: "eschedule", 5: "enoconv", 6: "ediverged"}


class SrjError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _Grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("n", ctypes.c_int64 * 3), ("h", ctypes.c_double * 3),
                ("dtype", ctypes.c_int32), ("bc", ctypes.c_int32)]


class _Schedule(ctypes.Structure):
    _fields_ = [("P", ctypes.c_int32), ("omega", ctypes.POINTER(ctypes.c_double)),
                ("q", ctypes.POINTER(ctypes.c_int64)), ("kappa_min", ctypes.c_double),
                ("n_eff", ctypes.c_double), ("q_rounding", ctypes.c_int32),
                ("ordering", ctypes.c_int32), ("sequence", ctypes.POINTER(ctypes.c_int32)),
                ("M", ctypes.c_int64)]


BCS = {"dirichlet": 0, "neumann": 1}


def _fill_grid(g, n, h, dtype, bc="dirichlet"):
    """n = (n_x, n_y[, n_z]); h one spacing for every axis or one per axis (h_x, h_y[, h_z]);
    bc 'dirichlet' or 'neumann'."""
    g.bc = BCS[bc] if isinstance(bc, str) else int(bc)
    g.ndim = len(n)
    for i, v in enumerate(n):
        g.n[i] = int(v)
    hs = [float(h)] * len(n) if np.isscalar(h) else [float(x) for x in h]
    if len(hs) != len(n):
        raise ValueError("one spacing per axis")
    for i, v in enumerate(hs):
        g.h[i] = v
    g.dtype = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)


class _Desc(ctypes.Structure):
    _fields_ = [("P", ctypes.c_int32), ("M", ctypes.c_int64),
                ("omega", ctypes.c_double * MAX_LEVELS), ("beta", ctypes.c_double * MAX_LEVELS),
                ("q", ctypes.c_int64 * MAX_LEVELS), ("kappa_min", ctypes.c_double),
                ("kappa_max", ctypes.c_double), ("rho", ctypes.c_double),
                ("gamma_q_max", ctypes.c_double), ("prefix_peak_log10", ctypes.c_double),
                ("suffix_peak_log10", ctypes.c_double), ("fused_sweeps", ctypes.c_int32),
                ("resident", ctypes.c_int32), ("store_nt", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int64), ("cycles", ctypes.c_int64), ("relres", ctypes.c_double),
                ("seconds", ctypes.c_double), ("status", ctypes.c_int32)]


class _SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_sweeps", ctypes.c_int64), ("start_offset", ctypes.c_int64),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_cap", ctypes.c_int64),
                ("history_len", ctypes.c_int64)]


class _Tune(ctypes.Structure):
    _fields_ = [("fused_sweeps", ctypes.c_int32), ("seg_rows", ctypes.c_int32), ("candidates", ctypes.c_int32),
                ("us_per_sweep", ctypes.c_double), ("us_per_sweep_before", ctypes.c_double)]


_lib = None

EXPORTS = ["srj_plan", "srj_plan_destroy", "srj_plan_describe", "srj_plan_sequence",
           "srj_plan_set_fusion", "srj_solve", "srj_sweeps", "srj_residual", "srj_solve_ir",
           "srj_schedule_optimal", "srj_schedule_order", "srj_status_string", "srj_last_error",
           "srj_adjoint", "srj_batch_plan", "srj_batch_solve", "srj_batch_destroy", "srj_plan_tune",
           "srj_batch_tune", "srj_residual_static", "srj_schedule_counts", "srj_plan_operator", "srj_solve_ex",
           "srj_plan_tune_cached", "srj_plan_poison"]


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(SO):
        raise ImportError(f"libsrj.so is not built ({SO}); run __graft_entry__.build()")
    # The tensors handed to the library come from torch's HIP runtime.  Loading torch first
    # makes libsrj's libamdhip64.so.7 dependency resolve to that same, already mapped
    # runtime; loaded the other way round the process would hold two HIP (and two HSA)
    # runtimes, and the second one to reach the device fails its allocations.
    import torch  # noqa: F401
    L = ctypes.CDLL(SO)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.srj_plan.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Schedule), vp, ctypes.POINTER(vp)]
    L.srj_plan_operator.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Schedule), vp, vp, vp, ctypes.POINTER(vp)]
    L.srj_plan_destroy.argtypes = [vp]
    L.srj_plan_destroy.restype = None
    L.srj_plan_describe.argtypes = [vp, ctypes.POINTER(_Desc)]
    L.srj_plan_sequence.argtypes = [vp, ctypes.POINTER(i32), i64]
    L.srj_plan_set_fusion.argtypes = [vp, i32, i32]
    L.srj_solve.argtypes = [vp, vp, vp, dbl, i64, ctypes.POINTER(_Info)]
    L.srj_solve_ex.argtypes = [vp, vp, vp, ctypes.POINTER(_SolveOpts), ctypes.POINTER(_Info)]
    L.srj_sweeps.argtypes = [vp, vp, vp, i64, i64, ctypes.POINTER(dbl)]
    L.srj_residual.argtypes = [vp, vp, vp, vp, ctypes.POINTER(dbl)]
    L.srj_solve_ir.argtypes = [vp, vp, vp, dbl, i32, i32, ctypes.POINTER(_Info)]
    L.srj_residual_static.argtypes = [ctypes.POINTER(_Grid), vp, vp, vp, vp, vp]
    L.srj_adjoint.argtypes = [vp, vp, dbl, i64, vp, vp, ctypes.POINTER(_Info)]
    L.srj_batch_plan.argtypes = [i32, ctypes.POINTER(_Grid), ctypes.POINTER(_Schedule), vp, ctypes.POINTER(vp)]
    L.srj_batch_solve.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), dbl, i32, i32, ctypes.POINTER(_Info),
                                  ctypes.POINTER(dbl)]
    L.srj_batch_destroy.argtypes = [vp]
    L.srj_batch_destroy.restype = None
    L.srj_plan_tune.argtypes = [vp, ctypes.POINTER(_Tune)]
    L.srj_plan_tune_cached.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(_Tune)]
    L.srj_plan_poison.argtypes = [vp]
    L.srj_batch_tune.argtypes = [vp, ctypes.POINTER(_Tune)]
    L.srj_schedule_optimal.argtypes = [i32, dbl, dbl, ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                       ctypes.POINTER(i64), ctypes.POINTER(dbl)]
    L.srj_schedule_counts.argtypes = [i32, ctypes.POINTER(dbl), ctypes.POINTER(dbl), dbl, dbl, i32,
                                      ctypes.POINTER(i64)]
    L.srj_schedule_order.argtypes = [i32, ctypes.POINTER(dbl), ctypes.POINTER(i64), dbl, dbl, i32,
                                     ctypes.POINTER(i32)]
    L.srj_status_string.argtypes = [i32]
    L.srj_status_string.restype = ctypes.c_char_p
    L.srj_last_error.argtypes = []
    L.srj_last_error.restype = ctypes.c_char_p
    for name in ["srj_plan", "srj_plan_describe", "srj_plan_sequence", "srj_plan_set_fusion", "srj_solve",
                 "srj_sweeps", "srj_residual", "srj_solve_ir", "srj_schedule_optimal", "srj_schedule_order",
                 "srj_adjoint", "srj_batch_plan", "srj_batch_solve", "srj_plan_tune", "srj_batch_tune",
                 "srj_residual_static", "srj_schedule_counts", "srj_plan_operator", "srj_solve_ex",
                 "srj_plan_tune_cached", "srj_plan_poison"]:
        getattr(L, name).restype = i32
    _lib = L
    return L


def _check(st, allowed=(0,)):
    if st not in allowed:
        raise SrjError(st, lib().srj_last_error().decode())
    return st


def _dptr(t, shape=None):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Plan:
    """Owns an srj_plan_t; destroyed with the object."""

    def __init__(self, handle, n, ndim):
        self.handle = handle
        self.n = tuple(n)
        self.ndim = ndim

    @property
    def full_shape(self):
        return tuple(x + 2 for x in reversed(self.n[:self.ndim]))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.srj_plan_destroy(h)
            self.handle = None


def _fill_schedule(s, P, omega, q, kappa_min, ordering, sequence, n_eff, q_rounding, keep):
    """Fill an srj_schedule; arrays it points to are appended to keep (the caller holds them
    until the call returns)."""
    if omega is not None:
        w = np.ascontiguousarray(omega, dtype=np.float64)
        qq = np.ascontiguousarray(q, dtype=np.int64)
        keep += [w, qq]
        s.P = len(w)
        s.omega = w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        s.q = qq.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    else:
        s.P = int(P)
    s.kappa_min = float(kappa_min)
    s.n_eff = float(n_eff)
    s.q_rounding = int(q_rounding)
    s.ordering = int(ordering)
    if sequence is not None:
        sq = np.ascontiguousarray(sequence, dtype=np.int32)
        keep.append(sq)
        s.sequence = sq.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        s.M = len(sq)
        s.ordering = 2


def srj_plan(n, h, P=None, omega=None, q=None, kappa_min=0.0, ordering=0, sequence=None,
             dtype="f64", stream=None, n_eff=0.0, q_rounding=0, bc="dirichlet"):
    """Create a plan for a grid of interior sizes n = (n_x, n_y[, n_z]) and spacing h (one
    number, or one per axis).

    Either P (optimised schedule) or omega/q (explicit) is given; ordering 0 balanced,
    1 even spread, 2 explicit sequence; n_eff > 0 optimises for the Neumann table row of
    resolution n_eff; q_rounding 0 floor, 1 nearest, 2 ceiling, 3 best per level.
    """
    L = lib()
    g = _Grid()
    _fill_grid(g, n, h, dtype, bc)
    s = _Schedule()
    keep = []
    _fill_schedule(s, P, omega, q, kappa_min, ordering, sequence, n_eff, q_rounding, keep)
    out = ctypes.c_void_p()
    st = stream if stream is not None else _stream_handle()
    _check(L.srj_plan(ctypes.byref(g), ctypes.byref(s), st, ctypes.byref(out)))
    return Plan(out, n, len(n))


def srj_plan_operator(n, coef, mask=None, P=None, omega=None, q=None, kappa_min=0.0, ordering=0,
                      sequence=None, stream=None, n_eff=0.0, q_rounding=0):
    """Plan for a variable-coefficient operator: coef a float64 CUDA tensor of shape
    (2d + 1,) + full grid holding a_P, a_W, a_E, a_S, a_N (, a_D, a_U); mask an optional uint8
    CUDA tensor of the full-grid shape (nonzero = fixed point)."""
    import torch

    L = lib()
    g = _Grid()
    _fill_grid(g, n, 1.0, "f64", "dirichlet")
    full = tuple(x + 2 for x in reversed(tuple(n)))
    if not (isinstance(coef, torch.Tensor) and coef.is_cuda and coef.dtype == torch.float64 and coef.is_contiguous()
            and tuple(coef.shape) == (2 * len(n) + 1,) + full):
        raise TypeError(f"coef must be a contiguous float64 CUDA tensor of shape {(2 * len(n) + 1,) + full}")
    mp = None
    if mask is not None:
        if not (isinstance(mask, torch.Tensor) and mask.is_cuda and mask.dtype == torch.uint8 and mask.is_contiguous()
                and tuple(mask.shape) == full):
            raise TypeError("mask must be a contiguous uint8 CUDA tensor of the full-grid shape")
        mp = ctypes.c_void_p(mask.data_ptr())
    s = _Schedule()
    keep = []
    _fill_schedule(s, P, omega, q, kappa_min, ordering, sequence, n_eff, q_rounding, keep)
    out = ctypes.c_void_p()
    st = stream if stream is not None else _stream_handle()
    _check(L.srj_plan_operator(ctypes.byref(g), ctypes.byref(s), ctypes.c_void_p(coef.data_ptr()), mp, st,
                               ctypes.byref(out)))
    return Plan(out, n, len(n))


def srj_plan_describe(plan):
    d = _Desc()
    _check(lib().srj_plan_describe(plan.handle, ctypes.byref(d)))
    P = d.P
    return dict(P=P, M=d.M, omega=np.array(d.omega[:P]), beta=np.array(d.beta[:P]),
                q=np.array(d.q[:P], dtype=np.int64), kappa_min=d.kappa_min, kappa_max=d.kappa_max,
                rho=d.rho, gamma_q_max=d.gamma_q_max, prefix_peak_log10=d.prefix_peak_log10,
                suffix_peak_log10=d.suffix_peak_log10, fused_sweeps=d.fused_sweeps, resident=d.resident,
                store_nt=d.store_nt)


def srj_plan_sequence(plan):
    M = srj_plan_describe(plan)["M"]
    seq = np.zeros(M, dtype=np.int32)
    _check(lib().srj_plan_sequence(plan.handle, seq.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), M))
    return seq


def srj_plan_set_fusion(plan, fused, seg_rows=0):
    _check(lib().srj_plan_set_fusion(plan.handle, int(fused), int(seg_rows)))


def _info(i):
    return dict(sweeps=i.sweeps, cycles=i.cycles, relres=i.relres, seconds=i.seconds,
                status=STATUS.get(i.status, i.status))


def srj_solve(plan, u, f, tol, max_sweeps, raise_on_noconv=False):
    """Solve in place on u; returns the info dict (status 'ok' | 'enoconv' | 'ediverged')."""
    info = _Info()
    st = lib().srj_solve(plan.handle, _dptr(u, plan.full_shape), _dptr(f, plan.full_shape), float(tol),
                         int(max_sweeps), ctypes.byref(info))
    _check(st, (0, 5, 6) if not raise_on_noconv else (0,))
    return _info(info)


def srj_solve_ex(plan, u, f, tol, max_sweeps, start_offset=0, history_cap=0):
    """srj_solve resumed at step start_offset of a cycle and/or recording the relres of every
    check (returned as info["history"], the first history_cap checks; info["checks"] counts
    them all when history_cap > 0, and is 0 otherwise)."""
    info = _Info()
    hist = (ctypes.c_double * max(1, int(history_cap)))()
    o = _SolveOpts(tol=float(tol), max_sweeps=int(max_sweeps), start_offset=int(start_offset),
                   history=ctypes.cast(hist, ctypes.POINTER(ctypes.c_double)) if history_cap > 0 else None,
                   history_cap=int(history_cap), history_len=0)
    st = lib().srj_solve_ex(plan.handle, _dptr(u, plan.full_shape), _dptr(f, plan.full_shape), ctypes.byref(o),
                            ctypes.byref(info))
    _check(st, (0, 5, 6))
    d = _info(info)
    d["checks"] = int(o.history_len)
    d["history"] = [hist[i] for i in range(min(int(o.history_len), int(history_cap)))]
    return d


def srj_sweeps(plan, u, f, k0, nsweeps):
    """Apply nsweeps scheduled sweeps in place; returns (device seconds of the sweep
    launches, number of launches)."""
    stats = (ctypes.c_double * 2)()
    _check(lib().srj_sweeps(plan.handle, _dptr(u, plan.full_shape), _dptr(f, plan.full_shape), int(k0),
                            int(nsweeps), stats))
    return stats[0], int(stats[1])


def srj_residual(plan, u, f, r_out=None):
    norms = (ctypes.c_double * 4)()
    rp = _dptr(r_out, plan.full_shape) if r_out is not None else None
    _check(lib().srj_residual(plan.handle, _dptr(u, plan.full_shape), _dptr(f, plan.full_shape), rp, norms))
    return dict(l2=norms[0], linf=norms[1], source_l2=norms[2], relres=norms[3])


def srj_residual_static(n, h, u, f, norms, r_out=None, stream=None):
    """Residual norms of u without a plan and without allocating device memory: writes
    (||r||_2, max |r|, ||b~||_2, relres) into the device tensor norms (4 float64) on the
    stream, asynchronously; r_out (optional) receives r with a zero ring."""
    g = _Grid()
    _fill_grid(g, n, h, SRJ_F64)
    shape = tuple(x + 2 for x in reversed(tuple(n)))
    if norms.numel() < 4:
        raise ValueError("norms needs 4 elements")
    st = stream if stream is not None else _stream_handle()
    _check(lib().srj_residual_static(ctypes.byref(g), _dptr(u, shape), _dptr(f, shape),
                                     _dptr(r_out, shape) if r_out is not None else None, _dptr(norms), st))


def srj_solve_ir(plan, u, f, tol, inner_cycles, max_outer):
    info = _Info()
    st = lib().srj_solve_ir(plan.handle, _dptr(u, plan.full_shape), _dptr(f, plan.full_shape), float(tol),
                            int(inner_cycles), int(max_outer), ctypes.byref(info))
    _check(st, (0, 5, 6))
    return _info(info)


def srj_adjoint(plan, grad_u, tol, max_sweeps, df=None, dg=None):
    """Adjoint solve: A lambda = grad_u, then df = h^2 lambda, dg = boundary gather of
    lambda (device tensors, full layout; either may be None).  Returns the info dict."""
    info = _Info()
    st = lib().srj_adjoint(plan.handle, _dptr(grad_u, plan.full_shape), float(tol), int(max_sweeps),
                           _dptr(df, plan.full_shape) if df is not None else None,
                           _dptr(dg, plan.full_shape) if dg is not None else None, ctypes.byref(info))
    _check(st, (0, 5, 6))
    return _info(info)


class Batch:
    """Owns an srj_batch_t."""

    def __init__(self, handle, shapes):
        self.handle = handle
        self.shapes = shapes  # full-grid shapes (ny + 2, nx + 2)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.srj_batch_destroy(h)
            self.handle = None


def srj_batch_plan(problems, dtype="f32", stream=None):
    """problems: list of dicts with n = (n_x, n_y), h, and either P or omega/q (optionally
    sequence, kappa_min, ordering)."""
    L = lib()
    cnt = len(problems)
    grids = (_Grid * cnt)()
    scheds = (_Schedule * cnt)()
    keep = []
    for j, pr in enumerate(problems):
        g = grids[j]
        _fill_grid(g, pr["n"], pr["h"], dtype)
        s = scheds[j]
        if pr.get("omega") is not None:
            w = np.ascontiguousarray(pr["omega"], dtype=np.float64)
            qq = np.ascontiguousarray(pr["q"], dtype=np.int64)
            keep += [w, qq]
            s.P = len(w)
            s.omega = w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            s.q = qq.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        else:
            s.P = int(pr["P"])
        s.kappa_min = float(pr.get("kappa_min", 0.0))
        s.n_eff = float(pr.get("n_eff", 0.0))
        s.q_rounding = int(pr.get("q_rounding", 0))
        s.ordering = int(pr.get("ordering", 0))
        if pr.get("sequence") is not None:
            sq = np.ascontiguousarray(pr["sequence"], dtype=np.int32)
            keep.append(sq)
            s.sequence = sq.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            s.M = len(sq)
            s.ordering = 2
    out = ctypes.c_void_p()
    st = stream if stream is not None else _stream_handle()
    _check(L.srj_batch_plan(cnt, grids, scheds, st, ctypes.byref(out)))
    return Batch(out, [(int(p["n"][1]) + 2, int(p["n"][0]) + 2) for p in problems])


def srj_batch_solve(batch, us, fs, tol, inner_cycles=1, max_outer=1000):
    """Solve every problem in place; returns (list of info dicts, seconds array)."""
    cnt = len(batch.shapes)
    if len(us) != cnt or len(fs) != cnt:
        raise ValueError("one u and one f per problem")
    up = (ctypes.c_void_p * cnt)(*[_dptr(u, sh).value for u, sh in zip(us, batch.shapes)])
    fp = (ctypes.c_void_p * cnt)(*[_dptr(f, sh).value for f, sh in zip(fs, batch.shapes)])
    infos = (_Info * cnt)()
    secs = (ctypes.c_double * cnt)()
    st = lib().srj_batch_solve(batch.handle, up, fp, float(tol), int(inner_cycles), int(max_outer), infos, secs)
    _check(st, (0, 5, 6))
    return [_info(i) for i in infos], np.array(secs[:])


def srj_schedule_optimal(P, kappa_min, kappa_max=2.0):
    w = np.zeros(P)
    b = np.zeros(P)
    q = np.zeros(P, dtype=np.int64)
    k = np.zeros(max(P - 1, 1))
    _check(lib().srj_schedule_optimal(int(P), float(kappa_min), float(kappa_max),
                                      w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      q.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                      k.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return dict(w=w, beta=b, q=q, kappa=k[:P - 1])


def srj_schedule_counts(beta, q_rounding=0, omega=None, kappa_min=0.0, kappa_max=2.0):
    """Integer counts from fractions (Sec. 4.3): 0 floor, 1 nearest, 2 ceiling, 3 best
    floor/ceiling combination for the weights omega on [kappa_min, kappa_max]."""
    b = np.ascontiguousarray(beta, dtype=np.float64)
    w = np.ascontiguousarray(omega, dtype=np.float64) if omega is not None else None
    q = np.zeros(len(b), dtype=np.int64)
    _check(lib().srj_schedule_counts(len(b), b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if w is not None else None,
                                     float(kappa_min), float(kappa_max), int(q_rounding),
                                     q.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
    return q


def srj_schedule_order(omega, q, kappa_min, kappa_max=2.0, ordering=0):
    w = np.ascontiguousarray(omega, dtype=np.float64)
    qq = np.ascontiguousarray(q, dtype=np.int64)
    seq = np.zeros(int(qq.sum()), dtype=np.int32)
    _check(lib().srj_schedule_order(len(w), w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    qq.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), float(kappa_min),
                                    float(kappa_max), int(ordering),
                                    seq.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return seq


def _tune_dict(t):
    return dict(fused_sweeps=t.fused_sweeps, seg_rows=t.seg_rows, candidates=t.candidates,
                us_per_sweep=t.us_per_sweep, us_per_sweep_before=t.us_per_sweep_before)


def srj_plan_tune(plan):
    """Time candidate launch shapes on the plan's scratch fields and keep the fastest."""
    t = _Tune()
    _check(lib().srj_plan_tune(plan.handle, ctypes.byref(t)))
    return _tune_dict(t)


def srj_plan_tune_cached(plan, path):
    """srj_plan_tune through the on-disk cache at path (candidates = 0 on a cache hit)."""
    t = _Tune()
    _check(lib().srj_plan_tune_cached(plan.handle, os.fsencode(path), ctypes.byref(t)))
    return _tune_dict(t)


def srj_plan_poison(plan):
    """Fill the plan's iterate, source and reduction buffers, padding included, with NaN bytes."""
    _check(lib().srj_plan_poison(plan.handle))


def srj_batch_tune(batch):
    """Time candidate largest tile heights of the batch's sweep launch and keep the fastest."""
    t = _Tune()
    _check(lib().srj_batch_tune(batch.handle, ctypes.byref(t)))
    return _tune_dict(t)
