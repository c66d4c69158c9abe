"""ctypes binding of libifgf (argument marshalling only).

Every computation happens in the HIP library; this module converts torch
tensors and numpy arrays into the pointers and sizes of the C-ABI declared in
include/ifgf.h and raises on any non-zero status.  If the shared library is
missing the import fails loudly: there is no Python fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libifgf.so")

IFGF_FP64 = 0
IFGF_FP32 = 1
IFGF_WNOCONV = 1
IFGF_EDEVICE = -5
IFGF_DERIV_ANALYTIC = 0
IFGF_DERIV_FD = 1


class IFGFError(RuntimeError):
    def __init__(self, msg, code=None):
        super().__init__(msg)
        self.code = code


class Options(C.Structure):
    _fields_ = [("Ps", C.c_int), ("Pa", C.c_int), ("ns_init", C.c_int), ("na_init", C.c_int),
                ("refine_radial", C.c_int), ("leaf_wavelengths", C.c_double),
                ("precision", C.c_int), ("max_nrhs", C.c_int), ("host_only", C.c_int),
                ("batch_columns", C.c_int), ("fp32_workspaces", C.c_int), ("verbose", C.c_int),
                ("deriv_mode", C.c_int), ("target_chunk_pairs", C.c_int64), ("plan_on_device", C.c_int),
                ("keep_pair_tables", C.c_int), ("kernel_at_a_time", C.c_int),
                ("cone_memory_budget", C.c_int64), ("target_tiles", C.c_int)]


class NMullerParams(C.Structure):
    _fields_ = [("P", C.c_int), ("Nc", C.c_int), ("eps_e", C.c_double), ("eps_i", C.c_double),
                ("mu_e", C.c_double), ("mu_i", C.c_double), ("omega", C.c_double),
                ("delta_factor", C.c_double), ("nbeta", C.c_int), ("d_cov", C.c_int),
                ("corrections_on_host", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("converged", C.c_int), ("true_relres", C.c_double),
                ("arnoldi_relres", C.c_double), ("seconds", C.c_double),
                ("precond_iters", C.c_int), ("fallbacks", C.c_int), ("residual_fp64", C.c_int)]


_lib = None


def lib():
    """Load libifgf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # torch ships its own libamdhip64.so.7; libifgf.so needs the same soname.
        # Loading torch first makes the process use one HIP runtime: the one
        # that owns the device memory and streams handed to the library.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libifgf.so not found at {LIB_PATH}: run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i64, dbl, ci = C.c_void_p, C.c_int64, C.c_double, C.c_int
        L.ifgf_default_options.argtypes = [C.POINTER(Options)]
        L.ifgf_default_options.restype = None
        L.ifgf_plan.argtypes = [C.POINTER(vp), i64, vp, vp, vp, dbl, dbl, dbl, C.POINTER(Options)]
        L.ifgf_apply.argtypes = [vp, vp, ci, vp, vp]
        L.ifgf_plan_counts.argtypes = [vp, C.POINTER(i64), ci]
        L.ifgf_plan_table.argtypes = [vp, ci, C.POINTER(i64), i64, C.POINTER(i64)]
        L.ifgf_stats.argtypes = [vp, C.c_char_p, C.c_size_t]
        L.ifgf_set_timing.argtypes = [vp, ci]
        L.ifgf_set_timing.restype = ci
        L.ifgf_set_precision.argtypes = [vp, ci, C.POINTER(ci)]
        L.ifgf_precisions.argtypes = [vp]
        L.ifgf_precisions.restype = ci
        L.ifgf_autotune.argtypes = [vp, vp, C.POINTER(ci)]
        L.ifgf_check.argtypes = [vp, vp, C.POINTER(C.c_uint)]
        L.ifgf_dipole_field.argtypes = [i64, vp, dbl, dbl, dbl, vp, vp, vp, vp]
        L.ifgf_dipole_field.restype = ci
        L.ifgf_set_normals.argtypes = [vp, vp]
        L.ifgf_set_normals.restype = ci
        L.ifgf_eval_plan.argtypes = [C.POINTER(vp), i64, vp, vp, i64, vp, vp, dbl, dbl, dbl, C.POINTER(Options)]
        L.ifgf_eval_plan.restype = ci
        L.ifgf_eval_apply.argtypes = [vp, vp, ci, vp, vp]
        L.ifgf_eval_apply.restype = ci
        L.ifgf_eval_set_directions.argtypes = [vp, vp]
        L.ifgf_eval_set_directions.restype = ci
        L.ifgf_eval_ifgf.argtypes = [vp]
        L.ifgf_eval_ifgf.restype = vp
        L.ifgf_eval_destroy.argtypes = [vp]
        L.ifgf_eval_destroy.restype = None
        L.ifgf_set_lock_spin_limit.argtypes = [vp, ci]
        L.ifgf_autotune.restype = ci
        L.ifgf_set_precision.restype = ci
        L.ifgf_destroy.argtypes = [vp]
        L.ifgf_destroy.restype = None
        L.ifgf_last_error.restype = C.c_char_p
        L.nmuller_default_params.argtypes = [C.POINTER(NMullerParams)]
        L.nmuller_default_params.restype = None
        L.nmuller_plan.argtypes = [C.POINTER(vp), C.POINTER(NMullerParams), vp, vp, vp, dbl,
                                   C.POINTER(Options)]
        L.nmuller_apply.argtypes = [vp, vp, ci, vp, vp]
        L.nmuller_rhs.argtypes = [vp, vp, vp, ci, vp, vp]
        L.nmuller_geometry.argtypes = [vp, ci, vp, i64]
        L.nmuller_corrections.argtypes = [vp, C.POINTER(i64), vp, vp, vp]
        L.nmuller_plan_info.argtypes = [vp, vp, ci]
        L.nmuller_solve.argtypes = [vp, vp, ci, vp, ci, dbl, ci, ci, C.POINTER(SolveInfo), vp]
        L.nmuller_solve_noalloc.argtypes = [vp, vp, vp, ci, dbl, ci, ci, C.POINTER(SolveInfo), vp]
        L.nmuller_solve_noalloc.restype = ci
        L.nmuller_solve.restype = ci
        L.nmuller_solve_trajectory.argtypes = [vp, vp, vp, dbl, ci, ci, vp, vp, ci, C.POINTER(ci),
                                               C.POINTER(SolveInfo), vp]
        L.nmuller_solve_trajectory.restype = ci
        L.nmuller_set_preconditioner.argtypes = [vp, vp, vp, ci, ci]
        L.nmuller_precond_apply.argtypes = [vp, vp, vp, ci, vp]
        L.nmuller_precond_pairs.argtypes = [vp, vp, vp, ci, vp, vp, vp]
        L.nmuller_patch_features.argtypes = [vp, vp, i64]
        L.mlp_create.argtypes = [C.POINTER(vp), ci, vp, ci, ci]
        L.mlp_num_params.argtypes = [vp, C.POINTER(i64)]
        L.mlp_set_params.argtypes = [vp, vp]
        L.mlp_get_params.argtypes = [vp, vp, vp]
        L.mlp_get_grad.argtypes = [vp, vp, vp]
        L.mlp_forward.argtypes = [vp, vp, ci, vp, vp]
        L.mlp_backward.argtypes = [vp, vp, ci, vp, vp]
        L.mlp_adam_step.argtypes = [vp, C.c_float, vp]
        L.mlp_train_step.argtypes = [vp, vp, vp, vp, ci, C.c_float, vp, vp]
        L.nmuller_graph_capture.argtypes = [C.POINTER(vp), ci, vp, vp, vp, vp]
        L.ifgf_graph_launch.argtypes = [vp, vp]
        L.ifgf_graph_nodes.argtypes = [vp, C.POINTER(i64)]
        L.ifgf_graph_destroy.argtypes = [vp]
        L.ifgf_graph_destroy.restype = None
        L.mlp_destroy.argtypes = [vp]
        L.mlp_destroy.restype = None
        L.nmuller_ifgf.argtypes = [vp]
        L.nmuller_ifgf.restype = vp
        L.nmuller_destroy.argtypes = [vp]
        L.nmuller_destroy.restype = None
        for name in ("ifgf_plan", "ifgf_apply", "ifgf_plan_counts", "ifgf_plan_table", "ifgf_stats",
                     "nmuller_plan", "nmuller_apply", "nmuller_rhs", "nmuller_geometry",
                     "nmuller_corrections", "nmuller_plan_info", "nmuller_set_preconditioner", "ifgf_precisions",
                     "nmuller_precond_apply",
                     "nmuller_precond_pairs", "nmuller_patch_features", "mlp_create", "mlp_num_params",
                     "mlp_set_params", "mlp_get_params", "mlp_get_grad", "mlp_forward", "mlp_backward",
                     "mlp_adam_step", "mlp_train_step", "nmuller_graph_capture", "ifgf_graph_launch",
                     "ifgf_graph_nodes", "ifgf_check", "ifgf_set_lock_spin_limit"):
            getattr(L, name).restype = ci
        _lib = L
    return _lib


def exported_symbols():
    """Names of the C-ABI entry points declared in include/ifgf.h."""
    hdr = os.path.join(os.path.dirname(_HERE), "include")
    names = []
    import re
    for f in sorted(os.listdir(hdr)):
        if f.endswith(".h"):
            txt = open(os.path.join(hdr, f)).read()
            names += re.findall(r"^\s*(?:int|void|const char\*)\s+(\w+)\s*\(", txt, flags=re.M)
    return names


def _check(rc, what):
    if rc < 0:
        raise IFGFError(f"{what} failed ({rc}): {lib().ifgf_last_error().decode()}", rc)
    return rc


def _stream_ptr(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return int(stream)


def _host_f64(a, shape):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def default_options():
    o = Options()
    lib().ifgf_default_options(C.byref(o))
    return o


def ifgf_plan(points, normals, weights, k_int, k_ext, tol=1e-4, **opts):
    """Build an IFGF plan; returns an opaque handle (int)."""
    x = np.asarray(points)
    n = x.shape[0]
    x = _host_f64(points, (n, 3))
    nr = _host_f64(normals, (n, 3))
    w = _host_f64(weights, (n,))
    o = default_options()
    for k, v in opts.items():
        setattr(o, k, v)
    h = C.c_void_p()
    _check(lib().ifgf_plan(C.byref(h), n, x.ctypes.data, nr.ctypes.data, w.ctypes.data,
                           float(k_int), float(k_ext), float(tol), C.byref(o)), "ifgf_plan")
    return h.value


def ifgf_apply(plan, densities, nrhs, out, stream=None):
    """densities: device [nrhs][8][n] complex128; out: device [nrhs][2][14][n] complex128."""
    _check(lib().ifgf_apply(plan, densities.data_ptr(), int(nrhs), out.data_ptr(),
                            _stream_ptr(stream)), "ifgf_apply")


def ifgf_plan_counts(plan, ncount=64):
    buf = (C.c_int64 * ncount)()
    _check(lib().ifgf_plan_counts(plan, buf, ncount), "ifgf_plan_counts")
    return list(buf)


def ifgf_plan_table(plan, which):
    cnt = C.c_int64()
    _check(lib().ifgf_plan_table(plan, int(which), None, 0, C.byref(cnt)), "ifgf_plan_table")
    arr = np.zeros(cnt.value, dtype=np.int64)
    _check(lib().ifgf_plan_table(plan, int(which), arr.ctypes.data_as(C.POINTER(C.c_int64)),
                                 cnt.value, C.byref(cnt)), "ifgf_plan_table")
    return arr


def ifgf_stats(plan):
    import json
    buf = C.create_string_buffer(1 << 16)
    _check(lib().ifgf_stats(plan, buf, len(buf)), "ifgf_stats")
    return json.loads(buf.value.decode())


def ifgf_set_timing(plan, on):
    _check(lib().ifgf_set_timing(plan, int(bool(on))), "ifgf_set_timing")


def ifgf_autotune(plan, stream=None):
    """Pick the fastest column batch (1, 2 or 4 RHS per pass); returns it."""
    r = C.c_int(0)
    _check(lib().ifgf_autotune(plan, _stream_ptr(stream), C.byref(r)), "ifgf_autotune")
    return r.value


def ifgf_set_precision(plan, precision):
    """Switch a built plan to IFGF_FP64 or IFGF_FP32; returns the previous one."""
    prev = C.c_int(0)
    _check(lib().ifgf_set_precision(plan, int(precision), C.byref(prev)), "ifgf_set_precision")
    return prev.value


def ifgf_check(plan, stream=None):
    """Synchronise and read the plan's device error word; raises IFGFError
    (code IFGF_EDEVICE) if a kernel reported a failure since the last check."""
    flags = C.c_uint(0)
    _check(lib().ifgf_check(plan, _stream_ptr(stream), C.byref(flags)), "ifgf_check")
    return flags.value


def ifgf_set_lock_spin_limit(plan, limit):
    _check(lib().ifgf_set_lock_spin_limit(plan, int(limit)), "ifgf_set_lock_spin_limit")


def ifgf_dipole_field(points, k, eps, omega, p, x0, beam, stream=None):
    """E, H [n][3] complex128 device tensors of a dipole p (3 complex) at the
    complex source point x0 + i beam; points: device [n][3] float64."""
    import torch
    n = points.shape[0]
    if points.dtype != torch.float64 or not points.is_contiguous() or tuple(points.shape[1:]) != (3,):
        raise ValueError("points must be a contiguous float64 device tensor [n, 3]")
    p = np.asarray(p, dtype=np.complex128)
    dip = np.concatenate([np.stack([p.real, p.imag], axis=1).ravel(), np.asarray(x0, float),
                          np.asarray(beam, float)]).astype(np.float64)
    E = torch.empty((n, 3), dtype=torch.complex128, device=points.device)
    H = torch.empty_like(E)
    _check(lib().ifgf_dipole_field(int(n), points.data_ptr(), float(k), float(eps), float(omega),
                                   dip.ctypes.data, E.data_ptr(), H.data_ptr(), _stream_ptr(stream)),
           "ifgf_dipole_field")
    return E, H


def ifgf_destroy(plan):
    if plan:
        lib().ifgf_destroy(plan)


class IFGFEval:
    """Sums at target points other than the sources (ifgf_eval_*)."""

    def __init__(self, src, weights, tgt, dirs, k_int, k_ext, tol=1e-4, **opts):
        ns = int(np.asarray(src).shape[0])
        self.nt = int(np.asarray(tgt).shape[0])
        self.ns = ns
        self.max_nrhs = int(opts.get("max_nrhs", 1))
        x = _host_f64(src, (ns, 3))
        w = _host_f64(weights, (ns,))
        t = _host_f64(tgt, (self.nt, 3))
        d = _host_f64(dirs, (self.nt, 3))
        o = default_options()
        for k, v in opts.items():
            setattr(o, k, v)
        h = C.c_void_p()
        _check(lib().ifgf_eval_plan(C.byref(h), ns, x.ctypes.data, w.ctypes.data, self.nt, t.ctypes.data,
                                    d.ctypes.data, float(k_int), float(k_ext), float(tol), C.byref(o)),
               "ifgf_eval_plan")
        self.handle = h.value

    def set_directions(self, dirs):
        d = _host_f64(dirs, (self.nt, 3))
        _check(lib().ifgf_eval_set_directions(self.handle, d.ctypes.data), "ifgf_eval_set_directions")

    def apply(self, densities, out=None, stream=None):
        import torch
        nrhs = densities.shape[0]
        if densities.dtype != torch.complex128 or not densities.is_contiguous() or \
                tuple(densities.shape[1:]) != (8, self.ns):
            raise ValueError(f"densities must be a contiguous complex128 tensor [nrhs, 8, {self.ns}]")
        if out is None:
            out = torch.empty((nrhs, 2, 14, self.nt), dtype=torch.complex128, device=densities.device)
        _check(lib().ifgf_eval_apply(self.handle, densities.data_ptr(), int(nrhs), out.data_ptr(),
                                     _stream_ptr(stream)), "ifgf_eval_apply")
        return out

    def close(self):
        if self.handle:
            lib().ifgf_eval_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class IFGFPlan:
    """Owning wrapper around an ifgf plan handle."""

    def __init__(self, points, normals, weights, k_int, k_ext, tol=1e-4, **opts):
        self.n = int(np.asarray(points).shape[0])
        self.max_nrhs = int(opts.get("max_nrhs", 1))
        self.handle = ifgf_plan(points, normals, weights, k_int, k_ext, tol, **opts)

    def apply(self, densities, out=None, stream=None):
        import torch
        nrhs = densities.shape[0]
        if densities.dtype != torch.complex128 or not densities.is_contiguous():
            raise ValueError("densities must be a contiguous complex128 device tensor")
        if tuple(densities.shape[1:]) != (8, self.n):
            raise ValueError(f"densities must have shape [nrhs, 8, {self.n}]")
        if out is None:
            out = torch.empty((nrhs, 2, 14, self.n), dtype=torch.complex128, device=densities.device)
        ifgf_apply(self.handle, densities, nrhs, out, stream)
        return out

    def counts(self):
        return ifgf_plan_counts(self.handle)

    def table(self, which):
        return ifgf_plan_table(self.handle, which)

    def stats(self):
        return ifgf_stats(self.handle)

    def set_timing(self, on=True):
        ifgf_set_timing(self.handle, on)

    def close(self):
        if self.handle:
            ifgf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def nmuller_plan(P, Nc, points, du, dv, eps_e, eps_i, mu_e=1.0, mu_i=1.0, omega=2 * np.pi,
                 tol=1e-4, delta_factor=0.0, nbeta=0, d_cov=0, corrections_on_host=0, **opts):
    """Build an N-Mueller operator plan; returns an opaque handle (int)."""
    n = P * Nc * Nc
    x = _host_f64(points, (n, 3))
    a = _host_f64(du, (n, 3))
    b = _host_f64(dv, (n, 3))
    prm = NMullerParams()
    lib().nmuller_default_params(C.byref(prm))
    prm.P, prm.Nc = int(P), int(Nc)
    prm.eps_e, prm.eps_i, prm.mu_e, prm.mu_i, prm.omega = eps_e, eps_i, mu_e, mu_i, omega
    prm.delta_factor, prm.nbeta = float(delta_factor), int(nbeta)
    if d_cov:
        prm.d_cov = int(d_cov)
    prm.corrections_on_host = int(corrections_on_host)
    o = default_options()
    for k, v in opts.items():
        setattr(o, k, v)
    h = C.c_void_p()
    _check(lib().nmuller_plan(C.byref(h), C.byref(prm), x.ctypes.data, a.ctypes.data,
                              b.ctypes.data, float(tol), C.byref(o)), "nmuller_plan")
    return h.value


def nmuller_apply(nm, y, nrhs, Ay, stream=None):
    """y, Ay: device [nrhs][4][n] complex128."""
    _check(lib().nmuller_apply(nm, y.data_ptr(), int(nrhs), Ay.data_ptr(), _stream_ptr(stream)),
           "nmuller_apply")


def nmuller_rhs(nm, E, H, nrhs, b, stream=None):
    """E, H: device [nrhs][n][3] complex128; b: device [nrhs][4][n] complex128."""
    _check(lib().nmuller_rhs(nm, E.data_ptr(), H.data_ptr(), int(nrhs), b.data_ptr(),
                             _stream_ptr(stream)), "nmuller_rhs")


def nmuller_geometry(nm, which, n):
    shape = (n,) if which in (1, 4) else (n, 3)
    out = np.zeros(shape)
    _check(lib().nmuller_geometry(nm, int(which), out.ctypes.data, out.size), "nmuller_geometry")
    return out


def nmuller_corrections(nm, n, nc, values=True):
    npairs = C.c_int64()
    _check(lib().nmuller_corrections(nm, C.byref(npairs), None, None, None), "nmuller_corrections")
    ro = np.zeros(n + 1, dtype=np.int64)
    pp = np.zeros(npairs.value, dtype=np.int32)
    vals = np.zeros((npairs.value, 4, nc * nc, 2)) if values else None
    _check(lib().nmuller_corrections(nm, C.byref(npairs), ro.ctypes.data, pp.ctypes.data,
                                     vals.ctypes.data if values else None), "nmuller_corrections")
    if values:
        vals = vals[..., 0] + 1j * vals[..., 1]
    return ro, pp, vals


def nmuller_solve(nm, rhs, nrhs, y, use_x0=False, rtol=1e-4, maxit=500, restart=0, stream=None):
    """GMRES; rhs, y device [nrhs][4][n] complex128.  Returns a list of dicts."""
    info = (SolveInfo * int(nrhs))()
    _check(lib().nmuller_solve(nm, rhs.data_ptr(), int(nrhs), y.data_ptr(), int(bool(use_x0)),
                               float(rtol), int(maxit), int(restart), info, _stream_ptr(stream)),
           "nmuller_solve")
    return [_info_dict(i) for i in info]


def nmuller_solve_noalloc(nm, rhs, y, use_x0=False, rtol=1e-4, maxit=500, restart=0, stream=None):
    """One-RHS GMRES in the library's static scratch; rhs, y device [1][4][n]
    complex128.  Returns the info dict."""
    info = SolveInfo()
    _check(lib().nmuller_solve_noalloc(nm, rhs.data_ptr(), y.data_ptr(), int(bool(use_x0)), float(rtol),
                                       int(maxit), int(restart), C.byref(info), _stream_ptr(stream)),
           "nmuller_solve_noalloc")
    return _info_dict(info)


def _info_dict(i):
    return {"iters": i.iters, "converged": bool(i.converged), "true_relres": i.true_relres,
            "arnoldi_relres": i.arnoldi_relres, "seconds": i.seconds,
            "precond_iters": i.precond_iters, "fallbacks": i.fallbacks, "residual_fp64": bool(i.residual_fp64)}


def nmuller_solve_trajectory(nm, rhs, y, X, R, rtol=1e-4, maxit=500, stride=1, stream=None):
    """Unrestarted GMRES from 0 recording (x_k, r_k) every `stride` iterations
    into X, R (device [cap][4][n] complex128).  Returns (count, info dict)."""
    info = SolveInfo()
    nrec = C.c_int(0)
    _check(lib().nmuller_solve_trajectory(nm, rhs.data_ptr(), y.data_ptr(), float(rtol), int(maxit),
                                          int(stride), X.data_ptr(), R.data_ptr(), int(X.shape[0]),
                                          C.byref(nrec), C.byref(info), _stream_ptr(stream)),
           "nmuller_solve_trajectory")
    return nrec.value, _info_dict(info)


class NMullerGraph:
    """One HIP graph replaying op.apply(y, Ay) for several (op, y, Ay):
    many bodies and right-hand sides in a single launch.  The tensors are
    referenced, not copied: keep them alive while the graph exists."""

    def __init__(self, ops, ys, Ays):
        if not (len(ops) == len(ys) == len(Ays)) or not ops:
            raise ValueError("need equally many operators, inputs and outputs")
        for op, y, a in zip(ops, ys, Ays):
            if y.shape != a.shape or tuple(y.shape[1:]) != (4, op.n) or not (y.is_contiguous() and a.is_contiguous()):
                raise ValueError(f"y and Ay must be contiguous [nrhs, 4, {op.n}] tensors")
        k = len(ops)
        self._keep = (list(ys), list(Ays))
        h = C.c_void_p()
        arr_ops = (C.c_void_p * k)(*[op.handle for op in ops])
        arr_y = (C.c_void_p * k)(*[y.data_ptr() for y in ys])
        arr_a = (C.c_void_p * k)(*[a.data_ptr() for a in Ays])
        arr_n = (C.c_int * k)(*[int(y.shape[0]) for y in ys])
        _check(lib().nmuller_graph_capture(C.byref(h), k, arr_ops, arr_y, arr_n, arr_a), "nmuller_graph_capture")
        self.handle = h.value
        n = C.c_int64()
        _check(lib().ifgf_graph_nodes(self.handle, C.byref(n)), "ifgf_graph_nodes")
        self.nodes = n.value

    def launch(self, stream=None):
        _check(lib().ifgf_graph_launch(self.handle, _stream_ptr(stream)), "ifgf_graph_launch")

    def close(self):
        if self.handle:
            lib().ifgf_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


MLP_BF16 = 0
MLP_FP32 = 1


def _dims_arr(dims):
    return (C.c_int * len(dims))(*[int(d) for d in dims])


def nmuller_set_preconditioner(nm, params, dims, dtype=MLP_BF16):
    if params is None:
        _check(lib().nmuller_set_preconditioner(nm, None, None, 0, int(dtype)), "nmuller_set_preconditioner")
        return
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
    _check(lib().nmuller_set_preconditioner(nm, p.ctypes.data, _dims_arr(dims), len(dims) - 1, int(dtype)),
           "nmuller_set_preconditioner")


def nmuller_precond_apply(nm, v, z, stream=None):
    """v, z: device [nvec][4][n] complex128."""
    _check(lib().nmuller_precond_apply(nm, v.data_ptr(), z.data_ptr(), int(v.shape[0]), _stream_ptr(stream)),
           "nmuller_precond_apply")


def nmuller_precond_pairs(nm, R, E, X, T, stream=None):
    """R, E: device [npairs][4][n] complex128; X, T: device float32 rows."""
    _check(lib().nmuller_precond_pairs(nm, R.data_ptr(), E.data_ptr(), int(R.shape[0]), X.data_ptr(),
                                       T.data_ptr(), _stream_ptr(stream)), "nmuller_precond_pairs")


def nmuller_patch_features(nm, P):
    out = np.zeros((P, 4), dtype=np.float32)
    _check(lib().nmuller_patch_features(nm, out.ctypes.data, out.size), "nmuller_patch_features")
    return out


class MLP:
    """Owning wrapper around an mlp_t network (device-resident)."""

    def __init__(self, dims, dtype=MLP_BF16, max_batch=1024):
        self.dims = [int(d) for d in dims]
        self.dtype = int(dtype)
        self.max_batch = int(max_batch)
        h = C.c_void_p()
        _check(lib().mlp_create(C.byref(h), len(dims) - 1, _dims_arr(dims), self.dtype, self.max_batch),
               "mlp_create")
        self.handle = h.value
        n = C.c_int64()
        _check(lib().mlp_num_params(self.handle, C.byref(n)), "mlp_num_params")
        self.n_params = n.value

    def set_params(self, theta):
        p = np.ascontiguousarray(np.asarray(theta, dtype=np.float32))
        if p.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {p.size}")
        _check(lib().mlp_set_params(self.handle, p.ctypes.data), "mlp_set_params")

    def params(self, stream=None):
        out = np.zeros(self.n_params, dtype=np.float32)
        _check(lib().mlp_get_params(self.handle, out.ctypes.data, _stream_ptr(stream)), "mlp_get_params")
        return out

    def grad(self, stream=None):
        out = np.zeros(self.n_params, dtype=np.float32)
        _check(lib().mlp_get_grad(self.handle, out.ctypes.data, _stream_ptr(stream)), "mlp_get_grad")
        return out

    def _f32(self, t, cols):
        import torch
        if t.dtype != torch.float32 or not t.is_contiguous() or t.shape[-1] != cols:
            raise ValueError(f"expected a contiguous float32 device tensor with {cols} columns")
        return t

    def forward(self, X, Y=None, stream=None):
        import torch
        X = self._f32(X, self.dims[0])
        if Y is None:
            Y = torch.empty((X.shape[0], self.dims[-1]), dtype=torch.float32, device=X.device)
        _check(lib().mlp_forward(self.handle, X.data_ptr(), int(X.shape[0]), Y.data_ptr(), _stream_ptr(stream)),
               "mlp_forward")
        return Y

    def backward(self, dY, dX=None, stream=None):
        dY = self._f32(dY, self.dims[-1])
        _check(lib().mlp_backward(self.handle, dY.data_ptr(), int(dY.shape[0]),
                                  dX.data_ptr() if dX is not None else None, _stream_ptr(stream)),
               "mlp_backward")
        return dX

    def adam_step(self, lr, stream=None):
        _check(lib().mlp_adam_step(self.handle, float(lr), _stream_ptr(stream)), "mlp_adam_step")

    def train_step(self, X, T, idx, lr, loss, stream=None):
        """idx: device int32 [B]; loss: device float32 [1]."""
        _check(lib().mlp_train_step(self.handle, X.data_ptr(), T.data_ptr(), idx.data_ptr(), int(idx.shape[0]),
                                    float(lr), loss.data_ptr(), _stream_ptr(stream)), "mlp_train_step")

    def close(self):
        if self.handle:
            lib().mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def nmuller_destroy(nm):
    if nm:
        lib().nmuller_destroy(nm)


class NMullerOperator:
    """Owning wrapper around an N-Mueller plan."""

    def __init__(self, surface, eps_e, eps_i, mu_e=1.0, mu_i=1.0, omega=2 * np.pi, tol=1e-4,
                 **kw):
        self.n = surface.n
        self.P, self.Nc = surface.P, surface.nc
        self.max_nrhs = int(kw.get("max_nrhs", 1))
        self.handle = nmuller_plan(surface.P, surface.nc, surface.x, surface.du, surface.dv,
                                   eps_e, eps_i, mu_e, mu_i, omega, tol, **kw)

    def apply(self, y, out=None, stream=None):
        import torch
        if y.dtype != torch.complex128 or not y.is_contiguous() or tuple(y.shape[1:]) != (4, self.n):
            raise ValueError(f"y must be a contiguous complex128 tensor [nrhs, 4, {self.n}]")
        if out is None:
            out = torch.empty_like(y)
        nmuller_apply(self.handle, y, y.shape[0], out, stream)
        return out

    def rhs(self, E, H, stream=None):
        import torch
        nrhs = E.shape[0]
        b = torch.empty((nrhs, 4, self.n), dtype=torch.complex128, device=E.device)
        nmuller_rhs(self.handle, E.contiguous(), H.contiguous(), nrhs, b, stream)
        return b

    def solve(self, b, y=None, rtol=1e-4, maxit=500, restart=0, stream=None):
        import torch
        use_x0 = y is not None
        if y is None:
            y = torch.empty_like(b)
        info = nmuller_solve(self.handle, b.contiguous(), b.shape[0], y, use_x0, rtol, maxit, restart,
                             stream)
        return y, info

    def geometry(self, which):
        return nmuller_geometry(self.handle, which, self.n)

    def corrections(self, values=True):
        return nmuller_corrections(self.handle, self.n, self.Nc, values)

    def plan_info(self):
        """Where and how fast the corrections were built, their pair count and bytes."""
        buf = (C.c_double * 4)()
        _check(lib().nmuller_plan_info(self.handle, buf, 4), "nmuller_plan_info")
        return {"corrections_on_device": bool(buf[0]), "corrections_seconds": buf[1],
                "correction_pairs": int(buf[2]), "correction_bytes": int(buf[3])}

    def solve_trajectory(self, b, X, R, rtol=1e-4, maxit=500, stride=1, stream=None):
        import torch
        y = torch.empty_like(b[0] if b.dim() == 3 else b)
        cnt, info = nmuller_solve_trajectory(self.handle, b.contiguous(), y, X, R, rtol, maxit, stride, stream)
        return y, cnt, info

    def set_preconditioner(self, params, dims=None, dtype=MLP_BF16):
        nmuller_set_preconditioner(self.handle, params, dims, dtype)

    def precond_apply(self, v, z=None, stream=None):
        import torch
        if z is None:
            z = torch.empty_like(v)
        nmuller_precond_apply(self.handle, v, z, stream)
        return z

    def precond_pairs(self, R, E, stream=None):
        import torch
        npairs, nq = R.shape[0], self.Nc * self.Nc
        X = torch.empty((npairs * self.P, 8 * nq + 4), dtype=torch.float32, device=R.device)
        T = torch.empty((npairs * self.P, 8 * nq), dtype=torch.float32, device=R.device)
        nmuller_precond_pairs(self.handle, R, E, X, T, stream)
        return X, T

    def patch_features(self):
        return nmuller_patch_features(self.handle, self.P)

    def ifgf_handle(self):
        return lib().nmuller_ifgf(self.handle)

    def close(self):
        if self.handle:
            nmuller_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
