"""Thin ctypes binding of liblmfmm.so (the C-ABI in include/lmfmm.h).

Argument marshalling only: every step of the computation runs inside the
library (host runtime + HIP kernels).  torch provides device memory and the
current stream.  There is no fallback: if the library is missing or a call
fails, an exception is raised.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblmfmm.so")

LM_OK, LM_NOT_CONVERGED = 0, 1
LM_FP64, LM_MIXED = 0, 1
LM_AUTO, LM_DENSE, LM_FMM = 0, 1, 2
LM_BC_DIRICHLET, LM_BC_NEUMANN, LM_BC_ROBIN = 0, 1, 2
LM_QUAD_LOWEST, LM_QUAD_SPECTRAL = 0, 1

_lib = None


class LmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lmfmm status {status}: {msg}")
        self.status = status


class GeomOpts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int), ("p", ctypes.c_int), ("leaf_size", ctypes.c_int), ("precond", ctypes.c_int),
                ("top_fft", ctypes.c_int), ("bc", ctypes.c_int), ("robin_beta", ctypes.c_double),
                ("quad", ctypes.c_int)]


class GmresOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("restart", ctypes.c_int),
                ("precond", ctypes.c_int)]


class SolveReport(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("rel_residual", ctypes.c_double)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_active_rhs", ctypes.c_int), ("precision", ctypes.c_int),
                ("precond_fp64", ctypes.c_int)]


class Request(ctypes.Structure):
    _fields_ = [("geom", ctypes.c_void_p), ("n_rhs", ctypes.c_int), ("theta_rad", ctypes.POINTER(ctypes.c_double)),
                ("gmres", GmresOpts), ("n_obs", ctypes.c_int), ("obs_rad", ctypes.POINTER(ctypes.c_double))]


LM_QUEUED, LM_RUNNING, LM_DONE, LM_FAILED, LM_CANCELLED = 0, 1, 2, 3, 4
LM_ENOMEM, LM_ENOTFOUND, LM_ECANCELLED = -2, -4, -5


_vp, _dp, _ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
_SIGS = {
    "lm_last_error": ([], ctypes.c_char_p),
    "lm_version": ([], ctypes.c_char_p),
    "lm_create_layers": ([_ip, _dp, _dp, _dp, ctypes.POINTER(_vp)], _ip),
    "lm_destroy_layers": ([_vp], _ip),
    "lm_create_geometry": ([_vp, _ip, ctypes.POINTER(ctypes.c_int64), _dp, ctypes.POINTER(GeomOpts), _vp,
                            ctypes.POINTER(_vp)], _ip),
    "lm_geometry_info": ([_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                          ctypes.POINTER(ctypes.c_int)], _ip),
    "lm_geometry_elements": ([_vp, _dp, _dp, _dp, ctypes.POINTER(ctypes.c_int32)], _ip),
    "lm_geometry_normals": ([_vp, _dp, _dp], _ip),
    "lm_destroy_geometry": ([_vp], _ip),
    "lm_fmm_stats": ([_vp, ctypes.POINTER(ctypes.c_int64)], _ip),
    "lm_matvec": ([_vp, _ip, _ip, _vp, _vp, _vp], _ip),
    "lm_matvec_noalloc": ([_vp, _ip, _ip, _vp, _vp, _vp], _ip),
    "lm_precond_apply": ([_vp, _ip, _ip, _vp, _vp, _vp], _ip),
    "lm_precond_subdomains": ([_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)], _ip),
    "lm_matvec_stage_times": ([_vp, _ip, _ip, _vp, _vp, _ip, _vp, _dp], _ip),
    "lm_rhs": ([_vp, _ip, _dp, _vp, _vp], _ip),
    "lm_gmres_solve": ([_vp, _ip, _ip, _dp, ctypes.POINTER(GmresOpts), _vp, ctypes.POINTER(SolveReport), _vp], _ip),
    "lm_gmres_solve_rhs": ([_vp, _ip, _ip, _vp, ctypes.POINTER(GmresOpts), _vp, ctypes.POINTER(SolveReport), _vp],
                           _ip),
    "lm_far_field": ([_vp, _ip, _vp, _ip, _dp, _vp, _vp], _ip),
    "lm_point_source_rhs": ([_vp, _ip, _dp, _vp, _vp], _ip),
    "lm_point_far_field": ([_vp, _ip, _dp, _ip, _dp, _vp, _vp], _ip),
    "lm_field": ([_vp, _ip, _vp, _ip, _dp, _vp, _vp], _ip),
    "lm_point_field": ([_vp, _ip, _dp, _ip, _dp, _vp, _vp], _ip),
    "lm_server_create": ([ctypes.POINTER(ServerOpts), ctypes.POINTER(_vp)], _ip),
    "lm_submit": ([_vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)], _ip),
    "lm_poll": ([_vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(SolveReport), _dp, _vp, _vp], _ip),
    "lm_cancel": ([_vp, ctypes.c_uint64], _ip),
    "lm_release": ([_vp, ctypes.c_uint64], _ip),
    "lm_server_stats": ([_vp, ctypes.POINTER(ctypes.c_int64)], _ip),
    "lm_server_phase_times": ([_vp, _dp], _ip),
    "lm_server_memory": ([_vp, ctypes.POINTER(ctypes.c_int64)], _ip),
    "lm_request_footprint": ([_vp, _ip, ctypes.POINTER(GmresOpts), ctypes.POINTER(ctypes.c_int64)], _ip),
    "lm_server_destroy": ([_vp], _ip),
}


def exported_symbols():
    return list(_SIGS)


def lib():
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(status):
    if status < 0:
        raise LmError(status, lib().lm_last_error().decode())
    return status


def _dptr(a):
    return a.ctypes.data_as(_dp)


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _tptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Layers:
    """Sec. 2.1 medium: interfaces y = -d[l], wavenumbers k, weights eta."""

    def __init__(self, d, k, eta=None):
        d = np.ascontiguousarray(np.atleast_1d(d), dtype=np.float64)
        k = np.ascontiguousarray(np.atleast_1d(k), dtype=np.float64)
        e = None if eta is None else np.ascontiguousarray(np.atleast_1d(eta), dtype=np.float64)
        h = ctypes.c_void_p()
        _check(lib().lm_create_layers(k.size, _dptr(d), _dptr(k), None if e is None else _dptr(e), ctypes.byref(h)))
        self.h = h
        self.d, self.k = d, k

    def close(self):
        if self.h:
            lib().lm_destroy_layers(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Geometry:
    """Elements of closed node polygons (Sec. 3.3) plus the operator data;
    with quad=LM_QUAD_SPECTRAL the elements are the nodes of smooth closed
    scatterers (see lm_quad in the header)."""

    def __init__(self, layers, node_offsets, nodes_xy, method=LM_AUTO, p=20, leaf_size=48, precond=-1, top_fft=0,
                 bc=LM_BC_DIRICHLET, robin_beta=0.0, quad=LM_QUAD_LOWEST):
        off = np.ascontiguousarray(node_offsets, dtype=np.int64)
        xy = np.ascontiguousarray(nodes_xy, dtype=np.float64)
        o = GeomOpts(method, p, leaf_size, precond, top_fft, bc, robin_beta, quad)
        h = ctypes.c_void_p()
        _check(lib().lm_create_geometry(layers.h, off.size - 1, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                        _dptr(xy), ctypes.byref(o), _stream(), ctypes.byref(h)))
        self.h = h
        self.layers = layers  # keeps the medium alive
        n = ctypes.c_int64()
        b = ctypes.c_int64()
        m = ctypes.c_int()
        _check(lib().lm_geometry_info(h, ctypes.byref(n), ctypes.byref(b), ctypes.byref(m)))
        self.n, self.device_bytes, self.method = n.value, b.value, m.value

    @classmethod
    def from_workload(cls, w, **kw):
        lay = Layers(w.d, w.k, w.eta)
        off, xy = w.flat_nodes()
        return cls(lay, off, xy, **kw)

    def elements(self):
        cx, cy, ww = (np.empty(self.n) for _ in range(3))
        lay = np.empty(self.n, dtype=np.int32)
        _check(lib().lm_geometry_elements(self.h, _dptr(cx), _dptr(cy), _dptr(ww),
                                          lay.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return cx, cy, ww, lay

    def normals(self):
        """Outward unit normals of the elements (lm_geometry_normals)."""
        nx, ny = np.empty(self.n), np.empty(self.n)
        _check(lib().lm_geometry_normals(self.h, _dptr(nx), _dptr(ny)))
        return nx, ny

    def fmm_stats(self):
        """Plan sizes of the fast method (see lm_fmm_stats)."""
        out = (ctypes.c_int64 * 10)()
        _check(lib().lm_fmm_stats(self.h, out))
        keys = ("boxes", "m2l_free_entries", "m2l_reaction_entries", "free_classes", "reaction_tables",
                "reaction_near_pairs", "free_leaf_level", "reaction_finest_level", "free_near_leaf_pairs",
                "free_near_pairs")
        return dict(zip(keys, list(out)))

    def close(self):
        if self.h:
            lib().lm_destroy_geometry(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- operations on torch device tensors -----------------------------------
    def matvec(self, x, y=None, precision=LM_FP64):
        import torch
        dt = torch.complex128 if precision == LM_FP64 else torch.complex64
        x = x.reshape(-1, self.n)
        assert x.dtype == dt and x.is_cuda and x.is_contiguous()
        if y is None:
            y = torch.empty_like(x)
        _check(lib().lm_matvec(self.h, precision, x.shape[0], _tptr(x), _tptr(y), _stream()))
        return y

    def matvec_noalloc(self, x, y, precision=LM_FP64):
        """y = K x through lm_matvec_noalloc (workspace in the library's
        static device array; y must be given)."""
        import torch
        dt = torch.complex128 if precision == LM_FP64 else torch.complex64
        x = x.reshape(-1, self.n)
        assert x.dtype == dt and x.is_cuda and x.is_contiguous()
        assert y.dtype == dt and y.is_cuda and y.is_contiguous() and y.numel() == x.numel()
        _check(lib().lm_matvec_noalloc(self.h, precision, x.shape[0], _tptr(x), _tptr(y), _stream()))
        return y

    def precond_apply(self, x, y=None, precision=LM_FP64):
        """y = M x (lm_precond_apply); x: complex128 [n_rhs][N] on the device."""
        import torch
        x = x.reshape(-1, self.n)
        assert x.dtype == torch.complex128 and x.is_cuda and x.is_contiguous()
        if y is None:
            y = torch.empty_like(x)
        _check(lib().lm_precond_apply(self.h, precision, x.shape[0], _tptr(x), _tptr(y), _stream()))
        return y

    def precond_subdomains(self):
        """(level, leaf level, [(own elements, neighbourhood elements)]) of
        the preconditioner (lm_precond_subdomains)."""
        i32 = ctypes.POINTER(ctypes.c_int32)
        info = np.zeros(4, dtype=np.int64)
        _check(lib().lm_precond_subdomains(self.h, info.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), None, None,
                                           None))
        S, lev, nj, lf = (int(v) for v in info)
        jptr = np.zeros(S + 1, dtype=np.int32)
        nb = np.zeros(S, dtype=np.int32)
        jidx = np.zeros(max(nj, 1), dtype=np.int32)
        _check(lib().lm_precond_subdomains(self.h, info.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                           jptr.ctypes.data_as(i32), nb.ctypes.data_as(i32), jidx.ctypes.data_as(i32)))
        subs = [(jidx[jptr[b]:jptr[b] + nb[b]].copy(), jidx[jptr[b]:jptr[b + 1]].copy()) for b in range(S)]
        return lev, lf, subs

    def stage_times(self, x, y, reps=10, precision=LM_FP64):
        """Average ms per FMM stage from HIP events inside the library: P2M,
        M2M, M2L lists, L2L, L2P, near field, M2L partial sums, whole matvec,
        level-0 convolution (lm_matvec_stage_times)."""
        out = np.zeros(9)
        _check(lib().lm_matvec_stage_times(self.h, precision, x.shape[0], _tptr(x), _tptr(y), reps, _stream(),
                                           _dptr(out)))
        return out

    def rhs(self, theta_rad):
        import torch
        th = np.ascontiguousarray(np.atleast_1d(theta_rad), dtype=np.float64)
        g = torch.empty((th.size, self.n), dtype=torch.complex128, device="cuda")
        _check(lib().lm_rhs(self.h, th.size, _dptr(th), _tptr(g), _stream()))
        return g

    def solve(self, theta_rad, tol=1e-8, max_iter=500, restart=200, precond=1, precision=LM_FP64):
        import torch
        th = np.ascontiguousarray(np.atleast_1d(theta_rad), dtype=np.float64)
        phi = torch.empty((th.size, self.n), dtype=torch.complex128, device="cuda")
        rep = (SolveReport * th.size)()
        o = GmresOpts(tol, max_iter, restart, precond)
        st = _check(lib().lm_gmres_solve(self.h, precision, th.size, _dptr(th), ctypes.byref(o), _tptr(phi), rep,
                                         _stream()))
        return phi, [(r.iterations, r.rel_residual) for r in rep], st

    def solve_rhs(self, g, tol=1e-8, max_iter=500, restart=200, precond=1, precision=LM_FP64):
        import torch
        g = g.reshape(-1, self.n).contiguous()
        phi = torch.empty_like(g)
        rep = (SolveReport * g.shape[0])()
        o = GmresOpts(tol, max_iter, restart, precond)
        st = _check(lib().lm_gmres_solve_rhs(self.h, precision, g.shape[0], _tptr(g), ctypes.byref(o), _tptr(phi),
                                             rep, _stream()))
        return phi, [(r.iterations, r.rel_residual) for r in rep], st

    def point_source_rhs(self, src_xy):
        """G(c_i | s_r) at the collocation points for point sources s_r
        (lm_point_source_rhs); src_xy: (n_src, 2)."""
        import torch
        sxy = np.ascontiguousarray(np.atleast_2d(src_xy), dtype=np.float64)
        g = torch.empty((sxy.shape[0], self.n), dtype=torch.complex128, device="cuda")
        _check(lib().lm_point_source_rhs(self.h, sxy.shape[0], _dptr(sxy), _tptr(g), _stream()))
        return g

    def field(self, phi, pts_xy):
        """Scattered field of densities phi at receivers pts_xy (n, 2)
        (lm_field): device complex128 [n_rhs][n_pts]."""
        import torch
        phi = phi.reshape(-1, self.n).contiguous()
        p = np.ascontiguousarray(np.atleast_2d(pts_xy), dtype=np.float64)
        out = torch.empty((phi.shape[0], p.shape[0]), dtype=torch.complex128, device="cuda")
        _check(lib().lm_field(self.h, phi.shape[0], _tptr(phi), p.shape[0], _dptr(p), _tptr(out), _stream()))
        return out

    def far_field(self, phi, obs_rad):
        import torch
        phi = phi.reshape(-1, self.n).contiguous()
        ob = np.ascontiguousarray(np.atleast_1d(obs_rad), dtype=np.float64)
        out = torch.empty((phi.shape[0], ob.size), dtype=torch.complex128, device="cuda")
        _check(lib().lm_far_field(self.h, phi.shape[0], _tptr(phi), ob.size, _dptr(ob), _tptr(out), _stream()))
        return out


def point_far_field(layers, src_xy, obs_rad):
    """Far-field patterns of unit point sources (lm_point_far_field), device
    complex128 [n_src][n_obs]."""
    import torch
    sxy = np.ascontiguousarray(np.atleast_2d(src_xy), dtype=np.float64)
    ob = np.ascontiguousarray(np.atleast_1d(obs_rad), dtype=np.float64)
    out = torch.empty((sxy.shape[0], ob.size), dtype=torch.complex128, device="cuda")
    _check(lib().lm_point_far_field(layers.h, sxy.shape[0], _dptr(sxy), ob.size, _dptr(ob), _tptr(out), _stream()))
    return out


def point_field(layers, src_xy, pts_xy):
    """G(p | s) of unit point sources at receivers (lm_point_field), device
    complex128 [n_src][n_pts]."""
    import torch
    sxy = np.ascontiguousarray(np.atleast_2d(src_xy), dtype=np.float64)
    p = np.ascontiguousarray(np.atleast_2d(pts_xy), dtype=np.float64)
    out = torch.empty((sxy.shape[0], p.shape[0]), dtype=torch.complex128, device="cuda")
    _check(lib().lm_point_field(layers.h, sxy.shape[0], _dptr(sxy), p.shape[0], _dptr(p), _tptr(out), _stream()))
    return out


def far_field_angles():
    """341 angles per side: 5..175 deg (top) and 185..355 deg (bottom), 0.5 deg steps."""
    top = np.radians(np.arange(5.0, 175.0 + 1e-9, 0.5))
    bot = np.radians(np.arange(185.0, 355.0 + 1e-9, 0.5))
    return np.concatenate([top, bot])


def request_footprint(geom, n_rhs, tol=1e-6, max_iter=1000, restart=500, precond=1):
    """Device bytes a server charges for a request (lm_request_footprint)."""
    b = ctypes.c_int64()
    _check(lib().lm_request_footprint(geom.h, int(n_rhs), ctypes.byref(GmresOpts(tol, max_iter, restart, precond)),
                                      ctypes.byref(b)))
    return b.value


class Server:
    """Continuous-batching GMRES server (lm_server_* in include/lmfmm.h).

    submit() returns a request id at once; poll() reports the state and, once
    done, the reports, phi (numpy c128 [n_rhs][N]) and far field (numpy c128
    [n_rhs][n_obs])."""

    def __init__(self, precision=LM_MIXED, max_active_rhs=64, hbm_budget_bytes=0, precond_fp64=False):
        o = ServerOpts(int(hbm_budget_bytes), int(max_active_rhs), int(precision), int(bool(precond_fp64)))
        h = ctypes.c_void_p()
        _check(lib().lm_server_create(ctypes.byref(o), ctypes.byref(h)))
        self.h = h
        self._req = {}

    def submit(self, geom, theta_rad, tol=1e-6, max_iter=1000, restart=500, precond=1, obs_rad=None):
        th = np.ascontiguousarray(np.atleast_1d(theta_rad), dtype=np.float64)
        ob = np.zeros(0) if obs_rad is None else np.ascontiguousarray(np.atleast_1d(obs_rad), dtype=np.float64)
        r = Request(geom.h, th.size, _dptr(th), GmresOpts(tol, max_iter, restart, precond), ob.size,
                    _dptr(ob) if ob.size else None)
        rid = ctypes.c_uint64()
        _check(lib().lm_submit(self.h, ctypes.byref(r), ctypes.byref(rid)))
        self._req[rid.value] = (geom.n, th.size, ob.size)
        return rid.value

    def poll(self, rid, results=False):
        """(state, status, latency_s, reports, phi, far_field); the last three
        are None unless the request is done and results=True."""
        n, R, no = self._req[rid]
        st = ctypes.c_int()
        lat = np.zeros(1)
        rep = (SolveReport * R)()
        phi = np.empty((R, n), dtype=np.complex128) if results else None
        ff = np.empty((R, no), dtype=np.complex128) if results and no else None
        status = lib().lm_poll(self.h, rid, ctypes.byref(st), rep, _dptr(lat),
                               None if phi is None else phi.ctypes.data_as(_vp),
                               None if ff is None else ff.ctypes.data_as(_vp))
        if st.value == LM_DONE:
            return st.value, status, float(lat[0]), [(x.iterations, x.rel_residual) for x in rep], phi, ff
        return st.value, status, float(lat[0]), None, None, None

    def wait(self, rid, timeout=600.0, results=True):
        import time
        t0 = time.time()
        while True:
            out = self.poll(rid, results=results)
            if out[0] in (LM_DONE, LM_FAILED, LM_CANCELLED):
                return out
            if time.time() - t0 > timeout:
                raise TimeoutError(f"request {rid} not finished after {timeout} s")
            time.sleep(0.002)

    def cancel(self, rid):
        _check(lib().lm_cancel(self.h, rid))

    def release(self, rid):
        _check(lib().lm_release(self.h, rid))
        self._req.pop(rid, None)

    def stats(self):
        out = np.zeros(6, dtype=np.int64)
        _check(lib().lm_server_stats(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return dict(zip(["queued", "active_rhs", "admitted_bytes", "rounds", "launches", "fused_rhs"],
                        [int(v) for v in out]))

    def memory(self):
        """dict: device bytes the server holds, of which spare solves, and the
        admitted footprint (lm_server_memory)."""
        out = np.zeros(3, dtype=np.int64)
        _check(lib().lm_server_memory(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return dict(zip(["held", "spare", "admitted"], [int(v) for v in out]))

    def phase_times(self):
        """dict: K M phase ms, Gram-Schmidt phase ms and algorithmic bytes,
        M2L launch ms, flops and count, host ms of rounds and finishing, and
        the rounds' host split: queueing, waiting, host step
        (lm_server_phase_times)."""
        out = np.zeros(11)
        _check(lib().lm_server_phase_times(self.h, _dptr(out)))
        return dict(zip(["km_ms", "gs_ms", "gs_bytes", "m2l_ms", "m2l_flops", "m2l_launches", "round_ms", "finish_ms",
                         "launch_ms", "wait_ms", "step_ms"], [float(v) for v in out]))

    def close(self):
        if self.h:
            lib().lm_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
