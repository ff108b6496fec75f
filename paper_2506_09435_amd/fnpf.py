"""ctypes binding of libfnpf.so (include/fnpf.h): argument marshalling only.

Every computation runs in the HIP library.  PyTorch provides device memory
and the current stream; tensors passed to the library must be contiguous and
on the context's device (float64 unless stated otherwise).  The binding
fails loudly if the library is missing: there is no CPU fallback.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfnpf.so")

F64, F32 = 0, 1

STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_ALLOC", 3: "ERR_HIP", 4: "ERR_GEOM", 5: "ERR_NOCONV",
          6: "ERR_BREAKDOWN", 7: "ERR_NAN", 8: "ERR_STATE"}


class FnpfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class MeshDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("p", C.c_int32), ("nz", C.c_int32), ("n_eh", C.c_int32),
                ("n_s", C.c_int64), ("eh_nodes", C.c_void_p), ("eh_corner", C.c_void_p),
                ("eh_arc", C.c_void_p), ("eh_face_tag", C.c_void_p), ("layer_s", C.c_void_p),
                ("g", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("precond", C.c_int32), ("rtol", C.c_double), ("atol", C.c_double),
                ("max_iter", C.c_int32), ("check_every", C.c_int32), ("inner_rtol", C.c_double),
                ("max_outer", C.c_int32), ("extrapolate", C.c_int32), ("cheb_degree", C.c_int32),
                ("use_graph", C.c_int32), ("line_smoother", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("outer_iters", C.c_int32), ("rel_res", C.c_double), ("bnorm", C.c_double)]

    def as_dict(self):
        return dict(iters=self.iters, outer_iters=self.outer_iters, rel_res=self.rel_res, bnorm=self.bnorm)


_lib = None

# exported symbols and their argument types (also used by the ABI test)
SIGNATURES = {
    "fnpf_default_opts": (None, [C.c_void_p]),
    "fnpf_status_string": (C.c_char_p, [C.c_int]),
    "fnpf_last_error": (C.c_char_p, [C.c_void_p]),
    "fnpf_gll": (C.c_int, [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fnpf_create": (C.c_int, [C.c_void_p, C.c_void_p]),
    "fnpf_destroy": (C.c_int, [C.c_void_p]),
    "fnpf_sizes": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fnpf_node_coords": (C.c_int, [C.c_void_p, C.c_void_p]),
    "fnpf_surface_interp_weights": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fnpf_enable_fp32": (C.c_int, [C.c_void_p]),
    "fnpf_set_apply_variant": (C.c_int, [C.c_void_p, C.c_int32]),
    "fnpf_geom": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fnpf_export_geometry": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fnpf_laplace_apply": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "fnpf_laplace_apply_noalloc": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "fnpf_line_smoother_apply": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fnpf_neumann_load": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fnpf_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fnpf_w_surface": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fnpf_rhs": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fnpf_set_linear": (C.c_int, [C.c_void_p, C.c_int32]),
    "fnpf_set_surface_quadrature": (C.c_int, [C.c_void_p, C.c_int32]),
    "fnpf_surface_quadrature_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                               C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "fnpf_multigrid_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                      C.POINTER(C.c_double), C.c_int32]),
    "fnpf_set_modal_filter": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.c_int32]),
    "fnpf_modal_filter": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fnpf_modal_filter_vjp": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fnpf_set_relaxation": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_double, C.c_double]),
    "fnpf_rk4_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_double,
                                C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fnpf_rhs_vjp": (C.c_int, [C.c_void_p] + [C.c_void_p] * 8 + [C.c_void_p]),
    "fnpf_w_surface_vjp": (C.c_int, [C.c_void_p] + [C.c_void_p] * 5 + [C.c_void_p]),
    "fnpf_solve_adjoint": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fnpf_geom_vjp": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fnpf_rk4_step_vjp": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fnpf_get_warm_start": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "fnpf_set_warm_start": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "fnpf_sync": (C.c_int, [C.c_void_p, C.c_void_p]),
}


def lib():
    """Load libfnpf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2506_09435_amd.build` "
                               "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    lib().fnpf_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def gll(p: int):
    x = np.zeros(p + 1)
    w = np.zeros(p + 1)
    D = np.zeros((p + 1, p + 1))
    st = lib().fnpf_gll(p, x.ctypes.data, w.ctypes.data, D.ctypes.data)
    if st:
        raise FnpfError(st, "fnpf_gll")
    return x, w, D


def _ptr(t, dtype=None, n=None, device=None):
    """Device address of tensor t after checking what the C ABI cannot: the element count n
    (the call reads or writes exactly n elements), the dtype, contiguity and the device."""
    if t is None:
        return None
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} elements, got {t.numel()}")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if device is not None and t.device != device:
        raise ValueError(f"expected a tensor on {device}, got one on {t.device}")
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Context:
    """One mesh on the current GPU.  Mirrors the fnpf_* calls of include/fnpf.h."""

    def __init__(self, mesh, g: float = 9.81):
        import torch
        self.linear = False
        self._h = C.c_void_p()
        nodes = np.ascontiguousarray(mesh.eh_nodes, dtype=np.int32)
        corner = np.ascontiguousarray(mesh.eh_corner, dtype=np.float64)
        arc = None if mesh.eh_arc is None else np.ascontiguousarray(mesh.eh_arc, dtype=np.float64)
        tags = np.ascontiguousarray(mesh.eh_face_tag, dtype=np.int32)
        layer = None if mesh.layer_s is None else np.ascontiguousarray(mesh.layer_s, dtype=np.float64)
        d = MeshDesc(dim=mesh.dim, p=mesh.p, nz=mesh.nz, n_eh=mesh.n_eh, n_s=mesh.n_s,
                     eh_nodes=nodes.ctypes.data, eh_corner=corner.ctypes.data,
                     eh_arc=None if arc is None else arc.ctypes.data, eh_face_tag=tags.ctypes.data,
                     layer_s=None if layer is None else layer.ctypes.data, g=g)
        torch.cuda.current_device()
        st = lib().fnpf_create(C.byref(d), C.byref(self._h))
        if st:
            raise FnpfError(st, lib().fnpf_last_error(None).decode())
        self.mesh = mesh
        self.dim, self.p, self.nz = mesh.dim, mesh.p, mesh.nz
        n_v, n_s, n_e = C.c_int64(), C.c_int64(), C.c_int64()
        ncol = C.c_int32()
        lib().fnpf_sizes(self._h, C.byref(n_v), C.byref(n_s), C.byref(n_e), C.byref(ncol))
        self.n_v, self.n_s, self.n_e, self.n_colours = n_v.value, n_s.value, n_e.value, ncol.value
        self.ng = 6 if mesh.dim == 3 else 3
        self.npt = (mesh.p + 1) ** mesh.dim
        self.device = torch.device("cuda", torch.cuda.current_device())

    def _v(self, t, dtype=None):
        """Pointer to a volume vector [n_v] on this context's device."""
        import torch
        return _ptr(t, torch.float64 if dtype is None else dtype, self.n_v, self.device)

    def _s(self, t):
        """Pointer to a surface vector [n_s] (FP64) on this context's device."""
        import torch
        return _ptr(t, torch.float64, self.n_s, self.device)

    def _check(self, st, where):
        if st:
            raise FnpfError(st, f"{where}: {lib().fnpf_last_error(self._h).decode()}")

    def close(self):
        if self._h:
            lib().fnpf_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- queries ------------------------------------------------------------------
    def node_coords(self):
        xy = np.zeros((self.n_s, self.dim - 1))
        self._check(lib().fnpf_node_coords(self._h, xy.ctypes.data), "fnpf_node_coords")
        return xy

    def surface_interp_weights(self, points):
        """Lagrange interpolation at horizontal points: (node [n, nh] int32, w [n, nh]) with
        f(point_k) = sum_t w[k, t] f[node[k, t]] (fnpf_surface_interp_weights)."""
        pts = np.ascontiguousarray(np.asarray(points, dtype=np.float64).reshape(-1, self.dim - 1))
        n = pts.shape[0]
        nh = (self.p + 1) ** (self.dim - 1)
        node = np.zeros((n, nh), dtype=np.int32)
        w = np.zeros((n, nh))
        self._check(lib().fnpf_surface_interp_weights(self._h, n, pts.ctypes.data, node.ctypes.data, w.ctypes.data),
                    "fnpf_surface_interp_weights")
        return node, w

    def node_xy(self):
        xy = self.node_coords()
        if self.dim == 2:
            return xy[:, 0], np.zeros(self.n_s)
        return xy[:, 0], xy[:, 1]

    # -- path ---------------------------------------------------------------------
    def set_apply_variant(self, variant: int):
        """0: fused geometry with owner-computes tile assembly (default); 1: stored per-point
        factors; 6: fused geometry, line schedule with colour assembly; 7: fused geometry, colour
        schedule (fnpf_set_apply_variant; all compute the same operator)."""
        self._check(lib().fnpf_set_apply_variant(self._h, int(variant)), "fnpf_set_apply_variant")

    def enable_fp32(self):
        self._check(lib().fnpf_enable_fp32(self._h), "fnpf_enable_fp32")

    def geom(self, eta, h, stream=None):
        import torch
        self._check(lib().fnpf_geom(self._h, self._s(eta), self._s(h), _stream(stream)),
                    "fnpf_geom")

    def export_geometry(self, dtype=F64, stream=None):
        import torch
        tdt = torch.float64 if dtype == F64 else torch.float32
        G = torch.empty((self.n_e, self.ng, self.npt), dtype=tdt, device=self.device)
        diag = torch.empty(self.n_v, dtype=torch.float64, device=self.device)
        self._check(lib().fnpf_export_geometry(self._h, dtype, _ptr(G, tdt, G.numel(), self.device),
                                               self._v(diag), _stream(stream)), "fnpf_export_geometry")
        return G, diag

    def laplace_apply(self, x, y=None, mask_dirichlet=False, stream=None):
        import torch
        if x.dtype not in (torch.float64, torch.float32):
            raise TypeError(f"expected float64 or float32, got {x.dtype}")
        dtype = F64 if x.dtype == torch.float64 else F32
        if y is None:
            y = torch.empty_like(x)
        self._check(lib().fnpf_laplace_apply(self._h, dtype, self._v(x, x.dtype), self._v(y, x.dtype),
                                             int(mask_dirichlet), _stream(stream)), "fnpf_laplace_apply")
        return y

    def line_smoother_apply(self, r, z=None, stream=None):
        """z = B^-1 r with the vertical line blocks of the current geometry (fnpf_line_smoother_apply)."""
        import torch
        if r.dtype not in (torch.float64, torch.float32):
            raise TypeError(f"expected float64 or float32, got {r.dtype}")
        if z is None:
            z = torch.empty_like(r)
        self._check(lib().fnpf_line_smoother_apply(self._h, F64 if r.dtype == torch.float64 else F32,
                                                   self._v(r, r.dtype), self._v(z, r.dtype), _stream(stream)),
                    "fnpf_line_smoother_apply")
        return z

    def neumann_load(self, q, f=None, stream=None):
        import torch
        if f is None:
            f = torch.empty(self.n_v, dtype=torch.float64, device=self.device)
        qp = _ptr(q, torch.float64, self.dim * self.n_v, self.device)
        self._check(lib().fnpf_neumann_load(self._h, qp, self._v(f), _stream(stream)), "fnpf_neumann_load")
        return f

    def solve(self, phi_surface, phi=None, neumann_f=None, opts=None, stream=None, raise_on_error=True):
        import torch
        if phi is None:
            phi = torch.zeros(self.n_v, dtype=torch.float64, device=self.device)
        info = SolveInfo()
        o = opts if opts is not None else default_opts()
        st = lib().fnpf_solve(self._h, self._s(phi_surface), self._v(neumann_f),
                              self._v(phi), C.byref(o), C.byref(info), _stream(stream))
        if raise_on_error:
            self._check(st, "fnpf_solve")
        return phi, info.as_dict() | dict(status=STATUS[st])

    def w_surface(self, phi, w=None, stream=None):
        import torch
        if w is None:
            w = torch.empty(self.n_s, dtype=torch.float64, device=self.device)
        self._check(lib().fnpf_w_surface(self._h, self._v(phi), self._s(w),
                                         _stream(stream)), "fnpf_w_surface")
        return w

    def rhs(self, eta, phi_s, w, stream=None):
        import torch
        de = torch.empty(self.n_s, dtype=torch.float64, device=self.device)
        dp = torch.empty_like(de)
        self._check(lib().fnpf_rhs(self._h, self._s(eta), self._s(phi_s),
                                   self._s(w), self._s(de), self._s(dp), _stream(stream)), "fnpf_rhs")
        return de, dp

    def set_linear(self, linear=True):
        """Linear potential flow (fixed domain at eta = 0, linear free-surface conditions).  Also
        drops the cached flat geometry (call again after changing the depth array in place)."""
        self._check(lib().fnpf_set_linear(self._h, int(bool(linear))), "fnpf_set_linear")
        self.linear = bool(linear)

    def set_surface_quadrature(self, nq):
        """0: lumped GLL collocation of the free-surface equations; nq >= p+1: consistent form."""
        self._check(lib().fnpf_set_surface_quadrature(self._h, int(nq)), "fnpf_set_surface_quadrature")

    def surface_quadrature_info(self):
        nq, it = C.c_int32(), C.c_int32()
        lo, hi = C.c_double(), C.c_double()
        self._check(lib().fnpf_surface_quadrature_info(self._h, C.byref(nq), C.byref(it), C.byref(lo), C.byref(hi)),
                    "fnpf_surface_quadrature_info")
        return dict(nq=nq.value, iters=it.value, lam_lo=lo.value, lam_hi=hi.value)

    def multigrid_info(self, cap=8):
        lv = C.c_int32()
        l64, l32 = (C.c_double * cap)(), (C.c_double * cap)()
        self._check(lib().fnpf_multigrid_info(self._h, C.byref(lv), l64, l32, int(cap)), "fnpf_multigrid_info")
        n = min(lv.value, cap)
        return dict(levels=lv.value, lam64=list(l64)[:n], lam32=list(l32)[:n])

    def set_modal_filter(self, cutoff, alpha=0.0, order=1):
        """Modal filter (cutoff < 0 removes it); rk4_step filters eta and phi_s while it is set."""
        self._check(lib().fnpf_set_modal_filter(self._h, int(cutoff), float(alpha), int(order)),
                    "fnpf_set_modal_filter")

    def modal_filter(self, f, stream=None):
        import torch
        out = torch.empty(self.n_s, dtype=torch.float64, device=self.device)
        self._check(lib().fnpf_modal_filter(self._h, self._s(f), self._s(out), _stream(stream)),
                    "fnpf_modal_filter")
        return out

    def modal_filter_vjp(self, out_bar, f_bar, stream=None):
        import torch
        self._check(lib().fnpf_modal_filter_vjp(self._h, self._s(out_bar), self._s(f_bar),
                                                _stream(stream)), "fnpf_modal_filter_vjp")
        return f_bar

    def set_relaxation(self, cr, eta_c, eta_s, phi_c, phi_s, omega, t_ramp):
        if cr is None:
            self._check(lib().fnpf_set_relaxation(self._h, None, None, None, None, None, 0.0, 0.0),
                        "fnpf_set_relaxation")
            return
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (cr, eta_c, eta_s, phi_c, phi_s)]
        for a in arrs:
            if a.shape != (self.n_s,):
                raise ValueError("relaxation arrays must have shape [n_s]")
        self._check(lib().fnpf_set_relaxation(self._h, *[a.ctypes.data for a in arrs], float(omega),
                                              float(t_ramp)), "fnpf_set_relaxation")

    def rk4_step(self, eta, phi_s, h, t, dt, opts=None, tape=None, stream=None):
        import torch
        infos = (SolveInfo * 4)()
        o = opts if opts is not None else default_opts()
        st = lib().fnpf_rk4_step(self._h, self._s(eta), self._s(phi_s),
                                 self._s(h), float(t), float(dt), C.byref(o),
                                 _ptr(tape, torch.float64, 4 * self.tape_record, self.device), infos, _stream(stream))
        self._check(st, "fnpf_rk4_step")
        return [infos[k].as_dict() for k in range(4)]

    # -- adjoint --------------------------------------------------------------------
    @property
    def tape_record(self):
        """Doubles per stage in an fnpf_rk4_step tape: n_v + 2 n_s."""
        return self.n_v + 2 * self.n_s

    def new_tape(self):
        import torch
        return torch.empty(4 * self.tape_record, dtype=torch.float64, device=self.device)

    def rhs_vjp(self, eta, phi_s, w, deta_bar, dphi_bar, eta_bar, phis_bar, w_bar, stream=None):
        import torch
        f = torch.float64
        self._check(lib().fnpf_rhs_vjp(self._h, self._s(eta), self._s(phi_s), self._s(w), self._s(deta_bar),
                                       self._s(dphi_bar), self._s(eta_bar), self._s(phis_bar), self._s(w_bar),
                                       _stream(stream)), "fnpf_rhs_vjp")

    def w_surface_vjp(self, w, w_bar, phi_bar, eta_bar, h_bar, stream=None):
        import torch
        f = torch.float64
        self._check(lib().fnpf_w_surface_vjp(self._h, self._s(w), self._s(w_bar), self._v(phi_bar),
                                             self._s(eta_bar), self._s(h_bar), _stream(stream)),
                    "fnpf_w_surface_vjp")

    def solve_adjoint(self, phi_bar, lam=None, opts=None, stream=None):
        import torch
        if lam is None:
            lam = torch.zeros(self.n_v, dtype=torch.float64, device=self.device)
        info = SolveInfo()
        o = opts if opts is not None else default_opts()
        self._check(lib().fnpf_solve_adjoint(self._h, self._v(phi_bar), self._v(lam),
                                             C.byref(o), C.byref(info), _stream(stream)), "fnpf_solve_adjoint")
        return lam, info.as_dict()

    def geom_vjp(self, lam, phi, eta_bar, h_bar, stream=None):
        import torch
        f = torch.float64
        self._check(lib().fnpf_geom_vjp(self._h, self._v(lam), self._v(phi), self._s(eta_bar), self._s(h_bar),
                                        _stream(stream)), "fnpf_geom_vjp")

    def rk4_step_vjp(self, h, t, dt, tape, eta_bar, phis_bar, h_bar, opts=None, stream=None):
        """In place: (eta_bar, phis_bar) of the step output -> of its input; h_bar accumulated."""
        import torch
        f = torch.float64
        infos = (SolveInfo * 4)()
        o = opts if opts is not None else default_opts()
        self._check(lib().fnpf_rk4_step_vjp(self._h, self._s(h), float(t), float(dt),
                                            _ptr(tape, f, 4 * self.tape_record, self.device),
                                            self._s(eta_bar), self._s(phis_bar), self._s(h_bar), C.byref(o),
                                            infos, _stream(stream)), "fnpf_rk4_step_vjp")
        return [infos[k].as_dict() for k in range(4)]

    def get_warm_start(self, stream=None):
        import torch
        phi = torch.empty(self.n_v, dtype=torch.float64, device=self.device)
        self._check(lib().fnpf_get_warm_start(self._h, self._v(phi), _stream(stream)), "fnpf_get_warm_start")
        return phi

    def set_warm_start(self, phi=None, stream=None):
        import torch
        self._check(lib().fnpf_set_warm_start(self._h, self._v(phi) if phi is not None else None,
                                              _stream(stream)), "fnpf_set_warm_start")

    def sync(self, stream=None):
        self._check(lib().fnpf_sync(self._h, _stream(stream)), "fnpf_sync")


@dataclass
class Setup:
    """A workload prepared on the device: context, depth, initial state, relaxation."""
    ctx: Context
    h: object
    eta0: object
    phi0: object
    x: np.ndarray
    y: np.ndarray


def setup_workload(wl, fp32=False):
    """Create a context for a workloads.configs.Workload and evaluate its data at the library's nodes."""
    import torch
    ctx = Context(wl.mesh, g=wl.g)
    x, y = ctx.node_xy()
    dev = ctx.device
    h = torch.tensor(np.asarray(wl.depth(x, y), dtype=np.float64), device=dev)
    eta0 = torch.tensor(np.asarray(wl.eta0(x, y), dtype=np.float64), device=dev)
    phi0 = torch.tensor(np.asarray(wl.phi0(x, y), dtype=np.float64), device=dev)
    ra = wl.relaxation_arrays(x, y)
    if ra is not None:
        ctx.set_relaxation(*ra, omega=wl.relax_wave.omega, t_ramp=wl.t_ramp)
    if fp32:
        ctx.enable_fp32()
    return Setup(ctx=ctx, h=h, eta0=eta0, phi0=phi0, x=x, y=y)
