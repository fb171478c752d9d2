"""Python binding of libxf.so (include/xf.h).

The functions named xf_* mirror the C ABI one to one and only marshal
arguments (raw device pointers, sizes, the stream).  `Context` wraps a context
and its workspaces for torch tensors; `rhs` is a torch.autograd.Function whose
backward calls xf_rhs_vjp; `rollout` runs SSP-RK3 steps with checkpoints and
differentiates them with xf_rk3_step_vjp.  Every arithmetic step runs in the
library's HIP kernels; torch provides device memory and the current stream.
If libxf.so is missing this module raises on import: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libxf.so")

XF_OK, XF_EINVAL, XF_EDEVICE, XF_ENOMEM, XF_ENONPHYS, XF_EUNSUPPORTED, XF_ETOOLARGE = 0, -1, -2, -3, -4, -5, -6
XF_NOALLOC_BYTES = 64 << 20
XF_BC_PERIODIC, XF_BC_OUTFLOW = 0, 1
XF_PREC_FP64, XF_PREC_MIXED = 0, 1
XF_OP_RHS, XF_OP_RK3, XF_OP_VJP, XF_OP_RK3_VJP = 0, 1, 2, 3
XF_VISC_LLF, XF_VISC_ROE, XF_VISC_GLF = 0, 1, 2
VISC = {"LLF": XF_VISC_LLF, "ROE": XF_VISC_ROE, "GLF": XF_VISC_GLF}
XF_RECON_WENO5, XF_RECON_CU6, XF_RECON_WENO7 = 0, 1, 2
RECON = {"WENO5": XF_RECON_WENO5, "CU6": XF_RECON_CU6, "WENO7": XF_RECON_WENO7}
FLAGS = {1: "rho<=0", 2: "Y<0", 4: "p<=0 or T<=0", 8: "T out of range", 16: "Newton not converged",
         32: "Roe c^2<=0", 64: "NaN/Inf"}

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2403_05910_amd.build`")
_lib = ctypes.CDLL(LIB_PATH)

_c_int, _c_double, _c_size_t, _vp = ctypes.c_int, ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)


class xf_grid(ctypes.Structure):
    _fields_ = [("nx", _c_int), ("ny", _c_int), ("nz", _c_int),
                ("dx", _c_double), ("dy", _c_double), ("dz", _c_double),
                ("bc", _c_int * 6)]


class xf_thermo(ctypes.Structure):
    _fields_ = [("ns", _c_int), ("W", _dp), ("a", _dp), ("T_lo", _c_double), ("T_hi", _c_double)]


_ip = ctypes.POINTER(ctypes.c_int)


class xf_mechanism(ctypes.Structure):
    _fields_ = [("ns", _c_int), ("nr", _c_int), ("nu_f", _ip), ("nu_b", _ip), ("A", _dp), ("B", _dp), ("E", _dp),
                ("third", _ip), ("eff", _dp), ("reversible", _ip), ("s0", _dp)]


class xf_transport(ctypes.Structure):
    _fields_ = [("ns", _c_int), ("mu", _dp), ("kappa", _dp), ("D", _dp), ("p_ref", _c_double)]


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_create = _sig("xf_create", _c_int, ctypes.POINTER(xf_grid), ctypes.POINTER(xf_thermo), _c_int, ctypes.POINTER(_vp))
_create_ghosts = _sig("xf_create_ghosts", _c_int, ctypes.POINTER(xf_grid), ctypes.POINTER(xf_thermo), _c_int, _c_int,
                      ctypes.POINTER(_vp))
_destroy = _sig("xf_destroy", _c_int, _vp)
_state_elems = _sig("xf_state_elems", _c_size_t, _vp)
_ws_bytes = _sig("xf_workspace_bytes", _c_size_t, _vp, _c_int)
_fill = _sig("xf_fill_ghosts", _c_int, _vp, _vp, _vp)
_fill_vjp = _sig("xf_fill_ghosts_vjp", _c_int, _vp, _vp, _vp)
_rhs = _sig("xf_rhs", _c_int, _vp, _vp, _vp, _vp, _vp)
_rhs_noalloc = _sig("xf_rhs_noalloc", _c_int, _vp, _vp, _vp, _vp)
_rhs_alpha = _sig("xf_rhs_alpha", _c_int, _vp, _vp, _vp, _vp, _vp, _vp, _vp)
_prims = _sig("xf_primitives", _c_int, _vp, _vp, _vp, _vp)
_cfl = _sig("xf_cfl_dt", _c_int, _vp, _vp, _c_double, _vp, _vp, _vp)
_rk3 = _sig("xf_rk3_step", _c_int, _vp, _vp, _c_double, _vp, _vp, _vp)
_set_pp = _sig("xf_set_positivity", _c_int, _vp, _c_int)
_set_visc = _sig("xf_set_dissipation", _c_int, _vp, _c_int)
_set_recon = _sig("xf_set_reconstruction", _c_int, _vp, _c_int)
_set_viscous = _sig("xf_set_viscous", _c_int, _vp, ctypes.POINTER(xf_transport), _c_int)
_set_reactions = _sig("xf_set_reactions", _c_int, _vp, ctypes.POINTER(xf_mechanism), _c_int, _c_int)
_react = _sig("xf_react", _c_int, _vp, _vp, _c_double, _vp, _vp)
_rk3_cfl = _sig("xf_rk3_step_cfl", _c_int, _vp, _vp, _c_double, _vp, _vp, _vp)
_rhs_vjp = _sig("xf_rhs_vjp", _c_int, _vp, _vp, _vp, _vp, _vp, _vp)
_rk3_vjp = _sig("xf_rk3_step_vjp", _c_int, _vp, _vp, _c_double, _vp, _vp, _vp)
_status = _sig("xf_status", _c_int, _vp, _vp, ctypes.POINTER(ctypes.c_uint))
_timing = _sig("xf_timing", _c_int, _vp, _c_int)
_timing_read = _sig("xf_timing_read", _c_int, _vp, _vp, _dp, ctypes.POINTER(ctypes.c_longlong))
_strerror = _sig("xf_strerror", ctypes.c_char_p, _c_int)

EXPORTED = ["xf_create", "xf_create_ghosts", "xf_destroy", "xf_state_elems", "xf_workspace_bytes", "xf_fill_ghosts",
            "xf_fill_ghosts_vjp", "xf_rhs", "xf_rhs_noalloc", "xf_rhs_alpha", "xf_primitives", "xf_cfl_dt", "xf_rk3_step", "xf_rk3_step_cfl",
            "xf_set_dissipation", "xf_set_reconstruction", "xf_set_positivity", "xf_set_viscous", "xf_set_reactions", "xf_react", "xf_rhs_vjp", "xf_rk3_step_vjp",
            "xf_status", "xf_strerror", "xf_timing", "xf_timing_read"]
XF_VISCOUS_STRESS, XF_VISCOUS_HEAT, XF_VISCOUS_DIFFUSION = 1, 2, 4
VISCOUS_TERMS = {"stress": XF_VISCOUS_STRESS, "heat": XF_VISCOUS_HEAT, "diffusion": XF_VISCOUS_DIFFUSION}
KERNEL_CLASSES = ["prims", "sweep_x", "sweep_y", "sweep_z", "fill", "stage", "cfl", "zero",
                  "vjp_x", "vjp_y", "vjp_z", "prims_vjp", "fill_vjp", "transport", "viscous_x", "viscous_y",
                  "viscous_z", "react"]
XF_SPLIT_STRANG, XF_SPLIT_LIE = 0, 1
SPLITTING = {"strang": XF_SPLIT_STRANG, "lie": XF_SPLIT_LIE}


class XfError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {xf_strerror(code)} ({code})")
        self.code = code


def _check(code, what):
    if code != XF_OK:
        raise XfError(code, what)
    return code


# ---------------------------------------------------------------------------
# one-to-one wrappers of the C ABI (pointers are ints; streams are ints)
# ---------------------------------------------------------------------------
def xf_strerror(code):
    return _strerror(code).decode()


def xf_create(grid: xf_grid, thermo: xf_thermo, precision: int):
    h = _vp()
    _check(_create(ctypes.byref(grid), ctypes.byref(thermo), precision, ctypes.byref(h)), "xf_create")
    return h.value


def xf_create_ghosts(grid: xf_grid, thermo: xf_thermo, precision: int, ghost_width: int):
    h = _vp()
    _check(_create_ghosts(ctypes.byref(grid), ctypes.byref(thermo), precision, ghost_width, ctypes.byref(h)),
           "xf_create_ghosts")
    return h.value


def xf_destroy(ctx):
    return _check(_destroy(ctx), "xf_destroy")


def xf_state_elems(ctx):
    return int(_state_elems(ctx))


def xf_workspace_bytes(ctx, op):
    return int(_ws_bytes(ctx, op))


def xf_fill_ghosts(ctx, U, stream):
    return _check(_fill(ctx, U, stream), "xf_fill_ghosts")


def xf_fill_ghosts_vjp(ctx, Ubar, stream):
    return _check(_fill_vjp(ctx, Ubar, stream), "xf_fill_ghosts_vjp")


def xf_rhs(ctx, U, rhs, ws, stream):
    return _check(_rhs(ctx, U, rhs, ws, stream), "xf_rhs")


def xf_rhs_noalloc(ctx, U, rhs, stream):
    return _check(_rhs_noalloc(ctx, U, rhs, stream), "xf_rhs_noalloc")


def xf_rhs_alpha(ctx, U, alpha_in, alpha_out, rhs, ws, stream):
    return _check(_rhs_alpha(ctx, U, alpha_in, alpha_out, rhs, ws, stream), "xf_rhs_alpha")


def xf_primitives(ctx, U, prim, stream):
    return _check(_prims(ctx, U, prim, stream), "xf_primitives")


def xf_cfl_dt(ctx, U, cfl, dt_dev, ws, stream):
    return _check(_cfl(ctx, U, cfl, dt_dev, ws, stream), "xf_cfl_dt")


def xf_rk3_step(ctx, U, dt, dt_dev, ws, stream):
    return _check(_rk3(ctx, U, dt, dt_dev, ws, stream), "xf_rk3_step")


def xf_set_dissipation(ctx, visc):
    return _check(_set_visc(ctx, int(visc)), "xf_set_dissipation")


def xf_set_reconstruction(ctx, recon):
    return _check(_set_recon(ctx, int(recon)), "xf_set_reconstruction")


def xf_set_positivity(ctx, enable):
    return _check(_set_pp(ctx, int(bool(enable))), "xf_set_positivity")


def xf_set_reactions(ctx, mechanism, substeps, splitting):
    ptr = None if mechanism is None else ctypes.byref(mechanism)
    return _check(_set_reactions(ctx, ptr, int(substeps), int(splitting)), "xf_set_reactions")


def xf_react(ctx, U, dt, dt_dev, stream):
    return _check(_react(ctx, U, float(dt), dt_dev, stream), "xf_react")


def xf_set_viscous(ctx, transport, terms):
    ptr = None if transport is None else ctypes.byref(transport)
    return _check(_set_viscous(ctx, ptr, int(terms)), "xf_set_viscous")


def xf_rk3_step_cfl(ctx, U, cfl, dt_dev, ws, stream):
    return _check(_rk3_cfl(ctx, U, cfl, dt_dev, ws, stream), "xf_rk3_step_cfl")


def xf_rhs_vjp(ctx, U, rhs_bar, U_bar, ws, stream):
    return _check(_rhs_vjp(ctx, U, rhs_bar, U_bar, ws, stream), "xf_rhs_vjp")


def xf_rk3_step_vjp(ctx, U_n, dt, U_bar, ws, stream):
    return _check(_rk3_vjp(ctx, U_n, dt, U_bar, ws, stream), "xf_rk3_step_vjp")


def xf_timing(ctx, enable):
    return _check(_timing(ctx, int(bool(enable))), "xf_timing")


def xf_timing_read(ctx, stream):
    """{class name: (total ms, launches)} of the launches since the last read"""
    n = len(KERNEL_CLASSES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_longlong * n)()
    _check(_timing_read(ctx, stream, ms, cnt), "xf_timing_read")
    return {KERNEL_CLASSES[k]: (ms[k], cnt[k]) for k in range(n)}


def xf_status(ctx, stream):
    """returns (code, flags); code is XF_ENONPHYS when flags != 0"""
    f = ctypes.c_uint(0)
    code = _status(ctx, stream, ctypes.byref(f))
    if code not in (XF_OK, XF_ENONPHYS):
        raise XfError(code, "xf_status")
    return code, int(f.value)


# ---------------------------------------------------------------------------
# torch-facing context
# ---------------------------------------------------------------------------
def _torch():
    import torch
    return torch


class Context:
    """A libxf context on the current torch device plus its workspaces.

    n = (nx, ny, nz), d = (dx, dy, dz), bc = 6 ints (-x,+x,-y,+y,-z,+z),
    W (ns,) kg/mol, a (ns, 6) thermo coefficients, [T_lo, T_hi] Newton bracket
    (T_hi <= 0: none), precision "fp64" or "mixed", ghost_width 3 or 4 (4 is
    needed by the WENO7 reconstruction).
    """

    def __init__(self, n, d, bc, W, a, T_lo=0.0, T_hi=0.0, precision="fp64", ghost_width=3):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("libxf needs a HIP device")
        self.n = tuple(int(v) for v in n)
        self.d = tuple(float(v) for v in d)
        self.bc = tuple(int(v) for v in bc)
        self.W = np.ascontiguousarray(W, dtype=np.float64)
        self.a = np.ascontiguousarray(a, dtype=np.float64).reshape(len(self.W), 6)
        self.ns = len(self.W)
        self.nv = self.ns + 4
        self.precision = precision
        self.positivity = False
        self.visc = "LLF"
        self.recon = "WENO5"
        self.viscous = 0
        self.reactions = None
        self.ghost_width = int(ghost_width)
        g = [self.ghost_width if k > 1 else 0 for k in self.n]
        self.shape = (self.nv, self.n[2] + 2 * g[2], self.n[1] + 2 * g[1], self.n[0] + 2 * g[0])
        self.interior = (slice(None), slice(g[2], g[2] + self.n[2]), slice(g[1], g[1] + self.n[1]),
                         slice(g[0], g[0] + self.n[0]))
        grid = xf_grid(self.n[0], self.n[1], self.n[2], self.d[0], self.d[1], self.d[2], (_c_int * 6)(*self.bc))
        th = xf_thermo(self.ns, self.W.ctypes.data_as(_dp), self.a.ctypes.data_as(_dp), float(T_lo), float(T_hi))
        prec = {"fp64": XF_PREC_FP64, "mixed": XF_PREC_MIXED}[precision]
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.handle = xf_create_ghosts(grid, th, prec, self.ghost_width)
        assert xf_state_elems(self.handle) == int(np.prod(self.shape))
        self._ws = {}

    @classmethod
    def from_case(cls, case, precision="fp64"):
        t = case.thermo
        return cls(case.n, case.d, case.bc, t.W, t.a, t.T_lo, t.T_hi, precision, case.ng)

    def close(self):
        if getattr(self, "handle", None):
            xf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- buffers --------------------------------------------------------
    def workspace(self, op):
        torch = _torch()
        if op not in self._ws:
            nb = xf_workspace_bytes(self.handle, op)
            self._ws[op] = torch.empty(nb, dtype=torch.uint8, device=self.device)
        return self._ws[op].data_ptr()

    def new_state(self):
        torch = _torch()
        return torch.zeros(self.shape, dtype=torch.float64, device=self.device)

    def state_from_numpy(self, U):
        torch = _torch()
        assert tuple(U.shape) == self.shape, (U.shape, self.shape)
        return torch.from_numpy(np.ascontiguousarray(U, dtype=np.float64)).to(self.device)

    def _ptr(self, t, shape=None):
        torch = _torch()
        shape = self.shape if shape is None else shape
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and tuple(t.shape) == shape):
            raise ValueError(f"expected a contiguous float64 device tensor of shape {shape}")
        return t.data_ptr()

    @staticmethod
    def _stream():
        return _torch().cuda.current_stream().cuda_stream

    # -- operations -----------------------------------------------------
    def fill_ghosts(self, U):
        xf_fill_ghosts(self.handle, self._ptr(U), self._stream())
        return U

    def fill_ghosts_vjp(self, Ubar):
        xf_fill_ghosts_vjp(self.handle, self._ptr(Ubar), self._stream())
        return Ubar

    def rhs(self, U, out=None):
        out = self.new_state() if out is None else out
        xf_rhs(self.handle, self._ptr(U), self._ptr(out), self.workspace(XF_OP_RHS), self._stream())
        return out

    def face_counts(self):
        """faces of the x, y and z directions (0 for an inactive one)"""
        nx, ny, nz = self.n
        return tuple(0 if self.n[d] <= 1 else (nx + (d == 0)) * (ny + (d == 1)) * (nz + (d == 2)) for d in range(3))

    def alpha_elems(self):
        """doubles of an alpha buffer of rhs_alpha: 3 per face of every direction"""
        return 3 * sum(self.face_counts())

    def rhs_alpha(self, U, alpha_in=None, alpha_out=None, out=None):
        """xf_rhs with the dissipation speeds given (alpha_in) and/or returned
        (alpha_out): float64 device tensors of alpha_elems() entries"""
        torch = _torch()
        out = self.new_state() if out is None else out

        def aptr(a):
            if a is None:
                return None
            if not (a.is_cuda and a.dtype == torch.float64 and a.is_contiguous() and a.numel() == self.alpha_elems()):
                raise ValueError(f"expected a contiguous float64 device tensor of {self.alpha_elems()} entries")
            return a.data_ptr()
        xf_rhs_alpha(self.handle, self._ptr(U), aptr(alpha_in), aptr(alpha_out), self._ptr(out),
                     self.workspace(XF_OP_RHS), self._stream())
        return out

    def primitives(self, U, out=None):
        """(T, p, c, 1/rho) of every padded cell, shape (4,) + the padded grid"""
        torch = _torch()
        out = torch.empty((4,) + self.shape[1:], dtype=torch.float64, device=self.device) if out is None else out
        xf_primitives(self.handle, self._ptr(U), self._ptr(out, (4,) + self.shape[1:]), self._stream())
        return out

    def cfl_dt(self, U, cfl, out=None):
        torch = _torch()
        out = torch.empty(1, dtype=torch.float64, device=self.device) if out is None else out
        xf_cfl_dt(self.handle, self._ptr(U), float(cfl), out.data_ptr(), self.workspace(XF_OP_RHS), self._stream())
        return out

    def set_dissipation(self, visc="LLF"):
        """artificial viscosity of the flux splitting: "LLF", "ROE" or "GLF" """
        xf_set_dissipation(self.handle, VISC[visc])
        self.visc = visc
        return self

    def set_reconstruction(self, recon="WENO5"):
        """reconstruction of the characteristic fluxes: "WENO5", "CU6" or
        "WENO7" (the last needs ghost_width 4)"""
        xf_set_reconstruction(self.handle, RECON[recon])
        self.recon = recon
        return self

    def set_viscous(self, table, terms=("stress", "heat", "diffusion")):
        """viscous and diffusive fluxes in every residual of the context:
        table with mu (ns, 4), kappa (ns, 4), D (ns, ns, 4) and p_ref (the
        fitted transport), terms a subset of "stress", "heat", "diffusion"
        (an empty one, or table None, switches them off)"""
        bits = 0
        for t in terms:
            bits |= VISCOUS_TERMS[t]
        if table is None or bits == 0:
            xf_set_viscous(self.handle, None, 0)
        else:
            mu = np.ascontiguousarray(table.mu, dtype=np.float64).reshape(self.ns, 4)
            kappa = np.ascontiguousarray(table.kappa, dtype=np.float64).reshape(self.ns, 4)
            D = np.ascontiguousarray(table.D, dtype=np.float64).reshape(self.ns, self.ns, 4)
            tr = xf_transport(self.ns, mu.ctypes.data_as(_dp), kappa.ctypes.data_as(_dp), D.ctypes.data_as(_dp),
                              float(table.p_ref))
            xf_set_viscous(self.handle, tr, bits)
        self.viscous = bits if table is not None else 0
        self._ws.clear()          # the workspaces grow while the fluxes are on
        return self

    def set_reactions(self, mech, substeps=4, splitting="strang"):
        """reaction source split off every step (xf_rk3_step): mech with
        nu_f, nu_b (nr, ns) ints, A, B, E (nr,), third (nr,), eff (nr, ns),
        reversible (nr,) and s0 (ns,), or None to switch reactions off"""
        if mech is None or substeps == 0:
            xf_set_reactions(self.handle, None, 0, 0)
            self.reactions = None
            return self
        nr = int(np.asarray(mech.A).shape[0])
        arr = {
            "nu_f": np.ascontiguousarray(mech.nu_f, dtype=np.int32).reshape(nr, self.ns),
            "nu_b": np.ascontiguousarray(mech.nu_b, dtype=np.int32).reshape(nr, self.ns),
            "A": np.ascontiguousarray(mech.A, dtype=np.float64), "B": np.ascontiguousarray(mech.B, dtype=np.float64),
            "E": np.ascontiguousarray(mech.E, dtype=np.float64),
            "third": np.ascontiguousarray(mech.third, dtype=np.int32),
            "eff": np.ascontiguousarray(mech.eff, dtype=np.float64).reshape(nr, self.ns),
            "reversible": np.ascontiguousarray(mech.reversible, dtype=np.int32),
            "s0": np.ascontiguousarray(mech.s0, dtype=np.float64)}
        ptr = {k: v.ctypes.data_as(_ip if v.dtype == np.int32 else _dp) for k, v in arr.items()}
        m = xf_mechanism(self.ns, nr, ptr["nu_f"], ptr["nu_b"], ptr["A"], ptr["B"], ptr["E"], ptr["third"],
                         ptr["eff"], ptr["reversible"], ptr["s0"])
        xf_set_reactions(self.handle, m, substeps, SPLITTING[splitting])
        self.reactions = (substeps, splitting)
        return self

    def react(self, U, dt):
        """one reaction step over dt (float or one-element device tensor) in place; ghosts refilled"""
        torch = _torch()
        if isinstance(dt, torch.Tensor):
            xf_react(self.handle, self._ptr(U), 0.0, dt.data_ptr(), self._stream())
        else:
            xf_react(self.handle, self._ptr(U), float(dt), None, self._stream())
        return U

    def set_positivity(self, enable=True):
        """positivity-preserving flux blend in rk3_step / rk3_step_cfl"""
        xf_set_positivity(self.handle, enable)
        self.positivity = bool(enable)
        return self

    def rk3_step(self, U, dt):
        """dt: a float, or a one-element float64 device tensor (no host round trip)"""
        torch = _torch()
        if isinstance(dt, torch.Tensor):
            xf_rk3_step(self.handle, self._ptr(U), 0.0, dt.data_ptr(), self.workspace(XF_OP_RK3), self._stream())
        else:
            xf_rk3_step(self.handle, self._ptr(U), float(dt), None, self.workspace(XF_OP_RK3), self._stream())
        return U

    def rk3_step_cfl(self, U, cfl, dt_out=None):
        """one RK3 step with dt = CFL limit of U^n computed on the device;
        returns the one-element device tensor holding dt"""
        torch = _torch()
        dt_out = torch.empty(1, dtype=torch.float64, device=self.device) if dt_out is None else dt_out
        xf_rk3_step_cfl(self.handle, self._ptr(U), float(cfl), dt_out.data_ptr(), self.workspace(XF_OP_RK3),
                        self._stream())
        return dt_out

    def rhs_vjp(self, U, rhs_bar, U_bar=None):
        U_bar = self.new_state() if U_bar is None else U_bar
        xf_rhs_vjp(self.handle, self._ptr(U), self._ptr(rhs_bar), self._ptr(U_bar), self.workspace(XF_OP_VJP),
                   self._stream())
        return U_bar

    def rk3_step_vjp(self, U_n, dt, U_bar):
        xf_rk3_step_vjp(self.handle, self._ptr(U_n), float(dt), self._ptr(U_bar), self.workspace(XF_OP_RK3_VJP),
                        self._stream())
        return U_bar

    def timing(self, enable=True):
        xf_timing(self.handle, enable)

    def timing_read(self):
        return xf_timing_read(self.handle, self._stream())

    def status(self):
        """synchronises; returns the accumulated non-physical-state bits (and clears them)"""
        return xf_status(self.handle, self._stream())[1]


# ---------------------------------------------------------------------------
# autograd
# ---------------------------------------------------------------------------
def _make_functions():
    torch = _torch()

    class RhsFunction(torch.autograd.Function):
        """L(G(U)): ghost fill then the right-hand side; backward is
        G^T J^T (xf_rhs_vjp then xf_fill_ghosts_vjp), LLF speeds held fixed."""

        @staticmethod
        def forward(fctx, ctx, U):
            V = U.detach().clone()
            ctx.fill_ghosts(V)
            out = ctx.rhs(V)
            fctx.ctx = ctx
            fctx.save_for_backward(V)
            return out

        @staticmethod
        def backward(fctx, g):
            (V,) = fctx.saved_tensors
            ctx = fctx.ctx
            Ub = ctx.rhs_vjp(V, g.contiguous())
            ctx.fill_ghosts_vjp(Ub)
            return None, Ub

    class RolloutFunction(torch.autograd.Function):
        """nsteps SSP-RK3 steps of fixed dt from U0; states are kept every
        ckpt_every steps and the backward recomputes each segment from its
        checkpoint, then runs xf_rk3_step_vjp step by step in reverse."""

        @staticmethod
        def forward(fctx, ctx, U0, dt, nsteps, ckpt_every):
            U = U0.detach().clone()
            ckpts = []
            for k in range(nsteps):
                if k % ckpt_every == 0:
                    ckpts.append(U.clone())
                ctx.rk3_step(U, dt)
            fctx.ctx, fctx.dt, fctx.nsteps, fctx.every = ctx, dt, nsteps, ckpt_every
            fctx.ckpts = ckpts
            return U

        @staticmethod
        def backward(fctx, g):
            ctx, dt, nsteps, every = fctx.ctx, fctx.dt, fctx.nsteps, fctx.every
            lam = g.detach().clone().contiguous()
            for seg in reversed(range(len(fctx.ckpts))):
                k0 = seg * every
                k1 = min(k0 + every, nsteps)
                states = [fctx.ckpts[seg]]
                for k in range(k0, k1 - 1):
                    states.append(ctx.rk3_step(states[-1].clone(), dt))
                for st in reversed(states):
                    ctx.rk3_step_vjp(st, dt, lam)
            fctx.ckpts = None
            return None, lam, None, None, None

    return RhsFunction, RolloutFunction


_FUNCS = None


def _funcs():
    global _FUNCS
    if _FUNCS is None:
        _FUNCS = _make_functions()
    return _FUNCS


def rhs(ctx: Context, U):
    """differentiable L(G(U)) for a padded state U (ghost values are replaced)"""
    return _funcs()[0].apply(ctx, U)


def rollout(ctx: Context, U0, dt, nsteps, ckpt_every=8):
    """differentiable state after nsteps SSP-RK3 steps of fixed dt"""
    return _funcs()[1].apply(ctx, U0, float(dt), int(nsteps), int(ckpt_every))


def rollout_memory_bytes(ctx: Context, nsteps, ckpt_every):
    """device memory of a checkpointed rollout and its backward: checkpoints,
    one segment of step states, the rollout output/cotangent and the RK3 and
    RK3-VJP workspaces"""
    S = int(np.prod(ctx.shape)) * 8
    C = (nsteps + ckpt_every - 1) // ckpt_every
    return C * S + ckpt_every * S + 2 * S + xf_workspace_bytes(ctx.handle, XF_OP_RK3) + \
        xf_workspace_bytes(ctx.handle, XF_OP_RK3_VJP)
