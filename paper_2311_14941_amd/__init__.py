"""stiffchem: batched stiff chemistry integration on MI355X.

Thin ctypes binding of libstiffchem.so (C ABI in include/stiffchem.h).  It
only marshals arguments: every step of the integration runs in the HIP
kernels.  PyTorch supplies device memory and the stream; arrays are torch
tensors on the plan's device:

* ``T``, ``p``, ``dt``: float64 [n]
* ``Y``: float64 [N, n] (species-major, so ``Y[k]`` is species k of every
  cell, matching the library's ``Y[k*ld + c]`` with ld = n)

If the shared library is missing this module raises: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libstiffchem.so")

SC_OK, SC_EINVAL, SC_EPARSE, SC_ENOMEM, SC_EHIP, SC_EUNSUPPORTED, SC_EBUDGET = 0, -1, -2, -3, -4, -5, -6
CELL_OK, CELL_MAX_STEPS, CELL_H_UNDERFLOW, CELL_NONFINITE, CELL_BAD_INPUT = range(5)
MODES = {"plain": 0, "persistent": 1, "static": 2}
ORDERS = {"none": 0, "dt": 1, "cost": 2}
REACTORS = {"const_p": 0, "const_v": 1}
METHODS = {"ros4": 0, "extrap": 1}
LINALGS = {"auto": 0, "dense": 1, "sparse": 2}


class StiffchemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"stiffchem error {code}: {msg}")
        self.code = code


class Options(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("max_steps", C.c_int32),
                ("mode", C.c_int32), ("tile", C.c_int32), ("grid", C.c_int32),
                ("order", C.c_int32), ("fixed_step", C.c_int32), ("hmax_frac", C.c_double),
                ("reactor", C.c_int32), ("method", C.c_int32), ("linalg", C.c_int32),
                ("cells_per_wave", C.c_int32), ("thermo_tol", C.c_double), ("thermo_Tmin", C.c_double),
                ("thermo_Tmax", C.c_double), ("thermo_degree", C.c_int32)]


class Mapping(C.Structure):
    _fields_ = [("z_tol", C.c_double), ("dT", C.c_double), ("dlnp", C.c_double)]


class MechInfo(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("n_species", "n_reactions", "n_third_body", "n_troe",
                                         "n_elements", "n_state", "n_padded", "nnz_jac", "nnz_lu",
                                         "n_stages", "rhs_evals_per_step", "exp_per_rhs")] + \
               [(n, C.c_int64) for n in ("flops_rhs", "flops_jac", "flops_lu", "flops_solve",
                                         "flops_step")] + \
               [(n, C.c_int32) for n in ("nnz_a_sparse", "nnz_lu_sparse", "lu_levels", "solve_levels")] + \
               [(n, C.c_int64) for n in ("lu_updates_sparse", "flops_lu_sparse", "flops_solve_sparse",
                                         "flops_step_sparse")] + \
               [("lu_tail_sparse", C.c_int32)]


_lib = None
_P = C.c_void_p
_I64 = C.c_int64


def lib():
    """Load the in-tree libstiffchem.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise ImportError(f"{LIBPATH} is missing: build it with paper_2311_14941_amd.build.build()")
        L = C.CDLL(LIBPATH)
        L.sc_last_error.restype = C.c_char_p
        L.sc_default_options.argtypes = [C.POINTER(Options)]
        L.sc_mech_load.argtypes = [C.c_char_p, C.c_size_t, C.POINTER(_P)]
        L.sc_mech_info_get.argtypes = [_P, C.POINTER(MechInfo)]
        L.sc_species_index.argtypes = [_P, C.c_char_p, C.POINTER(C.c_int32)]
        L.sc_mech_sparse_array.argtypes = [_P, C.c_char_p, _P, C.POINTER(C.c_size_t)]
        L.sc_mech_thermo_fit.argtypes = [_P, C.c_double, C.c_double, C.c_double, C.c_int32,
                                         C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                         _P, C.POINTER(C.c_size_t)]
        L.sc_mech_thermo_fit.restype = C.c_int
        L.sc_mech_sparse_array.restype = C.c_int
        L.sc_mech_free.argtypes = [_P]
        L.sc_mech_free.restype = None
        L.sc_plan_create.argtypes = [_P, C.c_int, C.POINTER(Options), C.POINTER(_P)]
        L.sc_plan_free.argtypes = [_P]
        L.sc_plan_free.restype = None
        L.sc_rhs.argtypes = [_P, _I64, _P, _P, _P, _I64, _P, _P, _P, _P]
        L.sc_jacobian.argtypes = [_P, _I64, _P, _P, _P, _I64, _P, _P, _P]
        L.sc_linsolve.argtypes = [_P, _I64, _P, _P, _P, _I64, _P, _P, _P, _P, _P]
        L.sc_integrate.argtypes = [_P, _I64, _P, _P, _P, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _P]
        L.sc_integrate_noalloc.argtypes = L.sc_integrate.argtypes
        L.sc_plan_set_mapping.argtypes = [_P, _P, _P, C.POINTER(Mapping)]
        L.sc_integrate_mapped.argtypes = [_P, _I64, _P, _P, _P, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]
        L.sc_vjp.argtypes = [_P, _I64, _P, _P, _P, _I64, _P, _P, _P, _P, _P, _P, _P]
        L.sc_adjoint.argtypes = [_P, _I64, _P, _P, _P, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                 _P, _P, _P, _P, C.c_size_t, C.POINTER(C.c_size_t), _P]
        L.sc_transport2d.argtypes = [C.c_int32, C.c_int32, C.c_int32, _P, _I64, _P, _P, C.c_double, C.c_double,
                                     _P, _P, _P]
        L.sc_transport2d.restype = C.c_int
        L.sc_adjoint_slot_bytes.argtypes = [_P]
        L.sc_adjoint_slot_bytes.restype = C.c_size_t
        for f in ("sc_mech_load", "sc_mech_info_get", "sc_species_index", "sc_plan_create", "sc_rhs",
                  "sc_jacobian", "sc_linsolve", "sc_integrate", "sc_integrate_noalloc", "sc_vjp", "sc_adjoint",
                  "sc_plan_set_mapping", "sc_integrate_mapped"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != SC_OK:
        raise StiffchemError(rc, lib().sc_last_error().decode())
    return rc


def last_error() -> str:
    return lib().sc_last_error().decode()


class Mechanism:
    """A parsed and compiled mechanism (host side)."""

    def __init__(self, text: str):
        h = _P()
        b = text.encode()
        _check(lib().sc_mech_load(b, len(b), C.byref(h)))
        self._h = h
        info = MechInfo()
        _check(lib().sc_mech_info_get(h, C.byref(info)))
        self.info = {n: getattr(info, n) for n, _ in MechInfo._fields_}
        self.N = self.info["n_species"]
        self.R = self.info["n_reactions"]

    @classmethod
    def load(cls, path):
        with open(path) as f:
            return cls(f.read())

    def species_index(self, name: str) -> int:
        k = C.c_int32()
        _check(lib().sc_species_index(self._h, name.encode(), C.byref(k)))
        return k.value

    _SPARSE_DTYPES = {"perm": "int32", "pattern": "uint8", "apat": "uint8", "erow": "int32", "ecol": "int32",
                      "lu_b_lvl": "int32", "lu_c_lvl": "int32", "fw_lvl": "int32", "bw_lvl": "int32",
                      "tfw_lvl": "int32", "tbw_lvl": "int32", "lu_b": "uint32", "lu_u": "uint32",
                      "diag": "uint32", "lu_c": "uint64", "fw": "uint64", "bw": "uint64", "tfw": "uint64",
                      "tbw": "uint64", "rxi": "uint16", "cstart": "int32", "cmask": "uint64",
                      "sweep_f": "uint32", "sweep_b": "uint32", "sweep_fi": "uint16", "sweep_bi": "uint16"}

    def thermo_fit(self, tol, Tmin=250.0, Tmax=4000.0, degree=0):
        """The interpolation tables of the reactions' -dG/RT and dH/RT
        (sc_mech_thermo_fit, host only): dict with degree, nint, max_err, the
        grid (u0 = ln Tmin, du) and coef[nint, R, 2, degree + 1]."""
        import numpy as np
        d, ni, err, nc = C.c_int32(0), C.c_int32(0), C.c_double(0.0), C.c_size_t(0)
        _check(lib().sc_mech_thermo_fit(self._h, Tmin, Tmax, tol, degree, C.byref(d), C.byref(ni), C.byref(err),
                                        None, C.byref(nc)))
        coef = np.empty(nc.value, dtype=np.float64)
        _check(lib().sc_mech_thermo_fit(self._h, Tmin, Tmax, tol, degree, C.byref(d), C.byref(ni), C.byref(err),
                                        coef.ctypes.data_as(C.c_void_p), C.byref(nc)))
        import math
        return dict(degree=d.value, nint=ni.value, max_err=err.value, u0=math.log(Tmin),
                    du=(math.log(Tmax) - math.log(Tmin)) / ni.value,
                    coef=coef.reshape(ni.value, self.R, 2, d.value + 1))

    def sparse_array(self, name: str):
        """One array of the compiled sparse algebra (sc_mech_sparse_array) as
        a NumPy array (host only)."""
        import numpy as np
        nb = C.c_size_t(0)
        _check(lib().sc_mech_sparse_array(self._h, name.encode(), None, C.byref(nb)))
        a = np.empty(nb.value // np.dtype(self._SPARSE_DTYPES[name]).itemsize, dtype=self._SPARSE_DTYPES[name])
        _check(lib().sc_mech_sparse_array(self._h, name.encode(), a.ctypes.data_as(C.c_void_p), C.byref(nb)))
        return a

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.sc_mech_free(h)
            self._h = None


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(torch, device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Plan:
    """A mechanism on one device with integration options.

    reactor: "const_p" (the per-cell p arguments are pressures) or "const_v"
    (a rigid vessel: they are densities in kg/m^3; forward calls only).
    method: "ros4" (the Rosenbrock method) or "extrap" (the linearly implicit
    Euler extrapolation baseline; forward only).
    linalg: "auto", "dense" or "sparse"; cells_per_wave (sparse): 1, 2 or 4
    cells side by side in one wave, 0 for the most that fit."""

    def __init__(self, mech: Mechanism, device: int = 0, rtol=1e-6, atol=1e-12, max_steps=100000,
                 mode="plain", tile=1, grid=0, order="none", fixed_step=False, hmax_frac=0.0,
                 reactor="const_p", method="ros4", linalg="auto", cells_per_wave=0, thermo_tol=0.0,
                 thermo_Tmin=250.0, thermo_Tmax=4000.0, thermo_degree=0):
        import torch
        self.torch = torch
        self.mech = mech
        self.device = device
        opt = Options()
        lib().sc_default_options(C.byref(opt))
        opt.rtol, opt.atol, opt.max_steps = rtol, atol, max_steps
        opt.mode, opt.tile, opt.grid, opt.order = MODES[mode], tile, grid, ORDERS[order]
        opt.fixed_step = 1 if fixed_step else 0
        opt.hmax_frac = float(hmax_frac)
        opt.reactor = REACTORS[reactor]
        opt.method = METHODS[method]
        opt.linalg = LINALGS[linalg]
        opt.cells_per_wave = int(cells_per_wave)
        opt.thermo_tol, opt.thermo_Tmin, opt.thermo_Tmax = float(thermo_tol), float(thermo_Tmin), float(thermo_Tmax)
        opt.thermo_degree = int(thermo_degree)
        self.reactor, self.method, self.linalg = reactor, method, linalg
        self.config = dict(mode=mode, tile=tile, grid=grid, order=order)
        self.options = opt
        h = _P()
        _check(lib().sc_plan_create(mech._h, device, C.byref(opt), C.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.sc_plan_free(h)
            self._h = None

    # -- argument marshalling ------------------------------------------------
    def _dev(self, x, dtype=None):
        t = self.torch
        dtype = dtype or t.float64
        x = t.as_tensor(x, dtype=dtype, device=f"cuda:{self.device}")
        return x.contiguous()

    def _cells(self, x, n, name, dtype=None):
        """A per-cell device array of n entries (a scalar is broadcast).  The
        kernels index every per-cell array up to n, so shapes are checked
        here, before any launch."""
        x = self._dev(x, dtype)
        if x.dim() == 0:
            x = x.expand(n).contiguous()
        if tuple(x.shape) != (n,):
            raise ValueError(f"{name} must have one entry per cell ({n}), got {tuple(x.shape)}")
        return x

    def _state(self, T, p, Y):
        T, Y = self._dev(T), self._dev(Y)
        if T.dim() != 1:
            raise ValueError(f"T must be [n], got {tuple(T.shape)}")
        n = T.shape[0]
        p = self._cells(p, n, "p")
        if Y.shape != (self.mech.N, n):
            raise ValueError(f"Y must be [N={self.mech.N}, n={n}], got {tuple(Y.shape)}")
        return T, p, Y, n

    def _dlnA(self, dlnA):
        if dlnA is None:
            return None
        d = self._dev(dlnA)
        if d.shape != (self.mech.R,):
            raise ValueError("dlnA must have one entry per reaction")
        return d

    # -- entry points ----------------------------------------------------------
    def rhs(self, T, p, Y, dlnA=None):
        T, p, Y, n = self._state(T, p, Y)
        d = self._dlnA(dlnA)
        fT = self.torch.empty_like(T)
        fY = self.torch.empty_like(Y)
        _check(lib().sc_rhs(self._h, n, _ptr(T), _ptr(p), _ptr(Y), n, _ptr(d), _ptr(fT), _ptr(fY),
                            _stream(self.torch, self.device)))
        return fT, fY

    def jacobian(self, T, p, Y, dlnA=None):
        """J[c, i, j] = d f_i / d y_j with y = (Y_0..Y_{N-1}, T)."""
        T, p, Y, n = self._state(T, p, Y)
        d = self._dlnA(dlnA)
        m = self.mech.N + 1
        J = self.torch.empty((n, m, m), dtype=self.torch.float64, device=T.device)
        _check(lib().sc_jacobian(self._h, n, _ptr(T), _ptr(p), _ptr(Y), n, _ptr(d), _ptr(J),
                                 _stream(self.torch, self.device)))
        return J

    def linsolve(self, T, p, Y, hg, b, dlnA=None):
        """x with (I/hg - J) x = b per cell; b [n, N+1]."""
        T, p, Y, n = self._state(T, p, Y)
        d = self._dlnA(dlnA)
        hg = self._cells(hg, n, "hg")
        b = self._dev(b)
        if tuple(b.shape) != (n, self.mech.N + 1):
            raise ValueError(f"b must be [n, N+1] = [{n}, {self.mech.N + 1}], got {tuple(b.shape)}")
        x = self.torch.empty_like(b)
        _check(lib().sc_linsolve(self._h, n, _ptr(T), _ptr(p), _ptr(Y), n, _ptr(d), _ptr(hg), _ptr(b),
                                 _ptr(x), _stream(self.torch, self.device)))
        return x

    def integrate_noalloc(self, T0, p, Y0, dt, dlnA=None, h=None, out=None):
        """integrate() through sc_integrate_noalloc: the library allocates no
        device memory in the call (queue and ordering workspace in its fixed
        scratch; at most 262,144 cells).  Pass `out` (and h) to keep the
        binding itself from allocating result tensors."""
        return self.integrate(T0, p, Y0, dt, dlnA=dlnA, h=h, out=out, _entry="sc_integrate_noalloc")

    def integrate(self, T0, p, Y0, dt, dlnA=None, h=None, out=None, _entry="sc_integrate"):
        """Integrate every cell over its own dt.  Returns a dict with T, Y,
        status, n_acc, n_rej and (when h is given) the carried step h."""
        T0, p, Y0, n = self._state(T0, p, Y0)
        dt = self._cells(dt, n, "dt")
        d = self._dlnA(dlnA)
        hio = None if h is None else self._cells(h, n, "h").clone()
        t = self.torch
        if out is None:
            out = dict(T=t.empty_like(T0), Y=t.empty_like(Y0),
                       status=t.empty(n, dtype=t.int32, device=T0.device),
                       n_acc=t.zeros(n, dtype=t.int32, device=T0.device),
                       n_rej=t.zeros(n, dtype=t.int32, device=T0.device))
        else:
            want = dict(T=(n,), Y=(self.mech.N, n), status=(n,), n_acc=(n,), n_rej=(n,))
            for k, shp in want.items():
                if tuple(out[k].shape) != shp or not out[k].is_contiguous():
                    raise ValueError(f"out[{k!r}] must be a contiguous tensor of shape {shp}")
        _check(getattr(lib(), _entry)(self._h, n, _ptr(T0), _ptr(p), _ptr(Y0), n, _ptr(dt), _ptr(d),
                                      _ptr(hio), _ptr(out["T"]), _ptr(out["Y"]), _ptr(out["status"]),
                                      _ptr(out["n_acc"]), _ptr(out["n_rej"]), _stream(t, self.device)))
        if hio is not None:
            out["h"] = hio
        return out

    def set_mapping(self, Y_fuel, Y_ox, z_tol, dT, dlnp=0.0):
        """Zonal reference-cell mapping for integrate_mapped(): fuel and
        oxidiser stream mass fractions (N each), the mixture-fraction bound
        z_tol, the temperature band dT [K] and the ln p band dlnp (0: none)."""
        import numpy as np
        N = self.mech.N
        yf = np.ascontiguousarray(Y_fuel, dtype=np.float64)
        yo = np.ascontiguousarray(Y_ox, dtype=np.float64)
        if yf.shape != (N,) or yo.shape != (N,):
            raise ValueError(f"stream compositions must have {N} mass fractions")
        opt = Mapping(float(z_tol), float(dT), float(dlnp))
        _check(lib().sc_plan_set_mapping(self._h, yf.ctypes.data, yo.ctypes.data, C.byref(opt)))

    def integrate_mapped(self, T0, p, Y0, dt, dlnA=None, h=None, out=None):
        """integrate() with the mapping of set_mapping(): returns the same dict
        plus ref [n] (int32), each cell's reference (itself when integrated)."""
        T0, p, Y0, n = self._state(T0, p, Y0)
        dt = self._cells(dt, n, "dt")
        d = self._dlnA(dlnA)
        hio = None if h is None else self._cells(h, n, "h").clone()
        t = self.torch
        dev = T0.device
        if out is None:
            out = dict(T=t.empty_like(T0), Y=t.empty_like(Y0), status=t.empty(n, dtype=t.int32, device=dev),
                       n_acc=t.zeros(n, dtype=t.int32, device=dev), n_rej=t.zeros(n, dtype=t.int32, device=dev))
        if "ref" not in out:
            out["ref"] = t.empty(n, dtype=t.int32, device=dev)
        _check(lib().sc_integrate_mapped(self._h, n, _ptr(T0), _ptr(p), _ptr(Y0), n, _ptr(dt), _ptr(d), _ptr(hio),
                                         _ptr(out["T"]), _ptr(out["Y"]), _ptr(out["status"]), _ptr(out["n_acc"]),
                                         _ptr(out["n_rej"]), _ptr(out["ref"]), _stream(t, self.device)))
        if hio is not None:
            out["h"] = hio
        return out

    def vjp(self, T, p, Y, wT, wY, dlnA=None, per_cell=False):
        """J(y)^T w per cell; returns (gT, gY) and, with per_cell, the
        parameter part [R, n]."""
        T, p, Y, n = self._state(T, p, Y)
        d = self._dlnA(dlnA)
        wT, wY = self._cells(wT, n, "wT"), self._dev(wY)
        if wY.shape != Y.shape:
            raise ValueError("w must have the shape of the state")
        gT, gY = self.torch.empty_like(T), self.torch.empty_like(Y)
        gc = self.torch.empty((self.mech.R, n), dtype=self.torch.float64, device=T.device) if per_cell else None
        _check(lib().sc_vjp(self._h, n, _ptr(T), _ptr(p), _ptr(Y), n, _ptr(d), _ptr(wT), _ptr(wY), _ptr(gT),
                            _ptr(gY), _ptr(gc), _stream(self.torch, self.device)))
        return (gT, gY, gc) if per_cell else (gT, gY)

    def adjoint(self, T0, p, Y0, dt, gT1, gY1, dlnA=None, h=None, cost=None, per_cell=False, budget=0,
                forward_out=False):
        """Discrete adjoint of integrate(): gradients of <gT1, T1> + <gY1, Y1>
        with respect to T0, Y0 and dlnA, the accepted step sequence frozen.
        Returns a dict with gT0, gY0, g_dlnA [R], status, n_acc, peak_bytes and,
        when asked, g_dlnA_cell [R, n] and the recorded forward T1, Y1."""
        t = self.torch
        T0, p, Y0, n = self._state(T0, p, Y0)
        dt = self._cells(dt, n, "dt")
        d = self._dlnA(dlnA)
        gT1, gY1 = self._dev(gT1), self._dev(gY1)
        if gT1.shape != T0.shape or gY1.shape != Y0.shape:
            raise ValueError("cotangents must have the shape of the state")
        h0 = None if h is None else self._cells(h, n, "h")
        cst = None if cost is None else self._cells(cost, n, "cost", t.int32)
        dev = T0.device
        out = dict(gT0=t.empty_like(T0), gY0=t.empty_like(Y0),
                   g_dlnA=t.empty(self.mech.R, dtype=t.float64, device=dev),
                   status=t.empty(n, dtype=t.int32, device=dev), n_acc=t.empty(n, dtype=t.int32, device=dev))
        gc = t.empty((self.mech.R, n), dtype=t.float64, device=dev) if per_cell else None
        T1 = t.empty_like(T0) if forward_out else None
        Y1 = t.empty_like(Y0) if forward_out else None
        peak = C.c_size_t(0)
        _check(lib().sc_adjoint(self._h, n, _ptr(T0), _ptr(p), _ptr(Y0), n, _ptr(dt), _ptr(d), _ptr(h0),
                                _ptr(gT1), _ptr(gY1), _ptr(out["gT0"]), _ptr(out["gY0"]), _ptr(out["g_dlnA"]),
                                _ptr(gc), _ptr(cst), _ptr(T1), _ptr(Y1), _ptr(out["status"]), _ptr(out["n_acc"]),
                                budget, C.byref(peak), _stream(t, self.device)))
        out["peak_bytes"] = peak.value
        if per_cell:
            out["g_dlnA_cell"] = gc
        if forward_out:
            out["T"], out["Y"] = T1, Y1
        return out

    def adjoint_slot_bytes(self) -> int:
        return lib().sc_adjoint_slot_bytes(self._h)


def transport2d(nx, ny, q, u, dt, dx, diffusivity, inflow, out=None):
    """One transport step (sc_transport2d) of the rows of q [ncomp, nx*ny]
    on the nx x ny grid; inflow [ncomp, ny].  Returns out."""
    import torch
    if q.dim() != 2 or q.shape[1] != nx * ny or inflow.shape != (q.shape[0], ny):
        raise ValueError("q must be [ncomp, nx*ny] and inflow [ncomp, ny]")
    if u.shape != (nx * ny,) or dt.shape != (nx * ny,):
        raise ValueError("u and dt must have one entry per cell")
    if out is not None and (out.shape != q.shape or not out.is_contiguous() or out.dtype != torch.float64):
        raise ValueError("out must be a contiguous float64 tensor shaped like q")
    for t in (q, u, dt, inflow):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("transport arrays must be contiguous float64 device tensors")
    out = torch.empty_like(q) if out is None else out
    _check(lib().sc_transport2d(nx, ny, q.shape[0], _ptr(q), nx * ny, _ptr(u), _ptr(dt), float(dx),
                                float(diffusivity), _ptr(inflow), _ptr(out),
                                _stream(torch, q.device.index or 0)))
    return out


def _chem_integrate_fn():
    import torch

    class ChemIntegrate(torch.autograd.Function):
        """(T0, Y0, dlnA) -> (T1, Y1, h1) through sc_integrate; backward
        through sc_adjoint (recording forward + reverse sweep: nothing is
        stored at forward time beyond the inputs).  p, dt, the plan and the
        initial step h are constants; h1 (the step proposed for a following
        substep) is not differentiable.  Y is [N, n] species-major."""

        @staticmethod
        def forward(ctx, T0, Y0, dlnA, p, dt, plan, h):
            hin = torch.zeros_like(T0) if h is None else plan._dev(h)
            out = plan.integrate(T0, p, Y0, dt, dlnA=dlnA, h=hin)
            if not bool((out["status"] == 0).all()):
                bad = int((out["status"] != 0).sum())
                raise RuntimeError(f"{bad} cells failed to integrate; no gradient is defined for them")
            ctx.plan = plan
            ctx.save_for_backward(T0, Y0, dlnA if dlnA is not None else T0.new_zeros(0), p, dt, hin,
                                  out["n_acc"] + out["n_rej"])
            ctx.has_dlnA = dlnA is not None
            ctx.mark_non_differentiable(out["h"])
            return out["T"], out["Y"], out["h"]

        @staticmethod
        def backward(ctx, gT1, gY1, gh1):
            T0, Y0, dlnA, p, dt, hin, cost = ctx.saved_tensors
            plan = ctx.plan
            gT1 = torch.zeros_like(T0) if gT1 is None else gT1.contiguous()
            gY1 = torch.zeros_like(Y0) if gY1 is None else gY1.contiguous()
            r = plan.adjoint(T0, p, Y0, dt, gT1, gY1, dlnA=dlnA if ctx.has_dlnA else None, h=hin, cost=cost,
                             budget=getattr(plan, "adjoint_budget", 0))
            g_d = r["g_dlnA"] if ctx.has_dlnA and ctx.needs_input_grad[2] else None
            return r["gT0"], r["gY0"], g_d, None, None, None, None

    return ChemIntegrate


_CHEM = None


def chem_integrate(T0, Y0, dlnA, p, dt, plan, h=None):
    """Differentiable integration: returns (T1, Y1, h1); gradients flow to T0,
    Y0 and dlnA (a tensor of R log multipliers, or None).  h: initial step
    per cell (None: dt); h1 carries the controller's next step to a
    following substep (operator splitting)."""
    global _CHEM
    if _CHEM is None:
        _CHEM = _chem_integrate_fn()
    return _CHEM.apply(T0, Y0, dlnA, p, dt, plan, h)


class Chain:
    """Successive integrations of the same cells (operator-split substeps:
    the state and the step size carry from one substep to the next), captured
    once into a HIP graph and replayed.  Buffers are allocated up front so the
    captured launches read and write fixed addresses."""

    def __init__(self, plan: "Plan", T0, p, Y0, dt, nsub: int, dlnA=None, graph=True):
        t = plan.torch
        self.plan, self.nsub = plan, nsub
        T0, p, Y0, n = plan._state(T0, p, Y0)
        dt = plan._cells(dt, n, "dt")
        self.n = n
        self.T = [T0.clone() for _ in range(2)]
        self.Y = [Y0.clone() for _ in range(2)]
        self.p, self.dt = p, dt
        self.d = plan._dlnA(dlnA)
        self.h = t.zeros(n, dtype=t.float64, device=T0.device)
        mk = lambda: t.zeros(n, dtype=t.int32, device=T0.device)
        self.status, self.n_acc, self.n_rej = mk(), mk(), mk()
        self.steps = mk()
        self.graph = None
        if graph:
            s = t.cuda.Stream(device=T0.device)
            s.wait_stream(t.cuda.current_stream(T0.device))
            with t.cuda.stream(s):  # warm-up outside capture (lazy setup)
                self._launch_all()
            t.cuda.current_stream(T0.device).wait_stream(s)
            self.graph = t.cuda.CUDAGraph()
            with t.cuda.graph(self.graph):
                self._launch_all()

    def _launch_all(self):
        plan, L = self.plan, lib()
        for k in range(self.nsub):
            a, b = k % 2, (k + 1) % 2
            _check(L.sc_integrate(plan._h, self.n, _ptr(self.T[a]), _ptr(self.p), _ptr(self.Y[a]), self.n,
                                  _ptr(self.dt), _ptr(self.d), _ptr(self.h), _ptr(self.T[b]), _ptr(self.Y[b]),
                                  _ptr(self.status), _ptr(self.n_acc), _ptr(self.n_rej),
                                  _stream(plan.torch, plan.device)))
            self.steps.add_(self.n_acc).add_(self.n_rej)

    def run(self, T0, Y0, h0=None):
        """Load the initial state, run all substeps; returns (T, Y, h, steps)."""
        self.T[0].copy_(self.plan._dev(T0))
        self.Y[0].copy_(self.plan._dev(Y0))
        self.h.zero_() if h0 is None else self.h.copy_(self.plan._dev(h0))
        self.steps.zero_()
        if self.graph is not None:
            self.graph.replay()
        else:
            self._launch_all()
        last = self.nsub % 2
        return self.T[last], self.Y[last], self.h, self.steps


def ensure_built():
    """Build the library only if it is missing (tests and benchmarks)."""
    if not os.path.exists(LIBPATH):
        from . import build as _b
        _b.build()
    return LIBPATH
