"""Test infrastructure: Python face of the CPU oracle (liboracle.so).

Only tests, the smoke check and the benchmark's CPU-baseline leg use this
module.  It builds and loads the plain C oracle (oracle.c) and exposes its
functions on NumPy arrays.  State vectors are ordered (Y_0..Y_{N-1}, T).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = [os.path.join(HERE, "oracle.c"), os.path.join(HERE, "rhs_tmpl.h")]

CELL_OK, CELL_MAX_STEPS, CELL_H_UNDERFLOW, CELL_NONFINITE, CELL_BAD_INPUT = range(5)


def build(force=False):
    """Compile liboracle.so with gcc (-O2, OpenMP, no intrinsics)."""
    if not force and os.path.exists(LIB) and all(
            os.path.getmtime(LIB) >= os.path.getmtime(s) for s in SRC):
        return LIB
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-o", LIB + ".tmp",
           SRC[0], "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def _mode(isothermal, constv):
    """Reactor mode bits of the C functions (isothermal 1, constant volume 2)."""
    return (1 if isothermal else 0) | (2 if constv else 0)


def _opt_dp(x):
    return None if x is None else np.ascontiguousarray(x, np.float64).ctypes.data_as(C.POINTER(C.c_double))


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        L.om_load.restype = C.c_void_p
        L.om_load.argtypes = [C.c_char_p, C.c_char_p, C.c_int]
        L.om_free.argtypes = [C.c_void_p]
        L.om_n_species.argtypes = [C.c_void_p]
        L.om_n_reactions.argtypes = [C.c_void_p]
        L.om_thermo.argtypes = [C.c_void_p, C.c_double, _dp, _dp, _dp]
        L.om_rates.argtypes = [C.c_void_p, C.c_double, _dp, C.c_void_p, _dp, _dp, _dp, _dp, _dp, C.c_int]
        L.om_rhs.argtypes = [C.c_void_p, C.c_double, _dp, C.c_void_p, _dp, C.c_int]
        L.om_jac_fd.argtypes = [C.c_void_p, C.c_double, _dp, C.c_void_p, _dp, C.c_int]
        L.om_jac_cs.argtypes = [C.c_void_p, C.c_double, _dp, C.c_void_p, _dp, C.c_int]
        L.om_dfdp_cs.argtypes = [C.c_void_p, C.c_double, _dp, C.c_void_p, _dp]
        L.om_dense_solve.argtypes = [C.c_int, _dp, _dp]
        L.om_radau_coeffs.argtypes = [_dp, _dp]
        L.om_integrate.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp, _dp, C.c_void_p, C.c_double,
                                   C.c_double, C.c_int, _dp, _dp, _ip, _ip, _ip, C.c_int, C.c_int]
        L.om_integrate_sens_batch.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp, C.c_void_p, C.c_int,
                                              _dp, C.c_void_p, C.c_double, C.c_double, C.c_int, _ip,
                                              C.c_int]
        L.om_max_threads.restype = C.c_int
        _lib = L
    return _lib


class Oracle:
    """A mechanism loaded into the oracle."""

    def __init__(self, text: str):
        err = C.create_string_buffer(256)
        h = lib().om_load(text.encode(), err, 256)
        if not h:
            raise ValueError("oracle: " + err.value.decode())
        self.h = h
        self.N = lib().om_n_species(h)
        self.R = lib().om_n_reactions(h)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.om_free(self.h)
            self.h = None

    # -- pointwise quantities ------------------------------------------------
    def thermo(self, T):
        cp, h, s = (np.empty(self.N) for _ in range(3))
        lib().om_thermo(self.h, float(T), cp, h, s)
        return cp, h, s

    def rates(self, T, p, Y, dlnA=None, constv=False):
        """Returns kf, kr, q [R], wdot [N] (mol/m^3/s) and aux (rho, cp, sum h wdot, Wbar).
        constv: p is the density of a constant-volume reactor."""
        y = np.ascontiguousarray(np.append(np.asarray(Y, np.float64), T))
        kf, kr, q = (np.empty(self.R) for _ in range(3))
        wdot, aux = np.empty(self.N), np.empty(4)
        lib().om_rates(self.h, float(p), y, _opt_dp(dlnA), kf, kr, q, wdot, aux, int(constv))
        return kf, kr, q, wdot, aux

    def rhs(self, y, p, dlnA=None, isothermal=False, constv=False):
        y = np.ascontiguousarray(y, np.float64)
        f = np.empty(self.N + 1)
        lib().om_rhs(self.h, float(p), y, _opt_dp(dlnA), f, _mode(isothermal, constv))
        return f

    def jac_fd(self, y, p, dlnA=None, isothermal=False, constv=False):
        y = np.ascontiguousarray(y, np.float64)
        J = np.empty((self.N + 1, self.N + 1))
        lib().om_jac_fd(self.h, float(p), y, _opt_dp(dlnA), J, _mode(isothermal, constv))
        return J

    def jac_cs(self, y, p, dlnA=None, isothermal=False, constv=False):
        y = np.ascontiguousarray(y, np.float64)
        J = np.empty((self.N + 1, self.N + 1))
        lib().om_jac_cs(self.h, float(p), y, _opt_dp(dlnA), J, _mode(isothermal, constv))
        return J

    def dfdp_cs(self, y, p, dlnA=None):
        y = np.ascontiguousarray(y, np.float64)
        F = np.empty((self.N + 1, self.R))
        lib().om_dfdp_cs(self.h, float(p), y, _opt_dp(dlnA), F)
        return F

    # -- integration ---------------------------------------------------------
    def integrate(self, T0, p, Y0, dt, dlnA=None, rtol=1e-6, atol=1e-12, max_steps=100000,
                  nthreads=0, isothermal=False, constv=False):
        """Integrate cells over dt[c]; p is the pressure, or with constv the
        density of a constant-volume reactor (rho fixed, p varies)."""
        T0 = np.ascontiguousarray(T0, np.float64)
        n = T0.shape[0]
        p = np.ascontiguousarray(np.broadcast_to(p, (n,)), np.float64)
        dt = np.ascontiguousarray(np.broadcast_to(dt, (n,)), np.float64)
        Y0 = np.ascontiguousarray(Y0, np.float64).reshape(n, self.N)
        T1, Y1 = np.empty(n), np.empty((n, self.N))
        nacc, nrej, st = (np.zeros(n, np.int32) for _ in range(3))
        lib().om_integrate(self.h, n, T0, p, Y0, dt, _opt_dp(dlnA), rtol, atol, max_steps, T1, Y1,
                           nacc, nrej, st, int(nthreads), _mode(isothermal, constv))
        return dict(T=T1, Y=Y1, n_acc=nacc, n_rej=nrej, status=st)

    def integrate_sens(self, T0, p, Y0, dt, s0, dpar=None, dlnA=None, rtol=1e-10, atol=1e-16,
                       max_steps=200000, nthreads=0):
        """Forward sensitivities.  s0[c, d, :] initial tangent (N+1, (Y, T) order)
        of direction d in cell c; dpar[c, d, :] the matching dlnA direction.
        Returns final states y[c, N+1] and tangents s[c, d, N+1]."""
        T0 = np.ascontiguousarray(T0, np.float64)
        n = T0.shape[0]
        y = np.ascontiguousarray(np.concatenate([np.asarray(Y0).reshape(n, self.N), T0[:, None]], 1))
        s = np.ascontiguousarray(s0, np.float64).copy()
        ns = s.shape[1]
        p = np.ascontiguousarray(np.broadcast_to(p, (n,)), np.float64)
        dt = np.ascontiguousarray(np.broadcast_to(dt, (n,)), np.float64)
        st = np.zeros(n, np.int32)
        lib().om_integrate_sens_batch(self.h, n, p, y, dt, _opt_dp(dlnA), ns, s,
                                      _opt_dp(dpar), rtol, atol, max_steps, st, int(nthreads))
        return y, s, st


def dense_solve(A, b):
    A = np.ascontiguousarray(A, np.float64).copy()
    b = np.ascontiguousarray(b, np.float64).copy()
    if lib().om_dense_solve(A.shape[0], A, b) != 0:
        raise np.linalg.LinAlgError("singular")
    return b


def radau_coeffs():
    c, A = np.empty(3), np.empty(9)
    lib().om_radau_coeffs(c, A)
    return c, A.reshape(3, 3)


def max_threads():
    return lib().om_max_threads()
