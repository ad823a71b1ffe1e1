"""ctypes wrapper of the FP64 CPU oracle (test infrastructure only).

Only tests/, the smoke check and the benchmark's CPU-baseline leg import this module.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_LIB = None


class OrcDomain(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("y_periodic", C.c_int32), ("bc_x", C.c_int32),
        ("u_in", C.c_double), ("rho_out", C.c_double),
        ("nu", C.c_double * 3), ("sigma", C.c_double * 3), ("theta_deg", C.c_double * 2),
        ("beta0", C.c_double), ("body_force", C.c_double * 2),
        ("n_circles", C.c_int32), ("force_half_q", C.c_int32),
        ("circles", C.POINTER(C.c_double)), ("solid", C.POINTER(C.c_uint8)),
        ("rho_init", C.POINTER(C.c_double)),
    ]


def lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(OrcDomain), C.c_char_p, C.c_int]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_max_threads.restype = C.c_int
        L.orc_step.argtypes = [C.c_void_p, C.c_int]
        L.orc_prepare.argtypes = [C.c_void_p]
        L.orc_info.argtypes = [C.c_void_p, ip]
        L.orc_get_ext.argtypes = [C.c_void_p, C.c_int, dp]
        L.orc_get_f.argtypes = [C.c_void_p, dp]
        L.orc_set_f.argtypes = [C.c_void_p, dp]
        L.orc_get_rho.argtypes = [C.c_void_p, dp]
        L.orc_mass.argtypes = [C.c_void_p, dp]
        L.orc_fill_nodes.argtypes = [C.c_void_p, ip, dp]
        L.orc_link_q.restype = C.c_double
        L.orc_link_q.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int]
        L.orc_theta12.restype = C.c_double
        L.orc_theta12.argtypes = [C.c_void_p]
        L.orc_march.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double, C.c_double, ip, dp]
        L.orc_gradient.argtypes = [C.c_void_p, dp, dp]
        L.orc_isotropic_sum.argtypes = [C.POINTER(C.c_long), C.POINTER(C.c_long)]
        L.orc_lattice.argtypes = [ip, ip, dp]
        L.orc_matrix.argtypes = [dp, dp]
        L.orc_equilibrium.argtypes = [C.c_double, C.c_double, C.c_double, dp]
        L.orc_force_populations.argtypes = [C.c_double] * 4 + [dp]
        L.orc_relaxation_rates.argtypes = [C.c_double, dp]
        L.orc_relaxation_time.restype = C.c_double
        L.orc_relaxation_time.argtypes = [dp, dp]
        L.orc_collide.argtypes = [dp, dp, dp, C.c_double, C.c_double, dp, dp]
        L.orc_g_of_X.restype = C.c_double
        L.orc_g_of_X.argtypes = [C.c_double]
        L.orc_segregation_X.argtypes = [dp, dp]
        L.orc_recolour.argtypes = [dp, dp, dp, dp, C.c_double, dp]
        _LIB = L
    return _LIB


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


class Oracle:
    """One domain advanced by the oracle.  Fields are returned as numpy arrays [.., ny, nx]."""

    def __init__(self, w, force_half_q: bool = False):
        L = lib()
        self.w = w
        self._solid = np.ascontiguousarray(w.solid, dtype=np.uint8)
        self._rho = np.ascontiguousarray(w.rho_init, dtype=np.float64)
        self._circ = np.ascontiguousarray(np.asarray(w.circles, dtype=np.float64).reshape(-1))
        if self._circ.size == 0:
            self._circ = np.zeros(3)
        d = OrcDomain()
        d.nx, d.ny, d.y_periodic, d.bc_x = w.nx, w.ny, w.y_periodic, w.bc_x
        d.u_in, d.rho_out = w.u_in, w.rho_out
        for k in range(3):
            d.nu[k] = w.nu[k]
            d.sigma[k] = w.sigma[k]
        d.theta_deg[0], d.theta_deg[1] = w.theta_deg
        d.beta0 = w.beta0
        d.body_force[0], d.body_force[1] = w.body_force
        d.n_circles = int(np.asarray(w.circles).reshape(-1, 3).shape[0])
        d.force_half_q = 1 if force_half_q else 0
        d.circles = _dp(self._circ)
        d.solid = self._solid.ctypes.data_as(C.POINTER(C.c_uint8))
        d.rho_init = _dp(self._rho)
        err = C.create_string_buffer(256)
        h = L.orc_create(C.byref(d), err, 256)
        if not h:
            raise ValueError(err.value.decode())
        self.h = C.c_void_p(h)
        info = np.zeros(8, np.int32)
        L.orc_info(self.h, _ip(info))
        self.nx, self.ny, self.GX, self.PY, self.NXE, self.NYE, self.n_fill, self.n_sb = map(int, info)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and _LIB is not None:
            _LIB.orc_destroy(h)
            self.h = None

    def step(self, n: int = 1) -> None:
        lib().orc_step(self.h, int(n))

    def prepare(self) -> None:
        lib().orc_prepare(self.h)

    def ext(self, which: int, comps: int) -> np.ndarray:
        out = np.zeros((comps, self.NYE, self.NXE))
        lib().orc_get_ext(self.h, which, _dp(out))
        return out

    def ext_C(self):
        return self.ext(0, 3)

    def ext_type(self):
        return self.ext(2, 1)[0].astype(np.int32)

    def ext_stress(self):
        return self.ext(3, 3)

    def ext_force(self):
        return self.ext(4, 2)

    def ext_velocity(self):
        return self.ext(5, 2)

    def crop(self, a: np.ndarray) -> np.ndarray:
        """In-grid part of an extended-grid array."""
        return a[..., self.PY:self.PY + self.ny, self.GX:self.GX + self.nx]

    def f(self) -> np.ndarray:
        out = np.zeros((3, 9, self.ny, self.nx))
        lib().orc_get_f(self.h, _dp(out))
        return out

    def set_f(self, f: np.ndarray) -> None:
        a = np.ascontiguousarray(f, dtype=np.float64)
        lib().orc_set_f(self.h, _dp(a))

    def rho(self) -> np.ndarray:
        out = np.zeros((3, self.ny, self.nx))
        lib().orc_get_rho(self.h, _dp(out))
        return out

    def mass(self) -> np.ndarray:
        out = np.zeros(3)
        lib().orc_mass(self.h, _dp(out))
        return out

    def fill_nodes(self):
        idx = np.zeros((self.n_fill, 4), np.int32)
        nrm = np.zeros((self.n_fill, 2))
        lib().orc_fill_nodes(self.h, _ip(idx), _dp(nrm))
        return idx, nrm

    def link_q(self, i: int, j: int, a: int) -> float:
        return float(lib().orc_link_q(self.h, i, j, a))

    def theta12(self) -> float:
        return float(lib().orc_theta12(self.h))

    def gradient(self, field_ext: np.ndarray) -> np.ndarray:
        a = np.ascontiguousarray(field_ext, dtype=np.float64)
        out = np.zeros((2, self.NYE, self.NXE))
        lib().orc_gradient(self.h, _dp(a), _dp(out))
        return out

    def march(self, i, j, dx, dy):
        out = np.zeros(5, np.int32)
        w = C.c_double(0.0)
        lib().orc_march(self.h, i, j, dx, dy, _ip(out), C.byref(w))
        return bool(out[0]), (int(out[1]), int(out[2])), (int(out[3]), int(out[4])), w.value


# ---- single-node building blocks ----------------------------------------------------------

def lattice():
    ex = np.zeros(9, np.int32)
    ey = np.zeros(9, np.int32)
    w = np.zeros(9)
    lib().orc_lattice(_ip(ex), _ip(ey), _dp(w))
    return ex, ey, w


def isotropic_sum(block5x5) -> np.ndarray:
    b = np.ascontiguousarray(np.asarray(block5x5, dtype=np.int64).reshape(25))
    out = np.zeros(2, np.int64)
    lib().orc_isotropic_sum(b.ctypes.data_as(C.POINTER(C.c_long)), out.ctypes.data_as(C.POINTER(C.c_long)))
    return out


def matrices():
    m = np.zeros(81)
    mi = np.zeros(81)
    lib().orc_matrix(_dp(m), _dp(mi))
    return m.reshape(9, 9), mi.reshape(9, 9)


def equilibrium(rho, ux, uy):
    out = np.zeros(9)
    lib().orc_equilibrium(rho, ux, uy, _dp(out))
    return out


def force_populations(ux, uy, fx, fy):
    out = np.zeros(9)
    lib().orc_force_populations(ux, uy, fx, fy, _dp(out))
    return out


def relaxation_rates(tau):
    out = np.zeros(9)
    lib().orc_relaxation_rates(tau, _dp(out))
    return out


def relaxation_time(rk, nu):
    rk = np.ascontiguousarray(rk, dtype=np.float64)
    nu = np.ascontiguousarray(nu, dtype=np.float64)
    return float(lib().orc_relaxation_time(_dp(rk), _dp(nu)))


def collide(f, rk, nu, fx, fy):
    f = np.ascontiguousarray(f, dtype=np.float64)
    rk = np.ascontiguousarray(rk, dtype=np.float64)
    nu = np.ascontiguousarray(nu, dtype=np.float64)
    out = np.zeros(9)
    u = np.zeros(2)
    lib().orc_collide(_dp(f), _dp(rk), _dp(nu), fx, fy, _dp(out), _dp(u))
    return out, u


def g_of_X(X):
    return float(lib().orc_g_of_X(X))


def segregation_X(sigma):
    s = np.ascontiguousarray(sigma, dtype=np.float64)
    out = np.zeros(3)
    lib().orc_segregation_X(_dp(s), _dp(out))
    return out


def recolour(fdag, rk, n, gX, beta0):
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (fdag, rk, n, gX)]
    out = np.zeros(27)
    lib().orc_recolour(_dp(a[0]), _dp(a[1]), _dp(a[2]), _dp(a[3]), beta0, _dp(out))
    return out.reshape(3, 9)
