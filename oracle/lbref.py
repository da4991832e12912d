"""ctypes binding of the FP64 C oracle (``lbref.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the package smoke check
and by the benchmark's CPU-baseline leg.  The GPU library never loads it.

All arrays are float64, C-contiguous, laid out ``f[alpha][y][x]`` for the
distributions and ``[y][x]`` for fields.  Velocities follow the standard
D2Q9 ordering (rest, +x, +y, -x, -y, then the diagonals (1,1), (-1,1),
(-1,-1), (1,-1)); the paper uses an orthogonal moment basis without printing
it, and this ordering/basis is the usual one.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbref.c")
_LIB = os.path.join(_HERE, "liblbref.so")

OK, EINVAL, ENOMEM, EUNSTABLE = 0, -1, -2, -4
PERIODIC, WALLS_Y = 0, 1
FORM_MOMENT, FORM_VELOCITY = 0, 1
PSI_CS, PSI_SS = 0, 1  # pseudopotential of Eq. (24) / of Eq. (23)
NEAREST, MULTIRANGE = 0, 1  # interaction stencil of Eq. (7): 8 nearest / 24 nearest and next-nearest


class LbrefParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("bc", ctypes.c_int32), ("pad_", ctypes.c_int32),
        ("a", ctypes.c_double), ("b", ctypes.c_double), ("R", ctypes.c_double), ("T", ctypes.c_double),
        ("G", ctypes.c_double), ("sigma", ctypes.c_double),
        ("s_rho", ctypes.c_double), ("s_e", ctypes.c_double), ("s_zeta", ctypes.c_double),
        ("s_j", ctypes.c_double), ("s_q", ctypes.c_double),
        ("nu_l", ctypes.c_double), ("nu_g", ctypes.c_double), ("rho_switch", ctypes.c_double),
        ("psi_form", ctypes.c_int32), ("stencil", ctypes.c_int32), ("psi_eps", ctypes.c_double),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP over rows, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
            _SRC, "-o", tmp, "-lm",
        ])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        P = ctypes.POINTER(LbrefParams)
        L.lbref_matrices.argtypes = [dp, dp]
        L.lbref_p_eos.argtypes = [P, ctypes.c_double]
        L.lbref_p_eos.restype = ctypes.c_double
        L.lbref_psi2.argtypes = [P, ctypes.c_double]
        L.lbref_psi2.restype = ctypes.c_double
        L.lbref_pressure.argtypes = [P, ctypes.c_double]
        L.lbref_pressure.restype = ctypes.c_double
        L.lbref_collide_site.argtypes = [P, dp] + [ctypes.c_double] * 6 + [ctypes.c_int, dp]
        L.lbref_init.argtypes = [P, dp, dp, dp, dp]
        L.lbref_moments.argtypes = [P, dp, dp, dp, dp, dp, dp, dp]
        L.lbref_step.argtypes = [P, dp, dp, ctypes.c_int64, ctypes.c_int, ctypes.POINTER(ctypes.c_int64)]
        L.lbref_stream.argtypes = [P, dp, dp]
        L.lbref_threads.argtypes = []
        L.lbref_threads.restype = ctypes.c_int
        L.lbref_collide_at.argtypes = [P, dp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), dp]
        L.lbref_stencil_weights.argtypes = [ctypes.c_int, dp]
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Params:
    """Physical and numerical parameters of one run (absolute temperature T)."""
    nx: int
    ny: int
    bc: int = PERIODIC
    a: float = 0.5
    b: float = 4.0
    R: float = 1.0
    T: float = 0.6 * 0.047
    G: float = -1.0
    sigma: float = 0.11
    s_rho: float = 1.0
    s_e: float = 1.1
    s_zeta: float = 1.1
    s_j: float = 1.0
    s_q: float = 1.1
    nu_l: float = 0.1
    nu_g: float = 0.3
    rho_switch: float = 0.13045
    psi_form: int = PSI_CS   # Eq. (24) from the EOS, or Eq. (23) with parameter psi_eps
    psi_eps: float = 0.0
    stencil: int = NEAREST   # interaction stencil of Eq. (7)

    def c(self) -> LbrefParams:
        return LbrefParams(self.nx, self.ny, self.bc, 0, self.a, self.b, self.R, self.T, self.G,
                           self.sigma, self.s_rho, self.s_e, self.s_zeta, self.s_j, self.s_q,
                           self.nu_l, self.nu_g, self.rho_switch, int(self.psi_form), int(self.stencil),
                           float(self.psi_eps))


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle status {code}: {msg}")
        self.code = code


def threads() -> int:
    """Threads used by the oracle's OpenMP loops."""
    return int(lib().lbref_threads())


def matrices():
    M = np.zeros(81)
    Minv = np.zeros(81)
    lib().lbref_matrices(_ptr(M), _ptr(Minv))
    return M.reshape(9, 9), Minv.reshape(9, 9)


def stencil_weights(stencil: int):
    """Weights w(q) of Eq. (7) by squared neighbour distance q = 0..8 (0 where absent)."""
    w = np.zeros(9)
    lib().lbref_stencil_weights(int(stencil), _ptr(w))
    return w


def p_eos(p: Params, rho: float) -> float:
    c = p.c()
    return lib().lbref_p_eos(ctypes.byref(c), float(rho))


def psi2(p: Params, rho: float) -> float:
    c = p.c()
    return lib().lbref_psi2(ctypes.byref(c), float(rho))


def pressure(p: Params, rho: float) -> float:
    """Bulk pressure rho/3 + G psi^2 / 2 (p_EOS of Eq. (30) for the Eq. (24) psi)."""
    c = p.c()
    return lib().lbref_pressure(ctypes.byref(c), float(rho))


def collide_site(p: Params, f9, rho, vx, vy, Fx, Fy, psi2_, form=FORM_MOMENT):
    f9 = np.ascontiguousarray(f9, dtype=np.float64)
    out = np.zeros(9)
    c = p.c()
    lib().lbref_collide_site(ctypes.byref(c), _ptr(f9), rho, vx, vy, Fx, Fy, psi2_, form, _ptr(out))
    return out


def stream(p: Params, fstar):
    """Eq. (5) streaming of a post-collision field f*[9][ny][nx] -> post-streaming f."""
    fstar = np.ascontiguousarray(fstar, dtype=np.float64)
    out = np.empty_like(fstar)
    c = p.c()
    st = lib().lbref_stream(ctypes.byref(c), _ptr(fstar), _ptr(out))
    if st:
        raise OracleError(st, "stream")
    return out


def collide_at(p: Params, f, sites):
    """Post-collision f* ([n][9]) at flat site indices of the post-streaming state f."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.zeros((sites.size, 9))
    c = p.c()
    st = lib().lbref_collide_at(ctypes.byref(c), _ptr(f), sites.size,
                                sites.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _ptr(out))
    if st:
        raise OracleError(st, "collide_at")
    return out


class State:
    """FP64 oracle state: post-streaming distributions f[9][ny][nx] at time t."""

    def __init__(self, p: Params, rho0, ux0=None, uy0=None):
        self.p = p
        self._c = p.c()
        n = (p.ny, p.nx)
        rho0 = np.ascontiguousarray(rho0, dtype=np.float64).reshape(n)
        ux0 = None if ux0 is None else np.ascontiguousarray(ux0, dtype=np.float64).reshape(n)
        uy0 = None if uy0 is None else np.ascontiguousarray(uy0, dtype=np.float64).reshape(n)
        self.f = np.zeros((9, p.ny, p.nx))
        self.work = np.zeros_like(self.f)
        self.t = 0
        st = lib().lbref_init(ctypes.byref(self._c), _ptr(rho0), _ptr(ux0), _ptr(uy0), _ptr(self.f))
        if st:
            raise OracleError(st, "init")

    def step(self, n: int, form: int = FORM_MOMENT):
        done = ctypes.c_int64(0)
        st = lib().lbref_step(ctypes.byref(self._c), _ptr(self.f), _ptr(self.work), int(n), form,
                              ctypes.byref(done))
        self.t += done.value
        if st:
            raise OracleError(st, f"step (completed {done.value} of {n})")
        return self

    def moments(self):
        """rho, ux, uy, Fx, Fy, psi at the current time (Eqs. 6, 7, 24)."""
        shp = (self.p.ny, self.p.nx)
        out = [np.zeros(shp) for _ in range(6)]
        st = lib().lbref_moments(ctypes.byref(self._c), _ptr(self.f), *[_ptr(o) for o in out])
        if st:
            raise OracleError(st, "moments")
        return tuple(out)
