"""ctypes front end of the FP64 CPU oracle (``oracle/lbm_ref.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of the benchmark
may import this module; the product path never does.  The oracle shares no code with the HIP
path; only plain parameter dictionaries and seeded NumPy arrays cross between the two.

Parameters are plain dicts with the keys of :data:`DEFAULTS` (the paper's values, Sec. 4).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_ref.c")
LIB = os.path.join(HERE, "liblbmref.so")

ISOTHERMAL, ADIABATIC, PERIODIC = 0, 1, 2

# Paper defaults (Sec. 4): rho0 = 1, varpi = -2, J = 1, sigma = 1, Ma = 0.1, rates 1.1/1.1/1.2
# and 1.5/1.5; hot west wall T = 1, cold east wall T = 0, adiabatic south/north walls.
DEFAULTS = dict(
    nx=64, ny=64,
    bc=(ISOTHERMAL, ISOTHERMAL, ADIABATIC, ADIABATIC),
    T_wall=(1.0, 0.0, 0.0, 0.0),
    Ra=1e3, Pr=1.0, Da=1e-2, J=1.0,
    Ma=0.1, sigma=1.0, varpi=-2.0, rho0=1.0,
    s_e=1.1, s_eps=1.1, s_q=1.2, zeta3=1.5, zeta4=1.5,
    forchheimer=1, T_init=0.5, ext_accel=(0.0, 0.0),
    tau_v=-1.0, tau_T=-1.0, gbeta=-1.0,
    uniform_rates=0, Ra_I=0.0, Qv=0.0,
)

DERIVED_NAMES = ("L", "cs2", "csT2", "tau_v", "tau_T", "nu_e", "nu", "gbeta", "dT", "T0",
                 "K_uniform", "Q")


class RefParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("bc", C.c_int32 * 4),
        ("T_wall", C.c_double * 4),
        ("Ra", C.c_double), ("Pr", C.c_double), ("Da", C.c_double), ("J", C.c_double),
        ("Ma", C.c_double), ("sigma", C.c_double), ("varpi", C.c_double), ("rho0", C.c_double),
        ("s_e", C.c_double), ("s_eps", C.c_double), ("s_q", C.c_double),
        ("zeta3", C.c_double), ("zeta4", C.c_double),
        ("forchheimer", C.c_int32),
        ("T_init", C.c_double),
        ("ext_accel", C.c_double * 2),
        ("tau_v", C.c_double), ("tau_T", C.c_double),
        ("gbeta", C.c_double),
        ("uniform_rates", C.c_int32),
        ("Ra_I", C.c_double), ("Qv", C.c_double),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain FP64, no fast-math, no contraction, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    """The oracle library; LBM_REF_LIB names another build of it (the mutation tests load
    deliberately broken copies of the oracle this way)."""
    global _lib
    if _lib is None:
        path = os.environ.get("LBM_REF_LIB")
        if not path:
            build()
            path = LIB
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        L.ref_create.restype = C.c_void_p
        L.ref_create.argtypes = [C.POINTER(RefParams), dp, C.c_double, dp]
        L.ref_destroy.argtypes = [C.c_void_p]
        L.ref_step.argtypes = [C.c_void_p, C.c_int64]
        L.ref_observables.argtypes = [C.c_void_p, dp, dp, dp, dp, dp]
        L.ref_get_step.restype = C.c_int64
        L.ref_get_step.argtypes = [C.c_void_p]
        L.ref_get_state.argtypes = [C.c_void_p, dp, dp]
        L.ref_set_state.argtypes = [C.c_void_p, dp, dp, C.c_int64]
        L.ref_set_threads.argtypes = [C.c_int]
        L.ref_get_threads.restype = C.c_int
        L.ref_derive.argtypes = [C.POINTER(RefParams), dp]
        L.ref_matrices.argtypes = [dp, dp, dp, dp]
        L.ref_feq.argtypes = [C.c_double] * 5 + [dp]
        L.ref_meq.argtypes = [C.c_double] * 5 + [dp]
        L.ref_forcing.argtypes = [C.c_double] * 6 + [dp]
        L.ref_geq.argtypes = [C.c_double] * 5 + [dp]
        L.ref_neq.argtypes = [C.c_double] * 5 + [dp]
        L.ref_macros.argtypes = [C.POINTER(RefParams), dp, dp, C.c_double, C.c_double, dp]
        L.ref_collide_fluid_node.argtypes = [C.POINTER(RefParams), dp, dp, C.c_double,
                                             C.c_double, dp, dp]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(**kw) -> RefParams:
    d = dict(DEFAULTS)
    unknown = set(kw) - set(d)
    if unknown:
        raise KeyError(f"unknown oracle parameters {sorted(unknown)}")
    d.update(kw)
    p = RefParams()
    for k, v in d.items():
        if k in ("bc", "T_wall", "ext_accel"):
            arr = getattr(p, k)
            for i, x in enumerate(v):
                arr[i] = x
        else:
            setattr(p, k, v)
    return p


def derived(**kw) -> dict:
    out = np.zeros(len(DERIVED_NAMES))
    lib().ref_derive(C.byref(make_params(**kw)), _ptr(out))
    return dict(zip(DERIVED_NAMES, out.tolist()))


def set_threads(n: int) -> None:
    lib().ref_set_threads(int(n))


def get_threads() -> int:
    return int(lib().ref_get_threads())


class RefLattice:
    """One cavity on the CPU.  phi and K are [ny][nx] float64 arrays or None (uniform)."""

    def __init__(self, phi=None, K=None, phi_uniform: float = 0.6, **params):
        self.params = dict(DEFAULTS)
        self.params.update(params)
        self.nx, self.ny = int(self.params["nx"]), int(self.params["ny"])
        self._p = make_params(**params)
        self._phi = None if phi is None else np.ascontiguousarray(phi, dtype=np.float64)
        self._K = None if K is None else np.ascontiguousarray(K, dtype=np.float64)
        for a in (self._phi, self._K):
            if a is not None and a.shape != (self.ny, self.nx):
                raise ValueError(f"field shape {a.shape} != {(self.ny, self.nx)}")
        self._phi_uniform = float(phi_uniform)
        self._h = lib().ref_create(C.byref(self._p), _ptr(self._phi), float(phi_uniform),
                                   _ptr(self._K))
        if not self._h:
            raise MemoryError("ref_create failed")

    def close(self):
        if self._h:
            lib().ref_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1) -> None:
        lib().ref_step(self._h, int(n))

    @property
    def time(self) -> int:
        return int(lib().ref_get_step(self._h))

    def observables(self, dynamic_pressure: bool = False) -> dict:
        """Fields u_x, u_y, p (Eq. (23)), T (Eq. (36)) and Nu_hot, Nu_cold (Eq. (38)); with
        ``dynamic_pressure`` p less its rest value rho0 cs^2 / phi (cs^2 = 1/3), node by node.
        Also max |u|, the mass deviation, min and max T, max |phi p - rho0 cs^2| and the
        divergence flag (non-finite u, p, T or |v|; |u| > cs; T outside the bounds of the
        walls, T_init and the heat source widened by dT)."""
        shp = (self.ny, self.nx)
        ux, uy, p, T = (np.empty(shp) for _ in range(4))
        out = np.zeros(8)
        lib().ref_observables(self._h, _ptr(ux), _ptr(uy), _ptr(p), _ptr(T), _ptr(out))
        if dynamic_pressure:
            phi = self._phi if self._phi is not None else self._phi_uniform
            p = p - self.params["rho0"] / 3.0 / phi
        return dict(ux=ux, uy=uy, p=p, T=T, nu_hot=out[0], nu_cold=out[1], max_speed=out[2],
                    mass_err=out[3], diverged=bool(out[4]), T_min=out[5], T_max=out[6],
                    phip_dev_max=out[7])

    def get_state(self):
        f = np.empty((9, self.ny, self.nx))
        g = np.empty((5, self.ny, self.nx))
        lib().ref_get_state(self._h, _ptr(f), _ptr(g))
        return f, g

    def set_state(self, f, g, step: int = 0) -> None:
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(9, self.ny, self.nx)
        g = np.ascontiguousarray(g, dtype=np.float64).reshape(5, self.ny, self.nx)
        lib().ref_set_state(self._h, _ptr(f), _ptr(g), int(step))


# ---- single formulas, for the pin tests -------------------------------------------------------

def matrices():
    M, Mi = np.zeros((9, 9)), np.zeros((9, 9))
    N, Ni = np.zeros((5, 5)), np.zeros((5, 5))
    lib().ref_matrices(_ptr(M), _ptr(Mi), _ptr(N), _ptr(Ni))
    return M, Mi, N, Ni


def feq(phip, ux, uy, phi, rho0=1.0):
    out = np.zeros(9)
    lib().ref_feq(phip, ux, uy, phi, rho0, _ptr(out))
    return out


def meq(phip, ux, uy, phi, rho0=1.0):
    out = np.zeros(9)
    lib().ref_meq(phip, ux, uy, phi, rho0, _ptr(out))
    return out


def forcing(ux, uy, Fx, Fy, phi, rho0=1.0):
    out = np.zeros(9)
    lib().ref_forcing(ux, uy, Fx, Fy, phi, rho0, _ptr(out))
    return out


def geq(T, ux, uy, sigma=1.0, varpi=-2.0):
    out = np.zeros(5)
    lib().ref_geq(T, ux, uy, sigma, varpi, _ptr(out))
    return out


def neq(T, ux, uy, sigma=1.0, varpi=-2.0):
    out = np.zeros(5)
    lib().ref_neq(T, ux, uy, sigma, varpi, _ptr(out))
    return out


def macros(fh, gh, phi, K, **params):
    """Fluid-node macroscopics: dict(T, ux, uy, phip, Fx, Fy)."""
    out = np.zeros(6)
    fh = np.ascontiguousarray(fh, dtype=np.float64)
    gh = np.ascontiguousarray(gh, dtype=np.float64)
    lib().ref_macros(C.byref(make_params(**params)), _ptr(fh), _ptr(gh), phi, K, _ptr(out))
    return dict(zip(("T", "ux", "uy", "phip", "Fx", "Fy"), out.tolist()))


def collide_fluid_node(fh, gh, phi, K, **params):
    fp, gp = np.zeros(9), np.zeros(5)
    fh = np.ascontiguousarray(fh, dtype=np.float64)
    gh = np.ascontiguousarray(gh, dtype=np.float64)
    lib().ref_collide_fluid_node(C.byref(make_params(**params)), _ptr(fh), _ptr(gh), phi, K,
                                 _ptr(fp), _ptr(gp))
    return fp, gp


if __name__ == "__main__":
    build(force="--force" in sys.argv)
    print(LIB)
