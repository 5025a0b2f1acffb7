"""ctypes wrapper of the plain FP64 CPU oracle (felbm_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests, by the smoke check and by the
benchmark's CPU-baseline leg; never by the product path.  Arrays use the
caller's node order; vector fields are [n_nodes, dim], populations
[2Q, n_nodes] (f then g), matching the oracle's C layout.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "felbm_oracle.c")
_LIB = os.path.join(_HERE, "libfelbm_oracle.so")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


def build(force: bool = False) -> str:
    """Compile the oracle with plain gcc (no fast-math, no vector ISA flags)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fopenmp", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = C.CDLL(_LIB)
        lib.orc_create.restype = C.c_void_p
        lib.orc_create.argtypes = [C.c_int, C.c_int, C.c_int64, _dp, C.c_int64, _ip,
                                   C.POINTER(C.c_int8), _dp, C.POINTER(C.c_uint8), _dp,
                                   C.POINTER(C.c_int)]
        lib.orc_destroy.argtypes = [C.c_void_p]
        for name in ["orc_set_phys", "orc_set_options", "orc_apply_M", "orc_apply_A",
                     "orc_recover_grad", "orc_lumped_mass", "orc_solve_M", "orc_node_terms",
                     "orc_init", "orc_step", "orc_fields", "orc_aux", "orc_last_cg",
                     "orc_conserved", "orc_get_state", "orc_set_state", "orc_beta_kappa",
                     "orc_weak_laplacian", "orc_set_threads", "orc_max_threads"]:
            getattr(lib, name).restype = C.c_int
        lib.orc_set_phys.argtypes = [C.c_void_p, _dp]
        lib.orc_set_options.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double, C.c_int]
        lib.orc_apply_M.argtypes = [C.c_void_p, _dp, _dp]
        lib.orc_apply_A.argtypes = [C.c_void_p, C.c_int, _dp, _dp]
        lib.orc_recover_grad.argtypes = [C.c_void_p, _dp, _dp]
        lib.orc_lumped_mass.argtypes = [C.c_void_p, _dp]
        lib.orc_solve_M.argtypes = [C.c_void_p, _dp, _dp, C.POINTER(C.c_int), _dp]
        lib.orc_node_terms.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, _dp, _dp]
        lib.orc_init.argtypes = [C.c_void_p, _dp, _dp, _dp]
        lib.orc_step.argtypes = [C.c_void_p, C.c_int]
        lib.orc_fields.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
        lib.orc_aux.argtypes = [C.c_void_p, C.c_int, _dp]
        lib.orc_last_cg.argtypes = [C.c_void_p, C.POINTER(C.c_int), _dp]
        lib.orc_conserved.argtypes = [C.c_void_p, _dp]
        lib.orc_get_state.argtypes = [C.c_void_p, _dp]
        lib.orc_set_state.argtypes = [C.c_void_p, _dp]
        lib.orc_beta_kappa.argtypes = [C.c_void_p, _dp]
        lib.orc_weak_laplacian.argtypes = [C.c_void_p, _dp, _dp]
        lib.orc_set_threads.argtypes = [C.c_void_p, C.c_int]
        lib.orc_max_threads.argtypes = []
        _lib = lib
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed with status {rc}")


class Oracle:
    """One mesh, one set of physical parameters, FP64 state on the host."""

    def __init__(self, mesh: dict, lattice: int, phys=None, *, mass_mode: int = 0,
                 lap_mode: int = 0, cg_tol: float = 1e-15, cg_maxit: int = 500):
        lib = _load()
        self.lib = lib
        self.dim = int(mesh["dim"])
        self.Q = int(lattice)
        self._xyz = np.ascontiguousarray(mesh["xyz"], np.float64)
        self._conn = np.ascontiguousarray(mesh["conn"], np.int32)
        self._shift = np.ascontiguousarray(mesh["shift"], np.int8)
        self._box = np.ascontiguousarray(mesh["box"], np.float64)
        self._wall = np.ascontiguousarray(mesh["wall"], np.uint8)
        self._wn = np.ascontiguousarray(mesh["wall_normal"], np.float64)
        self.N = self._xyz.shape[0]
        err = C.c_int(0)
        h = lib.orc_create(self.Q, self.dim, self.N, _d(self._xyz), self._conn.shape[0],
                           self._conn.ctypes.data_as(_ip),
                           self._shift.ctypes.data_as(C.POINTER(C.c_int8)), _d(self._box),
                           self._wall.ctypes.data_as(C.POINTER(C.c_uint8)), _d(self._wn),
                           C.byref(err))
        if not h:
            raise OracleError(f"orc_create failed with status {err.value}")
        self.h = h
        _check(lib.orc_set_options(h, mass_mode, lap_mode, cg_tol, cg_maxit), "set_options")
        if phys is not None:
            self.set_phys(phys)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.orc_destroy(h)
            self.h = None

    # -- parameters and state ------------------------------------------------
    def set_phys(self, phys):
        vals = np.ascontiguousarray(phys.as_tuple() if hasattr(phys, "as_tuple") else phys,
                                    np.float64)
        _check(self.lib.orc_set_phys(self.h, _d(vals)), "set_phys")

    def beta_kappa(self):
        out = np.zeros(2)
        self.lib.orc_beta_kappa(self.h, _d(out))
        return float(out[0]), float(out[1])

    def init(self, rho, u, p):
        rho = np.ascontiguousarray(rho, np.float64)
        u = np.ascontiguousarray(u, np.float64).reshape(self.N, self.dim)
        p = np.ascontiguousarray(p, np.float64)
        _check(self.lib.orc_init(self.h, _d(rho), _d(u), _d(p)), "init")

    def step(self, n: int = 1, *, allow_notconv: bool = False):
        rc = self.lib.orc_step(self.h, int(n))
        if rc == -5 and allow_notconv:
            return rc
        _check(rc, "step")
        return rc

    def fields(self):
        rho = np.zeros(self.N)
        u = np.zeros((self.N, self.dim))
        p = np.zeros(self.N)
        Cc = np.zeros(self.N)
        _check(self.lib.orc_fields(self.h, _d(rho), _d(u), _d(p), _d(Cc)), "fields")
        return dict(rho=rho, u=u, p=p, C=Cc)

    def aux(self, which: str):
        shapes = {"gradrho": (0, (self.N, self.dim)), "lap": (1, (self.N,)),
                  "S": (2, (self.N, self.dim)), "mu": (3, (self.N,)),
                  "gradmu": (4, (self.N, self.dim)), "delta": (5, (2 * self.Q, self.N))}
        idx, shape = shapes[which]
        out = np.zeros(shape)
        _check(self.lib.orc_aux(self.h, idx, _d(out)), "aux")
        return out

    def last_cg(self):
        it = C.c_int(0)
        rel = np.zeros(1)
        self.lib.orc_last_cg(self.h, C.byref(it), _d(rel))
        return it.value, float(rel[0])

    def conserved(self):
        out = np.zeros(6)
        _check(self.lib.orc_conserved(self.h, _d(out)), "conserved")
        return out

    def get_state(self):
        out = np.zeros((2 * self.Q, self.N))
        _check(self.lib.orc_get_state(self.h, _d(out)), "get_state")
        return out

    def set_state(self, psibar):
        a = np.ascontiguousarray(psibar, np.float64).reshape(2 * self.Q, self.N)
        _check(self.lib.orc_set_state(self.h, _d(a)), "set_state")

    def set_threads(self, n: int):
        """Threads over populations in the streaming stage (0 = OpenMP
        default, 1 = serial); results do not depend on it."""
        _check(self.lib.orc_set_threads(self.h, int(n)), "set_threads")

    # -- operators (for the pins) --------------------------------------------
    def weak_laplacian(self, phi):
        """-m^-1 K phi, K = int grad N . grad N^T (natural boundary)."""
        phi = np.ascontiguousarray(phi, np.float64)
        out = np.zeros(self.N)
        _check(self.lib.orc_weak_laplacian(self.h, _d(phi), _d(out)), "weak_laplacian")
        return out

    def apply_M(self, x):
        x = np.ascontiguousarray(x, np.float64)
        y = np.zeros(self.N)
        _check(self.lib.orc_apply_M(self.h, _d(x), _d(y)), "apply_M")
        return y

    def apply_A(self, alpha, x):
        x = np.ascontiguousarray(x, np.float64)
        y = np.zeros(self.N)
        _check(self.lib.orc_apply_A(self.h, int(alpha), _d(x), _d(y)), "apply_A")
        return y

    def recover_grad(self, phi):
        phi = np.ascontiguousarray(phi, np.float64)
        out = np.zeros((self.N, self.dim))
        _check(self.lib.orc_recover_grad(self.h, _d(phi), _d(out)), "recover_grad")
        return out

    def lumped_mass(self):
        m = np.zeros(self.N)
        self.lib.orc_lumped_mass(self.h, _d(m))
        return m

    def solve_M(self, b):
        b = np.ascontiguousarray(b, np.float64)
        x = np.zeros(self.N)
        it = C.c_int(0)
        rel = np.zeros(1)
        rc = self.lib.orc_solve_M(self.h, _d(b), _d(x), C.byref(it), _d(rel))
        if rc not in (0, -5):
            _check(rc, "solve_M")
        return x, it.value, float(rel[0])

    def node_terms(self, rho, u, p, gradrho, S, gradmu):
        v = np.zeros(14)
        v[0] = rho
        v[1:1 + len(u)] = u
        v[4] = p
        v[5:5 + len(gradrho)] = gradrho
        v[8:8 + len(S)] = S
        v[11:11 + len(gradmu)] = gradmu
        outs = [np.zeros(self.Q) for _ in range(5)]
        _check(self.lib.orc_node_terms(self.h, _d(v), *[_d(o) for o in outs]), "node_terms")
        return dict(zip(["feq", "geq", "F", "G", "Gb"], outs))


def max_threads() -> int:
    """Threads the oracle's OpenMP runtime uses by default."""
    return int(_load().orc_max_threads())


def run(instance, lattice: int, steps: int, **kw):
    """Convenience: build an oracle for an inputs.Instance, init, step."""
    o = Oracle(instance.mesh, lattice, instance.phys, **kw)
    o.init(instance.rho0, instance.u0, instance.p0)
    if steps:
        o.step(steps)
    return o
