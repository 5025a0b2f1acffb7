"""Thin ctypes binding of libfelbm.so (the HIP library, C ABI in include/felbm.h).

Argument marshalling only: every step of the method runs in the library's
kernels.  PyTorch supplies the device workspace (one uint8 tensor) and the
stream.  Importing this module fails loudly if the library is not built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfelbm.so")

FEL_OK, FEL_EINVAL, FEL_ENOMEM, FEL_EDEVICE, FEL_ESTATE, FEL_ENOTCONV, FEL_ENONFINITE = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "FEL_OK", -1: "FEL_EINVAL", -2: "FEL_ENOMEM", -3: "FEL_EDEVICE", -4: "FEL_ESTATE",
                -5: "FEL_ENOTCONV", -6: "FEL_ENONFINITE"}
PREC = {"fp64": 0, "fp32": 1, "fp32_fp16": 2}
AUX = {"gradrho": 0, "mu": 1, "S": 2, "delta": 3}

# every symbol declared in include/felbm.h
ABI_SYMBOLS = ["fel_create", "fel_upload_mesh", "fel_workspace_size", "fel_bind", "fel_bind_static", "fel_init_fields",
               "fel_step", "fel_sync", "fel_read_fields", "fel_conserved_sums", "fel_get_state",
               "fel_set_state", "fel_read_aux", "fel_profile", "fel_profile_read", "fel_layout_info",
               "fel_stage_tables", "fel_tuning", "fel_destroy", "fel_last_error", "fel_version"]


class FelOptions(C.Structure):
    _fields_ = [("lattice", C.c_int), ("precision", C.c_int), ("mass_mode", C.c_int), ("cg_iters", C.c_int),
                ("cg_tol", C.c_double), ("laplacian_mode", C.c_int), ("max_instances", C.c_int),
                ("node_order", C.c_int), ("solver_batch", C.c_int), ("lds_staging", C.c_int),
                ("fused_reductions", C.c_int)]


class FelPhys(C.Structure):
    _fields_ = [("rho_l", C.c_double), ("rho_v", C.c_double), ("tau_l", C.c_double), ("tau_v", C.c_double),
                ("sigma", C.c_double), ("xi", C.c_double), ("dt", C.c_double), ("grav", C.c_double * 3)]


class FelError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None
_vp = C.c_void_p
_dp = C.POINTER(C.c_double)


def load_library():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(the HIP library has no fallback)")
    # torch ships its own HIP runtime under the same soname (libamdhip64.so.7);
    # loading torch first makes the dynamic loader reuse that one runtime for
    # the library, so device pointers and streams from torch are native to it.
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    for name in ABI_SYMBOLS:
        getattr(lib, name)
    lib.fel_create.argtypes = [C.POINTER(FelOptions), C.POINTER(_vp)]
    lib.fel_upload_mesh.argtypes = [_vp, C.c_int, C.c_int, C.c_int64, _dp, C.c_int64, C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int8), _dp, C.POINTER(C.c_uint8), _dp]
    lib.fel_workspace_size.argtypes = [_vp, C.POINTER(C.c_size_t)]
    lib.fel_bind.argtypes = [_vp, _vp, C.c_size_t, _vp]
    lib.fel_bind_static.argtypes = [_vp, _vp]
    lib.fel_init_fields.argtypes = [_vp, C.c_int, C.POINTER(FelPhys), _dp, _dp, _dp]
    lib.fel_step.argtypes = [_vp, C.c_int]
    lib.fel_sync.argtypes = [_vp]
    lib.fel_read_fields.argtypes = [_vp, C.c_int, _dp, _dp, _dp, _dp]
    lib.fel_conserved_sums.argtypes = [_vp, C.c_int, _dp]
    lib.fel_get_state.argtypes = [_vp, C.c_int, _dp]
    lib.fel_set_state.argtypes = [_vp, C.c_int, _dp]
    lib.fel_read_aux.argtypes = [_vp, C.c_int, C.c_int, _dp]
    lib.fel_profile.argtypes = [_vp, C.c_int]
    lib.fel_profile_read.argtypes = [_vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int64), _dp,
                                     C.POINTER(C.c_char_p)]
    lib.fel_layout_info.argtypes = [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                    C.POINTER(C.c_int), C.POINTER(C.c_int), _dp]
    lib.fel_stage_tables.argtypes = [_vp, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int64), _vp, _vp, _vp]
    lib.fel_tuning.argtypes = [_vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                               C.POINTER(C.c_int)]
    lib.fel_destroy.argtypes = [_vp]
    lib.fel_last_error.argtypes = [_vp]
    lib.fel_last_error.restype = C.c_char_p
    lib.fel_version.restype = C.c_char_p
    for name in ABI_SYMBOLS:
        if name not in ("fel_last_error", "fel_version"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _d(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _phys(ph) -> FelPhys:
    t = ph.as_tuple() if hasattr(ph, "as_tuple") else tuple(ph)
    p = FelPhys()
    p.rho_l, p.rho_v, p.tau_l, p.tau_v, p.sigma, p.xi, p.dt = t[:7]
    for i in range(3):
        p.grav[i] = t[7 + i] if len(t) > 7 + i else 0.0
    return p


class Context:
    """One felbm context: instances uploaded, bound to a torch workspace/stream."""

    def __init__(self, lattice: int, *, precision: str = "fp64", mass_mode: int = 0, cg_iters: int = 0,
                 cg_tol: float = 0.0, laplacian_mode: int = 0, max_instances: int = 1, node_order: int = 0,
                 solver_batch: int = 0, lds_staging: int = 0, fused_reductions: int = 0):
        self.lib = load_library()
        opt = FelOptions(lattice, PREC[precision], mass_mode, cg_iters, cg_tol, laplacian_mode, max_instances,
                         node_order, solver_batch, lds_staging, fused_reductions)
        h = _vp()
        st = self.lib.fel_create(C.byref(opt), C.byref(h))
        if st != FEL_OK:
            raise FelError(st, "fel_create rejected the options")
        self.h = h
        self.lattice = lattice
        self.dim = 2 if lattice == 9 else 3
        self.n_nodes = {}
        self.workspace = None
        self.stream = None

    def _check(self, st, what):
        if st != FEL_OK:
            msg = self.lib.fel_last_error(self.h)
            raise FelError(st, f"{what}: {msg.decode() if msg else ''}")
        return st

    def close(self):
        if getattr(self, "h", None):
            self.lib.fel_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- setup ----------------------------------------------------------------
    def upload_mesh(self, inst: int, mesh: dict):
        xyz = np.ascontiguousarray(mesh["xyz"], np.float64)
        conn = np.ascontiguousarray(mesh["conn"], np.int32)
        shift = np.ascontiguousarray(mesh["shift"], np.int8) if mesh.get("shift") is not None else None
        box = np.ascontiguousarray(mesh["box"], np.float64) if mesh.get("box") is not None else None
        wall = np.ascontiguousarray(mesh["wall"], np.uint8) if mesh.get("wall") is not None else None
        wn = np.ascontiguousarray(mesh["wall_normal"], np.float64) if mesh.get("wall_normal") is not None else None
        self._check(self.lib.fel_upload_mesh(
            self.h, inst, int(mesh["dim"]), xyz.shape[0], _d(xyz), conn.shape[0],
            conn.ctypes.data_as(C.POINTER(C.c_int32)),
            shift.ctypes.data_as(C.POINTER(C.c_int8)) if shift is not None else None, _d(box),
            wall.ctypes.data_as(C.POINTER(C.c_uint8)) if wall is not None else None, _d(wn)),
            "fel_upload_mesh")
        self.n_nodes[inst] = xyz.shape[0]

    def workspace_size(self) -> int:
        n = C.c_size_t(0)
        self._check(self.lib.fel_workspace_size(self.h, C.byref(n)), "fel_workspace_size")
        return n.value

    def bind(self, device: str = "cuda:0", stream=None):
        import torch
        nbytes = self.workspace_size()
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        self._check(self.lib.fel_bind(self.h, C.c_void_p(aligned), nbytes, C.c_void_p(self.stream.cuda_stream)),
                    "fel_bind")

    def bind_static(self, device: str = "cuda:0", stream=None):
        """Binds to the library's static device workspace (no device memory
        is allocated for the context); `stream` as in bind."""
        import torch
        torch.cuda.set_device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        self._check(self.lib.fel_bind_static(self.h, C.c_void_p(self.stream.cuda_stream)), "fel_bind_static")

    def init_fields(self, inst: int, phys, rho, u=None, p=None):
        rho = np.ascontiguousarray(rho, np.float64)
        u = np.ascontiguousarray(u, np.float64).reshape(rho.size, self.dim) if u is not None else None
        p = np.ascontiguousarray(p, np.float64) if p is not None else None
        ph = _phys(phys)
        self._check(self.lib.fel_init_fields(self.h, inst, C.byref(ph), _d(rho), _d(u), _d(p)), "fel_init_fields")

    # -- stepping -------------------------------------------------------------
    def step(self, n: int = 1):
        self._check(self.lib.fel_step(self.h, int(n)), "fel_step")

    def sync(self, *, allow_notconv: bool = False):
        st = self.lib.fel_sync(self.h)
        if st == FEL_ENOTCONV and allow_notconv:
            return st
        return self._check(st, "fel_sync")

    # -- read-back ------------------------------------------------------------
    def read_fields(self, inst: int = 0):
        N = self.n_nodes[inst]
        rho, u, p, Cc = np.zeros(N), np.zeros((N, self.dim)), np.zeros(N), np.zeros(N)
        self._check(self.lib.fel_read_fields(self.h, inst, _d(rho), _d(u), _d(p), _d(Cc)), "fel_read_fields")
        return dict(rho=rho, u=u, p=p, C=Cc)

    def conserved_sums(self, inst: int = 0):
        out = np.zeros(6)
        self._check(self.lib.fel_conserved_sums(self.h, inst, _d(out)), "fel_conserved_sums")
        return out

    def get_state(self, inst: int = 0):
        out = np.zeros((2 * self.lattice, self.n_nodes[inst]))
        self._check(self.lib.fel_get_state(self.h, inst, _d(out)), "fel_get_state")
        return out

    def set_state(self, inst: int, psibar):
        a = np.ascontiguousarray(psibar, np.float64)
        self._check(self.lib.fel_set_state(self.h, inst, _d(a)), "fel_set_state")

    def read_aux(self, inst: int, which: str):
        N = self.n_nodes[inst]
        shape = {"gradrho": (N, self.dim), "mu": (N,), "S": (N, self.dim), "delta": (2 * self.lattice, N)}[which]
        out = np.zeros(shape)
        self._check(self.lib.fel_read_aux(self.h, inst, AUX[which], _d(out)), "fel_read_aux")
        return out

    def profile(self, enable: bool):
        self._check(self.lib.fel_profile(self.h, 1 if enable else 0), "fel_profile")

    def profile_read(self):
        n = C.c_int(0)
        counts = (C.c_int64 * 32)()
        ms = (C.c_double * 32)()
        names = (C.c_char_p * 32)()
        self._check(self.lib.fel_profile_read(self.h, 32, C.byref(n), counts, ms, names), "fel_profile_read")
        return {names[k].decode(): (int(counts[k]), float(ms[k])) for k in range(n.value)}

    def layout_info(self):
        rows, w, pops, it = C.c_int64(0), C.c_int(0), C.c_int(0), C.c_int(0)
        hmax, hmean = C.c_int(0), C.c_double(0.0)
        self._check(self.lib.fel_layout_info(self.h, C.byref(rows), C.byref(w), C.byref(pops), C.byref(it),
                                             C.byref(hmax), C.byref(hmean)), "fel_layout_info")
        return dict(rows=rows.value, ell_width=w.value, pops=pops.value, cg_iters=it.value, halo_max=hmax.value,
                    halo_mean=hmean.value)

    def stage_tables(self, form: int):
        """LDS staging tables of the layout before binding (form 2 per tile,
        3 per wavefront): lcol [ell_width][rows] uint16, list_ptr, list_col."""
        nl, nc = C.c_int64(0), C.c_int64(0)
        self._check(self.lib.fel_stage_tables(self.h, form, C.byref(nl), C.byref(nc), None, None, None),
                    "fel_stage_tables")
        info = self.layout_info()
        lcol = np.zeros((info["ell_width"], info["rows"]), np.uint16)
        ptr = np.zeros(nl.value + 1, np.int32)
        col = np.zeros(max(nc.value, 1), np.int32)
        self._check(self.lib.fel_stage_tables(self.h, form, C.byref(nl), C.byref(nc), lcol.ctypes.data,
                                              ptr.ctypes.data, col.ctypes.data), "fel_stage_tables")
        return dict(lcol=lcol, list_ptr=ptr, list_col=col[:nc.value])

    def tuning(self):
        """Schedule in use, keyed by kernel class name: (population batch,
        staging: 1 direct gathers, 2 LDS-staged per tile, 3 per wavefront);
        under "fused" the CG reduction form (1 finalize launches, 2 fused)."""
        n, fused = C.c_int(0), C.c_int(0)
        batch, staging = (C.c_int * 32)(), (C.c_int * 32)()
        self._check(self.lib.fel_tuning(self.h, 32, C.byref(n), batch, staging, C.byref(fused)), "fel_tuning")
        names = self.profile_read()
        out = {name: (batch[k], staging[k]) for k, name in enumerate(list(names)[:n.value])}
        out["fused"] = fused.value
        return out


def from_workload(workload, *, precision: str = "fp64", device: str = "cuda:0", stream=None, **opts) -> Context:
    """Context with every instance of an inputs.Workload uploaded, bound and initialised."""
    ctx = Context(workload.lattice, precision=precision, max_instances=len(workload.instances), **opts)
    for i, inst in enumerate(workload.instances):
        ctx.upload_mesh(i, inst.mesh)
    ctx.bind(device, stream)
    for i, inst in enumerate(workload.instances):
        ctx.init_fields(i, inst.phys, inst.rho0, inst.u0, inst.p0)
    return ctx
