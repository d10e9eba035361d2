"""ctypes binding of ``libccmsav.so`` (the C ABI of ``include/ccmsav.h``).

Argument marshalling only: every step of the scheme runs in the HIP library.
Fields may be numpy arrays (host memory) or torch tensors (device memory);
PyTorch supplies device memory and the stream, nothing else. If the shared
library is missing this module raises instead of falling back to anything.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Dict, Optional

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libccmsav.so")

FP64 = 0
MIXED = 1
MIXED_GEMM_BF16X3 = 2
PRECISIONS = {"fp64": FP64, "mixed": MIXED, "gemm": MIXED_GEMM_BF16X3}

STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "EDOMAIN",
          -5: "ENONFINITE", -6: "EUNSUPPORTED", -7: "ECONVERGE", -8: "EBARRIER"}

FLAG_GRAPH = 1
FLAG_BDF1 = 2
FLAG_PERIODIC = 4
FLAG_CLASSICAL = 8
FLAG_PERSISTENT = 16
BC_NEUMANN, BC_DIRICHLET, BC_PERIODIC = 0, 1, 2

EXPORTED = (
    "ccmsav_workspace_bytes", "ccmsav_init", "ccmsav_step", "ccmsav_energy",
    "ccmsav_mass", "ccmsav_get_fields", "ccmsav_get_savs", "ccmsav_level",
    "ccmsav_sync", "ccmsav_elliptic_solve", "ccmsav_destroy", "ccmsav_strerror",
    "ccmsav_profile_steps", "ccmsav_workspace_bytes_batch", "ccmsav_init_batch",
    "ccmsav_members", "ccmsav_energy_m", "ccmsav_mass_m", "ccmsav_get_fields_m",
    "ccmsav_get_savs_m", "ccmsav_tuning", "ccmsav_smooth_ic", "ccmsav_physical_energy",
    "ccmsav_physical_energy_m", "ccmsav_set_launch_variants", "ccmsav_elliptic_solve_bc",
    "ccmsav_elliptic_solve_noalloc", "ccmsav_pcg_config", "ccmsav_pcg_stats",
    "ccmsav_set_spin_limit",
)
PHASES = ("stencil", "row_dct", "col_gram", "solve5", "col_solve", "row_idct")


class Params(ctypes.Structure):
    """Mirror of ``ccmsav_params``."""
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("h", ctypes.c_double), ("dt", ctypes.c_double), ("eps", ctypes.c_double),
        ("M_phi", ctypes.c_double), ("M0", ctypes.c_double),
        ("gamma_surf", ctypes.c_double), ("gamma_bend", ctypes.c_double),
        ("gamma_area", ctypes.c_double), ("A", ctypes.c_double),
        ("gamma_in", ctypes.c_double), ("gamma_out", ctypes.c_double),
        ("psi_in", ctypes.c_double), ("psi_out", ctypes.c_double),
        ("beta_in", ctypes.c_double), ("beta_out", ctypes.c_double),
        ("theta", ctypes.c_double), ("lam", ctypes.c_double), ("beta", ctypes.c_double),
        ("precision", ctypes.c_int32), ("flags", ctypes.c_int32),
    ]

    @classmethod
    def from_dict(cls, d: Dict, precision=FP64, flags=0) -> "Params":
        p = cls()
        for name, _ in cls._fields_:
            if name in ("precision", "flags"):
                continue
            setattr(p, name, d[name])
        p.precision = PRECISIONS.get(precision, precision) if isinstance(precision, str) else precision
        p.flags = flags
        return p


class CcmsavError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        self.name = STATUS.get(code, str(code))
        super().__init__(f"{what}: {self.name} ({code}): {strerror(code)}")


_lib = None


def load() -> ctypes.CDLL:
    """Load the in-tree library, or raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing; build it with "
                          "`python -m paper_2601_10057_amd.build`")
    # torch ships its own HIP runtime; loading it first makes the library bind
    # to that same runtime, so that device pointers and streams from torch are
    # valid in the library's calls (a second runtime instance would reject them).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
    lib.ccmsav_workspace_bytes.argtypes = [ctypes.POINTER(Params)]
    lib.ccmsav_workspace_bytes.restype = ctypes.c_size_t
    lib.ccmsav_init.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Params), vp, vp, vp,
                                ctypes.c_size_t, vp]
    lib.ccmsav_step.argtypes = [vp, ctypes.c_int32]
    lib.ccmsav_energy.argtypes = [vp, dp, dp]
    lib.ccmsav_mass.argtypes = [vp, dp, dp]
    lib.ccmsav_get_fields.argtypes = [vp, vp, vp]
    lib.ccmsav_get_savs.argtypes = [vp, dp]
    lib.ccmsav_level.argtypes = [vp]
    lib.ccmsav_level.restype = ctypes.c_int64
    lib.ccmsav_sync.argtypes = [vp]
    lib.ccmsav_profile_steps.argtypes = [vp, ctypes.c_int32, dp]
    lib.ccmsav_elliptic_solve.argtypes = [vp, vp, vp, vp]
    lib.ccmsav_elliptic_solve_bc.argtypes = [vp, ctypes.c_int32, vp, vp, vp]
    lib.ccmsav_elliptic_solve_noalloc.argtypes = [ctypes.POINTER(Params), vp, vp, vp, vp]
    lib.ccmsav_pcg_config.argtypes = [vp, ctypes.c_double, ctypes.c_int32]
    lib.ccmsav_pcg_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), dp]
    lib.ccmsav_set_spin_limit.argtypes = [vp, ctypes.c_uint32]
    lib.ccmsav_smooth_ic.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_int32, vp, vp]
    lib.ccmsav_physical_energy.argtypes = [vp, dp]
    lib.ccmsav_physical_energy_m.argtypes = [vp, ctypes.c_int32, dp]
    lib.ccmsav_set_launch_variants.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    lib.ccmsav_destroy.argtypes = [vp]
    lib.ccmsav_workspace_bytes_batch.argtypes = [ctypes.c_int32, ctypes.POINTER(Params)]
    lib.ccmsav_workspace_bytes_batch.restype = ctypes.c_size_t
    lib.ccmsav_init_batch.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.POINTER(Params),
                                      ctypes.POINTER(vp), ctypes.POINTER(vp), vp,
                                      ctypes.c_size_t, vp]
    lib.ccmsav_members.argtypes = [vp]
    lib.ccmsav_members.restype = ctypes.c_int32
    lib.ccmsav_energy_m.argtypes = [vp, ctypes.c_int32, dp, dp]
    lib.ccmsav_mass_m.argtypes = [vp, ctypes.c_int32, dp, dp]
    lib.ccmsav_get_fields_m.argtypes = [vp, ctypes.c_int32, vp, vp]
    lib.ccmsav_get_savs_m.argtypes = [vp, ctypes.c_int32, dp]
    lib.ccmsav_tuning.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), dp]
    lib.ccmsav_tuning.restype = ctypes.c_int32
    lib.ccmsav_strerror.argtypes = [ctypes.c_int]
    lib.ccmsav_strerror.restype = ctypes.c_char_p
    for fn in ("ccmsav_init", "ccmsav_step", "ccmsav_energy", "ccmsav_mass",
               "ccmsav_get_fields", "ccmsav_get_savs", "ccmsav_sync",
               "ccmsav_elliptic_solve", "ccmsav_smooth_ic", "ccmsav_destroy",
               "ccmsav_physical_energy", "ccmsav_physical_energy_m",
               "ccmsav_set_launch_variants", "ccmsav_elliptic_solve_bc",
               "ccmsav_elliptic_solve_noalloc", "ccmsav_profile_steps",
               "ccmsav_pcg_config", "ccmsav_pcg_stats", "ccmsav_set_spin_limit",
               "ccmsav_init_batch", "ccmsav_energy_m", "ccmsav_mass_m",
               "ccmsav_get_fields_m", "ccmsav_get_savs_m"):
        getattr(lib, fn).restype = ctypes.c_int
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load().ccmsav_strerror(code).decode()


def workspace_bytes(params: Dict, precision=FP64) -> int:
    p = Params.from_dict(params, precision)
    return int(load().ccmsav_workspace_bytes(ctypes.byref(p)))


def elliptic_solve_noalloc(params: Dict, rhs, out_chi, out_zeta, precision="fp64",
                           stream=None):
    """chi^{-1} rhs and zeta^{-1} rhs (device tensors) without a context and
    without allocating: ccmsav_elliptic_solve_noalloc on ``stream`` (default:
    torch's current stream)."""
    p = Params.from_dict(dict(params, A=params.get("A", float("nan"))), precision)
    if stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    _check(load().ccmsav_elliptic_solve_noalloc(ctypes.byref(p), _ptr(rhs), _ptr(out_chi),
                                                _ptr(out_zeta), stream),
           "ccmsav_elliptic_solve_noalloc")


def _ptr(x) -> Optional[int]:
    """Address of a numpy array or torch tensor (None passes through)."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        if x.dtype != np.float64 or not x.flags["C_CONTIGUOUS"]:
            raise ValueError("fields must be C-contiguous float64 arrays")
        return x.ctypes.data
    if hasattr(x, "data_ptr"):
        import torch
        if x.dtype != torch.float64 or not x.is_contiguous():
            raise ValueError("fields must be contiguous float64 tensors")
        return x.data_ptr()
    raise TypeError(f"unsupported field type {type(x)}")


def _check(code: int, what: str):
    if code != 0:
        raise CcmsavError(code, what)


class Context:
    """CC-MSAV simulation of one vesicle, or of an ensemble of independent
    vesicles advanced in lock step, on the GPU and bound to a HIP stream.

    ``Context(params, phi0, psi0)`` holds one member; ``Context.ensemble``
    builds a context of several (each with its own parameters and grid).
    Member-indexed queries take ``member`` (default 0). ``bdf1=True`` takes
    every step with the first-order CC-MSAV-BDF1 scheme; ``periodic=True``
    takes periodic boundaries (FP64, one member); ``classical=True`` the
    classical MSAV scheme with its PCG solves (FP64, one member);
    ``persistent=True`` runs every step as one persistent kernel launch
    (mixed precision, grids of 64 to 512).
    """

    def __init__(self, params, phi0, psi0, precision="fp64", workspace=None,
                 stream=None, torch_workspace: bool = True, graph: bool = False,
                 bdf1: bool = False, periodic: bool = False, classical: bool = False,
                 persistent: bool = False):
        self._init([params], [phi0], [psi0], precision, workspace, stream, torch_workspace, graph,
                   bdf1, periodic, classical, persistent)

    @classmethod
    def ensemble(cls, params_list, phi0_list, psi0_list, precision="fp64", workspace=None,
                 stream=None, torch_workspace: bool = True, graph: bool = False,
                 bdf1: bool = False, periodic: bool = False,
                 classical: bool = False, persistent: bool = False) -> "Context":
        self = cls.__new__(cls)
        self._init(list(params_list), list(phi0_list), list(psi0_list), precision, workspace,
                   stream, torch_workspace, graph, bdf1, periodic, classical, persistent)
        return self

    def _init(self, params_list, phi0_list, psi0_list, precision, workspace, stream,
              torch_workspace, graph, bdf1=False, periodic=False, classical=False,
              persistent=False):
        lib = load()
        self._h = None
        n = len(params_list)
        if n == 0 or len(phi0_list) != n or len(psi0_list) != n:
            raise ValueError("one parameter set and two initial fields per member")
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else precision
        flags = ((FLAG_GRAPH if graph else 0) | (FLAG_BDF1 if bdf1 else 0)
                 | (FLAG_PERIODIC if periodic else 0) | (FLAG_CLASSICAL if classical else 0)
                 | (FLAG_PERSISTENT if persistent else 0))
        self.params_list = [dict(p) for p in params_list]
        self.params = self.params_list[0]
        parr = (Params * n)(*[Params.from_dict(p, self.precision, flags) for p in params_list])
        self._p = parr
        self.shapes = [(int(p["ny"]), int(p["nx"])) for p in params_list]
        self.ny, self.nx = self.shapes[0]
        nbytes = int(lib.ccmsav_workspace_bytes_batch(n, parr))
        self._ws = workspace
        if self._ws is None and torch_workspace and nbytes:
            import torch
            if torch.cuda.is_available():
                self._ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        if stream is None:
            try:
                import torch
                stream = torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else None
            except ImportError:
                stream = None
        self._stream = stream
        ptr_phi = (ctypes.c_void_p * n)(*[_ptr(x) for x in phi0_list])
        ptr_psi = (ctypes.c_void_p * n)(*[_ptr(x) for x in psi0_list])
        h = ctypes.c_void_p()
        ws_ptr = self._ws.data_ptr() if self._ws is not None else None
        ws_len = nbytes if self._ws is not None else 0
        code = lib.ccmsav_init_batch(ctypes.byref(h), n, parr, ptr_phi, ptr_psi, ws_ptr, ws_len,
                                     stream)
        _check(code, "ccmsav_init_batch")
        self._h = h

    # -- stepping and diagnostics ------------------------------------------
    @property
    def members(self) -> int:
        return int(load().ccmsav_members(self._h))

    def step(self, nsteps: int = 1):
        _check(load().ccmsav_step(self._h, int(nsteps)), "ccmsav_step")

    def profile_steps(self, nsteps: int) -> Dict[str, float]:
        """Take ``nsteps`` steps with HIP events around each kernel; mean ms per launch."""
        buf = (ctypes.c_double * len(PHASES))()
        _check(load().ccmsav_profile_steps(self._h, int(nsteps), buf), "ccmsav_profile_steps")
        return dict(zip(PHASES, list(buf)))

    def sync(self):
        _check(load().ccmsav_sync(self._h), "ccmsav_sync")

    def tuning(self):
        """Autotuner choices per grid shape: [{nx, ny, variants, ms}], empty before step 1."""
        lib = load()
        n = int(lib.ccmsav_tuning(self._h, 0, None, None))
        if n < 0:
            _check(n, "ccmsav_tuning")
        if n == 0:
            return []
        info = (ctypes.c_int32 * (5 * n))()
        ms = (ctypes.c_double * (6 * n))()
        lib.ccmsav_tuning(self._h, n, info, ms)
        names = ("row_dct", "col_solve", "row_idct")
        return [dict(nx=info[5 * s], ny=info[5 * s + 1],
                     variants={names[t]: info[5 * s + 2 + t] for t in range(3)},
                     ms={names[t]: [ms[6 * s + 2 * t], ms[6 * s + 2 * t + 1]] for t in range(3)})
                for s in range(n)]

    @property
    def level(self) -> int:
        return int(load().ccmsav_level(self._h))

    def energy(self, parts: bool = False, member: int = 0):
        e = ctypes.c_double()
        buf = (ctypes.c_double * 9)()
        _check(load().ccmsav_energy_m(self._h, member, ctypes.byref(e), buf), "ccmsav_energy")
        return (e.value, list(buf)) if parts else e.value

    def mass(self, member: int = 0):
        a, b = ctypes.c_double(), ctypes.c_double()
        _check(load().ccmsav_mass_m(self._h, member, ctypes.byref(a), ctypes.byref(b)),
               "ccmsav_mass")
        return a.value, b.value

    def fields(self, member: int = 0):
        """(phi^n, psi^n) of a member copied to host numpy arrays."""
        ny, nx = self.shapes[member]
        phi = np.empty((ny, nx))
        psi = np.empty((ny, nx))
        _check(load().ccmsav_get_fields_m(self._h, member, phi.ctypes.data, psi.ctypes.data),
               "ccmsav_get_fields")
        return phi, psi

    def fields_into(self, phi, psi, member: int = 0):
        _check(load().ccmsav_get_fields_m(self._h, member, _ptr(phi), _ptr(psi)),
               "ccmsav_get_fields")

    def savs(self, member: int = 0):
        """(V, U, W, Z) at level n and at level n-1."""
        buf = (ctypes.c_double * 8)()
        _check(load().ccmsav_get_savs_m(self._h, member, buf), "ccmsav_get_savs")
        v = np.array(list(buf))
        return v[:4], v[4:]

    def elliptic_solve(self, rhs, out_chi, out_zeta, bc: str = "neumann"):
        """chi^{-1} rhs and zeta^{-1} rhs (device tensors) with the BDF2
        operators, for homogeneous Neumann (DCT), Dirichlet (DST) or periodic
        (FFT) boundaries."""
        code = {"neumann": BC_NEUMANN, "dirichlet": BC_DIRICHLET, "periodic": BC_PERIODIC}[bc]
        _check(load().ccmsav_elliptic_solve_bc(self._h, code, _ptr(rhs), _ptr(out_chi),
                                               _ptr(out_zeta)), "ccmsav_elliptic_solve_bc")

    def pcg_config(self, tol: float = 1e-12, max_iter: int = 40):
        """Classical scheme: PCG stopping tolerance and iterations per step."""
        _check(load().ccmsav_pcg_config(self._h, float(tol), int(max_iter)), "ccmsav_pcg_config")

    def set_spin_limit(self, polls: int):
        """Persistent launch: polls a workgroup waits at a grid barrier before
        giving up (EBARRIER at the next synchronising call)."""
        _check(load().ccmsav_set_spin_limit(self._h, int(polls)), "ccmsav_set_spin_limit")

    def pcg_stats(self):
        """Classical scheme: ([iterations], [relative residuals]) of the last step's two solves."""
        it = (ctypes.c_int32 * 2)()
        rr = (ctypes.c_double * 2)()
        _check(load().ccmsav_pcg_stats(self._h, it, rr), "ccmsav_pcg_stats")
        return list(it), list(rr)

    def set_launch_variants(self, row_dct: int = -1, col_solve: int = -1, row_idct: int = -1):
        """Fix the launch variants (0 or 1; -1 keeps the current choice)."""
        v = (ctypes.c_int32 * 3)(row_dct, col_solve, row_idct)
        _check(load().ccmsav_set_launch_variants(self._h, v), "ccmsav_set_launch_variants")

    def physical_energy(self, member: int = 0):
        """F and its parts (Sec. 2.1) at the current level, and the arc length."""
        out = (ctypes.c_double * 6)()
        _check(load().ccmsav_physical_energy_m(self._h, int(member), out),
               "ccmsav_physical_energy_m")
        return dict(zip(("F", "surf", "bend", "area", "osm", "arc_length"), list(out)))

    def smooth_ic(self, phi_sharp, M: float = 0.01, dt: float = 1e-6, nsteps: int = 10):
        """App. F relaxation of a sharp phase field on this context's grid;
        returns the smoothed, clipped field as a numpy array."""
        src = phi_sharp
        if isinstance(src, np.ndarray):
            src = np.ascontiguousarray(src, dtype=np.float64)
        if tuple(src.shape) != self.shapes[0]:
            raise ValueError(f"phi_sharp must have shape {self.shapes[0]}")
        out = np.empty(self.shapes[0], dtype=np.float64)
        _check(load().ccmsav_smooth_ic(self._h, float(M), float(dt), int(nsteps), _ptr(src),
                                       _ptr(out)), "ccmsav_smooth_ic")
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().ccmsav_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def mcell_steps(n_cells: int, steps: int, seconds: float) -> float:
    return n_cells * steps / seconds / 1e6 if seconds > 0 else math.nan
