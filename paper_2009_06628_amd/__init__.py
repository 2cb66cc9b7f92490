"""MI355X-native split time step of the two-phase Cahn-Hilliard Navier-Stokes
model (Khanwale et al., arXiv 2009.06628) -- Python binding.

The binding only marshals arguments: every step of the path runs in the HIP
kernels of libchns.so (built in-tree by ``paper_2009_06628_amd.build``).
PyTorch supplies device memory and the stream.  There is no CPU fallback: if
the library or a GPU is missing, every entry point raises.

Names follow the C ABI in include/chns.h: create_grid / set_properties /
step / solve_pressure / adjoint_step (plus workspace_size,
apply_pressure_operator and the timing calls).  The differentiable rollout
(torch.autograd.Function with checkpointing) is in ``.adjoint``.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libchns.so")

CHNS_OK, CHNS_ENOCONV, CHNS_EINVAL, CHNS_ENOMEM, CHNS_EDEVICE, CHNS_ENONFINITE = 0, 1, -1, -2, -3, -4
CHNS_BC_PERIODIC, CHNS_BC_WALL = 0, 1
CHNS_FP64, CHNS_FP32_REFINE = 0, 1
CHNS_OPT_CH_SOLVER, CHNS_OPT_SERIAL_COMPONENTS, CHNS_OPT_TIME_SCHEME, CHNS_OPT_PICARD_ITERATIONS = 1, 2, 3, 4
CHNS_OPT_MARCH_SWEEP_CELLS = 5
CHNS_OPT_TILE_CYCLE_CELLS = 6
CHNS_OPT_TIME_GUESS = 7
CHNS_CH_DIRECT, CHNS_CH_PCG, CHNS_CH_DIRECT_DENSE = 0, 1, 2
CHNS_SCHEME_SPLIT, CHNS_SCHEME_CN = 0, 1


class chns_grid_desc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("h", ctypes.c_double),
                ("bc", ctypes.c_int * 3), ("precision", ctypes.c_int), ("nphases", ctypes.c_int)]


class chns_props(ctypes.Structure):
    _fields_ = [("rho_minus", ctypes.c_double), ("eta_minus", ctypes.c_double),
                ("Re", ctypes.c_double), ("We", ctypes.c_double), ("Cn", ctypes.c_double),
                ("Pe", ctypes.c_double), ("inv_Fr", ctypes.c_double),
                ("dt", ctypes.c_double), ("S", ctypes.c_double),
                ("rtol_ch", ctypes.c_double), ("rtol_mom", ctypes.c_double), ("rtol_p", ctypes.c_double),
                ("max_iter", ctypes.c_int), ("reserved", ctypes.c_int),
                ("rho3", ctypes.c_double * 3), ("eta3", ctypes.c_double * 3), ("sigma3", ctypes.c_double * 3)]


class chns_state(ctypes.Structure):
    _fields_ = [("phi", ctypes.c_void_p), ("u", ctypes.c_void_p * 3), ("p", ctypes.c_void_p),
                ("mu", ctypes.c_void_p), ("phi2", ctypes.c_void_p), ("mu2", ctypes.c_void_p)]


class chns_step_stats(ctypes.Structure):
    _fields_ = [("iters_ch", ctypes.c_int), ("iters_mom", ctypes.c_int * 3), ("iters_p", ctypes.c_int),
                ("unconverged", ctypes.c_int),
                ("res_ch", ctypes.c_double), ("res_mom", ctypes.c_double * 3), ("res_p", ctypes.c_double),
                ("mass_plus", ctypes.c_double), ("mass_minus", ctypes.c_double),
                ("energy", ctypes.c_double), ("umax", ctypes.c_double), ("divmax", ctypes.c_double),
                ("mass_phase", ctypes.c_double * 3)]


class chns_energy_monitor(ctypes.Structure):
    _fields_ = [("visc", ctypes.c_double), ("chem", ctypes.c_double), ("cubic", ctypes.c_double),
                ("inert", ctypes.c_double), ("dt_max", ctypes.c_double), ("energy_before", ctypes.c_double),
                ("energy_after", ctypes.c_double), ("holds", ctypes.c_int), ("reserved", ctypes.c_int)]


class chns_kernel_timing(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("launches", ctypes.c_int), ("ms", ctypes.c_double),
                ("bytes", ctypes.c_double)]


class chns_adj(ctypes.Structure):
    _fields_ = [("phi", ctypes.c_void_p), ("u", ctypes.c_void_p * 3)]


class chns_record(ctypes.Structure):
    _fields_ = [("phihat", ctypes.c_void_p), ("phi_new", ctypes.c_void_p), ("mu", ctypes.c_void_p),
                ("p", ctypes.c_void_p), ("ustar", ctypes.c_void_p * 3)]


class chns_batch_stats(ctypes.Structure):
    _fields_ = [("iters_ch", ctypes.c_int), ("iters_mom", ctypes.c_int * 3), ("iters_p", ctypes.c_int),
                ("flags", ctypes.c_int), ("steps", ctypes.c_int), ("pad", ctypes.c_int),
                ("total_iters", ctypes.c_longlong),
                ("res_ch", ctypes.c_double), ("res_mom", ctypes.c_double * 3), ("res_p", ctypes.c_double)]


CHNS_MAX_TUNING = 16


CHNS_BATCH_PERSISTENT, CHNS_BATCH_TILED = 0, 1


class chns_batch_tuning(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("block", ctypes.c_int), ("grid", ctypes.c_int), ("tile_cells", ctypes.c_int),
                ("ms_per_step", ctypes.c_double),
                ("budget_ch", ctypes.c_int), ("budget_mom", ctypes.c_int), ("budget_p", ctypes.c_int),
                ("ncand", ctypes.c_int), ("cand_mode", ctypes.c_int * CHNS_MAX_TUNING),
                ("cand_block", ctypes.c_int * CHNS_MAX_TUNING),
                ("cand_grid", ctypes.c_int * CHNS_MAX_TUNING), ("cand_ms", ctypes.c_double * CHNS_MAX_TUNING)]


class chns_solve_stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("rel_res", ctypes.c_double)]


EXPORTS = {
    "chns_workspace_size": (ctypes.c_int, [ctypes.POINTER(chns_grid_desc), ctypes.POINTER(ctypes.c_size_t)]),
    "chns_create_grid": (ctypes.c_int, [ctypes.POINTER(chns_grid_desc), ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "chns_set_properties": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(chns_props)]),
    "chns_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(chns_state), ctypes.c_int,
                                 ctypes.POINTER(chns_step_stats)]),
    "chns_step_monitor": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(chns_state),
                                         ctypes.POINTER(chns_energy_monitor)]),
    "chns_solve_pressure": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_double, ctypes.c_int, ctypes.POINTER(chns_solve_stats)]),
    "chns_apply_pressure_operator": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                    ctypes.c_void_p]),
    "chns_adjoint_workspace_size": (ctypes.c_int, [ctypes.POINTER(chns_grid_desc), ctypes.POINTER(ctypes.c_size_t)]),
    "chns_attach_adjoint_workspace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "chns_adjoint_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(chns_state), ctypes.POINTER(chns_adj),
                                         ctypes.POINTER(chns_adj), ctypes.POINTER(ctypes.c_double)]),
    "chns_step_record": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(chns_state), ctypes.POINTER(chns_record)]),
    "chns_adjoint_step_recorded": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(chns_state),
                                                  ctypes.POINTER(chns_record), ctypes.POINTER(chns_adj),
                                                  ctypes.POINTER(chns_adj), ctypes.POINTER(ctypes.c_double)]),
    "chns_batch_workspace_size": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(chns_grid_desc),
                                                 ctypes.POINTER(ctypes.c_size_t)]),
    "chns_create_batch": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(chns_grid_desc), ctypes.POINTER(chns_props),
                                         ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_void_p)]),
    "chns_batch_offsets": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_longlong)]),
    "chns_batch_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(chns_state), ctypes.c_int, ctypes.c_int,
                                       ctypes.POINTER(chns_batch_stats)]),
    "chns_batch_set_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
    "chns_batch_set_tiled": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "chns_batch_set_budget": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "chns_batch_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(chns_state), ctypes.c_int,
                                           ctypes.POINTER(chns_batch_tuning)]),
    "chns_destroy_batch": (ctypes.c_int, [ctypes.c_void_p]),
    "chns_set_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "chns_get_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(chns_kernel_timing), ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_int)]),
    "chns_solve_pressure_noalloc": (ctypes.c_int, [ctypes.POINTER(chns_grid_desc), ctypes.c_void_p, ctypes.c_void_p,
                                                   ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_void_p,
                                                   ctypes.POINTER(chns_solve_stats)]),
    "chns_solve_pressure_noalloc_capacity": (ctypes.c_size_t, []),
    "chns_set_option": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
    "chns_set_wall_velocity": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                              ctypes.c_void_p]),
    "chns_destroy_grid": (ctypes.c_int, [ctypes.c_void_p]),
    "chns_error_string": (ctypes.c_char_p, [ctypes.c_int]),
    "chns_last_error": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_size_t]),
}

_LIB = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libchns.so (no GPU needed to load).  Raises if it is not built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run `python -m paper_2009_06628_amd.build`")
    # torch first: its HIP runtime must be the one libchns.so binds to (a
    # library loaded before torch would bring up a second runtime instance
    # that sees no device)
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


class CHNSError(RuntimeError):
    def __init__(self, code: int, where: str):
        lib = load_library()
        buf = ctypes.create_string_buffer(1024)
        lib.chns_last_error(buf, 1024)
        super().__init__(f"{where}: {lib.chns_error_string(code).decode()} ({code}): {buf.value.decode()}")
        self.code = code


def _check(code: int, where: str, allow_noconv: bool = False) -> int:
    if code == CHNS_OK or (code == CHNS_ENOCONV and allow_noconv):
        return code
    raise CHNSError(code, where)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("paper_2009_06628_amd needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


def _ptr(t, dtype=None) -> int:
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    if t.dtype != torch.float64:
        raise ValueError("expected float64")
    return t.data_ptr()


def make_desc(n: Sequence[int], h: float, bc: Sequence[str], precision: int = CHNS_FP64,
              nphases: int = 2) -> chns_grid_desc:
    d = chns_grid_desc()
    d.dim = len(n)
    for a in range(3):
        d.n[a] = int(n[a]) if a < len(n) else 1
        d.bc[a] = (CHNS_BC_WALL if bc[a] == "wall" else CHNS_BC_PERIODIC) if a < len(n) else 0
    d.h = float(h)
    d.precision = precision
    d.nphases = int(nphases)
    return d


def workspace_size(n: Sequence[int], h: float, bc: Sequence[str], precision: int = CHNS_FP64,
                   nphases: int = 2) -> int:
    lib = load_library()
    d = make_desc(n, h, bc, precision, nphases)
    out = ctypes.c_size_t(0)
    _check(lib.chns_workspace_size(ctypes.byref(d), ctypes.byref(out)), "chns_workspace_size")
    return out.value


class Grid:
    """Handle of one uniform grid (create_grid); owns its workspace tensor."""

    def __init__(self, n: Sequence[int], h: float, bc: Sequence[str], precision: int = CHNS_FP64,
                 device: str = "cuda", stream=None, nphases: int = 2):
        torch = _torch()
        lib = load_library()
        self.n = tuple(int(x) for x in n)
        self.dim = len(self.n)
        self.shape = tuple(reversed(self.n))
        self.h = float(h)
        self.bc = tuple(bc)
        self.device = torch.device(device)
        self.nphases = int(nphases)
        self._desc = make_desc(self.n, h, bc, precision, self.nphases)
        nbytes = workspace_size(self.n, h, bc, precision, self.nphases)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        handle = ctypes.c_void_p()
        _check(lib.chns_create_grid(ctypes.byref(self._desc), ctypes.c_void_p(aligned), ctypes.c_size_t(nbytes),
                                    ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(handle)),
               "chns_create_grid")
        self._h = handle
        self._lib = lib

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.chns_destroy_grid(h)
            self._h = None

    # -- set_properties ------------------------------------------------------
    def set_properties(self, props) -> None:
        _check(self._lib.chns_set_properties(self._h, ctypes.byref(_props_struct(props))), "chns_set_properties")

    # -- state ---------------------------------------------------------------
    def new_state(self, init: Optional[Dict] = None) -> Dict:
        """Allocate a device state (float64) and fill it from numpy arrays."""
        torch = _torch()
        z = lambda: torch.zeros(self.shape, dtype=torch.float64, device=self.device)
        if self.nphases == 3:
            # phases 1 and 2 (phase 3 is implied); mu~_1, mu~_2
            st = {"phi": [z(), z()], "u": [z() for _ in range(self.dim)], "p": z(), "mu": [z(), z()]}
        else:
            st = {"phi": z(), "u": [z() for _ in range(self.dim)], "p": z(), "mu": z()}
        if init is not None:
            if self.nphases == 3:
                for i in range(2):
                    st["phi"][i].copy_(torch.as_tensor(init["phi"][i]))
            else:
                st["phi"].copy_(torch.as_tensor(init["phi"]))
            for a in range(self.dim):
                st["u"][a].copy_(torch.as_tensor(init["u"][a]))
            if "p" in init:
                st["p"].copy_(torch.as_tensor(init["p"]))
        return st

    def _cstate(self, st: Dict) -> chns_state:
        cs = chns_state()
        if self.nphases == 3:
            cs.phi, cs.phi2 = _ptr(st["phi"][0]), _ptr(st["phi"][1])
            cs.mu, cs.mu2 = _ptr(st["mu"][0]), _ptr(st["mu"][1])
        else:
            cs.phi = _ptr(st["phi"])
            cs.mu = _ptr(st["mu"])
        for a in range(3):
            cs.u[a] = _ptr(st["u"][a]) if a < self.dim else None
        cs.p = _ptr(st["p"])
        return cs

    # -- step ----------------------------------------------------------------
    def step(self, st: Dict, nsteps: int = 1, stats: bool = True, allow_noconv: bool = False) -> Optional[Dict]:
        cs = self._cstate(st)
        out = chns_step_stats()
        rc = self._lib.chns_step(self._h, ctypes.byref(cs), int(nsteps), ctypes.byref(out) if stats else None)
        _check(rc, "chns_step", allow_noconv)
        if not stats:
            return None
        return {
            "iters_ch": out.iters_ch, "iters_mom": list(out.iters_mom)[: self.dim], "iters_p": out.iters_p,
            "unconverged": out.unconverged, "res_ch": out.res_ch, "res_mom": list(out.res_mom)[: self.dim],
            "res_p": out.res_p, "mass_plus": out.mass_plus, "mass_minus": out.mass_minus,
            "energy": out.energy, "umax": out.umax, "divmax": out.divmax, "rc": rc,
            "mass_phase": list(out.mass_phase)[: self.nphases],
        }

    # -- step_monitor ------------------------------------------------------------
    def step_monitor(self, st: Dict, allow_noconv: bool = False) -> Dict:
        """One step with the energy-law monitor (chns_step_monitor)."""
        cs = self._cstate(st)
        out = chns_energy_monitor()
        rc = self._lib.chns_step_monitor(self._h, ctypes.byref(cs), ctypes.byref(out))
        _check(rc, "chns_step_monitor", allow_noconv)
        return {"visc": out.visc, "chem": out.chem, "cubic": out.cubic, "inert": out.inert, "dt_max": out.dt_max,
                "holds": bool(out.holds), "energy_before": out.energy_before, "energy_after": out.energy_after,
                "rc": rc}

    # -- solve_pressure --------------------------------------------------------
    def solve_pressure(self, rho, rhs, p, rtol: float = 1e-12, max_iter: int = 200) -> Dict:
        out = chns_solve_stats()
        rc = self._lib.chns_solve_pressure(self._h, ctypes.c_void_p(_ptr(rho)), ctypes.c_void_p(_ptr(rhs)),
                                           ctypes.c_void_p(_ptr(p)), float(rtol), int(max_iter), ctypes.byref(out))
        _check(rc, "chns_solve_pressure", allow_noconv=True)
        return {"iters": out.iters, "rel_res": out.rel_res, "rc": rc}

    # -- adjoint_step ------------------------------------------------------------
    def attach_adjoint(self) -> None:
        """Allocate and attach the adjoint workspace (once per handle)."""
        if getattr(self, "adj_workspace", None) is not None:
            return
        torch = _torch()
        out = ctypes.c_size_t(0)
        _check(self._lib.chns_adjoint_workspace_size(ctypes.byref(self._desc), ctypes.byref(out)),
               "chns_adjoint_workspace_size")
        nbytes = out.value
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        aligned = (ws.data_ptr() + 255) & ~255
        _check(self._lib.chns_attach_adjoint_workspace(self._h, ctypes.c_void_p(aligned), ctypes.c_size_t(nbytes)),
               "chns_attach_adjoint_workspace")
        self.adj_workspace = ws

    def _cadj(self, lam: Dict) -> chns_adj:
        ca = chns_adj()
        ca.phi = _ptr(lam["phi"])
        for a in range(3):
            ca.u[a] = _ptr(lam["u"][a]) if a < self.dim else None
        return ca

    def adjoint_step(self, fwd: Dict, lam_in: Dict, lam_out: Dict, grad=None, allow_noconv: bool = False) -> int:
        """One reverse step (chns_adjoint_step).  fwd: state dict at the start of
        the forward step (phi, u, p; mu unused); lam_in / lam_out: dicts with
        phi and u (may be the same dict).  grad: optional ctypes double[2]
        accumulating dL/dsigma, dL/dM."""
        if getattr(self, "adj_workspace", None) is None:
            self.attach_adjoint()
        cs = chns_state()
        cs.phi = _ptr(fwd["phi"])
        for a in range(3):
            cs.u[a] = _ptr(fwd["u"][a]) if a < self.dim else None
        cs.p = _ptr(fwd["p"])
        cs.mu = None
        li, lo = self._cadj(lam_in), self._cadj(lam_out)
        rc = self._lib.chns_adjoint_step(self._h, ctypes.byref(cs), ctypes.byref(li), ctypes.byref(lo), grad)
        return _check(rc, "chns_adjoint_step", allow_noconv)

    def new_record(self) -> Dict:
        """Device buffers for the forward fields of one step (chns_record)."""
        torch = _torch()
        z = lambda: torch.empty(self.shape, dtype=torch.float64, device=self.device)
        return {"phihat": z(), "phi_new": z(), "mu": z(), "p": z(), "ustar": [z() for _ in range(self.dim)]}

    def _crec(self, rec: Dict) -> chns_record:
        cr = chns_record()
        cr.phihat, cr.phi_new = _ptr(rec["phihat"]), _ptr(rec["phi_new"])
        cr.mu, cr.p = _ptr(rec["mu"]), _ptr(rec["p"])
        for a in range(3):
            cr.ustar[a] = _ptr(rec["ustar"][a]) if a < self.dim else None
        return cr

    def step_record(self, st: Dict, rec: Dict, allow_noconv: bool = False) -> int:
        """One step (chns_step_record) that also stores its forward fields in
        rec (from new_record)."""
        cs = self._cstate(st)
        rc = self._lib.chns_step_record(self._h, ctypes.byref(cs), ctypes.byref(self._crec(rec)))
        return _check(rc, "chns_step_record", allow_noconv)

    def adjoint_step_recorded(self, fwd: Dict, rec: Dict, lam_in: Dict, lam_out: Dict, grad=None,
                              allow_noconv: bool = False) -> int:
        """One reverse step from the recorded forward fields of the step that
        started at fwd (chns_adjoint_step_recorded)."""
        if getattr(self, "adj_workspace", None) is None:
            self.attach_adjoint()
        cs = chns_state()
        cs.phi = _ptr(fwd["phi"])
        for a in range(3):
            cs.u[a] = _ptr(fwd["u"][a]) if a < self.dim else None
        cs.p = None
        cs.mu = None
        li, lo = self._cadj(lam_in), self._cadj(lam_out)
        rc = self._lib.chns_adjoint_step_recorded(self._h, ctypes.byref(cs), ctypes.byref(self._crec(rec)),
                                                  ctypes.byref(li), ctypes.byref(lo), grad)
        return _check(rc, "chns_adjoint_step_recorded", allow_noconv)

    # -- moving walls ------------------------------------------------------------
    def set_wall_velocity(self, axis: int, side: int, component: int, values) -> None:
        """chns_set_wall_velocity: values is a face tensor of `component`
        (kept referenced by the grid) or None to stop that wall."""
        if not hasattr(self, "_walls"):
            self._walls = {}
        key = (axis, side, component)
        if values is None:
            self._walls.pop(key, None)
            ptr = None
        else:
            self._walls[key] = values
            ptr = ctypes.c_void_p(_ptr(values))
        _check(self._lib.chns_set_wall_velocity(self._h, int(axis), int(side), int(component), ptr),
               "chns_set_wall_velocity")

    # -- options ---------------------------------------------------------------
    def set_option(self, option: int, value: int) -> None:
        """chns_set_option: CHNS_OPT_CH_SOLVER (CHNS_CH_DIRECT / CHNS_CH_PCG /
        CHNS_CH_DIRECT_DENSE),
        CHNS_OPT_SERIAL_COMPONENTS (0 / 1), CHNS_OPT_TIME_SCHEME
        (CHNS_SCHEME_SPLIT / CHNS_SCHEME_CN), CHNS_OPT_PICARD_ITERATIONS (>= 1),
        CHNS_OPT_MARCH_SWEEP_CELLS (>= 1), CHNS_OPT_TILE_CYCLE_CELLS (>= 0),
        CHNS_OPT_TIME_GUESS (0 / 1)."""
        _check(self._lib.chns_set_option(self._h, int(option), int(value)), "chns_set_option")

    # -- per-kernel timing ------------------------------------------------------
    def set_timing(self, enable: bool) -> None:
        _check(self._lib.chns_set_timing(self._h, 1 if enable else 0), "chns_set_timing")

    def get_timing(self) -> List[Dict]:
        arr = (chns_kernel_timing * 64)()
        cnt = ctypes.c_int(0)
        _check(self._lib.chns_get_timing(self._h, arr, 64, ctypes.byref(cnt)), "chns_get_timing")
        return [{"name": arr[i].name.decode(), "launches": arr[i].launches, "ms": arr[i].ms,
                 "bytes": arr[i].bytes} for i in range(cnt.value)]

    def apply_pressure_operator(self, rho, x, y) -> None:
        _check(self._lib.chns_apply_pressure_operator(self._h, ctypes.c_void_p(_ptr(rho)), ctypes.c_void_p(_ptr(x)),
                                                      ctypes.c_void_p(_ptr(y))), "chns_apply_pressure_operator")


def _props_struct(props) -> chns_props:
    p = chns_props()
    for name, ctype in chns_props._fields_:
        if name == "reserved":
            continue
        if name in ("rho3", "eta3", "sigma3"):
            setattr(p, name, ctype(*[float(x) for x in getattr(props, name, (1.0, 1.0, 1.0))]))
        else:
            setattr(p, name, getattr(props, name))
    return p


class Batch:
    """Batched ensemble (chns_create_batch / chns_batch_step): problems of
    uneven size packed back to back, advanced by one persistent kernel per
    step.  problems: objects with n, h, bc, props (e.g. workloads.Problem)."""

    def __init__(self, problems, precision: int = CHNS_FP64, device: str = "cuda", stream=None):
        torch = _torch()
        lib = load_library()
        self._lib = lib
        self.count = len(problems)
        self.dim = len(problems[0].n)
        self.device = torch.device(device)
        self.shapes = [tuple(reversed(tuple(int(x) for x in p.n))) for p in problems]
        descs = (chns_grid_desc * self.count)()
        props = (chns_props * self.count)()
        for i, p in enumerate(problems):
            descs[i] = make_desc(p.n, p.h, p.bc, precision)
            props[i] = _props_struct(p.props)
        self._descs, self._props = descs, props
        nbytes = ctypes.c_size_t(0)
        _check(lib.chns_batch_workspace_size(self.count, descs, ctypes.byref(nbytes)), "chns_batch_workspace_size")
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        aligned = (self.workspace.data_ptr() + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        handle = ctypes.c_void_p()
        _check(lib.chns_create_batch(self.count, descs, props, ctypes.c_void_p(aligned), nbytes,
                                     ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(handle)),
               "chns_create_batch")
        self._h = handle
        offs = (ctypes.c_longlong * (self.count + 1))()
        _check(lib.chns_batch_offsets(handle, offs), "chns_batch_offsets")
        self.offsets = [int(offs[i]) for i in range(self.count + 1)]
        self.total_cells = self.offsets[-1]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.chns_destroy_batch(h)
            self._h = None

    def new_state(self, inits=None) -> Dict:
        """Packed device state; inits: list of per-problem dicts (numpy)."""
        torch = _torch()
        z = lambda: torch.zeros(self.total_cells, dtype=torch.float64, device=self.device)
        st = {"phi": z(), "u": [z() for _ in range(self.dim)], "p": z(), "mu": z()}
        if inits is not None:
            import numpy as np
            host = {"phi": np.zeros(self.total_cells), "u": [np.zeros(self.total_cells) for _ in range(self.dim)],
                    "p": np.zeros(self.total_cells)}
            for i, ini in enumerate(inits):
                a, b = self.offsets[i], self.offsets[i + 1]
                host["phi"][a:b] = np.asarray(ini["phi"]).ravel()
                for d in range(self.dim):
                    host["u"][d][a:b] = np.asarray(ini["u"][d]).ravel()
                if "p" in ini:
                    host["p"][a:b] = np.asarray(ini["p"]).ravel()
            st["phi"].copy_(torch.as_tensor(host["phi"]))
            for d in range(self.dim):
                st["u"][d].copy_(torch.as_tensor(host["u"][d]))
            st["p"].copy_(torch.as_tensor(host["p"]))
        return st

    def view(self, st: Dict, i: int) -> Dict:
        """Views of problem i's arrays in a packed state (cell / face shape)."""
        a, b = self.offsets[i], self.offsets[i + 1]
        sh = self.shapes[i]
        return {"phi": st["phi"][a:b].view(sh), "u": [x[a:b].view(sh) for x in st["u"]],
                "p": st["p"][a:b].view(sh), "mu": st["mu"][a:b].view(sh)}

    def _cstate(self, st: Dict) -> chns_state:
        cs = chns_state()
        cs.phi = _ptr(st["phi"])
        for a in range(3):
            cs.u[a] = _ptr(st["u"][a]) if a < self.dim else None
        cs.p = _ptr(st["p"])
        cs.mu = _ptr(st["mu"])
        return cs

    def step(self, st: Dict, nsteps: int = 1, use_graph: bool = False, stats: bool = True,
             allow_noconv: bool = False):
        cs = self._cstate(st)
        arr = (chns_batch_stats * self.count)() if stats else None
        rc = self._lib.chns_batch_step(self._h, ctypes.byref(cs), int(nsteps), 1 if use_graph else 0, arr)
        _check(rc, "chns_batch_step", allow_noconv)
        if not stats:
            return None
        return [{"iters_ch": s.iters_ch, "iters_mom": list(s.iters_mom)[: self.dim], "iters_p": s.iters_p,
                 "flags": s.flags, "steps": s.steps, "total_iters": s.total_iters, "res_ch": s.res_ch,
                 "res_mom": list(s.res_mom)[: self.dim], "res_p": s.res_p} for s in arr]

    def set_launch(self, block: int, grid: int) -> None:
        """Persistent form: block threads per workgroup, grid workgroups."""
        _check(self._lib.chns_batch_set_launch(self._h, int(block), int(grid)), "chns_batch_set_launch")

    def set_tiled(self, tile_cells: int = 1024) -> None:
        """Tiled form: one launch per sweep over all problems, tile_cells per tile."""
        _check(self._lib.chns_batch_set_tiled(self._h, int(tile_cells)), "chns_batch_set_tiled")

    def set_budget(self, ch: int, mom: int, p: int) -> None:
        _check(self._lib.chns_batch_set_budget(self._h, int(ch), int(mom), int(p)), "chns_batch_set_budget")

    def autotune(self, st: Dict, steps_per_trial: int = 1) -> Dict:
        cs = self._cstate(st)
        r = chns_batch_tuning()
        _check(self._lib.chns_batch_autotune(self._h, ctypes.byref(cs), int(steps_per_trial), ctypes.byref(r)),
               "chns_batch_autotune")
        name = {CHNS_BATCH_PERSISTENT: "persistent", CHNS_BATCH_TILED: "tiled"}
        return {"mode": name[r.mode], "block": r.block, "grid": r.grid, "tile_cells": r.tile_cells,
                "ms_per_step": r.ms_per_step, "budgets": (r.budget_ch, r.budget_mom, r.budget_p),
                "candidates": [(name[r.cand_mode[i]], r.cand_block[i], r.cand_grid[i], r.cand_ms[i])
                               for i in range(r.ncand)]}


def solve_pressure_noalloc(n: Sequence[int], h: float, bc: Sequence[str], rho, rhs, p, rtol: float = 1e-12,
                           max_iter: int = 200, precision: int = CHNS_FP64, stream=None) -> Dict:
    """Stand-alone pressure solve that allocates nothing
    (chns_solve_pressure_noalloc): the solver storage is the library's
    fixed device array, so calls on one GPU must not overlap."""
    torch = _torch()
    lib = load_library()
    d = make_desc(n, h, bc, precision)
    s = stream if stream is not None else torch.cuda.current_stream(rho.device)
    out = chns_solve_stats()
    rc = lib.chns_solve_pressure_noalloc(ctypes.byref(d), ctypes.c_void_p(_ptr(rho)), ctypes.c_void_p(_ptr(rhs)),
                                         ctypes.c_void_p(_ptr(p)), float(rtol), int(max_iter),
                                         ctypes.c_void_p(s.cuda_stream), ctypes.byref(out))
    _check(rc, "chns_solve_pressure_noalloc", allow_noconv=True)
    return {"iters": out.iters, "rel_res": out.rel_res, "rc": rc}


def create_batch(problems, precision=CHNS_FP64, device="cuda", stream=None) -> Batch:
    return Batch(problems, precision, device, stream)


def create_grid(n, h, bc, precision=CHNS_FP64, device="cuda", stream=None, nphases: int = 2) -> Grid:
    return Grid(n, h, bc, precision, device, stream, nphases)


def grid_for_problem(problem, precision=CHNS_FP64, device="cuda") -> Grid:
    """Grid + properties (and moving-wall data) for a workloads.Problem."""
    g = Grid(problem.n, problem.h, problem.bc, precision, device, nphases=getattr(problem.props, "nphases", 2))
    walls = getattr(problem, "wall_velocity", None)
    if walls:
        torch = _torch()
        for (b, side, a), U in walls.items():
            g.set_wall_velocity(b, side, a, torch.tensor(U, dtype=torch.float64, device=g.device).contiguous())
    g.set_properties(problem.props)
    return g
