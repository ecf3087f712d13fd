"""ctypes binding of libtcplb.so (the C interface declared in include/tcplb.h).

Argument marshalling only: every step of the sweep runs in the library's HIP
kernels.  PyTorch, when present, supplies device memory (through the
allocator callbacks) and the HIP stream.  There is no CPU fallback: if the
library has not been built, constructing a Domain raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtcplb.so")

PHI, UX, UY, UZ, T, P, PSTAR, RHO = range(8)
FIELDS = {"phi": PHI, "ux": UX, "uy": UY, "uz": UZ, "T": T, "p": P, "pstar": PSTAR, "rho": RHO}
PDFS = {"h": 0, "g": 1, "f": 2}
THERMAL = {"lb": 0, "rk2": 1, "rk4": 2}
PRECISION = {"fp64": 0, "fp32": 1, "fp16": 2}
KERNELS = ("phase", "hydro", "thermal", "rk", "step", "adjoint", "coupled_adjoint")

# names of every entry point the header declares
EXPORTS = (
    "tcp_params_default", "tcp_create", "tcp_destroy", "tcp_set_field", "tcp_set_field_f32", "tcp_set_droplets",
    "tcp_set_heat_sources", "tcp_set_wall_temperature", "tcp_initialize", "tcp_step", "tcp_step_taped", "tcp_tape_adjoint",
    "tcp_warm_temperature", "tcp_thermal_adjoint", "tcp_get_field", "tcp_get_field_f32",
    "tcp_get_field_noalloc",
    "tcp_get_pdfs", "tcp_reduce", "tcp_state_bytes", "tcp_save_state", "tcp_load_state", "tcp_synchronize",
    "tcp_set_profiling", "tcp_set_fusion", "tcp_set_graphs", "tcp_kernel_times", "tcp_algorithmic_bytes", "tcp_bandwidth_probe", "tcp_pdf_copy_probe",
    "tcp_error_string",
    "tcp_last_error",
)


class Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("walls_y", C.c_int32),
        ("q_pf", C.c_int32), ("q_thermal", C.c_int32), ("thermal", C.c_int32), ("precision", C.c_int32),
        ("rho_h", C.c_double), ("rho_l", C.c_double), ("nu_h", C.c_double), ("nu_l", C.c_double),
        ("mobility", C.c_double), ("xi", C.c_double), ("sigma_ref", C.c_double), ("sigma_t", C.c_double),
        ("t_ref", C.c_double), ("kappa_h", C.c_double), ("kappa_l", C.c_double),
        ("g", C.c_double * 3), ("omega_bulk", C.c_double), ("normal_eps", C.c_double),
        ("u_wall_bot", C.c_double * 3), ("u_wall_top", C.c_double * 3),
        ("t_wall_bot", C.c_double), ("t_wall_top", C.c_double), ("t_shift", C.c_double),
        ("contact_angle_bot", C.c_double), ("contact_angle_top", C.c_double),
    ]


class HeatSource(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("Q", "x", "y", "z", "w", "d_cut")]


class Droplet(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("x", "y", "z", "r")]


class Allocator(C.Structure):
    _fields_ = [("alloc", C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)),
                ("free", C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)),
                ("ctx", C.c_void_p)]


class TcpError(RuntimeError):
    pass


_lib = None


def load() -> C.CDLL:
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with python paper_2401_03041_amd/csrc/build.py "
                          "(there is no CPU fallback)")
    # One process must hold one HIP runtime.  PyTorch ships its own libamdhip64
    # with the same soname as the system one; loading torch first makes the
    # library bind to that copy instead of starting a second runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    vp, dp, i64 = C.c_void_p, C.POINTER(C.c_double), C.c_int64
    sig = {
        "tcp_params_default": [C.POINTER(Params)],
        "tcp_create": [C.POINTER(Params), C.POINTER(Allocator), vp, C.POINTER(vp)],
        "tcp_destroy": [vp],
        "tcp_set_field": [vp, C.c_int, dp, vp],
        "tcp_set_field_f32": [vp, C.c_int, vp],
        "tcp_set_droplets": [vp, C.POINTER(Droplet), C.c_int],
        "tcp_set_heat_sources": [vp, C.POINTER(HeatSource), C.c_int],
        "tcp_set_wall_temperature": [vp, C.c_int, dp],
        "tcp_initialize": [vp],
        "tcp_step": [vp, i64],
        "tcp_step_taped": [vp, i64, i64],
        "tcp_tape_adjoint": [vp, dp, dp, dp, dp, dp],
        "tcp_warm_temperature": [vp, i64, C.c_double, i64, C.POINTER(i64), dp],
        "tcp_thermal_adjoint": [vp, i64, dp, dp, dp, dp],
        "tcp_get_field": [vp, C.c_int, dp, vp],
        "tcp_get_field_f32": [vp, C.c_int, vp],
        "tcp_get_field_noalloc": [vp, C.c_int, dp],
        "tcp_get_pdfs": [vp, C.c_int, dp],
        "tcp_reduce": [vp, dp, dp],
        "tcp_state_bytes": [vp, C.POINTER(C.c_size_t)],
        "tcp_save_state": [vp, vp],
        "tcp_load_state": [vp, vp],
        "tcp_synchronize": [vp],
        "tcp_set_profiling": [vp, C.c_int],
        "tcp_set_graphs": [vp, C.c_int],
        "tcp_set_fusion": [vp, C.c_int],
        "tcp_kernel_times": [vp, dp, C.POINTER(i64)],
        "tcp_algorithmic_bytes": [vp, dp],
        "tcp_bandwidth_probe": [C.c_size_t, C.c_int, dp],
        "tcp_pdf_copy_probe": [C.c_int64, C.c_int, dp],
        "tcp_error_string": [C.c_int],
        "tcp_last_error": [vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.tcp_error_string.restype = C.c_char_p
    lib.tcp_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def params_from_config(cfg: dict) -> Params:
    """Fill tcp_params from a workload description (see workloads.py)."""
    lib = load()
    p = Params()
    lib.tcp_params_default(C.byref(p))
    p.nx, p.ny, p.nz = (int(v) for v in cfg["shape"])
    p.walls_y = 0 if cfg.get("periodic_y", True) else 1
    p.q_pf = int(cfg.get("q_pf", 15))
    p.q_thermal = int(cfg.get("q_thermal", 7))
    p.thermal = THERMAL[cfg.get("thermal", "lb")]
    p.precision = PRECISION[cfg.get("precision", "fp64")]
    for k in ("rho_h", "rho_l", "nu_h", "nu_l", "mobility", "xi", "sigma_ref", "sigma_t", "t_ref",
              "kappa_h", "kappa_l"):
        setattr(p, k, float(cfg[k]))
    for a in range(3):
        p.g[a] = float(cfg.get("g", (0, 0, 0))[a])
        p.u_wall_bot[a] = float(cfg.get("u_wall_bot", (0, 0, 0))[a])
        p.u_wall_top[a] = float(cfg.get("u_wall_top", (0, 0, 0))[a])
    p.omega_bulk = float(cfg.get("omega_bulk", 1.0))
    p.normal_eps = float(cfg.get("normal_eps", 1e-6))
    p.t_wall_bot = float(cfg.get("t_wall_bot", 0.0))
    p.t_wall_top = float(cfg.get("t_wall_top", 0.0))
    p.t_shift = float(cfg.get("t_shift", 0.0))
    p.contact_angle_bot = float(cfg.get("contact_angle_bot", 90.0))
    p.contact_angle_top = float(cfg.get("contact_angle_top", 90.0))
    return p


class _TorchAllocator:
    """Backs library allocations with torch CUDA (HIP) tensors."""

    def __init__(self, device):
        import torch
        self.torch = torch
        self.device = device
        self.live = {}
        self.c_alloc = Allocator._fields_[0][1](self._alloc)
        self.c_free = Allocator._fields_[1][1](self._free)
        self.struct = Allocator(self.c_alloc, self.c_free, None)

    def _alloc(self, nbytes, ctx):
        try:
            t = self.torch.empty(int(nbytes), dtype=self.torch.uint8, device=self.device)
        except RuntimeError:
            return None
        ptr = t.data_ptr()
        self.live[ptr] = t
        return ptr

    def _free(self, ptr, ctx):
        self.live.pop(ptr, None)


class Domain:
    """One simulation domain living on the GPU (see include/tcplb.h)."""

    def __init__(self, cfg: dict, device: int = 0, use_torch: bool = True):
        self._lib = load()
        self.cfg = dict(cfg)
        self.nx, self.ny, self.nz = (int(v) for v in cfg["shape"])
        self._p = params_from_config(cfg)
        self.n_sources = 0
        self.device = int(device)
        self._alloc = None
        stream = None
        if use_torch:
            import torch
            dev = torch.device("cuda", device)
            self._alloc = _TorchAllocator(dev)
            stream = torch.cuda.current_stream(dev).cuda_stream
        h = C.c_void_p()
        rc = self._lib.tcp_create(C.byref(self._p), C.byref(self._alloc.struct) if self._alloc else None,
                                  C.c_void_p(stream) if stream else None, C.byref(h))
        if rc != 0:
            raise TcpError(f"tcp_create: {self._lib.tcp_error_string(rc).decode()}: "
                           f"{self._lib.tcp_last_error(None).decode()}")
        self._h = h

    # -- helpers --------------------------------------------------------------------
    def _check(self, rc: int, what: str):
        if rc != 0:
            raise TcpError(f"{what}: {self._lib.tcp_error_string(rc).decode()}: "
                           f"{self._lib.tcp_last_error(self._h).decode()}")

    @property
    def shape3(self):
        return (self.nz, self.ny, self.nx)

    @property
    def ncell(self) -> int:
        return self.nx * self.ny * self.nz

    def close(self):
        if getattr(self, "_h", None):
            self._lib.tcp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- problem set-up --------------------------------------------------------------
    def _device_array(self, t, what: str):
        """Check that a CUDA tensor holds exactly one field (nx*ny*nz values,
        contiguous) before its address crosses the boundary."""
        import torch
        if t.dtype not in (torch.float32, torch.float64):
            raise TypeError(f"{what}: device arrays are float32 or float64, not {t.dtype}")
        if t.numel() != self.nx * self.ny * self.nz or not t.is_contiguous():
            raise ValueError(f"{what}: a contiguous device array of {self.nx * self.ny * self.nz} values is required")
        if t.device.index is not None and t.device.index != self.device:
            raise ValueError(f"{what}: the array is on cuda:{t.device.index}, the domain on cuda:{self.device}")
        return t

    def set_field(self, name: str, value) -> None:
        """Set phi, ux, uy, uz or T from a host array (FP64), or from a CUDA
        tensor: float32 through the FP32 entry point, anything else as FP64."""
        which = FIELDS[name]
        if hasattr(value, "is_cuda") and value.is_cuda:
            import torch
            t = value.contiguous()
            if t.dtype != torch.float32:
                t = t.to(dtype=torch.float64)
            self._device_array(t, "set_field")
            if t.dtype == torch.float32:
                self._check(self._lib.tcp_set_field_f32(self._h, which, C.c_void_p(t.data_ptr())), "set_field")
            else:
                self._check(self._lib.tcp_set_field(self._h, which, None, C.c_void_p(t.data_ptr())), "set_field")
            self._lib.tcp_synchronize(self._h)
            return
        a = np.ascontiguousarray(np.broadcast_to(np.asarray(value, dtype=np.float64), self.shape3))
        self._check(self._lib.tcp_set_field(self._h, which, _dptr(a), None), "set_field")

    def set_droplets(self, drops) -> None:
        n = len(drops)
        arr = (Droplet * max(n, 1))(*[Droplet(*map(float, d)) for d in drops])
        self._check(self._lib.tcp_set_droplets(self._h, arr, n), "set_droplets")

    def set_heat_sources(self, sources) -> None:
        n = len(sources)
        arr = (HeatSource * max(n, 1))(*[HeatSource(*map(float, s)) for s in sources])
        self._check(self._lib.tcp_set_heat_sources(self._h, arr, n), "set_heat_sources")
        self.n_sources = n

    def set_wall_temperature(self, wall: int, tw) -> None:
        a = np.ascontiguousarray(np.broadcast_to(np.asarray(tw, dtype=np.float64), (self.nz, self.nx)))
        self._check(self._lib.tcp_set_wall_temperature(self._h, int(wall), _dptr(a)), "set_wall_temperature")

    def initialize(self) -> None:
        self._check(self._lib.tcp_initialize(self._h), "initialize")

    def step(self, n: int = 1) -> None:
        self._check(self._lib.tcp_step(self._h, int(n)), "step")

    def step_taped(self, n: int, segment: int = 0) -> None:
        """Advance n coupled steps and keep the tape tape_adjoint needs
        (checkpoints every `segment` steps; 0: ceil(sqrt(n)))."""
        self._check(self._lib.tcp_step_taped(self._h, int(n), int(segment)), "step_taped")

    def tape_adjoint(self, dL_dcentroid, dL_dphi=None):
        """Gradients of a loss of the final phase field (through its centroid,
        dL_dcentroid (3,), plus an optional per-cell dL_dphi) after the taped run,
        with respect to the taped heat sources and the wall temperatures:
        (dsrc[n_sources, 4] = dL/d(Q, x, y, z) per source, dTw_bot[nz, nx], dTw_top[nz, nx])."""
        gc = np.ascontiguousarray(np.asarray(dL_dcentroid, dtype=np.float64).reshape(3))
        m = None
        if dL_dphi is not None:
            m = np.ascontiguousarray(np.broadcast_to(np.asarray(dL_dphi, dtype=np.float64), self.shape3))
        dq = np.zeros(64)
        bot = np.zeros((self.nz, self.nx))
        top = np.zeros((self.nz, self.nx))
        self._check(self._lib.tcp_tape_adjoint(self._h, _dptr(gc), _dptr(m) if m is not None else None, _dptr(dq),
                                               _dptr(bot), _dptr(top)), "tape_adjoint")
        return dq[:4 * self.n_sources].reshape(self.n_sources, 4), bot, top

    def warm_temperature(self, max_steps: int, tol: float = 0.0, check_every: int = 100):
        """Thermal updates alone (phi, u held) until the per-update change of T is at
        most tol or max_steps have run; returns (steps run, last change)."""
        n = C.c_int64()
        ch = np.zeros(1)
        self._check(self._lib.tcp_warm_temperature(self._h, int(max_steps), float(tol), int(check_every),
                                                   C.byref(n), _dptr(ch)), "warm_temperature")
        return int(n.value), float(ch[0])

    def thermal_adjoint(self, nsteps: int, dL_dT):
        """Gradients of L = sum(dL_dT * T), T after nsteps warm-up updates (phi, u
        held), with respect to the heat sources and the wall temperatures:
        (dsrc[n_sources, 4] = dL/d(Q, x, y, z) per source, dTw_bot[nz, nx], dTw_top[nz, nx])."""
        m = np.ascontiguousarray(np.broadcast_to(np.asarray(dL_dT, dtype=np.float64), self.shape3))
        dq = np.zeros(64)
        bot = np.zeros((self.nz, self.nx))
        top = np.zeros((self.nz, self.nx))
        self._check(self._lib.tcp_thermal_adjoint(self._h, int(nsteps), _dptr(m), _dptr(dq), _dptr(bot), _dptr(top)),
                    "thermal_adjoint")
        return dq[:4 * self.n_sources].reshape(self.n_sources, 4), bot, top

    # -- read-back ---------------------------------------------------------------------
    def get_field(self, name: str, out=None):
        """Field, shape (nz, ny, nx): FP64 numpy array, or into `out`, a CUDA
        float64 or float32 tensor of nx*ny*nz values (asynchronous)."""
        which = FIELDS[name]
        if out is not None:
            import torch
            if not out.is_cuda:
                raise ValueError("get_field: out must be a CUDA tensor")
            self._device_array(out, "get_field")
            if out.dtype == torch.float32:
                self._check(self._lib.tcp_get_field_f32(self._h, which, C.c_void_p(out.data_ptr())), "get_field")
            else:
                self._check(self._lib.tcp_get_field(self._h, which, None, C.c_void_p(out.data_ptr())), "get_field")
            return out
        a = np.empty(self.shape3, dtype=np.float64)
        self._check(self._lib.tcp_get_field(self._h, which, _dptr(a), None), "get_field")
        return a

    def get_field_noalloc(self, name: str):
        """FP64 field, shape (nz, ny, nx), read back through the library's fixed
        staging array (no device allocation; at most 4194304 cells)."""
        a = np.empty(self.shape3, dtype=np.float64)
        self._check(self._lib.tcp_get_field_noalloc(self._h, FIELDS[name], _dptr(a)), "get_field_noalloc")
        return a

    def fields(self, names=("phi", "ux", "uy", "uz", "p", "T")) -> dict:
        return {k: self.get_field(k) for k in names}

    def get_pdfs(self, which: str) -> np.ndarray:
        q = {"h": self._p.q_pf, "g": 27, "f": self._p.q_thermal}[which]
        a = np.empty((q,) + self.shape3, dtype=np.float64)
        self._check(self._lib.tcp_get_pdfs(self._h, PDFS[which], _dptr(a)), "get_pdfs")
        return a

    def reduce(self):
        m = np.zeros(1)
        c = np.zeros(3)
        self._check(self._lib.tcp_reduce(self._h, _dptr(m), _dptr(c)), "reduce")
        return float(m[0]), c

    def state_bytes(self) -> int:
        n = C.c_size_t()
        self._check(self._lib.tcp_state_bytes(self._h, C.byref(n)), "state_bytes")
        return int(n.value)

    def save_state(self) -> np.ndarray:
        buf = np.empty(self.state_bytes(), dtype=np.uint8)
        self._check(self._lib.tcp_save_state(self._h, buf.ctypes.data_as(C.c_void_p)), "save_state")
        return buf

    def load_state(self, buf: np.ndarray) -> None:
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        if buf.size != self.state_bytes():
            raise ValueError("state size mismatch")
        self._check(self._lib.tcp_load_state(self._h, buf.ctypes.data_as(C.c_void_p)), "load_state")

    def synchronize(self) -> None:
        self._check(self._lib.tcp_synchronize(self._h), "synchronize")

    # -- measurement --------------------------------------------------------------------
    def set_profiling(self, on: bool) -> None:
        self._check(self._lib.tcp_set_profiling(self._h, int(bool(on))), "set_profiling")

    def set_fusion(self, on: bool) -> None:
        """Thermal LB: one fused kernel per step (default) or the three kernels."""
        self._check(self._lib.tcp_set_fusion(self._h, int(bool(on))), "set_fusion")

    def set_graphs(self, mode: int) -> None:
        """Step graphs: 0 never, 1 grids up to 2^21 cells (default), 2 always."""
        self._check(self._lib.tcp_set_graphs(self._h, int(mode)), "set_graphs")

    def kernel_times(self) -> dict:
        ms = np.zeros(len(KERNELS))
        n = (C.c_int64 * len(KERNELS))()
        self._check(self._lib.tcp_kernel_times(self._h, _dptr(ms), n), "kernel_times")
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNELS)}

    def algorithmic_bytes(self) -> dict:
        b = np.zeros(len(KERNELS))
        self._check(self._lib.tcp_algorithmic_bytes(self._h, _dptr(b)), "algorithmic_bytes")
        return {k: float(b[i]) for i, k in enumerate(KERNELS)}


def bandwidth_probe(nbytes: int = 1 << 32, reps: int = 10) -> float:
    """Best device-to-device copy rate (GB/s, read + write) of a plain streaming kernel."""
    lib = load()
    out = np.zeros(1)
    rc = lib.tcp_bandwidth_probe(int(nbytes), int(reps), _dptr(out))
    if rc != 0:
        raise TcpError(f"bandwidth probe: {lib.tcp_last_error(None).decode()}")
    return float(out[0])


def pdf_copy_probe(ncells: int = 1 << 27, reps: int = 5) -> float:
    """Best rate (GB/s, read + write) of copying a 27-component FP32 field of
    ncells cells in the blocked PDF layout: the step kernel's access pattern."""
    lib = load()
    out = np.zeros(1)
    rc = lib.tcp_pdf_copy_probe(int(ncells), int(reps), _dptr(out))
    if rc != 0:
        raise TcpError(f"PDF copy probe: {lib.tcp_last_error(None).decode()}")
    return float(out[0])


def domain_from_workload(cfg: dict, device: int = 0, temperature=None, velocity=None) -> Domain:
    """Create a domain and load the workload's inputs (droplets, temperature,
    velocity, heat sources), then set the PDFs to equilibrium."""
    from . import workloads as W
    d = Domain(cfg, device=device)
    if cfg["droplets"]:
        d.set_droplets(cfg["droplets"])
    d.set_field("T", W.temperature(cfg) if temperature is None else temperature)
    u = W.velocity(cfg) if velocity is None else velocity
    for name, comp in zip(("ux", "uy", "uz"), u):
        d.set_field(name, comp)
    if cfg["heat_sources"]:
        d.set_heat_sources(cfg["heat_sources"])
    d.initialize()
    return d


def thermal_warmup(domain: Domain, nsteps: int):
    """The temperature warm-up as a differentiable function for torch.

    Returns f(sources, tw_bot, tw_top) -> T: `sources` an (n, 6) float64 tensor
    of heat sources (Q, x, y, z, w, d_cut), `tw_bot` / `tw_top` (nz, nx) wall
    temperatures.  Each call restores the domain's state as it was when this
    function was made, loads the inputs and runs nsteps warm-up updates (phi
    and u held); T comes back as an (nz, ny, nx) float64 tensor.  The backward
    pass reloads that call's own inputs (another call may have run in between)
    and runs tcp_thermal_adjoint: gradients for Q, x, y, z of every source and
    for both walls (w and d_cut get none)."""
    import torch
    snapshot = domain.save_state()

    def load_inputs(src, bot, top):
        domain.load_state(snapshot)
        domain.set_heat_sources(src.tolist())
        domain.set_wall_temperature(0, bot)
        domain.set_wall_temperature(1, top)

    class _Warmup(torch.autograd.Function):
        @staticmethod
        def forward(ctx, sources, tw_bot, tw_top):
            # the backward pass reloads these: the domain may have been given other
            # inputs by another forward call in between
            ctx.inputs = (sources.detach().cpu().numpy().copy(), tw_bot.detach().cpu().numpy().copy(),
                          tw_top.detach().cpu().numpy().copy())
            load_inputs(*ctx.inputs)
            domain.warm_temperature(nsteps, 0.0, max(int(nsteps), 1))
            return torch.from_numpy(domain.get_field("T")).to(sources.device)

        @staticmethod
        def backward(ctx, grad_T):
            load_inputs(*ctx.inputs)
            dsrc, dbot, dtop = domain.thermal_adjoint(nsteps, grad_T.detach().cpu().numpy())
            n = dsrc.shape[0]
            g = torch.zeros((n, 6), dtype=torch.float64)
            g[:, :4] = torch.from_numpy(dsrc)
            dev = grad_T.device
            return g.to(dev), torch.from_numpy(dbot).to(dev), torch.from_numpy(dtop).to(dev)

    return _Warmup.apply


def centroid_run(domain: Domain, nsteps: int, segment: int = 0):
    """A coupled run as a differentiable function for torch.

    Returns f(sources, tw_bot, tw_top) -> centroid: `sources` an (n, 6) float64
    tensor of heat sources (Q, x, y, z, w, d_cut), `tw_bot` / `tw_top` (nz, nx)
    wall temperatures.  Each call restores the domain's state as it was when
    this function was made, loads the inputs, runs nsteps taped coupled steps
    and returns the FP64 centroid of the final phase field, a (3,) tensor.  The
    backward pass runs tcp_tape_adjoint with dL/dcentroid; if another call has
    replaced the tape in between, it first reloads this call's inputs and
    tapes the run again.  Gradients for Q, x, y, z of every source and for both
    walls (w and d_cut get none)."""
    import torch
    snapshot = domain.save_state()
    counter = [0]

    def run(src, bot, top):
        domain.load_state(snapshot)
        domain.set_heat_sources(src.tolist())
        domain.set_wall_temperature(0, bot)
        domain.set_wall_temperature(1, top)
        domain.step_taped(nsteps, segment)
        counter[0] += 1
        domain._tape_owner = counter[0]
        return domain.reduce()[1]

    class _Centroid(torch.autograd.Function):
        @staticmethod
        def forward(ctx, sources, tw_bot, tw_top):
            ctx.inputs = (sources.detach().cpu().numpy().copy(), tw_bot.detach().cpu().numpy().copy(),
                          tw_top.detach().cpu().numpy().copy())
            c = run(*ctx.inputs)
            ctx.tape = domain._tape_owner
            return torch.from_numpy(c.copy()).to(sources.device)

        @staticmethod
        def backward(ctx, grad_c):
            if getattr(domain, "_tape_owner", None) != ctx.tape:
                run(*ctx.inputs)
                ctx.tape = domain._tape_owner
            dsrc, dbot, dtop = domain.tape_adjoint(grad_c.detach().cpu().numpy())
            n = dsrc.shape[0]
            g = torch.zeros((n, 6), dtype=torch.float64)
            g[:, :4] = torch.from_numpy(dsrc)
            dev = grad_c.device
            return g.to(dev), torch.from_numpy(dbot).to(dev), torch.from_numpy(dtop).to(dev)

    return _Centroid.apply
