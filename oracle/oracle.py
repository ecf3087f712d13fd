"""Python access to the FP64 CPU oracle (``tcp_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  Nothing here imports the GPU package,
and the GPU package never imports this module.

Arrays are numpy ``float64`` with shape ``(nz, ny, nx)`` (x fastest), the
same cell order ``x + nx*(y + ny*z)`` the C code uses.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tcp_oracle.c")
_LIB = os.path.join(_HERE, "libtcp_oracle.so")

FIELDS_IN = {"phi": 0, "ux": 1, "uy": 2, "uz": 3, "T": 4}
FIELDS_OUT = {"phi": 0, "ux": 1, "uy": 2, "uz": 3, "p": 4, "pstar": 5, "T": 6, "rho": 7}
PDFS = {"h": 0, "g": 1, "f": 2}
THERMAL = {"lb": 0, "rk2": 1, "rk4": 2}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
               _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("walls_y", C.c_int32), ("q_pf", C.c_int32), ("q_thermal", C.c_int32),
        ("thermal", C.c_int32), ("pad", C.c_int32),
        ("rho_h", C.c_double), ("rho_l", C.c_double), ("nu_h", C.c_double), ("nu_l", C.c_double),
        ("mobility", C.c_double), ("xi", C.c_double),
        ("sigma_ref", C.c_double), ("sigma_t", C.c_double), ("t_ref", C.c_double),
        ("kappa_h", C.c_double), ("kappa_l", C.c_double),
        ("g", C.c_double * 3), ("omega_bulk", C.c_double),
        ("u_wall_bot", C.c_double * 3), ("u_wall_top", C.c_double * 3),
        ("t_wall_bot", C.c_double), ("t_wall_top", C.c_double),
        ("normal_eps", C.c_double),
        ("contact_angle_bot", C.c_double), ("contact_angle_top", C.c_double),
    ]


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = C.CDLL(_LIB)
    dp = C.POINTER(C.c_double)
    vp = C.c_void_p
    lib.ora_create.restype = vp
    lib.ora_create.argtypes = [C.POINTER(_Params)]
    lib.ora_destroy.argtypes = [vp]
    lib.ora_set_field.argtypes = [vp, C.c_int, dp]
    lib.ora_set_droplets.argtypes = [vp, dp, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                     C.POINTER(C.c_int32)]
    lib.ora_set_heat_sources.argtypes = [vp, dp, C.c_int]
    lib.ora_set_wall_temperature.argtypes = [vp, C.c_int, dp]
    lib.ora_initialize.argtypes = [vp]
    lib.ora_step.argtypes = [vp, C.c_int64]
    lib.ora_warm_temperature.argtypes = [vp, C.c_int64, C.c_double, C.c_int64, C.POINTER(C.c_int64), dp]
    lib.ora_get_field.argtypes = [vp, C.c_int, dp]
    lib.ora_get_pdfs.argtypes = [vp, C.c_int, dp]
    lib.ora_set_pdfs.argtypes = [vp, C.c_int, dp]
    lib.ora_reduce.argtypes = [vp, dp, dp]
    lib.ora_num_threads.restype = C.c_int
    lib.ora_set_num_threads.argtypes = [C.c_int]
    lib.ora_stencil.argtypes = [C.c_int, C.POINTER(C.c_int), dp, C.POINTER(C.c_int)]
    lib.ora_moment_matrix.argtypes = [C.c_int, C.c_int, dp, dp, C.POINTER(C.c_int), C.POINTER(C.c_int)]
    lib.ora_cm_collide.argtypes = [C.c_int, C.c_int, dp, dp, dp, dp, dp, dp]
    lib.ora_equilibrium.argtypes = [C.c_int, C.c_int, C.c_double, dp, dp]
    lib.ora_iso_grad_lap.argtypes = [vp, dp, C.c_int, C.c_int, C.c_int, C.c_int, dp, dp]
    lib.ora_guo_source.argtypes = [dp, dp, dp]
    lib.ora_heat_source.restype = C.c_double
    lib.ora_heat_source.argtypes = [vp, C.c_double, C.c_double, C.c_double]
    _lib = lib
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return _load().ora_num_threads()


def set_num_threads(n: int) -> None:
    _load().ora_set_num_threads(int(n))


def make_params(cfg: dict) -> _Params:
    """Fill the oracle's own parameter struct from a configuration dict."""
    p = _Params()
    p.nx, p.ny, p.nz = (int(v) for v in cfg["shape"])
    p.walls_y = 0 if cfg.get("periodic_y", True) else 1
    p.q_pf = int(cfg.get("q_pf", 15))
    p.q_thermal = int(cfg.get("q_thermal", 7))
    p.thermal = THERMAL[cfg.get("thermal", "lb")]
    for k in ("rho_h", "rho_l", "nu_h", "nu_l", "mobility", "xi", "sigma_ref", "sigma_t", "t_ref",
              "kappa_h", "kappa_l"):
        setattr(p, k, float(cfg[k]))
    g = cfg.get("g", (0.0, 0.0, 0.0))
    for a in range(3):
        p.g[a] = float(g[a])
        p.u_wall_bot[a] = float(cfg.get("u_wall_bot", (0, 0, 0))[a])
        p.u_wall_top[a] = float(cfg.get("u_wall_top", (0, 0, 0))[a])
    p.omega_bulk = float(cfg.get("omega_bulk", 1.0))
    p.t_wall_bot = float(cfg.get("t_wall_bot", 0.0))
    p.t_wall_top = float(cfg.get("t_wall_top", 0.0))
    p.normal_eps = float(cfg.get("normal_eps", 1e-6))
    p.contact_angle_bot = float(cfg.get("contact_angle_bot", 90.0))
    p.contact_angle_top = float(cfg.get("contact_angle_top", 90.0))
    return p


class OracleDomain:
    """One oracle domain; mirrors the problem statement of the GPU library."""

    def __init__(self, cfg: dict):
        self._lib = _load()
        self.cfg = dict(cfg)
        self.nx, self.ny, self.nz = (int(v) for v in cfg["shape"])
        self._p = make_params(cfg)
        self._h = self._lib.ora_create(C.byref(self._p))
        if not self._h:
            raise ValueError("oracle rejected the parameters")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ora_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    @property
    def shape3(self):
        return (self.nz, self.ny, self.nx)

    def set_field(self, name: str, arr) -> None:
        a = _f64(np.broadcast_to(np.asarray(arr, dtype=np.float64), self.shape3))
        if self._lib.ora_set_field(self._h, FIELDS_IN[name], _dptr(a)) != 0:
            raise ValueError(name)

    def set_droplets(self, drops, gdim=None, origin=(0, 0, 0), periodic=None) -> None:
        d = _f64(np.asarray(drops, dtype=np.float64).reshape(-1, 4))
        gdim = (self.nx, self.ny, self.nz) if gdim is None else gdim
        if periodic is None:
            periodic = (1, 1 if self.cfg.get("periodic_y", True) else 0, 1)
        g = (C.c_int64 * 3)(*[int(v) for v in gdim])
        o = (C.c_int64 * 3)(*[int(v) for v in origin])
        pr = (C.c_int32 * 3)(*[int(v) for v in periodic])
        self._lib.ora_set_droplets(self._h, _dptr(d), d.shape[0], g, o, pr)

    def set_heat_sources(self, sources) -> None:
        s = _f64(np.asarray(sources, dtype=np.float64).reshape(-1, 6))
        if self._lib.ora_set_heat_sources(self._h, _dptr(s), s.shape[0]) != 0:
            raise ValueError("too many heat sources")

    def set_wall_temperature(self, wall: int, tw) -> None:
        a = _f64(np.broadcast_to(np.asarray(tw, dtype=np.float64), (self.nz, self.nx)))
        if self._lib.ora_set_wall_temperature(self._h, int(wall), _dptr(a)) != 0:
            raise ValueError("wall")

    def initialize(self) -> None:
        self._lib.ora_initialize(self._h)

    def step(self, n: int = 1) -> None:
        if self._lib.ora_step(self._h, int(n)) != 0:
            raise RuntimeError("oracle collision matrix became singular")

    def warm_temperature(self, max_steps: int, tol: float = 0.0, check_every: int = 100):
        """Thermal updates alone (Sec. 4.1 temperature initialisation); returns
        (updates run, last per-update change of T)."""
        n = C.c_int64()
        ch = np.zeros(1)
        rc = self._lib.ora_warm_temperature(self._h, int(max_steps), float(tol), int(check_every), C.byref(n),
                                            _dptr(ch))
        if rc != 0:
            raise RuntimeError(f"oracle warm-up failed ({rc})")
        return int(n.value), float(ch[0])

    def get_field(self, name: str) -> np.ndarray:
        out = np.empty(self.shape3, dtype=np.float64)
        self._lib.ora_get_field(self._h, FIELDS_OUT[name], _dptr(out))
        return out

    def fields(self, names=("phi", "ux", "uy", "uz", "p", "T")) -> dict:
        return {k: self.get_field(k) for k in names}

    def get_pdfs(self, which: str) -> np.ndarray:
        q = {"h": int(self._p.q_pf), "g": 27, "f": int(self._p.q_thermal)}[which]
        out = np.empty((q,) + self.shape3, dtype=np.float64)
        self._lib.ora_get_pdfs(self._h, PDFS[which], _dptr(out))
        return out

    def set_pdfs(self, which: str, arr) -> None:
        a = _f64(arr)
        self._lib.ora_set_pdfs(self._h, PDFS[which], _dptr(a))

    def reduce(self):
        m = np.zeros(1)
        c = np.zeros(3)
        self._lib.ora_reduce(self._h, _dptr(m), _dptr(c))
        return float(m[0]), c

    def iso_grad_lap(self, psi, x, y, z, ghost: str = "mirror"):
        a = _f64(psi)
        g = np.zeros(3)
        l = np.zeros(1)
        self._lib.ora_iso_grad_lap(self._h, _dptr(a), int(x), int(y), int(z), int(ghost != "mirror"),
                                   _dptr(g), _dptr(l))
        return g, float(l[0])

    def heat_source(self, x, y, z) -> float:
        return float(self._lib.ora_heat_source(self._h, float(x), float(y), float(z)))


# ---- building blocks for the pin tests -------------------------------------------------
def stencil(q: int):
    lib = _load()
    e = (C.c_int * (3 * q))()
    w = np.zeros(q)
    opp = (C.c_int * q)()
    if lib.ora_stencil(q, e, _dptr(w), opp) != 0:
        raise ValueError(q)
    return np.array(list(e), dtype=np.int64).reshape(q, 3), w, np.array(list(opp), dtype=np.int64)


def moment_matrix(q: int, u, kind: int = 0):
    lib = _load()
    T = np.zeros((q, q))
    order = (C.c_int * q)()
    tag = (C.c_int * q)()
    uu = _f64(u)
    if lib.ora_moment_matrix(q, kind, _dptr(uu), _dptr(T), order, tag) != 0:
        raise ValueError(q)
    return T, np.array(list(order)), np.array(list(tag))


def cm_collide(q: int, kind: int, rate, u, f, feq, S) -> np.ndarray:
    lib = _load()
    out = np.zeros(q)
    args = [_f64(a) for a in (rate, u, f, feq, S)]
    if lib.ora_cm_collide(q, kind, *[_dptr(a) for a in args], _dptr(out)) != 0:
        raise RuntimeError("singular moment matrix")
    return out


def guo_source(u, acc) -> np.ndarray:
    lib = _load()
    out = np.zeros(27)
    lib.ora_guo_source(_dptr(_f64(u)), _dptr(_f64(acc)), _dptr(out))
    return out


def equilibrium(q: int, kind: int, zeroth: float, u) -> np.ndarray:
    lib = _load()
    out = np.zeros(q)
    uu = _f64(u)
    lib.ora_equilibrium(q, kind, float(zeroth), _dptr(uu), _dptr(out))
    return out
