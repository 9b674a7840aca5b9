"""ctypes wrapper of the FP64 CPU oracle (``lbib_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.  All arrays use
the public layout [component][y][x] (fields) and [node][2] (capsule nodes).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Any, Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "lbib_oracle.c")
# LBIB_ORACLE_LIB points the wrapper at another build of this source (the
# mutation checks of the pins load deliberately broken copies this way)
LIB = os.environ.get("LBIB_ORACLE_LIB") or os.path.join(_HERE, "liblbib_oracle.so")

KINEMATIC, DYNAMIC = 0, 1
E_WALL, E_NONFINITE = 1, 2

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP over lattice columns)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC",
                               "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def build_native(out: str) -> str:
    """The same source built for the host it runs on (gcc -O3 -march=native),
    used for the CPU-baseline timing; ``LIB`` must point at it before the
    first ``lib()`` call."""
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", "-O3", "-march=native", "-std=c11", "-D_DEFAULT_SOURCE",
                           "-fopenmp", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"])
    os.replace(tmp, out)
    return out


_lib: Optional[C.CDLL] = None


def lib() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        build()
    L = C.CDLL(LIB)
    vp = C.c_void_p
    L.orc_equilibrium.argtypes = [C.c_double, C.c_double, C.c_double, _dp]
    L.orc_forcing.argtypes = [C.c_double] * 5 + [_dp]
    L.orc_mls.argtypes = [C.c_double, C.c_double, _ip, _ip, _dp, _dp, _dp]
    L.orc_internal_forces.argtypes = [C.c_int, _dp, _dp, _dp, _dp, C.c_double, C.c_double,
                                      C.c_double, _dp, _dp, _dp]
    L.orc_polygon_diag.argtypes = [C.c_int, _dp, _dp]
    L.orc_create.restype = vp
    L.orc_create.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int, C.c_double, C.c_double,
                             C.c_double, C.c_double, C.c_int, C.c_double, C.c_double, C.c_int,
                             C.c_double, C.c_double]
    L.orc_destroy.argtypes = [vp]
    L.orc_add_capsule.argtypes = [vp, C.c_int, _dp, _dp, C.c_int, C.c_double, C.c_double,
                                  C.c_double]
    L.orc_step.argtypes = [vp, C.c_int, C.c_int]
    L.orc_status.argtypes = [vp]
    L.orc_steps.argtypes = [vp]
    L.orc_steps.restype = C.c_long
    for name in ("orc_get_pops", "orc_set_pops", "orc_get_moments", "orc_get_force",
                 "orc_set_force", "orc_set_moments"):
        getattr(L, name).argtypes = [vp, _dp]
    L.orc_get_capsule.argtypes = [vp, C.c_int, _dp, _dp, _dp]
    L.orc_set_capsule.argtypes = [vp, C.c_int, _dp, _dp, _dp]
    L.orc_get_capsule_forces.argtypes = [vp, C.c_int, _dp, _dp]
    L.orc_get_diag.argtypes = [vp, C.c_int, _dp]
    L.orc_external_forces.argtypes = [vp, C.c_int, _dp, _dp]
    L.orc_interpolate.argtypes = [vp, C.c_int, _dp, _dp]
    L.orc_spread.argtypes = [vp, C.c_int, _dp, _dp, _dp, _dp]
    L.orc_set_contact.argtypes = [vp, C.c_double]
    L.orc_add_rigid.argtypes = [vp, C.c_int, _dp, C.c_double, C.c_double]
    L.orc_get_rigid.argtypes = [vp, C.c_int, _dp]
    L.orc_get_contact.argtypes = [vp, C.c_int, _dp]
    L.orc_set_threads.argtypes = [C.c_int]
    L.orc_get_threads.restype = C.c_int
    _lib = L
    return L


# ---- free functions -------------------------------------------------------

def equilibrium(rho: float, ux: float, uy: float) -> np.ndarray:
    out = np.zeros(9)
    lib().orc_equilibrium(rho, ux, uy, out)
    return out


def forcing(tau: float, ux: float, uy: float, fx: float, fy: float) -> np.ndarray:
    out = np.zeros(9)
    lib().orc_forcing(tau, ux, uy, fx, fy, out)
    return out


def mls(x: float, y: float):
    """Returns (cells [9][2] int, phi [9], dphi/dx [9], dphi/dy [9])."""
    cx = np.zeros(9, np.int32)
    cy = np.zeros(9, np.int32)
    phi, dx, dy = np.zeros(9), np.zeros(9), np.zeros(9)
    lib().orc_mls(x, y, cx, cy, phi, dx, dy)
    return np.stack([cx, cy], 1), phi, dx, dy


def internal_forces(x: np.ndarray, l0, theta0, ks, kb: float, ka: float, A0: float):
    """Returns (stretch, bending, area) nodal forces, each [nv][2]."""
    x = np.ascontiguousarray(x, np.float64)
    nv = x.shape[0]
    ks = np.broadcast_to(np.asarray(ks, np.float64), (nv,)).copy()
    fs, fb, fa = np.zeros((nv, 2)), np.zeros((nv, 2)), np.zeros((nv, 2))
    lib().orc_internal_forces(nv, x, np.ascontiguousarray(l0, np.float64),
                              np.ascontiguousarray(theta0, np.float64), ks, kb, ka, A0, fs, fb, fa)
    return fs, fb, fa


def polygon_diag(x: np.ndarray) -> Dict[str, float]:
    out = np.zeros(9)
    x = np.ascontiguousarray(x, np.float64)
    lib().orc_polygon_diag(x.shape[0], x, out)
    keys = ["area", "perimeter", "cx", "cy", "D", "Sw", "Jxx", "Jyy", "Jxy"]
    return dict(zip(keys, out.tolist()))


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


# ---- simulation -----------------------------------------------------------

class Sim:
    """FP64 reference simulation built from a workload dictionary."""

    def __init__(self, cfg: Dict[str, Any]):
        L = lib()
        self.cfg = cfg
        self.nx, self.ny = int(cfg["nx"]), int(cfg["ny"])
        ux0, uy0 = cfg.get("init_u", (0.0, 0.0))
        self.h = L.orc_create(self.nx, self.ny, float(cfg["tau"]), int(cfg.get("periodic_y", 0)),
                              float(cfg.get("u_bottom", 0.0)), float(cfg.get("u_top", 0.0)),
                              float(cfg.get("body_force_x", 0.0)), 0.0,
                              int(cfg.get("init_profile", 0)), float(ux0), float(uy0),
                              int(cfg.get("periodic_x", 1)), float(cfg.get("inlet_umax", 0.0)),
                              float(cfg.get("outlet_rho", 1.0)))
        self.nodes = []
        for cap in cfg.get("capsules", []):
            nodes = np.ascontiguousarray(cap["nodes"], np.float64)
            if cap.get("rigid"):
                L.orc_add_rigid(self.h, nodes.shape[0], nodes, float(cap["mass"]),
                                float(cap["inertia"]))
            else:
                ks = np.atleast_1d(np.asarray(cap["ks"], np.float64)).copy()
                L.orc_add_capsule(self.h, nodes.shape[0], nodes, ks, ks.size, float(cap["kb"]),
                                  float(cap["ka"]), float(cap["mass"]))
            self.nodes.append(nodes.shape[0])
        if cfg.get("contact_cutoff", 0.0):
            L.orc_set_contact(self.h, float(cfg["contact_cutoff"]))

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().orc_destroy(h)
            self.h = None

    def step(self, n: int, mode: Optional[str] = None) -> None:
        mode = mode or self.cfg["mode"]
        m = DYNAMIC if mode == "dynamic" else KINEMATIC
        rc = lib().orc_step(self.h, int(n), m)
        if rc != 0:
            raise RuntimeError(f"orc_step returned {rc}")

    @property
    def status(self) -> int:
        return int(lib().orc_status(self.h))

    @property
    def steps(self) -> int:
        return int(lib().orc_steps(self.h))

    def pops(self) -> np.ndarray:
        out = np.zeros((9, self.ny, self.nx))
        lib().orc_get_pops(self.h, out)
        return out

    def set_pops(self, f: np.ndarray) -> None:
        lib().orc_set_pops(self.h, np.ascontiguousarray(f, np.float64))

    def moments(self) -> np.ndarray:
        """[3][ny][nx]: rho, ux, uy (velocity with half of the last force)."""
        out = np.zeros((3, self.ny, self.nx))
        lib().orc_get_moments(self.h, out)
        return out

    def set_moments(self, m: np.ndarray) -> None:
        lib().orc_set_moments(self.h, np.ascontiguousarray(m, np.float64))

    def force(self) -> np.ndarray:
        out = np.zeros((2, self.ny, self.nx))
        lib().orc_get_force(self.h, out)
        return out

    def set_force(self, F: np.ndarray) -> None:
        lib().orc_set_force(self.h, np.ascontiguousarray(F, np.float64))

    def capsule(self, c: int):
        nv = self.nodes[c]
        x, xm1, uv = np.zeros((nv, 2)), np.zeros((nv, 2)), np.zeros((nv, 2))
        lib().orc_get_capsule(self.h, c, x, xm1, uv)
        return x, xm1, uv

    def set_capsule(self, c: int, x, xm1, uv) -> None:
        lib().orc_set_capsule(self.h, c, *(np.ascontiguousarray(a, np.float64) for a in (x, xm1, uv)))

    def rigid(self, c: int) -> Dict[str, float]:
        """Rigid particle state: centroid, angle, velocity, angular velocity, last
        hydrodynamic force and torque."""
        out = np.zeros(10)
        lib().orc_get_rigid(self.h, c, out)
        return dict(zip(["X", "Y", "theta", "ux", "uy", "w", "Fx", "Fy", "M", "rigid"],
                        out.tolist()))

    def contact(self, c: int) -> np.ndarray:
        """Contact forces (Eq. 27) of the positions at the last force evaluation."""
        out = np.zeros((self.nodes[c], 2))
        lib().orc_get_contact(self.h, c, out)
        return out

    def capsule_forces(self, c: int):
        nv = self.nodes[c]
        ft, fe = np.zeros((nv, 2)), np.zeros((nv, 2))
        lib().orc_get_capsule_forces(self.h, c, ft, fe)
        return ft, fe

    def diag(self, c: int) -> Dict[str, float]:
        out = np.zeros(13)
        lib().orc_get_diag(self.h, c, out)
        keys = ["area", "perimeter", "cx", "cy", "D", "Sw", "Jxx", "Jyy", "Jxy", "dp", "dA",
                "A0", "P0"]
        return dict(zip(keys, out.tolist()))

    def external_forces(self, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, np.float64)
        out = np.zeros_like(x)
        lib().orc_external_forces(self.h, x.shape[0], x, out)
        return out

    def interpolate(self, xy: np.ndarray) -> np.ndarray:
        xy = np.ascontiguousarray(xy, np.float64)
        out = np.zeros_like(xy)
        lib().orc_interpolate(self.h, xy.shape[0], xy, out)
        return out

    def spread(self, xy: np.ndarray, c: np.ndarray, F: np.ndarray) -> np.ndarray:
        xy = np.ascontiguousarray(xy, np.float64)
        out = np.zeros((2, self.ny, self.nx))
        lib().orc_spread(self.h, xy.shape[0], xy, np.ascontiguousarray(c, np.float64),
                         np.ascontiguousarray(F, np.float64), out)
        return out


# ---- gradients by central differences ----------------------------------------

def objective(cfg: Dict[str, Any], steps: int, which: str = "D", capsule: int = 0) -> float:
    """Objective of the final shape after ``steps`` steps of the FP64 oracle:
    the Taylor deformation D or the area-centroid height y_c (Sec. 3)."""
    s = Sim(cfg)
    s.step(steps)
    if s.status:
        raise RuntimeError(f"oracle status {s.status}")
    return s.diag(capsule)["D" if which == "D" else "cy"]


def perturbed(cfg: Dict[str, Any], param: Any, delta: float) -> Dict[str, Any]:
    """Copy of cfg with one parameter moved by delta: ("ks", capsule, element)
    for one element's stretching constant, or "g" for the uniform body force
    (which also sets the initial Poiseuille profile)."""
    new = dict(cfg)
    if param == "g":
        new["body_force_x"] = float(cfg["body_force_x"]) + delta
        return new
    _, c, l = param
    caps = [dict(k) for k in cfg["capsules"]]
    nv = len(caps[c]["nodes"])
    ks = np.broadcast_to(np.asarray(caps[c]["ks"], np.float64), (nv,)).copy()
    ks[l] += delta
    caps[c]["ks"] = ks
    new["capsules"] = caps
    return new


def central_difference(cfg: Dict[str, Any], steps: int, param: Any, h: float,
                       which: str = "D", capsule: int = 0) -> float:
    """dJ/dparam ~ (J(p + h) - J(p - h)) / (2 h): the definition of the
    derivative with a symmetric difference, error O(h^2)."""
    jp = objective(perturbed(cfg, param, h), steps, which, capsule)
    jm = objective(perturbed(cfg, param, -h), steps, which, capsule)
    return (jp - jm) / (2.0 * h)
