"""Thin ctypes binding of the C-ABI library ``liblbib.so`` (include/lbib.h).

Argument marshalling only.  Every step of the method runs in the HIP kernels
behind the ABI.  PyTorch supplies the device buffers (``torch.empty`` on the
current device) and the HIP stream (``torch.cuda.current_stream()``).  If the
compiled library is missing, loading fails loudly.  There is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Any, Dict, List, Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblbib.so")

# lbib_status
OK, EINVAL, ECAPACITY, EDEVICE, ESTATE, ENUMERIC = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ECAPACITY", -3: "EDEVICE", -4: "ESTATE",
                -5: "ENUMERIC"}
KINEMATIC, DYNAMIC = 0, 1
(FLAG_WALL, FLAG_NONFINITE, FLAG_PATCH, FLAG_OVERFLOW, FLAG_MOVE, FLAG_NEAR, FLAG_SYNC,
 FLAG_EDGE, FLAG_AREA) = 1, 2, 4, 8, 16, 32, 64, 128, 256
NUM_BUFFERS = 8
BUFFER_NAMES = ["pops_a", "pops_b", "force", "flags", "nodes", "caps", "diag", "stage"]
# lbib_state_id
F_POPS, F_POPS_DEV, F_MOMENTS, F_FORCE = 0, 1, 2, 3
C_NODES, C_PREV, C_VEL, C_FORCE, C_STATE, C_DIAG, STATUS, C_RIGID = 4, 5, 6, 7, 8, 9, 10, 11
DIAG_KEYS = ["area", "perimeter", "cx", "cy", "D", "Sw", "dp", "dA", "Jxx", "Jyy", "Jxy", "A0",
             "P0"]

EXPORTS = ["lbib_required_bytes", "lbib_create", "lbib_add_capsule", "lbib_step",
           "lbib_get_state", "lbib_set_state", "lbib_check", "lbib_set_timing",
           "lbib_get_timing", "lbib_steps_done", "lbib_last_error", "lbib_destroy",
           "lbib_required_bytes_batch", "lbib_create_batch", "lbib_add_capsule_to",
           "lbib_num_lattices", "lbib_adjoint_bytes", "lbib_adjoint", "lbib_adjoint_noalloc",
           "lbib_set_overlap", "lbib_set_graph", "lbib_graph_replays", "lbib_set_tile", "lbib_autotune",
           "lbib_set_contact", "lbib_add_rigid_to", "lbib_set_limits"]
OBJ_TAYLOR, OBJ_CENTROID_Y = 0, 1
ADJOINT_SCRATCH_BYTES = 64 * 1024 * 1024  # LBIB_ADJOINT_SCRATCH_BYTES
TILE_ORDERS = ("banded", "linear", "chunked")  # tile orders of the batched grid pass


class lbib_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("real_bytes", C.c_int32),
                ("max_capsules", C.c_int32), ("max_nodes_total", C.c_int32),
                ("max_nodes_capsule", C.c_int32)]


class lbib_walls(C.Structure):
    _fields_ = [("periodic_x", C.c_int32), ("periodic_y", C.c_int32),
                ("u_bottom", C.c_double), ("u_top", C.c_double),
                ("body_force_x", C.c_double), ("init_profile", C.c_int32),
                ("init_ux", C.c_double), ("init_uy", C.c_double),
                ("inlet_umax", C.c_double), ("outlet_rho", C.c_double)]


class LbibError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib: Optional[C.CDLL] = None


def load() -> C.CDLL:
    """Loads liblbib.so (built by ``python -m paper_1903_03356_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch carries its own HIP runtime; loading it first makes the library
    # bind to that same runtime (one device context, torch's streams and
    # synchronisation), instead of a second copy from the ROCm install
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1903_03356_amd.build` (hipcc, gfx950)")
    L = C.CDLL(LIB_PATH)
    vp, i32 = C.c_void_p, C.c_int32
    L.lbib_required_bytes.restype = C.c_size_t
    L.lbib_required_bytes.argtypes = [C.POINTER(lbib_grid), i32]
    L.lbib_create.restype = i32
    L.lbib_create.argtypes = [C.POINTER(lbib_grid), C.c_double, C.POINTER(lbib_walls),
                              C.POINTER(vp), i32, vp, C.POINTER(vp)]
    L.lbib_add_capsule.restype = i32
    L.lbib_add_capsule.argtypes = [vp, C.POINTER(C.c_double), i32, C.POINTER(C.c_double), i32,
                                   C.c_double, C.c_double, C.c_double, C.POINTER(i32)]
    L.lbib_step.restype = i32
    L.lbib_step.argtypes = [vp, i32, i32]
    L.lbib_get_state.restype = i32
    L.lbib_get_state.argtypes = [vp, i32, i32, vp, C.c_size_t, i32]
    L.lbib_set_state.restype = i32
    L.lbib_set_state.argtypes = [vp, i32, i32, vp, C.c_size_t, i32]
    L.lbib_check.restype = i32
    L.lbib_check.argtypes = [vp, C.POINTER(i32)]
    L.lbib_set_timing.restype = i32
    L.lbib_set_timing.argtypes = [vp, i32]
    L.lbib_set_overlap.restype = i32
    L.lbib_set_overlap.argtypes = [vp, i32]
    L.lbib_set_contact.restype = i32
    L.lbib_set_contact.argtypes = [vp, C.c_double]
    L.lbib_add_rigid_to.restype = i32
    L.lbib_add_rigid_to.argtypes = [vp, i32, C.POINTER(C.c_double), i32, C.c_double, C.c_double,
                                    C.POINTER(i32)]
    L.lbib_get_timing.restype = i32
    L.lbib_get_timing.argtypes = [vp, C.POINTER(C.c_double)]
    L.lbib_steps_done.restype = C.c_int64
    L.lbib_steps_done.argtypes = [vp]
    L.lbib_last_error.restype = C.c_char_p
    L.lbib_last_error.argtypes = [vp]
    L.lbib_destroy.restype = None
    L.lbib_destroy.argtypes = [vp]
    L.lbib_required_bytes_batch.restype = C.c_size_t
    L.lbib_required_bytes_batch.argtypes = [C.POINTER(lbib_grid), i32, i32]
    L.lbib_create_batch.restype = i32
    L.lbib_create_batch.argtypes = [C.POINTER(lbib_grid), C.POINTER(C.c_double),
                                    C.POINTER(lbib_walls), i32, C.POINTER(vp), i32, vp,
                                    C.POINTER(vp)]
    L.lbib_add_capsule_to.restype = i32
    L.lbib_add_capsule_to.argtypes = [vp, i32, C.POINTER(C.c_double), i32, C.POINTER(C.c_double),
                                      i32, C.c_double, C.c_double, C.c_double, C.POINTER(i32)]
    L.lbib_num_lattices.restype = i32
    L.lbib_num_lattices.argtypes = [vp]
    L.lbib_set_graph.restype = i32
    L.lbib_set_graph.argtypes = [vp, i32]
    L.lbib_graph_replays.restype = C.c_int64
    L.lbib_graph_replays.argtypes = [vp]
    L.lbib_set_tile.restype = i32
    L.lbib_set_tile.argtypes = [vp, i32, i32, i32]
    L.lbib_autotune.restype = i32
    L.lbib_autotune.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32),
                                C.POINTER(C.c_double), i32]
    L.lbib_adjoint_bytes.restype = C.c_size_t
    L.lbib_adjoint_bytes.argtypes = [vp, i32, i32]
    dp = C.POINTER(C.c_double)
    L.lbib_adjoint.restype = i32
    L.lbib_adjoint.argtypes = [vp, i32, i32, i32, i32, i32, vp, C.c_size_t, dp, dp, dp, i32]
    L.lbib_set_limits.restype = i32
    L.lbib_set_limits.argtypes = [vp, C.c_double, C.c_double]
    L.lbib_adjoint_noalloc.restype = i32
    L.lbib_adjoint_noalloc.argtypes = [vp, i32, i32, i32, i32, i32, dp, dp, dp, i32]
    _lib = L
    return L


def _check(rc: int, ctx=None) -> None:
    if rc != OK:
        msg = load().lbib_last_error(ctx)
        raise LbibError(rc, msg.decode() if msg else "")


def make_grid(nx: int, ny: int, real_bytes: int, max_capsules: int = 1,
              max_nodes_total: int = 3, max_nodes_capsule: int = 3) -> lbib_grid:
    return lbib_grid(nx, ny, real_bytes, max(1, max_capsules), max(3, max_nodes_total),
                     max(3, max_nodes_capsule))


def required_bytes(grid: lbib_grid, buffer_id: int) -> int:
    return int(load().lbib_required_bytes(C.byref(grid), buffer_id))


def required_bytes_batch(grids, buffer_id: int) -> int:
    arr = (lbib_grid * len(grids))(*grids)
    return int(load().lbib_required_bytes_batch(arr, len(grids), buffer_id))


def grid_of(cfg: Dict[str, Any], max_capsules: int = 0, max_nodes_total: int = 0,
            max_nodes_capsule: int = 0) -> lbib_grid:
    caps = cfg.get("capsules", [])
    nodes_total = sum(len(c["nodes"]) for c in caps)
    nv_max = max([len(c["nodes"]) for c in caps] + [3])
    return make_grid(int(cfg["nx"]), int(cfg["ny"]), int(cfg["real_bytes"]),
                     max(1, len(caps), max_capsules), max(3, nodes_total, max_nodes_total),
                     max(nv_max, max_nodes_capsule))


def walls_of(cfg: Dict[str, Any]) -> lbib_walls:
    ux0, uy0 = cfg.get("init_u", (0.0, 0.0))
    return lbib_walls(int(cfg.get("periodic_x", 1)), int(cfg.get("periodic_y", 0)),
                      float(cfg.get("u_bottom", 0.0)), float(cfg.get("u_top", 0.0)),
                      float(cfg.get("body_force_x", 0.0)), int(cfg.get("init_profile", 0)),
                      float(ux0), float(uy0), float(cfg.get("inlet_umax", 0.0)),
                      float(cfg.get("outlet_rho", 1.0)))


class Sim:
    """One context: device buffers allocated with torch, kernels in liblbib.so.

    ``cfg`` is a workload dictionary (paper_1903_03356_amd.workloads)."""

    def __init__(self, cfg: Dict[str, Any], device: Optional[Any] = None, stream=None,
                 max_capsules: int = 0, max_nodes_total: int = 0, max_nodes_capsule: int = 0):
        import torch
        L = load()
        self.torch = torch
        self.cfg = cfg
        self.device = torch.device(device if device is not None else "cuda")
        caps = cfg.get("capsules", [])
        self.grid = grid_of(cfg, max_capsules, max_nodes_total, max_nodes_capsule)
        self.walls = walls_of(cfg)
        self.buffers: List[Any] = []
        with torch.cuda.device(self.device):
            for i in range(NUM_BUFFERS):
                nb = required_bytes(self.grid, i)
                if nb == 0:
                    raise LbibError(ECAPACITY, "invalid grid for buffer sizing")
                self.buffers.append(torch.empty(nb, dtype=torch.uint8, device=self.device))
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            ptrs = (C.c_void_p * NUM_BUFFERS)(*[b.data_ptr() for b in self.buffers])
            h = C.c_void_p()
            _check(L.lbib_create(C.byref(self.grid), float(cfg["tau"]), C.byref(self.walls), ptrs,
                                 NUM_BUFFERS, C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        self.nv: List[int] = []
        self.dims = [(int(cfg["nx"]), int(cfg["ny"]))]
        for cap in caps:
            if cap.get("rigid"):
                self.add_rigid_to(0, cap["nodes"], cap["mass"], cap["inertia"])
            else:
                self.add_capsule(cap["nodes"], cap["ks"], cap["kb"], cap["ka"], cap["mass"])
        self.nx, self.ny = int(cfg["nx"]), int(cfg["ny"])
        if cfg.get("contact_cutoff", 0.0):
            self.set_contact(float(cfg["contact_cutoff"]))

    # -- ABI wrappers with the same names ------------------------------------
    def add_capsule(self, nodes, ks, kb: float, ka: float, mass: float) -> int:
        nodes = np.ascontiguousarray(nodes, np.float64)
        ks = np.ascontiguousarray(np.atleast_1d(np.asarray(ks, np.float64)))
        cid = C.c_int32()
        dp = C.POINTER(C.c_double)
        with self.torch.cuda.device(self.device):
            _check(load().lbib_add_capsule(self.h, nodes.ctypes.data_as(dp), nodes.shape[0],
                                           ks.ctypes.data_as(dp), ks.size, float(kb), float(ka),
                                           float(mass), C.byref(cid)), self.h)
        self.nv.append(nodes.shape[0])
        return cid.value

    def add_capsule_to(self, lattice: int, nodes, ks, kb: float, ka: float, mass: float) -> int:
        nodes = np.ascontiguousarray(nodes, np.float64)
        ks = np.ascontiguousarray(np.atleast_1d(np.asarray(ks, np.float64)))
        cid = C.c_int32()
        dp = C.POINTER(C.c_double)
        with self.torch.cuda.device(self.device):
            _check(load().lbib_add_capsule_to(self.h, int(lattice), nodes.ctypes.data_as(dp),
                                              nodes.shape[0], ks.ctypes.data_as(dp), ks.size,
                                              float(kb), float(ka), float(mass), C.byref(cid)),
                   self.h)
        self.nv.append(nodes.shape[0])
        return cid.value

    def add_rigid_to(self, lattice: int, nodes, mass: float, inertia: float) -> int:
        nodes = np.ascontiguousarray(nodes, np.float64)
        cid = C.c_int32()
        with self.torch.cuda.device(self.device):
            _check(load().lbib_add_rigid_to(self.h, int(lattice),
                                            nodes.ctypes.data_as(C.POINTER(C.c_double)),
                                            nodes.shape[0], float(mass), float(inertia),
                                            C.byref(cid)), self.h)
        self.nv.append(nodes.shape[0])
        return cid.value

    def rigid(self, c: int) -> Dict[str, float]:
        """Rigid particle state: centroid, angle, velocity, angular velocity and
        the last force and torque (LBIB_C_RIGID)."""
        out = np.zeros(10)
        with self.torch.cuda.device(self.device):
            _check(load().lbib_get_state(self.h, C_RIGID, int(c), out.ctypes.data_as(C.c_void_p),
                                         out.nbytes, 0), self.h)
        return dict(zip(["X", "Y", "theta", "ux", "uy", "w", "Fx", "Fy", "M", "rigid"],
                        out.tolist()))

    @property
    def num_lattices(self) -> int:
        return int(load().lbib_num_lattices(self.h))

    def step(self, n: int, mode: Optional[str] = None) -> None:
        mode = mode or self.cfg.get("mode", "dynamic")
        m = DYNAMIC if mode == "dynamic" else KINEMATIC
        with self.torch.cuda.device(self.device):
            _check(load().lbib_step(self.h, int(n), m), self.h)

    def get_state(self, what: int, capsule: int = 0, out=None):
        """Host copy (numpy FP64) or, with ``out`` a CUDA FP64 tensor, a queued device copy.
        ``capsule`` is the capsule id, or the lattice index for the field states."""
        field = what in (F_POPS, F_POPS_DEV, F_MOMENTS, F_FORCE)
        # an index out of range goes to the library, which rejects it (EINVAL)
        nx, ny = self.dims[capsule] if field and 0 <= capsule < len(self.dims) else (1, 1)
        shapes = {F_POPS: (9, ny, nx), F_POPS_DEV: (9, ny, nx),
                  F_MOMENTS: (3, ny, nx), F_FORCE: (2, ny, nx),
                  C_DIAG: (16,), STATUS: (1,)}
        if what in shapes:
            shape = shapes[what]
        else:
            nv = self.nv[capsule] if 0 <= capsule < len(self.nv) else 1
            shape = (3, nv, 2) if what == C_STATE else (nv, 2)
        with self.torch.cuda.device(self.device):
            if out is not None:
                _check(load().lbib_get_state(self.h, what, capsule, C.c_void_p(out.data_ptr()),
                                             out.numel() * out.element_size(), 1), self.h)
                return out
            arr = np.zeros(shape, np.int32 if what == STATUS else np.float64)
            _check(load().lbib_get_state(self.h, what, capsule, arr.ctypes.data_as(C.c_void_p),
                                         arr.nbytes, 0), self.h)
        return arr

    def set_state(self, what: int, src, capsule: int = 0) -> None:
        with self.torch.cuda.device(self.device):
            if hasattr(src, "data_ptr"):
                _check(load().lbib_set_state(self.h, what, capsule, C.c_void_p(src.data_ptr()),
                                             src.numel() * src.element_size(), 1), self.h)
            else:
                a = np.ascontiguousarray(src, np.float64)
                _check(load().lbib_set_state(self.h, what, capsule, a.ctypes.data_as(C.c_void_p),
                                             a.nbytes, 0), self.h)

    def check(self) -> int:
        flags = C.c_int32()
        with self.torch.cuda.device(self.device):
            rc = load().lbib_check(self.h, C.byref(flags))
        if rc not in (OK, ENUMERIC):
            _check(rc, self.h)
        return flags.value

    def set_timing(self, enable: bool) -> None:
        _check(load().lbib_set_timing(self.h, 1 if enable else 0), self.h)

    def get_timing(self) -> Dict[str, float]:
        out = (C.c_double * 6)()
        with self.torch.cuda.device(self.device):
            _check(load().lbib_get_timing(self.h, out), self.h)
        return {"grid_ms": out[0], "grid_launches": out[1], "ib_ms": out[2],
                "ib_launches": out[3], "near_ms": out[4], "near_launches": out[5]}

    def set_contact(self, cutoff: float) -> None:
        with self.torch.cuda.device(self.device):
            _check(load().lbib_set_contact(self.h, float(cutoff)), self.h)

    def set_overlap(self, enable, queue_waits: bool = False) -> None:
        """True / False force the overlapped schedule on / off; None restores
        the automatic choice (a single lattice of 2^22 cells or more).
        queue_waits=True (with enable=True) keeps every hand-off between the
        two streams on the queue (lbib_set_overlap(ctx, 2)), for tools that run
        kernels one at a time."""
        v = -1 if enable is None else ((2 if queue_waits else 1) if enable else 0)
        _check(load().lbib_set_overlap(self.h, v), self.h)

    def set_limits(self, max_edge: float = 0.0, max_area_change: float = 0.0) -> None:
        """lbib_set_limits: element length and area-change checks (0 = off)."""
        _check(load().lbib_set_limits(self.h, float(max_edge), float(max_area_change)), self.h)

    def set_graph(self, enable) -> None:
        """True replays captured 16-step blocks; False and None (the
        default) launch every step directly."""
        v = -1 if enable is None else (1 if enable else 0)
        _check(load().lbib_set_graph(self.h, v), self.h)

    @property
    def graph_replays(self) -> int:
        return int(load().lbib_graph_replays(self.h))

    def set_tile(self, rows: int, resident: int = 0, linear=False) -> None:
        """Tile shape of the batched grid pass (lbib_set_tile).  ``linear`` is
        the tile order: False / 0 banded, True / 1 linear, "chunked" / 2."""
        order = TILE_ORDERS.index(linear) if isinstance(linear, str) else int(linear)
        _check(load().lbib_set_tile(self.h, int(rows), order, int(resident)), self.h)

    def autotune(self, launches: int = 20) -> Dict[str, Any]:
        """lbib_autotune: times the 36 tile shapes of the batched grid pass and
        keeps the fastest; returns the choice (``order`` one of TILE_ORDERS,
        ``linear`` its index) and the mean time per pass (us) of every (order,
        rows, resident) candidate."""
        rows, lin, res = C.c_int32(), C.c_int32(), C.c_int32()
        n = 4 * 3 * len(TILE_ORDERS)
        us = (C.c_double * n)()
        with self.torch.cuda.device(self.device):
            _check(load().lbib_autotune(self.h, int(launches), C.byref(rows), C.byref(lin),
                                        C.byref(res), us, n), self.h)
        cands = [(o, r, k) for o in TILE_ORDERS for r in (1, 2, 4) for k in (0, 2, 4, 8)]
        return {"rows": rows.value, "linear": lin.value, "order": TILE_ORDERS[lin.value],
                "resident": res.value,
                "us": {f"{o}_rows{r}_resident{k}": round(us[i], 2)
                       for i, (o, r, k) in enumerate(cands)}}

    def adjoint_bytes(self, nsteps: int, checkpoint_every: int = 0) -> int:
        return int(load().lbib_adjoint_bytes(self.h, int(nsteps), int(checkpoint_every)))

    def adjoint(self, nsteps: int, objective: int = OBJ_TAYLOR, capsule: int = 0,
                mode: Optional[str] = None, workspace=None,
                checkpoint_every: int = 0) -> Dict[str, Any]:
        """lbib_adjoint: J and dJ/dg, dJ/dk_s (per element, node order) of an
        nsteps run from step 0.  checkpoint_every = 0 tapes the whole
        trajectory; K > 0 keeps every K-th grid state and recomputes the
        segments in the reverse sweep.  Allocates the workspace unless given."""
        mode = mode or self.cfg.get("mode", "dynamic")
        m = DYNAMIC if mode == "dynamic" else KINEMATIC
        nb = self.adjoint_bytes(nsteps, checkpoint_every)
        if nb == 0:
            raise LbibError(EINVAL, "no adjoint layout for this context")
        with self.torch.cuda.device(self.device):
            ws = workspace if workspace is not None else self.torch.empty(
                nb, dtype=self.torch.uint8, device=self.device)
            nks = max(1, sum(self.nv))
            ks = np.zeros(nks, np.float64)
            J, g = C.c_double(), C.c_double()
            _check(load().lbib_adjoint(self.h, int(nsteps), int(checkpoint_every), m,
                                       int(objective), int(capsule),
                                       C.c_void_p(ws.data_ptr()), ws.numel(), C.byref(J),
                                       C.byref(g), ks.ctypes.data_as(C.POINTER(C.c_double)),
                                       nks), self.h)
        caps, o = [], 0
        for n in self.nv:
            caps.append(ks[o:o + n].copy())
            o += n
        return {"J": J.value, "dJ_dg": g.value, "dJ_dks": caps}

    def adjoint_noalloc(self, nsteps: int, objective: int = OBJ_TAYLOR, capsule: int = 0,
                        mode: Optional[str] = None, checkpoint_every: int = 0) -> Dict[str, Any]:
        """lbib_adjoint_noalloc: as ``adjoint``, with the library's static
        workspace (at most ADJOINT_SCRATCH_BYTES) instead of a caller-owned one."""
        mode = mode or self.cfg.get("mode", "dynamic")
        m = DYNAMIC if mode == "dynamic" else KINEMATIC
        nks = max(1, sum(self.nv))
        ks = np.zeros(nks, np.float64)
        J, g = C.c_double(), C.c_double()
        with self.torch.cuda.device(self.device):
            _check(load().lbib_adjoint_noalloc(self.h, int(nsteps), int(checkpoint_every), m,
                                               int(objective), int(capsule), C.byref(J),
                                               C.byref(g),
                                               ks.ctypes.data_as(C.POINTER(C.c_double)), nks),
                   self.h)
        caps, o = [], 0
        for n in self.nv:
            caps.append(ks[o:o + n].copy())
            o += n
        return {"J": J.value, "dJ_dg": g.value, "dJ_dks": caps}

    @property
    def steps_done(self) -> int:
        return int(load().lbib_steps_done(self.h))

    # -- conveniences -----------------------------------------------------------
    def pops(self, lattice: int = 0) -> np.ndarray:
        return self.get_state(F_POPS, lattice)

    def pops_dev(self, lattice: int = 0) -> np.ndarray:
        return self.get_state(F_POPS_DEV, lattice)

    def set_pops(self, f, lattice: int = 0) -> None:
        self.set_state(F_POPS, f, lattice)

    def moments(self, lattice: int = 0) -> np.ndarray:
        return self.get_state(F_MOMENTS, lattice)

    def force(self, lattice: int = 0) -> np.ndarray:
        return self.get_state(F_FORCE, lattice)

    def capsule(self, c: int):
        s = self.get_state(C_STATE, c)
        return s[0], s[1], s[2]

    def set_capsule(self, c: int, x, xm1, uv) -> None:
        self.set_state(C_STATE, np.stack([np.asarray(x), np.asarray(xm1), np.asarray(uv)]), c)

    def capsule_force(self, c: int) -> np.ndarray:
        return self.get_state(C_FORCE, c)

    def diag(self, c: int) -> Dict[str, float]:
        d = self.get_state(C_DIAG, c)
        return dict(zip(DIAG_KEYS, d.tolist()))

    def close(self) -> None:
        h = getattr(self, "h", None)
        if h:
            load().lbib_destroy(h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch(Sim):
    """Ensemble context: one lattice per workload dictionary in ``cfgs``, stepped
    together (lbib_create_batch).  Capsule ids run over the whole batch, lattice
    by lattice; ``cap_ids[i]`` lists those of lattice i.  Field getters take
    the lattice index."""

    def __init__(self, cfgs: List[Dict[str, Any]], device: Optional[Any] = None, stream=None):
        import torch
        L = load()
        if not cfgs:
            raise ValueError("a batch needs at least one lattice")
        modes = {c.get("mode", "dynamic") for c in cfgs}
        if len(modes) != 1:
            raise ValueError("all lattices of a batch share the coupling mode")
        self.torch = torch
        self.cfg = dict(cfgs[0])
        self.cfgs = cfgs
        self.device = torch.device(device if device is not None else "cuda")
        grids = [grid_of(c) for c in cfgs]
        self.grids = (lbib_grid * len(cfgs))(*grids)
        self.walls_arr = (lbib_walls * len(cfgs))(*[walls_of(c) for c in cfgs])
        taus = (C.c_double * len(cfgs))(*[float(c["tau"]) for c in cfgs])
        self.buffers: List[Any] = []
        with torch.cuda.device(self.device):
            for i in range(NUM_BUFFERS):
                nb = int(L.lbib_required_bytes_batch(self.grids, len(cfgs), i))
                if nb == 0:
                    raise LbibError(ECAPACITY, "invalid lattices for buffer sizing")
                self.buffers.append(torch.empty(nb, dtype=torch.uint8, device=self.device))
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            ptrs = (C.c_void_p * NUM_BUFFERS)(*[b.data_ptr() for b in self.buffers])
            h = C.c_void_p()
            _check(L.lbib_create_batch(self.grids, taus, self.walls_arr, len(cfgs), ptrs,
                                       NUM_BUFFERS, C.c_void_p(self.stream.cuda_stream),
                                       C.byref(h)))
        self.h = h
        self.nv: List[int] = []
        self.dims = [(int(c["nx"]), int(c["ny"])) for c in cfgs]
        self.cap_ids: List[List[int]] = []
        for i, c in enumerate(cfgs):
            ids = [self.add_rigid_to(i, cap["nodes"], cap["mass"], cap["inertia"])
                   if cap.get("rigid") else
                   self.add_capsule_to(i, cap["nodes"], cap["ks"], cap["kb"], cap["ka"],
                                       cap["mass"]) for cap in c.get("capsules", [])]
            self.cap_ids.append(ids)
        self.nx, self.ny = self.dims[0]
        cut = max(float(c.get("contact_cutoff", 0.0)) for c in cfgs)
        if cut:
            self.set_contact(cut)


def capsule_objectives(ks, u_max, build, nsteps: int, capsule: int = 0,
                       mode: Optional[str] = None, checkpoint_every: int = 0):
    """Differentiable (D, y_c) of one capsule after ``nsteps`` steps from the
    initial state, as a function of the per-element stretching constants
    ``ks`` (1-D tensor) and the channel's peak speed ``u_max`` (0-D tensor).

    ``build(ks_array, u_max_float)`` returns the workload dictionary; its body
    force must be linear in u_max (g = 8 nu u_max / H^2, as the channel
    builders set it).  Forward: two lbib_adjoint runs (objectives D and y_c),
    whose gradients the backward combines with the incoming weights; dJ/du_max =
    dJ/dg * dg/du_max, with the slope dg/du_max = the body force ``build`` gives
    for u_max = 1 (also at u_max = 0).  The output and each gradient live on
    the device and in the dtype of their input.  ``checkpoint_every`` as in
    Sim.adjoint."""
    return _CapsuleObjectives.apply(ks, u_max, build, int(nsteps), int(capsule), mode,
                                    int(checkpoint_every))


def _make_objectives_function():
    import torch

    class CapsuleObjectives(torch.autograd.Function):
        @staticmethod
        def forward(ctx, ks, u_max, build, nsteps, capsule, mode, every):
            ks_np = ks.detach().cpu().double().numpy()
            um = float(u_max.detach().cpu())
            cfg = build(ks_np, um)
            slope = float(build(ks_np, 1.0)["body_force_x"])  # g is linear in u_max
            out, gks, gum = [], [], []
            for obj in (OBJ_TAYLOR, OBJ_CENTROID_Y):
                r = Sim(cfg).adjoint(nsteps, obj, capsule, mode, checkpoint_every=every)
                out.append(r["J"])
                gks.append(torch.as_tensor(r["dJ_dks"][capsule], dtype=ks.dtype,
                                           device=ks.device))
                gum.append(r["dJ_dg"] * slope)
            ctx.save_for_backward(torch.stack(gks))
            ctx.gum = gum
            ctx.um_meta = (u_max.dtype, u_max.device, u_max.shape)
            return torch.tensor(out, dtype=ks.dtype, device=ks.device)

        @staticmethod
        def backward(ctx, grad_out):
            (gks,) = ctx.saved_tensors
            w = grad_out.to(device=gks.device, dtype=gks.dtype)
            grad_ks = w[0] * gks[0] + w[1] * gks[1]
            dtype, device, shape = ctx.um_meta
            wc = w.detach().cpu().double()
            grad_um = torch.tensor(float(wc[0]) * ctx.gum[0] + float(wc[1]) * ctx.gum[1],
                                   dtype=dtype, device=device).reshape(shape)
            return grad_ks, grad_um, None, None, None, None, None

    return CapsuleObjectives


class _LazyFunction:
    def __init__(self):
        self.fn = None

    def apply(self, *args):
        if self.fn is None:
            self.fn = _make_objectives_function()
        return self.fn.apply(*args)


_CapsuleObjectives = _LazyFunction()
