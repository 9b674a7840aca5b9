"""Seeded synthetic workloads for the LBM - immersed-boundary capsule solver.

This module only generates inputs: lattice sizes, wall speeds, the uniform
body force that drives a periodic channel, capsule node coordinates and the
membrane constants handed to the solver.  It performs no step of the method
(no equilibrium, collision, interpolation, spreading or membrane force).  Both
the HIP library and the FP64 reference consume the dictionaries built here.

Shapes follow the paper's test cases (Sec. 3.1 shear capsule, Sec. 3.2-3.3
Poiseuille capsules, Eq. 26 biconcave outline); every random draw comes from
``numpy.random.default_rng(seed)`` in the order documented in each builder.

Units are lattice units: dx = dt = 1, reference density 1, c_s^2 = 1/3, so the
kinematic viscosity is nu = (tau - 1/2)/3 (Sec. 2.1).
"""
from __future__ import annotations

import math
from typing import Any, Dict, List

import numpy as np

# init_profile codes understood by both implementations
INIT_REST = 0
INIT_COUETTE = 1      # linear profile between the two wall speeds
INIT_POISEUILLE = 2   # u(y) = g/(2 nu) * y * (H - y), H = ny - 1
INIT_UNIFORM = 3      # uniform (ux, uy) everywhere (fully periodic boxes)
INIT_INLET = 4        # the inlet parabola 4 u_max y (H - y) / H^2 everywhere (open channels)


def viscosity(tau: float) -> float:
    """Lattice kinematic viscosity for relaxation time tau (Sec. 2.1)."""
    return (tau - 0.5) / 3.0


def poiseuille_body_force(tau: float, ny: int, u_max: float) -> float:
    """Uniform x-force that gives peak speed u_max in a channel with on-node walls
    at y = 0 and y = ny - 1 (channel height H = ny - 1):  g = 8 nu u_max / H^2."""
    H = ny - 1
    return 8.0 * viscosity(tau) * u_max / (H * H)


def ks_from_ca(tau: float, u_max: float, ca: float, rho_ref: float = 1.0) -> float:
    """Capillary-number definition Ca = nu rho u_max / k_s (Sec. 2.2.1)."""
    return viscosity(tau) * rho_ref * u_max / ca


def ks_from_g(tau: float, shear_rate: float, diameter: float, g_num: float,
              rho_ref: float = 1.0) -> float:
    """Dimensionless shear rate G = nu rho gamma d / k_s (Sec. 2.2.1, Sec. 3.1)."""
    return viscosity(tau) * rho_ref * shear_rate * diameter / g_num


def polygon_area(nodes: np.ndarray) -> float:
    """Signed area of a closed polygon (positive for counter-clockwise order).
    Used only to turn a density ratio into the capsule mass handed to the solver."""
    x, y = nodes[:, 0], nodes[:, 1]
    return 0.5 * float(np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y))


def circle_nodes(cx: float, cy: float, radius: float, n: int, phase: float = 0.5) -> np.ndarray:
    """n counter-clockwise nodes on a circle at angles 2 pi (k + phase) / n.
    phase = 0.5 keeps nodes off the symmetry axes, so no node sits exactly on a
    half-integer lattice coordinate for the centred shear case."""
    ang = 2.0 * math.pi * (np.arange(n) + phase) / n
    return np.stack([cx + radius * np.cos(ang), cy + radius * np.sin(ang)], axis=1)


def _resample_closed(curve: np.ndarray, n: int) -> np.ndarray:
    """Place n points equispaced in arc length along a densely sampled closed curve."""
    closed = np.vstack([curve, curve[:1]])
    seg = np.hypot(np.diff(closed[:, 0]), np.diff(closed[:, 1]))
    s = np.concatenate([[0.0], np.cumsum(seg)])
    targets = np.arange(n) * (s[-1] / n)
    x = np.interp(targets, s, closed[:, 0])
    y = np.interp(targets, s, closed[:, 1])
    return np.stack([x, y], axis=1)


def biconcave_nodes(cx: float, cy: float, length: float, n: int, angle: float = 0.0,
                    dense: int = 40000) -> np.ndarray:
    """Biconcave outline of Eq. 26 with the printed alpha/2 thickness factor.

    x = (L/2) sin q,  y = (L/4)(0.207 + 2.003 sin^2 q - 1.123 sin^4 q) cos q,
    q in [-pi/2, 3pi/2).  The paper's a*alpha only sets the scale, so it is
    chosen to make the long axis equal to ``length``.  As printed, increasing q
    runs clockwise; the samples are reversed to counter-clockwise order, then
    n nodes are placed equispaced in arc length and the shape is rotated by
    ``angle`` about its centre and moved to (cx, cy)."""
    q = -0.5 * math.pi + 2.0 * math.pi * np.arange(dense) / dense
    s = np.sin(q)
    half = 0.5 * length
    x = half * s
    y = 0.5 * half * (0.207 + 2.003 * s * s - 1.123 * s ** 4) * np.cos(q)
    curve = np.stack([x, y], axis=1)[::-1]
    pts = _resample_closed(curve, n)
    c, sn = math.cos(angle), math.sin(angle)
    rot = np.stack([c * pts[:, 0] - sn * pts[:, 1], sn * pts[:, 0] + c * pts[:, 1]], axis=1)
    return rot + np.array([cx, cy])


def capsule(nodes: np.ndarray, ks: float, kb: float = 0.0, ka: float = 1.0,
            density_ratio: float = 1.0) -> Dict[str, Any]:
    """Capsule record: nodes (n, 2) FP64 counter-clockwise, per-element stiffness
    (a scalar here), bending and area constants, and the total membrane mass
    m = (rho_s / rho_f) * rho_ref * A0 spread evenly over the n nodes (Eq. 21)."""
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    return {
        "nodes": nodes,
        "ks": float(ks),
        "kb": float(kb),
        "ka": float(ka),
        "mass": float(density_ratio * polygon_area(nodes)),
        "density_ratio": float(density_ratio),
    }


def rigid_particle(nodes: np.ndarray, density_ratio: float = 1.0) -> Dict[str, Any]:
    """Rigid particle record (Sec. 2.3.1): outline (n, 2) counter-clockwise,
    mass m = (rho_s / rho_f) A and moment of inertia I = (rho_s / rho_f) J about
    the area centroid, with A and J (polar second moment of area) from the
    polygon by Green's theorem."""
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    x, y = nodes[:, 0], nodes[:, 1]
    xn, yn = np.roll(x, -1), np.roll(y, -1)
    cr = x * yn - xn * y
    A = 0.5 * cr.sum()
    cx = ((x + xn) * cr).sum() / (6.0 * A)
    cy = ((y + yn) * cr).sum() / (6.0 * A)
    Jxx = ((y * y + y * yn + yn * yn) * cr).sum() / 12.0 - A * cy * cy
    Jyy = ((x * x + x * xn + xn * xn) * cr).sum() / 12.0 - A * cx * cx
    return {"nodes": nodes, "rigid": True, "ks": 0.0, "kb": 0.0, "ka": 0.0,
            "mass": float(density_ratio * A), "inertia": float(density_ratio * (Jxx + Jyy)),
            "density_ratio": float(density_ratio)}


def _base(name: str, nx: int, ny: int, tau: float, real_bytes: int, mode: str, steps: int,
          **kw: Any) -> Dict[str, Any]:
    cfg = {
        "name": name, "nx": nx, "ny": ny, "tau": tau, "real_bytes": real_bytes,
        "periodic_y": 0, "u_bottom": 0.0, "u_top": 0.0, "body_force_x": 0.0,
        "init_profile": INIT_REST, "init_u": (0.0, 0.0), "mode": mode, "steps": steps,
        "capsules": [],
    }
    cfg.update(kw)
    return cfg


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def shear_capsule(nx: int = 64, ny: int = 64, tau: float = 1.0, u_wall: float = 0.01,
                  radius: float = 8.0, n_nodes: int = 64, g_num: float = 0.05,
                  eb: float = 0.05, mode: str = "kinematic", steps: int = 2000,
                  real_bytes: int = 8) -> Dict[str, Any]:
    """Circular capsule centred in a wall-driven shear flow (Sec. 3.1 analogue).

    Walls at y = 0 and y = ny-1 move at -u_wall and +u_wall; x is periodic; the
    fluid starts from the linear profile.  Stiffness from the G form with
    gamma = 2 u_wall / H and d = 2R; k_b = E_b k_s R^2; density ratio 1."""
    H = ny - 1
    gamma = 2.0 * u_wall / H
    ks = ks_from_g(tau, gamma, 2.0 * radius, g_num)
    kb = eb * ks * radius * radius
    cx, cy = 0.5 * (nx - 1), 0.5 * H
    caps = [capsule(circle_nodes(cx, cy, radius, n_nodes), ks, kb, 1.0, 1.0)]
    return _base("shear64", nx, ny, tau, real_bytes, mode, steps,
                 u_bottom=-u_wall, u_top=u_wall, init_profile=INIT_COUETTE, capsules=caps)


def poiseuille_biconcave(ca: float, nx: int = 1024, ny: int = 256, tau: float = 0.8,
                         u_max: float = 0.02, length: float = 40.0, n_nodes: int = 128,
                         centre=(256.0, None), steps: int = 20000, mode: str = "dynamic",
                         real_bytes: int = 4) -> Dict[str, Any]:
    """Biconcave capsule in a body-force-driven periodic channel (Sec. 3.3 analogue).

    Centre height 6.5/15 of the channel (the paper's lowest start, Sec. 3.2);
    fluid starts from the analytic parabola; E_b = 0, k_a = 1, density ratio 1."""
    H = ny - 1
    g = poiseuille_body_force(tau, ny, u_max)
    cx = centre[0]
    cy = centre[1] if centre[1] is not None else 6.5 / 15.0 * H
    ks = ks_from_ca(tau, u_max, ca)
    caps = [capsule(biconcave_nodes(cx, cy, length, n_nodes), ks, 0.0, 1.0, 1.0)]
    return _base(f"poiseuille_biconcave_ca{ca:g}", nx, ny, tau, real_bytes, mode, steps,
                 body_force_x=g, init_profile=INIT_POISEUILLE, capsules=caps)


def stability_ratio(ks: float, mass: float, n_nodes: int) -> float:
    """Gershgorin bound on half the largest spring-network eigenvalue over the
    nodal mass, 2 k_s / m_v: the explicit node update needs it below 2."""
    return 2.0 * ks / (mass / n_nodes)


def inertial_capsules(seed: int = 0, nx: int = 2048, ny: int = 512, n_caps: int = 32,
                      tau: float = 0.8, u_max: float = 0.02, steps: int = 50000,
                      screen_limit: float = 1.5, real_bytes: int = 4,
                      mode: str = "dynamic", max_tries: int = 200000) -> Dict[str, Any]:
    """32 circular or biconcave capsules in a periodic channel.

    Draw order per capsule, from default_rng(seed): shape (biconcave if
    u < 0.5), node count U{96..160}, radius U[6, 12] (biconcave half-length),
    orientation U[0, 2 pi), density ratio U[1, 2], log10 Ca U[-3, -1], centre x
    U[0, nx), centre y U[R + 4, H - R - 4].  A draw is rejected (and drawn
    again) if its bounding circle comes within 3 lu of an earlier capsule, or if
    its stability ratio 2 k_s / m_v exceeds ``screen_limit``."""
    rng = np.random.default_rng(seed)
    H = ny - 1
    g = poiseuille_body_force(tau, ny, u_max)
    caps: List[Dict[str, Any]] = []
    placed: List[tuple] = []
    tries = 0
    while len(caps) < n_caps:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place all capsules")
        biconcave = rng.uniform() < 0.5
        n = int(rng.integers(96, 161))
        R = float(rng.uniform(6.0, 12.0))
        angle = float(rng.uniform(0.0, 2.0 * math.pi))
        ratio = float(rng.uniform(1.0, 2.0))
        ca = float(10.0 ** rng.uniform(-3.0, -1.0))
        cx = float(rng.uniform(0.0, nx))
        cy = float(rng.uniform(R + 4.0, H - R - 4.0))
        ok = True
        for (px, py, pr) in placed:
            dx = abs(cx - px)
            dx = min(dx, nx - dx)
            if math.hypot(dx, cy - py) < R + pr + 3.0:
                ok = False
                break
        if not ok:
            continue
        if biconcave:
            nodes = biconcave_nodes(cx, cy, 2.0 * R, n, angle)
        else:
            nodes = circle_nodes(cx, cy, R, n, phase=0.5)
        ks = ks_from_ca(tau, u_max, ca)
        cap = capsule(nodes, ks, 0.0, 1.0, ratio)
        if stability_ratio(ks, cap["mass"], n) > screen_limit:
            continue
        cap.update({"shape": "biconcave" if biconcave else "circle", "radius": R, "ca": ca})
        caps.append(cap)
        placed.append((cx, cy, R))
    return _base(f"inertial{n_caps}_{nx}x{ny}", nx, ny, tau, real_bytes, mode, steps,
                 body_force_x=g, init_profile=INIT_POISEUILLE, capsules=caps)


def fused_bench(seed: int = 0, n: int = 4096, n_caps: int = 32, steps: int = 1000,
                tau: float = 0.8, u_max: float = 0.02) -> Dict[str, Any]:
    """n x n channel with the capsules of ``inertial_capsules`` (2048 x 512 draw)
    moved to the larger domain by scaling their centres (x by n/2048, y by the
    ratio of channel heights).  Shapes and constants are unchanged."""
    base = inertial_capsules(seed=seed, n_caps=n_caps, tau=tau, u_max=u_max)
    sx = n / 2048.0
    sy = (n - 1) / 511.0
    caps = []
    for cap in base["capsules"]:
        nodes = cap["nodes"]
        c = nodes.mean(axis=0)
        shift = np.array([c[0] * (sx - 1.0), c[1] * (sy - 1.0)])
        new = dict(cap)
        new["nodes"] = np.ascontiguousarray(nodes + shift)
        caps.append(new)
    g = poiseuille_body_force(tau, n, u_max)
    return _base(f"fused{n}x{n}_{n_caps}caps", n, n, tau, 4, "dynamic", steps,
                 body_force_x=g, init_profile=INIT_POISEUILLE, capsules=caps)


def grid_bench(n: int = 4096, tau: float = 0.8, u_max: float = 0.02, steps: int = 1000,
               real_bytes: int = 4) -> Dict[str, Any]:
    """n x n channel without capsules (grid-only roofline case)."""
    g = poiseuille_body_force(tau, n, u_max)
    return _base(f"grid{n}x{n}", n, n, tau, real_bytes, "dynamic", steps,
                 body_force_x=g, init_profile=INIT_POISEUILLE)


def ensemble(seed: int = 0, n_inst: int = 256, u_max: float = 0.02, screen_limit: float = 1.5,
             real_bytes: int = 4, mode: str = "dynamic", steps: int = 10000,
             nx_range=(128, 512), ny_range=(64, 128), tau_range=(0.6, 1.2),
             max_tries: int = 100000) -> List[Dict[str, Any]]:
    """Independent capsule channels for the batched ensemble.

    Draw order per lattice, from default_rng(seed): nx U{nx_range}, ny
    U{ny_range}, tau U[tau_range], capsule count U{1, 2}; then per capsule:
    shape (biconcave if u < 0.5), node count U{64..128}, radius U[5, 9]
    (biconcave half-length), orientation U[0, 2 pi), density ratio U[1, 2],
    log10 Ca U[-3, -1], centre x offset U[-4, 4] from (k + 1/2) nx / count,
    centre y U[R + 4, H - R - 4].  A capsule whose stability ratio
    2 k_s / m_v exceeds ``screen_limit`` is drawn again (all of its draws).
    Each channel is driven by the body force for peak speed u_max and starts
    from the analytic parabola; E_b = 0, k_a = 1."""
    rng = np.random.default_rng(seed)
    out: List[Dict[str, Any]] = []
    for i in range(n_inst):
        nx = int(rng.integers(nx_range[0], nx_range[1] + 1))
        ny = int(rng.integers(ny_range[0], ny_range[1] + 1))
        tau = float(rng.uniform(*tau_range))
        count = int(rng.integers(1, 3))
        H = ny - 1
        g = poiseuille_body_force(tau, ny, u_max)
        caps: List[Dict[str, Any]] = []
        tries = 0
        while len(caps) < count:
            tries += 1
            if tries > max_tries:
                raise RuntimeError(f"lattice {i}: no capsule passes the screen")
            biconcave = rng.uniform() < 0.5
            n = int(rng.integers(64, 129))
            R = float(rng.uniform(5.0, 9.0))
            angle = float(rng.uniform(0.0, 2.0 * math.pi))
            ratio = float(rng.uniform(1.0, 2.0))
            ca = float(10.0 ** rng.uniform(-3.0, -1.0))
            cx = (len(caps) + 0.5) * nx / count + float(rng.uniform(-4.0, 4.0))
            cy = float(rng.uniform(R + 4.0, H - R - 4.0))
            if biconcave:
                nodes = biconcave_nodes(cx, cy, 2.0 * R, n, angle)
            else:
                nodes = circle_nodes(cx, cy, R, n, phase=0.5)
            ks = ks_from_ca(tau, u_max, ca)
            cap = capsule(nodes, ks, 0.0, 1.0, ratio)
            if stability_ratio(ks, cap["mass"], n) > screen_limit:
                continue
            cap.update({"shape": "biconcave" if biconcave else "circle", "radius": R, "ca": ca})
            caps.append(cap)
        out.append(_base(f"ensemble{seed}_{i}_{nx}x{ny}", nx, ny, tau, real_bytes, mode, steps,
                         body_force_x=g, init_profile=INIT_POISEUILLE, capsules=caps))
    return out


def adjoint_channel(nx: int = 512, ny: int = 128, tau: float = 0.8, u_max: float = 0.02,
                    radius: float = 10.0, n_nodes: int = 96, ca: float = 1e-2,
                    steps: int = 5000) -> Dict[str, Any]:
    """Circular capsule at 0.4 H in a 512 x 128 channel (the differentiated case)."""
    H = ny - 1
    g = poiseuille_body_force(tau, ny, u_max)
    ks = ks_from_ca(tau, u_max, ca)
    caps = [capsule(circle_nodes(128.0, 0.4 * H, radius, n_nodes), ks, 0.0, 1.0, 1.0)]
    return _base("adjoint512x128", nx, ny, tau, 4, "dynamic", steps,
                 body_force_x=g, init_profile=INIT_POISEUILLE, capsules=caps)


def couette_migration(nx: int = 256, H: int = 100, tau: float = 0.8, reynolds: float = 10.0,
                      ca: float = 1e-3, eb: float = 0.0, n_nodes: int = 100,
                      start: float = 0.25, density_ratio: float = 1.0,
                      steps: int = 2000000, mode: str = "kinematic",
                      real_bytes: int = 4) -> Dict[str, Any]:
    """Circular capsule released near the bottom wall of a Couette flow (the
    Sec. 3.5 set-up): the wall at y = 0 at rest, the wall at y = H moving at
    u_max = nu Re / H, x periodic, the fluid starting from the linear profile;
    diameter 0.25 H, centroid at (nx / 2, start * H); k_s from Ca (the same
    definition as the channel cases, Sec. 2.2.1), k_b = E_b k_s R^2.

    The paper's E_b = 0.1 gives k_b = 15.6 at Ca = 1e-3, which the explicit
    node update does not survive (both couplings leave the finite range within
    100 steps); the default is E_b = 0.  The default horizon, 2e6 steps
    (t u_max / H = 200), is long enough for the capsule to reach the centreline."""
    ny = H + 1
    u_top = viscosity(tau) * reynolds / H
    R = 0.125 * H
    ks = ks_from_ca(tau, u_top, ca)
    caps = [capsule(circle_nodes(0.5 * nx, start * H, R, n_nodes), ks, eb * ks * R * R, 1.0,
                    density_ratio)]
    return _base(f"couette{nx}x{ny}", nx, ny, tau, real_bytes, mode, steps,
                 u_bottom=0.0, u_top=u_top, init_profile=INIT_COUETTE, capsules=caps)


def wall_detachment(nx: int = 128, H: int = 100, tau: float = 3.5, reynolds: float = 1e-2,
                    ca: float = 1e-3, eb: float = 0.0, n_nodes: int = 100, gap: float = 3.0,
                    horizon: float = 2.0, density_ratio: float = 1.0, mode: str = "kinematic",
                    real_bytes: int = 4) -> Dict[str, Any]:
    """Circular capsule released against the bottom wall of a plane-Poiseuille
    flow (the second Sec. 3.5 set-up): x periodic, the channel driven by the
    body force for peak speed u_max = nu Re / H (H = ny - 1) and starting from
    the analytic parabola; diameter 0.25 H, centroid at (nx / 2, R + gap), so
    that the lowest node sits ``gap`` lattice units above the wall and its MLS
    support clears the wall row; k_s from Ca (the channel definition,
    Sec. 2.2.1), k_b = E_b k_s R^2, E_b = 0 as in the Couette case.

    The paper prints neither tau nor the domain length for this case.  At
    Re = 1e-2 the run to t u_max / H = ``horizon`` takes horizon H^2 / (nu Re)
    steps, so the default tau = 3.5 (nu = 1, u_max = 1e-4) keeps the paper's
    horizon of 2 at 2e6 steps; nx = 128 leaves about four diameters between
    periodic images."""
    ny = H + 1
    nu = viscosity(tau)
    u_max = nu * reynolds / H
    R = 0.125 * H
    ks = ks_from_ca(tau, u_max, ca)
    steps = int(round(horizon * H / u_max))
    caps = [capsule(circle_nodes(0.5 * nx, R + gap, R, n_nodes), ks, eb * ks * R * R, 1.0,
                    density_ratio)]
    cfg = _base(f"detach{nx}x{ny}", nx, ny, tau, real_bytes, mode, steps,
                body_force_x=poiseuille_body_force(tau, ny, u_max), init_profile=INIT_POISEUILLE,
                capsules=caps)
    cfg["u_max"] = u_max
    return cfg


def open_channel(nx: int, ny: int, tau: float, u_max: float, real_bytes: int = 8,
                 mode: str = "dynamic", steps: int = 0, init_profile: int = INIT_REST,
                 outlet_rho: float = 1.0) -> Dict[str, Any]:
    """Open channel of Sec. 3.2: stationary walls, parabolic velocity inlet
    u_x(0, y) = 4 u_max y (H - y) / H^2 and outlet density outlet_rho; no body
    force; the flow starts at rest (or from the inlet parabola)."""
    return _base(f"open{nx}x{ny}", nx, ny, tau, real_bytes, mode, steps, periodic_x=0,
                 inlet_umax=float(u_max), outlet_rho=float(outlet_rho), init_profile=init_profile)


def multi_capsule_channel(seed: int = 0, nx: int = 1536, ny: int = 256, tau: float = 0.8,
                          u_max: float = 0.02, n_caps: int = 16, n_rigid: int = 2,
                          length: float = 30.0, ca: float = 1e-2, gap: float = 0.5,
                          real_bytes: int = 4, steps: int = 1000) -> Dict[str, Any]:
    """Open channel (velocity inlet, pressure outlet, Sec. 3.2) carrying a
    4 x 4 block of bodies a few lattice units apart, the Sec. 3.4 set-up: 16
    biconcave capsules of the given length (Ca from u_max), of which the first
    ``n_rigid`` are replaced by rigid discs of the same length; contact force
    (Eq. 27, cutoff 2).  Draws from default_rng(seed): per body, orientation
    U[-0.3, 0.3] rad and a centre jitter U[-1, 1] lu in x and y.  The flow starts
    from the inlet parabola everywhere."""
    rng = np.random.default_rng(seed)
    H = ny - 1
    ks = ks_from_ca(tau, u_max, ca)
    pitch_x = length + gap + 2.0
    pitch_y = 0.5 * length + gap + 2.0
    x0 = 0.25 * nx
    y0 = 0.5 * H - 1.5 * pitch_y
    caps: List[Dict[str, Any]] = []
    for k in range(n_caps):
        i, j = k % 4, k // 4
        angle = float(rng.uniform(-0.3, 0.3))
        jx, jy = rng.uniform(-1.0, 1.0, 2)
        cx, cy = x0 + i * pitch_x + jx, y0 + j * pitch_y + jy
        if k < n_rigid:
            caps.append(rigid_particle(circle_nodes(cx, cy, 0.25 * length, 64), 1.0))
        else:
            caps.append(capsule(biconcave_nodes(cx, cy, length, 96, angle), ks, 0.0, 1.0, 1.0))
    cfg = open_channel(nx, ny, tau, u_max, real_bytes=real_bytes, mode="dynamic", steps=steps,
                       init_profile=INIT_INLET)
    cfg["name"] = f"multi{n_caps}_{nx}x{ny}"
    cfg["capsules"] = caps
    cfg["contact_cutoff"] = 2.0
    return cfg


def dense_suspension(seed: int = 0, length: float = 30.0, gap: float = 0.5, tau: float = 0.8,
                     u_max: float = 0.02, ca: float = 1e-2, n_nodes: int = 96,
                     max_angle: float = 0.1, horizon: float = 2.0, mode: str = "kinematic",
                     real_bytes: int = 4) -> Dict[str, Any]:
    """Sixteen biconcave capsules filling a plane-Poiseuille channel at the
    paper's hematocrit of about 30 % (the Sec. 3.4 set-up, at a capsule length
    the IB kernel's on-chip patch holds): a 4 x 4 block at pitches
    (L + gap + 2, L/2 + gap + 2) that tiles the periodic x direction, with
    five lattice units between the block and each wall; body-force channel
    starting from the parabola (as the other channel cases); Ca from u_max,
    E_b = 0, k_a = 1, density ratio 1; contact force (Eq. 27, cutoff 2).
    Draws from default_rng(seed): per capsule, orientation U[-max_angle,
    max_angle] rad and a centre jitter U[-1, 1] lu in x and y.  The horizon
    is t u_max / H (Fig. 5 shows the fields at 2)."""
    rng = np.random.default_rng(seed)
    pitch_x = length + gap + 2.0
    pitch_y = 0.5 * length + gap + 2.0
    nx = int(round(4 * pitch_x))
    H = int(math.ceil(4 * pitch_y + 10.0))
    ny = H + 1
    ks = ks_from_ca(tau, u_max, ca)
    caps: List[Dict[str, Any]] = []
    for k in range(16):
        i, j = k % 4, k // 4
        angle = float(rng.uniform(-max_angle, max_angle))
        jx, jy = rng.uniform(-1.0, 1.0, 2)
        cx = (i + 0.5) * nx / 4.0 + jx
        cy = 0.5 * H + (j - 1.5) * pitch_y + jy
        caps.append(capsule(biconcave_nodes(cx, cy, length, n_nodes, angle), ks, 0.0, 1.0, 1.0))
    steps = int(round(horizon * H / u_max))
    cfg = _base(f"dense16_{nx}x{ny}", nx, ny, tau, real_bytes, mode, steps,
                body_force_x=poiseuille_body_force(tau, ny, u_max), init_profile=INIT_POISEUILLE,
                capsules=caps)
    cfg["contact_cutoff"] = 2.0
    cfg["u_max"] = u_max
    cfg["hematocrit"] = sum(polygon_area(c["nodes"]) for c in caps) / float(nx * H)
    return cfg


def periodic_box(nx: int, ny: int, tau: float, u0=(0.0, 0.0), real_bytes: int = 8,
                 mode: str = "dynamic", steps: int = 10) -> Dict[str, Any]:
    """Fully periodic box at uniform velocity u0 (no walls, no body force)."""
    return _base(f"box{nx}x{ny}", nx, ny, tau, real_bytes, mode, steps, periodic_y=1,
                 init_profile=INIT_UNIFORM, init_u=tuple(float(v) for v in u0))


def random_populations(nx: int, ny: int, seed: int, amp: float = 0.02) -> np.ndarray:
    """Seeded non-equilibrium population field, layout [9][ny][nx] FP64.

    Each population is a typical magnitude (4/9 rest, 1/9 axis, 1/36 diagonal)
    times (1 + amp * N(0, 1)): positive, of realistic size, and far from any
    equilibrium, so every term of a collision is exercised."""
    rng = np.random.default_rng(seed)
    mag = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    return mag[:, None, None] * (1.0 + amp * rng.standard_normal((9, ny, nx)))
