"""Shared helpers of the GPU parity tests: build the HIP simulation and the FP64
oracle from one workload dictionary and compare their states."""
from __future__ import annotations

import math
import os
import sys

import numpy as np

W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def oracle_threads(orc) -> None:
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    orc.set_threads(max(1, min(16, n)))


def pair(cfg):
    """(HIP simulation, oracle simulation) built from the same inputs."""
    from oracle import oracle as orc
    from paper_1903_03356_amd import lbib
    oracle_threads(orc)
    return lbib.Sim(cfg), orc.Sim(cfg)


def vel_l2_rel(mg, mo) -> float:
    """||u_gpu - u_oracle||_2 / ||u_oracle||_2 over all cells (both components)."""
    num = np.sqrt(np.sum((mg[1:] - mo[1:]) ** 2))
    den = np.sqrt(np.sum(mo[1:] ** 2))
    return float(num / den) if den > 0 else float(num)


def compare_fields(g, o, vel_tol, rho_tol, pop_tol=None):
    mg, mo = g.moments(), o.moments()
    err_u = vel_l2_rel(mg, mo)
    err_rho = float(np.abs(mg[0] - mo[0]).max())
    out = {"u_l2_rel": err_u, "rho_max_abs": err_rho}
    if pop_tol is not None:
        dg = g.pops_dev()
        do = o.pops() - W[:, None, None]
        out["pop_dev_max_abs"] = float(np.abs(dg - do).max())
        assert out["pop_dev_max_abs"] <= pop_tol, out
    assert err_u <= vel_tol, out
    assert err_rho <= rho_tol, out
    return out


def compare_capsules(g, o, pos_tol, d_tol):
    errs = []
    for c in range(len(g.nv)):
        xg, pg, ug = g.capsule(c)
        xo, po, uo = o.capsule(c)
        dg, do = g.diag(c), o.diag(c)
        e = {"cap": c, "x_max_abs": float(np.abs(xg - xo).max()),
             "xprev_max_abs": float(np.abs(pg - po).max()),
             "dD": abs(dg["D"] - do["D"]), "dSw": abs(dg["Sw"] - do["Sw"]),
             "ddp": abs(dg["dp"] - do["dp"]), "dA": abs(dg["area"] - do["area"]) / do["area"]}
        errs.append(e)
        assert e["x_max_abs"] <= pos_tol and e["xprev_max_abs"] <= pos_tol, e
        assert e["dD"] <= d_tol and e["dSw"] <= d_tol and e["ddp"] <= d_tol, e
    return errs


def regular_polygon_force(N, R, R0, ks, ka):
    """Radial (outward) internal force per node of a regular N-gon of radius R
    with stress-free radius R0, from the membrane energy: stretch
    sum 1/2 k_s (l - l0)^2 (Eq. 10) and area k_a p_ref (A - A0)^2 / (2 A0) with
    p_ref = 1/3 (Eq. 12).  By symmetry each node carries -dE/dR / N."""
    s1, s2 = math.sin(math.pi / N), math.sin(2.0 * math.pi / N)
    l, l0 = 2.0 * R * s1, 2.0 * R0 * s1
    A, A0 = 0.5 * N * R * R * s2, 0.5 * N * R0 * R0 * s2
    dE_dR = N * ks * (l - l0) * 2.0 * s1 + ka / 3.0 * (A - A0) / A0 * N * R * s2
    return -dE_dR / N, A0


def uneven_polygon(cx, cy, a, b, n, seed):
    """Counter-clockwise nodes on an ellipse at unevenly spaced angles (seeded
    jitter of a third of the mean spacing)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    ang = 2.0 * math.pi * (np.arange(n) + 0.5 + rng.uniform(-1 / 3, 1 / 3, n)) / n
    return np.stack([cx + a * np.cos(ang), cy + b * np.sin(ang)], axis=1)


def edge_line_integrals(x):
    """Perimeter P and the line integral of the position, sum over the
    straight edges of length * midpoint (exact for a polygon)."""
    import numpy as np
    y = np.roll(x, -1, axis=0)
    l = np.hypot(*(y - x).T)
    return l.sum(), (l[:, None] * 0.5 * (x + y)).sum(axis=0)
