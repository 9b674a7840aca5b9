"""Shared helpers of the GPU parity tests: build the HIP simulation and the FP64
oracle from one workload dictionary and compare their states."""
from __future__ import annotations

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
