"""Parity over the full horizons of the channel workloads: the HIP library in
FP32 (and in FP64) against the FP64 oracle's state after the whole run.

The oracle runs take minutes to an hour on the CPU, so their sampled state is
stored under tests/golden/ by make_long_runs.py, which calls only the oracle
and the seeded input generators.  The GPU side rebuilds the same workload from
the same generator and steps it through the C-ABI.

Bars (after the run):
- velocity: relative L2 error <= 1e-5, over the 256 sampled cells (both
  components) and over the row means of u_x (the channel profile);
- Taylor deformation D of every capsule: |D_gpu - D_oracle| <= 1e-4;
- nodes: within 1e-5 u_max T of the oracle's (T steps at peak speed u_max:
  the displacement a 1e-5 relative velocity error accumulates), 4e-3 lattice
  units over 20000 steps;
- density at the sampled cells: within 1e-5.
An FP64 run takes 1e-3 of each bar.

The printed Dynamic coupling does not stay finite over these horizons (its
membrane zigzag mode grows; the oracle shows the same), so the runs use the
Kinematic coupling of Eq. 25 over the same lattice, MLS and membrane path."""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

from paper_1903_03356_amd import lbib
from paper_1903_03356_amd import workloads as wl
from tests.parity import log

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
U_MAX = 0.02


def golden(name: str):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not generated (tests/golden/make_long_runs.py)")
    with open(path) as f:
        return json.load(f)


def compare_snapshot(sim, lattice: int, cap_ids, ref, steps: int, tag: str, u_max: float = U_MAX,
                     scale: float = 1.0):
    """Checks one lattice of ``sim`` against an oracle snapshot; returns the errors.
    ``scale`` multiplies every bar (below 1 for an FP64 run)."""
    m = sim.moments(lattice)
    cells = np.asarray(ref["cells"])
    got = m[:, cells[:, 1], cells[:, 0]].T
    want = np.asarray(ref["moments"])
    du = got[:, 1:] - want[:, 1:]
    e_u = float(np.sqrt((du ** 2).sum() / (want[:, 1:] ** 2).sum()))
    e_rho = float(np.abs(got[:, 0] - want[:, 0]).max())
    prof = m[1].mean(axis=1)
    pw = np.asarray(ref["ux_row_mean"])
    e_prof = float(np.sqrt(((prof - pw) ** 2).sum() / (pw ** 2).sum()))
    e_x, e_d = 0.0, 0.0
    assert len(cap_ids) == len(ref["capsules"])
    for c, rc in zip(cap_ids, ref["capsules"]):
        x = sim.capsule(c)[0]
        e_x = max(e_x, float(np.abs(x - np.asarray(rc["nodes"])).max()))
        e_d = max(e_d, abs(sim.diag(c)["D"] - rc["diag"]["D"]))
    out = {"u_l2_rel": e_u, "profile_rel": e_prof, "rho_max_abs": e_rho, "x_max_abs": e_x,
           "D_max_abs": e_d}
    log(f"{tag}: " + ", ".join(f"{k} {v:.2e}" for k, v in out.items()))
    assert e_u <= 1e-5 * scale, (tag, out)
    assert e_prof <= 1e-5 * scale, (tag, out)
    assert e_rho <= 1e-5 * scale, (tag, out)
    assert e_d <= 1e-4 * scale, (tag, out)
    assert e_x <= 1e-5 * u_max * steps * scale, (tag, out)
    return out


def bar_scale(real_bytes: int) -> float:
    """FP32 runs take the bars above; FP64 runs 1e-3 of them (the oracle's
    arithmetic in another order, against values stored to ten digits)."""
    return 1.0 if real_bytes == 4 else 1e-3


@pytest.mark.gpu
@pytest.mark.parametrize("real_bytes", [4, 8])
@pytest.mark.parametrize("ca", [1e-3, 1e-2, 1e-1])
def test_channel_full_horizon(ca, real_bytes):
    """1024 x 256 biconcave channel, all 20000 steps."""
    ref = golden(f"long_channel_ca{ca:g}.json")
    cfg = wl.poiseuille_biconcave(ca, mode="kinematic", real_bytes=real_bytes)
    steps = ref["steps"]
    assert steps == cfg["steps"] == 20000
    sim = lbib.Sim(cfg)
    sim.step(steps, "kinematic")
    assert sim.check() == 0
    compare_snapshot(sim, 0, [0], ref, steps, f"channel Ca {ca:g} ({8 * real_bytes} bit), {steps} steps",
                     scale=bar_scale(real_bytes))


@pytest.mark.gpu
@pytest.mark.parametrize("real_bytes", [4, 8])
def test_ensemble_full_horizon(real_bytes):
    """The 256-lattice ensemble in one batched context, all 10000 steps;
    8 seeded lattices against the oracle."""
    ref = golden("long_ensemble.json")
    cfgs = wl.ensemble(seed=0, mode="kinematic", real_bytes=real_bytes)
    steps = ref["steps"]
    assert steps == cfgs[0]["steps"] == 10000
    bat = lbib.Batch(cfgs)
    bat.step(steps, "kinematic")
    assert bat.check() == 0
    for r in ref["lattices"]:
        i = r["lattice"]
        compare_snapshot(bat, i, bat.cap_ids[i], r, steps, f"ensemble lattice {i} ({8 * real_bytes} bit)",
                         scale=bar_scale(real_bytes))


@pytest.mark.gpu
@pytest.mark.parametrize("real_bytes", [4, 8])
def test_inertial_channel_horizon(real_bytes):
    """2048 x 512 channel with 32 capsules, over the stored horizon."""
    ref = golden("long_inertial.json")
    cfg = wl.inertial_capsules(seed=0, mode="kinematic", real_bytes=real_bytes)
    steps = ref["steps"]
    sim = lbib.Sim(cfg)
    sim.step(steps, "kinematic")
    assert sim.check() == 0
    compare_snapshot(sim, 0, list(range(len(cfg["capsules"]))), ref, steps,
                     f"inertial 2048x512 ({8 * real_bytes} bit), {steps} steps",
                     scale=bar_scale(real_bytes))


@pytest.mark.gpu
def test_adjoint_full_horizon():
    """The 512 x 128 gradient channel over all 5000 steps: the FP32 gradient
    with a checkpoint every 70 steps against the oracle's central differences,
    for D and y_c, k_s of two elements and the body force g.

    The stored differences use three step sizes each, large enough to average
    over the small jumps of the discrete map at the nodes' MLS stencil switches
    (thousands over 5000 steps; a step of 1e-6 g straddles a few and scatters
    by 25 %).  The bar is 1e-3 of the largest difference of that objective and
    parameter kind, plus the scatter of the three differences (max - min), which
    measures how far the difference itself is settled: about 1e-3 for D, about
    0.5 % for y_c, whose stencil jumps are larger relative to its slope."""
    ref = golden("long_adjoint.json")
    cfg = dict(wl.adjoint_channel(), mode="kinematic")
    steps = ref["steps"]
    for obj, key, jkey in ((lbib.OBJ_TAYLOR, "dD", "D"), (lbib.OBJ_CENTROID_Y, "dyc", "yc")):
        r = lbib.Sim(cfg).adjoint(steps, obj, 0, "kinematic", checkpoint_every=70)
        assert abs(r["J"] - ref[jkey]) <= 1e-4 * max(1.0, abs(ref[jkey]))
        by = {}
        for e in ref["fd"]:
            by.setdefault(e["param"], []).append(e[key])
        ks_scale = max(max(abs(v) for v in vals) for p, vals in by.items() if p != "g")
        for p, vals in by.items():
            assert len(vals) == 3
            got = r["dJ_dg"] if p == "g" else float(r["dJ_dks"][0][int(p[2:])])
            fd = vals[1]
            spread = max(vals) - min(vals)
            scale = max(abs(v) for v in vals) if p == "g" else ks_scale
            bar = 1e-3 * scale + spread
            log(f"adjoint {jkey} {p}: fp32 {got:.9g} fd {fd:.9g} (h scatter {spread:.2e}), "
                f"bar {bar:.2e}")
            assert abs(got - fd) <= bar, (jkey, p, got, vals, bar)


@pytest.mark.gpu
@pytest.mark.parametrize("real_bytes", [4, 8])
def test_couette_migration_full_horizon(real_bytes):
    """The Sec. 3.5 Couette case (256 x 101, capsule released at 0.25 H,
    density ratio 1), all 2e6 steps: the centroid and the deformation along
    the whole migration, and the sampled state at the end.  FP32 to the bars
    of this file; FP64 to 1e-3 of them (the same arithmetic as the oracle in
    another order; the stored values keep ten significant digits)."""
    ref = golden("long_couette.json")
    cfg = wl.couette_migration(real_bytes=real_bytes)
    scale = bar_scale(real_bytes)
    steps = ref["steps"]
    assert steps == cfg["steps"] == ref["trajectory"][-1]["steps"]
    u_top = cfg["u_top"]
    sim = lbib.Sim(cfg)
    worst = {"c": 0.0, "D": 0.0}
    done = 0
    for r in ref["trajectory"]:
        sim.step(r["steps"] - done, "kinematic")
        done = r["steps"]
        d = sim.diag(0)
        e_c = max(abs(d["cx"] - r["cx"]), abs(d["cy"] - r["cy"]))
        e_d = abs(d["D"] - r["D"])
        worst = {"c": max(worst["c"], e_c), "D": max(worst["D"], e_d)}
        assert e_c <= 1e-5 * u_top * r["steps"] * scale, (r["steps"], d["cx"], d["cy"], r)
        assert e_d <= 1e-4 * scale, (r["steps"], d["D"], r["D"])
    log(f"couette trajectory ({8 * real_bytes} bit): centroid {worst['c']:.2e}, D {worst['D']:.2e}, "
        f"final y_c {sim.diag(0)['cy']:.4f} (oracle {ref['trajectory'][-1]['cy']:.4f})")
    assert sim.check() == 0
    compare_snapshot(sim, 0, [0], ref, steps, f"couette 256x101 ({8 * real_bytes} bit), {steps} steps",
                     u_max=u_top, scale=scale)


def test_couette_migration_reaches_centreline():
    """Sec. 3.5: a capsule released at 0.25 H in Couette flow settles at 0.5 H,
    and it takes its deformed shape at once and keeps it while it migrates.
    Checked on the oracle's stored trajectory (density ratio 1, the case the
    Kinematic coupling covers): the centroid rises monotonically and ends
    within 0.01 H of the centreline; at every sample (every 50,000 steps,
    from the first on) D and the perimeter are within 10 % and 1 % of their
    final values (host only)."""
    ref = golden("long_couette.json")
    H = ref["H"]
    tr = ref["trajectory"]
    ys = [r["cy"] for r in tr]
    assert all(b >= a for a, b in zip(ys, ys[1:])), ys
    assert abs(ys[-1] - 0.5 * H) <= 0.01 * H, ys[-1]
    assert ys[0] < 0.3 * H, ys[0]
    d_end, p_end = tr[-1]["D"], tr[-1]["perimeter"]
    assert d_end > 0.01, d_end
    for r in tr:
        assert abs(r["D"] - d_end) <= 0.1 * d_end, r
        assert abs(r["perimeter"] - p_end) <= 0.01 * p_end, r


def detach_config(ref, real_bytes: int):
    """The wall-detachment workload at the horizon the stored run covers."""
    return wl.wall_detachment(real_bytes=real_bytes, horizon=ref["workload"]["horizon"])


@pytest.mark.gpu
@pytest.mark.parametrize("real_bytes", [4, 8])
def test_wall_detachment_full_horizon(real_bytes):
    """The Sec. 3.5 wall-detachment case (128 x 101 Poiseuille channel at
    Re = 1e-2, capsule released against the bottom wall, density ratio 1) over
    the stored run: centroid, deformation and perimeter change at every stored
    interval, and the sampled state at the end.  FP32 to the bars of this
    file; FP64 to 1e-3 of them."""
    ref = golden("long_detach.json")
    cfg = detach_config(ref, real_bytes)
    scale = bar_scale(real_bytes)
    steps = ref["steps"]
    assert steps == cfg["steps"] == ref["trajectory"][-1]["steps"]
    u_max = cfg["u_max"]
    sim = lbib.Sim(cfg)
    worst = {"c": 0.0, "D": 0.0, "dp": 0.0}
    done = 0
    for r in ref["trajectory"]:
        sim.step(r["steps"] - done, "kinematic")
        done = r["steps"]
        d = sim.diag(0)
        e_c = max(abs(d["cx"] - r["cx"]), abs(d["cy"] - r["cy"]))
        e_d = abs(d["D"] - r["D"])
        e_p = abs(d["dp"] - r["dp"])
        worst = {"c": max(worst["c"], e_c), "D": max(worst["D"], e_d), "dp": max(worst["dp"], e_p)}
        assert e_c <= 1e-5 * u_max * r["steps"] * scale, (r["steps"], d["cx"], d["cy"], r)
        assert e_d <= 1e-4 * scale, (r["steps"], d["D"], r["D"])
        assert e_p <= 1e-4 * scale, (r["steps"], d["dp"], r["dp"])
    log(f"detach trajectory ({8 * real_bytes} bit): centroid {worst['c']:.2e}, D {worst['D']:.2e}, "
        f"dp {worst['dp']:.2e}, final y_c {sim.diag(0)['cy']:.6f} "
        f"(oracle {ref['trajectory'][-1]['cy']:.6f})")
    assert sim.check() == 0
    compare_snapshot(sim, 0, [0], ref, steps, f"detach 128x101 ({8 * real_bytes} bit), {steps} steps",
                     u_max=u_max, scale=scale)


def test_wall_detachment_leaves_the_wall():
    """Sec. 3.5, the capsule released against the wall of a Poiseuille flow at
    density ratio 1 (the case the Kinematic coupling covers), checked on the
    oracle's stored run (host only):
    - it detaches: the centroid's height above the wall rises at every stored
      interval;
    - it lags the flow: over every interval its mean x-velocity is below the
      undisturbed parabola 4 u_max y (H - y) / H^2 at the interval's lowest
      centroid height (a body near a wall, and in a curved profile, trails the
      fluid at its centre);
    - it travels deformed: at every stored interval D > 0.05, the perimeter
      change dp > 0 and the swelling ratio Sw < 1;
    - its deformation follows the shear it meets: the shear rate of the
      parabola falls with the height above the wall, and once past its
      largest value D does not grow again (within 1e-4) while the capsule
      rises."""
    ref = golden("long_detach.json")
    H, u_max = ref["H"], ref["u_max"]
    tr = ref["trajectory"]
    cfg = detach_config(ref, 8)
    x0 = cfg["capsules"][0]["nodes"]
    start = {"steps": 0, "cx": float(np.mean(x0[:, 0])), "cy": float(np.mean(x0[:, 1]))}
    pts = [start] + tr
    ys = [p["cy"] for p in pts]
    assert all(b > a for a, b in zip(ys, ys[1:])), ys
    for a, b in zip(pts, pts[1:]):
        dx = b["cx"] - a["cx"]
        if dx < -0.5 * cfg["nx"]:
            dx += cfg["nx"]
        v = dx / (b["steps"] - a["steps"])
        y = min(a["cy"], b["cy"])
        u_ref = 4.0 * u_max * y * (H - y) / H ** 2
        assert 0.0 < v < u_ref, (b["steps"], v, u_ref)
    assert all(r["D"] > 0.05 and r["dp"] > 0.0 and r["Sw"] < 1.0 for r in tr), tr
    ds = [r["D"] for r in tr]
    peak = ds.index(max(ds))
    assert all(b <= a + 1e-4 for a, b in zip(ds[peak:], ds[peak + 1:])), ds


@pytest.mark.gpu
@pytest.mark.parametrize("real_bytes", [4, 8])
def test_dense_suspension_full_horizon(real_bytes):
    """The Sec. 3.4 dense suspension (130 x 81 channel, 16 biconcave capsules
    at about 30 % hematocrit, contact force on) over t u_max / H = 2 (8000
    steps): every capsule's centroid, D and perimeter change at each quarter
    of the run, and the sampled state with all 16 capsules at the end.  FP32
    to the bars of this file; FP64 to 1e-3 of them."""
    ref = golden("long_dense.json")
    cfg = wl.dense_suspension(real_bytes=real_bytes)
    scale = bar_scale(real_bytes)
    steps = ref["steps"]
    assert steps == cfg["steps"] == ref["trajectory"][-1]["steps"]
    u_max = cfg["u_max"]
    sim = lbib.Sim(cfg)
    worst = {"c": 0.0, "D": 0.0, "dp": 0.0}
    done = 0
    for r in ref["trajectory"]:
        sim.step(r["steps"] - done, "kinematic")
        done = r["steps"]
        for c, rd in enumerate(r["diag"]):
            d = sim.diag(c)
            e_c = max(abs(d["cx"] - rd["cx"]), abs(d["cy"] - rd["cy"]))
            worst = {"c": max(worst["c"], e_c), "D": max(worst["D"], abs(d["D"] - rd["D"])),
                     "dp": max(worst["dp"], abs(d["dp"] - rd["dp"]))}
            assert e_c <= 1e-5 * u_max * r["steps"] * scale, (r["steps"], c, d, rd)
            assert abs(d["D"] - rd["D"]) <= 1e-4 * scale, (r["steps"], c, d["D"], rd["D"])
            assert abs(d["dp"] - rd["dp"]) <= 1e-4 * scale, (r["steps"], c, d["dp"], rd["dp"])
    log(f"dense suspension ({8 * real_bytes} bit): centroid {worst['c']:.2e}, D {worst['D']:.2e}, "
        f"dp {worst['dp']:.2e}")
    assert sim.check() == 0
    compare_snapshot(sim, 0, list(range(16)), ref, steps,
                     f"dense 130x81 ({8 * real_bytes} bit), {steps} steps", u_max=u_max, scale=scale)


def test_golden_samples_follow_their_seed():
    """The stored sample cells are the ones the generator's seed draws on each
    workload's lattice, the ensemble lattices the ones its pick seed draws, and
    every stored value is finite (host only)."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_long_runs",
                                                  os.path.join(GOLDEN, "make_long_runs.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    dims = {"poiseuille_biconcave": (1024, 256), "inertial_capsules": (2048, 512),
            "couette_migration": (256, 101), "wall_detachment": (128, 101),
            "dense_suspension": (130, 81)}
    found = 0
    for name in sorted(os.listdir(GOLDEN)):
        if not (name.startswith("long_") and name.endswith(".json")):
            continue
        with open(os.path.join(GOLDEN, name)) as f:
            ref = json.load(f)
        fn = ref["workload"]["fn"]
        if fn == "adjoint_channel":
            assert {e["param"] for e in ref["fd"]} == {"g"} | {f"ks{l}" for l in mk.ADJ_ELEMENTS}
            assert all(np.isfinite([e["dD"], e["dyc"]]).all() for e in ref["fd"])
            found += 1
            continue
        if fn == "ensemble":
            cfgs = wl.ensemble(seed=0, mode="kinematic")
            assert [r["lattice"] for r in ref["lattices"]] == mk.ensemble_pick(len(cfgs))
            snaps = [(r, (cfgs[r["lattice"]]["nx"], cfgs[r["lattice"]]["ny"]))
                     for r in ref["lattices"]]
        else:
            snaps = [(ref, dims[fn])]
        for s, (nx, ny) in snaps:
            assert np.array_equal(np.asarray(s["cells"]), mk.sample_cells(nx, ny)), name
            assert len(s["moments"]) == mk.N_SAMPLE and len(s["ux_row_mean"]) == ny
            assert s["status"] == 0
            assert np.isfinite(np.asarray(s["moments"])).all()
            assert all(np.isfinite(c["diag"]["D"]) for c in s["capsules"])
        found += 1
    if found == 0:
        pytest.skip("no long-run fixtures generated")
