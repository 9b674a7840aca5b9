"""The seeded synthetic inputs are reproducible and keep the figures quoted
with the measurements (seed 0): the ensemble's cell and capsule counts, the
4096^2 workload's node count, and the stability screen of the drawn capsules."""
import numpy as np

from paper_1903_03356_amd import workloads as wl


def test_ensemble_seed0_figures():
    cfgs = wl.ensemble(seed=0)
    assert len(cfgs) == 256
    assert sum(c["nx"] * c["ny"] for c in cfgs) == 8005365
    assert sum(len(c["capsules"]) for c in cfgs) == 388
    for c in cfgs:
        assert 128 <= c["nx"] <= 512 and 64 <= c["ny"] <= 128
        for cap in c["capsules"]:
            assert wl.stability_ratio(cap["ks"], cap["mass"], len(cap["nodes"])) <= 1.5


def test_fused_workload_figures():
    cfg = wl.fused_bench(seed=0, n=4096)
    assert (cfg["nx"], cfg["ny"], len(cfg["capsules"])) == (4096, 4096, 32)
    assert sum(len(c["nodes"]) for c in cfg["capsules"]) == 4177
    assert cfg["real_bytes"] == 4 and cfg["mode"] == "dynamic"


def test_inputs_are_reproducible():
    a, b = wl.inertial_capsules(seed=3), wl.inertial_capsules(seed=3)
    for ca, cb in zip(a["capsules"], b["capsules"]):
        assert np.array_equal(ca["nodes"], cb["nodes"]) and ca["ks"] == cb["ks"]
    c = wl.inertial_capsules(seed=4)
    assert not np.array_equal(a["capsules"][0]["nodes"], c["capsules"][0]["nodes"])
    for cap in a["capsules"]:
        assert wl.stability_ratio(cap["ks"], cap["mass"], len(cap["nodes"])) <= 1.5


def test_couette_migration_figures():
    """Sec. 3.5 set-up: H = 100, Re = 10 at tau = 0.8 gives a top-wall speed of
    0.01; d = 0.25 H released at 0.25 H; Ca = 1e-3 gives k_s = 1."""
    cfg = wl.couette_migration()
    assert (cfg["nx"], cfg["ny"]) == (256, 101)
    assert cfg["u_bottom"] == 0.0 and abs(cfg["u_top"] - 0.01) < 1e-15
    assert cfg["init_profile"] == wl.INIT_COUETTE and cfg["mode"] == "kinematic"
    cap = cfg["capsules"][0]
    nodes = cap["nodes"]
    np.testing.assert_allclose(nodes.mean(axis=0), (128.0, 25.0), atol=1e-12)
    np.testing.assert_allclose(np.hypot(*(nodes - (128.0, 25.0)).T), 12.5, atol=1e-12)
    assert abs(cap["ks"] - 1.0) < 1e-12 and cap["kb"] == 0.0 and len(nodes) == 100
    assert abs(wl.couette_migration(eb=0.1)["capsules"][0]["kb"] - 15.625) < 1e-9


def test_wall_detachment_figures():
    """Sec. 3.5 detachment set-up: H = 100 and Re = 1e-2 at tau = 3.5 (nu = 1)
    give u_max = 1e-4, body force 8 nu u_max / H^2 = 8e-8 and 2e6 steps to
    t u_max / H = 2; d = 0.25 H with its lowest node 3 lattice units above
    the wall; Ca = 1e-3 gives k_s = 0.1."""
    cfg = wl.wall_detachment()
    assert (cfg["nx"], cfg["ny"]) == (128, 101)
    assert abs(cfg["u_max"] - 1e-4) < 1e-18 and abs(cfg["body_force_x"] - 8e-8) < 1e-20
    assert cfg["steps"] == 2000000 and wl.wall_detachment(horizon=0.25)["steps"] == 250000
    assert cfg["init_profile"] == wl.INIT_POISEUILLE and cfg["mode"] == "kinematic"
    assert cfg["u_bottom"] == cfg["u_top"] == 0.0
    cap = cfg["capsules"][0]
    nodes = cap["nodes"]
    np.testing.assert_allclose(nodes.mean(axis=0), (64.0, 15.5), atol=1e-12)
    np.testing.assert_allclose(np.hypot(*(nodes - (64.0, 15.5)).T), 12.5, atol=1e-12)
    assert nodes[:, 1].min() >= 3.0
    assert abs(cap["ks"] - 0.1) < 1e-12 and cap["kb"] == 0.0 and len(nodes) == 100


def test_dense_suspension_figures():
    """Sec. 3.4 set-up at about 30 % hematocrit: 16 biconcave capsules of
    length 30 fill a 130 x 81 channel (capsule area over channel area between
    0.29 and 0.32); every node keeps 3 lattice units off the walls; capsules
    of neighbouring rows and columns (x periodic) start within the contact
    cutoff of one another but do not overlap; the horizon t u_max / H = 2 is
    8000 steps; the draw repeats for a seed and changes with it."""
    cfg = wl.dense_suspension()
    assert (cfg["nx"], cfg["ny"]) == (130, 81) and cfg["steps"] == 8000
    assert 0.29 <= cfg["hematocrit"] <= 0.32, cfg["hematocrit"]
    assert cfg["contact_cutoff"] == 2.0 and cfg["init_profile"] == wl.INIT_POISEUILLE
    caps = [c["nodes"] for c in cfg["capsules"]]
    assert len(caps) == 16
    ys = np.concatenate([c[:, 1] for c in caps])
    assert ys.min() >= 3.0 and ys.max() <= cfg["ny"] - 4
    dmin = np.inf
    for a in range(16):
        for b in range(a + 1, 16):
            for sh in (-cfg["nx"], 0, cfg["nx"]):
                d = caps[a][:, None, :] - (caps[b][None, :, :] + [sh, 0.0])
                dmin = min(dmin, float(np.hypot(d[..., 0], d[..., 1]).min()))
    assert 0.5 < dmin < cfg["contact_cutoff"], dmin
    again = wl.dense_suspension()
    assert all(np.array_equal(a["nodes"], b["nodes"]) for a, b in zip(cfg["capsules"], again["capsules"]))
    other = wl.dense_suspension(seed=1)
    assert not np.array_equal(cfg["capsules"][0]["nodes"], other["capsules"][0]["nodes"])
