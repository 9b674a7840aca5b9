"""Captured step blocks (lbib_set_graph) against direct launches.

A replayed block runs the very kernel launches of the direct path, so every
case must give the same bits: populations, force field, node state and rigid
state, over calls of uneven length whose blocks start on even and on odd
steps, with contact on (the Dynamic and the split Kinematic launch order), in
a batch context and with rigid particles; and again after a change of the
contact cutoff, which must re-capture."""
import numpy as np
import pytest

from paper_1903_03356_amd import workloads as wl
from tests.parity import log

pytestmark = pytest.mark.gpu


def _contact_pair(mode):
    cfg = wl._base("contact", 64, 48, 0.9, 4, mode, 0, u_bottom=-0.005, u_top=0.005,
                   init_profile=wl.INIT_COUETTE)
    cfg["capsules"] = [wl.capsule(wl.circle_nodes(24.0, 23.0, 6.0, 48), 0.02, 0.0, 1.0, 1.0),
                       wl.capsule(wl.circle_nodes(37.5, 25.0, 6.0, 48), 0.02, 0.0, 1.0, 1.3)]
    cfg["contact_cutoff"] = 2.0
    return cfg


def _rigid_mix():
    cfg = wl._base("mix", 96, 48, 0.8, 4, "dynamic", 0,
                   body_force_x=wl.poiseuille_body_force(0.8, 48, 0.02),
                   init_profile=wl.INIT_POISEUILLE)
    ks = wl.ks_from_ca(0.8, 0.02, 1e-2)
    cfg["capsules"] = [wl.rigid_particle(wl.circle_nodes(30.0, 22.0, 6.0, 48), 1.2),
                       wl.capsule(wl.circle_nodes(43.7, 24.0, 6.0, 48), ks, 0.0, 1.0, 1.0)]
    cfg["contact_cutoff"] = 2.0
    return cfg


CASES = {
    "dynamic_contact": lambda: _contact_pair("dynamic"),
    "kinematic_contact": lambda: _contact_pair("kinematic"),
    "grid_only": lambda: wl.grid_bench(n=256),
    "rigid_mix": _rigid_mix,
    "inertial": lambda: wl.inertial_capsules(seed=1, nx=512, ny=128, n_caps=6, steps=0),
}


def _same(a, b, ncap, lattices=1):
    for l in range(lattices):
        assert np.array_equal(a.pops_dev(l), b.pops_dev(l))
        assert np.array_equal(a.force(l), b.force(l))
    for c in range(ncap):
        for x, y in zip(a.capsule(c), b.capsule(c)):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("case", sorted(CASES))
def test_graph_replays_match_direct_launches(case):
    from paper_1903_03356_amd import lbib
    cfg = CASES[case]()
    ncap = len(cfg["capsules"])
    log(f"graph vs direct: {case}")
    a, b = lbib.Sim(cfg), lbib.Sim(cfg)
    a.set_graph(True)
    b.set_graph(False)
    # blocks start at steps 2, 18 (even), 42 (even), 59, 75 (odd)
    for chunk in (1, 40, 17, 33):
        a.step(chunk)
        b.step(chunk)
    assert a.graph_replays == 5 and b.graph_replays == 0
    assert a.check() == 0 and b.check() == 0
    _same(a, b, ncap)
    if ncap > 1:
        a.set_contact(0.0)
        b.set_contact(0.0)
        a.step(20)
        b.step(20)
        assert a.graph_replays == 6
        _same(a, b, ncap)


def test_graph_replays_in_a_batch():
    from paper_1903_03356_amd import lbib
    cfgs = wl.ensemble(seed=1, n_inst=6)
    a, b = lbib.Batch(cfgs), lbib.Batch(cfgs)
    a.set_graph(True)
    b.set_graph(False)
    for chunk in (1, 40, 17):
        a.step(chunk)
        b.step(chunk)
    assert a.graph_replays == 3
    _same(a, b, sum(len(c["capsules"]) for c in cfgs), lattices=len(cfgs))
    # a new tile shape is captured again (the replays then launch that shape)
    a.set_tile(2, 4)
    a.step(20)
    b.step(20)
    assert a.graph_replays == 4
    _same(a, b, sum(len(c["capsules"]) for c in cfgs), lattices=len(cfgs))


def test_timing_runs_launch_directly():
    from paper_1903_03356_amd import lbib
    s = lbib.Sim(wl.grid_bench(n=128))
    s.set_timing(True)
    s.step(40)
    t = s.get_timing()
    assert s.graph_replays == 0 and t["grid_launches"] == 40
