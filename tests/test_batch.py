"""Batched ensembles: many independent lattices in one context
(lbib_create_batch), stepped by one grid launch and one IB launch per step.

GPU tests compare every lattice of a batch with the FP64 oracle run on that
lattice alone (same tolerances as the single-lattice parity tests), and check
that a batch is bit-identical to the same lattices stepped in contexts of
their own.  The CPU tests cover buffer sizing, argument checks that fail
before any device work, and the seeded ensemble draw."""
import ctypes as C

import numpy as np
import pytest

from paper_1903_03356_amd import lbib
from paper_1903_03356_amd import workloads as wl
from tests.parity import W, log, oracle_threads, vel_l2_rel


# ------------------------------------------------------------------ CPU ----

def test_required_bytes_batch_is_the_sum_of_the_lattices():
    grids = [lbib.make_grid(100, 37, 4, 2, 200, 100), lbib.make_grid(130, 64, 4, 1, 128, 128),
             lbib.make_grid(1024, 9, 4, 1, 3, 3)]
    for bid in (0, 1, 2):
        assert lbib.required_bytes_batch(grids, bid) == sum(lbib.required_bytes(g, bid)
                                                            for g in grids)
    assert lbib.required_bytes_batch(grids, 3) >= sum(2 * g.ny * 2 * 4 for g in grids)
    assert lbib.required_bytes_batch(grids, 4) == \
        -(-20 * (200 + 128 + 3) * 4 // 256) * 256
    assert lbib.required_bytes_batch(grids, 5) >= 4 * 272 + 3 * 112
    assert lbib.required_bytes_batch(grids, 7) >= 3 * 1024 * 9 * 8
    assert lbib.required_bytes_batch(grids[:1], 0) == lbib.required_bytes(grids[0], 0)
    for bid in range(8):
        assert lbib.required_bytes_batch(grids, bid) % 256 == 0
    mixed = grids[:2] + [lbib.make_grid(64, 64, 8)]
    assert all(lbib.required_bytes_batch(mixed, i) == 0 for i in range(8))
    L = lbib.load()
    arr = (lbib.lbib_grid * 1)(grids[0])
    assert L.lbib_required_bytes_batch(arr, 0, 0) == 0
    assert L.lbib_required_bytes_batch(None, 1, 0) == 0


def _create_batch(grids, taus, walls, null_taus=False):
    L = lbib.load()
    n = len(grids)
    g = (lbib.lbib_grid * max(1, n))(*grids)
    t = None if null_taus else (C.c_double * max(1, n))(*taus)
    w = (lbib.lbib_walls * max(1, n))(*walls)
    ptrs = (C.c_void_p * lbib.NUM_BUFFERS)(*[C.c_void_p(256 * (i + 1))
                                            for i in range(lbib.NUM_BUFFERS)])
    h = C.c_void_p()
    rc = L.lbib_create_batch(g, t, w, n, ptrs, lbib.NUM_BUFFERS, None, C.byref(h))
    return rc, h


def test_create_batch_rejects_invalid_arguments():
    L = lbib.load()
    w = lbib.lbib_walls(1, 0, 0.0, 0.0, 0.0, 0, 0.0, 0.0)
    g4, g8 = lbib.make_grid(64, 64, 4), lbib.make_grid(64, 64, 8)
    rc, h = _create_batch([g4, g8], [0.8, 0.8], [w, w])
    assert rc == lbib.EINVAL and not h.value
    assert b"real_bytes" in L.lbib_last_error(None)
    rc, _ = _create_batch([g4, g4, g4], [0.8, 0.5, 0.8], [w, w, w])
    assert rc == lbib.EINVAL and b"tau" in L.lbib_last_error(None)
    rc, _ = _create_batch([], [], [])
    assert rc == lbib.EINVAL
    rc, _ = _create_batch([g4], [0.8], [w], null_taus=True)
    assert rc == lbib.EINVAL
    w0 = lbib.lbib_walls(2, 0, 0.0, 0.0, 0.0, 0, 0.0, 0.0)
    rc, _ = _create_batch([g4, g4], [0.8, 0.8], [w, w0])
    assert rc == lbib.EINVAL and b"periodic_x" in L.lbib_last_error(None)
    assert L.lbib_num_lattices(None) == -1
    assert L.lbib_add_capsule_to(None, 0, None, 3, None, 1, 0.0, 1.0, 1.0, None) == lbib.EINVAL


def test_ensemble_draw():
    """Seeded ensemble: sizes, taus and capsule counts inside the documented
    ranges, every capsule inside its channel with the wall margin and below the
    stability screen, and the same seed gives the same draw."""
    E = wl.ensemble(seed=0, n_inst=24)
    E2 = wl.ensemble(seed=0, n_inst=24)
    for a, b in zip(E, E2):
        assert (a["nx"], a["ny"], a["tau"]) == (b["nx"], b["ny"], b["tau"])
        for ca, cb in zip(a["capsules"], b["capsules"]):
            assert np.array_equal(ca["nodes"], cb["nodes"])
    for cfg in E:
        assert 128 <= cfg["nx"] <= 512 and 64 <= cfg["ny"] <= 128
        assert 0.6 <= cfg["tau"] <= 1.2
        assert 1 <= len(cfg["capsules"]) <= 2
        g = wl.poiseuille_body_force(cfg["tau"], cfg["ny"], 0.02)
        assert cfg["body_force_x"] == pytest.approx(g, rel=1e-15)
        for cap in cfg["capsules"]:
            n = len(cap["nodes"])
            assert 64 <= n <= 128
            y = cap["nodes"][:, 1]
            assert y.min() >= 3.0 and y.max() <= cfg["ny"] - 4.0
            assert wl.polygon_area(cap["nodes"]) > 0
            assert wl.stability_ratio(cap["ks"], cap["mass"], n) <= 1.5
    assert wl.ensemble(seed=1, n_inst=4)[0]["nx"] != E[0]["nx"] or \
        wl.ensemble(seed=1, n_inst=4)[0]["tau"] != E[0]["tau"]


# ------------------------------------------------------------------ GPU ----

def _oracle(cfg):
    from oracle import oracle as orc
    oracle_threads(orc)
    return orc.Sim(cfg)


def _compare_lattice(b, i, o, vel_tol, rho_tol, pos_tol, d_tol):
    mg, mo = b.moments(i), o.moments()
    err_u = vel_l2_rel(mg, mo)
    err_rho = float(np.abs(mg[0] - mo[0]).max())
    out = {"lattice": i, "u_l2_rel": err_u, "rho_max_abs": err_rho}
    assert err_u <= vel_tol and err_rho <= rho_tol, out
    for k, cid in enumerate(b.cap_ids[i]):
        xg, pg, _ = b.capsule(cid)
        xo, po, _ = o.capsule(k)
        dg, do = b.diag(cid), o.diag(k)
        e = {"lattice": i, "cap": k, "x": float(np.abs(xg - xo).max()),
             "xprev": float(np.abs(pg - po).max()), "dD": abs(dg["D"] - do["D"]),
             "dSw": abs(dg["Sw"] - do["Sw"]), "ddp": abs(dg["dp"] - do["dp"])}
        assert e["x"] <= pos_tol and e["xprev"] <= pos_tol, e
        assert e["dD"] <= d_tol and e["dSw"] <= d_tol and e["ddp"] <= d_tol, e
    return out


def _mixed_lattices(real_bytes=4, mode="dynamic"):
    """Three lattices of different sizes, taus and walls: a ragged channel with
    two capsules, a capsule-free Couette channel, and a periodic box."""
    a = wl._base("a", 130, 70, 0.7, real_bytes, mode, 0,
                 body_force_x=wl.poiseuille_body_force(0.7, 70, 0.02),
                 init_profile=wl.INIT_POISEUILLE)
    ks = wl.ks_from_ca(0.7, 0.02, 1e-2)
    a["capsules"] = [wl.capsule(wl.circle_nodes(32.0, 30.0, 6.0, 64), ks, 0.0, 1.0, 1.5),
                     wl.capsule(wl.biconcave_nodes(97.0, 38.0, 14.0, 80, 0.4), ks, 0.0, 1.0, 1.0)]
    b = wl._base("b", 200, 64, 1.1, real_bytes, mode, 0, u_bottom=-0.01, u_top=0.01,
                 init_profile=wl.INIT_COUETTE)
    c = wl.periodic_box(96, 72, 0.9, u0=(0.015, -0.005), real_bytes=real_bytes, mode=mode)
    c["capsules"] = [wl.capsule(wl.circle_nodes(40.0, 36.0, 7.0, 72),
                                wl.ks_from_ca(0.9, 0.02, 3e-2), 0.0, 1.0, 1.2)]
    return [a, b, c]


@pytest.mark.gpu
def test_batch_bitwise_matches_single_contexts():
    cfgs = wl.ensemble(seed=3, n_inst=5)
    log("batch vs single contexts: " + ", ".join(f"{c['nx']}x{c['ny']}" for c in cfgs))
    bat = lbib.Batch(cfgs)
    singles = [lbib.Sim(c) for c in cfgs]
    bat.step(80)
    for s in singles:
        s.step(80)
    assert bat.check() == 0
    for i, s in enumerate(singles):
        assert np.array_equal(bat.pops_dev(i), s.pops_dev()), i
        assert np.array_equal(bat.force(i), s.force()), i
        for k, cid in enumerate(bat.cap_ids[i]):
            for a, b in zip(bat.capsule(cid), s.capsule(k)):
                assert np.array_equal(a, b), (i, k)
            assert bat.diag(cid) == s.diag(k)


@pytest.mark.gpu
def test_batch_fp32_dynamic_vs_oracle():
    cfgs = _mixed_lattices(4, "dynamic")
    log("batch fp32 dynamic: 3 lattices, 150 steps")
    bat = lbib.Batch(cfgs)
    bat.step(150)
    assert bat.check() == 0
    for i, cfg in enumerate(cfgs):
        o = _oracle(cfg)
        o.step(150)
        log(str(_compare_lattice(bat, i, o, 1e-5, 1e-6, 1e-4, 1e-4)))


@pytest.mark.gpu
def test_batch_fp64_kinematic_vs_oracle():
    cfgs = _mixed_lattices(8, "kinematic")
    log("batch fp64 kinematic: 3 lattices, 200 steps")
    bat = lbib.Batch(cfgs)
    bat.step(200)
    assert bat.check() == 0
    for i, cfg in enumerate(cfgs):
        o = _oracle(cfg)
        o.step(200)
        log(str(_compare_lattice(bat, i, o, 1e-10, 1e-12, 1e-10, 1e-10)))


@pytest.mark.gpu
def test_ensemble_full_size_sampled():
    """The 256-lattice seeded ensemble (about 8.0 M cells, 388 capsules) in
    one batch; four lattices spread over the batch are checked against the
    oracle after 20 steps."""
    cfgs = wl.ensemble(seed=0)
    log(f"ensemble: {len(cfgs)} lattices, {sum(c['nx'] * c['ny'] for c in cfgs)} cells")
    bat = lbib.Batch(cfgs)
    bat.step(20)
    assert bat.check() == 0
    for i in (0, 1, 128, 255):
        o = _oracle(cfgs[i])
        o.step(20)
        log(str(_compare_lattice(bat, i, o, 1e-5, 1e-6, 1e-4, 1e-4)))


@pytest.mark.gpu
def test_batch_state_transfer_per_lattice():
    """set/get of the populations addresses one lattice and leaves the others
    alone (FP64 periodic boxes: no wall rows, so the round trip is exact)."""
    cfgs = [wl.periodic_box(40 + 24 * i, 20 + 8 * i, 0.8, real_bytes=8) for i in range(3)]
    bat = lbib.Batch(cfgs)
    before = [bat.pops(i) for i in range(3)]
    f1 = wl.random_populations(64, 28, seed=5)
    bat.set_pops(f1, 1)
    assert np.array_equal(bat.pops(1), f1)
    assert np.array_equal(bat.pops(0), before[0])
    assert np.array_equal(bat.pops(2), before[2])
    with pytest.raises(lbib.LbibError) as e:
        bat.get_state(lbib.F_MOMENTS, 3)
    assert e.value.code == lbib.EINVAL
    with pytest.raises(lbib.LbibError) as e:
        bat.add_capsule_to(3, wl.circle_nodes(20, 10, 4, 16), 0.01, 0.0, 1.0, 1.0)
    assert e.value.code == lbib.EINVAL
    assert bat.num_lattices == 3
    o = _oracle(cfgs[1])
    o.set_pops(f1)
    bat.step(30)
    o.step(30)
    dg = bat.pops_dev(1)
    do = o.pops() - W[:, None, None]
    assert np.abs(dg - do).max() < 1e-13


def _same_batches(a, b, n_lattices):
    for i in range(n_lattices):
        assert np.array_equal(a.pops_dev(i), b.pops_dev(i)), i
        assert np.array_equal(a.force(i), b.force(i)), i
        for cid in a.cap_ids[i]:
            for x, y in zip(a.capsule(cid), b.capsule(cid)):
                assert np.array_equal(x, y), (i, cid)


@pytest.mark.gpu
@pytest.mark.parametrize("linear", [False, True, "chunked"])
@pytest.mark.parametrize("rows", [1, 2, 4])
def test_every_tile_shape_is_bit_identical(rows, linear):
    """The tile shapes of the batched grid pass (rows per thread, banded,
    linear or chunked tile order, one block per tile or a persistent launch) compute the
    same bits as the default, on lattices with ragged rows and segments, walls,
    a Couette channel and a periodic box."""
    cfgs = _mixed_lattices() + wl.ensemble(seed=4, n_inst=4)
    ref = lbib.Batch(cfgs)
    ref.step(40)
    for resident in (0, 1, 3, 8):
        log(f"tile rows={rows} linear={linear} resident={resident}")
        b = lbib.Batch(cfgs)
        b.set_tile(rows, resident, linear)
        b.step(40)
        assert b.check() == 0
        _same_batches(b, ref, len(cfgs))


@pytest.mark.gpu
def test_autotune_picks_a_shape_and_keeps_the_state():
    cfgs = wl.ensemble(seed=5, n_inst=16)
    a, b = lbib.Batch(cfgs), lbib.Batch(cfgs)
    a.step(9)
    b.step(9)
    r = a.autotune(3)
    log(f"autotune: {r}")
    assert r["rows"] in (1, 2, 4) and r["resident"] in (0, 2, 4, 8)
    assert len(r["us"]) == 36 and all(v > 0 for v in r["us"].values())
    assert r["order"] in lbib.TILE_ORDERS
    _same_batches(a, b, len(cfgs))  # tuning leaves the state alone
    a.step(25)
    b.step(25)
    _same_batches(a, b, len(cfgs))


@pytest.mark.gpu
def test_tile_arguments_are_checked():
    s = lbib.Sim(wl.grid_bench(n=64))
    with pytest.raises(lbib.LbibError) as e:
        s.autotune(2)
    assert e.value.code == lbib.EINVAL
    b = lbib.Batch(wl.ensemble(seed=5, n_inst=2))
    for rows, res in ((3, 0), (1, -1), (2, 65)):
        with pytest.raises(lbib.LbibError) as e:
            b.set_tile(rows, res)
        assert e.value.code == lbib.EINVAL
    with pytest.raises(lbib.LbibError) as e:
        b.autotune(0)
    assert e.value.code == lbib.EINVAL


@pytest.mark.gpu
@pytest.mark.parametrize("rows,linear,resident", [(1, False, 0), (2, True, 0), (4, True, 8),
                                                  (1, "chunked", 0), (2, "chunked", 4)])
def test_overlapped_batch_is_bit_identical(rows, linear, resident):
    """The near / far split over a batch (each capsule's near region on its own
    lattice, the far part as the batched pass in the chosen tile shape, beside
    the IB launch) gives the bits of the single pass: a ragged channel with two
    capsules, a capsule-free Couette channel, a periodic box and seeded
    ensemble channels."""
    cfgs = _mixed_lattices() + wl.ensemble(seed=6, n_inst=5)
    a, b = lbib.Batch(cfgs), lbib.Batch(cfgs)
    a.set_overlap(True)
    b.set_overlap(False)
    a.set_tile(rows, resident, linear)
    for chunk in (1, 25, 34):
        a.set_timing(chunk == 34)  # the last chunk counts the near launches
        a.step(chunk)
        b.step(chunk)
    assert a.get_timing()["near_launches"] == 34  # the split did run
    assert a.check() == 0 and b.check() == 0
    _same_batches(a, b, len(cfgs))
