"""Reverse-mode gradients (lbib_adjoint) against the FP64 oracle.

The oracle of a gradient is the definition of the derivative: the central
difference (J(p + h) - J(p - h)) / 2h of the oracle's objective after the same
number of steps.  The CPU test pins that difference (second-order convergence
in h, so h is in the asymptotic range and the objective is smooth there).
The GPU tests compare the FP64 adjoint with it (relative 1e-5 of the largest
component, both schemes, both objectives, k_s of single elements and the body
force g), the FP32 adjoint with the FP64 adjoint, and check that the taped
forward run leaves the context exactly where lbib_step would."""
import math

import numpy as np
import pytest

from paper_1903_03356_amd import lbib
from paper_1903_03356_amd import workloads as wl
from tests.parity import log, oracle_threads


def ellipse_channel(real_bytes=8, mode="dynamic", nx=64, ny=40, n_nodes=32, ca=0.02,
                    tau=0.8, a=6.0, b=4.5, centre=(24.0, 17.0), ratio=1.0):
    """Elliptical capsule (D = (a - b)/(a + b) at rest, so D stays away from
    its non-smooth zero) in a body-force Poiseuille channel."""
    ang = 2.0 * math.pi * (np.arange(n_nodes) + 0.5) / n_nodes
    nodes = np.stack([centre[0] + a * np.cos(ang), centre[1] + b * np.sin(ang)], axis=1)
    ks = wl.ks_from_ca(tau, 0.02, ca)
    cfg = wl._base("ellipse", nx, ny, tau, real_bytes, mode, 0,
                   body_force_x=wl.poiseuille_body_force(tau, ny, 0.02),
                   init_profile=wl.INIT_POISEUILLE)
    cfg["capsules"] = [wl.capsule(nodes, ks, 0.0, 1.0, ratio)]
    return cfg


def test_central_difference_is_second_order(orc):
    """Pins the oracle's gradient.  For an element's k_s the differences with
    h, h/2, h/4 converge at second order (the gap shrinks about 4x per
    halving).  The MLS support (floor(x + 1/2)) makes the objective piecewise
    smooth with small jumps where a node crosses a half-integer, so a
    difference is only meaningful with h below the distance to the nearest
    switch: for the body force (which moves every node) h = 1e-4 and 1e-5
    relative give the same value to 1e-6, while 1e-2 straddles a switch."""
    oracle_threads(orc)
    cfg = ellipse_channel(mode="dynamic", nx=48, ny=32, n_nodes=24, centre=(20.0, 13.0))
    steps = 30
    ks0 = cfg["capsules"][0]["ks"]
    h = 0.2 * ks0
    d1 = orc.central_difference(cfg, steps, ("ks", 0, 3), h, "D")
    d2 = orc.central_difference(cfg, steps, ("ks", 0, 3), h / 2, "D")
    d4 = orc.central_difference(cfg, steps, ("ks", 0, 3), h / 4, "D")
    e1, e2 = abs(d1 - d2), abs(d2 - d4)
    assert d1 != 0.0 and 0.15 * e1 < e2 < 0.35 * e1, (d1, d2, d4)
    g0 = cfg["body_force_x"]
    a = orc.central_difference(cfg, steps, "g", 1e-4 * g0, "D")
    b = orc.central_difference(cfg, steps, "g", 1e-5 * g0, "D")
    far = orc.central_difference(cfg, steps, "g", 1e-2 * g0, "D")
    assert abs(a - b) < 1e-6 * abs(a), (a, b)
    assert abs(far - a) > 1e-3 * abs(a)  # a support switch inside [g - h, g + h]


def _fd(cfg, steps, param, h, which):
    from oracle import oracle as orc
    oracle_threads(orc)
    return orc.central_difference(cfg, steps, param, h, which)


def _check_against_fd(mode, which, steps, elements=(0, 7, 19), eb=0.0):
    cfg = ellipse_channel(real_bytes=8, mode=mode)
    # bending k_b = E_b k_s R^2 (Sec. 3.1), R the ellipse's mean radius
    cfg["capsules"][0]["kb"] = eb * cfg["capsules"][0]["ks"] * 6.0 * 4.5
    sim = lbib.Sim(cfg)
    r = sim.adjoint(steps, lbib.OBJ_TAYLOR if which == "D" else lbib.OBJ_CENTROID_Y, 0, mode)
    from oracle import oracle as orc
    J_orc = orc.objective(cfg, steps, which)
    assert abs(r["J"] - J_orc) < 1e-9 * max(1.0, abs(J_orc)), (r["J"], J_orc)
    ks0 = cfg["capsules"][0]["ks"]
    grads, fds = [], []
    for l in elements:
        grads.append(r["dJ_dks"][0][l])
        fds.append(_fd(cfg, steps, ("ks", 0, l), 1e-4 * ks0, which))
    gg = r["dJ_dg"]
    # h = 1e-5 g keeps MLS support switches out of [g - h, g + h] (at 1e-4 g the
    # Dynamic run already crosses one); the difference then carries a rounding
    # error of up to 2 eps |J| / (2 h), which the g tolerance includes
    hg = 1e-5 * cfg["body_force_x"]
    fg = _fd(cfg, steps, "g", hg, which)
    noise_g = 4.0 * 2.0 * 2.2e-16 * max(1.0, abs(r["J"])) / (2.0 * hg)
    log(f"{mode} {which} E_b={eb} steps={steps}: ks adjoint {grads} fd {fds}; g adjoint {gg} fd {fg}")
    scale = max(abs(v) for v in fds)
    for a, f in zip(grads, fds):
        assert abs(a - f) <= 1e-5 * scale + 1e-12, (a, f)
    assert abs(gg - fg) <= 1e-5 * abs(fg) + noise_g, (gg, fg, noise_g)
    return r


@pytest.mark.gpu
@pytest.mark.parametrize("which", ["D", "yc"])
def test_adjoint_kinematic_fp64_vs_fd(which):
    _check_against_fd("kinematic", which, 60)


@pytest.mark.gpu
@pytest.mark.parametrize("which", ["D", "yc"])
def test_adjoint_dynamic_fp64_vs_fd(which):
    _check_against_fd("dynamic", which, 60)


@pytest.mark.gpu
@pytest.mark.parametrize("mode", ["kinematic", "dynamic"])
@pytest.mark.parametrize("which", ["D", "yc"])
def test_adjoint_bending_fp64_vs_fd(mode, which):
    """With bending (Eq. 13, E_b = 0.2): the reverse sweep carries the
    transpose of the bending forces too.  At this E_b the gradients differ
    from those without bending by 10-50 %, far outside the bar."""
    _check_against_fd(mode, which, 60, eb=0.2)


@pytest.mark.gpu
def test_adjoint_full_size_channel_vs_fd():
    """The 512 x 128 gradient channel itself (circle R = 10, 96 nodes at 0.4 H,
    Ca = 1e-2), FP64, 200 Dynamic steps: dD/dk_s of the element with the
    largest gradient and of element 37, and dD/dg, against the oracle's
    central differences; then the FP32 gradient of the same run against the
    FP64 one, and a 500-step FP32 Kinematic run with a checkpoint every 70
    steps against its whole-tape run.

    At this size the MLS support switches put jumps of about 1e-12 into D, so
    a difference is only trusted where those stay small against h: k_s with
    h = 1e-3 k_s (1e-3, 5e-4, 2.5e-4 agree within 2e-5 of the largest
    component), g with h = 1e-7 g (1e-6 and 1e-7 agree within 2e-6, while 1e-5
    straddles a switch).  The bar is 1e-4 of the largest k_s component, and
    1e-5 for g."""
    from oracle import oracle as orc
    oracle_threads(orc)
    steps = 200
    cfg = wl.adjoint_channel()
    cfg["real_bytes"] = 8
    r = lbib.Sim(cfg).adjoint(steps, lbib.OBJ_TAYLOR, 0, "dynamic")
    assert abs(r["J"] - orc.objective(cfg, steps, "D")) < 1e-9
    ks0 = cfg["capsules"][0]["ks"]
    k8 = r["dJ_dks"][0]
    top = int(np.argmax(np.abs(k8)))
    fds = {l: orc.central_difference(cfg, steps, ("ks", 0, l), 1e-3 * ks0, "D") for l in (top, 37)}
    scale = abs(fds[top])
    for l, fd in fds.items():
        log(f"512x128 dD/dks[{l}]: adjoint {k8[l]} fd {fd}")
        assert abs(k8[l] - fd) <= 1e-4 * scale, (l, k8[l], fd)
    hg = 1e-7 * cfg["body_force_x"]
    fg = orc.central_difference(cfg, steps, "g", hg, "D")
    log(f"512x128 dD/dg: adjoint {r['dJ_dg']} fd {fg}")
    assert abs(r["dJ_dg"] - fg) <= 1e-5 * abs(fg)
    cfg4 = wl.adjoint_channel()
    r4 = lbib.Sim(cfg4).adjoint(steps, lbib.OBJ_TAYLOR, 0, "dynamic")
    k4 = r4["dJ_dks"][0]
    assert np.abs(k4 - k8).max() <= 1e-3 * np.abs(k8).max()
    assert abs(r4["dJ_dg"] - r["dJ_dg"]) <= 1e-3 * abs(r["dJ_dg"])
    # Checkpoints against the whole tape over 500 steps, with the Kinematic
    # scheme: the forward runs are bit-identical, and the gradients differ only
    # by the summation order of the reverse IB kernel's floating-point atomics.
    # With the Dynamic scheme the growing mode of its weak coupling amplifies
    # that rounding through the reverse sweep (about 100x over 500 steps here,
    # up to 1.4e-4 relative in dJ/dg), so the comparison is made where the
    # sweep is stable; the Dynamic checkpoint paths are compared at shorter
    # horizons in test_checkpointed_adjoint_equals_full_tape.
    kin = dict(cfg4, mode="kinematic")
    full = lbib.Sim(kin).adjoint(500, lbib.OBJ_CENTROID_Y, 0, "kinematic")
    ck = lbib.Sim(kin).adjoint(500, lbib.OBJ_CENTROID_Y, 0, "kinematic", checkpoint_every=70)
    assert ck["J"] == full["J"]
    assert abs(ck["dJ_dg"] - full["dJ_dg"]) <= 1e-4 * abs(full["dJ_dg"])
    assert np.abs(ck["dJ_dks"][0] - full["dJ_dks"][0]).max() <= 1e-4 * np.abs(full["dJ_dks"][0]).max()


def two_capsule_channel(real_bytes=8, mode="dynamic"):
    """Two elliptical capsules one behind the other in a body-force channel:
    the first acts on the second only through the fluid."""
    cfg = ellipse_channel(real_bytes=real_bytes, mode=mode, nx=96, ny=40, centre=(22.0, 17.0))
    ang = 2.0 * math.pi * (np.arange(28) + 0.5) / 28
    nodes = np.stack([52.0 + 5.0 * np.cos(ang), 21.0 + 4.0 * np.sin(ang)], axis=1)
    cfg["capsules"].append(wl.capsule(nodes, wl.ks_from_ca(0.8, 0.02, 0.03), 0.0, 1.0, 1.2))
    return cfg


@pytest.mark.gpu
@pytest.mark.parametrize("mode", ["dynamic", "kinematic"])
def test_adjoint_two_capsules_vs_fd(mode):
    """The objective of the second capsule, differentiated with respect to an
    element of each capsule and g, against the oracle's central differences
    (FP64): the cross-capsule term travels through the fluid adjoint."""
    from oracle import oracle as orc
    oracle_threads(orc)
    steps = 50
    cfg = two_capsule_channel(mode=mode)
    r = lbib.Sim(cfg).adjoint(steps, lbib.OBJ_TAYLOR, 1, mode)
    assert abs(r["J"] - orc.objective(cfg, steps, "D", capsule=1)) < 1e-9
    fds, grads = [], []
    for c, l in ((0, 5), (1, 3), (1, 17)):
        ks0 = cfg["capsules"][c]["ks"]
        # h = 1e-3 k_s: below it the differences of this run carry support-switch
        # noise (1e-3 and 3e-3 agree within 3e-7; 1e-4 scatters by 1e-4)
        fds.append(orc.central_difference(cfg, steps, ("ks", c, l), 1e-3 * ks0, "D", capsule=1))
        grads.append(r["dJ_dks"][c][l])
    log(f"two capsules {mode}: adjoint {grads} fd {fds}")
    scale = max(abs(v) for v in fds)
    assert abs(fds[0]) > 1e-6 * scale  # capsule 0 does move the objective
    for a, f in zip(grads, fds):
        assert abs(a - f) <= 1e-5 * scale, (a, f)
    # 1e-6 g: at 1e-5 g the two-capsule run already straddles a support switch
    hg = 1e-6 * cfg["body_force_x"]
    fg = orc.central_difference(cfg, steps, "g", hg, "D", capsule=1)
    noise = 4.0 * 2.0 * 2.2e-16 * max(1.0, abs(r["J"])) / (2.0 * hg)
    log(f"two capsules {mode}: dJ/dg adjoint {r['dJ_dg']} fd {fg} (noise {noise:.1e})")
    assert abs(r["dJ_dg"] - fg) <= 1e-5 * abs(fg) + noise, (r["dJ_dg"], fg)


@pytest.mark.gpu
@pytest.mark.parametrize("eb", [0.0, 0.2])
def test_adjoint_fp32_vs_fp64(eb):
    """The FP32 adjoint of the same run, against the FP64 adjoint (without
    and with bending)."""
    cfgs = []
    for rb in (8, 4):
        cfg = ellipse_channel(real_bytes=rb)
        cfg["capsules"][0]["kb"] = eb * cfg["capsules"][0]["ks"] * 6.0 * 4.5
        cfgs.append(cfg)
    r8 = lbib.Sim(cfgs[0]).adjoint(100, lbib.OBJ_TAYLOR)
    r4 = lbib.Sim(cfgs[1]).adjoint(100, lbib.OBJ_TAYLOR)
    k8, k4 = r8["dJ_dks"][0], r4["dJ_dks"][0]
    err = np.abs(k4 - k8).max() / np.abs(k8).max()
    log(f"fp32 vs fp64 adjoint, E_b {eb}: ks rel {err:.2e}, g {r4['dJ_dg']} vs {r8['dJ_dg']}")
    assert err < 1e-3
    assert abs(r4["dJ_dg"] - r8["dJ_dg"]) < 1e-3 * abs(r8["dJ_dg"])


@pytest.mark.gpu
def test_adjoint_leaves_the_forward_state():
    """After lbib_adjoint(N) the context holds exactly the state lbib_step(N)
    produces (the taped forward run is the same computation)."""
    cfg = ellipse_channel(real_bytes=4)
    a = lbib.Sim(cfg)
    b = lbib.Sim(cfg)
    a.adjoint(40)
    b.step(40)
    assert a.steps_done == 40
    assert np.array_equal(a.pops_dev(), b.pops_dev())
    assert np.array_equal(a.force(), b.force())
    for x, y in zip(a.capsule(0), b.capsule(0)):
        assert np.array_equal(x, y)
    a.step(5)
    b.step(5)
    assert np.array_equal(a.pops_dev(), b.pops_dev())


@pytest.mark.gpu
@pytest.mark.parametrize("mode,rb,every", [("dynamic", 8, 7), ("dynamic", 4, 1),
                                           ("kinematic", 4, 7), ("kinematic", 8, 29)])
def test_checkpointed_adjoint_equals_full_tape(mode, rb, every):
    """Checkpoints every K steps with recomputed segments (K = 7 over 30 steps:
    four full segments and a ragged one of 2; K = 1; K = N - 1) against the
    whole-trajectory tape: J and the state left behind are bit-identical (the
    recomputed forward steps repeat the first run exactly); the gradients agree
    to the rounding of the reverse kernel's floating-point atomics, whose
    summation order is free (relative 1e-4 in FP32, 1e-11 in FP64 of the
    largest component)."""
    steps = 30
    full = lbib.Sim(ellipse_channel(real_bytes=rb, mode=mode))
    ck = lbib.Sim(ellipse_channel(real_bytes=rb, mode=mode))
    r0 = full.adjoint(steps, lbib.OBJ_CENTROID_Y, 0, mode)
    r1 = ck.adjoint(steps, lbib.OBJ_CENTROID_Y, 0, mode, checkpoint_every=every)
    tol = 1e-4 if rb == 4 else 1e-11
    assert r1["J"] == r0["J"]
    assert abs(r1["dJ_dg"] - r0["dJ_dg"]) <= tol * abs(r0["dJ_dg"])
    k0, k1 = r0["dJ_dks"][0], r1["dJ_dks"][0]
    assert np.abs(k1 - k0).max() <= tol * np.abs(k0).max()
    assert np.array_equal(ck.pops_dev(), full.pops_dev())
    assert np.array_equal(ck.force(), full.force())
    for x, y in zip(ck.capsule(0), full.capsule(0)):
        assert np.array_equal(x, y)
    ck.step(3)
    full.step(3)
    assert np.array_equal(ck.pops_dev(), full.pops_dev())


@pytest.mark.gpu
def test_checkpoint_workspace_size():
    """The checkpointed workspace of the 512 x 128 gradient channel (5000
    steps, a checkpoint every 70) against the whole-trajectory tape."""
    s = lbib.Sim(wl.adjoint_channel())
    full = s.adjoint_bytes(5000, 0)
    ck = s.adjoint_bytes(5000, 70)
    cells = 512 * 128
    log(f"adjoint workspace: full {full / 1e9:.2f} GB, checkpoint 70 {ck / 1e9:.3f} GB")
    assert full > 5000 * 52 * cells
    per_level = full / 5001  # one grid slot and one node slot (padded rows)
    assert ck < (72 + 71 + 3) * per_level + 5001 * 8192
    assert s.adjoint_bytes(5000, 5000) == full == s.adjoint_bytes(5000, 9999)
    assert s.adjoint_bytes(5000, -1) == 0


@pytest.mark.gpu
def test_adjoint_argument_checks():
    cfg = ellipse_channel(real_bytes=4)
    s = lbib.Sim(cfg)
    for kw, code in (({"objective": 5}, lbib.EINVAL), ({"capsule": 1}, lbib.EINVAL)):
        with pytest.raises(lbib.LbibError) as e:
            s.adjoint(10, **kw)
        assert e.value.code == code
    s.step(1)
    with pytest.raises(lbib.LbibError) as e:
        s.adjoint(10)
    assert e.value.code == lbib.ESTATE
    bat = lbib.Batch([cfg, cfg])
    with pytest.raises(lbib.LbibError) as e:
        bat.adjoint(10)
    assert e.value.code == lbib.EINVAL
    with pytest.raises(lbib.LbibError) as e:
        lbib.Sim(cfg).adjoint(10, checkpoint_every=-1)
    assert e.value.code == lbib.EINVAL


@pytest.mark.gpu
def test_autograd_function_chain_rule():
    """torch.autograd through lbib.capsule_objectives: the forward values
    against the oracle's objectives, and the gradient of a D + b y_c with
    respect to the per-element k_s and the peak speed u_max against central
    differences of the oracle (FP64)."""
    import torch
    from oracle import oracle as orc
    oracle_threads(orc)
    steps = 40
    base = ellipse_channel(real_bytes=8)
    nv = len(base["capsules"][0]["nodes"])
    ks0 = base["capsules"][0]["ks"]
    u0 = 0.02

    def build(ks, um):
        cfg = ellipse_channel(real_bytes=8)
        cfg["body_force_x"] = wl.poiseuille_body_force(cfg["tau"], cfg["ny"], um)
        cfg["capsules"][0]["ks"] = np.asarray(ks, np.float64)
        return cfg

    ks = torch.full((nv,), ks0, dtype=torch.float64, requires_grad=True)
    um = torch.tensor(u0, dtype=torch.float64, requires_grad=True)
    out = lbib.capsule_objectives(ks, um, build, steps)
    a, b = 1.0, 0.3
    (a * out[0] + b * out[1]).backward()

    def f(ks_np, u):
        cfg = build(ks_np, u)
        return a * orc.objective(cfg, steps, "D") + b * orc.objective(cfg, steps, "yc")

    k = np.full(nv, ks0)
    cfg0 = build(k, u0)
    out = out.detach()
    assert abs(float(out[0]) - orc.objective(cfg0, steps, "D")) < 1e-9
    assert abs(float(out[1]) - orc.objective(cfg0, steps, "yc")) < 1e-9
    h = 2e-7  # 1e-5 relative: clear of MLS support switches
    fd_um = (f(k, u0 + h) - f(k, u0 - h)) / (2 * h)
    e = np.zeros(nv)
    e[5] = 1e-4 * ks0
    fd_k5 = (f(k + e, u0) - f(k - e, u0)) / (2 * e[5])
    log(f"autograd: du_max {float(um.grad)} fd {fd_um}; dks[5] {float(ks.grad[5])} fd {fd_k5}")
    assert abs(float(um.grad) - fd_um) <= 1e-5 * abs(fd_um)
    assert abs(float(ks.grad[5]) - fd_k5) <= 1e-5 * abs(fd_k5)


@pytest.mark.gpu
def test_autograd_function_device_tensors():
    """capsule_objectives with ks and u_max on the GPU: the output and both
    gradients come back on the GPU, equal to those of CPU inputs.  At u_max = 0
    the gradient in u_max is the slope of g (linear in u_max) times dJ/dg,
    which is not zero."""
    import torch
    steps = 20
    base = ellipse_channel(real_bytes=8)
    nv = len(base["capsules"][0]["nodes"])
    ks0 = base["capsules"][0]["ks"]

    def build(ks, um):
        cfg = ellipse_channel(real_bytes=8)
        cfg["body_force_x"] = wl.poiseuille_body_force(cfg["tau"], cfg["ny"], um)
        cfg["capsules"][0]["ks"] = np.asarray(ks, np.float64)
        return cfg

    grads = {}
    for dev in ("cpu", "cuda"):
        ks = torch.full((nv,), ks0, dtype=torch.float64, device=dev, requires_grad=True)
        um = torch.tensor(0.02, dtype=torch.float64, device=dev, requires_grad=True)
        out = lbib.capsule_objectives(ks, um, build, steps)
        assert out.device.type == dev
        (out[0] + 0.3 * out[1]).backward()
        assert ks.grad.device.type == dev and um.grad.device.type == dev
        grads[dev] = (out.detach().cpu(), ks.grad.cpu(), um.grad.cpu())
    for a, b in zip(grads["cpu"], grads["cuda"]):
        assert torch.equal(a, b)
    ks = torch.full((nv,), ks0, dtype=torch.float64, device="cuda", requires_grad=True)
    um = torch.zeros((), dtype=torch.float64, device="cuda", requires_grad=True)
    out = lbib.capsule_objectives(ks, um, build, steps)
    out[1].backward()
    r = lbib.Sim(build(np.full(nv, ks0), 0.0)).adjoint(steps, lbib.OBJ_CENTROID_Y, 0)
    slope = build(np.full(nv, ks0), 1.0)["body_force_x"]
    assert float(um.grad) == pytest.approx(r["dJ_dg"] * slope, rel=1e-12)
    assert float(um.grad) != 0.0
