"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test ties one part of the oracle to something other than the oracle's
own formulas: lattice identities, closed-form flows, MLS reproduction
properties, conservation laws, energy gradients, polygon closed forms,
symmetry, and the paper's printed values (tests/golden/paper_values.json).
"""
import json
import math
import os

import numpy as np
import pytest

from paper_1903_03356_amd import workloads as wl
from tests.parity import edge_line_integrals, regular_polygon_force, uneven_polygon

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def lattice_from_eq3():
    """Velocities of Eq. 3 evaluated from their trigonometric definition."""
    e = [(0, 0)]
    for i in range(1, 5):
        a = (i - 1) * math.pi / 2
        e.append((round(math.cos(a)), round(math.sin(a))))
    for i in range(5, 9):
        a = (2 * i - 9) * math.pi / 4
        e.append((round(math.sqrt(2) * math.cos(a)), round(math.sqrt(2) * math.sin(a))))
    w = json.load(open(GOLDEN))["lattice_weights"]["value"]
    wts = [w[0]] + [w[1]] * 4 + [w[2]] * 4
    return np.array(e, dtype=float), np.array(wts)


E, WTS = lattice_from_eq3()


# ---------------------------------------------------------------- P1, P2 ----

def test_p1_equilibrium_moments(orc):
    rng = np.random.default_rng(1)
    for _ in range(20):
        rho = 1 + 0.1 * rng.standard_normal()
        u = 0.05 * rng.standard_normal(2)
        f = orc.equilibrium(rho, u[0], u[1])
        assert abs(f.sum() - rho) < 1e-14
        np.testing.assert_allclose(f @ E, rho * u, atol=1e-15)
        second = np.einsum("i,ia,ib->ab", f, E, E)
        np.testing.assert_allclose(second, rho * (np.eye(2) / 3 + np.outer(u, u)), atol=1e-15)
    assert abs(WTS.sum() - 1) < 1e-15


def test_p2_forcing_moments(orc):
    rng = np.random.default_rng(2)
    for tau in (0.6, 0.8, 1.3):
        for _ in range(10):
            u = 0.05 * rng.standard_normal(2)
            F = 1e-3 * rng.standard_normal(2)
            s = orc.forcing(tau, u[0], u[1], F[0], F[1])
            pre = 1 - 1 / (2 * tau)
            assert abs(s.sum()) < 1e-17
            np.testing.assert_allclose(s @ E, pre * F, atol=1e-18)
            second = np.einsum("i,ia,ib->ab", s, E, E)
            np.testing.assert_allclose(second, pre * (np.outer(u, F) + np.outer(F, u)), atol=1e-18)


def test_p2_one_step_adds_force_periodic(orc):
    """Fully periodic box, uniform force g: one step adds exactly N g of momentum."""
    nx, ny = 12, 9
    g = 3e-5
    cfg = wl._base("box", nx, ny, 0.7, 8, "kinematic", 1, periodic_y=1, body_force_x=g)
    sim = orc.Sim(cfg)
    sim.set_pops(wl.random_populations(nx, ny, seed=3))
    f0 = sim.pops()
    p0 = np.einsum("iyx,ia->a", f0, E)
    m0 = f0.sum()
    sim.step(1)
    f1 = sim.pops()
    p1 = np.einsum("iyx,ia->a", f1, E)
    assert abs(f1.sum() - m0) < 1e-12 * m0
    # momentum sums of ~100 cells of O(0.1): rounding ~1e-15
    np.testing.assert_allclose(p1 - p0, [nx * ny * g, 0.0], atol=2e-14)


# ---------------------------------------------------------------- P3 --------

def test_p3_mass_conserved_with_ib_forcing(orc):
    """Periodic box with a deforming capsule: total mass constant to rounding."""
    nx, ny = 40, 32
    cfg = wl.periodic_box(nx, ny, 0.8, u0=(0.01, 0.0), mode="kinematic")
    nodes = wl.circle_nodes(20.2, 15.7, 6.0, 48)
    stretched = nodes.copy()
    stretched[:, 0] = 20.2 + 1.2 * (nodes[:, 0] - 20.2)
    cfg["capsules"] = [wl.capsule(nodes, 0.02, 0.002, 1.0)]
    sim = orc.Sim(cfg)
    sim.set_pops(wl.random_populations(nx, ny, seed=5))
    sim.set_capsule(0, stretched, stretched, np.zeros_like(stretched))
    m0 = sim.pops().sum()
    sim.step(50)
    assert abs(sim.pops().sum() - m0) < 1e-13 * m0
    assert sim.status == 0


# ---------------------------------------------------------------- P4, P5 ----

@pytest.mark.parametrize("tau", [0.6, 0.8, 1.0])
def test_p4_poiseuille_closed_form(orc, tau):
    """Body-force channel with Zou-He walls converges to g/(2 nu) y (H - y)."""
    ny, g = 17, 1e-6
    cfg = wl._base("p", 4, ny, tau, 8, "kinematic", 0, body_force_x=g)
    sim = orc.Sim(cfg)
    sim.step(40000)
    nu = (tau - 0.5) / 3
    y = np.arange(ny)
    ua = g / (2 * nu) * y * (ny - 1 - y)
    m = sim.moments()
    assert np.abs(m[1] - ua[:, None]).max() < 1e-10 * ua.max()
    assert np.abs(m[2]).max() < 1e-14


def test_p5_couette_closed_form(orc):
    ny = 17
    cfg = wl._base("c", 4, ny, 0.8, 8, "kinematic", 0, u_bottom=-0.01, u_top=0.02)
    sim = orc.Sim(cfg)
    sim.step(40000)
    y = np.arange(ny)
    ua = -0.01 + 0.03 * y / (ny - 1)
    m = sim.moments()
    assert np.abs(m[1] - ua[:, None]).max() < 1e-12
    assert np.abs(m[2]).max() < 1e-14


def test_p4_init_profile_is_analytic(orc):
    """The Poiseuille start state carries the analytic profile (plus half of g)."""
    cfg = wl.poiseuille_biconcave(1e-2, nx=16, ny=33)
    cfg["capsules"] = []
    sim = orc.Sim(cfg)
    m = sim.moments()
    nu = (cfg["tau"] - 0.5) / 3
    g = cfg["body_force_x"]
    y = np.arange(33)
    ua = g / (2 * nu) * y * (32 - y)
    # walls carry the Zou-He velocity exactly; interior: equilibrium + g/2
    assert np.abs(m[1, 0]).max() < 1e-16 and np.abs(m[1, -1]).max() < 1e-16
    np.testing.assert_allclose(m[1, 1:-1], (ua[1:-1] + 0.5 * g)[:, None] * np.ones((1, 16)),
                               rtol=0, atol=1e-16)


# ---------------------------------------------------------------- P6 --------

def test_p6_mls_reproduction(orc):
    rng = np.random.default_rng(6)
    for _ in range(200):
        x, y = rng.uniform(5, 50, 2)
        cells, phi, dx, dy = orc.mls(x, y)
        # support: 3x3 around the nearest node (ties up)
        c0 = np.array([math.floor(x + 0.5), math.floor(y + 0.5)])
        assert set(map(tuple, cells - c0)) == {(a, b) for a in (-1, 0, 1) for b in (-1, 0, 1)}
        assert abs(phi.sum() - 1) < 1e-14
        np.testing.assert_allclose(phi @ cells, [x, y], atol=1e-12)
        # gradient rows reproduce the gradient of linear fields exactly
        np.testing.assert_allclose([dx.sum(), dy.sum()], [0, 0], atol=1e-13)
        np.testing.assert_allclose(dx @ cells, [1, 0], atol=1e-12)
        np.testing.assert_allclose(dy @ cells, [0, 1], atol=1e-12)
        # a random linear field and its gradient
        a, b, c = rng.standard_normal(3)
        vals = a + b * cells[:, 0] + c * cells[:, 1]
        assert abs(phi @ vals - (a + b * x + c * y)) < 1e-11
        assert abs(dx @ vals - b) < 1e-12 and abs(dy @ vals - c) < 1e-12


def test_p6_mls_node_centred_closed_form(orc):
    """At a lattice node the symmetric support makes the moment matrix diagonal,
    so phi_k = W_k / sum W (Eq. 9 weight with r_w, alpha as printed)."""
    gv = json.load(open(GOLDEN))
    rw, alpha = gv["mls_support_side"]["value"], gv["mls_alpha"]["value"]
    cells, phi, _, _ = orc.mls(17.0, 23.0)
    r = np.hypot(cells[:, 0] - 17.0, cells[:, 1] - 23.0) / rw
    W = np.exp(-(r / alpha) ** 2)
    np.testing.assert_allclose(phi, W / W.sum(), atol=1e-15)
    assert abs(phi.max() - 0.5201545) < 1e-7


# ---------------------------------------------------------------- P7 --------

def test_p7_spread_conserves_force_and_is_adjoint(orc):
    nx, ny = 32, 24
    cfg = wl.periodic_box(nx, ny, 0.8)
    sim = orc.Sim(cfg)
    rng = np.random.default_rng(7)
    field = np.zeros((3, ny, nx))
    field[0] = 1.0
    field[1:] = rng.standard_normal((2, ny, nx))
    sim.set_moments(field)
    n = 25
    xy = np.stack([rng.uniform(0, nx, n), rng.uniform(0, ny, n)], 1)
    c = rng.uniform(0.2, 1.5, n)
    F = rng.standard_normal((n, 2))
    fib = sim.spread(xy, c, F)
    np.testing.assert_allclose(fib.sum(axis=(1, 2)), (c[:, None] * F).sum(0), atol=1e-12)
    U = sim.interpolate(xy)
    lhs = np.sum(fib * field[1:])
    rhs = np.sum(c[:, None] * F * U)
    assert abs(lhs - rhs) < 1e-11 * max(1, abs(rhs))


# ---------------------------------------------------------------- P8, P9 ----

def _stress_free(nodes):
    nv = len(nodes)
    nxt = np.roll(nodes, -1, 0)
    prv = np.roll(nodes, 1, 0)
    l0 = np.hypot(*(nxt - nodes).T)
    a = nodes - prv
    b = nxt - nodes
    th = np.arctan2(a[:, 0] * b[:, 1] - a[:, 1] * b[:, 0], (a * b).sum(1))
    return l0, th, wl.polygon_area(nodes)


def _perturbed(seed, nv=40):
    rng = np.random.default_rng(seed)
    ref = wl.circle_nodes(10.0, 12.0, 5.0, nv)
    cur = ref + 0.15 * rng.standard_normal(ref.shape)
    ks = rng.uniform(0.5, 2.0, nv)
    return ref, cur, ks


def test_p8_zero_net_force_and_torque(orc):
    ref, cur, ks = _perturbed(8)
    l0, th0, A0 = _stress_free(ref)
    for part in orc.internal_forces(cur, l0, th0, ks, 0.3, 1.0, A0):
        np.testing.assert_allclose(part.sum(0), [0, 0], atol=1e-13)
        r = cur - cur.mean(0)
        torque = np.sum(r[:, 0] * part[:, 1] - r[:, 1] * part[:, 0])
        assert abs(torque) < 1e-12
    for part in orc.internal_forces(ref, l0, th0, ks, 0.3, 1.0, A0):
        assert np.abs(part).max() < 1e-14


def _energies(x, l0, th0, ks, kb, ka, A0):
    """Stretch (Eq. 10), bending (reading of Eq. 12-13: k_b(1 - cos)) and the
    area-penalty energy k_a p_ref (A - A0)^2 / (2 A0) whose gradient Eq. 14 is."""
    nxt = np.roll(x, -1, 0)
    prv = np.roll(x, 1, 0)
    l = np.hypot(*(nxt - x).T)
    es = 0.5 * np.sum(ks * (l - l0) ** 2)
    a = x - prv
    b = nxt - x
    th = np.arctan2(a[:, 0] * b[:, 1] - a[:, 1] * b[:, 0], (a * b).sum(1))
    eb = kb * np.sum(1 - np.cos(th - th0))
    A = wl.polygon_area(x)
    ea = ka * (1 / 3) * (A - A0) ** 2 / (2 * A0)
    return es, eb, ea


def test_p9_forces_are_energy_gradients(orc):
    ref, cur, ks = _perturbed(9, nv=24)
    l0, th0, A0 = _stress_free(ref)
    kb, ka = 0.37, 1.0
    fs, fb, fa = orc.internal_forces(cur, l0, th0, ks, kb, ka, A0)
    h = 1e-6
    for v in range(len(cur)):
        for d in range(2):
            xp, xm = cur.copy(), cur.copy()
            xp[v, d] += h
            xm[v, d] -= h
            ep = _energies(xp, l0, th0, ks, kb, ka, A0)
            em = _energies(xm, l0, th0, ks, kb, ka, A0)
            grad = [(p - m) / (2 * h) for p, m in zip(ep, em)]
            for F, gr in zip((fs, fb, fa), grad):
                assert abs(F[v, d] + gr) < 1e-8 * max(1.0, abs(gr)), (v, d)


# ---------------------------------------------------------------- P10 -------

@pytest.mark.parametrize("N", [3, 5, 12, 64])
def test_p10_regular_polygon(orc, N):
    R = 7.3
    x = wl.circle_nodes(3.0, -2.0, R, N, phase=0.13)
    d = orc.polygon_diag(x)
    assert abs(d["Sw"] - (math.pi / N) / math.tan(math.pi / N)) < 1e-13
    assert abs(d["perimeter"] - 2 * N * R * math.sin(math.pi / N)) < 1e-12
    assert abs(d["area"] - 0.5 * N * R * R * math.sin(2 * math.pi / N)) < 1e-11
    assert abs(d["D"]) < 1e-9
    assert abs(d["cx"] - 3.0) < 1e-12 and abs(d["cy"] + 2.0) < 1e-12


@pytest.mark.parametrize("N,a,b,rot", [(3, 2.0, 1.0, 0.3), (7, 5.0, 4.0, 1.1), (64, 9.0, 3.0, -0.4)])
def test_p10_affine_polygon_taylor(orc, N, a, b, rot):
    u = wl.circle_nodes(0.0, 0.0, 1.0, N, phase=0.37)
    p = u * np.array([a, b])
    c, s = math.cos(rot), math.sin(rot)
    p = p @ np.array([[c, s], [-s, c]]) + np.array([40.0, 20.0])
    d = orc.polygon_diag(p)
    assert abs(d["D"] - (a - b) / (a + b)) < 1e-12


def test_p11_biconcave_swelling_ratio(orc):
    """Eq. 26 as printed gives Sw0 = 0.4609, not the 0.481 printed beside it."""
    gv = json.load(open(GOLDEN))
    nodes = wl.biconcave_nodes(100.0, 50.0, 40.0, 2000)
    d = orc.polygon_diag(nodes)
    assert abs(d["Sw"] - 0.4609) < 5e-4
    assert abs(d["Sw"] - gv["biconcave_sw0_printed"]["value"]) > 0.015
    assert wl.polygon_area(nodes) > 0  # counter-clockwise


# ------------------------------------------------------ Eqs. 15-16 pins -----

def test_hydro_linear_pressure_field(orc):
    """rho = 1 + beta . x, u = 0: each element gets -(p+ - p-) n+ l with
    p+ - p- = (beta . 2.4 n+)/3 exactly (linear reproduction)."""
    nx, ny = 48, 40
    sim = orc.Sim(wl.periodic_box(nx, ny, 0.8))
    beta = np.array([2e-3, -1.3e-3])
    yy, xx = np.mgrid[0:ny, 0:nx]
    field = np.zeros((3, ny, nx))
    field[0] = 1 + beta[0] * xx + beta[1] * yy
    sim.set_moments(field)
    x = wl.circle_nodes(24.3, 19.6, 6.0, 30)
    fext = sim.external_forces(x)
    probe = json.load(open(GOLDEN))["probe_length"]["value"]
    exp = np.zeros_like(x)
    for l in range(len(x)):
        t = x[(l + 1) % len(x)] - x[l]
        L = np.hypot(*t)
        n = np.array([t[1], -t[0]]) / L
        Fl = -(beta @ (2 * probe * n)) / 3 * n * L
        exp[l] += 0.5 * Fl
        exp[(l + 1) % len(x)] += 0.5 * Fl
    np.testing.assert_allclose(fext, exp, atol=1e-14)


def test_hydro_piecewise_shear(orc):
    """Two-node element (both orientations) across a kink in u_x(y): the
    viscous force is nu (g1 - g2) L along -x on each node."""
    nx, ny = 40, 24
    tau = 0.9
    nu = (tau - 0.5) / 3
    sim = orc.Sim(wl.periodic_box(nx, ny, tau))
    g1, g2 = 3e-3, -1e-3
    yy, xx = np.mgrid[0:ny, 0:nx].astype(float)
    field = np.zeros((3, ny, nx))
    field[0] = 1.0
    field[1] = np.where(yy <= 10.5, g1 * (yy - 10.5), g2 * (yy - 10.5))
    sim.set_moments(field)
    L = 0.8
    x = np.array([[20.1, 10.4], [20.1 + L, 10.4]])  # element 0 has n+ = (0, -1)
    fext = sim.external_forces(x)
    np.testing.assert_allclose(fext, [[-nu * (g1 - g2) * L, 0]] * 2, atol=1e-15)


def test_hydro_piecewise_cross_shear(orc):
    """The same element across a kink in du_y/dx instead: only the transposed
    gradient of the symmetric stress nu (grad u + grad u^T) (Eq. 16) reaches
    the element's normal, so the force is again nu (h1 - h2) L along -x on each
    node, and zero if the stress missed its transpose."""
    nx, ny = 40, 24
    tau = 0.9
    nu = (tau - 0.5) / 3
    sim = orc.Sim(wl.periodic_box(nx, ny, tau))
    h1, h2 = 2e-3, -1.5e-3
    yy, xx = np.mgrid[0:ny, 0:nx].astype(float)
    field = np.zeros((3, ny, nx))
    field[0] = 1.0
    field[2] = np.where(yy <= 10.5, h1 * (xx - 20.0), h2 * (xx - 20.0))
    sim.set_moments(field)
    L = 0.8
    x = np.array([[20.1, 10.4], [20.1 + L, 10.4]])  # element 0 has n+ = (0, -1)
    fext = sim.external_forces(x)
    np.testing.assert_allclose(fext, [[-nu * (h1 - h2) * L, 0]] * 2, atol=1e-15)


# ---------------------------------------------------------------- P12 -------

def _area_drift(orc, mode, ka, steps):
    cfg = wl.shear_capsule(mode=mode, g_num=0.1)
    cfg["capsules"][0]["ka"] = ka
    sim = orc.Sim(cfg)
    A0 = sim.diag(0)["A0"]
    worst = 0.0
    for _ in range(steps // 500):
        sim.step(500)
        worst = max(worst, abs(sim.diag(0)["area"] / A0 - 1.0))
    assert sim.status == 0
    return worst


@pytest.mark.parametrize("mode,steps", [("kinematic", 6000), ("dynamic", 3000)])
def test_p12_area_penalty_limits_the_drift(orc, mode, steps):
    """Area conservation (Eq. 14 with k_a = 1): a capsule sheared at G = 0.1
    keeps |A / A0 - 1| below 1e-4, and the penalty more than halves the drift
    of the same run without it.  A penalty with the wrong sign or scale would
    widen the drift instead.  (Dynamic: 3000 steps, inside the stable period
    of the Dynamic loop.)"""
    with_penalty = _area_drift(orc, mode, 1.0, steps)
    without = _area_drift(orc, mode, 0.0, steps)
    assert with_penalty < 1e-4
    assert with_penalty < 0.5 * without


# ---------------------------------------------------------------- P13 -------

@pytest.mark.parametrize("mode", ["kinematic", "dynamic"])
def test_p13_uniform_translation(orc, mode):
    U = (0.013, -0.007)
    cfg = wl.periodic_box(48, 40, 0.8, u0=U, mode=mode)
    nodes = wl.circle_nodes(22.3, 19.1, 6.0, 60)
    cfg["capsules"] = [wl.capsule(nodes, 0.05, 0.01, 1.0)]
    sim = orc.Sim(cfg)
    D0 = sim.diag(0)["D"]
    n = 60
    sim.step(n)
    x, xm1, uv = sim.capsule(0)
    np.testing.assert_allclose(x, nodes + n * np.array(U), atol=1e-11)
    np.testing.assert_allclose(x - xm1, np.tile(U, (60, 1)), atol=1e-13)
    if mode == "dynamic":
        np.testing.assert_allclose(uv, np.tile(U, (60, 1)), atol=1e-13)
    assert abs(sim.diag(0)["D"] - D0) < 1e-12
    m = sim.moments()
    assert np.abs(m[1] - U[0]).max() < 1e-13 and np.abs(m[2] - U[1]).max() < 1e-13


# ---------------------------------------------------------------- P14 -------

@pytest.mark.parametrize("mode", ["kinematic", "dynamic"])
def test_p14_point_symmetry_shear(orc, mode):
    """Centred capsule in symmetric shear: the state is symmetric under the
    point reflection (x, y) -> (63 - x, 63 - y), so the centroid stays put and
    u(63 - x, 63 - y) = -u(x, y)."""
    cfg = wl.shear_capsule(mode=mode)
    sim = orc.Sim(cfg)
    sim.step(300)
    d = sim.diag(0)
    assert abs(d["cx"] - 31.5) < 1e-11 and abs(d["cy"] - 31.5) < 1e-11
    m = sim.moments()
    np.testing.assert_allclose(m[1], -m[1][::-1, ::-1], atol=1e-14)
    np.testing.assert_allclose(m[2], -m[2][::-1, ::-1], atol=1e-14)
    np.testing.assert_allclose(m[0], m[0][::-1, ::-1], atol=1e-14)
    x, _, _ = sim.capsule(0)
    np.testing.assert_allclose(x[32:], 63.0 - x[:32], atol=1e-11)
    assert d["D"] > 0 and sim.status == 0


@pytest.mark.parametrize("R,ratio", [(8.4, 1.0), (7.7, 1.6)])
def test_dynamic_first_step_closed_form(orc, R, ratio):
    """Eqs. 21-24 on one step.  A regular polygon stretched (or squeezed) from
    its stress-free radius, nodes at rest, fluid at rest: the direct forcing is
    zero, so the fluid stays at rest, the hydrodynamic force and the
    interpolated velocity are zero, and the update moves every node by exactly
    half the internal force over the node mass m_v = (rho_s / rho_f) A0 / N
    (Eq. 23), with node velocity 3/2 of that displacement (Eq. 24, BDF2 from a
    node at rest).  The internal force is the energy gradient in closed form."""
    N, R0, ks, ka = 48, 8.0, 0.05, 1.0
    c = (20.0, 20.0)
    cfg = wl.periodic_box(40, 40, 0.8, real_bytes=8, mode="dynamic")
    cfg["capsules"] = [wl.capsule(wl.circle_nodes(c[0], c[1], R0, N), ks, 0.0, ka, ratio)]
    o = orc.Sim(cfg)
    x0 = wl.circle_nodes(c[0], c[1], R, N)
    o.set_capsule(0, x0, x0, np.zeros_like(x0))
    o.step(1)
    x1, _, uv = o.capsule(0)
    Fr, A0 = regular_polygon_force(N, R, R0, ks, ka)
    mv = ratio * A0 / N
    rhat = (x0 - np.array(c)) / R
    d = x1 - x0
    radial = np.einsum("va,va->v", d, rhat)
    tangential = d - radial[:, None] * rhat
    expect = 0.5 * Fr / mv
    assert abs(expect) > 1e-4
    np.testing.assert_allclose(radial, expect, rtol=1e-10)
    assert np.abs(tangential).max() < 1e-12
    np.testing.assert_allclose(uv, 1.5 * d, rtol=0, atol=1e-14)
    assert np.abs(np.einsum("iyx,ia->a", o.pops(), E)).max() < 1e-13  # the fluid is still at rest


def test_dynamic_forcing_weight_is_arc_length(orc):
    """Dyn. steps 1-3 with c_v = the arc length of node v, half of each adjacent
    element (A11).  The nodes of a resting, unevenly spaced polygon are given a
    uniform velocity u0 over a fluid at rest, so F_v = c_v u0.  Spreading keeps
    the total (partition of unity) and its first moment (linear reproduction);
    one collision adds the force to the momentum (P2), and streaming keeps the
    angular momentum.  After one step the fluid therefore holds exactly the line
    integrals of u0 along the membrane: momentum P u0, and angular momentum
    (integral of x ds) x u0.  Both are exact for a polygon as sums of edge length
    times midpoint.  Per-node weights 1, or one-sided element lengths, give
    other values."""
    n = 40
    u0 = np.array([3e-3, -1e-3])
    cfg = wl.periodic_box(40, 36, 0.8, real_bytes=8, mode="dynamic")
    x0 = uneven_polygon(20.0, 18.0, 8.0, 6.0, n, seed=7)
    cfg["capsules"] = [wl.capsule(x0, 0.02, 0.0, 1.0, 1.0)]
    o = orc.Sim(cfg)
    o.set_capsule(0, x0, x0 - u0, np.tile(u0, (n, 1)))
    f0 = o.pops()
    o.step(1)
    f1 = o.pops()
    P, Ix = edge_line_integrals(x0)
    ys, xs = np.mgrid[0:36, 0:40].astype(np.float64)
    j = np.einsum("iyx,ia->ayx", f1 - f0, E)
    p1 = j.sum(axis=(1, 2))
    L1 = (xs * j[1] - ys * j[0]).sum()
    # sums over 1440 cells of O(0.1) populations: rounding ~1e-13 (x 40 for the moment)
    np.testing.assert_allclose(p1, P * u0, rtol=0, atol=5e-13)
    assert abs(L1 - (Ix[0] * u0[1] - Ix[1] * u0[0])) < 2e-11
    one_sided = (np.hypot(*(np.roll(x0, -1, axis=0) - x0).T)[:, None] * x0).sum(axis=0)
    assert abs((one_sided[0] - Ix[0]) * u0[1] - (one_sided[1] - Ix[1]) * u0[0]) > 1e-6


def test_wall_support_flag(orc):
    """A node whose MLS support reaches a wall row is flagged."""
    cfg = wl._base("w", 32, 24, 0.8, 8, "kinematic", 1)
    cfg["capsules"] = [wl.capsule(wl.circle_nodes(16.0, 6.0, 5.0, 40), 0.01)]
    sim = orc.Sim(cfg)
    sim.step(1)
    assert sim.status & orc.E_WALL


def test_mode_is_fixed(orc):
    cfg = wl.periodic_box(16, 16, 0.8)
    sim = orc.Sim(cfg)
    sim.step(1, "dynamic")
    with pytest.raises(RuntimeError):
        sim.step(1, "kinematic")


# ---------------------------------------------------------------- P15 -------

def _affine_taylor(shear):
    """Taylor deformation of a circle carried by the simple shear x' = x + s y:
    (s1 - s2)/(s1 + s2) for the singular values of [[1, s], [0, 1]]."""
    sv = np.linalg.svd(np.array([[1.0, shear], [0.0, 1.0]]), compute_uv=False)
    return (sv[0] - sv[1]) / (sv[0] + sv[1])


@pytest.mark.parametrize("g_num", [0.05, 0.00625])
def test_p15_short_time_material_line(orc, g_num):
    """Shear capsule (Sec. 3.1 geometry, shrunk): before the membrane has time
    to react, both schemes deform the circle like a material line, so D
    follows the affine closed form, and the two schemes agree (Sec. 3.1)."""
    gamma = 0.02 / 63
    res = {}
    for mode in ("kinematic", "dynamic"):
        sim = orc.Sim(wl.shear_capsule(g_num=g_num, eb=0.0, mode=mode))
        sim.step(160)
        res[mode] = sim.diag(0)["D"]
        assert abs(res[mode] / _affine_taylor(gamma * 160) - 1) < 0.1, (mode, res)
    assert abs(res["dynamic"] - res["kinematic"]) / res["kinematic"] < 0.05, res


def _box_with_stretched_capsule(orc, mode):
    cfg = wl.periodic_box(48, 48, 0.8, mode=mode)
    ref = wl.circle_nodes(23.7, 24.2, 8.0, 64)
    cfg["capsules"] = [wl.capsule(ref, 0.05, 0.0, 1.0)]
    sim = orc.Sim(cfg)
    st = ref.copy()
    st[:, 0] = 23.7 + 1.1 * (ref[:, 0] - 23.7)
    st[:, 1] = 24.2 + (ref[:, 1] - 24.2) / 1.1
    sim.set_capsule(0, st, st, np.zeros_like(st))
    return sim, cfg["capsules"][0], ref


def _energy_momentum(sim, cap, ref):
    """Stretch energy (Eq. 10), area-penalty energy (the potential of Eq. 14),
    fluid kinetic energy and fluid momentum."""
    x, _, _ = sim.capsule(0)
    l = np.hypot(*(np.roll(x, -1, 0) - x).T)
    l0 = np.hypot(*(np.roll(ref, -1, 0) - ref).T)
    A, A0 = wl.polygon_area(x), wl.polygon_area(ref)
    e_el = 0.5 * cap["ks"] * np.sum((l - l0) ** 2) + cap["ka"] / 3 * (A - A0) ** 2 / (2 * A0)
    m = sim.moments()
    ke = 0.5 * np.sum(m[0] * (m[1] ** 2 + m[2] ** 2))
    p = np.einsum("iyx,ia->a", sim.pops(), E)
    return e_el + ke, p


def test_p15_kinematic_energy_decay_and_momentum(orc):
    """Periodic box at rest, pre-stretched capsule, Kinematic IB: the force put
    into the fluid is the membrane force, which sums to zero, so the fluid
    momentum stays zero; the coupled system dissipates, so elastic plus
    kinetic energy never grows."""
    sim, cap, ref = _box_with_stretched_capsule(orc, "kinematic")
    e0, _ = _energy_momentum(sim, cap, ref)
    prev = e0
    for _ in range(12):
        sim.step(25)
        e, p = _energy_momentum(sim, cap, ref)
        assert e <= prev * (1 + 1e-12), (sim.steps, e, prev)
        assert np.abs(p).max() < 1e-11
        prev = e
    assert prev < 0.1 * e0


def test_p15_dynamic_relaxes(orc):
    sim, cap, ref = _box_with_stretched_capsule(orc, "dynamic")
    e0, _ = _energy_momentum(sim, cap, ref)
    sim.step(900)
    e, _ = _energy_momentum(sim, cap, ref)
    assert e < 0.1 * e0 and sim.status == 0


@pytest.mark.slow
def test_p15_kinematic_deformation_grows_with_g(orc):
    """Steady shear deformation increases with the dimensionless shear rate G."""
    orc.set_threads(min(8, os.cpu_count() or 1))
    d = []
    for g_num in (0.00625, 0.0125, 0.05):
        sim = orc.Sim(wl.shear_capsule(g_num=g_num, eb=0.0, mode="kinematic"))
        sim.step(4000)
        d.append(sim.diag(0)["D"])
        assert sim.status == 0
    assert d[0] < d[1] < d[2], d


# Sec. 3.1 and Sec. 3.2 report the two couplings in close agreement (both
# within 1 % of the benchmark in shear; a relative gap in the perimeter change
# that falls with Ca, 3.8e-3 at Ca = 1e-1 down to 1e-4 at Ca = 1e-4).  The
# Dynamic steps as printed do not reach that: the tentative velocity of Eq. 23
# is the fluid's, so each step the node restarts from the fluid velocity and
# its BDF2 velocity (Eq. 24) exceeds the fluid's by about F_tot / (2 m_v); the
# direct forcing (steps 1-3) hands the fluid c_v times that slip, i.e. only
# kappa / (1 + beta kappa) of the membrane force, kappa = ds / (2 m_v) (= 1/R
# for a circle with the area mass) and beta the share of the traction jump the
# probes of Eqs. 15-16 see (about 0.5 measured).  The capsule therefore deforms
# as a much softer one, and the loop with the BDF2 target grows a node-scale
# mode once its gain passes about 2/3.  These two pins state the paper's
# results and fail on the printed scheme; they stay as strict expected
# failures so that a change of reading that meets them shows up.
DYN_XFAIL = ("the printed weak Dynamic coupling passes the fluid only about ds / (2 m_v) of "
             "the membrane force and grows a node-scale mode (see the note above)")


@pytest.mark.xfail(strict=True, reason=DYN_XFAIL)
def test_p15_steady_shear_dynamic_agrees_with_kinematic(orc):
    """Sec. 3.1: the centred capsule in shear (64 x 64, G = 0.05, E_b = 0.05,
    rho_s / rho_f = 1) reaches the same steady Taylor deformation with both
    couplings, within 2 %."""
    orc.set_threads(min(8, os.cpu_count() or 1))
    d = {}
    for mode in ("kinematic", "dynamic"):
        sim = orc.Sim(wl.shear_capsule(mode=mode))
        sim.step(6000)
        d[mode] = sim.diag(0)["D"]
    assert abs(d["dynamic"] / d["kinematic"] - 1.0) < 0.02, d


@pytest.mark.slow
@pytest.mark.xfail(strict=True, reason=DYN_XFAIL)
def test_p16_dynamic_kinematic_gap_falls_with_ca(orc):
    """Sec. 3.2: a circular capsule at 6.5 / 15 of a Poiseuille channel, both
    couplings run to t u_max / H = 2; the relative gap in the perimeter change
    eps = |dp_Dyn - dp_Kin| / |dp_Kin| falls as Ca falls and is of the order of
    the paper's values (below 1e-2 at Ca = 1e-3)."""
    orc.set_threads(min(8, os.cpu_count() or 1))
    nx, ny, tau, u_max = 128, 49, 0.8, 0.02
    H = ny - 1
    steps = int(2 * H / u_max)
    eps = {}
    for ca in (1e-1, 1e-2, 1e-3):
        dp = {}
        for mode in ("kinematic", "dynamic"):
            cfg = wl._base("p16", nx, ny, tau, 8, mode, steps,
                           body_force_x=wl.poiseuille_body_force(tau, ny, u_max),
                           init_profile=wl.INIT_POISEUILLE)
            cfg["capsules"] = [wl.capsule(wl.circle_nodes(40.0, 6.5 / 15.0 * H, 6.0, 48),
                                          wl.ks_from_ca(tau, u_max, ca), 0.0, 1.0, 1.0)]
            sim = orc.Sim(cfg)
            sim.step(steps)
            dp[mode] = sim.diag(0)["dp"]
        eps[ca] = abs(dp["dynamic"] - dp["kinematic"]) / abs(dp["kinematic"])
    assert all(np.isfinite(v) for v in eps.values()), eps
    assert eps[1e-3] < eps[1e-2] < eps[1e-1], eps
    assert eps[1e-3] < 1e-2, eps


# ---- Eq. 27: contact repulsion between capsules ------------------------------

def _diamond(cx, cy, h=2.0):
    """Counter-clockwise square rotated 45 degrees: right, top, left, bottom
    vertices; the outward vertex normal of the right vertex is +x."""
    return np.array([[cx + h, cy], [cx, cy + h], [cx - h, cy], [cx, cy - h]])


@pytest.mark.parametrize("d,shift", [(0.8, False), (1.5, False), (2.5, False), (1.0, True)])
def test_contact_force_formula(orc, d, shift):
    """Two diamonds whose facing vertices are d apart (one pair inside the
    2 dx cutoff, every other pair beyond it): each of the two vertices gets
    (1e-4 / (8 sqrt 2)) d^(-5/2) along its own inward normal, nothing beyond
    the cutoff, and no other vertex is pushed.  With shift the pair faces
    across the periodic x boundary."""
    from paper_1903_03356_amd import workloads as wl
    nx = 40
    cfg = wl.periodic_box(nx, 24, 0.8, real_bytes=8, mode="kinematic")
    if shift:
        a, b = _diamond(nx - 2.0 - d / 2, 12.0), _diamond(2.0 + d / 2, 12.0)
    else:
        a, b = _diamond(16.0, 12.0), _diamond(16.0 + 4.0 + d, 12.0)
    cfg["capsules"] = [wl.capsule(a, 0.0, 0.0, 0.0), wl.capsule(b, 0.0, 0.0, 0.0)]
    cfg["contact_cutoff"] = 2.0
    s = orc.Sim(cfg)
    s.step(1)
    fa, fb = s.contact(0), s.contact(1)
    mag = 1e-4 / (8.0 * math.sqrt(2.0)) * d ** -2.5 if d < 2.0 else 0.0
    np.testing.assert_allclose(fa[0], [-mag, 0.0], rtol=1e-12, atol=1e-20)
    np.testing.assert_allclose(fb[2], [mag, 0.0], rtol=1e-12, atol=1e-20)
    assert np.all(fa[1:] == 0.0) and np.all(fb[[0, 1, 3]] == 0.0)


def test_contact_force_off_by_default(orc):
    from paper_1903_03356_amd import workloads as wl
    cfg = wl.periodic_box(40, 24, 0.8, real_bytes=8, mode="kinematic")
    cfg["capsules"] = [wl.capsule(_diamond(16.0, 12.0), 0.0, 0.0, 0.0),
                       wl.capsule(_diamond(21.0, 12.0), 0.0, 0.0, 0.0)]
    s = orc.Sim(cfg)
    s.step(1)
    assert np.all(s.contact(0) == 0.0)


# ---- open channel: Zou-He velocity inlet and pressure outlet (Sec. 3.2) ---

def test_open_channel_poiseuille(orc):
    """Channel driven by the parabolic inlet profile and the outlet density,
    started at rest (Sec. 3.2).  The inlet velocity and the outlet density are
    imposed exactly; at steady state the mid-channel profile is the parabola
    and the pressure gradient is the plane-Poiseuille one, dp/dx = -8 nu rho
    u_max / H^2 (closed forms); the corner density is the inner diagonal
    neighbour's."""
    from paper_1903_03356_amd import workloads as wl
    orc.set_threads(4)
    nx, ny, umax, tau = 60, 21, 0.01, 1.0
    cfg = wl.open_channel(nx, ny, tau, umax, real_bytes=8, mode="kinematic")
    s = orc.Sim(cfg)
    s.step(19000)
    m0 = s.moments()
    s.step(1000)
    rho, ux, uy = s.moments()
    assert np.abs(np.stack([rho, ux, uy]) - m0).max() < 1e-12  # steady
    H = ny - 1
    y = np.arange(ny)
    prof = 4.0 * umax * y * (H - y) / H ** 2
    assert np.abs(ux[:, 0] - prof).max() < 1e-14
    assert np.abs(rho[1:-1, -1] - 1.0).max() < 1e-14
    mid = nx // 2
    assert np.abs(ux[:, mid] / ux[H // 2, mid] - prof / umax).max() < 1e-4
    nu = (tau - 0.5) / 3.0
    dpdx = np.polyfit(np.arange(10, nx - 10), rho[H // 2, 10:nx - 10] / 3.0, 1)[0]
    theory = -8.0 * nu * umax / H ** 2 * rho.mean()
    assert abs(dpdx / theory - 1.0) < 0.01, (dpdx, theory)
    for (cx, cy), (nbx, nby) in (((0, 0), (1, 1)), ((0, H), (1, H - 1)),
                                 ((nx - 1, 0), (nx - 2, 1)), ((nx - 1, H), (nx - 2, H - 1))):
        assert abs(rho[cy, cx] - rho[nby, nbx]) < 1e-15


# ---- rigid particles (Sec. 2.3.1, Eqs. 17-20) --------------------------------

def test_rigid_mass_and_inertia_of_a_regular_polygon():
    """Regular N-gon of circumradius R: A = N R^2 sin(2 pi / N) / 2 and polar
    moment J = A R^2 (2 + cos(2 pi / N)) / 6 about its centre (-> pi R^4 / 2)."""
    from paper_1903_03356_amd import workloads as wl
    for n in (6, 40):
        R = 5.0
        p = wl.rigid_particle(wl.circle_nodes(3.0, 4.0, R, n), density_ratio=1.5)
        A = n * R * R * math.sin(2 * math.pi / n) / 2.0
        J = A * R * R * (2.0 + math.cos(2 * math.pi / n)) / 6.0
        assert p["mass"] == pytest.approx(1.5 * A, rel=1e-13)
        assert p["inertia"] == pytest.approx(1.5 * J, rel=1e-12)


def test_rigid_particle_translates_with_uniform_flow(orc):
    """Uniform flow in a periodic box: the start-up takes the flow's velocity,
    the direct forcing and the outer-probe loads vanish (uniform pressure gives
    no net force or torque on a closed polygon), so the particle translates
    exactly and does not turn."""
    from paper_1903_03356_amd import workloads as wl
    u0 = (0.02, -0.01)
    cfg = wl.periodic_box(48, 32, 0.8, u0=u0, real_bytes=8, mode="dynamic")
    nodes = wl.circle_nodes(20.0, 15.0, 5.0, 40)
    cfg["capsules"] = [wl.rigid_particle(nodes, 1.5)]
    s = orc.Sim(cfg)
    r0 = s.rigid(0)
    s.step(100)
    r = s.rigid(0)
    assert abs(r["X"] - (r0["X"] + 100 * u0[0])) < 1e-11
    assert abs(r["Y"] - (r0["Y"] + 100 * u0[1])) < 1e-11
    assert abs(r["w"]) < 1e-14 and abs(r["theta"]) < 1e-12
    x, _, _ = s.capsule(0)
    np.testing.assert_allclose(x, nodes + 100 * np.array(u0), atol=1e-11)


def test_rigid_disc_rotates_at_half_the_shear_rate(orc):
    """A free disc at the centre of a Couette flow turns at -gamma/2 in the
    unconfined Stokes limit (the fluid's local angular velocity); confinement
    R/H = 5/47 slows it by a few per cent.  The steady rate must lie in
    (0.95, 1.0) x (-gamma / 2)."""
    from paper_1903_03356_amd import workloads as wl
    orc.set_threads(4)
    nx, ny = 64, 48
    H = ny - 1
    cfg = wl._base("rot", nx, ny, 0.9, 8, "dynamic", 0, u_bottom=-0.01, u_top=0.01,
                   init_profile=wl.INIT_COUETTE)
    cfg["capsules"] = [wl.rigid_particle(wl.circle_nodes(0.5 * (nx - 1), 0.5 * H, 5.0, 40), 1.0)]
    s = orc.Sim(cfg)
    s.step(4000)
    r = s.rigid(0)
    ratio = r["w"] / (-0.5 * 0.02 / H)
    assert 0.95 < ratio < 1.0, ratio
    assert abs(r["X"] - 0.5 * (nx - 1)) < 1e-4 and abs(r["Y"] - 0.5 * H) < 1e-4
