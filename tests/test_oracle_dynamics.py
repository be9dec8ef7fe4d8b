"""Pins of the oracle's time integration and coupling against invariants and
exact solutions: free fall, exactness of the corrected gradient on linear
fields, rigid motions, momentum conservation of the multi-step coupling, the
hydrostatic layer, viscous shear decay, density reinitialisation, normals and
the inflow profile."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1911_13255_amd import scenes


def _lone_fluid(n=3, g=-9.81):
    sc = scenes.hydrostatic_layer(seed=None)
    # three particles far apart, no walls: free fall
    sc["x_fluid"] = np.array([[0.05, 0.2], [0.1, 0.25], [0.15, 0.3]])[:n]
    sc["x_wall"] = np.zeros((0, 2))
    sc["n_wall"] = np.zeros((0, 2))
    sc["periodic"][:] = 0
    sc["g"] = np.array([0.0, g, 0.0])
    sc["hydro_H"] = 0.0
    return sc


def test_free_fall_is_exact_quadratic():
    # Position Verlet integrates constant acceleration exactly (Section 3.3).
    sc = _lone_fluid()
    o = O.Oracle(sc)
    x0 = o.get(O.F_X).copy()
    o.step(37)
    t = o.scalars()["t"]
    x = o.get(O.F_X)
    v = o.get(O.F_V)
    assert np.allclose(x[:, 0], x0[:, 0], atol=0)
    assert np.allclose(x[:, 1], x0[:, 1] - 0.5 * 9.81 * t * t, rtol=0, atol=1e-14)
    assert np.allclose(v[:, 1], -9.81 * t, rtol=1e-13)
    assert np.allclose(o.get(O.F_A)[:, 1], -9.81, rtol=0, atol=1e-15)


def test_solid_free_fall_and_time_averages():
    # Unstressed block in free fall: every sub-step has a = g, so the averages
    # over one acoustic step are abar = g and vbar = g (t_n + dt/2).
    sc = scenes.solid_block(dim=2, n=(6, 5, 1))
    sc["g"] = np.array([0.0, -9.81, 0.0])
    o = O.Oracle(sc)
    o.step(3)
    s = o.scalars()
    assert s["kappa"] > 1
    t1 = s["t"]
    t0 = t1 - s["dt_ac"]
    assert np.allclose(o.get(O.S_ABAR)[:, 1], -9.81, atol=1e-10)
    assert np.allclose(o.get(O.S_VBAR)[:, 1], -9.81 * 0.5 * (t0 + t1), rtol=1e-10)
    assert np.allclose(o.get(O.S_U)[:, 1], -0.5 * 9.81 * t1 * t1, rtol=1e-10)
    assert np.abs(o.get(O.S_F) - np.eye(2)).max() < 1e-12


@pytest.mark.parametrize("d", [2, 3])
def test_deformation_rate_is_exact_for_linear_velocity(d):
    # The corrected gradient reproduces any linear field exactly, edge and
    # corner particles included; a transposed operand or a missing volume fails.
    sc = scenes.solid_block(dim=d, n=(7, 6, 5), E=1e3)
    sc["v_solid"] = np.zeros((len(sc["x_solid"]), d))
    rng = np.random.default_rng(4)
    G = rng.standard_normal((d, d))
    sc["v_solid"] = sc["x_solid"] @ G.T
    o = O.Oracle(sc)
    o.rebuild()
    o.fluid_step()
    o.couple()
    o.set_scalars({"dt_ac": 1e-9})
    o.solid_substeps()
    dF = o.get(O.S_DF)
    assert np.abs(dF - G[None]).max() < 1e-9 * np.abs(G).max()


def test_rigid_rotation_is_stress_free():
    # F = R and u = (R - I) r0: no acceleration anywhere (g = 0, no fluid).
    sc = scenes.solid_block(dim=2, n=(8, 6, 1))
    o = O.Oracle(sc)
    x0 = o.get(O.S_X0)
    th = 0.4
    R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    o.set(O.S_F, np.broadcast_to(R, (len(x0), 2, 2)))
    o.set(O.S_U, x0 @ R.T - x0)
    o.rebuild()
    o.fluid_step()
    o.couple()
    o.set_scalars({"dt_ac": 1e-12})
    o.solid_substeps()
    a = o.get(O.S_A)
    s = o.scalars()
    scale = s["K"] / (1000.0 * 0.01)
    assert np.abs(a).max() < 1e-8 * scale


def test_uniform_stretch_restores():
    # A uniformly stretched block: constant stress gives no force inside and
    # pulls the faces back (sign of the stress divergence, Section 2.2).
    sc = scenes.solid_block(dim=2, n=(16, 16, 1), E=1e6, nu=0.3)
    o = O.Oracle(sc)
    x0 = o.get(O.S_X0)
    F = np.diag([1.001, 1.0])
    o.set(O.S_F, np.broadcast_to(F, (len(x0), 2, 2)))
    o.set(O.S_U, x0 @ F.T - x0)
    o.rebuild()
    o.fluid_step()
    o.couple()
    o.set_scalars({"dt_ac": 1e-12})
    o.solid_substeps()
    a = o.get(O.S_A)
    lo, hi = x0.min(0), x0.max(0)
    deep = np.all((x0 > lo + 0.045) & (x0 < hi - 0.045), axis=1)
    left = np.abs(x0[:, 0] - lo[0]) < 1e-9
    right = np.abs(x0[:, 0] - hi[0]) < 1e-9
    face = np.abs(a[right, 0]).mean()
    assert face > 0
    assert np.abs(a[deep]).max() < 1e-9 * face
    assert np.all(a[right, 0] < 0) and np.all(a[left, 0] > 0)


@pytest.mark.parametrize("d,eta", [(2, 0.0), (2, 2.0), (3, 0.5)])
def test_total_momentum_is_conserved_exactly(d, eta):
    # Periodic box, g = 0, free solid, kappa > 1 sub-steps: the position-based
    # Verlet scheme with the time-averaged coupling conserves fluid + solid
    # momentum to round-off (Section 3.3), and every coupling pair is exactly
    # antisymmetric (Section 2.2).
    sc = scenes.periodic_box_with_solid(dim=d, n=12 if d == 2 else 8, eta=eta, amp=0.3)
    o = O.Oracle(sc)
    mf, ms = o.masses()

    def total():
        return mf @ o.get(O.F_V) + ms @ o.get(O.S_V)

    def scale():
        return mf @ np.abs(o.get(O.F_V)).sum(1) + ms @ np.abs(o.get(O.S_V)).sum(1)

    p0 = total()
    kap = []
    for _ in range(25):
        if o.scalars()["need_rebuild"]:
            o.rebuild()
        o.fluid_step()
        o.couple()
        # same snapshot on both sides: the pair forces cancel
        pair = o.fluid_side_coupling()[:d] + o.totals()["sum_fF"][:d]
        assert np.abs(pair).max() <= 1e-13 * np.abs(o.get(O.S_FF)).sum()
        o.solid_substeps()
        kap.append(o.scalars()["kappa"])
    assert max(kap) > 1
    assert o.counters()["rebuilds"] >= 2
    assert o.counters()["n_sf"] > 0
    assert np.abs(total() - p0).max() < 1e-12 * scale()


def test_hydrostatic_layer_stays_at_rest():
    # Flat floor at rest: the imaginary wall pressure extrapolates hydrostatically
    # along the normal, so the layer keeps p = rho0 g (H - y) (walls, Section 2.2).
    sc = scenes.hydrostatic_layer()
    o = O.Oracle(sc, density_reinit=0)
    g, H = 9.81, 0.4
    o.step(1000)
    x, v, p = o.get(O.F_X), o.get(O.F_V), o.get(O.F_P)
    assert np.linalg.norm(v, axis=1).max() < 0.01 * math.sqrt(g * H)
    sel = (x[:, 1] > 0.05) & (x[:, 1] < 0.3)
    err = np.abs(p[sel] - 1000.0 * g * (H - x[sel, 1])).max()
    assert err < 0.1 * 1000.0 * g * H
    # nothing has gone through the floor
    assert x[:, 1].min() > 0.0


def test_shear_decay_loses_energy():
    # A viscous layer sliding over a static wall must lose kinetic energy
    # monotonically and be dragged backwards (the imaginary velocity mirrors the
    # fluid velocity about the wall's, no-slip).
    sc = scenes.shear_layer()
    o = O.Oracle(sc, density_reinit=0)
    mf, _ = o.masses()
    ke = [o.totals()["ke_fluid"]]
    px = [mf @ o.get(O.F_V)[:, 0]]
    for _ in range(40):
        o.step(1)
        ke.append(o.totals()["ke_fluid"])
        px.append(mf @ o.get(O.F_V)[:, 0])
    assert np.all(np.diff(ke) < 0)
    assert np.all(np.diff(px) < 0)
    assert ke[-1] < 0.999 * ke[0]


def test_density_reinit_on_an_unjittered_lattice():
    # At rest on an exact lattice the number density equals the lattice value
    # wherever the support is full (walls on the same lattice fill it), and
    # is clipped to rho0 at the free surface.
    sc = scenes.hydrostatic_column(seed=None)
    o = O.Oracle(sc, density_reinit=1)
    o.rebuild()
    rho = o.get(O.F_RHO)
    assert np.abs(rho / 1000.0 - 1.0).max() < 1e-12
    # without the walls in the sum, particles near the floor would be clipped,
    # but a lattice compressed by 1% must give psi > psi0 in the interior
    sc2 = scenes.hydrostatic_column(seed=None)
    sc2["x_fluid"] = sc2["x_fluid"] * 0.99
    o2 = O.Oracle(sc2, density_reinit=1)
    o2.rebuild()
    x = o2.get(O.F_X)
    inner = (x[:, 0] > 0.05) & (x[:, 0] < 0.15) & (x[:, 1] > 0.05) & (x[:, 1] < 0.3)
    r = o2.get(O.F_RHO)[inner] / 1000.0
    assert np.all(r > 1.015) and np.ptp(r) < 1e-9


def test_plate_normals():
    # Unjittered plate: faces have +-x normals, the middle column none; a rigid
    # rotation of F rotates them at the next rebuild.
    sc = scenes.dam_break_plate(seed=None)
    o = O.Oracle(sc)
    x0 = o.get(O.S_X0)
    n0 = o.get(O.S_N0)
    nfree = len(x0) - sc["n_clamp"]
    col = np.rint((x0[:, 0] - 0.2) / 0.001 - 0.5).astype(int)
    mid_h = (x0[:, 1] > 0.01) & (x0[:, 1] < 0.06)
    sel = np.arange(len(x0)) < nfree
    assert np.allclose(n0[sel & mid_h & (col == 0)], [-1.0, 0.0], atol=1e-12)
    assert np.allclose(n0[sel & mid_h & (col == 4)], [1.0, 0.0], atol=1e-12)
    assert np.all(n0[sel & mid_h & (col == 2)] == 0.0)
    assert np.allclose(n0[sel & mid_h & (col == 1)], [-1.0, 0.0], atol=1e-12)
    th = 0.3
    R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    o.set(O.S_F, np.broadcast_to(R, (len(x0), 2, 2)))
    o.rebuild()
    assert np.allclose(o.get(O.S_N), n0 @ R.T, atol=1e-12)


def test_inflow_profile_mean_and_peak():
    # The buffer profile has mean Ubar(t) over the channel height and peak
    # 1.5 Ubar at mid-height, with Ubar following the cosine ramp.
    sc = scenes.plate_behind_cylinder(dp_f=0.01)
    o = O.Oracle(sc)
    o.step(3)
    t = o.scalars()["t"]
    ubar = 0.5 * (1.0 - math.cos(0.5 * math.pi * t))
    x, v = o.get(O.F_X), o.get(O.F_V)
    buf = x[:, 0] < sc["inflow_len"]
    assert np.all(v[buf, 1] == 0.0)
    col = np.rint(x[:, 0] / sc["dp_f"] - 0.5).astype(int)
    first = buf & (col == 0)
    y, u = x[first, 1], v[first, 0]
    order = np.argsort(y)
    # trapezoid over one buffer column with the zero end points at the walls
    yy = np.concatenate([[0.0], y[order], [sc["inflow_H"]]])
    uu = np.concatenate([[0.0], u[order], [0.0]])
    mean = np.trapezoid(uu, yy) / sc["inflow_H"]
    assert len(y) > 30
    assert abs(mean - ubar) < 0.01 * ubar
    assert abs(v[buf, 0].max() - 1.5 * ubar) < 0.01 * ubar


def test_density_variation_is_about_one_percent():
    # With c = 10 v_max the density varies by about 1% (Section 2.1).
    o = O.Oracle(scenes.dam_break_plate(seed=2))
    o.step(200)
    rho = o.get(O.F_RHO)
    assert np.abs(rho / 1000.0 - 1.0).max() < 0.015
