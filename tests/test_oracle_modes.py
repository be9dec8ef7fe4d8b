"""Pins of the oracle's two contrasts to the multi-resolution, multi-time-step
method: the linear elastic (Kirchhoff) material of Section 2.1, and the single
time step of fluid and structure that Section 3.2 sets the multiple time steps
against.

The material is checked against what the mathematics fixes: no stress under a
rigid rotation, the infinitesimal Hooke law at small strain, S = dW/dE of its
own strain energy, agreement with the Neo-Hookean law to first order, and the
closed form of a plane-strain stretch.  The single step is checked against its
definition (one solid step, the smaller of the two criteria) and against the
multi-step method on a scene where that method already takes one sub-step.
"""
import math

import numpy as np
import pytest
from scipy import linalg

from oracle import oracle as O
from paper_1911_13255_amd import scenes


def _rot(d, ang):
    if d == 2:
        return np.array([[math.cos(ang), -math.sin(ang)], [math.sin(ang), math.cos(ang)]])
    ax = np.array([0.3, -1.0, 0.6])
    ax /= np.linalg.norm(ax)
    K = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
    return linalg.expm(ang * K)


# ---------------------------------------------------------------- Kirchhoff material

@pytest.mark.parametrize("d", [2, 3])
def test_svk_rigid_motion_is_stress_free(d):
    mu, lam = 3.0e6, 1.4e7
    assert np.abs(O.svk_stress(np.eye(d), mu, lam)).max() == 0.0
    assert np.abs(O.svk_stress(_rot(d, 1.1), mu, lam)).max() < 1e-8 * mu
    assert abs(O.svk_energy(_rot(d, 1.1), mu, lam)) < 1e-20 * mu


@pytest.mark.parametrize("d", [2, 3])
def test_svk_small_strain_is_infinitesimal_hooke(d):
    # sigma = lambda tr(eps) I + 2 mu eps with eps = sym(F - I): the textbook
    # small-strain law; the difference is second order in the strain
    mu, lam = 3.0e6, 1.4e7
    rng = np.random.default_rng(11)
    G = rng.standard_normal((d, d))
    errs = []
    for eps in (1e-3, 1e-4):
        F = np.eye(d) + eps * G
        P = O.svk_stress(F, mu, lam)
        e = 0.5 * (F - np.eye(d) + (F - np.eye(d)).T)
        sig = lam * np.trace(e) * np.eye(d) + 2 * mu * e
        errs.append(np.abs(P - sig).max())
        assert errs[-1] < 30 * eps * eps * (mu + lam)
    # quadratic, not linear, convergence: a dropped or doubled term fails
    assert errs[0] / errs[1] > 50


@pytest.mark.parametrize("d", [2, 3])
def test_svk_stress_is_energy_derivative(d):
    mu, lam = 2.0, 5.0
    rng = np.random.default_rng(12)
    F = np.eye(d) + 0.2 * rng.standard_normal((d, d))
    S = np.linalg.solve(F, O.svk_stress(F, mu, lam))
    E = 0.5 * (F.T @ F - np.eye(d))

    def W_of_E(Em):
        return O.svk_energy(linalg.sqrtm(np.eye(d) + 2 * Em).real, mu, lam)

    h = 1e-6
    for i in range(d):
        for j in range(d):
            dE = np.zeros((d, d))
            dE[i, j] += 0.5 * h
            dE[j, i] += 0.5 * h
            fd = (W_of_E(E + dE) - W_of_E(E - dE)) / (2 * h)
            assert abs(fd - 0.5 * (S[i, j] + S[j, i])) < 1e-7 * (mu + lam)


@pytest.mark.parametrize("d", [2, 3])
def test_svk_and_neo_hooke_share_the_linearisation(d):
    mu, lam = 1.0e6, 2.0e6
    rng = np.random.default_rng(13)
    G = rng.standard_normal((d, d))
    diffs = []
    for eps in (1e-2, 1e-3):
        F = np.eye(d) + eps * G
        diffs.append(np.abs(O.svk_stress(F, mu, lam) - O.nh_stress(F, mu, lam)).max())
    assert diffs[1] < 1e-4 * (mu + lam)
    assert diffs[0] / diffs[1] > 50
    # and they part at large strain
    F = np.eye(d) + 0.4 * G / np.abs(G).max()
    assert np.abs(O.svk_stress(F, mu, lam) - O.nh_stress(F, mu, lam)).max() > 1e-2 * mu


def test_svk_plane_strain_stretch_closed_form():
    # F = diag(s, 1): E11 = (s^2 - 1)/2, the only strain; S11 = (lambda + 2 mu) E11,
    # S22 = lambda E11, P = F S
    mu, lam = 3.0, 7.0
    for s in (0.6, 1.0, 1.5):
        P = O.svk_stress(np.diag([s, 1.0]), mu, lam)
        e11 = 0.5 * (s * s - 1.0)
        assert abs(P[0, 0] - s * (lam + 2 * mu) * e11) < 1e-14
        assert abs(P[1, 1] - lam * e11) < 1e-14
        assert P[0, 1] == 0.0 and P[1, 0] == 0.0
        assert abs(O.svk_energy(np.diag([s, 1.0]), mu, lam) - 0.5 * (lam + 2 * mu) * e11 * e11) < 1e-14


def test_svk_block_dynamics_rigid_rotation_and_stretch():
    # Through the whole sub-step: a rotated block feels no force, a stretched
    # one is pulled back at its faces and force-free inside.
    sc = scenes.solid_block(dim=2, n=(16, 16, 1), E=1e6, nu=0.3)
    sc["material"] = 1
    x0 = scenes.solid_block(dim=2, n=(16, 16, 1))["x_solid"]
    for F, kind in ((_rot(2, 0.5), "rot"), (np.diag([1.001, 1.0]), "stretch")):
        o = O.Oracle(sc)
        o.set(O.S_F, np.broadcast_to(F, (len(x0), 2, 2)))
        o.set(O.S_U, x0 @ F.T - x0)
        o.rebuild()
        o.fluid_step()
        o.couple()
        o.set_scalars({"dt_ac": 1e-12})
        o.solid_substeps()
        a = o.get(O.S_A)
        if kind == "rot":
            assert np.abs(a).max() < 1e-8 * o.scalars()["K"] / (1000.0 * 0.01)
        else:
            lo, hi = x0.min(0), x0.max(0)
            deep = np.all((x0 > lo + 0.045) & (x0 < hi - 0.045), axis=1)
            right = np.abs(x0[:, 0] - hi[0]) < 1e-9
            left = np.abs(x0[:, 0] - lo[0]) < 1e-9
            face = np.abs(a[right, 0]).mean()
            assert face > 0 and np.abs(a[deep]).max() < 1e-9 * face
            assert np.all(a[right, 0] < 0) and np.all(a[left, 0] > 0)


# ---------------------------------------------------------------- single time step

def test_single_step_takes_the_solid_step():
    # The dam break's plate is stiff (kappa > 10 in the multi-step method):
    # with one shared step, every acoustic step is the solid step and kappa = 1.
    sc = scenes.dam_break_plate(seed=1)
    multi = O.Oracle(sc)
    multi.step(1)
    assert multi.scalars()["kappa"] > 10
    sc["single_step"] = 1
    o = O.Oracle(sc)
    for _ in range(5):
        o.step(1)
        s = o.scalars()
        assert s["kappa"] == 1
        assert s["dt_ac"] == s["dt_s"]
    assert o.counters()["substeps"] == 5


def _soft_box(single):
    sc = scenes.periodic_box_with_solid(dim=2, n=12, amp=0.3)
    sc["E"] = 2e4
    sc["single_step"] = single
    return sc


def test_single_step_is_the_multi_step_method_when_kappa_is_one():
    # A soft block whose solid step exceeds the fluid step: both forms take the
    # same steps, so the trajectories are identical.
    a, b = O.Oracle(_soft_box(0)), O.Oracle(_soft_box(1))
    for _ in range(30):
        a.step(1)
        b.step(1)
        assert a.scalars()["kappa"] == 1
    assert a.counters()["rebuilds"] >= 2
    for f in (O.F_X, O.F_V, O.F_RHO, O.S_U, O.S_V, O.S_F, O.S_VBAR, O.S_ABAR):
        assert np.array_equal(a.get(f), b.get(f))
    assert a.scalars()["t"] == b.scalars()["t"]


def test_single_step_conserves_momentum():
    # One shared step is the kappa = 1 case of the same scheme: fluid + solid
    # momentum is conserved to round-off (Section 3.3).
    sc = scenes.periodic_box_with_solid(dim=2, n=12, amp=0.3)
    sc["single_step"] = 1
    o = O.Oracle(sc)
    mf, ms = o.masses()

    def total():
        return mf @ o.get(O.F_V) + ms @ o.get(O.S_V)

    scale = mf @ np.abs(o.get(O.F_V)).sum(1) + ms @ np.abs(o.get(O.S_V)).sum(1)
    p0 = total()
    dts = []
    for _ in range(25):
        o.step(1)
        s = o.scalars()
        assert s["kappa"] == 1
        dts.append(s["dt_ac"] / s["dt_s"])
    assert max(dts) == 1.0  # the solid step set the shared step
    assert np.abs(total() - p0).max() < 1e-12 * scale


# ---------------------------------------------------------------- velocity-based Verlet

def test_velocity_verlet_drift_is_the_marching_interval_mismatch():
    # Section 3.3: with multiple time steps the velocity-based scheme does not
    # conserve momentum, because the fluid applies the coupling force of an
    # evaluation over half of each neighbouring acoustic step while the solid
    # applies it over its own sub-steps.  The force of evaluation n reaches
    # the fluid with weight (dt_n + dt_{n+1})/2 and the solid with weight
    # dt_n - delta_n/2 + delta_{n+1}/2 (delta = dt / kappa); every other force
    # cancels in pairs.  The observed drift must be exactly that mismatch,
    # while the position-based scheme keeps the total to round-off.
    sc = scenes.periodic_box_with_solid(dim=2, n=12, amp=0.3)
    sc["velocity_verlet"] = 1
    o = O.Oracle(sc)
    mf, ms = o.masses()

    def total():
        return mf @ o.get(O.F_V) + ms @ o.get(O.S_V)

    scale = mf @ np.abs(o.get(O.F_V)).sum(1) + ms @ np.abs(o.get(O.S_V)).sum(1)
    p0 = total()
    forces, dts, kaps = [], [], []
    for _ in range(30):
        if o.scalars()["need_rebuild"]:
            o.rebuild()
        o.fluid_step()
        o.couple()
        pair = o.fluid_side_coupling()[:2] + o.totals()["sum_fF"][:2]
        assert np.abs(pair).max() <= 1e-13 * np.abs(o.get(O.S_FF)).sum()
        forces.append(o.totals()["sum_fF"][:2].copy())
        o.solid_substeps()
        s = o.scalars()
        dts.append(s["dt_ac"])
        kaps.append(s["kappa"])
    assert max(kaps) > 1 and len(set(dts)) > 1
    n = len(dts)
    pred = np.zeros(2)
    for k in range(n):
        last = k == n - 1
        w_solid = dts[k] - 0.5 * dts[k] / kaps[k] + (0.0 if last else 0.5 * dts[k + 1] / kaps[k + 1])
        w_fluid = 0.5 * dts[k] + (0.0 if last else 0.5 * dts[k + 1])
        pred += (w_solid - w_fluid) * forces[k]
    drift = total() - p0
    assert np.abs(drift).max() > 1e3 * 1e-13 * scale  # a real drift
    assert np.abs(drift - pred).max() <= 1e-12 * scale
