"""Pins of the FP64 surrogate-step reference: the coupling force's pressure
part, the reference neighbour count, features of a state at rest, the
neighbour differences of a linear velocity field and of a uniform drift, and
the kinematic identities u_end = u + dt vbar and v_end = v + dt abar of the
plain step when the exact averages are fed back."""
import numpy as np

from oracle import oracle as O
from oracle import surrogate_oracle as SO
from paper_1911_13255_amd import scenes


def test_pressure_part_equals_the_whole_coupling_force_without_viscosity():
    sc = scenes.periodic_box_with_solid(dim=2, n=16, eta=0.0, amp=0.3)
    o = O.Oracle(sc)
    o.step(2)
    assert np.abs(o.get(O.S_FF)).max() > 0
    assert np.array_equal(o.get(O.S_FF), o.get(O.S_FFP))
    sc = scenes.periodic_box_with_solid(dim=2, n=16, eta=2.0, amp=0.3)
    o = O.Oracle(sc)
    o.step(2)
    assert np.abs(o.get(O.S_FF) - o.get(O.S_FFP)).max() > 0


def test_reference_pairs_and_features_at_rest():
    sc = scenes.dam_break_plate(seed=1)
    o = O.Oracle(sc)
    o.rebuild()  # the first step's start: fluid phase and coupling done, the solid at rest
    o.fluid_step()
    o.couple()
    pairs = SO.reference_pairs(sc, o)
    assert sum(len(nb) for nb, _ in pairs) == o.counters()["n_ss"]
    X = SO.features(sc, o, pairs)
    # initial state: F = I, v = a = 0, no fluid contact -> every feature is zero
    assert X.shape == (len(sc["x_solid"]), 24)
    assert np.abs(X).max() == 0.0
    # and the scale is gravity's plus the floor
    s, dt = SO.scales(sc, o, pairs)
    assert np.allclose(s, 9.81 + 1e-3, rtol=1e-15, atol=0) and dt == o.scalars()["dt_ac"]


def _moving_plate():
    sc = scenes.dam_break_plate(seed=1)
    o = O.Oracle(sc)
    o.step(20)
    if o.scalars()["need_rebuild"]:
        o.rebuild()
    o.fluid_step()
    o.couple()
    return sc, o, SO.reference_pairs(sc, o)


def test_features_of_a_linear_velocity_field_and_of_a_uniform_drift():
    sc, o, pairs = _moving_plate()
    x0 = o.get(O.S_X0)
    nfree = len(x0) - int(sc["n_clamp"])
    X = SO.features(sc, o, pairs)
    assert np.abs(X[:nfree, 6:12]).max() > 0  # the state moves and feels the fluid
    # v = A x0: the neighbour mean minus the own value, A (mean x0_b - x0_a),
    # vanishes up to the lattice jitter (|delta x0| <= 1e-4 dp_S) wherever the
    # reference neighbourhood is complete and symmetric (the plate's middle
    # column away from its ends: all 20 lattice points within 2 h_S)
    A = np.array([[0.3, -1.2], [2.0, 0.7]])
    o.set(O.S_V, x0 @ A.T)
    X = SO.features(sc, o, pairs)
    s, dt = SO.scales(sc, o, pairs)
    full = np.array([len(pairs[a][0]) == 20 for a in range(nfree)])
    assert full.sum() >= 20
    dv = X[:nfree, 16:18] * (s[:nfree, None] * dt)  # back to m/s
    bound = np.linalg.norm(A, 2) * 2e-4 * sc["dp_s"]
    assert np.linalg.norm(dv[full], axis=1).max() <= bound
    assert np.linalg.norm(dv[~full], axis=1).max() > 100 * bound
    # a uniform drift added to every velocity moves the own-velocity columns
    # by the drift and leaves every other feature
    drift = np.array([0.25, -0.5])
    o.set(O.S_V, o.get(O.S_V) + drift)
    Y = SO.features(sc, o, pairs)
    assert np.allclose(Y[:nfree, 4:6] - X[:nfree, 4:6], drift, rtol=0, atol=1e-14)
    others = np.r_[0:4, 6:24]
    assert np.allclose(Y[:, others], X[:, others], rtol=1e-12, atol=1e-12 * np.abs(X[:, others]).max())


def _plain_step_and_start(seed=1, steps=30):
    sc = scenes.dam_break_plate(seed=seed)
    o = O.Oracle(sc)
    o.step(steps)
    if o.scalars()["need_rebuild"]:
        o.rebuild()
    o.fluid_step()
    o.couple()
    pairs = SO.reference_pairs(sc, o)
    X = SO.features(sc, o, pairs)
    state = {f: o.get(f).copy() for f in (O.S_U, O.S_V, O.S_A, O.S_F, O.S_DF, O.S_FF, O.S_FFP)}
    dt = o.scalars()["dt_ac"]
    o.solid_substeps()
    end = {f: o.get(f).copy() for f in (O.S_U, O.S_V, O.S_VBAR, O.S_ABAR)}
    for f, val in state.items():  # back to the step start
        o.set(f, val)
    o.set_scalars({"dt_ac": dt})
    return sc, o, pairs, X, end, dt


def test_exact_averages_reproduce_the_plain_step_end_and_pass_the_judge():
    # Fed back as the network's output, the exact averages of the plain
    # sub-steps reproduce the plain step end (u + dt vbar, v + dt abar: the
    # averages' definition) and give a judge residual of exactly 0, so a
    # judge step passes them at any threshold.
    sc, o, pairs, X, end, dt = _plain_step_and_start()
    u0 = o.get(O.S_U)
    nfree = len(u0) - int(sc["n_clamp"])
    vbar, abar = end[O.S_VBAR], end[O.S_ABAR]
    assert np.abs(abar[:nfree]).max() > 0 and np.abs(vbar[:nfree]).max() > 0
    y = SO.targets(sc, o, pairs, vbar, abar)
    s, _ = SO.scales(sc, o, pairs)
    assert np.abs(y[:nfree]).max() < 1e3 * np.abs(y[:nfree]).mean()  # of one size
    r = SO.learned_step(sc, o, pairs, y, np.zeros(4), np.ones(4))
    ue, ve = end[O.S_U], end[O.S_V]
    assert np.allclose(r["u"][:nfree], ue[:nfree], rtol=0, atol=1e-15 + 1e-12 * np.abs(ue).max())
    assert np.allclose(r["v"][:nfree], ve[:nfree], rtol=0, atol=1e-15 + 1e-12 * np.abs(ve).max())
    vp, ap = SO.predicted_averages(sc, o, pairs, y, np.zeros(4), np.ones(4))
    assert SO.judge_residual(sc, vp, ap, vbar, abar, dt) < 1e-14


def test_judge_residual_measures_relative_error():
    # A uniform relative error eps in the predicted acceleration gives
    # R = eps |abar| / (|abar| + |g| sqrt(N)) <= eps; in the velocity likewise.
    sc, o, pairs, X, end, dt = _plain_step_and_start()
    vbar, abar = end[O.S_VBAR], end[O.S_ABAR]
    nfree = len(vbar) - int(sc["n_clamp"])
    g = 9.81
    for eps in (1e-4, 1e-2):
        R = SO.judge_residual(sc, vbar, abar * (1 + eps), vbar, abar, dt)
        na = np.linalg.norm(abar[:nfree])
        assert abs(R - eps * na / (na + g * np.sqrt(nfree))) < 1e-9 * eps
        R = SO.judge_residual(sc, vbar * (1 - eps), abar, vbar, abar, dt)
        nv = np.linalg.norm(vbar[:nfree])
        assert abs(R - eps * nv / (nv + g * dt * np.sqrt(nfree))) < 1e-9 * eps
