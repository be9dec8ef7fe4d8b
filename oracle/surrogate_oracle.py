"""FP64 reference of the learned sub-step surrogate's per-particle arithmetic
(test infrastructure only).

TEST INFRASTRUCTURE ONLY: only the tests may import it; the product path never
does.  It shares no code with the GPU library and works on the FP64 oracle's
state (oracle.Oracle) between `couple` and `solid_substeps` of a 2D scene.

Definitions (the paper has no learned part; Sections 2.1, 2.2 and 3.2 give the
quantities involved):
  own values of a free solid particle: F - I (4, row-major), v, a, the
  pressure part fp and the viscous part fv of the coupling force (12);
  their plain mean over its reference neighbours (|r0_ab| < 2 h_S, b != a;
  the own values when it has none);
  the row's acceleration scale s = |a| + |mean a| + |g| + |fp + fv| / m + s0
  with m = rho0_S V_S and s0 = 1e-3 m/s^2, and dt the acoustic step;
  features (24): F - I, v, a / s, fp / (m s), fv / (m s), then the
  neighbour mean minus the own value of each of the 12, the velocity's
  divided by s dt, the acceleration's by s, the forces' by m s, F's as is
  (the same information as the own values and their means, scaled so that
  quiet and violent states give features and targets of one size);
  training targets: ((vbar - v) / (s dt), (abar - a) / s);
  the network output y (standardised) gives, with d = y std + mean,
  vbar = v + s dt d_v and abar = a + s d_a;
  a learned step: dF/dt = sum_b (vbar_b - vbar_a) (x) (B_a V_b grad0 W_ab),
  F_end = F + dt dF/dt, u_end = u + dt vbar, v_end = v + dt abar, and the
  stored acceleration becomes abar;
  a judge step compares the predicted averages with those of the plain
  sub-steps over the N free particles,
    R = max(|vbar_pred - vbar|_2 / (|vbar|_2 + |g| dt sqrt(N)),
            |abar_pred - abar|_2 / (|abar|_2 + |g| sqrt(N))),
  and passes when R <= threshold.
"""
import numpy as np

from oracle import oracle as O


def scene_constants(sc):
    nu, E = sc["nu"], sc["E"]
    return dict(hs=sc["h_ratio"] * sc["dp_s"], Vs=sc["dp_s"] ** 2, rho0s=sc["rho0_s"],
                mu=E / (2.0 * (1.0 + nu)), lam=E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu)),
                g=np.array(sc["g"][:2], dtype=np.float64), nclamp=int(sc["n_clamp"]))


def reference_pairs(sc, o):
    """Neighbour lists and V_b grad0_a W_ab of the reference configuration, by brute force."""
    k = scene_constants(sc)
    x0 = o.get(O.S_X0)
    ns = len(x0)
    out = []
    for a in range(ns):
        r = x0[a] - x0
        dist = np.linalg.norm(r, axis=1)
        nb = np.where((dist < 2.0 * k["hs"]) & (np.arange(ns) != a))[0]
        gr = np.array([k["Vs"] * r[b] / dist[b] * O.kernel_dW(2, dist[b], k["hs"]) for b in nb]).reshape(-1, 2)
        out.append((nb, gr))
    return out


def own_features(o):
    F = o.get(O.S_F)
    own = np.zeros((len(F), 12))
    own[:, 0:4] = (F - np.eye(2)).reshape(-1, 4)
    own[:, 4:6] = o.get(O.S_V)
    own[:, 6:8] = o.get(O.S_A)
    fp = o.get(O.S_FFP)
    own[:, 8:10] = fp
    own[:, 10:12] = o.get(O.S_FF) - fp
    return own


SCALE_FLOOR = 1e-3  # s0, m/s^2


def own_and_means(sc, o, pairs):
    """Own values (n_solid x 12) and their neighbour means (own values where a
    particle has no neighbour); rows of the free particles only matter."""
    own = own_features(o)
    means = own.copy()
    nfree = len(own) - int(sc["n_clamp"])
    for a in range(nfree):
        nb, _ = pairs[a]
        if len(nb):
            means[a] = own[nb].mean(axis=0)
    return own, means


def scales(sc, o, pairs):
    """(s, dt): the acceleration scale of every solid particle (see the module
    docstring) and the acoustic step."""
    k = scene_constants(sc)
    own, means = own_and_means(sc, o, pairs)
    m = k["rho0s"] * k["Vs"]
    s = (np.linalg.norm(own[:, 6:8], axis=1) + np.linalg.norm(means[:, 6:8], axis=1) + np.linalg.norm(k["g"])
         + np.linalg.norm(own[:, 8:10] + own[:, 10:12], axis=1) / m + SCALE_FLOOR)
    return s, o.scalars()["dt_ac"]


def features(sc, o, pairs):
    """(n_solid, 24) raw features, clamp rows zero."""
    k = scene_constants(sc)
    own, means = own_and_means(sc, o, pairs)
    s, dt = scales(sc, o, pairs)
    m = k["rho0s"] * k["Vs"]
    diff = means - own
    X = np.zeros((len(own), 24))
    X[:, 0:4] = own[:, 0:4]
    X[:, 4:6] = own[:, 4:6]
    X[:, 6:8] = own[:, 6:8] / s[:, None]
    X[:, 8:12] = own[:, 8:12] / (m * s[:, None])
    X[:, 12:16] = diff[:, 0:4]
    X[:, 16:18] = diff[:, 4:6] / (s[:, None] * dt)
    X[:, 18:20] = diff[:, 6:8] / s[:, None]
    X[:, 20:24] = diff[:, 8:12] / (m * s[:, None])
    X[len(own) - k["nclamp"]:] = 0.0
    return X


def targets(sc, o_start, pairs, vbar, abar):
    """Training targets of the free particles, ((vbar - v) / (s dt),
    (abar - a) / s), from the step-start state o_start and the averages of
    the plain sub-steps; clamp rows zero."""
    s, dt = scales(sc, o_start, pairs)
    v0, a0 = o_start.get(O.S_V), o_start.get(O.S_A)
    nfree = len(v0) - int(sc["n_clamp"])
    T = np.zeros((len(v0), 4))
    T[:nfree, 0:2] = (vbar[:nfree] - v0[:nfree]) / (s[:nfree, None] * dt)
    T[:nfree, 2:4] = (abar[:nfree] - a0[:nfree]) / s[:nfree, None]
    return T


def predicted_averages(sc, o, pairs, y, out_mean, out_std):
    """(vbar, abar) from standardised network outputs y (n_solid x 4), clamp
    rows zero."""
    nfree = len(y) - int(sc["n_clamp"])
    v0, a0 = o.get(O.S_V), o.get(O.S_A)
    s, dt = scales(sc, o, pairs)
    d = y * out_std + out_mean
    vbar = np.zeros((len(y), 2))
    abar = np.zeros((len(y), 2))
    vbar[:nfree] = v0[:nfree] + (s[:nfree] * dt)[:, None] * d[:nfree, 0:2]
    abar[:nfree] = a0[:nfree] + s[:nfree, None] * d[:nfree, 2:4]
    return vbar, abar


def learned_step(sc, o, pairs, y, out_mean, out_std):
    """The state a learned step ends at, from standardised outputs y."""
    k = scene_constants(sc)
    dt = o.scalars()["dt_ac"]
    F0, u0, v0, B = o.get(O.S_F), o.get(O.S_U), o.get(O.S_V), o.get(O.S_B)
    ns = len(F0)
    nfree = ns - k["nclamp"]
    vbar, abar = predicted_averages(sc, o, pairs, y, out_mean, out_std)
    Fend = F0.copy()
    dFs = np.zeros_like(F0)
    for a in range(nfree):
        nb, gr = pairs[a]
        G = np.zeros((2, 2))
        for b, gg in zip(nb, gr):
            G += np.outer(vbar[b] - vbar[a], gg)
        dFs[a] = G @ B[a].T
        Fend[a] = F0[a] + dt * dFs[a]
    u, v = u0.copy(), v0.copy()
    u[:nfree] += dt * vbar[:nfree]
    v[:nfree] += dt * abar[:nfree]
    a = o.get(O.S_A).copy()
    a[:nfree] = abar[:nfree]
    return dict(vbar=vbar, abar=abar, F=Fend, dF=dFs, u=u, v=v, a=a)


def judge_residual(sc, vbar_pred, abar_pred, vbar, abar, dt):
    """R of a judge step over the free particles (see the module docstring)."""
    k = scene_constants(sc)
    nfree = len(vbar) - k["nclamp"]
    g = np.linalg.norm(k["g"])
    rn = np.sqrt(max(nfree, 1))
    rv = np.linalg.norm(vbar_pred[:nfree] - vbar[:nfree]) / (np.linalg.norm(vbar[:nfree]) + g * dt * rn + 1e-300)
    ra = np.linalg.norm(abar_pred[:nfree] - abar[:nfree]) / (np.linalg.norm(abar[:nfree]) + g * rn + 1e-300)
    return max(rv, ra)
