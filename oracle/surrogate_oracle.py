"""FP64 reference of the learned sub-step surrogate's per-particle arithmetic
(test infrastructure only).

TEST INFRASTRUCTURE ONLY: only the tests may import it; the product path never
does.  It shares no code with the GPU library and works on the FP64 oracle's
state (oracle.Oracle) between `couple` and `solid_substeps` of a 2D scene.

Definitions (the paper has no learned part; Sections 2.1, 2.2 and 3.2 give the
quantities involved):
  features of a free solid particle: F - I (4, row-major), v, a, the pressure
  and viscous parts of the coupling force, then the plain mean of these 12
  values over its reference neighbours (|r0_ab| < 2 h_S, b != a);
  the network output y (standardised) gives vbar = v + y_v std + mean and
  abar = a + y_a std + mean;
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


def features(sc, o, pairs):
    """(n_solid, 24) raw features, clamp rows zero."""
    own = own_features(o)
    ns = len(own)
    nfree = ns - int(sc["n_clamp"])
    X = np.zeros((ns, 24))
    for a in range(nfree):
        nb, _ = pairs[a]
        X[a, :12] = own[a]
        X[a, 12:] = own[nb].mean(axis=0) if len(nb) else 0.0
    return X


def predicted_averages(sc, o, y, out_mean, out_std):
    """(vbar, abar) from standardised network outputs y (n_solid x 4), clamp
    rows zero."""
    nfree = len(y) - int(sc["n_clamp"])
    v0, a0 = o.get(O.S_V), o.get(O.S_A)
    d = y * out_std + out_mean
    vbar = np.zeros((len(y), 2))
    abar = np.zeros((len(y), 2))
    vbar[:nfree] = v0[:nfree] + d[:nfree, 0:2]
    abar[:nfree] = a0[:nfree] + d[:nfree, 2:4]
    return vbar, abar


def learned_step(sc, o, pairs, y, out_mean, out_std):
    """The state a learned step ends at, from standardised outputs y."""
    k = scene_constants(sc)
    dt = o.scalars()["dt_ac"]
    F0, u0, v0, B = o.get(O.S_F), o.get(O.S_U), o.get(O.S_V), o.get(O.S_B)
    ns = len(F0)
    nfree = ns - k["nclamp"]
    vbar, abar = predicted_averages(sc, o, y, out_mean, out_std)
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
