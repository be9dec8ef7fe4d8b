"""Magnitude pins of the oracle's pair sums against closed forms.

The rigid-motion, sign and invariant tests elsewhere cannot see a doubled or
dropped factor in a pair sum.  Here each sum is evaluated on an unjittered
lattice whose interior has a full kernel support, with g = 0 and uniform
reference density, for a field whose exact response is known:

- continuity (Section 3.1, the fluid mass equation) under a uniform expansion;
- the fluid viscous term (Section 3.1, the fluid momentum equation) under a
  parabolic shear;
- the fluid pressure term under a linear pressure field;
- the wall coupling terms (Section 2.2, forces of a solid on the fluid) against
  the fluid terms they mirror;
- the solid stress divergence (Section 3.1, the solid momentum equation at h_S)
  under a linearly varying stretch and shear;
- the unsaturated branch of the Riemann limiter (Section 2.2);
- density reinitialisation mode 2 and the viscous bound of the advection step
  (Section 3.2).

Each docstring names the mistakes it catches.  The lattice moment
A = sum_b V_b (r_b - r_a) (x) grad_a W_ab that several closed forms contain is
summed here over an integer lattice with the oracle's kernel derivative, which
the kernel tests pin by quadrature and finite differences.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1911_13255_amd import scenes

H_RATIO = 1.3


def lattice_moment(d, h_ratio=H_RATIO):
    """A of an unbounded lattice of unit spacing and unit volume (dimensionless)."""
    R = int(math.ceil(2 * h_ratio)) + 1
    ks = np.arange(-R, R + 1)
    pts = np.stack(np.meshgrid(*([ks] * d), indexing="ij"), -1).reshape(-1, d).astype(float)
    A = np.zeros((d, d))
    for p in pts:
        r = float(np.linalg.norm(p))
        if r == 0.0:
            continue
        dW = O.kernel_dW(d, r, h_ratio)
        # r_b - r_a = p and grad_a W_ab = e_ab dW/dr with e_ab = (r_a - r_b)/r = -p/r
        A += np.outer(p, -p / r * dW)
    return A


def test_lattice_moment_is_isotropic():
    # the values of the scratch computation quoted with the lattice constants
    for d, a in ((2, 0.97392148), (3, 0.97889584)):
        A = lattice_moment(d)
        assert np.abs(A - a * np.eye(d)).max() < 5e-8


def _fluid_block(dim, n, dp=0.01, eta=0.0, c=10.0, vel=None, walls=None, periodic_x=False):
    """An unjittered fluid lattice of n^dim particles (n[0] x n[1] x ... when n
    is a tuple) at rest or with velocity vel(x), g = 0, rho = rho0, optionally
    over wall layers (positions, normals)."""
    sc = scenes.solid_block(dim=dim)
    nn = (n,) * dim if np.isscalar(n) else tuple(n)
    hi = np.array([nn[k] * dp for k in range(dim)])
    x = scenes.lattice(np.zeros(dim), hi, dp)
    sc.update(dp_f=dp, dp_s=dp, rho0_f=1000.0, c_f=c, eta=eta, g=np.zeros(3), hydro_H=0.0,
              u_ref=c / 10.0, name="fluid_block")
    sc["x_fluid"] = x
    sc["v_fluid"] = None if vel is None else np.ascontiguousarray(vel(x), dtype=np.float64)
    sc["x_solid"] = np.zeros((0, dim))
    sc["n_clamp"] = 0
    sc["tip_index"] = -1
    if walls is None:
        sc["x_wall"], sc["n_wall"] = np.zeros((0, dim)), np.zeros((0, dim))
    else:
        sc["x_wall"], sc["n_wall"] = walls
    sc["lo"] = np.full(3, -0.1)
    sc["hi"] = np.full(3, 1.0)
    sc["lo"][:dim] = -0.1
    sc["hi"][:dim] = hi + 0.1
    if periodic_x:
        sc["lo"][0], sc["hi"][0] = 0.0, hi[0]
        sc["periodic"] = np.array([1, 0, 0], dtype=np.int32)
    return sc


def _inner(x, n, dp, layers):
    """Particles at least `layers` lattice rows from every face of the block."""
    nn = np.full(x.shape[1], n) if np.isscalar(n) else np.asarray(n)
    idx = np.rint(x / dp - 0.5).astype(int)
    return np.all((idx >= layers) & (idx <= nn - 1 - layers), axis=1)


def _first_step(sc, riemann=1, reinit=0):
    o = O.Oracle(sc, riemann=bool(riemann), density_reinit=reinit)
    o.step(1)
    return o


# ------------------------------------------------------------------ continuity

@pytest.mark.parametrize("d,riemann", [(2, 1), (2, 0), (3, 1)])
def test_continuity_of_a_uniform_expansion(d, riemann):
    """v = alpha (x - x_c): drho/dt = -rho0 alpha tr(A) exactly in the interior.

    At uniform pressure the interface velocity is the pair average, so
    v_i - v* = alpha r_ij / 2 and the sum 2 rho_i sum_j V_j (v_i - v*).grad_i W
    equals rho_i alpha sum_j V_j r dW/dr = -rho0 alpha tr(A).  The expansion
    keeps the Riemann pressure at the average (no compression), so the fluid
    does not accelerate.  Catches: the factor 2 dropped or doubled, the sign
    flipped, V_j or rho_i dropped, v_i - v_j in place of v_i - v*.
    """
    n = 16 if d == 2 else 10
    dp, alpha = 0.01, 0.05
    xc = 0.5 * n * dp
    sc = _fluid_block(d, n, dp, vel=lambda x: alpha * (x - xc))
    o = _first_step(sc, riemann)
    drho = o.get(O.F_DRHO)
    inner = _inner(sc["x_fluid"], n, dp, 3)
    assert inner.sum() >= 16
    expect = -1000.0 * alpha * np.trace(lattice_moment(d))
    assert np.abs(drho[inner] - expect).max() < 1e-10 * abs(expect)
    assert np.abs(o.get(O.F_A)).max() < 1e-12


def test_continuity_wall_term_mirrors_the_fluid_term():
    """A wall at rest under fluid moving with U adds rho_i V_a (v_i - 0).grad W
    per wall particle; the same lattice with the walls replaced by fluid at rest
    gives 2 rho_i V_j (v_i - (v_i + 0)/2).grad W, the identical number.

    Catches: the wall term (the continuity reading for walls and solid) dropped,
    doubled, sign-flipped, or without V_a.
    """
    d, dp, nx, ny = 2, 0.01, 12, 10
    U = np.array([0.02, -0.015])
    wall_x = scenes.lattice([0.0, -3 * dp], [nx * dp, 0.0], dp)
    wall_n = np.tile([0.0, 1.0], (len(wall_x), 1))
    a = _fluid_block(d, (nx, ny), dp, vel=lambda x: np.tile(U, (len(x), 1)), walls=(wall_x, wall_n),
                     periodic_x=True)
    b = _fluid_block(d, (nx, ny), dp, periodic_x=True)
    xb = np.concatenate([b["x_fluid"], wall_x])
    vb = np.concatenate([np.tile(U, (len(b["x_fluid"]), 1)), np.zeros_like(wall_x)])
    b["x_fluid"], b["v_fluid"] = xb, vb
    oa, ob = _first_step(a, riemann=0), _first_step(b, riemann=0)
    nf = len(a["x_fluid"])
    da, db = oa.get(O.F_DRHO), ob.get(O.F_DRHO)[:nf]
    near = a["x_fluid"][:, 1] < 2.0 * dp  # the two rows within 2h of a wall particle
    assert np.abs(da[near]).min() > 1e-3
    assert np.abs(da - db).max() < 1e-12 * np.abs(db).max()


# ------------------------------------------------------------------ fluid momentum

@pytest.mark.parametrize("d", [2, 3])
def test_viscous_term_of_a_parabolic_shear(d):
    """v = (beta y^2, 0): a_x = 2 eta beta A_yy / rho0 in the interior
    (the continuum eta nabla^2 v / rho0 = 2 eta beta / rho0 times the lattice
    moment).

    With simple averages the pressure stays zero.  Catches: the factor 2
    dropped or doubled, the sign flipped, V_j dropped, 1/r_ij dropped or
    squared, v_j - v_i in place of v_i - v_j.
    """
    n = 16 if d == 2 else 10
    dp, eta, beta = 0.01, 0.02, 3.0

    def vel(x):
        v = np.zeros_like(x)
        v[:, 0] = beta * x[:, 1] ** 2
        return v

    sc = _fluid_block(d, n, dp, eta=eta, vel=vel)
    o = _first_step(sc, riemann=0)
    a = o.get(O.F_A)
    inner = _inner(sc["x_fluid"], n, dp, 3)
    A = lattice_moment(d)
    expect = 2.0 * eta * beta * A[1, 1] / 1000.0
    assert np.abs(a[inner, 0] - expect).max() < 1e-9 * expect
    assert np.abs(a[inner, 1:]).max() < 1e-9 * expect


@pytest.mark.parametrize("riemann", [0, 1])
def test_pressure_term_of_a_linear_pressure_field(riemann):
    """p = p_c + G.(x - x_c) at rest: a = -A G / rho in the interior.

    sum_j V_j (p_i + p_j) grad_i W over a full support is A^T G; the density
    follows p through the equation of state, so the volumes vary by a part in
    1e6 and the bar is 1e-5.  Catches: the factor 2 dropped or doubled, the
    sign flipped, V_i V_j / m_i replaced by anything else, the Riemann pressure
    not reducing to the average for a pair at rest.
    """
    d, n, dp, c = 2, 16, 0.01, 10.0
    G = np.array([0.35, -0.2])
    sc = _fluid_block(d, n, dp, c=c)
    o = O.Oracle(sc, riemann=bool(riemann), density_reinit=0)
    x = sc["x_fluid"]
    p = (x - 0.5 * n * dp) @ G
    rho = np.array([O.eos_inv(q, 1000.0, c) for q in p])
    o.set(O.F_RHO, rho)
    o.step(1)
    a = o.get(O.F_A)
    inner = _inner(x, n, dp, 3)
    expect = -(lattice_moment(d) @ G)[None, :] / rho[inner, None]
    assert np.abs(a[inner] - expect).max() < 1e-5 * np.abs(expect).max()


def _wall_pair(U, eta, rho=1000.0, c=10.0):
    """Fluid over three wall layers (A) and the same lattice with the walls
    replaced by fluid (B) and with no walls at all (C); returns the three
    first-step accelerations of the original fluid particles and their
    positions."""
    d, dp, nx, ny = 2, 0.01, 12, 10
    wall_x = scenes.lattice([0.0, -3 * dp], [nx * dp, 0.0], dp)
    wall_n = np.tile([0.0, 1.0], (len(wall_x), 1))
    a = _fluid_block(d, (nx, ny), dp, eta=eta, c=c, walls=(wall_x, wall_n), periodic_x=True,
                     vel=lambda x: np.tile(U, (len(x), 1)))
    b = _fluid_block(d, (nx, ny), dp, eta=eta, c=c, periodic_x=True)
    b["x_fluid"] = np.concatenate([b["x_fluid"], wall_x])
    b["v_fluid"] = np.concatenate([np.tile(U, (nx * ny, 1)), np.tile(-np.asarray(U), (len(wall_x), 1))])
    cc = _fluid_block(d, (nx, ny), dp, eta=eta, c=c, periodic_x=True, vel=lambda x: np.tile(U, (len(x), 1)))
    out = []
    for sc in (a, b, cc):
        o = O.Oracle(sc, riemann=False, density_reinit=0)
        if rho != 1000.0:
            o.set(O.F_RHO, np.full(len(sc["x_fluid"]), rho))
        o.step(1)
        out.append(o.get(O.F_A)[: nx * ny])
    return out[0], out[1], out[2], a["x_fluid"]


def test_wall_viscous_term_mirrors_the_fluid_term():
    """Fluid sliding with U over a wall at rest feels
    2 eta V_a (v_i - v_d) / (r + 0.01 h) dW/dr per wall particle, with the
    imaginary velocity v_d = 2 vbar - v_i = -U.  Replacing the walls by fluid
    moving with -U gives the same terms with 1/r in place of 1/(r + 0.01 h), so
    the ratio lies in (r_min/(r_min + 0.01 h), 1) and is below 1.

    Catches: the wall viscous term doubled, halved, sign-flipped or without
    V_a; the printed imaginary velocity 2 v_i - vbar (ratio -1/2); the
    regulariser 0.01 h dropped (ratio exactly 1).
    """
    U = np.array([0.05, 0.0])
    aw, af, _, x = _wall_pair(U, eta=0.05)
    dp, h = 0.01, 0.013
    first = x[:, 1] < dp
    ratio = aw[first, 0] / af[first, 0]
    assert np.all(af[first, 0] < 0.0)
    assert np.all(ratio > dp / (dp + 0.01 * h)) and np.all(ratio < 1.0 - 1e-4)
    near = x[:, 1] < 2.0 * dp  # the two rows within 2h of a wall particle
    r2 = aw[near, 0] / af[near, 0]
    assert np.all(r2 > dp / (dp + 0.01 * h)) and np.all(r2 < 1.0)


def test_wall_pressure_term_mirrors_the_fluid_term():
    """At a uniform pressure p above walls at rest (g = 0), the imaginary
    pressure is p and the imaginary density rho, so a wall particle pushes with
    -2 V_i V_a p grad W / m_i, where the fluid it replaces pushes with
    -2 V_i V_j p grad W / m_i.  With V_a = dp^d and V_j = m_j / rho, the two
    wall-side contributions (each taken against the same lattice without the
    wall layers) differ by the factor rho / rho0 exactly.

    Catches: the wall pressure term doubled, sign-flipped or without V_a; the
    density-weighted pressure average wrong.
    """
    rho = 1003.0
    aw, af, a0, x = _wall_pair(np.zeros(2), eta=0.0, rho=rho)
    near = x[:, 1] < 0.02  # the two rows within 2h of a wall particle
    ww = aw[near] - a0[near]
    wf = af[near] - a0[near]
    assert np.abs(wf[:, 1]).min() > 1.0
    assert np.abs(ww - (rho / 1000.0) * wf).max() < 1e-9 * np.abs(wf).max()


# ------------------------------------------------------------------ solid momentum

def _stress_divergence(d, eps, mode):
    n = 14
    dp, rho_s, E, nu = 0.01, 1000.0, 1.0e6, 0.3
    sc = scenes.solid_block(dim=d, n=(n, n, n), dp=dp, E=E, nu=nu, rho_s=rho_s)
    o = O.Oracle(sc)
    x0 = o.get(O.S_X0)
    xc = 0.5 * n * dp
    ns = len(x0)
    F = np.broadcast_to(np.eye(d), (ns, d, d)).copy()
    u = np.zeros((ns, d))
    if mode == "stretch":  # u_x = eps (x - xc)^2 / 2
        s = x0[:, 0] - xc
        u[:, 0] = 0.5 * eps * s * s
        F[:, 0, 0] += eps * s
    else:  # shear: u_x = eps (y - xc)^2 / 2
        s = x0[:, 1] - xc
        u[:, 0] = 0.5 * eps * s * s
        F[:, 0, 1] += eps * s
    o.set(O.S_F, F)
    o.set(O.S_U, u)
    o.rebuild()
    o.fluid_step()
    o.couple()
    o.set_scalars({"dt_ac": 1e-12})
    o.solid_substeps()
    sc_ = o.scalars()
    inner = _inner(x0, n, dp, 5)  # neighbours of the sample have full supports too
    return o.get(O.S_A)[inner], sc_["mu"], sc_["lam"], rho_s


@pytest.mark.parametrize("d", [2, 3])
def test_stress_divergence_of_a_linearly_varying_stretch(d):
    """F = I + eps (x - x_c) e_x e_x: a_x -> (lambda + 2 mu) eps / rho0_S as
    eps -> 0, with a relative error of order eps (the Neo-Hookean stress is
    linear in the strain to first order; the corrected sum differentiates a
    linear stress field exactly where the neighbours' B are uniform).

    Catches: the sum (P_a B_a + P_b B_b) doubled or halved, a volume dropped,
    the sign flipped, the mass in place of the volume.
    """
    errs = []
    for eps in (1e-3, 1e-4):
        a, mu, lam, rho_s = _stress_divergence(d, eps, "stretch")
        k = (lam + 2 * mu) * eps / rho_s
        assert a.shape[0] >= 16
        rel = np.abs(a[:, 0] / k - 1.0).max()
        assert rel < 20 * eps
        assert np.abs(a[:, 1:]).max() < 1e-6 * k
        errs.append(rel)
    # first-order relative error: it falls with eps
    assert errs[1] < 0.2 * errs[0]


def test_stress_divergence_of_a_linearly_varying_shear():
    """F = I + eps (y - y_c) e_x e_y: a_x -> mu eps / rho0_S (the shear modulus
    alone), a_y -> 0.  Catches a wrong modulus combination or a dropped term of
    P = F S that the stretch test does not separate."""
    for d in (2, 3):
        eps = 1e-4
        a, mu, lam, rho_s = _stress_divergence(d, eps, "shear")
        k = mu * eps / rho_s
        assert np.abs(a[:, 0] / k - 1.0).max() < 20 * eps
        assert np.abs(a[:, 1:]).max() < 1e-3 * k


# ------------------------------------------------------------------ Riemann limiter (Section 2.2)

def test_riemann_limiter_below_saturation():
    """For 0 < U_L - U_R < c/3 the dissipation coefficient is 3 (U_L - U_R), so
    P* - pbar = 1.5 rhobar (U_L - U_R)^2: quadratic in the approach speed
    (doubling it multiplies the excess by 4), continuous with the saturated
    linear branch at c/3, and U* unaffected.  Catches: a factor 3 or 1/2
    dropped, min in place of max, the limiter applied to separating pairs."""
    c, ri, rj, pi_, pj = 12.0, 1000.0, 1006.0, 80.0, 20.0
    e = np.array([0.6, 0.8])
    rb, pbar = 0.5 * (ri + rj), 0.5 * (pi_ + pj)

    def excess(dU):
        # v_i approaches j along -e: U_L - U_R = -(v_i - v_j).e = dU
        vi, vj = -0.5 * dU * e, 0.5 * dU * e
        P, vs = O.riemann(2, ri, rj, pi_, pj, vi, vj, e, c=c)
        return P - pbar, vs

    for dU in (0.01, 0.7, c / 6.0, 0.99 * c / 3.0):
        ex, vs = excess(dU)
        assert abs(ex - 1.5 * rb * dU * dU) < 1e-12 * max(1.0, rb * dU * dU)
        # the interface velocity carries only the pressure-difference term
        us = -(vs @ e)
        assert abs(us - (pi_ - pj) / (2 * rb * c)) < 1e-14
    assert abs(excess(1.0)[0] / excess(0.5)[0] - 4.0) < 1e-12
    # the saturated branch continues the same value at c/3 and then grows linearly
    lo, hi = excess(c / 3.0 * (1 - 1e-12))[0], excess(c / 3.0 * (1 + 1e-12))[0]
    assert abs(hi - lo) < 1e-6 * hi
    assert abs(excess(c)[0] - 0.5 * rb * c * c) < 1e-9 * rb * c * c
    # separating pairs: no dissipation
    assert excess(-0.5)[0] == 0.0


# ------------------------------------------------------------------ density reinitialisation and dt_ad (Section 3.2)

def test_density_reinit_mode_2_keeps_the_compressed_continuity_density():
    """Mode 2: rho = max(rho, rho0 psi/psi0).  On the exact lattice at rest
    (psi = psi0 wherever the support is full) the hydrostatic densities, all
    >= rho0, are kept bit for bit, and at the free surface (psi < psi0) too,
    where mode 1 sets rho0; a lattice compressed by 1% lifts the interior to
    rho0 psi/psi0, the value of mode 1.  Catches: min in place of max, psi0/psi
    in place of psi/psi0, mode 1's clip applied."""
    sc = scenes.hydrostatic_column(seed=None)
    o0 = O.Oracle(sc, density_reinit=0)
    rho_init = o0.get(O.F_RHO)
    o2 = O.Oracle(sc, density_reinit=2)
    o2.rebuild()
    assert np.array_equal(o2.get(O.F_RHO), rho_init)
    assert rho_init.min() >= 1000.0 and rho_init.max() > 1000.0 * 1.004
    o1 = O.Oracle(sc, density_reinit=1)
    o1.rebuild()
    top = sc["x_fluid"][:, 1] > 0.4 - 0.01
    assert np.any(rho_init[top] > 1000.0) and np.all(o1.get(O.F_RHO)[top] == 1000.0)
    sc2 = scenes.hydrostatic_column(seed=None)
    sc2["x_fluid"] = sc2["x_fluid"] * 0.99
    o2c, o1c = O.Oracle(sc2, density_reinit=2), O.Oracle(sc2, density_reinit=1)
    o2c.rebuild()
    o1c.rebuild()
    x = sc2["x_fluid"]
    inner = (x[:, 0] > 0.05) & (x[:, 0] < 0.15) & (x[:, 1] > 0.05) & (x[:, 1] < 0.3)
    r2, r1 = o2c.get(O.F_RHO)[inner], o1c.get(O.F_RHO)[inner]
    assert np.all(r1 > 1000.0 * 1.015)
    # the two modes round rho0 psi / psi0 in different orders
    ref = np.maximum(r1, O.Oracle(sc2, density_reinit=0).get(O.F_RHO)[inner])
    assert np.abs(r2 - ref).max() < 1e-13 * 1000.0


def test_advection_step_viscous_bound_uses_the_kinematic_viscosity():
    """dt_ad = CFL_ad min(h/|v|max, h^2 rho0/eta): with a strong viscosity the
    second bound binds at the hand value 0.25 * 0.013^2 * 1000 / 100; scaling
    rho0 and eta together leaves it unchanged (it depends on eta/rho0 only),
    doubling eta halves it, and eta = 0 drops it.  Catches: h^2/eta (the
    printed dimensionally inconsistent form), a missing CFL factor, max in place
    of min."""
    def dt_ad(eta, rho0=1000.0):
        sc = scenes.hydrostatic_layer(seed=None)
        sc["eta"] = eta
        sc["rho0_f"] = rho0
        o = O.Oracle(sc)
        o.rebuild()
        return o.scalars()["dt_ad"]

    h = 1.3 * 0.01
    assert abs(dt_ad(100.0) - 0.25 * h * h * 1000.0 / 100.0) < 1e-15
    assert abs(dt_ad(400.0, rho0=4000.0) - dt_ad(100.0)) < 1e-15
    assert abs(dt_ad(200.0) - 0.5 * dt_ad(100.0)) < 1e-15
    c0 = 10.0 * math.sqrt(2 * 9.81 * 0.4)
    assert abs(dt_ad(0.0) - 0.25 * h / (c0 / 10.0)) < 1e-15
    # a weak viscosity does not bind
    assert dt_ad(1e-3) == dt_ad(0.0)
