"""Parity at the benchmark sizes.

The 2D channel (17,444 fluid particles) and all 64 batched dam breaks are small
enough for the FP64 oracle to run whole.  The 3D dam break (2.0M fluid) is
checked on sampled particles: the first-step acceleration of a fluid particle
depends only on particles within 4 h_F of it (its neighbours within 2 h_F and
their own neighbourhoods through the density reinitialisation), so the oracle
runs a crop of radius 4 h_F + dp_F around each sample and must give that
particle the same acceleration as the full GPU run.

The plate of the 3D dam break (354k solid particles, the streamed sub-step
passes on 1,800 lattice blocks) is checked the same way: within one acoustic step a
solid particle's state depends on the solid within 4 h_S per sub-step (its
neighbours' stress, which depends on their neighbours' velocities), so after
kappa sub-steps on the solid within (4 kappa + 2) h_S, and on correct
correction matrices there, 2 h_S further.  The step's kappa depends on the
largest solid speed of the whole plate: a written velocity bump puts that
maximum on one particle deep in the plate's index range, and every crop also
holds that particle, so each crop takes the same kappa as the full run.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1911_13255_amd import scenes, sph

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)


def rel_inf(g, r):
    den = np.abs(r).max()
    return np.abs(g - r).max() / den if den > 0 else np.abs(g - r).max()


FIELDS = ((sph.F_RHO, "rho"), (sph.F_DRHO, "drho"), (sph.F_A, "a_f"), (sph.F_V, "v_f"), (sph.S_U, "u_s"),
          (sph.S_V, "v_s"), (sph.S_VBAR, "vbar"), (sph.S_ABAR, "abar"), (sph.S_A, "a_s"))


def compare_all(sim, o, scene, label, tol=1e-4):
    for f, name in FIELDS:
        r = o.get(f)
        if np.abs(r).max() == 0.0:
            continue
        e = rel_inf(sim.read(f, scene), r)
        assert e <= tol, (label, name, e)


@pytest.mark.parametrize("lpp,block", [(0, 0), (16, 64)])
def test_channel_full_size(gpu, lpp, block):
    sc = scenes.plate_behind_cylinder(seed=1)
    note(f"channel full size {len(sc['x_fluid'])} fluid, lpp {lpp} block {block}")
    sim = sph.Simulation(sc, lanes_per_particle=lpp, block_pair=block)
    o = O.Oracle(sc)
    for k in range(3):
        sim.step()
        o.step(1)
        compare_all(sim, o, 0, f"channel step {k + 1}")
    sim.sync()
    sim.close()


def test_all_64_batched_scenes(gpu):
    scs = scenes.batched_dam_breaks(64)
    note("batched 64 scenes, 2 steps")
    sim = sph.Simulation(scs)
    oras = [O.Oracle(s) for s in scs]
    for k in range(2):
        sim.advance(1)
        for o in oras:
            o.step(1)
    for i, o in enumerate(oras):
        compare_all(sim, o, i, f"scene {i}")
        assert sim.scalars(i)["kappa"] == o.scalars()["kappa"]
    sim.sync()
    sim.close()


def crop(sc, center, radius, extra=()):
    """The scene restricted to the particles within `radius` of `center`, and
    within each (center, radius) of `extra` (order kept, so the clamp block
    stays last)."""
    out = dict(sc)

    def within(x):
        keep = np.linalg.norm(x - center, axis=1) <= radius
        for c, r in extra:
            keep |= np.linalg.norm(x - c, axis=1) <= r
        return np.where(keep)[0]

    fi = within(sc["x_fluid"])
    wi = within(sc["x_wall"])
    si = within(sc["x_solid"])
    n_s = len(sc["x_solid"])
    out["x_fluid"] = sc["x_fluid"][fi]
    out["x_wall"] = sc["x_wall"][wi]
    out["n_wall"] = sc["n_wall"][wi]
    out["x_solid"] = sc["x_solid"][si] if len(si) else np.zeros((0, sc["dim"]))
    out["n_clamp"] = int(np.sum(si >= n_s - int(sc["n_clamp"])))
    out["tip_index"] = 0
    out["_solid_index"] = si
    return out, fi


SOLID_FIELDS = ((sph.S_U, "u_s"), (sph.S_V, "v_s"), (sph.S_F, "F"), (sph.S_DF, "dF"), (sph.S_VBAR, "vbar"),
                (sph.S_ABAR, "abar"), (sph.S_A, "a_s"))


def plate_bump(sc):
    """Velocity bump of 1 m/s on the free plate (Gaussian, 15 mm), its unique
    maximum on the free particle nearest (0.8345, 0.45, 0.2), deep in the plate's
    index range (the last blocks of the solid reductions)."""
    xs = sc["x_solid"]
    nfree = len(xs) - int(sc["n_clamp"])
    p = int(np.argmin(np.linalg.norm(xs[:nfree] - np.array([0.8345, 0.45, 0.2]), axis=1)))
    dirv = np.array([1.0, 0.3, -0.5])
    dirv /= np.linalg.norm(dirv)
    w = np.exp(-np.sum((xs - xs[p]) ** 2, axis=1) / 0.015 ** 2)
    v = w[:, None] * dirv[None, :]
    v[nfree:] = 0.0
    return v, p


def test_dam_break_3d_sampled_first_step(gpu):
    sc = scenes.dam_break_plate_3d(seed=1)
    nf = len(sc["x_fluid"])
    ns = len(sc["x_solid"])
    note(f"3D dam break full size: {nf} fluid, {ns} solid")
    sim = sph.Simulation(sc)
    # the plate's reference configuration is its lattice: the streamed solid
    # passes run on lattice blocks (13 x 200 x 136 cells with the clamp: 4 x
    # 50 x 9 blocks of 4 x 4 x 16)
    tab = sim.solid_table()
    assert tab["compact"] == 1 and tab["lattice_blocks"] == 1800, tab
    assert not sim.solid_register_resident()
    vs, pstar = plate_bump(sc)
    assert pstar > 0.7 * ns
    sim.write(sph.S_V, vs)
    sim.step()
    a_gpu = sim.read(sph.F_A)
    rho_gpu = sim.read(sph.F_RHO)
    solid_gpu = {f: sim.read(f) for f, _ in SOLID_FIELDS}
    kappa_gpu = sim.scalars()["kappa"]
    sim.sync()
    sim.close()
    note(f"3D dam break: GPU step done, kappa {kappa_gpu:.0f}")
    x = sc["x_fluid"]
    rng = np.random.default_rng(2024)
    hf, dpf = sc["h_ratio"] * sc["dp_f"], sc["dp_f"]
    interior = np.where((x[:, 0] > 0.1) & (x[:, 0] < 0.5) & (x[:, 1] > 0.1) & (x[:, 1] < 0.5) &
                        (x[:, 2] > 0.1) & (x[:, 2] < 1.1))[0]
    surface = np.where(x[:, 2] > 1.2 - 2 * dpf)[0]
    walls = np.where((x[:, 0] < 2 * dpf) | (x[:, 2] < 2 * dpf) | (x[:, 1] < 2 * dpf))[0]
    samples = np.concatenate([rng.choice(interior, 8, replace=False), rng.choice(surface, 6, replace=False),
                              rng.choice(walls, 6, replace=False)])
    a_ref, a_smp, rho_ref, rho_smp = [], [], [], []
    for i in samples:
        sub, fi = crop(sc, x[i], 4.0 * hf + dpf)
        o = O.Oracle(sub)
        o.step(1)
        k = int(np.where(fi == i)[0][0])
        a_ref.append(o.get(O.F_A)[k])
        rho_ref.append(o.get(O.F_RHO)[k])
        a_smp.append(a_gpu[i])
        rho_smp.append(rho_gpu[i])
    a_ref, a_smp = np.array(a_ref), np.array(a_smp)
    err_a = np.abs(a_smp - a_ref).max() / max(np.abs(a_ref).max(), 9.81)
    err_rho = np.abs(np.array(rho_smp) - np.array(rho_ref)).max() / np.abs(np.array(rho_ref)).max()
    note(f"3D sampled first step: {len(samples)} samples, acceleration error {err_a:.2e}, density error {err_rho:.2e}")
    assert err_a <= 1e-4
    assert err_rho <= 1e-6
    # the plate: samples at the bump, beside it, at the clamp, the free top
    # edge, a side edge and inside
    xs = sc["x_solid"]
    nfree = ns - int(sc["n_clamp"])
    hs, dps = sc["h_ratio"] * sc["dp_s"], sc["dp_s"]

    def nearest(p):
        return int(np.argmin(np.linalg.norm(xs[:nfree] - np.asarray(p), axis=1)))

    ssamples = [pstar, nearest(xs[pstar] + [0.0, 0.02, 0.01]), nearest([0.8015, 0.3, 0.0015]),
                nearest([0.8385, 0.05, 0.0045]), nearest([0.82, 0.2, 0.3985]), nearest([0.8015, 0.0015, 0.2]),
                int(rng.integers(0, nfree))]
    kap = int(round(kappa_gpu))
    R = (4 * kap + 4) * hs + dps
    ref = {name: [] for _, name in SOLID_FIELDS}
    smp = {name: [] for _, name in SOLID_FIELDS}
    for a in ssamples:
        sub, _ = crop(sc, xs[a], R, extra=((xs[pstar], 1.5 * dps),))
        si = sub.pop("_solid_index")
        o = O.Oracle(sub)
        o.set(O.S_V, vs[si])
        o.step(1)
        assert int(o.scalars()["kappa"]) == kap, (a, o.scalars()["kappa"], kap)
        k = int(np.where(si == a)[0][0])
        for f, name in SOLID_FIELDS:
            r, g = o.get(f)[k], solid_gpu[f][a]
            if f == sph.S_F:
                r, g = r - np.eye(3), g - np.eye(3)
            ref[name].append(r)
            smp[name].append(g)
    errs = {}
    for name in ref:
        r, g = np.array(ref[name]), np.array(smp[name])
        errs[name] = np.abs(g - r).max() / np.abs(r).max()
    note(f"3D plate: {len(ssamples)} samples, kappa {kap}, crop radius {R:.4f} m, errors " +
         ", ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for name, e in errs.items():
        assert e <= 1e-4, (name, e)


@pytest.mark.parametrize("solid_lattice", [True, False])
def test_dam_break_3d_lattice_blocks_match_table(gpu, solid_lattice):
    # The streamed solid passes on lattice blocks and on the reference table
    # sum the same pairs, in class order and in table order (on the jittered
    # plate with each pair's gradient formed in FP32 from its lattice vector
    # and the two offsets, against the table's FP64 gradients rounded to
    # FP32): with a velocity bump in the plate, over three acoustic steps,
    # the whole plate's state agrees to the FP32 rounding of those sums.
    sc = scenes.dam_break_plate_3d(seed=1, solid_lattice=solid_lattice)
    vs, _ = plate_bump(sc)
    out = {}
    for blocks in (0, -1):
        note(f"3D dam break, lattice plate {solid_lattice}, solid_blocks {blocks}")
        sim = sph.Simulation(sc, solid_blocks=blocks)
        assert (sim.solid_table()["lattice_blocks"] > 0) == (blocks == 0)
        sim.write(sph.S_V, vs)
        for _ in range(3):
            sim.step()
        out[blocks] = {name: sim.read(f) for f, name in SOLID_FIELDS}
        out[blocks]["kappa"] = sim.scalars()["kappa"]
        sim.sync()
        sim.close()
    assert out[0]["kappa"] == out[-1]["kappa"] > 1
    errs = {}
    for _, name in SOLID_FIELDS:
        g, r = out[0][name], out[-1][name]
        if name == "F":
            g, r = g - np.eye(3), r - np.eye(3)
        errs[name] = np.abs(g - r).max() / np.abs(r).max()
    note(f"3D plate (lattice {solid_lattice}), lattice blocks against the table: " +
         ", ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for name, e in errs.items():
        assert e <= 1e-5, (name, e)
