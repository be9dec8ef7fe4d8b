"""Seeded synthetic scenes shaped like the paper's fluid-structure benchmarks.

This module only generates inputs: particle lattices, wall shells with their
geometric outward normals, material parameters and a seeded jitter.  It holds
none of the SPH method's arithmetic (no kernel, no equation of state, no
density or mass initialisation); both the GPU library and the FP64 oracle take
a scene dict from here and initialise their own state from it.

Scene dict keys (SI units; positions are row-major ``(n, dim)`` float64):

``dim, dp_f, dp_s, h_ratio, rho0_f, c_f, eta, gamma, g(3), rho0_s, E, nu,
cfl_ac, cfl_ad, cfl_s, u_ref, lo(3), hi(3), periodic(3), hydro_H,
inflow_U0, inflow_ts, inflow_H, inflow_len, x_fluid, v_fluid, x_wall, n_wall,
x_solid, v_solid, n_clamp, tip_index, name``

Solid particles are listed free ones first; the last ``n_clamp`` of them form
the rigid base block that holds the plate (Section 4.2 "constraints of the
rigid base").  Walls are rigid dummy particles at the fluid spacing.

Jitter: every fluid and free-solid coordinate is displaced by an independent
uniform draw in [-1e-4 dp, +1e-4 dp) taken from a counter-based SplitMix64
stream (Steele, Lea & Flood 2014): output k of the stream seeded with s is the
SplitMix64 finaliser applied to s + (k+1) * 0x9E3779B97F4A7C15 (mod 2^64).
"""
from __future__ import annotations

import math

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counters) -> np.ndarray:
    """Counter-based SplitMix64: output number ``counters`` of the stream ``seed``."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (c + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, counters) -> np.ndarray:
    """Doubles in [0, 1) from the top 53 bits of the SplitMix64 outputs."""
    z = splitmix64(seed, counters)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def _jitter(seed: int, first_counter: int, n: int, dim: int, dp: float) -> np.ndarray:
    cnt = first_counter + np.arange(n * 4, dtype=np.uint64).reshape(n, 4)[:, :dim]
    return (2.0 * uniform01(seed, cnt) - 1.0) * (1e-4 * dp)


def lattice(lo, hi, dp) -> np.ndarray:
    """Cell-centred lattice points of spacing dp filling the box [lo, hi)."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    counts = np.maximum(np.rint((hi - lo) / dp).astype(int), 0)
    axes = [lo[k] + (np.arange(counts[k]) + 0.5) * dp for k in range(len(lo))]
    if any(len(a) == 0 for a in axes):
        return np.zeros((0, len(lo)))
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack([m.ravel() for m in mesh], axis=1)


def _base(dim: int) -> dict:
    return dict(
        dim=dim, dp_f=0.0, dp_s=0.0, h_ratio=1.3, rho0_f=1000.0, c_f=10.0, eta=0.0,
        gamma=7.0, g=np.zeros(3), rho0_s=1000.0, E=1e6, nu=0.3, cfl_ac=0.25, cfl_ad=0.25,
        cfl_s=0.6, u_ref=1.0, lo=np.zeros(3), hi=np.ones(3), periodic=np.zeros(3, dtype=np.int32),
        hydro_H=0.0, inflow_U0=0.0, inflow_ts=0.0, inflow_H=0.0, inflow_len=0.0,
        x_fluid=np.zeros((0, dim)), v_fluid=None, x_wall=np.zeros((0, dim)),
        n_wall=np.zeros((0, dim)), x_solid=np.zeros((0, dim)), v_solid=None,
        n_clamp=0, tip_index=-1, name="", material=0, single_step=0,
    )


def _tank_walls(extent, dp, layers=3, open_top=True):
    """Wall shell of ``layers`` dummy layers outside the box [0, extent).

    The last axis is vertical.  Each wall particle carries the unit vector from
    itself towards the nearest point of the box (the outward normal of the wall
    seen from the fluid, diagonal in edges and corners).
    """
    extent = np.asarray(extent, float)
    dim = len(extent)
    t = layers * dp
    lo = -t * np.ones(dim)
    hi = extent + t
    if open_top:
        hi[-1] = extent[-1]
    pts = lattice(lo, hi, dp)
    inside = np.all((pts > 0.0) & (pts < extent), axis=1)
    pts = pts[~inside]
    nearest = np.clip(pts, 0.0, extent)
    nrm = nearest - pts
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    return pts, nrm


def _finish(sc: dict, seed: int, solid_lattice: bool = False) -> dict:
    """Seeded jitter of 1e-4 dp on the fluid and (unless ``solid_lattice``)
    on the free solid particles, then contiguous FP64 arrays."""
    dim = sc["dim"]
    nf = len(sc["x_fluid"])
    ns = len(sc["x_solid"])
    nfree = ns - sc["n_clamp"]
    if seed is not None:
        sc["x_fluid"] = sc["x_fluid"] + _jitter(seed, 0, nf, dim, sc["dp_f"])
        if nfree > 0 and not solid_lattice:
            xs = sc["x_solid"].copy()
            xs[:nfree] += _jitter(seed, 4 * nf, nfree, dim, sc["dp_s"])
            sc["x_solid"] = xs
    for k in ("x_fluid", "x_wall", "n_wall", "x_solid"):
        sc[k] = np.ascontiguousarray(sc[k], dtype=np.float64).reshape(-1, dim)
    for k in ("v_fluid", "v_solid"):
        if sc[k] is not None:
            sc[k] = np.ascontiguousarray(sc[k], dtype=np.float64).reshape(-1, dim)
    sc["seed"] = seed
    return sc


def _plate(x0, x1, y0, y1, dp, clamp_rows, dim=2, z=None, clamp_axis="bottom"):
    """Plate lattice plus a clamp block of ``clamp_rows`` layers past one end."""
    if dim == 2:
        plate = lattice([x0, y0], [x1, y1], dp)
        if clamp_axis == "bottom":
            clamp = lattice([x0, y0 - clamp_rows * dp], [x1, y0], dp)
        else:  # clamp extends to the left (-x) of the plate root
            clamp = lattice([x0 - clamp_rows * dp, y0], [x0, y1], dp)
    else:
        plate = lattice([x0, z[0], y0], [x1, z[1], y1], dp)
        clamp = lattice([x0, z[0], y0 - clamp_rows * dp], [x1, z[1], y0], dp)
    return plate, clamp


def dam_break_plate(seed: int = 1, dp_f: float = 0.004, dp_s: float = 0.001,
                    water=(0.1, 0.14), tank=(0.4, 0.2), plate_x=0.2,
                    plate_w=0.005, plate_h=0.079, E=1e7, nu=0.4, rho_s=1100.0,
                    cfl_ac=0.25) -> dict:
    """2D dam break on an elastic plate clamped at its base (Section 4.2 shape).

    Water column ``water`` in the corner of an open tank ``tank`` with three wall
    layers; a Neo-Hookean plate of width ``plate_w`` and height ``plate_h``
    standing on the tank floor at ``plate_x``, held by three clamp rows below
    the floor.  Defaults give 875 fluid, 618 wall and 395 + 15 solid particles.
    """
    sc = _base(2)
    g = 9.81
    H = water[1]
    c0 = 10.0 * math.sqrt(2.0 * g * H)
    sc.update(dp_f=dp_f, dp_s=dp_s, rho0_f=1000.0, c_f=c0, eta=0.0,
              g=np.array([0.0, -g, 0.0]), rho0_s=rho_s, E=E, nu=nu,
              cfl_ac=cfl_ac, cfl_ad=0.25, cfl_s=0.6, u_ref=c0 / 10.0, hydro_H=H,
              name="dam_break_plate_2d")
    sc["x_fluid"] = lattice([0.0, 0.0], list(water), dp_f)
    sc["x_wall"], sc["n_wall"] = _tank_walls(tank, dp_f)
    nw = max(3, int(round(plate_w / dp_s)))
    nh = int(round(plate_h / dp_s))
    plate, clamp = _plate(plate_x, plate_x + nw * dp_s, 0.0, nh * dp_s, dp_s, 3)
    sc["x_solid"] = np.concatenate([plate, clamp])
    sc["n_clamp"] = len(clamp)
    # tip sensor: free end, mid thickness
    top = plate[:, 1].max()
    cand = np.where(np.abs(plate[:, 1] - top) < 1e-12)[0]
    mid = plate_x + 0.5 * nw * dp_s
    sc["tip_index"] = int(cand[np.argmin(np.abs(plate[cand, 0] - mid))])
    m = 3 * dp_f + 0.01
    sc["lo"] = np.array([-m, -m, 0.0])
    sc["hi"] = np.array([tank[0] + m, tank[1] + 0.1, 1.0])
    return _finish(sc, seed)


def plate_behind_cylinder(seed: int = 1, D: float = 0.1, dp_f: float = None,
                          dp_ratio: float = 2.0, Re: float = 100.0, rho_ratio: float = 10.0,
                          E_star: float = 1.4e3, nu: float = 0.4, U0: float = 1.0,
                          cfl_ac: float = 0.6) -> dict:
    """2D flexible plate behind a rigid cylinder in a channel (Section 4.1 shape).

    Channel 11D x 4.1D with no-slip walls top and bottom (three layers), periodic
    in x with an inflow buffer; rigid cylinder of diameter D centred at (2D, 2D);
    plate 3.5D x 0.2D from the cylinder's downstream surface with a three-column
    clamp block inside the cylinder.  rho_f = 1, U0 = 1, c_f = 10 U0.
    """
    sc = _base(2)
    if dp_f is None:
        dp_f = D / 20.0
    dp_s = dp_f / dp_ratio
    L, Hc = 11.0 * D, 4.1 * D
    cx, cy, R = 2.0 * D, 2.0 * D, 0.5 * D
    rho_f = 1.0
    eta = rho_f * U0 * D / Re
    c0 = 10.0 * U0
    sc.update(dp_f=dp_f, dp_s=dp_s, rho0_f=rho_f, c_f=c0, eta=eta, g=np.zeros(3),
              rho0_s=rho_ratio * rho_f, E=E_star * rho_f * U0 * U0, nu=nu,
              cfl_ac=cfl_ac, cfl_ad=0.25, cfl_s=0.6, u_ref=c0 / 10.0, hydro_H=0.0,
              inflow_U0=U0, inflow_ts=2.0, inflow_H=Hc, inflow_len=4.0 * 1.3 * dp_f,
              name="plate_behind_cylinder_2d")
    px0 = cx + math.sqrt(R * R - (0.1 * D) ** 2)
    px0 = math.floor(px0 / dp_s + 0.5) * dp_s
    nlen = int(round(3.5 * D / dp_s))
    nth = int(round(0.2 * D / dp_s))
    py0 = cy - 0.5 * nth * dp_s
    plate, clamp = _plate(px0, px0 + nlen * dp_s, py0, py0 + nth * dp_s, dp_s, 3,
                          clamp_axis="left")
    fl = lattice([0.0, 0.0], [L, Hc], dp_f)
    r = np.hypot(fl[:, 0] - cx, fl[:, 1] - cy)
    in_cyl = r < R
    in_plate = ((fl[:, 0] > px0) & (fl[:, 0] < px0 + nlen * dp_s)
                & (fl[:, 1] > py0) & (fl[:, 1] < py0 + nth * dp_s))
    sc["x_fluid"] = fl[~in_cyl & ~in_plate]
    cyl = fl[in_cyl]
    ncyl = cyl - np.array([cx, cy])
    ncyl /= np.maximum(np.linalg.norm(ncyl, axis=1, keepdims=True), 1e-300)
    t = 3 * dp_f
    bot = lattice([0.0, -t], [L, 0.0], dp_f)
    top = lattice([0.0, Hc], [L, Hc + t], dp_f)
    sc["x_wall"] = np.concatenate([bot, top, cyl])
    sc["n_wall"] = np.concatenate([np.tile([0.0, 1.0], (len(bot), 1)),
                                   np.tile([0.0, -1.0], (len(top), 1)), ncyl])
    sc["x_solid"] = np.concatenate([plate, clamp])
    sc["n_clamp"] = len(clamp)
    tipx = plate[:, 0].max()
    cand = np.where(np.abs(plate[:, 0] - tipx) < 1e-12)[0]
    sc["tip_index"] = int(cand[np.argmin(np.abs(plate[cand, 1] - cy))])
    sc["lo"] = np.array([0.0, -t - 0.01, 0.0])
    sc["hi"] = np.array([L, Hc + t + 0.01, 1.0])
    sc["periodic"] = np.array([1, 0, 0], dtype=np.int32)
    return _finish(sc, seed)


def dam_break_plate_3d(seed: int = 1, dp_f: float = 0.006, dp_ratio: float = 2.0,
                       water=(0.6, 0.6, 1.2), tank=(1.6, 0.6, 1.2),
                       plate=(0.04, 0.6, 0.4), plate_x=0.8, E=5e6, nu=0.45,
                       rho_s=1100.0, cfl_ac=0.25, solid_lattice: bool = True) -> dict:
    """3D dam break on an elastic plate clamped at its base (z is vertical).

    The plate's reference configuration is its exact lattice unless
    ``solid_lattice`` is False (then it is jittered like the fluid).
    """
    sc = _base(3)
    g = 9.81
    H = water[2]
    c0 = 10.0 * math.sqrt(2.0 * g * H)
    dp_s = dp_f / dp_ratio
    sc.update(dp_f=dp_f, dp_s=dp_s, rho0_f=1000.0, c_f=c0, eta=0.0,
              g=np.array([0.0, 0.0, -g]), rho0_s=rho_s, E=E, nu=nu, cfl_ac=cfl_ac,
              cfl_ad=0.25, cfl_s=0.6, u_ref=c0 / 10.0, hydro_H=H,
              name="dam_break_plate_3d")
    sc["x_fluid"] = lattice([0.0, 0.0, 0.0], list(water), dp_f)
    sc["x_wall"], sc["n_wall"] = _tank_walls(tank, dp_f)
    nx = max(3, int(math.floor(plate[0] / dp_s + 1e-9)))
    ny = int(math.floor(plate[1] / dp_s + 1e-9))
    nz = int(math.floor(plate[2] / dp_s + 1e-9))
    pl = lattice([plate_x, 0.0, 0.0], [plate_x + nx * dp_s, ny * dp_s, nz * dp_s], dp_s)
    cl = lattice([plate_x, 0.0, -3 * dp_s], [plate_x + nx * dp_s, ny * dp_s, 0.0], dp_s)
    sc["x_solid"] = np.concatenate([pl, cl])
    sc["n_clamp"] = len(cl)
    top = pl[:, 2].max()
    cand = np.where(np.abs(pl[:, 2] - top) < 1e-12)[0]
    ctr = np.array([plate_x + 0.5 * nx * dp_s, 0.5 * ny * dp_s])
    sc["tip_index"] = int(cand[np.argmin(np.linalg.norm(pl[cand, :2] - ctr, axis=1))])
    m = 3 * dp_f + 0.02
    sc["lo"] = np.array([-m, -m, -m])
    sc["hi"] = np.array([tank[0] + m, tank[1] + m, tank[2] + 0.2])
    return _finish(sc, seed, solid_lattice)


def batched_dam_breaks(n_scenes: int = 64, master_seed: int = 2026) -> list:
    """Independent 2D dam-break/plate scenes with seeded parameters.

    Scene k draws, from the SplitMix64 stream seeded with output k of the master
    stream: water height in [0.08, 0.2] m, plate length in [0.05, 0.1] m,
    E in [2, 20] MPa, nu in [0.3, 0.47] and dp_f in [0.002, 0.005] m; the
    water is 0.1 m wide, the tank 0.4 m wide and max(0.2, H + 0.05) m high,
    the plate 5 mm thick at x = 0.2 m with dp_s = dp_f / 4.
    """
    seeds = splitmix64(master_seed, np.arange(n_scenes, dtype=np.uint64))
    out = []
    for k in range(n_scenes):
        s = int(seeds[k])
        u = uniform01(s, np.arange(5, dtype=np.uint64))
        H = 0.08 + 0.12 * u[0]
        Lp = 0.05 + 0.05 * u[1]
        E = 2e6 + 18e6 * u[2]
        nu = 0.3 + 0.17 * u[3]
        dp_f = 0.002 + 0.003 * u[4]
        dp_f = 1e-6 * round(dp_f / 1e-6)
        nwx = int(round(0.1 / dp_f))
        nwy = int(round(H / dp_f))
        sc = dam_break_plate(seed=s & 0x7FFFFFFF, dp_f=dp_f, dp_s=dp_f / 4.0,
                             water=(nwx * dp_f, nwy * dp_f),
                             tank=(0.4, max(0.2, H + 0.05)), plate_x=0.2,
                             plate_w=0.005, plate_h=Lp, E=E, nu=nu)
        sc["name"] = f"batched_dam_break_{k}"
        out.append(sc)
    return out


# ---------------------------------------------------------------- test scenes

def hydrostatic_column(seed: int = 3, dp: float = 0.01, width: float = 0.2,
                       H: float = 0.4) -> dict:
    """Water at rest filling a 2D open tank (no solid)."""
    sc = _base(2)
    g = 9.81
    c0 = 10.0 * math.sqrt(2.0 * g * H)
    sc.update(dp_f=dp, dp_s=dp, rho0_f=1000.0, c_f=c0, g=np.array([0.0, -g, 0.0]),
              cfl_ac=0.25, u_ref=c0 / 10.0, hydro_H=H, name="hydrostatic_column")
    sc["x_fluid"] = lattice([0.0, 0.0], [width, H], dp)
    sc["x_wall"], sc["n_wall"] = _tank_walls((width, H + 0.1), dp)
    m = 3 * dp + 0.01
    sc["lo"] = np.array([-m, -m, 0.0])
    sc["hi"] = np.array([width + m, H + 0.2, 1.0])
    return _finish(sc, seed)


def periodic_box_with_solid(seed: int = 5, dim: int = 2, n: int = 16, dp: float = 0.01,
                            solid=True, amp: float = 0.05, eta: float = 0.0,
                            solid_lattice: bool = False) -> dict:
    """Fully periodic fluid box with a free (unclamped) elastic block, g = 0.

    Velocities are a seeded random field of amplitude ``amp`` (times the fluid
    sound speed / 10), so that every pair term is exercised.
    """
    sc = _base(dim)
    Lb = n * dp
    c0 = 10.0
    dp_s = dp / 2.0
    sc.update(dp_f=dp, dp_s=dp_s, rho0_f=1000.0, c_f=c0, eta=eta, g=np.zeros(3),
              rho0_s=1200.0, E=2e5, nu=0.35, cfl_ac=0.25, u_ref=c0 / 10.0,
              name="periodic_box")
    lo = np.zeros(dim)
    hi = np.full(dim, Lb)
    fl = lattice(lo, hi, dp)
    if solid:
        blo = np.full(dim, 0.375 * Lb)
        bhi = np.full(dim, 0.625 * Lb)
        inside = np.all((fl > blo) & (fl < bhi), axis=1)
        fl = fl[~inside]
        sc["x_solid"] = lattice(blo, bhi, dp_s)
    sc["x_fluid"] = fl
    rng_f = uniform01(seed ^ 0x1234, np.arange(len(fl) * dim, dtype=np.uint64))
    sc["v_fluid"] = (2.0 * rng_f.reshape(-1, dim) - 1.0) * amp * c0 / 10.0
    if solid:
        ns = len(sc["x_solid"])
        rng_s = uniform01(seed ^ 0x5678, np.arange(ns * dim, dtype=np.uint64))
        sc["v_solid"] = (2.0 * rng_s.reshape(-1, dim) - 1.0) * amp * c0 / 10.0
        sc["tip_index"] = 0
    sc["lo"] = np.zeros(3)
    sc["hi"] = np.ones(3)
    sc["lo"][:dim] = 0.0
    sc["hi"][:dim] = Lb
    sc["periodic"] = np.array([1 if k < dim else 0 for k in range(3)], dtype=np.int32)
    return _finish(sc, seed, solid_lattice)


def shear_layer(seed: int = 7, dp: float = 0.01, n_x: int = 16, n_y: int = 8,
                U: float = 0.1, eta: float = 5.0) -> dict:
    """Viscous fluid layer sliding over a static wall, periodic in x, g = 0."""
    sc = _base(2)
    Lx, Hy = n_x * dp, n_y * dp
    c0 = 10.0
    sc.update(dp_f=dp, dp_s=dp, rho0_f=1000.0, c_f=c0, eta=eta, g=np.zeros(3),
              cfl_ac=0.25, u_ref=c0 / 10.0, name="shear_layer")
    fl = lattice([0.0, 0.0], [Lx, Hy], dp)
    sc["x_fluid"] = fl
    v = np.zeros_like(fl)
    v[:, 0] = U
    sc["v_fluid"] = v
    sc["x_wall"] = lattice([0.0, -3 * dp], [Lx, 0.0], dp)
    sc["n_wall"] = np.tile([0.0, 1.0], (len(sc["x_wall"]), 1))
    sc["lo"] = np.array([0.0, -0.05, 0.0])
    sc["hi"] = np.array([Lx, Hy + 0.05, 1.0])
    sc["periodic"] = np.array([1, 0, 0], dtype=np.int32)
    return _finish(sc, seed)


def solid_block(seed=None, dim: int = 2, n=(8, 6, 5), dp: float = 0.01, E=1e6, nu=0.3,
                rho_s=1000.0, n_clamp_rows: int = 0) -> dict:
    """A lone elastic block (no fluid, g = 0), optionally with clamp rows below."""
    sc = _base(dim)
    sc.update(dp_f=2 * dp, dp_s=dp, rho0_s=rho_s, E=E, nu=nu, c_f=10.0, u_ref=1.0,
              name="solid_block")
    hi = [n[k] * dp for k in range(dim)]
    blk = lattice(np.zeros(dim), hi, dp)
    if n_clamp_rows:
        lo_c = [0.0] * dim
        lo_c[-1] = -n_clamp_rows * dp
        hi_c = list(hi)
        hi_c[-1] = 0.0
        cl = lattice(lo_c, hi_c, dp)
        sc["x_solid"] = np.concatenate([blk, cl])
        sc["n_clamp"] = len(cl)
    else:
        sc["x_solid"] = blk
    sc["x_fluid"] = np.zeros((0, dim))
    sc["tip_index"] = 0
    sc["lo"] = np.full(3, -0.5)
    sc["hi"] = np.full(3, 0.5)
    return _finish(sc, seed)


def hydrostatic_layer(seed: int = 3, dp: float = 0.01, width: float = 0.2,
                      H: float = 0.4) -> dict:
    """Water at rest over a flat floor, periodic in x (no side walls, no solid)."""
    sc = _base(2)
    g = 9.81
    c0 = 10.0 * math.sqrt(2.0 * g * H)
    sc.update(dp_f=dp, dp_s=dp, rho0_f=1000.0, c_f=c0, g=np.array([0.0, -g, 0.0]),
              cfl_ac=0.25, u_ref=c0 / 10.0, hydro_H=H, name="hydrostatic_layer")
    sc["x_fluid"] = lattice([0.0, 0.0], [width, H], dp)
    sc["x_wall"] = lattice([0.0, -3 * dp], [width, 0.0], dp)
    sc["n_wall"] = np.tile([0.0, 1.0], (len(sc["x_wall"]), 1))
    sc["lo"] = np.array([0.0, -3 * dp - 0.01, 0.0])
    sc["hi"] = np.array([width, H + 0.2, 1.0])
    sc["periodic"] = np.array([1, 0, 0], dtype=np.int32)
    return _finish(sc, seed)
