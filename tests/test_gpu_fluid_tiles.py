"""Neighbour tiles of the 3D fluid force and continuity passes (Section 3.1
pair sums over the frozen pair lists of an advection step, Section 3.2).

A block of the pair launches stages its particles' distinct fluid neighbours
in LDS and walks rows that index that set instead of the neighbours
themselves.  Every pair's terms are the per-pair form's, in the same order,
from the same records, so the two forms agree bit for bit over steps that
rebuild the lists; the pair sets read back through sph_pairs are the same
too.  Groups that straddle two scenes, or have more distinct neighbours than
a tile holds, keep per-pair gathers, and the results still agree.
"""
import sys

import numpy as np
import pytest

from paper_1911_13255_amd import scenes, sph

pytestmark = pytest.mark.gpu

FIELDS = (sph.F_X, sph.F_V, sph.F_RHO, sph.F_DRHO, sph.F_A, sph.F_P, sph.F_NNB, sph.S_U, sph.S_V, sph.S_F,
          sph.S_VBAR, sph.S_ABAR, sph.S_FF)


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dam_break(dp_f):
    return [scenes.dam_break_plate_3d(seed=1, dp_f=dp_f)]


def box(seed=5, h_ratio=1.3, solid=True):
    sc = scenes.periodic_box_with_solid(seed=seed, dim=3, n=12, eta=0.5, amp=0.3, solid=solid)
    sc["h_ratio"] = h_ratio
    return sc


CASES = {
    # 16k fluid particles: the force pass forms the snapshot per pair
    "dam_break_coarse": lambda: dam_break(0.03),
    # 250k fluid particles: the snapshot pass runs first
    "dam_break_prep": lambda: dam_break(0.012),
    # periodic in all three axes: rows hold wrapped relative cells
    "periodic_box": lambda: [box()],
    # two scenes in one context: the group across their boundary gathers per pair
    "two_scenes": lambda: [box(5), box(9)],
    # support of 4 dp (no solid, whose reference table is sized for 2.6 dp)
    # and 64 particles per group: every group has more distinct neighbours
    # than a tile holds
    "wide_support": lambda: [box(h_ratio=2.0, solid=False)],
}
OPTIONS = {"wide_support": dict(lanes_per_particle=4)}


@pytest.mark.parametrize("name", sorted(CASES))
def test_tiles_equal_per_pair_gathers(gpu, name):
    scs = CASES[name]()
    steps = 40 if name.startswith("dam_break") else 30
    opt = OPTIONS.get(name, {})
    tiled = sph.Simulation(scs, **opt)
    plain = sph.Simulation(scs, fluid_tiles=-1, **opt)
    for sim in (tiled, plain):
        sim.advance(steps)
    t = tiled.fluid_tiles()
    note(f"{name}: {sum(len(s['x_fluid']) for s in scs)} fluid, tiles {t}, "
         f"rebuilds {tiled.counters()['rebuilds']}")
    assert plain.fluid_tiles()["group"] == 0
    assert t["group"] == tiled.launch_config()["block_pair"] // tiled.launch_config()["lpp_fluid"]
    assert t["groups"] == -(-sum(len(s["x_fluid"]) for s in scs) // t["group"])
    if name == "wide_support":
        assert t["tiled"] == 0
    elif name == "two_scenes":
        assert 0 < t["tiled"] < t["groups"]
    else:
        assert t["tiled"] == t["groups"]
    assert t["largest"] <= 768
    assert tiled.counters()["rebuilds"] >= 2
    for s in range(len(scs)):
        for f in FIELDS:
            if f >= sph.S_U and len(scs[s]["x_solid"]) == 0:
                continue
            assert np.array_equal(tiled.read(f, s), plain.read(f, s)), (name, s, f)
        assert tiled.scalars(s) == plain.scalars(s)
        if name != "dam_break_prep":
            for a, b in zip(tiled.pairs(0, s), plain.pairs(0, s)):
                assert np.array_equal(a, b), (name, s)
    assert tiled.counters() == plain.counters()
    assert tiled.sync() == sph.SPH_OK and plain.sync() == sph.SPH_OK
    tiled.close()
    plain.close()


def test_tiles_in_graph_replays_and_separate_calls(gpu):
    """The phases called one by one (rebuild, force, couple, solid,
    continuity) and sph_advance's steps give the same bits with tiles."""
    scs = [box()]
    tiled = sph.Simulation(scs)
    plain = sph.Simulation(scs, fluid_tiles=-1)
    for sim in (tiled, plain):
        sim.advance(10)
        for _ in range(12):
            sim.step()
        sim.advance(10)
    for f in FIELDS:
        assert np.array_equal(tiled.read(f), plain.read(f)), f
    tiled.close()
    plain.close()


def test_tile_option_checked(gpu):
    with pytest.raises(sph.SphError):
        sph.Simulation([box()], fluid_tiles=3)
