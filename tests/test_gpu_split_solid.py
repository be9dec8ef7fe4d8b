"""The block-resident solid kernel split over several workgroups per scene
(serial steps; Section 3.3's kappa sub-steps, Algorithm 1's solid loop).

Each workgroup keeps a slice of the free particles in registers and the
whole scene's P B and v in LDS, refreshed through global memory after every
half sub-step.  Every particle's sums are the ones of the one-workgroup form,
term for term and in the same order, so the two forms agree bit for bit; the
oracle's parity is checked on the split form as well.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1911_13255_amd import scenes, sph

pytestmark = pytest.mark.gpu

FIELDS = (sph.F_X, sph.F_V, sph.F_RHO, sph.S_U, sph.S_V, sph.S_A, sph.S_F, sph.S_DF, sph.S_VBAR, sph.S_ABAR)


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def cases(name):
    if name == "channel":
        return [scenes.plate_behind_cylinder(seed=1)]
    return scenes.batched_dam_breaks(64)[:8]


@pytest.mark.parametrize("name,target", [("channel", 128), ("channel", 512), ("batch", 64)])
def test_split_equals_one_workgroup_bit_for_bit(gpu, name, target):
    scs = cases(name)
    one = sph.Simulation(scs, serial_passes=1)
    split = sph.Simulation(scs, serial_passes=1, solid_parts=target)
    cfg = split.launch_config()
    note(f"split {name}: target {cfg['solid_parts']}, {cfg['solid_workgroups']} workgroups for {len(scs)} scenes")
    assert cfg["solid_parts"] > 0 and cfg["solid_workgroups"] > len(scs)
    assert one.launch_config()["solid_workgroups"] == 0
    # graph replays, then the separate calls (the launch that also ends the
    # step), then replays again
    for sim in (one, split):
        sim.advance(40)
        for _ in range(5):
            sim.step()
        sim.advance(40)
    for s in range(len(scs)):
        for f in FIELDS:
            assert np.array_equal(one.read(f, s), split.read(f, s)), (name, s, f)
        assert one.scalars(s) == split.scalars(s)
    assert one.counters()["substeps"] == split.counters()["substeps"]
    assert one.sync() == sph.SPH_OK and split.sync() == sph.SPH_OK
    one.close()
    split.close()


def test_split_channel_matches_the_oracle(gpu):
    sc = scenes.plate_behind_cylinder(seed=1)
    sim = sph.Simulation(sc, serial_passes=1, solid_parts=128)
    o = O.Oracle(sc)
    for k in range(3):
        sim.advance(4)
        o.step(4)
        for f, name in ((sph.F_RHO, "rho"), (sph.F_A, "a_f"), (sph.S_U, "u"), (sph.S_V, "v"), (sph.S_FF, "fF"),
                        (sph.S_VBAR, "vbar"), (sph.S_ABAR, "abar")):
            g, r = sim.read(f), o.get(f)
            err = np.abs(g - r).max() / np.abs(r).max()
            assert err <= 1e-4, (k, name, err)
        assert sim.scalars()["kappa"] == o.scalars()["kappa"]
    note(f"split channel: kappa {o.scalars()['kappa']}, parity within 1e-4 over 12 steps")
    assert sim.sync() == sph.SPH_OK
    sim.close()
