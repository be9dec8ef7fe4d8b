"""The entry point that allocates nothing (sph_reduce_noalloc) against the
reductions of sph_reduce, through the C-ABI: two calls in a row, the second
on a smaller scene (fewer blocks, stale partials of the first call left in the
static scratch), and the size limit of that scratch."""
import numpy as np
import pytest

from paper_1911_13255_amd import scenes, sph

pytestmark = pytest.mark.gpu


def _reduced(sim, scene, blocks=0):
    import torch

    out = torch.full((16,), float("nan"), dtype=torch.float64, device=sim.device)
    sim.reduce_noalloc(out, scene, blocks)
    torch.cuda.synchronize(sim.device)
    return out.cpu().numpy()


def _reference(sim, scene):
    r = sim.reduce(scene)
    return np.concatenate([r["mom_fluid"], r["mom_solid"], [r["ke_fluid"], r["ke_solid"], r["strain_energy"]],
                           r["sum_fF"], r["sum_fS"]])


def test_reduce_noalloc_matches_sph_reduce(gpu):
    scs = scenes.batched_dam_breaks(n_scenes=4)
    sizes = [max(len(s["x_fluid"]), len(s["x_solid"])) for s in scs]
    big, small = int(np.argmax(sizes)), int(np.argmin(sizes))
    assert (sizes[big] + 255) // 256 > (sizes[small] + 255) // 256
    print(f"scenes {sizes}: first call on scene {big}, second on scene {small}", flush=True)
    sim = sph.Simulation(scs)
    sim.advance(30)
    sim.sync()
    for scene in (big, small):  # two calls in a row, the second with fewer blocks
        got, ref = _reduced(sim, scene), _reference(sim, scene)
        assert np.all(np.isfinite(got[:15]))
        assert ref[6] > 0.0 and ref[8] != 0.0
        # same kernels over the same blocks: the same bits
        assert np.array_equal(got[:15], ref), (scene, got[:15], ref)
    # an explicit block count sums in another order: FP64 rounding only
    got = _reduced(sim, big, blocks=7)
    ref = _reference(sim, big)
    scale = np.abs(ref).max()
    assert np.abs(got[:15] - ref).max() <= 1e-12 * scale
    # the static scratch holds 1024 blocks' partials
    import torch

    out = torch.zeros(16, dtype=torch.float64, device=sim.device)
    with pytest.raises(sph.SphError) as e:
        sim.reduce_noalloc(out, 0, 1025)
    assert e.value.code == sph.SPH_E_ARG
    assert "1024" in str(e.value)
    sim.sync()
    sim.close()
