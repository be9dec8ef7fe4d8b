"""The stability limit of the batched dam breaks is the method's, not the GPU
path's: the FP64 oracle alone, on the coarse batched scene 1 (dp_F = 4.9 mm,
nu = 0.30, E = 10.8 MPa; 740 fluid and 256 solid particles), stays at rest-
like plate speeds through step 1,100 (the window the batch benchmark times),
is hit by the surge near step 1,400 and then blows up: the plate reaches tens
of metres per second (a surge of a 0.15 m column moves at about 2 m/s) and
the state turns non-finite before step 2,000."""
import numpy as np

from oracle import oracle as O
from paper_1911_13255_amd import scenes


def test_coarse_batched_scene_is_unstable_in_the_oracle():
    sc = scenes.batched_dam_breaks(64)[1]
    assert abs(sc["dp_f"] - 0.004946) < 1e-6 and abs(sc["nu"] - 0.3041) < 1e-3
    o = O.Oracle(sc)
    o.step(1100)
    F, vs = o.get(O.S_F), o.get(O.S_V)
    assert np.all(np.isfinite(F)) and np.all(np.isfinite(o.get(O.F_V)))
    assert np.linalg.det(F).min() > 0.99 and np.abs(vs).max() < 0.05
    blown = None
    for step in range(1100, 2000, 20):
        o.step(20)
        F, vs, vf = o.get(O.S_F), o.get(O.S_V), o.get(O.F_V)
        finite = np.all(np.isfinite(F)) and np.all(np.isfinite(vs)) and np.all(np.isfinite(vf))
        if not finite or np.abs(vs).max() > 20.0:
            blown = step + 20
            break
    assert blown is not None and 1400 < blown <= 2000, blown
