"""The C-ABI library loads and exports every symbol include/mrsph.h declares
(no GPU calls), and host-side argument checks reject bad scenes."""
import ctypes
import os

import numpy as np
import pytest

from paper_1911_13255_amd import scenes, sph


def _lib_or_skip():
    if not os.path.exists(sph.LIB_PATH):
        pytest.skip("libmrsph.so not built")
    return sph.lib()


def test_header_symbols_exported():
    _lib_or_skip()
    names = sph.exported_names()
    for must in ("sph_init", "neighbor_build", "fluid_step", "couple", "solid_substeps", "sph_advance",
                 "sph_read", "sph_write", "sph_reduce", "sph_counters", "sph_sync", "sph_destroy",
                 "sph_arena_bytes", "sph_scalars", "sph_set_scalars", "sph_last_error"):
        assert must in names
    L = ctypes.CDLL(sph.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing


def test_arena_bytes_and_argument_checks():
    L = _lib_or_skip()
    sc = scenes.dam_break_plate(seed=1)
    st, keep = sph.scene_struct(sc)
    arr = (sph.SphScene * 1)(st)
    opt = sph.make_options()
    n1 = L.sph_arena_bytes(arr, 1, ctypes.byref(opt))
    assert n1 > 0
    # more scenes need more memory
    arr2 = (sph.SphScene * 2)(st, st)
    assert L.sph_arena_bytes(arr2, 2, ctypes.byref(opt)) > n1
    # invalid descriptions give 0
    bad = sph.SphScene.from_buffer_copy(st)
    bad.dim = 4
    assert L.sph_arena_bytes((sph.SphScene * 1)(bad), 1, ctypes.byref(opt)) == 0
    bad = sph.SphScene.from_buffer_copy(st)
    bad.n_clamp = bad.n_solid + 1
    assert L.sph_arena_bytes((sph.SphScene * 1)(bad), 1, ctypes.byref(opt)) == 0
    bad = sph.SphScene.from_buffer_copy(st)
    bad.periodic[0] = 1
    bad.hi[0] = bad.lo[0] + 0.02  # fewer than 3 cells of 2 h_F
    assert L.sph_arena_bytes((sph.SphScene * 1)(bad), 1, ctypes.byref(opt)) == 0
    # pair-list capacities beyond the limit are rejected
    big = sph.make_options(max_fluid_nbr=5000)
    assert L.sph_arena_bytes(arr, 1, ctypes.byref(big)) == 0
    # larger capacities need more memory
    roomy = sph.make_options(max_fluid_nbr=256, max_boundary_nbr=512)
    assert L.sph_arena_bytes(arr, 1, ctypes.byref(roomy)) > n1
    mixed = sph.SphScene.from_buffer_copy(st)
    mixed.dim = 3
    assert L.sph_arena_bytes((sph.SphScene * 2)(st, mixed), 2, ctypes.byref(opt)) == 0
    # init with no context pointer or a null arena fails without touching the GPU
    out = ctypes.c_void_p()
    assert L.sph_init(arr, 1, ctypes.byref(opt), None, 0, None, ctypes.byref(out)) == sph.SPH_E_ARG
    assert L.sph_init(arr, 1, ctypes.byref(opt), None, 0, None, None) == sph.SPH_E_ARG


def test_calls_without_context_are_order_errors():
    L = _lib_or_skip()
    for name in ("neighbor_build", "fluid_step", "couple", "solid_substeps", "sph_sync"):
        assert getattr(L, name)(None) == sph.SPH_E_ORDER
    assert L.sph_advance(None, 1) == sph.SPH_E_ORDER
    cfg = (ctypes.c_int * 8)()
    assert L.sph_launch_config(None, cfg) == sph.SPH_E_ORDER
    buf = np.zeros(8)
    assert L.sph_scalars(None, 0, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == sph.SPH_E_ORDER


def test_autotune_and_option_checks_without_gpu():
    L = _lib_or_skip()
    sc = scenes.dam_break_plate(seed=1)
    arr, keep = sph.scene_array([sc])
    opt = sph.make_options()
    best = sph.SphOptions()
    ms = ctypes.c_double()
    # bad arguments are rejected before any GPU work
    assert L.sph_autotune(None, 1, ctypes.byref(opt), None, 0, None, 1, 1, ctypes.byref(best),
                          ctypes.byref(ms)) == sph.SPH_E_ARG
    assert L.sph_autotune(arr, 1, ctypes.byref(opt), None, 1 << 30, None, 1, 1, ctypes.byref(best),
                          ctypes.byref(ms)) == sph.SPH_E_ARG
    assert L.sph_autotune(arr, 1, ctypes.byref(opt), ctypes.c_void_p(1), 16, None, 1, 0, ctypes.byref(best),
                          ctypes.byref(ms)) == sph.SPH_E_ARG
    # serial_passes is 0 or 1
    assert L.sph_arena_bytes(arr, 1, ctypes.byref(sph.make_options(serial_passes=2))) == 0
    assert L.sph_arena_bytes(arr, 1, ctypes.byref(sph.make_options(serial_passes=1))) > 0
    # the autotuner's cache key depends on the scene shapes, not on the tuned fields
    import paper_1911_13255_amd.sph as S
    assert S.make_options(lanes_per_particle=4).as_dict()["lanes_per_particle"] == 4


def test_split_solid_option_is_validated_and_sized():
    # solid_parts: negative values are rejected; a target that splits the
    # channel's plate adds the exchange buffers to the arena
    import ctypes

    from paper_1911_13255_amd import scenes, sph

    L = sph.lib()
    arr, keep = sph.scene_array([scenes.plate_behind_cylinder(seed=1)])
    assert L.sph_arena_bytes(arr, 1, ctypes.byref(sph.make_options(solid_parts=-1))) == 0
    plain = L.sph_arena_bytes(arr, 1, ctypes.byref(sph.make_options()))
    split = L.sph_arena_bytes(arr, 1, ctypes.byref(sph.make_options(solid_parts=128)))
    assert plain > 0 and split > plain
    # a target above the plate's free particles splits nothing
    assert L.sph_arena_bytes(arr, 1, ctypes.byref(sph.make_options(solid_parts=100000))) == plain


def test_solid_blocks_option_is_validated_and_sized():
    # solid_blocks: 0 or -1. A 3D solid on or near a lattice (the default
    # jitter of 1e-4 dp_S) adds the lattice grid of its bounding box and the
    # particles' offsets (16 bytes per cell) to the arena; a solid further
    # off its lattice than a quarter spacing, a 2D scene and -1 add nothing
    import ctypes

    import numpy as np

    from paper_1911_13255_amd import scenes, sph

    L = sph.lib()

    def nbytes(sc, **o):
        arr, keep = sph.scene_array([sc])
        return L.sph_arena_bytes(arr, 1, ctypes.byref(sph.make_options(**o)))

    lat = scenes.periodic_box_with_solid(dim=3, n=12, solid_lattice=True)
    jit = scenes.periodic_box_with_solid(dim=3, n=12, solid_lattice=False)
    assert nbytes(lat, solid_blocks=2) == 0 and nbytes(lat, solid_blocks=-2) == 0
    ns = len(lat["x_solid"])
    assert nbytes(lat) >= nbytes(lat, solid_blocks=-1) + 16 * ns
    assert nbytes(jit) >= nbytes(jit, solid_blocks=-1) + 16 * ns
    off = scenes.periodic_box_with_solid(dim=3, n=12, solid_lattice=True)
    xs = off["x_solid"].copy()
    xs[::2, 0] += 0.4 * off["dp_s"]
    off["x_solid"] = np.ascontiguousarray(xs)
    assert nbytes(off) == nbytes(off, solid_blocks=-1)
    flat = scenes.periodic_box_with_solid(dim=2, n=12, solid_lattice=True)
    assert nbytes(flat) == nbytes(flat, solid_blocks=-1)
