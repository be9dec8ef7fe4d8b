"""Python binding of libmrsph (argument marshalling only).

Every step of the method runs in the library's HIP kernels; PyTorch provides
the device arena (one uint8 tensor) and the stream.  The entry points keep the
C names: ``neighbor_build``, ``fluid_step``, ``couple``, ``solid_substeps``,
``advance`` (sph_advance), ``read``/``write`` (sph_read/sph_write), ...
"""
from __future__ import annotations

import ctypes as C
import json
import os
import re

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmrsph.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "mrsph.h")

SPH_OK, SPH_E_ARG, SPH_E_HIP, SPH_E_ORDER, SPH_E_CAPACITY, SPH_E_UNSTABLE = 0, -1, -2, -3, -4, -5
SPH_FALLBACK = 1  # info code of sph_sync
K_FLUID_FORCE, K_CONTINUITY, K_COUPLE, K_SOLID, K_REBUILD = 0, 1, 2, 3, 4
F_X, F_V, F_RHO, F_DRHO, F_A, F_P, F_NNB = 0, 1, 2, 3, 4, 5, 6
S_U, S_V, S_A, S_F, S_DF, S_FF, S_VBAR, S_ABAR, S_N, S_B, S_N0, S_X0 = range(10, 22)
FLUID_FIELDS = {F_X, F_V, F_RHO, F_DRHO, F_A, F_P, F_NNB}
VECTOR_FIELDS = {F_X, F_V, F_A, S_U, S_V, S_A, S_FF, S_VBAR, S_ABAR, S_N, S_N0, S_X0}
TENSOR_FIELDS = {S_F, S_DF, S_B}

_dp = C.POINTER(C.c_double)


class SphError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mrsph error {code}: {msg}")
        self.code = code


class SphScene(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("n_fluid", C.c_int), ("n_wall", C.c_int), ("n_solid", C.c_int),
        ("n_clamp", C.c_int),
        ("dp_f", C.c_double), ("dp_s", C.c_double), ("h_ratio", C.c_double),
        ("rho0_f", C.c_double), ("c_f", C.c_double), ("eta", C.c_double), ("gamma", C.c_double),
        ("g", C.c_double * 3),
        ("rho0_s", C.c_double), ("E", C.c_double), ("nu", C.c_double),
        ("cfl_ac", C.c_double), ("cfl_ad", C.c_double), ("cfl_s", C.c_double), ("u_ref", C.c_double),
        ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("periodic", C.c_int * 3),
        ("hydro_H", C.c_double),
        ("inflow_U0", C.c_double), ("inflow_ts", C.c_double), ("inflow_H", C.c_double),
        ("inflow_len", C.c_double),
        ("x_fluid", _dp), ("v_fluid", _dp), ("x_wall", _dp), ("nrm_wall", _dp),
        ("x_solid", _dp), ("v_solid", _dp),
        ("material", C.c_int), ("single_step", C.c_int),
    ]


class SphOptions(C.Structure):
    _fields_ = [("riemann", C.c_int), ("density_reinit", C.c_int), ("max_solid_nbr", C.c_int),
                ("solid_block", C.c_int), ("lanes_per_particle", C.c_int), ("block_pair", C.c_int),
                ("solid_lds", C.c_int), ("max_fluid_nbr", C.c_int), ("max_boundary_nbr", C.c_int),
                ("serial_passes", C.c_int), ("solid_parts", C.c_int), ("fluid_tiles", C.c_int),
                ("solid_blocks", C.c_int)]

    def as_dict(self) -> dict:
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


def exported_names():
    """Function names declared in the headers under include/."""
    inc = os.path.dirname(HEADER)
    names = set()
    for h in sorted(os.listdir(inc)):
        if not h.endswith(".h"):
            continue
        txt = open(os.path.join(inc, h)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names |= set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", txt))
    return sorted(names - {"defined"})


_lib = None


def lib():
    """Load libmrsph.so; fails loudly when the HIP library is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                               "(python -c 'import __graft_entry__ as g; g.build()')")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.sph_arena_bytes.restype = C.c_size_t
        L.sph_arena_bytes.argtypes = [C.POINTER(SphScene), C.c_int, C.POINTER(SphOptions)]
        L.sph_init.argtypes = [C.POINTER(SphScene), C.c_int, C.POINTER(SphOptions), vp, C.c_size_t, vp,
                               C.POINTER(vp)]
        for name in ("neighbor_build", "fluid_step", "couple", "solid_substeps", "sph_sync"):
            getattr(L, name).argtypes = [vp]
        L.sph_advance.argtypes = [vp, C.c_int]
        L.sph_read.argtypes = [vp, C.c_int, C.c_int, _dp]
        L.sph_write.argtypes = [vp, C.c_int, C.c_int, _dp]
        L.sph_scalars.argtypes = [vp, C.c_int, _dp]
        L.sph_set_scalars.argtypes = [vp, C.c_int, _dp]
        L.sph_counters.argtypes = [vp, C.c_int, C.POINTER(C.c_ulonglong)]
        L.sph_launch_config.argtypes = [vp, C.POINTER(C.c_int)]
        L.sph_solid_table.argtypes = [vp, C.POINTER(C.c_int)]
        L.sph_fluid_tiles.argtypes = [vp, C.POINTER(C.c_longlong)]
        L.sph_set_surrogate.argtypes = [vp, vp, C.POINTER(C.c_float), C.c_float, C.c_int]
        L.sph_solid_features.argtypes = [vp, vp, vp]
        L.sph_solid_targets.argtypes = [vp, vp]
        L.sph_surrogate_counters.argtypes = [vp, C.c_int, C.POINTER(C.c_ulonglong)]
        L.sph_surrogate_residual.argtypes = [vp, C.c_int, C.POINTER(C.c_double)]
        L.sph_autotune.argtypes = [C.POINTER(SphScene), C.c_int, C.POINTER(SphOptions), vp, C.c_size_t, vp,
                                   C.c_int, C.c_int, C.POINTER(SphOptions), _dp]
        L.sph_reduce.argtypes = [vp, C.c_int, _dp]
        L.sph_reduce_noalloc.argtypes = [vp, C.c_int, C.c_int, vp]
        L.sph_time_kernel.argtypes = [vp, C.c_int, C.c_int, _dp]
        L.sph_pairs.argtypes = [vp, C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.sph_last_error.restype = C.c_char_p
        L.sph_last_error.argtypes = [vp]
        L.sph_destroy.argtypes = [vp]
        L.sph_destroy.restype = None
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def scene_struct(sc: dict):
    """Marshal a scene dict (see scenes.py) into the C struct; returns (struct, keepalive)."""
    keep = {}
    for k in ("x_fluid", "v_fluid", "x_wall", "n_wall", "x_solid", "v_solid"):
        a = sc.get(k)
        keep[k] = None if a is None else np.ascontiguousarray(a, dtype=np.float64)
    s = SphScene()
    s.dim = int(sc["dim"])
    s.n_fluid = len(keep["x_fluid"])
    s.n_wall = len(keep["x_wall"])
    s.n_solid = len(keep["x_solid"])
    s.n_clamp = int(sc["n_clamp"])
    for k in ("dp_f", "dp_s", "h_ratio", "rho0_f", "c_f", "eta", "gamma", "rho0_s", "E", "nu",
              "cfl_ac", "cfl_ad", "cfl_s", "u_ref", "hydro_H", "inflow_U0", "inflow_ts",
              "inflow_H", "inflow_len"):
        setattr(s, k, float(sc[k]))
    for k in range(3):
        s.g[k] = float(sc["g"][k])
        s.lo[k] = float(sc["lo"][k])
        s.hi[k] = float(sc["hi"][k])
        s.periodic[k] = int(sc["periodic"][k])
    for k, a in keep.items():
        setattr(s, "nrm_wall" if k == "n_wall" else k, _ptr(a))
    s.material = int(sc.get("material", 0))
    s.single_step = int(sc.get("single_step", 0))
    return s, keep


def scene_array(scenes):
    """C array of scene structs plus the host arrays it points into."""
    arr = (SphScene * len(scenes))()
    keep = []
    for i, sc in enumerate(scenes):
        st, k = scene_struct(sc)
        arr[i] = st
        keep.append(k)
    return arr, keep


def make_options(riemann=True, density_reinit=1, max_solid_nbr=0, solid_block=0, lanes_per_particle=0,
                 block_pair=0, solid_lds=0, max_fluid_nbr=0, max_boundary_nbr=0, serial_passes=0, solid_parts=0,
                 fluid_tiles=0, solid_blocks=0):
    return SphOptions(int(riemann), int(density_reinit), int(max_solid_nbr), int(solid_block),
                      int(lanes_per_particle), int(block_pair), int(solid_lds), int(max_fluid_nbr),
                      int(max_boundary_nbr), int(serial_passes), int(solid_parts), int(fluid_tiles),
                      int(solid_blocks))


def workload_signature(scenes, opt: dict) -> str:
    """Key of the autotuner cache: scene shapes and counts, fixed options, device."""
    import hashlib

    import torch

    h = hashlib.sha256()
    for sc in scenes:
        h.update(repr((int(sc["dim"]), len(sc["x_fluid"]), len(sc["x_wall"]), len(sc["x_solid"]),
                       int(sc["n_clamp"]), float(sc["dp_f"]), float(sc["dp_s"]))).encode())
    fixed = {k: v for k, v in opt.items()
             if k not in ("lanes_per_particle", "block_pair", "serial_passes", "solid_parts")}
    h.update(json.dumps(fixed, sort_keys=True).encode())
    h.update(torch.cuda.get_device_name(0).encode())
    return h.hexdigest()[:32]


def autotune(scenes, warmup: int = 20, steps: int = 200, cache: str = None, device: int = 0, **options) -> dict:
    """Launch shapes for these scenes chosen by the library's autotuner
    (sph_autotune), cached by workload signature in a JSON file.  Returns the
    full option set to pass to Simulation."""
    import torch

    if isinstance(scenes, dict):
        scenes = [scenes]
    L = lib()
    opt = make_options(**options)
    key = workload_signature(scenes, opt.as_dict())
    if cache and os.path.exists(cache):
        try:
            hit = json.load(open(cache)).get(key)
        except ValueError:
            hit = None
        if hit:
            return hit["options"]
    arr, keep = scene_array(scenes)
    nbytes = L.sph_arena_bytes(arr, len(scenes), C.byref(opt))
    if nbytes == 0:
        raise SphError(SPH_E_ARG, "invalid scene description")
    dev = torch.device("cuda", device)
    with torch.cuda.device(dev):
        stream = torch.cuda.Stream(device=dev)
        arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize(dev)
    best = SphOptions()
    ms = C.c_double(0.0)
    rc = L.sph_autotune(arr, len(scenes), C.byref(opt), C.c_void_p(arena.data_ptr()), nbytes + 256,
                        C.c_void_p(stream.cuda_stream), int(warmup), int(steps), C.byref(best), C.byref(ms))
    torch.cuda.synchronize(dev)
    del arena
    if rc != SPH_OK:
        raise SphError(rc, "sph_autotune failed")
    chosen = best.as_dict()
    if cache:
        try:
            db = json.load(open(cache)) if os.path.exists(cache) else {}
        except ValueError:
            db = {}
        db[key] = {"options": chosen, "ms_per_step": ms.value}
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        json.dump(db, open(cache, "w"), indent=1)
    return chosen


class Simulation:
    """One or more scenes on one GPU, advanced by the library's kernels."""

    def __init__(self, scenes, riemann: bool = True, density_reinit: int = 1,
                 max_solid_nbr: int = 0, solid_block: int = 0, lanes_per_particle: int = 0,
                 block_pair: int = 0, solid_lds: int = 0, max_fluid_nbr: int = 0,
                 max_boundary_nbr: int = 0, serial_passes: int = 0, solid_parts: int = 0, fluid_tiles: int = 0,
                 solid_blocks: int = 0, device: int = 0, arena_fill: int = None):
        """arena_fill: byte written over the whole arena before sph_init (tests
        use it to show that no result depends on the arena's prior contents)."""
        import torch

        if isinstance(scenes, dict):
            scenes = [scenes]
        self.L = lib()
        self.n_scenes = len(scenes)
        self.dim = int(scenes[0]["dim"])
        self.nf = [len(s["x_fluid"]) for s in scenes]
        self.ns = [len(s["x_solid"]) for s in scenes]
        arr, self._keep = scene_array(scenes)
        self._scene_dicts = scenes
        self._scenes = arr
        self.opt = make_options(riemann, density_reinit, max_solid_nbr, solid_block, lanes_per_particle,
                                block_pair, solid_lds, max_fluid_nbr, max_boundary_nbr, serial_passes, solid_parts,
                                fluid_tiles, solid_blocks)
        nbytes = self.L.sph_arena_bytes(arr, self.n_scenes, C.byref(self.opt))
        if nbytes == 0:
            raise SphError(SPH_E_ARG, "invalid scene description")
        self.device = torch.device("cuda", device)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.Stream(device=self.device)
            self.arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            if arena_fill is not None:
                self.arena.fill_(int(arena_fill) & 0xFF)
        torch.cuda.synchronize(self.device)
        self.arena_bytes = nbytes
        ctx = C.c_void_p()
        rc = self.L.sph_init(arr, self.n_scenes, C.byref(self.opt), C.c_void_p(self.arena.data_ptr()),
                             nbytes + 256, C.c_void_p(self.stream.cuda_stream), C.byref(ctx))
        if rc != SPH_OK:
            raise SphError(rc, "sph_init failed")
        self.ctx = ctx

    def _check(self, rc):
        """Raise on an error code; positive info codes are returned."""
        if rc < SPH_OK:
            raise SphError(rc, self.L.sph_last_error(self.ctx).decode())
        return rc

    # --- Algorithm 1 entry points (enqueue only)
    def neighbor_build(self):
        self._check(self.L.neighbor_build(self.ctx))

    def fluid_step(self):
        self._check(self.L.fluid_step(self.ctx))

    def couple(self):
        self._check(self.L.couple(self.ctx))

    def solid_substeps(self):
        self._check(self.L.solid_substeps(self.ctx))

    def step(self):
        """One acoustic step through the four separate entry points."""
        self.neighbor_build()
        self.fluid_step()
        self.couple()
        self.solid_substeps()

    def advance(self, n: int):
        """n acoustic steps, replayed from a captured HIP graph."""
        self._check(self.L.sph_advance(self.ctx, int(n)))

    def sync(self):
        return self._check(self.L.sph_sync(self.ctx))

    # --- state I/O
    def _shape(self, field, scene):
        n = self.nf[scene] if field in FLUID_FIELDS else self.ns[scene]
        if field in VECTOR_FIELDS:
            return (n, self.dim)
        if field in TENSOR_FIELDS:
            return (n, self.dim, self.dim)
        if field == F_NNB:
            return (n, 2)
        return (n,)

    def read(self, field: int, scene: int = 0) -> np.ndarray:
        out = np.zeros(self._shape(field, scene))
        self._check(self.L.sph_read(self.ctx, int(field), int(scene), _ptr(out)))
        return out

    def write(self, field: int, value, scene: int = 0):
        a = np.ascontiguousarray(np.broadcast_to(value, self._shape(field, scene)), dtype=np.float64)
        self._check(self.L.sph_write(self.ctx, int(field), int(scene), _ptr(a)))

    def scalars(self, scene: int = 0) -> dict:
        out = np.zeros(8)
        self._check(self.L.sph_scalars(self.ctx, int(scene), _ptr(out)))
        keys = ("t", "dt_ac", "dt_ad", "dt_s", "adv_accum", "kappa", "need_rebuild", "vmax")
        return dict(zip(keys, out.tolist()))

    def set_scalars(self, scene: int = 0, **kw):
        cur = self.scalars(scene)
        cur.update(kw)
        arr = np.array([cur["t"], 0.0, cur["dt_ad"], 0.0, cur["adv_accum"], 0.0,
                        float(cur["need_rebuild"]), 0.0])
        self._check(self.L.sph_set_scalars(self.ctx, int(scene), _ptr(arr)))

    # --- learned sub-step surrogate
    def _enter(self):
        import torch

        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _leave(self):
        import torch

        torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def solid_count(self) -> int:
        return sum(self.ns)

    def free_mask(self):
        """Boolean mask of the free (not clamped) solid particles, rows in solid order."""
        m = []
        for sc in self._scene_dicts:
            n, nc = len(sc["x_solid"]), int(sc["n_clamp"])
            m.append(np.r_[np.ones(n - nc, bool), np.zeros(nc, bool)])
        return np.concatenate(m) if m else np.zeros(0, bool)

    def solid_features(self, stats_dev=None, out=None):
        """(n_solid x 24) FP32 device tensor of the surrogate features now
        (call between couple and solid_substeps)."""
        import torch

        x = out if out is not None else torch.empty((self.solid_count(), 24), dtype=torch.float32, device=self.device)
        self._enter()
        self._check(self.L.sph_solid_features(self.ctx, None if stats_dev is None else C.c_void_p(stats_dev.data_ptr()),
                                              C.c_void_p(x.data_ptr())))
        self._leave()
        return x

    def solid_targets(self, out=None):
        """(n_solid x 4) FP32 device tensor of the training targets of the
        step whose features solid_features took (call after solid_substeps)."""
        import torch

        t = out if out is not None else torch.empty((self.solid_count(), 4), dtype=torch.float32, device=self.device)
        self._enter()
        self._check(self.L.sph_solid_targets(self.ctx, C.c_void_p(t.data_ptr())))
        self._leave()
        return t

    def set_surrogate(self, net, stats, threshold: float, every: int = 10):
        """net: mlp.Network (24 -> 4) or None; stats: 56 floats (feature mean,
        feature 1/std, output mean, output std); threshold and interval of the
        judge steps (see sph_set_surrogate)."""
        if net is None:
            self._check(self.L.sph_set_surrogate(self.ctx, None, None, 0.0, 1))
            self._net = None
            return
        st = np.ascontiguousarray(stats, dtype=np.float32)
        assert st.size == 56
        self._check(self.L.sph_set_surrogate(self.ctx, net.ctx, st.ctypes.data_as(C.POINTER(C.c_float)),
                                             float(threshold), int(every)))
        self._net = net  # keep the network alive while the context uses it

    def surrogate_counters(self, scene: int = -1) -> dict:
        """accepted: learned steps; fallback: plain-sub-step steps while a
        network is set (judge and plain steps); judged_ok / judged_fail."""
        out = (C.c_ulonglong * 4)()
        self._check(self.L.sph_surrogate_counters(self.ctx, int(scene), out))
        return {"accepted": int(out[0]), "fallback": int(out[1]), "judged_ok": int(out[2]),
                "judged_fail": int(out[3])}

    def surrogate_residual(self, scene: int = 0) -> float:
        """R of the scene's last judge step (NaN before the first)."""
        out = C.c_double()
        self._check(self.L.sph_surrogate_residual(self.ctx, int(scene), C.byref(out)))
        return float(out.value)

    def launch_config(self) -> dict:
        out = (C.c_int * 10)()
        self._check(self.L.sph_launch_config(self.ctx, out))
        keys = ("lpp_fluid", "lpp_couple", "block_pair", "solid_ppt", "block_solid", "cap_fluid_nbr",
                "cap_boundary_nbr", "graph", "solid_parts", "solid_workgroups")
        return dict(zip(keys, [int(x) for x in out]))

    def solid_table(self) -> dict:
        out = (C.c_int * 5)()
        self._check(self.L.sph_solid_table(self.ctx, out))
        return {"compact": int(out[0]), "capacity": int(out[1]), "bytes_per_pair": int(out[2]),
                "lattice_blocks": int(out[3]), "classes": int(out[4])}

    def fluid_tiles(self) -> dict:
        out = (C.c_longlong * 5)()
        self._check(self.L.sph_fluid_tiles(self.ctx, out))
        return dict(zip(("group", "groups", "tiled", "neighbours", "largest"), [int(x) for x in out]))

    def solid_register_resident(self) -> bool:
        return self.launch_config()["solid_ppt"] > 0

    def counters(self, scene: int = -1) -> dict:
        out = (C.c_ulonglong * 8)()
        self._check(self.L.sph_counters(self.ctx, int(scene), out))
        keys = ("n_ff", "n_fw", "n_fs", "n_ss", "steps", "rebuilds", "substeps", "interactions")
        return dict(zip(keys, [int(x) for x in out]))

    def reduce(self, scene: int = 0) -> dict:
        out = np.zeros(15)
        self._check(self.L.sph_reduce(self.ctx, int(scene), _ptr(out)))
        return dict(mom_fluid=out[0:3].copy(), mom_solid=out[3:6].copy(), ke_fluid=out[6],
                    ke_solid=out[7], strain_energy=out[8], sum_fF=out[9:12].copy(),
                    sum_fS=out[12:15].copy())

    def pairs(self, which: int, scene: int = 0):
        """(start, idx) CSR neighbour lists at the last rebuild in original
        order, rows sorted (see sph_pairs): which 0 fluid-fluid, 1 fluid-boundary
        (walls, then n_wall + free solid index), 2 free solid-fluid,
        3 solid-solid reference."""
        sc = self._scene_dicts[scene]
        n = {0: self.nf[scene], 1: self.nf[scene], 2: self.ns[scene] - int(sc["n_clamp"]),
             3: self.ns[scene]}[which]
        start = np.zeros(n + 1, dtype=np.int32)
        ip = C.POINTER(C.c_int)
        cnt = self._check(self.L.sph_pairs(self.ctx, int(which), int(scene), start.ctypes.data_as(ip), None))
        idx = np.zeros(max(cnt, 1), dtype=np.int32)
        self._check(self.L.sph_pairs(self.ctx, int(which), int(scene), start.ctypes.data_as(ip),
                                     idx.ctypes.data_as(ip)))
        return start, idx[:cnt]

    def reduce_noalloc(self, out_dev, scene: int = 0, blocks: int = 0):
        """Enqueue the reductions into out_dev (a float64 device tensor of 16
        elements) with sph_reduce_noalloc, ordered after torch's current
        stream and before its later work."""
        self._enter()
        self._check(self.L.sph_reduce_noalloc(self.ctx, int(scene), int(blocks), C.c_void_p(out_dev.data_ptr())))
        self._leave()
        return out_dev

    def time_kernel(self, kernel: int, reps: int = 100) -> float:
        """Average milliseconds per launch of one kernel (HIP events on the stream)."""
        out = C.c_double()
        self._check(self.L.sph_time_kernel(self.ctx, int(kernel), int(reps), C.byref(out)))
        return out.value

    def close(self):
        if getattr(self, "ctx", None):
            self.L.sph_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
