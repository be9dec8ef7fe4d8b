"""Python handle on the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline load this module; the GPU library never does.  It shares no code with
the GPU path; both take scene dicts from the seeded scene generator.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

# field ids (index order, FP64)
F_X, F_V, F_RHO, F_DRHO, F_A, F_P = 0, 1, 2, 3, 4, 5
S_U, S_V, S_A, S_F, S_DF, S_FF, S_VBAR, S_ABAR, S_N, S_B, S_N0, S_X0, S_FFP = range(10, 23)
VECTOR_FIELDS = {F_X, F_V, F_A, S_U, S_V, S_A, S_FF, S_VBAR, S_ABAR, S_N, S_N0, S_X0, S_FFP}
TENSOR_FIELDS = {S_F, S_DF, S_B}
FLUID_FIELDS = {F_X, F_V, F_RHO, F_DRHO, F_A, F_P}

_dp = C.POINTER(C.c_double)


class OraScene(C.Structure):
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
        ("riemann", C.c_int), ("density_reinit", C.c_int),
        ("material", C.c_int), ("single_step", C.c_int), ("velocity_verlet", C.c_int),
    ]


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (FP64, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-ffp-contract=off", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        vp = C.c_void_p
        L.ora_create.restype = vp
        L.ora_create.argtypes = [C.POINTER(OraScene)]
        for name in ("ora_destroy", "ora_rebuild", "ora_fluid_step", "ora_couple",
                     "ora_solid_substeps", "ora_step"):
            getattr(L, name).argtypes = [vp]
            getattr(L, name).restype = None
        L.ora_advance.argtypes = [vp, C.c_int]
        L.ora_get.argtypes = [vp, C.c_int, _dp]
        L.ora_set.argtypes = [vp, C.c_int, _dp]
        L.ora_scalars.argtypes = [vp, _dp]
        L.ora_set_scalars.argtypes = [vp, _dp]
        L.ora_counters.argtypes = [vp, C.POINTER(C.c_longlong)]
        L.ora_totals.argtypes = [vp, _dp]
        L.ora_fluid_side_coupling.argtypes = [vp, _dp]
        L.ora_masses.argtypes = [vp, _dp, _dp]
        L.ora_pairs.argtypes = [vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.ora_pairs.restype = C.c_int
        for name in ("ora_kernel_W", "ora_kernel_dW"):
            getattr(L, name).argtypes = [C.c_int, C.c_double, C.c_double]
            getattr(L, name).restype = C.c_double
        L.ora_eos.argtypes = [C.c_double] * 4
        L.ora_eos.restype = C.c_double
        L.ora_eos_inv.argtypes = [C.c_double] * 4
        L.ora_eos_inv.restype = C.c_double
        L.ora_psi0.argtypes = [C.c_int, C.c_double]
        L.ora_psi0.restype = C.c_double
        L.ora_riemann.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                                  C.c_double, C.c_double, _dp, _dp, _dp, _dp, _dp]
        L.ora_nh_stress.argtypes = [C.c_int, _dp, C.c_double, C.c_double, _dp]
        L.ora_nh_energy.argtypes = [C.c_int, _dp, C.c_double, C.c_double]
        L.ora_nh_energy.restype = C.c_double
        L.ora_svk_stress.argtypes = [C.c_int, _dp, C.c_double, C.c_double, _dp]
        L.ora_svk_energy.argtypes = [C.c_int, _dp, C.c_double, C.c_double]
        L.ora_svk_energy.restype = C.c_double
        for name in ("ora_brute_pairs", "ora_grid_pairs"):
            getattr(L, name).argtypes = [C.POINTER(OraScene), _dp, C.c_int, C.c_double,
                                         C.POINTER(C.c_int), C.POINTER(C.c_int)]
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def make_scene_struct(sc: dict, riemann: int = 1, density_reinit: int = 1):
    """Marshal a scene dict into the oracle's struct; returns (struct, keepalive)."""
    keep = {}
    for k in ("x_fluid", "v_fluid", "x_wall", "n_wall", "x_solid", "v_solid"):
        a = sc.get(k)
        keep[k] = None if a is None else np.ascontiguousarray(a, dtype=np.float64)
    s = OraScene()
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
    s.riemann = int(riemann)
    s.density_reinit = int(density_reinit)
    s.material = int(sc.get("material", 0))
    s.single_step = int(sc.get("single_step", 0))
    s.velocity_verlet = int(sc.get("velocity_verlet", 0))
    return s, keep


class Oracle:
    """One scene simulated by the FP64 oracle."""

    def __init__(self, sc: dict, riemann: bool = True, density_reinit: bool = True):
        self.L = lib()
        self.dim = int(sc["dim"])
        self.nf = len(sc["x_fluid"])
        self.ns = len(sc["x_solid"])
        self.n_clamp = int(sc["n_clamp"])
        self._s, self._keep = make_scene_struct(sc, riemann, density_reinit)
        self.h = self.L.ora_create(C.byref(self._s))

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.L.ora_destroy(h)
            self.h = None

    # --- Algorithm 1 pieces
    def rebuild(self):
        self.L.ora_rebuild(self.h)

    def fluid_step(self):
        self.L.ora_fluid_step(self.h)

    def couple(self):
        self.L.ora_couple(self.h)

    def solid_substeps(self):
        self.L.ora_solid_substeps(self.h)

    def step(self, n: int = 1):
        self.L.ora_advance(self.h, int(n))

    # --- state
    def _shape(self, f):
        n = self.nf if f in FLUID_FIELDS else self.ns
        if f in VECTOR_FIELDS:
            return (n, self.dim)
        if f in TENSOR_FIELDS:
            return (n, self.dim, self.dim)
        return (n,)

    def get(self, f) -> np.ndarray:
        out = np.zeros(self._shape(f))
        self.L.ora_get(self.h, f, _ptr(out))
        return out

    def set(self, f, val):
        a = np.ascontiguousarray(np.broadcast_to(val, self._shape(f)), dtype=np.float64)
        self.L.ora_set(self.h, f, _ptr(a))

    def scalars(self) -> dict:
        out = np.zeros(12)
        self.L.ora_scalars(self.h, _ptr(out))
        keys = ("t", "dt_ac", "dt_ad", "dt_s", "adv_accum", "kappa", "need_rebuild", "psi0",
                "K", "mu", "lam", "c_s")
        return dict(zip(keys, out.tolist()))

    def set_scalars(self, d: dict):
        cur = self.scalars()
        cur.update(d)
        keys = ("t", "dt_ac", "dt_ad", "dt_s", "adv_accum", "kappa", "need_rebuild")
        arr = np.array([cur[k] for k in keys] + [0.0] * 5)
        self.L.ora_set_scalars(self.h, _ptr(arr))

    def counters(self) -> dict:
        out = (C.c_longlong * 8)()
        self.L.ora_counters(self.h, out)
        keys = ("n_ff", "n_fb", "n_sf", "n_ss", "steps", "rebuilds", "substeps", "interactions")
        return dict(zip(keys, list(out)))

    def totals(self) -> dict:
        out = np.zeros(12)
        self.L.ora_totals(self.h, _ptr(out))
        return dict(mom_fluid=out[0:3].copy(), mom_solid=out[3:6].copy(), ke_fluid=out[6],
                    ke_solid=out[7], strain_energy=out[8], sum_fF=out[9:12].copy())

    def fluid_side_coupling(self) -> np.ndarray:
        out = np.zeros(3)
        self.L.ora_fluid_side_coupling(self.h, _ptr(out))
        return out

    def masses(self):
        mf = np.zeros(self.nf)
        ms = np.zeros(self.ns)
        self.L.ora_masses(self.h, _ptr(mf), _ptr(ms))
        return mf, ms

    def pairs(self, which: int):
        n = {0: self.nf, 1: self.nf, 2: self.ns - self.n_clamp, 3: self.ns}[which]
        start = np.zeros(n + 1, dtype=np.int32)
        cnt = self.L.ora_pairs(self.h, which, start.ctypes.data_as(C.POINTER(C.c_int)), None)
        if cnt < 0:
            raise RuntimeError("pairs not built")
        idx = np.zeros(max(cnt, 1), dtype=np.int32)
        self.L.ora_pairs(self.h, which, start.ctypes.data_as(C.POINTER(C.c_int)),
                         idx.ctypes.data_as(C.POINTER(C.c_int)))
        return start, idx[:cnt]


# --- point functions (for the pins)

def kernel_W(d, r, h):
    return lib().ora_kernel_W(int(d), float(r), float(h))


def kernel_dW(d, r, h):
    return lib().ora_kernel_dW(int(d), float(r), float(h))


def eos(rho, rho0, c, gam=7.0):
    return lib().ora_eos(float(rho), float(rho0), float(c), float(gam))


def eos_inv(p, rho0, c, gam=7.0):
    return lib().ora_eos_inv(float(p), float(rho0), float(c), float(gam))


def num_threads():
    L = lib()
    L.ora_num_threads.restype = C.c_int
    return L.ora_num_threads()


def set_threads(n: int):
    """OpenMP threads of the oracle's parallel loops from now on (timing only)."""
    L = lib()
    L.ora_set_threads.argtypes = [C.c_int]
    L.ora_set_threads.restype = None
    L.ora_set_threads(int(n))


def psi0(d, h_ratio=1.3):
    return lib().ora_psi0(int(d), float(h_ratio))


def riemann(d, rho_i, rho_j, p_i, p_j, vi, vj, e, c, use_riemann=True):
    vi3 = np.zeros(3)
    vj3 = np.zeros(3)
    e3 = np.zeros(3)
    vi3[:d] = vi
    vj3[:d] = vj
    e3[:d] = e
    ps = C.c_double()
    vs = np.zeros(3)
    lib().ora_riemann(int(d), int(use_riemann), float(c), float(rho_i), float(rho_j),
                      float(p_i), float(p_j), _ptr(vi3), _ptr(vj3), _ptr(e3), C.byref(ps), _ptr(vs))
    return ps.value, vs[:d]


def nh_stress(F, mu, lam):
    F = np.asarray(F, float)
    d = F.shape[0]
    F3 = np.eye(3)
    F3[:d, :d] = F
    P3 = np.zeros((3, 3))
    lib().ora_nh_stress(d, _ptr(np.ascontiguousarray(F3)), float(mu), float(lam), _ptr(P3))
    return P3[:d, :d]


def nh_energy(F, mu, lam):
    F = np.asarray(F, float)
    d = F.shape[0]
    F3 = np.eye(3)
    F3[:d, :d] = F
    return lib().ora_nh_energy(d, _ptr(np.ascontiguousarray(F3)), float(mu), float(lam))


def svk_stress(F, mu, lam):
    """First Piola-Kirchhoff stress of the linear elastic (Kirchhoff) law."""
    F = np.asarray(F, float)
    d = F.shape[0]
    F3 = np.eye(3)
    F3[:d, :d] = F
    P3 = np.zeros((3, 3))
    lib().ora_svk_stress(d, _ptr(np.ascontiguousarray(F3)), float(mu), float(lam), _ptr(P3))
    return P3[:d, :d]


def svk_energy(F, mu, lam):
    F = np.asarray(F, float)
    d = F.shape[0]
    F3 = np.eye(3)
    F3[:d, :d] = F
    return lib().ora_svk_energy(d, _ptr(np.ascontiguousarray(F3)), float(mu), float(lam))


def neighbour_lists(sc: dict, x: np.ndarray, radius: float, brute: bool):
    """CSR neighbour lists of the points x (index order) by brute force or by the
    oracle's bin grid, with the scene's box and periodic axes."""
    s, keep = make_scene_struct(sc)
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = len(x)
    fn = lib().ora_brute_pairs if brute else lib().ora_grid_pairs
    start = np.zeros(n + 1, dtype=np.int32)
    cnt = fn(C.byref(s), _ptr(x), n, float(radius), start.ctypes.data_as(C.POINTER(C.c_int)), None)
    idx = np.zeros(max(cnt, 1), dtype=np.int32)
    fn(C.byref(s), _ptr(x), n, float(radius), start.ctypes.data_as(C.POINTER(C.c_int)),
       idx.ctypes.data_as(C.POINTER(C.c_int)))
    return start, idx[:cnt]
