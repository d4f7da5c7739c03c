"""ctypes binding of the FP64 CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark.  The product path never imports this module.

The oracle computes one relaxation step of the multi-phase SPH mesh generator of
Ji, Fu, Hu & Adams (arXiv 1906.07925), Algorithm 1, in double precision; see
``mpsph_oracle.c`` for the equations each part follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")

GEOMETRY = {"periodic": 0, "box": 1, "annulus": 2, "ball": 3, "levelset": 4}
FIELD = {"uniform": 0, "radial_linear": 1, "sphere_distance": 2, "rbf_exp": 3, "grid": 4}
NORMAL, SURFACE, CURVE, FIXED = 0, 1, 2, 3


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (FP64, OpenMP).  Returns the library path."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           os.path.join(_HERE, "mpsph_oracle.c"), "-o", _SO + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(_SO + ".tmp", _SO)
    return _SO


class Params(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("geometry", C.c_int32),
        ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("centre", C.c_double * 3),
        ("r_in", C.c_double), ("r_out", C.c_double),
        ("field", C.c_int32), ("s0", C.c_double), ("fcentre", C.c_double * 3),
        ("fa", C.c_double), ("fb", C.c_double),
        ("n_rbf", C.c_int32), ("rbf_centre", C.POINTER(C.c_double)),
        ("rbf_coeff", C.POINTER(C.c_double)), ("rbf_width", C.c_double),
        ("tau", C.c_double), ("kappa", C.c_double), ("p0", C.c_double), ("sigma0", C.c_double),
        ("t0", C.c_int64), ("t1", C.c_int64),
        ("nu_coeff", C.c_double), ("c_acc", C.c_double), ("c_vel", C.c_double),
        ("c_visc", C.c_double), ("search", C.c_int32), ("seeded", C.c_int32),
        ("grid_n", C.c_int32 * 3), ("pad2_", C.c_int32),
        ("grid_phi", C.POINTER(C.c_double)), ("grid_s", C.POINTER(C.c_double)),
    ]


_DP = C.POINTER(C.c_double)


class Out(C.Structure):
    _fields_ = [(k, _DP) for k in ("rho", "rho_t", "h", "a", "a_abs", "vt", "at", "at_abs", "v",
                                   "dr", "nn", "a_kabs", "at_kabs", "at_prop", "at_prop_k", "at_prop_kn")] + [
        (k, C.c_double) for k in ("dt1", "dt2", "sigma", "residual_l2", "residual_linf", "kinetic",
                                  "elr_mean", "elr_std", "elr_min", "elr_max")] + [
        (k, C.c_int64) for k in ("pairs", "interface_pairs", "band_pairs", "n_normal", "n_elr",
                                 "nonfinite", "interface_particles")]


_N_ARRAYS = sum(1 for _, t in Out._fields_ if t is _DP)
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        L.orc_kernel_w.restype = C.c_double
        L.orc_kernel_w.argtypes = [C.c_double, C.c_double, C.c_int32]
        L.orc_kernel_dw.restype = C.c_double
        L.orc_kernel_dw.argtypes = [C.c_double, C.c_double, C.c_int32]
        L.orc_sigma.restype = C.c_double
        L.orc_sigma.argtypes = [C.POINTER(Params), C.c_int64]
        L.orc_spacing.restype = C.c_double
        L.orc_spacing.argtypes = [C.POINTER(Params), _DP]
        L.orc_level_set.restype = C.c_double
        L.orc_level_set.argtypes = [C.POINTER(Params), _DP]
        L.orc_field.restype = C.c_int
        L.orc_field.argtypes = [C.POINTER(Params), C.c_int64, _DP, _DP, _DP]
        L.orc_field_integral.restype = C.c_double
        L.orc_field_integral.argtypes = [C.POINTER(Params), C.c_int32]
        L.orc_step.restype = C.c_int
        L.orc_step.argtypes = [C.POINTER(Params), C.c_int64, _DP, C.POINTER(C.c_int32),
                               C.POINTER(C.c_int32), C.c_int64, C.POINTER(Out)]
        L.orc_pairs.restype = C.c_int
        L.orc_pairs.argtypes = [C.POINTER(Params), C.c_int64, _DP, C.c_int64,
                                C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.orc_threads.restype = C.c_int
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_DP)


class OracleParams:
    """Holds the ctypes parameter block plus the arrays it points to."""

    def __init__(self, spec: dict, s0: float | None = None, search: str = "grid"):
        p = Params()
        d = int(spec["dim"])
        p.dim = d
        p.geometry = GEOMETRY[spec["geometry"]]
        for a in range(3):
            p.lo[a] = spec["lo"][a] if a < d else 0.0
            p.hi[a] = spec["hi"][a] if a < d else 0.0
            p.centre[a] = spec.get("centre", (0.0, 0.0, 0.0))[a] if a < d else 0.0
            p.fcentre[a] = spec.get("fcentre", (0.0, 0.0, 0.0))[a] if a < d else 0.0
        p.r_in = spec.get("r_in", 0.0)
        p.r_out = spec.get("r_out", 0.0)
        p.field = FIELD[spec["field"]]
        p.fa = spec.get("fa", 0.0)
        p.fb = spec.get("fb", 0.0)
        self._rbf_c = np.ascontiguousarray(spec.get("rbf_centre", np.zeros((1, d))), dtype=np.float64)
        self._rbf_k = np.ascontiguousarray(spec.get("rbf_coeff", np.zeros(1)), dtype=np.float64)
        p.n_rbf = int(spec.get("n_rbf", 0))
        p.rbf_centre = _dp(self._rbf_c)
        p.rbf_coeff = _dp(self._rbf_k)
        p.rbf_width = spec.get("rbf_width", 0.15)
        p.tau = spec.get("tau", 1.3)
        p.kappa = spec.get("kappa", 2.0)
        p.p0 = spec.get("p0", 1.0)
        p.sigma0 = spec.get("sigma0", 3.0)
        p.t0 = int(spec.get("t0", -1))
        p.t1 = int(spec.get("t1", -1))
        p.nu_coeff = spec.get("nu_coeff", 0.1)
        p.c_acc = spec.get("c_acc", 0.25)
        p.c_vel = spec.get("c_vel", 1.0 / 40.0)
        p.c_visc = spec.get("c_visc", 0.125)
        p.search = 1 if search == "brute" else 0
        p.seeded = 1 if spec.get("seeded") else 0
        # background mesh: node values, x index fastest
        gn = spec.get("grid_n", (2, 2, 2))
        for a in range(3):
            p.grid_n[a] = int(gn[a]) if a < d else 1
        self._gphi = np.ascontiguousarray(np.asarray(spec.get("grid_phi", np.zeros(1)), dtype=np.float64).reshape(-1))
        self._gs = np.ascontiguousarray(np.asarray(spec.get("grid_s", np.zeros(1)), dtype=np.float64).reshape(-1))
        p.grid_phi = _dp(self._gphi)
        p.grid_s = _dp(self._gs)
        p.s0 = 1.0
        self.p = p
        self.dim = d
        if s0 is None:
            s0 = spec.get("s0")
        if s0 is None:
            s0 = normalised_s0(self, int(spec["n"]))
        self.p.s0 = float(s0)

    @property
    def s0(self) -> float:
        return self.p.s0


def grid_interp(op: OracleParams, which: str, x: np.ndarray):
    """Interpolated background-mesh value ('phi' or 's') and gradient at each row of x."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    nodes = op.p.grid_phi if which == "phi" else op.p.grid_s
    v = np.empty(x.shape[0])
    g = np.zeros((x.shape[0], 3))
    lib().orc_grid_interp.restype = C.c_double
    lib().orc_grid_interp.argtypes = [C.POINTER(Params), _DP, _DP, _DP]
    for i in range(x.shape[0]):
        gi = np.zeros(3)
        v[i] = lib().orc_grid_interp(C.byref(op.p), nodes, _dp(np.ascontiguousarray(x[i])), _dp(gi))
        g[i] = gi
    return v, g[:, :x.shape[1]]


def field_integral(op: OracleParams, nq: int = 2048) -> float:
    """Integral over the meshing region of rho_t with the current s0 (Eq. 4)."""
    return lib().orc_field_integral(C.byref(op.p), int(nq))


def normalised_s0(op: OracleParams, n: int, nq: int | None = None) -> float:
    """s0 such that the integral of rho_t = s^-d over the region equals n (Eq. 4 used to fix
    the field constant from the particle count, with unit particle mass, Eq. 15)."""
    if nq is None:
        nq = 4096 if op.dim == 2 else 400
    saved = op.p.s0
    op.p.s0 = 1.0
    integral = field_integral(op, nq)
    op.p.s0 = saved
    return (integral / n) ** (1.0 / op.dim)


def features(op: OracleParams, nq: int = 1024):
    """Boundary features of the region (Eq. 6 with the reading of orc_features): arrays of the
    integral of s^-power over each feature at the current s0, its particle type and its power."""
    I = np.zeros(26)
    typ = np.zeros(26, dtype=np.int32)
    pw = np.zeros(26, dtype=np.int32)
    lib().orc_features.restype = C.c_int32
    lib().orc_features.argtypes = [C.POINTER(Params), C.c_int32, _DP, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    m = lib().orc_features(C.byref(op.p), int(nq), _dp(I), typ.ctypes.data_as(C.POINTER(C.c_int32)),
                           pw.ctypes.data_as(C.POINTER(C.c_int32)))
    return I[:m], typ[:m], pw[:m]


def feature_budget(op: OracleParams, n: int, nq: int = 1024, nq_volume: int | None = None) -> dict:
    """Particle budget with the boundary features seeded explicitly: with unit particle mass
    (Eq. 15) the count is the total mass M_v + M_s (Eq. 4-6), so u = 1/s0 solves
    n = sum over terms of I u^power (volume: power dim).  Solved by bisection on u."""
    saved = op.p.s0
    op.p.s0 = 1.0
    if nq_volume is None:
        nq_volume = 4096 if op.dim == 2 else 400
    Iv = field_integral(op, nq_volume)
    I, typ, pw = features(op, nq)
    op.p.s0 = saved
    d = op.dim

    def total(u):
        return Iv * u ** d + float(np.sum(I * u ** pw.astype(np.float64)))

    lo_u, hi_u = 0.0, 1.0
    while total(hi_u) < n:
        hi_u *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo_u + hi_u)
        if total(mid) < n:
            lo_u = mid
        else:
            hi_u = mid
    u = 0.5 * (lo_u + hi_u)
    mass = I * u ** pw.astype(np.float64)
    count = np.where(pw == 0, 1, np.rint(mass)).astype(np.int64)
    return {"s0": 1.0 / u, "mass_volume": Iv * u ** d, "n_volume": int(n - count.sum()), "type": typ,
            "mass": mass, "count": count, "power": pw}


def kernel_w(r: float, h: float, dim: int) -> float:
    return lib().orc_kernel_w(r, h, dim)


def kernel_dw(r: float, h: float, dim: int) -> float:
    return lib().orc_kernel_dw(r, h, dim)


def sigma(op: OracleParams, step: int) -> float:
    return lib().orc_sigma(C.byref(op.p), int(step))


def field(op: OracleParams, x: np.ndarray):
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = x.shape[0]
    rt = np.empty(n)
    h = np.empty(n)
    lib().orc_field(C.byref(op.p), n, _dp(x), _dp(rt), _dp(h))
    return rt, h


def level_set(op: OracleParams, x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    return np.array([lib().orc_level_set(C.byref(op.p), _dp(np.ascontiguousarray(x[i])))
                     for i in range(x.shape[0])])


def step(op: OracleParams, x: np.ndarray, colour: np.ndarray, ptype: np.ndarray, step_index: int,
         want: tuple = ("rho", "rho_t", "h", "a", "a_abs", "vt", "at", "at_abs", "v", "dr", "nn", "a_kabs",
                        "at_kabs", "at_prop", "at_prop_k", "at_prop_kn")):
    """Run one step.  Returns (new_x, new_type, result dict)."""
    x = np.array(x, dtype=np.float64, order="C", copy=True)
    n, d = x.shape
    col = np.ascontiguousarray(colour, dtype=np.int32)
    typ = np.array(ptype, dtype=np.int32, order="C", copy=True)
    out = Out()
    arrays = {}
    for k in ("rho", "rho_t", "h", "a_abs", "at_abs", "nn", "a_kabs", "at_kabs", "at_prop", "at_prop_k", "at_prop_kn"):
        if k in want:
            arrays[k] = np.zeros(n)
    for k in ("a", "vt", "at", "v", "dr"):
        if k in want:
            arrays[k] = np.zeros((n, d))
    for k, arr in arrays.items():
        setattr(out, k, _dp(arr))
    rc = lib().orc_step(C.byref(op.p), n, _dp(x), col.ctypes.data_as(C.POINTER(C.c_int32)),
                        typ.ctypes.data_as(C.POINTER(C.c_int32)), int(step_index), C.byref(out))
    if rc != 0:
        raise RuntimeError(f"orc_step failed with code {rc}")
    res = dict(arrays)
    for k, _ in Out._fields_[_N_ARRAYS:]:
        res[k] = getattr(out, k)
    return x, typ, res


def pairs(op: OracleParams, x: np.ndarray):
    """Ordered pairs (i, j) with r_ij < kappa h_ij (no type mask), sorted lexicographically."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = x.shape[0]
    cnt = C.c_int64(0)
    z = np.zeros(1, dtype=np.int64)
    P64 = C.POINTER(C.c_int64)
    lib().orc_pairs(C.byref(op.p), n, _dp(x), 0, z.ctypes.data_as(P64), z.ctypes.data_as(P64),
                    C.byref(cnt))
    m = cnt.value
    pi = np.zeros(max(m, 1), dtype=np.int64)
    pj = np.zeros(max(m, 1), dtype=np.int64)
    lib().orc_pairs(C.byref(op.p), n, _dp(x), m, pi.ctypes.data_as(P64), pj.ctypes.data_as(P64),
                    C.byref(cnt))
    pi, pj = pi[:m], pj[:m]
    o = np.lexsort((pj, pi))
    return pi[o], pj[o]


def threads() -> int:
    return lib().orc_threads()
