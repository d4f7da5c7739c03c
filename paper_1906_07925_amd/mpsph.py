"""Python binding of the C ABI in ``include/mpsph.h`` (argument marshalling only).

Every step of the relaxation runs in the HIP kernels of ``libmpsph.so``.  PyTorch is used
for device memory and for the current HIP stream.  There is no CPU path: if the library is
missing, every entry point raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpsph.so")

GEOMETRY = {"periodic": 0, "box": 1, "annulus": 2, "ball": 3, "levelset": 4}
FIELD = {"uniform": 0, "radial_linear": 1, "sphere_distance": 2, "rbf_exp": 3, "grid": 4}
FIELDS = {"rho": 0, "rho_t": 1, "h": 2, "a": 3, "a_abs": 4, "vt": 5, "at": 6, "v": 7, "dr": 8, "nn": 9,
          "x0": 10}
VECTOR_FIELDS = {"a", "vt", "at", "v", "dr", "x0"}
ERRORS = {1: "invalid argument", 2: "out of memory", 3: "device error", 4: "bad context state",
          5: "non-finite values", 6: "unsupported configuration", 7: "exceeds the static scratch array"}


class MpsphError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {ERRORS.get(code, 'unknown')} (status {code})")
        self.code = code


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
        ("t0", C.c_int64), ("t1", C.c_int64), ("nu_coeff", C.c_double),
        ("c_acc", C.c_double), ("c_vel", C.c_double), ("c_visc", C.c_double),
        ("cell_log2", C.c_int32), ("debug", C.c_int32),
        ("t0_window", C.c_int32), ("t0_tol", C.c_double), ("theta", C.c_double),
        ("grid_n", C.c_int32 * 3), ("grid_phi", C.POINTER(C.c_double)), ("grid_s", C.POINTER(C.c_double)),
        ("seeded", C.c_int32),
    ]


class Metrics(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("step", "pairs", "interface_pairs", "candidates", "n_normal",
                                         "n_elr", "nonfinite", "n_feature", "pairs_total", "candidates_total")] + \
               [(k, C.c_double) for k in ("residual_l2", "residual_linf", "kinetic", "dt1", "dt2", "sigma",
                                          "elr_mean", "elr_std", "elr_min", "elr_max")] + \
               [(k, C.c_int64) for k in ("interface_particles", "t0")]


MAX_FEATURES = 26


class Features(C.Structure):
    _fields_ = [("s0", C.c_double), ("mass_volume", C.c_double), ("n_volume", C.c_int64),
                ("n_features", C.c_int32), ("type", C.c_int32 * MAX_FEATURES),
                ("mass", C.c_double * MAX_FEATURES), ("count", C.c_int64 * MAX_FEATURES)]


_lib = None


def lib():
    """Load ``libmpsph.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1906_07925_amd/build.py "
                               "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        P, V, I32, I64 = C.POINTER(Params), C.c_void_p, C.c_int32, C.c_int64
        sig = {
            "mpsph_field_scale": (C.c_int, [P, I64, C.POINTER(C.c_double)]),
            "mpsph_field_bounds": (C.c_int, [P, I64, C.POINTER(C.c_double)]),
            "mpsph_feature_budget": (C.c_int, [P, I64, C.POINTER(Features)]),
            "mpsph_workspace_bytes": (C.c_size_t, [P, I64]),
            "mpsph_batch_workspace_bytes": (C.c_size_t, [I32, P, C.POINTER(I64)]),
            "mpsph_create": (C.c_int, [P, I64, V, C.c_size_t, V, C.POINTER(V)]),
            "mpsph_create_static": (C.c_int, [P, I64, V, C.POINTER(V)]),
            "mpsph_batch_create": (C.c_int, [I32, P, C.POINTER(I64), V, C.c_size_t, V, C.POINTER(V)]),
            "mpsph_domain_count": (C.c_int, [V, C.POINTER(I32), C.POINTER(I64)]),
            "mpsph_step_graph": (C.c_int, [V, I32]),
            "mpsph_domain_metrics": (C.c_int, [V, I32, I32, C.POINTER(Metrics)]),
            "mpsph_load": (C.c_int, [V, V, V, V]),
            "mpsph_step": (C.c_int, [V, I32]),
            "mpsph_metrics": (C.c_int, [V, C.POINTER(Metrics)]),
            "mpsph_store": (C.c_int, [V, V, V]),
            "mpsph_debug_fields": (C.c_int, [V, I32, V]),
            "mpsph_debug_cells": (C.c_int, [V, V, V, C.POINTER(I64), C.POINTER(I32)]),
            "mpsph_debug_pairs": (C.c_int, [V, I64, V, V, C.POINTER(I64)]),
            "mpsph_set_field_coeff": (C.c_int, [V, I32, C.POINTER(C.c_double)]),
            "mpsph_autotune": (C.c_int, [V, V, V, V, I32, I32, C.POINTER(I32), C.POINTER(I32)]),
            "mpsph_configure": (C.c_int, [V, I32, I32]),
            "mpsph_set_pair_variant": (C.c_int, [V, I32]),
            "mpsph_grad": (C.c_int, [V, I32, I32, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double), V]),
            "mpsph_profile": (C.c_int, [V, I32]),
            "mpsph_profile_read": (C.c_int, [V, I32, C.POINTER(C.c_char_p), C.POINTER(I64),
                                             C.POINTER(C.c_double), C.POINTER(I32)]),
            "mpsph_destroy": (None, [V]),
            "mpsph_strerror": (C.c_char_p, [C.c_int]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        raise MpsphError(rc, what)


def make_params(spec: dict, s0: float | None = None, cell_log2: int = -1, debug: bool = False):
    """Build the parameter block from a workload spec.  Returns (Params, keep-alive arrays)."""
    p = Params()
    d = int(spec["dim"])
    p.dim = d
    geom = spec["geometry"]
    if geom not in GEOMETRY:
        raise ValueError(f"geometry {geom!r} is not supported by the GPU library")
    p.geometry = GEOMETRY[geom]
    for a in range(3):
        p.lo[a] = spec["lo"][a] if a < d else 0.0
        p.hi[a] = spec["hi"][a] if a < d else 0.0
        p.centre[a] = spec.get("centre", (0.0,) * 3)[a] if a < d else 0.0
        p.fcentre[a] = spec.get("fcentre", (0.0,) * 3)[a] if a < d else 0.0
    p.r_in = spec.get("r_in", 0.0)
    p.r_out = spec.get("r_out", 0.0)
    p.field = FIELD[spec["field"]]
    p.fa = spec.get("fa", 0.0)
    p.fb = spec.get("fb", 0.0)
    keep = []
    n_rbf = int(spec.get("n_rbf", 0))
    p.n_rbf = n_rbf
    if n_rbf:
        cen = np.ascontiguousarray(spec["rbf_centre"], dtype=np.float64)
        coe = np.ascontiguousarray(spec["rbf_coeff"], dtype=np.float64)
        keep += [cen, coe]
        p.rbf_centre = cen.ctypes.data_as(C.POINTER(C.c_double))
        p.rbf_coeff = coe.ctypes.data_as(C.POINTER(C.c_double))
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
    if s0 is None:
        s0 = spec.get("s0")
    p.s0 = float(s0) if s0 is not None else 0.0
    p.cell_log2 = int(cell_log2)
    p.debug = 1 if debug else 0
    gn = spec.get("grid_n", (0, 0, 0))
    for a in range(3):
        p.grid_n[a] = int(gn[a]) if a < d and a < len(gn) else 0
    for key in ("grid_phi", "grid_s"):
        if key in spec:
            arr = np.ascontiguousarray(np.asarray(spec[key], dtype=np.float64).reshape(-1))
            keep.append(arr)
            setattr(p, key, arr.ctypes.data_as(C.POINTER(C.c_double)))
    p.t0_window = int(spec.get("t0_window", 50))
    p.t0_tol = float(spec.get("t0_tol", 1e-3))
    p.theta = float(spec.get("theta", 0.2))
    p.seeded = 1 if spec.get("seeded") else 0
    return p, keep


def field_scale(spec: dict, n: int) -> float:
    p, keep = make_params(spec)
    out = C.c_double(0.0)
    _check(lib().mpsph_field_scale(C.byref(p), int(n), C.byref(out)), "mpsph_field_scale")
    return out.value


def field_bounds(spec: dict, n: int) -> dict:
    """Bounds of the size field the neighbour search relies on (mpsph_field_bounds): s0, s_min,
    s_max and a Lipschitz constant of s, domain units."""
    p, keep = make_params(spec)
    out = (C.c_double * 4)()
    _check(lib().mpsph_field_bounds(C.byref(p), int(n), out), "mpsph_field_bounds")
    return dict(s0=out[0], smin=out[1], smax=out[2], lip=out[3])


def feature_budget(spec: dict, n: int) -> dict:
    """Particle budget with the boundary features seeded explicitly (mpsph_feature_budget):
    s0, the interior count and, per feature in the library's order, type, mass and count."""
    p, keep = make_params(spec)
    out = Features()
    _check(lib().mpsph_feature_budget(C.byref(p), int(n), C.byref(out)), "mpsph_feature_budget")
    k = out.n_features
    return {"s0": out.s0, "mass_volume": out.mass_volume, "n_volume": int(out.n_volume),
            "type": np.array(out.type[:k], dtype=np.int32), "mass": np.array(out.mass[:k]),
            "count": np.array(out.count[:k], dtype=np.int64)}


class Relaxer:
    """A relaxation context on the current CUDA/HIP device and stream.

    ``spec`` is one workload spec (one domain of ``n`` particles) or a list of specs (a batch of
    independent domains advanced by the same launches; ``n`` and ``s0`` are then lists too, and
    the particle arrays hold the domains one after the other).  ``static`` creates a one-domain
    context on the library's static scratch array (mpsph_create_static: no device allocation)."""

    def __init__(self, spec, n=None, s0=None, cell_log2: int = -1, debug: bool = False, stream=None,
                 static: bool = False):
        import torch
        self._torch = torch
        specs = list(spec) if isinstance(spec, (list, tuple)) else [spec]
        ns = list(n) if isinstance(n, (list, tuple)) else [n] * len(specs)
        s0s = list(s0) if isinstance(s0, (list, tuple)) else [s0] * len(specs)
        ns = [int(sp["n"] if k is None else k) for sp, k in zip(specs, ns)]
        self.ndom = len(specs)
        self.dims = [int(sp["dim"]) for sp in specs]
        self.dim = self.dims[0] if len(set(self.dims)) == 1 else None   # None: mixed 2D / 3D batch
        self.counts = ns
        self.n = sum(ns)
        self.nfloat = sum(k * d for k, d in zip(ns, self.dims))   # floats of a position array
        made = [make_params(sp, s0=z, cell_log2=cell_log2, debug=debug) for sp, z in zip(specs, s0s)]
        self.params = (Params * self.ndom)(*[m[0] for m in made])
        self.lanes = 4
        self._keep = [m[1] for m in made]
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self._ctx = C.c_void_p()
        if static:
            if self.ndom != 1:
                raise ValueError("a static-scratch context holds one domain")
            _check(lib().mpsph_create_static(C.byref(self.params[0]), ns[0], C.c_void_p(stream.cuda_stream),
                                             C.byref(self._ctx)), "mpsph_create_static")
            return
        cnt = (C.c_int64 * self.ndom)(*ns)
        _check(lib().mpsph_batch_create(self.ndom, self.params, cnt, None, 0, C.c_void_p(stream.cuda_stream),
                                        C.byref(self._ctx)), "mpsph_batch_create")

    # -- lifecycle
    def close(self):
        if self._ctx:
            lib().mpsph_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, t, dtype):
        torch = self._torch
        t = torch.as_tensor(t)
        if t.device.type != "cuda" or t.dtype != dtype or not t.is_contiguous():
            t = t.to(device="cuda", dtype=dtype).contiguous()
        return t

    def _pos_shape(self):
        return (self.n, self.dim) if self.dim is not None else (self.nfloat,)

    def split(self, arr, vector: bool = True) -> list:
        """Per-domain views of a particle array in the context's layout (positions / vector
        quantities when ``vector``, else one value per particle)."""
        flat = arr.reshape(-1)
        out, o = [], 0
        for k, d in zip(self.counts, self.dims):
            w = k * d if vector else k
            out.append(flat[o:o + w].reshape((k, d) if vector else (k,)))
            o += w
        return out

    def load(self, x, colour, ptype=None):
        """Positions (n x dim, or for a mixed batch the flat concatenation of each domain's
        n_d x dim_d block), colours and optional types."""
        torch = self._torch
        x = self._dev(x, torch.float32)
        c = self._dev(colour, torch.int32)
        assert x.numel() == self.nfloat and c.shape == (self.n,)
        t = None if ptype is None else self._dev(ptype, torch.int32)
        self._hold = (x, c, t)
        _check(lib().mpsph_load(self._ctx, C.c_void_p(x.data_ptr()), C.c_void_p(c.data_ptr()),
                                C.c_void_p(t.data_ptr()) if t is not None else None), "mpsph_load")

    def configure(self, cell_log2: int = -1, lanes: int = 4):
        """Set the cell exponent (-1: size rule) and the lanes per particle; load again after."""
        _check(lib().mpsph_configure(self._ctx, int(cell_log2), int(lanes)), "mpsph_configure")
        self.lanes = int(lanes)

    def set_pair_variant(self, variant: str):
        """Pair-kernel variant: 'default', 'persistent' (work-queue launch over all domains) or
        'tile' (LDS-staged density pass, 3D).  Every variant computes the same step."""
        code = {"default": 0, "persistent": 1, "tile": 2}[variant]
        _check(lib().mpsph_set_pair_variant(self._ctx, code), "mpsph_set_pair_variant")

    def autotune(self, x, colour, ptype=None, probe_steps: int = 5, warm_steps: int | None = None):
        """Pick the cell size and lanes per particle by timing probe_steps steps after warm_steps
        untimed ones (default: probe_steps) from this state; the state is loaded afterwards.
        Returns (cell_log2, lanes)."""
        torch = self._torch
        x = self._dev(x, torch.float32)
        c = self._dev(colour, torch.int32)
        assert x.numel() == self.nfloat and c.shape == (self.n,)
        t = None if ptype is None else self._dev(ptype, torch.int32)
        self._hold = (x, c, t)
        k, ln = C.c_int32(0), C.c_int32(0)
        warm = probe_steps if warm_steps is None else warm_steps
        _check(lib().mpsph_autotune(self._ctx, C.c_void_p(x.data_ptr()), C.c_void_p(c.data_ptr()),
                                    C.c_void_p(t.data_ptr()) if t is not None else None, int(warm),
                                    int(probe_steps), C.byref(k), C.byref(ln)), "mpsph_autotune")
        self.lanes = ln.value
        return k.value, ln.value

    def step(self, nsteps: int = 1):
        _check(lib().mpsph_step(self._ctx, int(nsteps)), "mpsph_step")

    def step_graph(self, nsteps: int = 1):
        """The same steps as ``step``, launched as one captured HIP graph."""
        _check(lib().mpsph_step_graph(self._ctx, int(nsteps)), "mpsph_step_graph")

    def metrics(self, allow_nonfinite: bool = False) -> dict:
        """Metrics of the last step of domain 0."""
        return self.domain_metrics(allow_nonfinite)[0]

    def domain_metrics(self, allow_nonfinite: bool = False) -> list:
        """Metrics of the last step of every domain."""
        m = (Metrics * self.ndom)()
        rc = lib().mpsph_domain_metrics(self._ctx, 0, self.ndom, m)
        if rc != 0 and not (allow_nonfinite and rc == 5):
            raise MpsphError(rc, "mpsph_domain_metrics")
        return [{k: getattr(m[d], k) for k, _ in Metrics._fields_} for d in range(self.ndom)]

    def store(self):
        torch = self._torch
        x = torch.empty(self._pos_shape(), dtype=torch.float32, device="cuda")
        t = torch.empty((self.n,), dtype=torch.int32, device="cuda")
        _check(lib().mpsph_store(self._ctx, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr())), "mpsph_store")
        return x, t

    def field(self, name: str):
        torch = self._torch
        shape = self._pos_shape() if name in VECTOR_FIELDS else (self.n,)
        out = torch.empty(shape, dtype=torch.float32, device="cuda")
        _check(lib().mpsph_debug_fields(self._ctx, FIELDS[name], C.c_void_p(out.data_ptr())),
               f"mpsph_debug_fields({name})")
        return out

    def cells(self):
        torch = self._torch
        nc = C.c_int64(0)
        k = C.c_int32(0)
        _check(lib().mpsph_debug_cells(self._ctx, None, None, C.byref(nc), C.byref(k)), "mpsph_debug_cells")
        keys = torch.empty((self.n,), dtype=torch.int32, device="cuda")
        cstart = torch.empty((nc.value + 1,), dtype=torch.int32, device="cuda")
        _check(lib().mpsph_debug_cells(self._ctx, C.c_void_p(keys.data_ptr()), C.c_void_p(cstart.data_ptr()),
                                       C.byref(nc), C.byref(k)), "mpsph_debug_cells")
        return keys, cstart, k.value

    def pairs(self):
        """Ordered neighbour pairs (i, j) of the last step (load indices, unspecified order)."""
        torch = self._torch
        cnt = C.c_int64(0)
        _check(lib().mpsph_debug_pairs(self._ctx, 0, None, None, C.byref(cnt)), "mpsph_debug_pairs")
        m = cnt.value
        pi = torch.empty((max(m, 1),), dtype=torch.int32, device="cuda")
        pj = torch.empty((max(m, 1),), dtype=torch.int32, device="cuda")
        _check(lib().mpsph_debug_pairs(self._ctx, m, C.c_void_p(pi.data_ptr()), C.c_void_p(pj.data_ptr()),
                                       C.byref(cnt)), "mpsph_debug_pairs")
        assert cnt.value == m
        return pi[:m], pj[:m]

    def cell_log2(self) -> int:
        nc = C.c_int64(0)
        k = C.c_int32(0)
        _check(lib().mpsph_debug_cells(self._ctx, None, None, C.byref(nc), C.byref(k)), "mpsph_debug_cells")
        return k.value

    def ncells(self) -> int:
        """Cells of the cell table (all domains, x sub-cells included)."""
        nc = C.c_int64(0)
        k = C.c_int32(0)
        _check(lib().mpsph_debug_cells(self._ctx, None, None, C.byref(nc), C.byref(k)), "mpsph_debug_cells")
        return nc.value

    def set_field_coeff(self, coeff, domain: int = 0):
        """New RBF coefficients of one domain's size field (s0 and the cell grid are kept)."""
        c = np.ascontiguousarray(np.asarray(coeff, dtype=np.float64).reshape(-1))
        _check(lib().mpsph_set_field_coeff(self._ctx, int(domain), c.ctypes.data_as(C.POINTER(C.c_double))),
               "mpsph_set_field_coeff")

    def grad(self, nsteps: int, ckpt_every: int = 10, lam: float = 1.0, n_rbf: int = 0, want_pos: bool = False):
        """Run nsteps steps and return (loss, dL/dcoeff (numpy, n_rbf), dL/dx0 (device tensor or
        None)) by the library's adjoint."""
        torch = self._torch
        loss = C.c_double(0.0)
        gc = np.zeros(max(int(n_rbf), 1), dtype=np.float64)
        gx = torch.empty(self._pos_shape(), dtype=torch.float32, device="cuda") if want_pos else None
        _check(lib().mpsph_grad(self._ctx, int(nsteps), int(ckpt_every), float(lam), C.byref(loss),
                                gc.ctypes.data_as(C.POINTER(C.c_double)),
                                C.c_void_p(gx.data_ptr()) if gx is not None else None), "mpsph_grad")
        return loss.value, gc[:int(n_rbf)], gx

    def profile(self, on):
        """True: time every kernel launch; "pairs": only the pair passes; False: stop."""
        _check(lib().mpsph_profile(self._ctx, 2 if on == "pairs" else (1 if on else 0)), "mpsph_profile")

    def profile_read(self) -> dict:
        cap = 64
        names = (C.c_char_p * cap)()
        launches = (C.c_int64 * cap)()
        ms = (C.c_double * cap)()
        cnt = C.c_int32(0)
        _check(lib().mpsph_profile_read(self._ctx, cap, names, launches, ms, C.byref(cnt)), "mpsph_profile_read")
        return {names[i].decode(): (launches[i], ms[i]) for i in range(min(cnt.value, cap))}


def workspace_bytes(spec: dict, n: int, cell_log2: int = -1) -> int:
    p, keep = make_params(spec, cell_log2=cell_log2)
    return int(lib().mpsph_workspace_bytes(C.byref(p), int(n)))


def batch_workspace_bytes(specs: list, ns: list, cell_log2: int = -1) -> int:
    made = [make_params(sp, cell_log2=cell_log2) for sp in specs]
    ps = (Params * len(specs))(*[m[0] for m in made])
    cnt = (C.c_int64 * len(specs))(*[int(k) for k in ns])
    return int(lib().mpsph_batch_workspace_bytes(len(specs), ps, cnt))


def relax_loss_function():
    """A torch.autograd.Function: RelaxLoss.apply(coeff, x0, relaxer, colour, ptype, nsteps,
    ckpt_every, lam) runs the relaxation from positions x0 with RBF coefficients coeff (float64
    CPU tensor) and returns the loss; backward supplies dL/dcoeff and dL/dx0 from the library's
    adjoint, computed together with the forward."""
    import torch

    class RelaxLoss(torch.autograd.Function):
        @staticmethod
        def forward(fctx, coeff, x0, relaxer, colour, ptype, nsteps, ckpt_every, lam):
            relaxer.set_field_coeff(coeff.detach().cpu().numpy())
            relaxer.load(x0.detach(), colour, ptype)
            loss, gc, gx = relaxer.grad(nsteps, ckpt_every, lam, n_rbf=coeff.numel(), want_pos=True)
            fctx.save_for_backward(torch.as_tensor(gc, dtype=coeff.dtype), gx.reshape(x0.shape).to(x0.dtype))
            return torch.tensor(loss, dtype=torch.float64)

        @staticmethod
        def backward(fctx, gout):
            gc, gx = fctx.saved_tensors
            return (gout.to(gc.dtype) * gc, gout.to(gx.device, gx.dtype) * gx, None, None, None, None, None, None)

    return RelaxLoss
