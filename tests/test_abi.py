"""C ABI checks that need no GPU: the built library loads, exports every function declared in
include/*.h, the Python structs match the C layout, and host-only entry points behave."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

from paper_1906_07925_amd import mpsph as M
from paper_1906_07925_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpsph.h")


def declared_functions():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"MPSPH_API\s+[\w\s\*]*?\b(mpsph_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(M.LIB_PATH):
        pytest.fail("libmpsph.so is not built (run paper_1906_07925_amd/build.py)")
    return M.lib()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 12
    out = subprocess.run(["nm", "-D", "--defined-only", M.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(mpsph_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        getattr(lib, n)


def test_struct_layout_matches_header():
    prog = r"""
#include <stdio.h>
#include <stddef.h>
#include "mpsph.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(mpsph_params), sizeof(mpsph_metrics_t),
         offsetof(mpsph_params, rbf_centre), offsetof(mpsph_params, cell_log2),
         offsetof(mpsph_metrics_t, residual_l2), offsetof(mpsph_metrics_t, elr_max));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(src, "w").write(prog)
        subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), src, "-o", exe])
        vals = [int(v) for v in subprocess.check_output([exe]).split()]
    assert vals == [C.sizeof(M.Params), C.sizeof(M.Metrics), M.Params.rbf_centre.offset,
                    M.Params.cell_log2.offset, M.Metrics.residual_l2.offset, M.Metrics.elr_max.offset]


def test_strerror_and_invalid_params(lib):
    assert lib.mpsph_strerror(0) == b"ok"
    assert lib.mpsph_strerror(99) == b"unknown status"
    p, keep = M.make_params(W.unit_square(16))
    p.dim = 4
    out = C.c_double()
    assert lib.mpsph_field_scale(C.byref(p), 16, C.byref(out)) == 1
    assert lib.mpsph_workspace_bytes(C.byref(p), 16) == 0
    ctx = C.c_void_p()
    assert lib.mpsph_create(C.byref(p), 16, None, 0, None, C.byref(ctx)) == 1
    assert lib.mpsph_step(None, 1) == 1
    assert lib.mpsph_load(None, None, None, None) == 1


def test_field_scale_matches_closed_forms(lib):
    # uniform square: s0 = (1/n)^(1/2); uniform cube: (1/n)^(1/3)
    assert M.field_scale(W.unit_square(4096), 4096) == pytest.approx(1 / 64, rel=1e-12)
    assert M.field_scale(W.unit_cube(1 << 18), 1 << 18) == pytest.approx(1 / 64, rel=1e-12)
    # ball of radius 1/2: volume pi/6
    import math
    assert M.field_scale(W.ball(10000), 10000) == pytest.approx((math.pi / 6 / 10000) ** (1 / 3), rel=1e-6)


def test_field_scale_agrees_with_oracle(lib):
    """The library's Gauss-Legendre normalisation and the oracle's midpoint rule are
    independent; both approximate the integral of rho_t (Eq. 4)."""
    from oracle import oracle as O
    for spec in (W.annulus(262144), W.cube_with_inclusion(1 << 21), W.ball(50000, dim=2)):
        a = M.field_scale(spec, spec["n"])
        b = O.OracleParams(spec).s0
        assert a == pytest.approx(b, rel=2e-4), spec["geometry"]


def test_workspace_grows_with_n(lib):
    spec = W.cube_with_inclusion(1 << 21)
    small = M.workspace_bytes(spec, 1 << 10, cell_log2=6)
    big = M.workspace_bytes(spec, 1 << 21, cell_log2=6)
    assert 0 < small < big
    assert big >= (1 << 21) * 100


def test_batch_workspace(lib):
    """A batch needs at least the particle state of all its domains and no more than the solo
    contexts together (plus per-domain tables); a batch of one equals the solo context; bad
    batches are refused (0 bytes)."""
    specs = [W.unit_square(5000), W.unit_cube(20000), W.annulus(8000), W.ball(12000)]
    ns = [s["n"] for s in specs]
    solo = [M.workspace_bytes(s, k) for s, k in zip(specs, ns)]
    both = M.batch_workspace_bytes(specs, ns)
    assert sum(ns) * 100 <= both <= sum(solo) + 65536
    assert M.batch_workspace_bytes(specs[:1], ns[:1]) == solo[0]
    assert M.batch_workspace_bytes([], []) == 0
    bad = dict(specs[1], tau=-1.0)
    assert M.batch_workspace_bytes([specs[0], bad], ns[:2]) == 0
    # cut-offs beyond the kernel's support 2h are refused, smaller ones accepted
    assert M.batch_workspace_bytes([specs[0], dict(specs[1], kappa=2.5)], ns[:2]) == 0
    assert M.batch_workspace_bytes([specs[0], dict(specs[1], kappa=1.5)], ns[:2]) > 0
    assert M.batch_workspace_bytes(specs[:2], [ns[0], -1]) == 0
