"""Pair-kernel variants (mpsph_set_pair_variant): the persistent work-queue launch over all
domains and the LDS-staged density pass compute the default kernels' step bit for bit, meet the
oracle's single-step bounds, and replay correctly as captured graphs (the work queue is reset
by its own launch, so graph replays need no memset)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1906_07925_amd import workloads as W
from tests import parity_util as PU

pytestmark = pytest.mark.gpu

VARIANTS = ("default", "persistent", "tile")


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_07925_amd import mpsph as M
    M.lib()
    return torch


def _run(torch, specs, ns, x, col, typ, steps, variant, k=-1, lanes=None):
    from paper_1906_07925_amd import mpsph as M
    R = M.Relaxer(specs, n=ns)
    if lanes is not None:
        R.configure(k, lanes)
    R.set_pair_variant(variant)
    R.load(torch.from_numpy(x).cuda(), torch.from_numpy(col).cuda(), torch.from_numpy(typ).cuda())
    R.step(steps)
    m = R.domain_metrics()
    xs, ts = R.store()
    R.close()
    return xs.cpu().numpy(), ts.cpu().numpy(), m


@pytest.mark.parametrize("lanes", [2, 4, 8])
def test_variants_equal_default_on_graded_cube(torch_cuda, lanes):
    """The graded cube (3D; coarse blocks overflow the staged copy and read through the caches,
    fine ones are staged): every variant ends bit-identical to the default after 5 steps."""
    cfg = W.config("cube_inclusion_2m", scale=0.02)
    x, col, typ = PU.state_f32(cfg)
    spec = dict(cfg["spec"], n=x.shape[0])
    out = {v: _run(torch_cuda, spec, x.shape[0], x, col, typ, 5, v, k=6, lanes=lanes) for v in VARIANTS}
    for v in VARIANTS[1:]:
        assert np.array_equal(out[v][0], out["default"][0]), v
        assert np.array_equal(out[v][1], out["default"][1]), v
        assert out[v][2] == out["default"][2], v


def test_variants_equal_default_on_mixed_batch(torch_cuda):
    """A shuffled batch of squares, annuli, cubes and balls with an empty domain: the persistent
    launch serves both dimensions in one launch; every variant ends bit-identical to the default."""
    cfgs = W.batched_domains(scale=0.01, n_dom=8)
    rng = np.random.Generator(np.random.PCG64(13))
    doms = []
    for k in rng.permutation(len(cfgs)):
        xd, cd, td = W.make_state(cfgs[k])
        doms.append((dict(cfgs[k]["spec"], n=xd.shape[0]), xd.astype(np.float32), cd, td))
    doms.insert(2, (dict(W.unit_square(0), n=0), np.zeros((0, 2), np.float32), np.zeros(0, np.int32),
                    np.zeros(0, np.int32)))
    x = np.concatenate([d[1].reshape(-1) for d in doms]).astype(np.float32)
    col = np.concatenate([d[2] for d in doms]).astype(np.int32)
    typ = np.concatenate([d[3] for d in doms]).astype(np.int32)
    specs, ns = [d[0] for d in doms], [d[1].shape[0] for d in doms]
    out = {v: _run(torch_cuda, specs, ns, x, col, typ, 6, v) for v in VARIANTS}
    for v in VARIANTS[1:]:
        assert np.array_equal(out[v][0], out["default"][0]), v
        assert out[v][2] == out["default"][2], v


@pytest.mark.parametrize("variant", ["persistent", "tile"])
def test_variant_single_step_parity(torch_cuda, variant):
    """The variants against the oracle with the single-step bounds of the parity tests (graded
    cube, 2^5 cells, 8 lanes)."""
    cfg = W.config("cube_inclusion_2m", scale=0.008)
    x32, col, typ = PU.state_f32(cfg)
    spec = dict(cfg["spec"], n=x32.shape[0])
    s0 = O.OracleParams(spec).s0
    errs = PU.check_single_step(spec, s0, x32, col, typ, cell_log2=5, lanes=8, variant=variant)
    print(variant, {k: f"{v:.1e}" for k, v in errs.items()})


def test_persistent_graph_replays(torch_cuda):
    """Three replays of a two-step graph of the persistent variant, with unrelated work between
    them, equal six eager default steps bit for bit."""
    torch = torch_cuda
    from paper_1906_07925_amd import mpsph as M
    cfgs = W.batched_domains(scale=0.005, n_dom=4)
    states = [W.make_state(c) for c in cfgs]
    specs = [dict(c["spec"], n=s[0].shape[0]) for c, s in zip(cfgs, states)]
    ns = [s[0].shape[0] for s in states]
    x = np.concatenate([s[0].astype(np.float32).reshape(-1) for s in states])
    col = np.concatenate([s[1] for s in states]).astype(np.int32)
    typ = np.concatenate([s[2] for s in states]).astype(np.int32)
    args = (torch.from_numpy(x).cuda(), torch.from_numpy(col).cuda(), torch.from_numpy(typ).cuda())
    E = M.Relaxer(specs, n=ns)
    G = M.Relaxer(specs, n=ns)
    G.set_pair_variant("persistent")
    E.load(*args)
    G.load(*args)
    for rep in range(3):
        E.step(2)
        G.step_graph(2)
        (torch.randn(1 << 16, device="cuda") * 2.0).sum().item()
        torch.cuda.synchronize()
        assert torch.equal(E.store()[0], G.store()[0]), rep
        assert E.domain_metrics() == G.domain_metrics(), rep
    E.close()
    G.close()
