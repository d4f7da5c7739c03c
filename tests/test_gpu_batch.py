"""Batched contexts and graph replay on the GPU.

A domain of a batch must evolve bit for bit as in a context of its own: its particles are
sorted, visited and summed in the same order, and the only cross-domain coupling, the time-step
minimum, is kept per domain.  Metric sums are FP64 reductions over differently grouped block
partials, so they agree to rounding; counts and time steps agree exactly.  A captured step
graph replays the eager launches, including the step counter that drives the surface-tension
ramp.
"""
import numpy as np
import pytest

from paper_1906_07925_amd import workloads as W

pytestmark = pytest.mark.gpu

EXACT = ("step", "pairs", "interface_pairs", "candidates", "n_normal", "n_elr", "nonfinite", "n_feature",
         "pairs_total", "candidates_total", "dt1", "dt2", "sigma", "residual_linf", "elr_min", "elr_max")


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_07925_amd import mpsph as M
    M.lib()
    return torch


def _mixed_batch(scale=0.01, n_dom=8, seed=5):
    """Squares, annuli, cubes and balls in a seeded shuffled order (2D and 3D interleaved), plus
    one empty domain; a surface-tension ramp over the first steps."""
    cfgs = W.batched_domains(scale=scale, n_dom=n_dom)
    rng = np.random.Generator(np.random.PCG64(seed))
    order = rng.permutation(len(cfgs))
    out = []
    for k in order:
        c = cfgs[k]
        x, col, typ = W.make_state(c)
        spec = dict(c["spec"], n=x.shape[0], t0=1, t1=4)
        out.append((spec, x.astype(np.float32), col, typ))
    empty = dict(W.unit_square(0), n=0)
    out.insert(3, (empty, np.zeros((0, 2), np.float32), np.zeros(0, np.int32), np.zeros(0, np.int32)))
    return out


def _concat(doms):
    x = np.concatenate([d[1].reshape(-1) for d in doms]).astype(np.float32)
    col = np.concatenate([d[2] for d in doms]).astype(np.int32)
    typ = np.concatenate([d[3] for d in doms]).astype(np.int32)
    return x, col, typ


def _run_solo(torch, spec, x, col, typ, steps):
    from paper_1906_07925_amd import mpsph as M
    R = M.Relaxer(spec, n=x.shape[0])
    R.load(torch.from_numpy(x).cuda(), torch.from_numpy(col).cuda(), torch.from_numpy(typ).cuda())
    R.step(steps)
    m = R.metrics()
    xs, ts = R.store()
    R.close()
    return xs.cpu().numpy(), ts.cpu().numpy(), m


def _metrics_agree(mb, ms):
    for k in EXACT:
        assert mb[k] == ms[k], (k, mb[k], ms[k])
    for k in ("residual_l2", "kinetic", "elr_mean", "elr_std"):
        assert abs(mb[k] - ms[k]) <= 1e-12 * max(abs(ms[k]), 1e-300), (k, mb[k], ms[k])


def test_batch_equals_solo_runs(torch_cuda):
    torch = torch_cuda
    from paper_1906_07925_amd import mpsph as M
    doms = _mixed_batch()
    steps = 6
    x, col, typ = _concat(doms)
    specs = [d[0] for d in doms]
    B = M.Relaxer(specs, n=[d[1].shape[0] for d in doms])
    assert B.ndom == len(doms) and B.dim is None
    B.load(torch.from_numpy(x).cuda(), torch.from_numpy(col).cuda(), torch.from_numpy(typ).cuda())
    B.step(steps)
    mb = B.domain_metrics()
    xb, tb = B.store()
    xb = B.split(xb.cpu().numpy())
    tb = B.split(tb.cpu().numpy(), vector=False)
    B.close()
    for k, (spec, xd, cd, td) in enumerate(doms):
        if xd.shape[0] == 0:
            assert mb[k]["pairs"] == 0 and mb[k]["pairs_total"] == 0
            continue
        xs, ts, ms = _run_solo(torch, spec, xd, cd, td, steps)
        assert np.array_equal(xb[k], xs), k
        assert np.array_equal(tb[k], ts), k
        _metrics_agree(mb[k], ms)
        assert ms["sigma"] < spec.get("sigma0", 3.0)     # the ramp was active by the last step


def test_graph_replay_matches_eager(torch_cuda):
    """Three replays of a two-step graph against six eager steps, with unrelated eager work and
    synchronisation between the replays; every replay is checked."""
    torch = torch_cuda
    from paper_1906_07925_amd import mpsph as M
    doms = _mixed_batch(scale=0.005, n_dom=4, seed=9)
    x, col, typ = _concat(doms)
    specs = [d[0] for d in doms]
    ns = [d[1].shape[0] for d in doms]
    args = (torch.from_numpy(x).cuda(), torch.from_numpy(col).cuda(), torch.from_numpy(typ).cuda())
    E = M.Relaxer(specs, n=ns)
    G = M.Relaxer(specs, n=ns)
    E.load(*args)
    G.load(*args)
    for rep in range(3):
        E.step(2)
        G.step_graph(2)
        junk = torch.randn(1 << 16, device="cuda")
        (junk * 2.0).sum().item()
        torch.cuda.synchronize()
        xe, te = E.store()
        xg, tg = G.store()
        assert torch.equal(xe, xg) and torch.equal(te, tg), rep
        me, mg = E.domain_metrics(), G.domain_metrics()
        assert me == mg, rep
        assert me[0]["step"] == 2 * rep + 1
    # a reload restarts the step counter inside the replayed graph as well
    E.load(*args)
    G.load(*args)
    E.step(2)
    G.step_graph(2)
    assert torch.equal(E.store()[0], G.store()[0])
    assert E.domain_metrics() == G.domain_metrics()
    E.close()
    G.close()


def test_batch_of_identical_domains(torch_cuda):
    """The same domain twice in one batch gives two identical trajectories."""
    torch = torch_cuda
    from paper_1906_07925_amd import mpsph as M
    cfg = W.config("annulus_262k", scale=0.01)
    x, col, typ = W.make_state(cfg)
    x = x.astype(np.float32)
    spec = dict(cfg["spec"], n=x.shape[0])
    B = M.Relaxer([spec, spec], n=[x.shape[0]] * 2)
    B.load(torch.from_numpy(np.concatenate([x, x])).cuda(), torch.from_numpy(np.concatenate([col, col])).cuda())
    B.step(5)
    xa, xb = B.split(B.store()[0])
    assert torch.equal(xa, xb)
    ma, mb = B.domain_metrics()
    _metrics_agree(ma, mb)
    B.close()


def test_batch_first_step_matches_oracle(torch_cuda):
    """Every domain of a mixed batch (squares, annuli, cubes and balls in a shuffled order, an
    empty domain among them, 2D and 3D interleaved) against the oracle directly: the first step
    of each domain, read from the batched context, meets the single-step bounds of the parity
    tests (fields, time steps, counts, positions and types)."""
    torch = torch_cuda
    from oracle import oracle as O
    from paper_1906_07925_amd import mpsph as M
    from tests import parity_util as PU
    doms = _mixed_batch(scale=0.02, n_dom=8, seed=11)
    x, col, typ = _concat(doms)
    specs = [d[0] for d in doms]
    ns = [d[1].shape[0] for d in doms]
    s0s = [O.OracleParams(sp).s0 if sp["n"] > 0 else 0.03 for sp in specs]
    B = M.Relaxer(specs, n=ns, s0=s0s, debug=True)
    B.load(torch.from_numpy(x).cuda(), torch.from_numpy(col).cuda(), torch.from_numpy(typ).cuda())
    B.step(1)
    mb = B.domain_metrics()
    fields = {}
    for name in PU.FIELDS:
        arr = B.field(name).cpu().numpy().astype(np.float64)
        fields[name] = B.split(arr, vector=name in M.VECTOR_FIELDS)
    xb, tb = B.store()
    xb = B.split(xb.cpu().numpy().astype(np.float64))
    tb = B.split(tb.cpu().numpy(), vector=False)
    B.close()
    kinds = set()
    for k, (spec, xd, cd, td) in enumerate(doms):
        if xd.shape[0] == 0:
            continue
        solo = M.Relaxer(spec, n=xd.shape[0], s0=s0s[k])
        cell_log2 = solo.cell_log2()                  # a domain keeps its own grid in a batch
        solo.close()
        g = {name: fields[name][k] for name in PU.FIELDS}
        g["x1"], g["t1"] = xb[k], tb[k]
        op, x1, t1, r = PU.oracle_step(spec, s0s[k], xd, cd, td)
        errs = PU.compare_step(spec, xd, x1, t1, r, mb[k], g, cell_log2)
        kinds.add((spec["geometry"], spec["dim"]))
        print(k, spec["geometry"], spec["dim"], xd.shape[0], {kk: f"{v:.1e}" for kk, v in errs.items()})
    assert kinds == {("box", 2), ("annulus", 2), ("box", 3), ("ball", 3)}, kinds
