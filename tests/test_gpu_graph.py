"""GPU parity of the graph-specialised afterburner (every net of two pins; JET_OPT_GRAPH_KERNELS)
against the oracle, which treats a graph as a hypergraph of two-pin nets (Algorithm 2 replayed per
net):

* recomputed gains element by element from the oracle's candidates, on a triangulated mesh, a
  power-law graph with hubs, and weighted random graphs, k from 2 to 128;
* whole refinements (all temperature rounds, rebalancing, per-iteration records) with the graph
  kernels on and off;
* the 4M-vertex mesh at full size: candidates, recomputed gains and two Jet iterations.
"""
import hashlib
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def J():
    import paper_2504_12013_amd.jet as jet
    return jet


def dev(a, dtype=torch.int32):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.int32).tobytes()).hexdigest()


def random_graph(n, m, k, seed, nw_max=1, vw_max=1):
    rng = np.random.default_rng(seed)
    a = rng.integers(0, n, 2 * m)
    b = rng.integers(0, n, 2 * m)
    keep = a != b
    e = np.unique(np.stack([np.minimum(a[keep], b[keep]), np.maximum(a[keep], b[keep])], axis=1), axis=0)[:m]
    off = np.arange(0, 2 * len(e) + 1, 2, dtype=np.int64)
    nw = rng.integers(1, nw_max + 1, len(e)).astype(np.int32) if nw_max > 1 else None
    vw = rng.integers(1, vw_max + 1, n).astype(np.int32) if vw_max > 1 else None
    hg = W.Hypergraph(n=n, m=len(e), off=off, pins=e.astype(np.int32).ravel(), k=k, eps=0.03, net_w=nw, vtx_w=vw)
    return hg, W.part_uniform(n, k, seed)


GRAPHS = {
    "mesh-k8": lambda: W.mesh_graph(side=160, k=8, seed=1),
    "mesh-k64": lambda: W.mesh_graph(side=300, k=64, seed=2),
    "powerlaw-k16": lambda: W.powerlaw_graph(n=40_000, avg_deg=10, k=16, seed=3),
    "random-weighted-k2": lambda: random_graph(5000, 20000, 2, 4, nw_max=5, vw_max=3),
    "random-weighted-k128": lambda: random_graph(20000, 60000, 128, 5, nw_max=3),
}


@pytest.mark.parametrize("name", list(GRAPHS))
def test_graph_afterburner_matches_oracle(name):
    hg, part = GRAPHS[name]()
    say(f"graph afterburner {name}: n={hg.n} m={hg.m} k={hg.k}")
    ctx = J().JetContext(hg)
    for tau in (0.0, 0.75):
        tq = O.quantize_tau(tau)
        ot, og, om = O.candidates(hg, part, tq)
        org = O.afterburner(hg, part, ot, og, om)
        for graph in (1, 0):
            ctx.set_option(J().JET_OPT_GRAPH_KERNELS, graph)
            rg = ctx.afterburner(dev(part), dev(ot), dev(og), dev(om, torch.uint8))
            assert np.array_equal(rg.cpu().numpy(), org), (name, tau, graph)


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("graph", [1, 0], ids=["graph-kernels", "general"])
def test_graph_refine_matches_oracle(name, graph):
    hg, part = GRAPHS[name]()
    say(f"graph refine {name} graph_kernels={graph}")
    ctx = J().JetContext(hg)
    ctx.set_option(J().JET_OPT_GRAPH_KERNELS, graph)
    kw = dict(tau=(0.75, 0.375, 0.0), limit=8)
    p = dev(part)
    rc, st, tr = ctx.refine(p, trace_cap=4096, **kw)
    out, orc, ost, otr = O.refine(hg, part, **kw)
    assert rc == orc
    assert sha(p.cpu().numpy()) == sha(out)
    for key in ("km1_in", "km1_out", "iterations", "rebalance_rounds", "moves_executed", "max_block_weight"):
        assert st[key] == ost[key], key
    assert tr == otr


def test_mesh_full_size_steps():
    """The 4M-vertex triangulated mesh (k = 64) of the graph benchmark: all candidate records, all
    recomputed gains and two whole Jet iterations against the oracle."""
    say("mesh 4M: generate")
    hg, part = W.mesh_graph()
    ctx = J().JetContext(hg)
    tq = O.quantize_tau(0.75)
    say("mesh 4M: candidates")
    t, g, m = ctx.candidates(dev(part), tq)
    ot, og, om = O.candidates(hg, part, tq)
    assert np.array_equal(m.cpu().numpy(), om)
    sel = om.astype(bool)
    assert np.array_equal(t.cpu().numpy()[sel], ot[sel]) and np.array_equal(g.cpu().numpy()[sel], og[sel])
    say("mesh 4M: afterburner")
    rg = ctx.afterburner(dev(part), t, g, m)
    assert np.array_equal(rg.cpu().numpy(), O.afterburner(hg, part, ot, og, om))
    say("mesh 4M: two iterations")
    p = dev(part)
    rc, st, tr = ctx.refine(p, trace_cap=8, tau=(0.75,), limit=8, max_iters=2)
    out, orc, ost, otr = O.refine(hg, part, tau=(0.75,), limit=8, max_iters=2)
    assert rc == orc and tr == otr and sha(p.cpu().numpy()) == sha(out)
