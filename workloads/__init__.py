"""Seeded synthetic hypergraph workloads shared by the CPU oracle, the GPU library, tests and bench.

Only input construction lives here (structure, weights, starting partitions, the coarsening
hierarchy used to reach a multilevel starting point).  None of the refinement arithmetic does, so
the oracle and the HIP path stay independent of each other and of this module.

Every generator is deterministic in its seed (SplitMix64 streams, see ``wlgen.c``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = ["wlgen.c", "wlhier.c"]
_LIB_PATH = os.path.join(_HERE, "libwlgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the generator library with gcc (host code only)."""
    srcs = [os.path.join(_HERE, s) for s in _SRCS if os.path.exists(os.path.join(_HERE, s))]
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-o", tmp] + srcs + ["-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Spec(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("m", ctypes.c_int32), ("p_target", ctypes.c_int64),
        ("size_kind", ctypes.c_int32), ("size_a", ctypes.c_int32), ("size_b", ctypes.c_int32),
        ("size_q", ctypes.c_double), ("place_kind", ctypes.c_int32), ("win_fixed", ctypes.c_int32),
        ("win_mult", ctypes.c_int32), ("sort_by_anchor", ctypes.c_int32), ("pad_", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER
        L.wl_sizes.argtypes = [P(_Spec), P(ctypes.c_int32), P(ctypes.c_int64)]
        L.wl_fill.argtypes = [P(_Spec), ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
        L.wl_weights.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_void_p]
        L.wl_weights.restype = None
        L.wl_part_roundrobin.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_void_p]
        L.wl_part_roundrobin.restype = None
        L.wl_part_ranges_noise.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                           ctypes.c_void_p]
        L.wl_part_uniform.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_void_p]
        L.wl_part_uniform.restype = None
        L.wl_randint.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p]
        L.wl_randint.restype = None
        if hasattr(L, "wl_coarsen"):
            L.wl_coarsen.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                     P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_int64)]
            L.wl_coarsen.restype = ctypes.c_void_p
            L.wl_coarse_fill.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p]
            L.wl_coarse_fill.restype = None
            L.wl_coarse_free.argtypes = [ctypes.c_void_p]
            L.wl_coarse_free.restype = None
            L.wl_contract.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                      P(ctypes.c_int32), P(ctypes.c_int64)]
            L.wl_contract.restype = ctypes.c_void_p
            L.wl_greedy_initial.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_uint64,
                                            ctypes.c_void_p]
            L.wl_greedy_initial.restype = None
        _lib = L
    return _lib


@dataclass
class Hypergraph:
    """CSR hypergraph: pins of net e are pins[off[e]:off[e+1]]."""
    n: int
    m: int
    off: np.ndarray            # int64[m+1]
    pins: np.ndarray           # int32[p]
    k: int
    eps: float
    net_w: Optional[np.ndarray] = None   # int32[m] or None (unit)
    vtx_w: Optional[np.ndarray] = None   # int32[n] or None (unit)

    @property
    def p(self) -> int:
        return int(self.off[-1])

    def total_weight(self) -> int:
        return int(self.n if self.vtx_w is None else int(self.vtx_w.astype(np.int64).sum()))


SIZE_UNIFORM, SIZE_GEOMETRIC, SIZE_ZIPF = 0, 1, 2
PLACE_UNIFORM, PLACE_RANDOM_ANCHOR, PLACE_ROW_ANCHOR = 0, 1, 2


def generate(n, m=0, *, seed, size_kind=SIZE_UNIFORM, size_a=2, size_b=8, size_q=0.0,
             place_kind=PLACE_UNIFORM, win_fixed=0, win_mult=0, sort_by_anchor=False, p_target=0):
    """Structure only: returns (off int64[m+1], pins int32[p])."""
    sp = _Spec(n=n, m=m, p_target=p_target, size_kind=size_kind, size_a=size_a, size_b=size_b, size_q=size_q,
               place_kind=place_kind, win_fixed=win_fixed, win_mult=win_mult,
               sort_by_anchor=1 if sort_by_anchor else 0, pad_=0, seed=seed & (2**64 - 1))
    mm = ctypes.c_int32()
    pp = ctypes.c_int64()
    if lib().wl_sizes(ctypes.byref(sp), ctypes.byref(mm), ctypes.byref(pp)) != 0:
        raise RuntimeError("wl_sizes failed")
    off = np.empty(mm.value + 1, dtype=np.int64)
    pins = np.empty(pp.value, dtype=np.int32)
    rc = lib().wl_fill(ctypes.byref(sp), mm.value, pp.value, off.ctypes.data, pins.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"wl_fill failed ({rc})")
    return off, pins


def weights(count, wmax, seed, stream):
    w = np.empty(count, dtype=np.int32)
    lib().wl_weights(count, wmax, seed & (2**64 - 1), stream, w.ctypes.data)
    return w


def part_roundrobin(n, k, seed):
    part = np.empty(n, dtype=np.int32)
    lib().wl_part_roundrobin(n, k, seed & (2**64 - 1), part.ctypes.data)
    return part


def part_ranges_noise(n, k, n_noise, seed):
    part = np.empty(n, dtype=np.int32)
    if lib().wl_part_ranges_noise(n, k, n_noise, seed & (2**64 - 1), part.ctypes.data) != 0:
        raise RuntimeError("wl_part_ranges_noise failed")
    return part


def part_uniform(n, k, seed):
    part = np.empty(n, dtype=np.int32)
    lib().wl_part_uniform(n, k, seed & (2**64 - 1), part.ctypes.data)
    return part


def randint(seed, stream, count, rng):
    out = np.empty(count, dtype=np.int64)
    lib().wl_randint(seed & (2**64 - 1), stream, count, rng, out.ctypes.data)
    return out


# ---------------------------------------------------------------- named workloads

def random_hypergraph(n, m, k, seed, *, smin=2, smax=8, vw_max=1, nw_max=1, eps=0.03):
    """Uniform net sizes in [smin, smax], pins uniform without replacement over all vertices."""
    off, pins = generate(n, m, seed=seed, size_kind=SIZE_UNIFORM, size_a=smin, size_b=min(smax, n))
    vw = weights(n, vw_max, seed, 0) if vw_max > 1 else None
    nw = weights(m, nw_max, seed, 1) if nw_max > 1 else None
    return Hypergraph(n=n, m=m, off=off, pins=pins, k=k, eps=eps, net_w=nw, vtx_w=vw)


def banded_hypergraph(n, k, seed, *, window=6, nets_per_vertex=2, vw_max=1, eps=0.03):
    """A locally connected hypergraph and a partition of contiguous blocks: for each vertex i < n-1,
    `nets_per_vertex` nets of 2..4 pins, i and pins drawn from i+1 .. i+window-1 (clipped at n-1);
    blocks are ranges of n/k consecutive IDs.  Two blocks meet in a few vertices only, so searches
    from their boundary run over many levels.  Returns (hypergraph, partition)."""
    rng = np.random.default_rng(seed)
    nets = []
    for i in range(n - 1):
        for _ in range(nets_per_vertex):
            size = int(rng.integers(2, 5))
            nets.append(sorted({i} | {int(min(n - 1, i + rng.integers(1, window))) for _ in range(size - 1)}))
    off = np.zeros(len(nets) + 1, np.int64)
    off[1:] = np.cumsum([len(e) for e in nets])
    vw = rng.integers(1, vw_max + 1, n).astype(np.int32) if vw_max > 1 else None
    hg = Hypergraph(n=n, m=len(nets), off=off, pins=np.concatenate(nets).astype(np.int32), k=k, eps=eps,
                    net_w=None, vtx_w=vw)
    return hg, (np.arange(n) * k // n).astype(np.int32)


def overloaded_with_heavy_vertex(seed):
    """A 60-vertex random hypergraph with k = 3..5 and vertex weights 1..2, where vertex `heavy`
    (one of the first ten) weighs 6..15; vertices 0..11 and `heavy` start in block 0, the others
    in random other blocks.  Returns (hypergraph, partition, heavy)."""
    rng = np.random.default_rng(seed)
    k = 3 + seed % 3
    hg = random_hypergraph(60, 90, k, 5000 + seed, smin=2, smax=5, vw_max=2, nw_max=3)
    vw = hg.vtx_w.astype(np.int64).copy()
    heavy = int(rng.integers(0, 10))
    vw[heavy] = int(rng.integers(6, 16))
    hg.vtx_w = vw.astype(np.int32)
    part = rng.integers(1, k, hg.n).astype(np.int32)
    part[:12] = 0
    part[heavy] = 0
    return hg, part, heavy


def small_uniform(seed=1):
    """2,000 unit-weight vertices, 4,000 unit-weight nets of size U[2,8], k=4, eps=0.03,
    balanced seeded starting partition (a permutation dealt round robin into the 4 blocks)."""
    hg = random_hypergraph(2000, 4000, 4, seed, smin=2, smax=8)
    return hg, part_roundrobin(hg.n, hg.k, seed)


def vlsi_like(seed=2, n=1_000_000, m=1_100_000, k=8, noise_frac=0.1):
    """Netlist-like: weights U{1..4}; sizes 2+Geom(0.4) capped at 64 (mean 3.5); pins within
    +-2000 IDs of a random anchor; nets numbered in anchor order; start = contiguous ID ranges
    with 10% of the vertices reassigned uniformly at random."""
    off, pins = generate(n, m, seed=seed, size_kind=SIZE_GEOMETRIC, size_a=2, size_b=64, size_q=0.4,
                         place_kind=PLACE_RANDOM_ANCHOR, win_fixed=2000, sort_by_anchor=True)
    vw = weights(n, 4, seed, 0)
    hg = Hypergraph(n=n, m=m, off=off, pins=pins, k=k, eps=0.03, net_w=None, vtx_w=vw)
    return hg, part_ranges_noise(n, k, int(round(noise_frac * n)), seed)


def rownet_matrix(seed=4, n=4_000_000, k=64, cap=10_000):
    """Row-net hypergraph of a banded sparse matrix: n rows = n nets = n vertices, sizes Zipf(2.1)
    on [2, cap], pins within +-max(4|e|, 2048) of the row index, unit weights."""
    off, pins = generate(n, n, seed=seed, size_kind=SIZE_ZIPF, size_a=2, size_b=cap, size_q=2.1,
                         place_kind=PLACE_ROW_ANCHOR, win_fixed=2048, win_mult=4)
    return Hypergraph(n=n, m=n, off=off, pins=pins, k=k, eps=0.03)


def sat_like(seed=5, n=20_000_000, p_total=200_000_000, k=128, cap=1_000_000):
    """SAT-like heavy tail: sizes Zipf(1.8) on [2, cap] drawn until the pin total is reached (last
    net truncated), pins uniform without replacement over all vertices, vertex weights U{1..8}."""
    off, pins = generate(n, 0, seed=seed, size_kind=SIZE_ZIPF, size_a=2, size_b=min(cap, n), size_q=1.8,
                         place_kind=PLACE_UNIFORM, p_target=p_total)
    vw = weights(n, 8, seed, 0)
    return Hypergraph(n=n, m=len(off) - 1, off=off, pins=pins, k=k, eps=0.03, vtx_w=vw)


def mesh_graph(side=2048, k=64, seed=6, noise_frac=0.05, diag=True):
    """Regular graph: the side x side grid with edges to the right, lower and (diag) lower-right
    neighbour (a triangulated mesh, average degree 6), vertices row-major, unit weights, every net
    of two pins in row-major order of its lower endpoint.  Start: contiguous ID ranges with
    noise_frac of the vertices reassigned at random."""
    idx = np.arange(side * side, dtype=np.int64).reshape(side, side)
    parts = [np.stack([idx[:, :-1].ravel(), idx[:, 1:].ravel()], axis=1),
             np.stack([idx[:-1, :].ravel(), idx[1:, :].ravel()], axis=1)]
    if diag:
        parts.append(np.stack([idx[:-1, :-1].ravel(), idx[1:, 1:].ravel()], axis=1))
    e = np.concatenate(parts)
    e = e[np.lexsort((e[:, 1], e[:, 0]))]
    n, m = side * side, len(e)
    off = np.arange(0, 2 * m + 1, 2, dtype=np.int64)
    hg = Hypergraph(n=n, m=m, off=off, pins=e.astype(np.int32).ravel(), k=k, eps=0.03)
    return hg, part_ranges_noise(n, k, int(n * noise_frac), seed)


def powerlaw_graph(n=1_000_000, avg_deg=10, k=64, seed=7, noise_frac=0.05):
    """Irregular graph: Chung-Lu edges with expected degrees proportional to (i + 10)^(-1/1.2)
    (a power law with a few hubs), duplicate edges and self loops dropped, unit weights, nets in
    order of their lower endpoint; vertices numbered in decreasing expected degree.  Start:
    contiguous ID ranges with noise_frac of the vertices reassigned at random."""
    w = (np.arange(n, dtype=np.float64) + 10.0) ** (-1.0 / 1.2)
    cdf = np.cumsum(w / w.sum())
    m0 = n * avg_deg // 2
    u = randint(seed, 1, 2 * m0, 1 << 53).astype(np.float64) / float(1 << 53)
    ends = np.minimum(np.searchsorted(cdf, u, side="right"), n - 1).reshape(m0, 2)
    a, b = np.minimum(ends[:, 0], ends[:, 1]), np.maximum(ends[:, 0], ends[:, 1])
    keep = a != b
    e = np.unique(np.stack([a[keep], b[keep]], axis=1), axis=0)
    m = len(e)
    off = np.arange(0, 2 * m + 1, 2, dtype=np.int64)
    hg = Hypergraph(n=n, m=m, off=off, pins=e.astype(np.int32).ravel(), k=k, eps=0.03)
    return hg, part_ranges_noise(n, k, int(n * noise_frac), seed)


def batch_set(seed=3, count=512, nmin=1_000, nmax=100_000):
    """count independent hypergraphs of uneven size: n log-uniform in [nmin, nmax], m = round(1.2 n),
    sizes Zipf(2.1) on [2, min(1000, n)], pins uniform without replacement, unit weights, k uniform
    in {2, 8, 32}, eps = 0.03; each starts from a seeded balanced partition (a permutation dealt
    round robin).  Returns a list of (Hypergraph, part)."""
    u = randint(seed, 0, count, 1 << 53).astype(np.float64) / float(1 << 53)
    ns = np.rint(np.exp(np.log(nmin) + u * (np.log(nmax) - np.log(nmin)))).astype(np.int64)
    ks = np.array([2, 8, 32])[randint(seed, 1, count, 3)]
    out = []
    for i in range(count):
        n, k, sd = int(ns[i]), int(ks[i]), seed * 1_000_003 + i
        m = int(round(1.2 * n))
        off, pins = generate(n, m, seed=sd, size_kind=SIZE_ZIPF, size_a=2, size_b=min(1000, n), size_q=2.1,
                             place_kind=PLACE_UNIFORM)
        out.append((Hypergraph(n=n, m=m, off=off, pins=pins, k=k, eps=0.03), part_roundrobin(n, k, sd)))
    return out


# ---------------------------------------------------------------- multilevel starting points

def _ptr(a):
    return None if a is None else a.ctypes.data


def coarsen(hg: Hypergraph, seed: int):
    """One random-matching contraction: returns (coarse Hypergraph, parent int32[n])."""
    parent = np.empty(hg.n, dtype=np.int32)
    nc, mc, pc = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
    off = np.ascontiguousarray(hg.off, np.int64)
    pins = np.ascontiguousarray(hg.pins, np.int32)
    nw = None if hg.net_w is None else np.ascontiguousarray(hg.net_w, np.int32)
    vw = None if hg.vtx_w is None else np.ascontiguousarray(hg.vtx_w, np.int32)
    h = lib().wl_coarsen(hg.n, hg.m, hg.p, off.ctypes.data, pins.ctypes.data, _ptr(nw), _ptr(vw),
                         seed & (2**64 - 1), parent.ctypes.data, ctypes.byref(nc), ctypes.byref(mc), ctypes.byref(pc))
    try:
        coff = np.empty(mc.value + 1, np.int64)
        cpins = np.empty(pc.value, np.int32)
        cnw = None if nw is None else np.empty(mc.value, np.int32)
        cvw = np.empty(nc.value, np.int32)
        lib().wl_coarse_fill(h, coff.ctypes.data, cpins.ctypes.data, _ptr(cnw), cvw.ctypes.data)
    finally:
        lib().wl_coarse_free(h)
    return Hypergraph(n=nc.value, m=mc.value, off=coff, pins=cpins, k=hg.k, eps=hg.eps, net_w=cnw, vtx_w=cvw), parent


def _fill_coarse(h, nc, mc, pc, weighted_nets, hg):
    try:
        coff = np.empty(mc + 1, np.int64)
        cpins = np.empty(pc, np.int32)
        cnw = np.empty(mc, np.int32) if weighted_nets else None
        cvw = np.empty(nc, np.int32)
        lib().wl_coarse_fill(h, coff.ctypes.data, cpins.ctypes.data, _ptr(cnw), cvw.ctypes.data)
    finally:
        lib().wl_coarse_free(h)
    return Hypergraph(n=nc, m=mc, off=coff, pins=cpins, k=hg.k, eps=hg.eps, net_w=cnw, vtx_w=cvw)


def contract(hg: Hypergraph, parent: np.ndarray, nc: int) -> Hypergraph:
    """Contraction of a given clustering (parent[v] in [0, nc)): summed vertex weights, nets mapped
    and deduplicated, single-pin nets dropped, parallel nets kept (the same contraction as
    coarsen())."""
    parent = np.ascontiguousarray(parent, np.int32)
    assert parent.shape == (hg.n,)
    mc, pc = ctypes.c_int32(), ctypes.c_int64()
    off = np.ascontiguousarray(hg.off, np.int64)
    pins = np.ascontiguousarray(hg.pins, np.int32)
    nw = None if hg.net_w is None else np.ascontiguousarray(hg.net_w, np.int32)
    vw = None if hg.vtx_w is None else np.ascontiguousarray(hg.vtx_w, np.int32)
    h = lib().wl_contract(hg.n, hg.m, hg.p, off.ctypes.data, pins.ctypes.data, _ptr(nw), _ptr(vw),
                          parent.ctypes.data, int(nc), ctypes.byref(mc), ctypes.byref(pc))
    if not h:
        raise ValueError("parent out of range")
    return _fill_coarse(h, int(nc), mc.value, pc.value, nw is not None, hg)


def hierarchy(hg: Hypergraph, levels: int, seed: int):
    """levels hypergraphs, finest first; parents[l] maps level l to level l+1."""
    hgs, parents = [hg], []
    for lvl in range(levels - 1):
        c, par = coarsen(hgs[-1], seed * 1000 + lvl)
        hgs.append(c)
        parents.append(par)
    return hgs, parents


def greedy_initial(hg: Hypergraph, seed: int) -> np.ndarray:
    part = np.empty(hg.n, dtype=np.int32)
    vw = None if hg.vtx_w is None else np.ascontiguousarray(hg.vtx_w, np.int32)
    lib().wl_greedy_initial(hg.n, hg.k, _ptr(vw), seed & (2**64 - 1), part.ctypes.data)
    return part
