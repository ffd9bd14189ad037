"""ctypes binding of the CPU oracle (``jet_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The oracle is the plain single-threaded reference that the GPU library
is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package; the GPU library never does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# JET_ORACLE_LIB selects another build of the same source (the sanitizer build in the tests)
_LIB_PATH = os.environ.get("JET_ORACLE_LIB") or os.path.join(_HERE, "libjet_oracle.so")
_lib = None

DEFAULT_DEADZONE_PPM = 100_000


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile the oracle with gcc.  ``sanitize`` builds an ASan/UBSan variant next to it."""
    srcs = [os.path.join(_HERE, f) for f in ("jet_oracle.c", "coarsen_oracle.c", "flow_oracle.c")]
    out = os.path.join(_HERE, "libjet_oracle.so" if not sanitize else "libjet_oracle_san.so")
    if force or not os.path.exists(out):
        flags = ["-O2", "-g"] if not sanitize else ["-O1", "-g", "-fsanitize=address,undefined",
                                                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", *flags, "-o", tmp, *srcs,
                               "-lm"])
        os.replace(tmp, out)
    return out


class HG(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("p", ctypes.c_int64),
                ("off", ctypes.c_void_p), ("pins", ctypes.c_void_p), ("nw", ctypes.c_void_p),
                ("vw", ctypes.c_void_p), ("k", ctypes.c_int32), ("eps", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [("limit", ctypes.c_int32), ("max_iters", ctypes.c_int32), ("num_tau", ctypes.c_int32),
                ("tau", ctypes.c_float * 8), ("deadzone_ppm", ctypes.c_int32),
                ("max_rebalance_rounds", ctypes.c_int32), ("rb_unweighted", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("km1_in", ctypes.c_int64), ("km1_out", ctypes.c_int64), ("lmax", ctypes.c_int64),
                ("max_block_weight", ctypes.c_int64), ("iterations", ctypes.c_int32),
                ("rebalance_rounds", ctypes.c_int32), ("balanced", ctypes.c_int32),
                ("moves_executed", ctypes.c_int32), ("tau_q_used", ctypes.c_int32 * 8)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "tau_q_used"}
        d["tau_q_used"] = list(self.tau_q_used)
        return d


class Trace(ctypes.Structure):
    _fields_ = [("km1", ctypes.c_int64), ("overload", ctypes.c_int64), ("n_cand", ctypes.c_int32),
                ("n_moved", ctypes.c_int32), ("rb_rounds", ctypes.c_int32), ("rb_moved", ctypes.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER
        vp = ctypes.c_void_p
        L.jo_km1.argtypes = [P(HG), vp]
        L.jo_km1.restype = ctypes.c_int64
        L.jo_phi.argtypes = [P(HG), vp, vp]
        L.jo_phi.restype = None
        L.jo_block_weights.argtypes = [P(HG), vp, vp]
        L.jo_block_weights.restype = None
        L.jo_limits.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                P(ctypes.c_int64), P(ctypes.c_int64), P(ctypes.c_int64)]
        L.jo_limits.restype = None
        L.jo_quantize_tau.argtypes = [ctypes.c_float]
        L.jo_quantize_tau.restype = ctypes.c_int32
        L.jo_gain_bruteforce.argtypes = [P(HG), vp, ctypes.c_int32, ctypes.c_int32]
        L.jo_gain_bruteforce.restype = ctypes.c_int64
        L.jo_candidates.argtypes = [P(HG), vp, vp, ctypes.c_int32, vp, vp, vp]
        L.jo_candidates.restype = None
        L.jo_candidates_sample.argtypes = [P(HG), vp, vp, ctypes.c_int32, vp, ctypes.c_int64, vp, vp, vp]
        L.jo_candidates_sample.restype = None
        L.jo_afterburner.argtypes = [P(HG), vp, vp, vp, vp, vp]
        L.jo_afterburner.restype = None
        L.jo_afterburner_replay.argtypes = [P(HG), vp, vp, vp, vp, vp]
        L.jo_afterburner_replay.restype = None
        L.jo_rebalance_round.argtypes = [P(HG), vp, ctypes.c_int32, vp]
        L.jo_rebalance_round.restype = ctypes.c_int32
        L.jo_rebalance_round_w.argtypes = [P(HG), vp, ctypes.c_int32, ctypes.c_int32, vp]
        L.jo_rebalance_round_w.restype = ctypes.c_int32
        L.jo_rebalance.argtypes = [P(HG), vp, P(Params), P(Stats)]
        L.jo_rebalance.restype = ctypes.c_int
        L.jo_refine.argtypes = [P(HG), vp, P(Params), P(Stats), vp, ctypes.c_int32, P(ctypes.c_int32)]
        L.jo_refine.restype = ctypes.c_int
        L.jo_bruteforce_2way.argtypes = [P(HG)]
        L.jo_bruteforce_2way.restype = ctypes.c_int64
        L.jo_coarsen_schedule.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, ctypes.c_int64]
        L.jo_coarsen_schedule.restype = ctypes.c_int64
        L.jo_coarsen_subround.argtypes = [P(HG), vp, vp, vp, ctypes.c_int32, ctypes.c_int64, vp]
        L.jo_coarsen_subround.restype = ctypes.c_int32
        L.jo_coarsen.argtypes = [P(HG), vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, vp]
        L.jo_coarsen.restype = ctypes.c_int32
        L.jo_flow_region.argtypes = [P(HG), vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp]
        L.jo_flow_region.restype = ctypes.c_int32
        L.jo_flow_mincut.argtypes = [P(HG), vp, ctypes.c_int32, ctypes.c_int32, vp, vp, vp]
        L.jo_flow_mincut.restype = ctypes.c_int64
        L.jo_flow_pair.argtypes = [P(HG), vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P(FlowPairStats)]
        L.jo_flow_pair.restype = ctypes.c_int32
        L.jo_flow_refine.argtypes = [P(HG), vp, ctypes.c_int32, ctypes.c_int32, P(FlowStats)]
        L.jo_flow_refine.restype = ctypes.c_int32
        _lib = L
    return _lib


class FlowPairStats(ctypes.Structure):
    _fields_ = [("old_cut", ctypes.c_int64), ("new_cut", ctypes.c_int64), ("iterations", ctypes.c_int32),
                ("region_a", ctypes.c_int32), ("region_b", ctypes.c_int32), ("moved", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class FlowStats(ctypes.Structure):
    _fields_ = [("km1_in", ctypes.c_int64), ("km1_out", ctypes.c_int64), ("rounds", ctypes.c_int32),
                ("matchings", ctypes.c_int32), ("pairs", ctypes.c_int32), ("accepted", ctypes.c_int32),
                ("flow_calls", ctypes.c_int32), ("moved", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


FLOW_ALPHA = 16       # region scale alpha (reading F1)
FLOW_MAX_ROUNDS = 8   # rounds of the k-way schedule (reading F4)


class OracleHG:
    """Keeps the numpy arrays alive while the C struct points into them."""

    def __init__(self, hg):
        self.off = np.ascontiguousarray(hg.off, dtype=np.int64)
        self.pins = np.ascontiguousarray(hg.pins, dtype=np.int32)
        self.nw = None if hg.net_w is None else np.ascontiguousarray(hg.net_w, dtype=np.int32)
        self.vw = None if hg.vtx_w is None else np.ascontiguousarray(hg.vtx_w, dtype=np.int32)
        self.n, self.m, self.k = int(hg.n), int(hg.m), int(hg.k)
        self.c = HG(n=self.n, m=self.m, p=int(self.off[-1]), off=self.off.ctypes.data, pins=self.pins.ctypes.data,
                    nw=None if self.nw is None else self.nw.ctypes.data,
                    vw=None if self.vw is None else self.vw.ctypes.data, k=self.k, eps=float(hg.eps))

    @property
    def ref(self):
        return ctypes.byref(self.c)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def make_params(tau=(0.75,), limit=12, max_iters=1000, deadzone_ppm=DEFAULT_DEADZONE_PPM, max_rebalance_rounds=64,
                rb_unweighted=0):
    tau = list(tau)
    if not 1 <= len(tau) <= 8:
        raise ValueError("1..8 temperatures")
    arr = (ctypes.c_float * 8)(*(tau + [0.0] * (8 - len(tau))))
    return Params(limit=limit, max_iters=max_iters, num_tau=len(tau), tau=arr, deadzone_ppm=deadzone_ppm,
                  max_rebalance_rounds=max_rebalance_rounds, rb_unweighted=int(rb_unweighted))


def km1(hg, part) -> int:
    o = OracleHG(hg)
    part = _i32(part)
    return int(lib().jo_km1(o.ref, part.ctypes.data))


def phi(hg, part) -> np.ndarray:
    o = OracleHG(hg)
    part = _i32(part)
    out = np.empty(hg.m * hg.k, dtype=np.int32)
    lib().jo_phi(o.ref, part.ctypes.data, out.ctypes.data)
    return out.reshape(hg.m, hg.k)


def block_weights(hg, part) -> np.ndarray:
    o = OracleHG(hg)
    part = _i32(part)
    out = np.empty(hg.k, dtype=np.int64)
    lib().jo_block_weights(o.ref, part.ctypes.data, out.ctypes.data)
    return out


def limits(W, k, eps, deadzone_ppm=DEFAULT_DEADZONE_PPM):
    A, lm, dz = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    lib().jo_limits(W, k, eps, deadzone_ppm, ctypes.byref(A), ctypes.byref(lm), ctypes.byref(dz))
    return A.value, lm.value, dz.value


def quantize_tau(tau: float) -> int:
    return int(lib().jo_quantize_tau(tau))


def gain_bruteforce(hg, part, v, b) -> int:
    o = OracleHG(hg)
    part = _i32(part)
    return int(lib().jo_gain_bruteforce(o.ref, part.ctypes.data, v, b))


def candidates(hg, part, tau_q, lock: Optional[np.ndarray] = None):
    o = OracleHG(hg)
    part = _i32(part)
    t = np.empty(hg.n, dtype=np.int32)
    g = np.empty(hg.n, dtype=np.int32)
    inM = np.empty(hg.n, dtype=np.uint8)
    lk = None if lock is None else np.ascontiguousarray(lock, dtype=np.uint8)
    lib().jo_candidates(o.ref, part.ctypes.data, None if lk is None else lk.ctypes.data, tau_q, t.ctypes.data,
                        g.ctypes.data, inM.ctypes.data)
    return t, g, inM


def candidates_sample(hg, part, tau_q, verts, lock: Optional[np.ndarray] = None):
    """(t, g, in_m) of the listed vertices (arrays in the order of verts)."""
    o = OracleHG(hg)
    part = _i32(part)
    verts = _i32(verts)
    t = np.full(hg.n, -1, dtype=np.int32)
    g = np.zeros(hg.n, dtype=np.int32)
    inm = np.zeros(hg.n, dtype=np.uint8)
    lk = None if lock is None else np.ascontiguousarray(lock, dtype=np.uint8)
    lib().jo_candidates_sample(o.ref, part.ctypes.data, None if lk is None else lk.ctypes.data, tau_q,
                               verts.ctypes.data, len(verts), t.ctypes.data, g.ctypes.data, inm.ctypes.data)
    return t[verts], g[verts], inm[verts]


def afterburner(hg, part, t, g, inM):
    o = OracleHG(hg)
    part, t, g = _i32(part), _i32(t), _i32(g)
    inM = np.ascontiguousarray(inM, dtype=np.uint8)
    rg = np.empty(hg.n, dtype=np.int32)
    lib().jo_afterburner(o.ref, part.ctypes.data, t.ctypes.data, g.ctypes.data, inM.ctypes.data, rg.ctypes.data)
    return rg


def afterburner_replay(hg, part, t, g, inM):
    o = OracleHG(hg)
    part, t, g = _i32(part), _i32(t), _i32(g)
    inM = np.ascontiguousarray(inM, dtype=np.uint8)
    rg = np.empty(hg.n, dtype=np.int64)
    lib().jo_afterburner_replay(o.ref, part.ctypes.data, t.ctypes.data, g.ctypes.data, inM.ctypes.data,
                                rg.ctypes.data)
    return rg


def rebalance_round(hg, part, deadzone_ppm=DEFAULT_DEADZONE_PPM, unweighted=0):
    """Returns (new_part, sel_target, moved)."""
    o = OracleHG(hg)
    part = _i32(part).copy()
    sel = np.empty(hg.n, dtype=np.int32)
    moved = int(lib().jo_rebalance_round_w(o.ref, part.ctypes.data, deadzone_ppm, int(unweighted), sel.ctypes.data))
    return part, sel, moved


def rebalance(hg, part, **kw):
    o = OracleHG(hg)
    part = _i32(part).copy()
    prm = make_params(**kw)
    st = Stats()
    rc = int(lib().jo_rebalance(o.ref, part.ctypes.data, ctypes.byref(prm), ctypes.byref(st)))
    return part, rc, st.as_dict()


def refine(hg, part, trace_cap=4096, **kw):
    """Returns (new_part, rc, stats dict, trace list of dicts)."""
    o = OracleHG(hg)
    part = _i32(part).copy()
    prm = make_params(**kw)
    st = Stats()
    tr = (Trace * max(trace_cap, 1))()
    tlen = ctypes.c_int32()
    rc = int(lib().jo_refine(o.ref, part.ctypes.data, ctypes.byref(prm), ctypes.byref(st), tr, trace_cap,
                             ctypes.byref(tlen)))
    trace = [{f: getattr(tr[i], f) for f, _ in Trace._fields_} for i in range(min(tlen.value, trace_cap))]
    return part, rc, st.as_dict(), trace


def bruteforce_2way(hg) -> int:
    o = OracleHG(hg)
    return int(lib().jo_bruteforce_2way(o.ref))


def level_stats(hg, part) -> np.ndarray:
    """The 16 level statistics of the learned temperature, from their definitions (Section 2 terms):
    n, m, pins, largest net, k, W, Lmax, largest block weight, cut nets (lambda >= 2), metric, sum
    of net weights, boundary vertices (some incident net is cut), weight of cut nets, ceil(W/k)."""
    part = _i32(part)
    ph = phi(hg, part)
    lam = (ph > 0).sum(axis=1)
    cut = lam >= 2
    nw = np.ones(hg.m, dtype=np.int64) if hg.net_w is None else hg.net_w.astype(np.int64)
    sizes = np.diff(hg.off)
    boundary = np.zeros(hg.n, dtype=bool)
    for e in np.nonzero(cut)[0]:
        boundary[hg.pins[hg.off[e]:hg.off[e + 1]]] = True
    W = hg.total_weight()
    A, lmax, _ = limits(W, hg.k, hg.eps)
    bw = block_weights(hg, part)
    return np.array([hg.n, hg.m, hg.p, sizes.max(), hg.k, W, lmax, bw.max(), cut.sum(), km1(hg, part), nw.sum(),
                     boundary.sum(), nw[cut].sum(), A, 0, 0], dtype=np.int64)


# ---- synchronous clustering of the coarsening phase (Section 6, Algorithm 4) ----

INITIAL_SINGLE, CAP_DIV = 100, 100   # Section 6: 100 one-vertex sub-rounds, sizes doubling up to 1% of n


def coarsen_schedule(n, initial_single=INITIAL_SINGLE, cap_div=CAP_DIV) -> list:
    cnt = int(lib().jo_coarsen_schedule(n, initial_single, cap_div, None, 0))
    if cnt < 0:
        raise ValueError("bad schedule arguments")
    out = np.empty(max(cnt, 1), dtype=np.int32)
    lib().jo_coarsen_schedule(n, initial_single, cap_div, out.ctypes.data, cnt)
    return out[:cnt].tolist()


def coarsen_subround(hg, label, cw, B, wmax):
    """One sub-round on copies of (label, cw): returns (label, cw, T, moved)."""
    o = OracleHG(hg)
    label = _i32(label).copy()
    cw = np.ascontiguousarray(cw, dtype=np.int64).copy()
    B = _i32(B)
    T = np.empty(hg.n, dtype=np.int32)
    moved = int(lib().jo_coarsen_subround(o.ref, label.ctypes.data, cw.ctypes.data, B.ctypes.data, len(B), wmax,
                                          T.ctypes.data))
    return label, cw, T, moved


def coarsen(hg, order, wmax, initial_single=INITIAL_SINGLE, cap_div=CAP_DIV):
    """The clustering pass: returns (label[n], number of clusters)."""
    o = OracleHG(hg)
    order = _i32(order)
    label = np.empty(hg.n, dtype=np.int32)
    cnt = int(lib().jo_coarsen(o.ref, order.ctypes.data, wmax, initial_single, cap_div, label.ctypes.data))
    if cnt < 0:
        raise ValueError("order is not a permutation of the vertices, or bad schedule arguments")
    return label, cnt


# ---- flow-based refinement (Section 5) ----

def flow_region(hg, part, a, b, alpha=FLOW_ALPHA) -> np.ndarray:
    """Region of the pair (a, b): int8[n], 1 on block a's side, 2 on b's, 0 outside."""
    o = OracleHG(hg)
    region = np.zeros(hg.n, dtype=np.int8)
    if lib().jo_flow_region(o.ref, _i32(part).ctypes.data, a, b, alpha, region.ctypes.data) < 0:
        raise ValueError("bad pair or alpha")
    return region


def flow_mincut(hg, part, a, b, term):
    """Maximum flow for terminals term (int8[n]: 0 free, 1 source, 2 sink, for the vertices of a
    and b) and the residual reachable sets: (F, in_sr bool[n], in_tr bool[n])."""
    o = OracleHG(hg)
    term = np.ascontiguousarray(term, dtype=np.int8)
    sr = np.zeros(hg.n, dtype=np.uint8)
    tr = np.zeros(hg.n, dtype=np.uint8)
    F = int(lib().jo_flow_mincut(o.ref, _i32(part).ctypes.data, a, b, term.ctypes.data, sr.ctypes.data,
                                 tr.ctypes.data))
    return F, sr.astype(bool), tr.astype(bool)


def flow_pair(hg, part, a, b, alpha=FLOW_ALPHA):
    """Two-way refinement of (a, b) on a copy: (new part, replaced, stats dict)."""
    o = OracleHG(hg)
    part = _i32(part).copy()
    st = FlowPairStats()
    r = int(lib().jo_flow_pair(o.ref, part.ctypes.data, a, b, alpha, ctypes.byref(st)))
    if r < 0:
        raise ValueError("bad pair or alpha")
    return part, bool(r), st.as_dict()


def flow_refine(hg, part, alpha=FLOW_ALPHA, max_rounds=FLOW_MAX_ROUNDS):
    """k-way flow refinement on a copy: (new part, stats dict)."""
    o = OracleHG(hg)
    part = _i32(part).copy()
    st = FlowStats()
    if lib().jo_flow_refine(o.ref, part.ctypes.data, alpha, max_rounds, ctypes.byref(st)) < 0:
        raise ValueError("bad alpha or max_rounds")
    return part, st.as_dict()
