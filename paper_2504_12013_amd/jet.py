"""Thin ctypes binding of libjet.so (the C ABI in include/jet.h).

Argument marshalling only: every step of the method runs in the library's HIP kernels.  PyTorch
supplies device memory (tensors on ``cuda``) and the HIP stream (``torch.cuda.current_stream()``).
The functions keep the C names; ``JetContext`` is a small convenience wrapper around them.
If the library has not been built, importing works but every call raises ``JetError``.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libjet.so")

JET_OK, JET_IMBALANCED = 0, 1
JET_EINVAL, JET_ENOMEM, JET_EHIP, JET_EOVERFLOW, JET_EUNSUPPORTED = -1, -2, -3, -4, -5


class JetError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"jet error {code}: {msg}")
        self.code = code


class jet_params(ctypes.Structure):
    _fields_ = [("limit", ctypes.c_int32), ("max_iters", ctypes.c_int32), ("num_tau", ctypes.c_int32),
                ("tau", ctypes.c_float * 8), ("deadzone_ppm", ctypes.c_int32),
                ("max_rebalance_rounds", ctypes.c_int32), ("rb_unweighted", ctypes.c_int32)]


class jet_flow_pair_stats(ctypes.Structure):
    _fields_ = [("old_cut", ctypes.c_int64), ("new_cut", ctypes.c_int64), ("iterations", ctypes.c_int32),
                ("region_a", ctypes.c_int32), ("region_b", ctypes.c_int32), ("moved", ctypes.c_int32),
                ("replaced", ctypes.c_int32), ("arcs", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class jet_flow_stats(ctypes.Structure):
    _fields_ = [("km1_in", ctypes.c_int64), ("km1_out", ctypes.c_int64), ("rounds", ctypes.c_int32),
                ("matchings", ctypes.c_int32), ("pairs", ctypes.c_int32), ("accepted", ctypes.c_int32),
                ("flow_calls", ctypes.c_int32), ("moved", ctypes.c_int32), ("arcs", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


FLOW_ALPHA = 16       # default region scale of the flow refinement
FLOW_MAX_ROUNDS = 8   # default rounds of the k-way flow schedule


class jet_stats(ctypes.Structure):
    _fields_ = [("km1_in", ctypes.c_int64), ("km1_out", ctypes.c_int64), ("lmax", ctypes.c_int64),
                ("max_block_weight", ctypes.c_int64), ("iterations", ctypes.c_int32),
                ("rebalance_rounds", ctypes.c_int32), ("balanced", ctypes.c_int32),
                ("moves_executed", ctypes.c_int32), ("tau_q_used", ctypes.c_int32 * 8)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "tau_q_used"}
        d["tau_q_used"] = list(self.tau_q_used)
        return d


class jet_hg_desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("num_pins", ctypes.c_int64),
                ("net_offsets", ctypes.c_void_p), ("pins", ctypes.c_void_p), ("net_weights", ctypes.c_void_p),
                ("vertex_weights", ctypes.c_void_p), ("k", ctypes.c_int32), ("eps", ctypes.c_double)]


class jet_prof_entry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("alg_bytes", ctypes.c_double)]


class jet_trace(ctypes.Structure):
    _fields_ = [("km1", ctypes.c_int64), ("overload", ctypes.c_int64), ("n_cand", ctypes.c_int32),
                ("n_moved", ctypes.c_int32), ("rb_rounds", ctypes.c_int32), ("rb_moved", ctypes.c_int32)]


_lib = None


def lib():
    """The loaded library; raises JetError if it is not built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise JetError(JET_EUNSUPPORTED, f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, P = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER
        L.jet_params_default.argtypes = [P(jet_params)]
        L.jet_params_default.restype = None
        L.jet_init.argtypes = [P(vp), i32, i32, i64, vp, vp, vp, vp, i32, ctypes.c_double, vp]
        L.jet_refine.argtypes = [vp, vp, P(jet_params), P(jet_stats)]
        L.jet_refine_ex.argtypes = [vp, vp, P(jet_params), P(jet_stats), vp, i32, P(i32)]
        L.jet_rebalance.argtypes = [vp, vp, P(jet_params), P(jet_stats)]
        L.jet_km1.argtypes = [vp, vp, P(i64)]
        L.jet_phi.argtypes = [vp, vp, vp]
        L.jet_candidates.argtypes = [vp, vp, vp, i32, vp, vp, vp]
        L.jet_afterburner.argtypes = [vp, vp, vp, vp, vp, vp]
        L.jet_rebalance_round.argtypes = [vp, vp, i32, vp, P(i32)]
        L.jet_prof_enable.argtypes = [vp, i32]
        L.jet_prof_read.argtypes = [vp, P(jet_prof_entry), i32, P(i32)]
        L.jet_free.argtypes = [vp]
        L.jet_strerror.argtypes = [ctypes.c_int]
        L.jet_strerror.restype = ctypes.c_char_p
        L.jet_last_error.argtypes = [vp]
        L.jet_last_error.restype = ctypes.c_char_p
        f32p = P(ctypes.c_float)
        L.jet_level_stats.argtypes = [vp, vp, P(i64)]
        L.jet_tau_features.argtypes = [P(i64), ctypes.c_double, i32, i32, i64, i32, i32, ctypes.c_double, f32p]
        L.jet_mlp_create.argtypes = [P(vp), ctypes.c_uint64, vp]
        L.jet_mlp_set.argtypes = [vp, vp, vp, vp]
        L.jet_mlp_get.argtypes = [vp, vp, vp, vp]
        L.jet_mlp_forward.argtypes = [vp, vp, i32, vp]
        L.jet_mlp_grad.argtypes = [vp, vp, vp, i32, vp, f32p]
        L.jet_mlp_train_step.argtypes = [vp, vp, vp, i32, ctypes.c_float, f32p]
        L.jet_mlp_save.argtypes = [vp, ctypes.c_char_p]
        L.jet_mlp_load.argtypes = [vp, ctypes.c_char_p]
        L.jet_mlp_free.argtypes = [vp]
        L.jet_mlp_last_error.argtypes = [vp]
        L.jet_mlp_last_error.restype = ctypes.c_char_p
        L.jet_refine_learned.argtypes = [vp, vp, P(jet_params), vp, i32, i32, i64, P(jet_stats), f32p, P(i32)]
        L.jet_set_option.argtypes = [vp, i32, i64]
        L.jet_batch_init.argtypes = [P(vp), i32, P(jet_hg_desc), vp]
        L.jet_batch_set_option.argtypes = [vp, i32, i64]
        L.jet_batch_refine.argtypes = [vp, P(vp), P(jet_params), i32, P(jet_stats), P(i32)]
        L.jet_batch_free.argtypes = [vp]
        L.jet_batch_last_error.argtypes = [vp]
        L.jet_batch_last_error.restype = ctypes.c_char_p
        L.jet_batch_prof_enable.argtypes = [vp, i32]
        L.jet_batch_prof_read.argtypes = [vp, P(jet_prof_entry), i32, P(i32)]
        L.jet_km1_static.argtypes = [i32, i32, i64, vp, vp, vp, vp, i32, vp, vp]
        L.jet_km1_static_last_error.argtypes = []
        L.jet_km1_static_last_error.restype = ctypes.c_char_p
        L.jet_coarsen.argtypes = [vp, vp, i64, i32, i32, vp, P(i32)]
        L.jet_loop_counts.argtypes = [vp, P(i64), P(i64)]
        L.jet_coarsen_subround.argtypes = [vp, vp, vp, vp, i32, i64, vp]
        L.jet_flow_region.argtypes = [vp, vp, i32, i32, i32, vp]
        L.jet_flow_mincut.argtypes = [vp, vp, i32, i32, vp, P(i64), vp, vp]
        L.jet_flow_pair.argtypes = [vp, vp, i32, i32, i32, P(jet_flow_pair_stats)]
        L.jet_flow_refine.argtypes = [vp, vp, i32, i32, P(jet_flow_stats)]
        for f in ("jet_init", "jet_refine", "jet_refine_ex", "jet_rebalance", "jet_km1", "jet_phi", "jet_candidates",
                  "jet_afterburner", "jet_rebalance_round", "jet_free", "jet_prof_enable", "jet_prof_read",
                  "jet_level_stats", "jet_tau_features", "jet_mlp_create", "jet_mlp_set", "jet_mlp_get",
                  "jet_mlp_forward", "jet_mlp_grad", "jet_mlp_train_step", "jet_mlp_save", "jet_mlp_load",
                  "jet_mlp_free", "jet_refine_learned", "jet_set_option", "jet_batch_init", "jet_batch_set_option",
                  "jet_batch_refine", "jet_batch_free", "jet_km1_static", "jet_batch_prof_enable",
                  "jet_batch_prof_read", "jet_coarsen", "jet_coarsen_subround", "jet_loop_counts",
                  "jet_flow_region", "jet_flow_mincut", "jet_flow_pair", "jet_flow_refine"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


EXPORTED = ("jet_params_default", "jet_init", "jet_refine", "jet_refine_ex", "jet_rebalance", "jet_km1", "jet_phi",
            "jet_candidates", "jet_afterburner", "jet_rebalance_round", "jet_free", "jet_strerror", "jet_last_error",
            "jet_prof_enable", "jet_prof_read", "jet_level_stats", "jet_tau_features", "jet_mlp_create",
            "jet_mlp_set", "jet_mlp_get", "jet_mlp_forward", "jet_mlp_grad", "jet_mlp_train_step", "jet_mlp_save",
            "jet_mlp_load", "jet_mlp_free", "jet_mlp_last_error", "jet_refine_learned", "jet_set_option",
            "jet_batch_init", "jet_batch_set_option", "jet_batch_refine", "jet_batch_free", "jet_batch_last_error",
            "jet_km1_static", "jet_km1_static_last_error", "jet_batch_prof_enable", "jet_batch_prof_read",
            "jet_coarsen", "jet_coarsen_subround", "jet_loop_counts", "jet_flow_region", "jet_flow_mincut",
            "jet_flow_pair", "jet_flow_refine")
JET_OPT_APPLY_DIVISOR = 1
JET_OPT_APPLY_WIDE = 2
JET_OPT_PROF_FAMILIES = 3
JET_OPT_CAND_LANE_DEGREE = 4
JET_OPT_GRAPH = 6
JET_OPT_RB_SLOTS = 7
JET_OPT_REPLAYS = 8
JET_OPT_GRID = 9
JET_OPT_CO_TABLE_SLOTS = 10
JET_OPT_CAND_XCD = 11
JET_OPT_RB_XCD = 12
JET_OPT_GRAPH_KERNELS = 13
JET_OPT_APPLY_XCD = 14
JET_OPT_FLOW_WORKERS = 15
JET_OPT_SEL_SPLIT_MIN = 5
PROF_FAMILIES = ("candidates", "candidates_hub", "afterburner", "select_moves", "apply", "rebalance_gain",
                 "rebalance_select")
MLP_NPARAM = 5313


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(rc: int, ctx=None, allow_imbalanced=True):
    if rc == JET_OK or (rc == JET_IMBALANCED and allow_imbalanced):
        return rc
    msg = lib().jet_last_error(ctx).decode() or lib().jet_strerror(rc).decode()
    raise JetError(rc, msg)


def make_params(tau: Sequence[float] = (0.75, 0.375, 0.0), limit: int = 8, max_iters: int = 1000,
                deadzone_ppm: int = 100_000, max_rebalance_rounds: int = 64, rb_unweighted: int = 0) -> jet_params:
    tau = list(tau)
    if not 1 <= len(tau) <= 8:
        raise ValueError("1..8 temperatures")
    return jet_params(limit=limit, max_iters=max_iters, num_tau=len(tau),
                      tau=(ctypes.c_float * 8)(*(tau + [0.0] * (8 - len(tau)))), deadzone_ppm=deadzone_ppm,
                      max_rebalance_rounds=max_rebalance_rounds, rb_unweighted=int(rb_unweighted))


def jet_params_default() -> jet_params:
    p = jet_params()
    lib().jet_params_default(ctypes.byref(p))
    return p


def _dev(a, dtype):
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        return a.to(device="cuda", dtype=dtype).contiguous()
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def jet_init(n, m, num_pins, net_offsets, pins, net_weights, vertex_weights, k, eps):
    """Device arrays (tensors) in, context handle out."""
    h = ctypes.c_void_p()
    rc = lib().jet_init(ctypes.byref(h), n, m, num_pins, _ptr(net_offsets), _ptr(pins), _ptr(net_weights),
                        _ptr(vertex_weights), k, eps, _stream())
    _check(rc, None)
    return h


def jet_refine(ctx, part: torch.Tensor, params: jet_params, trace_cap: int = 0):
    st = jet_stats()
    if trace_cap > 0:
        tr = (jet_trace * trace_cap)()
        tlen = ctypes.c_int32()
        rc = lib().jet_refine_ex(ctx, _ptr(part), ctypes.byref(params), ctypes.byref(st), tr, trace_cap,
                                 ctypes.byref(tlen))
        _check(rc, ctx)
        trace = [{f: getattr(tr[i], f) for f, _ in jet_trace._fields_} for i in range(min(tlen.value, trace_cap))]
        return rc, st.as_dict(), trace
    rc = lib().jet_refine(ctx, _ptr(part), ctypes.byref(params), ctypes.byref(st))
    _check(rc, ctx)
    return rc, st.as_dict(), None


def jet_rebalance(ctx, part: torch.Tensor, params: jet_params):
    st = jet_stats()
    rc = lib().jet_rebalance(ctx, _ptr(part), ctypes.byref(params), ctypes.byref(st))
    _check(rc, ctx)
    return rc, st.as_dict()


def jet_km1(ctx, part: torch.Tensor) -> int:
    out = ctypes.c_int64()
    _check(lib().jet_km1(ctx, _ptr(part), ctypes.byref(out)), ctx, allow_imbalanced=False)
    return out.value


def jet_km1_static(net_offsets, pins, net_weights, part, n: int, k: int, out: torch.Tensor) -> None:
    """Enqueues the allocation-free metric (device tensors in; out: int64 device tensor of one
    element receiving the metric, -1 for an out-of-range input)."""
    m = int(net_offsets.numel()) - 1
    rc = lib().jet_km1_static(n, m, int(pins.numel()), _ptr(net_offsets), _ptr(pins), _ptr(net_weights), _ptr(part),
                              k, _ptr(out), _stream())
    if rc != JET_OK:
        raise JetError(rc, lib().jet_km1_static_last_error().decode())


def jet_phi(ctx, part: torch.Tensor, phi: torch.Tensor):
    _check(lib().jet_phi(ctx, _ptr(part), _ptr(phi)), ctx, allow_imbalanced=False)


def jet_candidates(ctx, part, lock, tau_q, t, g, in_m):
    _check(lib().jet_candidates(ctx, _ptr(part), _ptr(lock), tau_q, _ptr(t), _ptr(g), _ptr(in_m)), ctx,
           allow_imbalanced=False)


def jet_afterburner(ctx, part, t, g, in_m, rg):
    _check(lib().jet_afterburner(ctx, _ptr(part), _ptr(t), _ptr(g), _ptr(in_m), _ptr(rg)), ctx,
           allow_imbalanced=False)


def jet_rebalance_round(ctx, part, deadzone_ppm, sel_target) -> int:
    moved = ctypes.c_int32()
    _check(lib().jet_rebalance_round(ctx, _ptr(part), deadzone_ppm, _ptr(sel_target), ctypes.byref(moved)), ctx,
           allow_imbalanced=False)
    return moved.value


def jet_prof_enable(ctx, on: bool):
    _check(lib().jet_prof_enable(ctx, 1 if on else 0), ctx, allow_imbalanced=False)


def jet_prof_read(ctx):
    """{family: {"launches", "total_ms", "alg_bytes"}} accumulated since jet_prof_enable."""
    buf = (jet_prof_entry * 16)()
    cnt = ctypes.c_int32()
    _check(lib().jet_prof_read(ctx, buf, 16, ctypes.byref(cnt)), ctx, allow_imbalanced=False)
    return {buf[i].name.decode(): {"launches": buf[i].launches, "total_ms": buf[i].total_ms,
                                   "alg_bytes": buf[i].alg_bytes} for i in range(min(cnt.value, 16))}


def jet_level_stats(ctx, part: torch.Tensor) -> np.ndarray:
    out = (ctypes.c_int64 * 16)()
    _check(lib().jet_level_stats(ctx, _ptr(part), out), ctx, allow_imbalanced=False)
    return np.array(out[:], dtype=np.int64)


def jet_tau_features(stats, eps, level, levels, n_finest, rnd, rounds, prev_gain) -> np.ndarray:
    st = (ctypes.c_int64 * 16)(*[int(x) for x in stats])
    out = (ctypes.c_float * 16)()
    rc = lib().jet_tau_features(st, float(eps), level, levels, int(n_finest), rnd, rounds, float(prev_gain), out)
    if rc != JET_OK:
        raise JetError(rc, "feature arguments out of range")
    return np.array(out[:], dtype=np.float32)


def _check_mlp(rc, net):
    if rc != JET_OK:
        raise JetError(rc, lib().jet_mlp_last_error(net).decode() or lib().jet_strerror(rc).decode())


def _host_f32(a, n):
    if a is None:
        return None
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    if a.size != n:
        raise ValueError(f"{n} values expected")
    return a


class TauNet:
    """The temperature network (jet_mlp_*): device parameters, FP32 kernels for all of its work."""

    def __init__(self, seed: int = 0, path: Optional[str] = None):
        self.h = ctypes.c_void_p()
        _check_mlp(lib().jet_mlp_create(ctypes.byref(self.h), ctypes.c_uint64(seed), _stream()), None)
        if path is not None:
            self.load(path)

    def close(self):
        if self.h:
            lib().jet_mlp_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set(self, params=None, mean=None, std=None):
        p, mu, sd = _host_f32(params, MLP_NPARAM), _host_f32(mean, 16), _host_f32(std, 16)
        arg = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)
        _check_mlp(lib().jet_mlp_set(self.h, arg(p), arg(mu), arg(sd)), self.h)

    def get(self):
        p = np.empty(MLP_NPARAM, np.float32)
        mu = np.empty(16, np.float32)
        sd = np.empty(16, np.float32)
        _check_mlp(lib().jet_mlp_get(self.h, p.ctypes.data_as(ctypes.c_void_p), mu.ctypes.data_as(ctypes.c_void_p),
                                     sd.ctypes.data_as(ctypes.c_void_p)), self.h)
        return p, mu, sd

    def forward(self, X: torch.Tensor) -> torch.Tensor:
        X = X.to(device="cuda", dtype=torch.float32).contiguous()
        tau = torch.empty(X.shape[0], dtype=torch.float32, device="cuda")
        _check_mlp(lib().jet_mlp_forward(self.h, _ptr(X), X.shape[0], _ptr(tau)), self.h)
        return tau

    def grad(self, X: torch.Tensor, t: torch.Tensor):
        X = X.to(device="cuda", dtype=torch.float32).contiguous()
        t = t.to(device="cuda", dtype=torch.float32).contiguous()
        g = torch.empty(MLP_NPARAM, dtype=torch.float32, device="cuda")
        loss = ctypes.c_float()
        _check_mlp(lib().jet_mlp_grad(self.h, _ptr(X), _ptr(t), X.shape[0], _ptr(g), ctypes.byref(loss)), self.h)
        return loss.value, g

    def train_step(self, X: torch.Tensor, t: torch.Tensor, lr: float = 1e-3) -> float:
        X = X.to(device="cuda", dtype=torch.float32).contiguous()
        t = t.to(device="cuda", dtype=torch.float32).contiguous()
        loss = ctypes.c_float()
        _check_mlp(lib().jet_mlp_train_step(self.h, _ptr(X), _ptr(t), X.shape[0], lr, ctypes.byref(loss)), self.h)
        return loss.value

    def save(self, path: str):
        _check_mlp(lib().jet_mlp_save(self.h, path.encode()), self.h)

    def load(self, path: str):
        _check_mlp(lib().jet_mlp_load(self.h, path.encode()), self.h)


def jet_refine_learned(ctx, part: torch.Tensor, params: jet_params, net: Optional[TauNet], level: int, levels: int,
                       n_finest: int):
    st = jet_stats()
    tau_used = (ctypes.c_float * 8)()
    from_net = (ctypes.c_int32 * 8)()
    rc = lib().jet_refine_learned(ctx, _ptr(part), ctypes.byref(params), net.h if net is not None else None, level,
                                  levels, n_finest, ctypes.byref(st), tau_used, from_net)
    _check(rc, ctx)
    d = st.as_dict()
    d["tau_from_net"] = list(from_net[:params.num_tau])  # 0 where the fixed temperature was used
    return rc, d, list(tau_used[:params.num_tau])


def jet_set_option(ctx, option: int, value: int):
    _check(lib().jet_set_option(ctx, option, value), ctx, allow_imbalanced=False)


class JetBatch:
    """Many independent hypergraphs in one library batch (jet_batch_*)."""

    def __init__(self, hgs):
        self._keep = []
        descs = (jet_hg_desc * len(hgs))()
        for i, hg in enumerate(hgs):
            off, pins = _dev(hg.off, torch.int64), _dev(hg.pins, torch.int32)
            nw, vw = _dev(hg.net_w, torch.int32), _dev(hg.vtx_w, torch.int32)
            self._keep.append((off, pins, nw, vw))
            descs[i] = jet_hg_desc(int(hg.n), int(hg.m), int(pins.numel()), _ptr(off), _ptr(pins), _ptr(nw),
                                   _ptr(vw), int(hg.k), float(hg.eps))
        self.h = ctypes.c_void_p()
        rc = lib().jet_batch_init(ctypes.byref(self.h), len(hgs), descs, _stream())
        self._keep = None   # the contexts hold their own copies
        if rc != JET_OK:
            raise JetError(rc, lib().jet_batch_last_error(None).decode())
        self.count = len(hgs)

    def close(self):
        if self.h:
            lib().jet_batch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_option(self, option: int, value: int):
        rc = lib().jet_batch_set_option(self.h, option, value)
        if rc != JET_OK:
            raise JetError(rc, lib().jet_batch_last_error(self.h).decode())

    def refine(self, parts, replays: int = 8, **kw):
        """parts: list of device int32 tensors (refined in place); replays: iterations of the whole
        batch between two host polls.  Returns (rc, [stats], [rc_i])."""
        if len(parts) != self.count:
            raise ValueError("one partition per hypergraph")
        arr = (ctypes.c_void_p * self.count)(*[_ptr(p) for p in parts])
        st = (jet_stats * self.count)()
        rcs = (ctypes.c_int32 * self.count)()
        rc = lib().jet_batch_refine(self.h, arr, ctypes.byref(make_params(**kw)), replays, st, rcs)
        if rc < 0:
            raise JetError(rc, lib().jet_batch_last_error(self.h).decode())
        return rc, [st[i].as_dict() for i in range(self.count)], list(rcs)

    def prof_enable(self, on: bool = True):
        rc = lib().jet_batch_prof_enable(self.h, 1 if on else 0)
        if rc != JET_OK:
            raise JetError(rc, lib().jet_batch_last_error(self.h).decode())

    def prof_read(self):
        """{family: {"launches", "total_ms", "alg_bytes"}} summed over the batch's union contexts."""
        out = (jet_prof_entry * 16)()
        cnt = ctypes.c_int32()
        rc = lib().jet_batch_prof_read(self.h, out, 16, ctypes.byref(cnt))
        if rc != JET_OK:
            raise JetError(rc, lib().jet_batch_last_error(self.h).decode())
        return {out[i].name.decode(): {"launches": out[i].launches, "total_ms": out[i].total_ms,
                                       "alg_bytes": out[i].alg_bytes} for i in range(cnt.value)}


def jet_free(ctx):
    if ctx:
        lib().jet_free(ctx)


class JetContext:
    """Owns one library context for one hypergraph (a ``workloads.Hypergraph``-like object)."""

    def __init__(self, hg, k: Optional[int] = None, eps: Optional[float] = None):
        self.n, self.m = int(hg.n), int(hg.m)
        self.k = int(k if k is not None else hg.k)
        self.eps = float(eps if eps is not None else hg.eps)
        off = _dev(hg.off, torch.int64)
        pins = _dev(hg.pins, torch.int32)
        nw = _dev(hg.net_w, torch.int32)
        vw = _dev(hg.vtx_w, torch.int32)
        self.p = int(pins.numel())
        self.h = jet_init(self.n, self.m, self.p, off, pins, nw, vw, self.k, self.eps)

    def close(self):
        if self.h:
            jet_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def refine(self, part: torch.Tensor, trace_cap: int = 0, **kw):
        return jet_refine(self.h, part, make_params(**kw), trace_cap)

    def rebalance(self, part: torch.Tensor, **kw):
        return jet_rebalance(self.h, part, make_params(**kw))

    def km1(self, part: torch.Tensor) -> int:
        return jet_km1(self.h, part)

    def phi(self, part: torch.Tensor) -> torch.Tensor:
        out = torch.empty(self.m * self.k, dtype=torch.int32, device="cuda")
        jet_phi(self.h, part, out)
        return out.view(self.m, self.k)

    def candidates(self, part: torch.Tensor, tau_q: int, lock: Optional[torch.Tensor] = None):
        t = torch.empty(self.n, dtype=torch.int32, device="cuda")
        g = torch.empty(self.n, dtype=torch.int32, device="cuda")
        in_m = torch.empty(self.n, dtype=torch.uint8, device="cuda")
        jet_candidates(self.h, part, lock, tau_q, t, g, in_m)
        return t, g, in_m

    def afterburner(self, part, t, g, in_m) -> torch.Tensor:
        rg = torch.empty(self.n, dtype=torch.int32, device="cuda")
        jet_afterburner(self.h, part, t, g, in_m, rg)
        return rg

    def prof_enable(self, on: bool = True):
        jet_prof_enable(self.h, on)

    def prof_read(self):
        return jet_prof_read(self.h)

    def set_option(self, option: int, value: int):
        jet_set_option(self.h, option, value)

    def level_stats(self, part: torch.Tensor) -> np.ndarray:
        return jet_level_stats(self.h, part)

    def refine_learned(self, part: torch.Tensor, net: Optional[TauNet], level: int, levels: int, n_finest: int,
                       **kw):
        return jet_refine_learned(self.h, part, make_params(**kw), net, level, levels, n_finest)

    def loop_counts(self):
        """(host polls, iteration pieces) of the last refinement or rebalancing call."""
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().jet_loop_counts(self.h, ctypes.byref(a), ctypes.byref(b)), self.h)
        return a.value, b.value

    def coarsen(self, order: torch.Tensor, max_cluster_weight: int, initial_single: int = 100, cap_div: int = 100):
        """Synchronous clustering (jet_coarsen): returns (label int32[n] on the device, clusters)."""
        label = torch.empty(self.n, dtype=torch.int32, device="cuda")
        cnt = ctypes.c_int32()
        _check(lib().jet_coarsen(self.h, _ptr(order), int(max_cluster_weight), int(initial_single), int(cap_div),
                                 _ptr(label), ctypes.byref(cnt)), self.h, allow_imbalanced=False)
        return label, cnt.value

    def coarsen_subround(self, label: torch.Tensor, cw: torch.Tensor, verts: torch.Tensor, max_cluster_weight: int):
        """One clustering sub-round (jet_coarsen_subround) on label / cw in place; returns the targets."""
        targets = torch.empty(self.n, dtype=torch.int32, device="cuda")
        _check(lib().jet_coarsen_subround(self.h, _ptr(label), _ptr(cw), _ptr(verts) if verts.numel() else None,
                                          int(verts.numel()), int(max_cluster_weight), _ptr(targets)), self.h,
               allow_imbalanced=False)
        return targets

    def flow_region(self, part: torch.Tensor, a: int, b: int, alpha: int = FLOW_ALPHA) -> torch.Tensor:
        """Region of the block pair (a, b) (jet_flow_region): int8[n] on the device."""
        region = torch.empty(self.n, dtype=torch.int8, device="cuda")
        _check(lib().jet_flow_region(self.h, _ptr(part), int(a), int(b), int(alpha), _ptr(region)), self.h,
               allow_imbalanced=False)
        return region

    def flow_mincut(self, part: torch.Tensor, a: int, b: int, term: torch.Tensor):
        """Maximum flow for the terminals term (int8[n]) and the residual reachable sets
        (jet_flow_mincut): (flow, in_sr uint8[n], in_tr uint8[n])."""
        sr = torch.empty(self.n, dtype=torch.uint8, device="cuda")
        tr = torch.empty(self.n, dtype=torch.uint8, device="cuda")
        f = ctypes.c_int64()
        _check(lib().jet_flow_mincut(self.h, _ptr(part), int(a), int(b), _ptr(term), ctypes.byref(f), _ptr(sr),
                                     _ptr(tr)), self.h, allow_imbalanced=False)
        return f.value, sr, tr

    def flow_pair(self, part: torch.Tensor, a: int, b: int, alpha: int = FLOW_ALPHA) -> dict:
        """Two-way flow refinement of (a, b) on part in place (jet_flow_pair); returns its stats."""
        st = jet_flow_pair_stats()
        _check(lib().jet_flow_pair(self.h, _ptr(part), int(a), int(b), int(alpha), ctypes.byref(st)), self.h,
               allow_imbalanced=False)
        return st.as_dict()

    def flow_refine(self, part: torch.Tensor, alpha: int = FLOW_ALPHA, max_rounds: int = FLOW_MAX_ROUNDS) -> dict:
        """k-way flow refinement on part in place (jet_flow_refine); returns its stats."""
        st = jet_flow_stats()
        _check(lib().jet_flow_refine(self.h, _ptr(part), int(alpha), int(max_rounds), ctypes.byref(st)), self.h,
               allow_imbalanced=False)
        return st.as_dict()

    def rebalance_round(self, part: torch.Tensor, deadzone_ppm: int = 100_000):
        sel = torch.empty(self.n, dtype=torch.int32, device="cuda")
        moved = jet_rebalance_round(self.h, part, deadzone_ppm, sel)
        return sel, moved
