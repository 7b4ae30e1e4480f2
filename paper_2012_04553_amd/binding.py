"""ctypes binding of libpm.so (argument marshalling only).

Every computation runs in the HIP library; this module converts Python
values to the C-ABI declared in include/pm.h and back.  PyTorch provides the
device arena (one uint8 tensor) and the stream.  There is no fallback: when
the library is missing or cannot be loaded, :func:`lib` raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpm.so")

PM_OK = 0
STATUS = {0: "PM_OK", -1: "PM_E_INVAL", -2: "PM_E_NOMEM", -3: "PM_E_OVERFLOW",
          -4: "PM_E_UNSUPPORTED", -5: "PM_E_DEVICE", -6: "PM_E_BUSY", -7: "PM_E_TIMEOUT",
          -8: "PM_E_CANCELLED", -9: "PM_E_NOTFOUND"}
EDGE_INDUCED, VERTEX_INDUCED = 0, 1
AGG_COUNT, AGG_MNI = 0, 1
MORPH_NONE, MORPH_NAIVE, MORPH_COST = 0, 1, 2


class PMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class pm_pattern(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("edge_mask", ctypes.c_uint32),
                ("induce", ctypes.c_uint32), ("label", ctypes.c_int32 * 8)]


class pm_graph_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("m", ctypes.c_uint64), ("max_degree", ctypes.c_uint32),
                ("max_out_degree", ctypes.c_uint32), ("labeled", ctypes.c_uint32),
                ("device_bytes", ctypes.c_uint64)]


class pm_query_stats(ctypes.Structure):
    _fields_ = [("plan_ms", ctypes.c_double), ("kernel_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double), ("alg_bytes", ctypes.c_uint64),
                ("work_items", ctypes.c_uint64), ("num_alt", ctypes.c_uint32),
                ("launches", ctypes.c_uint32)]


class pm_launch_stat(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_char * 32), ("alg_bytes", ctypes.c_uint64), ("ms", ctypes.c_double)]


SERVE_MAX_PATTERNS = 8


class pm_serve_request(ctypes.Structure):
    _fields_ = [("arrival_s", ctypes.c_double), ("graph_id", ctypes.c_uint32),
                ("npat", ctypes.c_uint32), ("morph", ctypes.c_int32),
                ("pats", pm_pattern * SERVE_MAX_PATTERNS)]


class pm_serve_result(ctypes.Structure):
    _fields_ = [("latency_s", ctypes.c_double), ("queue_s", ctypes.c_double),
                ("status", ctypes.c_int32), ("batch_size", ctypes.c_uint32),
                ("values", ctypes.c_int64 * SERVE_MAX_PATTERNS), ("setup_s", ctypes.c_double),
                ("service_s", ctypes.c_double)]


class pm_serve_config(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_uint32), ("max_batch", ctypes.c_uint32),
                ("budget_bytes", ctypes.c_uint64), ("deadline_s", ctypes.c_double),
                ("progress_every", ctypes.c_uint32)]


class pm_serve_stats(ctypes.Structure):
    _fields_ = [("p50_s", ctypes.c_double), ("p99_s", ctypes.c_double), ("mean_s", ctypes.c_double),
                ("max_s", ctypes.c_double), ("makespan_s", ctypes.c_double),
                ("matches_per_s", ctypes.c_double), ("mean_inflight", ctypes.c_double),
                ("batches", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("timeouts", ctypes.c_uint64),
                ("mean_setup_s", ctypes.c_double), ("mean_service_s", ctypes.c_double),
                ("sustained_qps", ctypes.c_double), ("shed", ctypes.c_uint64)]


# name -> (restype, argtypes) for every function declared in include/pm.h
_P = ctypes.c_void_p
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_patp = ctypes.POINTER(pm_pattern)
SIGNATURES = {
    "pm_create": (ctypes.c_int32, [_P, ctypes.c_uint64, _P, ctypes.c_int, ctypes.POINTER(_P)]),
    "pm_destroy": (ctypes.c_int32, [_P]),
    "pm_graph_load": (ctypes.c_int32, [_P, ctypes.c_uint32, _u32p, _u32p, _u8p, _u32p]),
    "pm_graph_unload": (ctypes.c_int32, [_P, ctypes.c_uint32]),
    "pm_graph_stats": (ctypes.c_int32, [_P, ctypes.c_uint32, ctypes.POINTER(pm_graph_info)]),
    "pm_query_footprint": (ctypes.c_int32, [_P, ctypes.c_uint32, _patp, ctypes.c_uint32,
                                            ctypes.c_int32, ctypes.c_int32, _u64p]),
    "pm_submit": (ctypes.c_int32, [_P, ctypes.c_uint32, _patp, ctypes.c_uint32, ctypes.c_int32,
                                   ctypes.c_int32, _u64p]),
    "pm_wait": (ctypes.c_int32, [_P, ctypes.c_uint64, _i64p, ctypes.c_int64]),
    "pm_last_query_stats": (ctypes.c_int32, [_P, ctypes.POINTER(pm_query_stats)]),
    "pm_cancel": (ctypes.c_int32, [_P, ctypes.c_uint64]),
    "pm_last_launch_stats": (ctypes.c_int32, [_P, ctypes.POINTER(pm_launch_stat), ctypes.c_uint32,
                                              ctypes.POINTER(ctypes.c_uint32)]),
    "pm_morph_plan": (ctypes.c_int32, [_patp, ctypes.c_uint32, ctypes.c_int32, ctypes.c_int32,
                                       _patp, _u32p, _i64p]),
    "pm_morph_plan_costs": (ctypes.c_int32, [_patp, ctypes.c_uint32, _patp, ctypes.POINTER(ctypes.c_double),
                                             ctypes.c_uint32, _patp, _u32p, _i64p]),
    "pm_fsm": (ctypes.c_int32, [_P, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int64,
                                ctypes.c_int32, _i64p, _u8p, ctypes.c_uint64]),
    "pm_fsm_levelwise": (ctypes.c_int32, [_P, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                          ctypes.c_int64, ctypes.c_int32, _patp, _i64p, ctypes.c_uint64,
                                          _u64p]),
    "pm_list": (ctypes.c_int32, [_P, ctypes.c_uint32, _patp, ctypes.c_int32, _u32p, ctypes.c_uint64, _u64p]),
    "pm_fsm_num_slots": (ctypes.c_uint64, [ctypes.c_uint32]),
    "pm_fsm_slot": (ctypes.c_int32, [ctypes.c_uint32, ctypes.c_uint64, _patp]),
    "pm_set_option": (ctypes.c_int32, [_P, ctypes.c_char_p, ctypes.c_int64]),
    "pm_autotune": (ctypes.c_int32, [_P, ctypes.c_uint32, _patp, ctypes.c_uint32, ctypes.c_int32,
                                     _i64p, ctypes.POINTER(ctypes.c_double)]),
    "pm_plan_describe": (ctypes.c_int32, [_P, ctypes.c_uint32, _patp, ctypes.c_char_p,
                                          ctypes.c_uint64]),
    "pm_serve": (ctypes.c_int32, [_P, ctypes.POINTER(pm_serve_request), ctypes.c_uint32,
                                  ctypes.POINTER(pm_serve_config), ctypes.POINTER(pm_serve_result),
                                  ctypes.POINTER(pm_serve_stats)]),
    "pm_count_noalloc": (ctypes.c_int32, [_P, ctypes.c_uint32, _patp, ctypes.c_uint32,
                                          ctypes.c_int32, _i64p]),
    "pm_last_error": (ctypes.c_char_p, []),
    "pm_status_str": (ctypes.c_char_p, [ctypes.c_int32]),
}

_lib = None


def lib():
    """Load libpm.so; raises when it is missing (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2012_04553_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int):
    if status != PM_OK:
        msg = lib().pm_last_error()
        raise PMError(status, msg.decode() if msg else "")


def make_pattern(k: int, edge_mask: int, induced: bool, labels=None) -> pm_pattern:
    p = pm_pattern()
    p.k = k
    p.edge_mask = edge_mask
    p.induce = VERTEX_INDUCED if induced else EDGE_INDUCED
    for i in range(8):
        p.label[i] = -1
    if labels is not None:
        for i, l in enumerate(labels):
            p.label[i] = int(l)
    return p


def pattern_array(pats) -> ctypes.Array:
    arr = (pm_pattern * len(pats))()
    for i, p in enumerate(pats):
        if isinstance(p, pm_pattern):
            arr[i] = p
        else:
            arr[i] = make_pattern(*p)
    return arr


def fsm_slot(num_labels: int, slot: int):
    """Pattern (k, edge_mask, labels) of an FSM slot (host-only)."""
    p = pm_pattern()
    check(lib().pm_fsm_slot(num_labels, slot, ctypes.byref(p)))
    return p.k, p.edge_mask, [p.label[i] for i in range(p.k)]


def fsm_num_slots(num_labels: int) -> int:
    return int(lib().pm_fsm_num_slots(num_labels))


def morph_plan(pats, morph: int = MORPH_NAIVE, agg: int = AGG_COUNT):
    """Host-only: alternative pattern set and conversion matrix."""
    arr = pattern_array(pats)
    cap = ctypes.c_uint32(1024)
    alt = (pm_pattern * 1024)()
    mat = (ctypes.c_int64 * (len(pats) * 1024))()
    check(lib().pm_morph_plan(arr, len(pats), agg, morph, alt, ctypes.byref(cap), mat))
    na = cap.value
    alts = [(alt[j].k, alt[j].edge_mask, alt[j].induce == VERTEX_INDUCED,
             [alt[j].label[i] for i in range(alt[j].k)]) for j in range(na)]
    matrix = np.array([mat[i] for i in range(len(pats) * na)], dtype=np.int64).reshape(len(pats), na)
    return alts, matrix


def morph_plan_costs(pats, cost_pats, costs):
    """Host-only cost-based morph planning with caller-given costs: the
    cheapest mixed (vertex-/edge-induced) alternative set and its matrix."""
    arr = pattern_array(pats)
    carr = pattern_array(cost_pats)
    cst = (ctypes.c_double * max(1, len(costs)))(*[float(c) for c in costs])
    cap = ctypes.c_uint32(1024)
    alt = (pm_pattern * 1024)()
    mat = (ctypes.c_int64 * (len(pats) * 1024))()
    check(lib().pm_morph_plan_costs(arr, len(pats), carr, cst, len(costs), alt, ctypes.byref(cap), mat))
    na = cap.value
    alts = [(alt[j].k, alt[j].edge_mask, alt[j].induce == VERTEX_INDUCED,
             [alt[j].label[i] for i in range(alt[j].k)]) for j in range(na)]
    matrix = np.array([mat[i] for i in range(len(pats) * na)], dtype=np.int64).reshape(len(pats), na)
    return alts, matrix


class Engine:
    """One pm_ctx on one GPU: arena + stream come from torch."""

    def __init__(self, arena_bytes: int = 8 << 30, device: int = 0, stream=None):
        import torch
        self.torch = torch
        self.device = device
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=f"cuda:{device}")
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.ctx = ctypes.c_void_p()
        check(lib().pm_create(ctypes.c_void_p(self.arena.data_ptr()), arena_bytes,
                              ctypes.c_void_p(self.stream.cuda_stream), device,
                              ctypes.byref(self.ctx)))

    def close(self):
        if self.ctx:
            check(lib().pm_destroy(self.ctx))
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_option(self, key: str, value: int):
        check(lib().pm_set_option(self.ctx, key.encode(), int(value)))

    def graph_load(self, n, row_ptr, col, labels=None) -> int:
        rp = np.ascontiguousarray(row_ptr, dtype=np.uint32)
        cl = np.ascontiguousarray(col, dtype=np.uint32)
        if cl.size == 0:
            cl = np.zeros(1, dtype=np.uint32)
        lb = None if labels is None else np.ascontiguousarray(labels, dtype=np.uint8)
        gid = ctypes.c_uint32()
        check(lib().pm_graph_load(self.ctx, n, rp.ctypes.data_as(_u32p), cl.ctypes.data_as(_u32p),
                                  None if lb is None else lb.ctypes.data_as(_u8p),
                                  ctypes.byref(gid)))
        return gid.value

    def load(self, g) -> int:
        return self.graph_load(g.n, g.row_ptr, g.col, g.labels)

    def graph_unload(self, gid: int):
        check(lib().pm_graph_unload(self.ctx, gid))

    def graph_stats(self, gid: int) -> dict:
        info = pm_graph_info()
        check(lib().pm_graph_stats(self.ctx, gid, ctypes.byref(info)))
        return {f: getattr(info, f) for f, _ in pm_graph_info._fields_}

    def footprint(self, gid, pats, morph=MORPH_NAIVE) -> int:
        arr = pattern_array(pats)
        out = ctypes.c_uint64()
        check(lib().pm_query_footprint(self.ctx, gid, arr, len(pats), AGG_COUNT, morph,
                                       ctypes.byref(out)))
        return out.value

    def submit(self, gid, pats, morph=MORPH_NAIVE, agg=AGG_COUNT) -> int:
        arr = pattern_array(pats)
        t = ctypes.c_uint64()
        check(lib().pm_submit(self.ctx, gid, arr, len(pats), agg, morph, ctypes.byref(t)))
        return t.value

    def wait(self, ticket: int, npat: int, timeout_us: int = -1) -> list[int]:
        out = (ctypes.c_int64 * npat)()
        check(lib().pm_wait(self.ctx, ticket, out, timeout_us))
        return [int(x) for x in out]

    def count(self, gid, pats, morph=MORPH_NAIVE) -> list[int]:
        return self.wait(self.submit(gid, pats, morph), len(pats))

    def mni(self, gid, pats, morph=MORPH_NONE) -> list[int]:
        """MNI support of every pattern (pm_submit with PM_AGG_MNI)."""
        return self.wait(self.submit(gid, pats, morph, agg=AGG_MNI), len(pats))

    def fsm_levelwise(self, gid, num_labels: int, max_edges: int, threshold: int, morph=MORPH_NONE):
        """Frequent labeled patterns with 1..max_edges edges: [(k, mask, labels, support)]."""
        cnt = ctypes.c_uint64()
        n = 4096
        while True:
            pats = (pm_pattern * n)()
            sup = (ctypes.c_int64 * n)()
            st = lib().pm_fsm_levelwise(self.ctx, gid, num_labels, max_edges, threshold, morph, pats, sup,
                                        n, ctypes.byref(cnt))
            if st == PM_OK or cnt.value <= n:
                check(st)
                break
            n = cnt.value     # capacity was short: run again with room for all
        return [(pats[i].k, pats[i].edge_mask, [pats[i].label[j] for j in range(pats[i].k)], int(sup[i]))
                for i in range(cnt.value)]

    def list(self, gid, pat, morph=MORPH_NONE, capacity=None):
        """Distinct matched subgraphs of one pattern (pm_list): (rows of k
        vertex ids, total number).  Without `capacity` every row is returned."""
        arr = pattern_array([pat])
        k = arr[0].k
        cnt = ctypes.c_uint64()
        cap = capacity if capacity is not None else 1 << 16
        while True:
            out = np.zeros(max(cap, 1) * k, dtype=np.uint32)
            check(lib().pm_list(self.ctx, gid, arr, morph, out.ctypes.data_as(_u32p), cap, ctypes.byref(cnt)))
            if capacity is not None or cnt.value <= cap:
                break
            cap = cnt.value
        got = min(cnt.value, cap)
        return out[: got * k].reshape(got, k), int(cnt.value)

    def count_noalloc(self, gid, pats, morph=MORPH_NAIVE) -> list[int]:
        """pm_count_noalloc: the same counts without allocating device memory."""
        arr = pattern_array(pats)
        out = (ctypes.c_int64 * len(pats))()
        check(lib().pm_count_noalloc(self.ctx, gid, arr, len(pats), morph, out))
        return [int(x) for x in out]

    def last_stats(self) -> dict:
        s = pm_query_stats()
        check(lib().pm_last_query_stats(self.ctx, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in pm_query_stats._fields_}

    def launch_stats(self) -> list[dict]:
        """Per-launch kernel name, algorithmic bytes and device ms of the last query."""
        n = ctypes.c_uint32()
        arr = (pm_launch_stat * 64)()
        check(lib().pm_last_launch_stats(self.ctx, arr, 64, ctypes.byref(n)))
        return [{"kernel": arr[i].kernel.decode(), "alg_bytes": int(arr[i].alg_bytes), "ms": arr[i].ms}
                for i in range(n.value)]

    def autotune(self, gid, pats, morph=MORPH_NAIVE):
        arr = pattern_array(pats)
        cfg = (ctypes.c_int64 * 3)()
        ms = ctypes.c_double()
        check(lib().pm_autotune(self.ctx, gid, arr, len(pats), morph, cfg, ctypes.byref(ms)))
        return {"blocks_per_cu": cfg[0], "item_budget": cfg[1], "item_split": cfg[2], "ms": ms.value}

    def fsm(self, gid, num_labels: int, threshold: int, morph=MORPH_NONE):
        """MNI support of every labeled 3-edge pattern (dense slot order) and
        the frequent flags (support >= threshold)."""
        ns = int(lib().pm_fsm_num_slots(num_labels))
        sup = np.zeros(ns, dtype=np.int64)
        freq = np.zeros(ns, dtype=np.uint8)
        check(lib().pm_fsm(self.ctx, gid, num_labels, threshold, morph,
                           sup.ctypes.data_as(_i64p), freq.ctypes.data_as(_u8p), ns))
        return sup, freq

    def cancel(self, ticket: int):
        check(lib().pm_cancel(self.ctx, ticket))

    def serve(self, requests, max_slots=8, max_batch=8, budget_bytes=None, deadline_s=0.0,
              progress_every=0):
        """Replay a request trace through the serving loop.

        requests: [(arrival_s, graph_id, [(k, mask, induced, labels), ...], morph)]
        Returns (per-request dicts, stats dict)."""
        n = len(requests)
        arr = (pm_serve_request * n)()
        for i, (t, gid, pats, morph) in enumerate(requests):
            r = arr[i]
            r.arrival_s = float(t)
            r.graph_id = gid
            r.npat = len(pats)
            r.morph = morph
            for j, p in enumerate(pats):
                r.pats[j] = p if isinstance(p, pm_pattern) else make_pattern(*p)
        cfg = pm_serve_config()
        cfg.max_slots = max_slots
        cfg.max_batch = max_batch
        cfg.budget_bytes = budget_bytes if budget_bytes is not None else self.arena.numel() // 2
        cfg.deadline_s = deadline_s
        cfg.progress_every = progress_every
        res = (pm_serve_result * n)()
        st = pm_serve_stats()
        check(lib().pm_serve(self.ctx, arr, n, ctypes.byref(cfg), res, ctypes.byref(st)))
        out = []
        for i in range(n):
            R = res[i]
            out.append({"latency_s": R.latency_s, "queue_s": R.queue_s, "status": R.status,
                        "batch_size": R.batch_size, "setup_s": R.setup_s, "service_s": R.service_s,
                        "values": [int(R.values[j]) for j in range(arr[i].npat)]})
        return out, {f: getattr(st, f) for f, _ in pm_serve_stats._fields_}

    def plan_describe(self, gid, pat) -> str:
        buf = ctypes.create_string_buffer(8192)
        arr = pattern_array([pat])
        check(lib().pm_plan_describe(self.ctx, gid, arr, buf, 8192))
        return buf.value.decode()
