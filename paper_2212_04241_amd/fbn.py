"""ctypes binding of libfbn.so: the same calls as include/fbn.h, argument
marshalling only.  Every step of inference runs in the HIP library; there is
no CPU or PyTorch fallback -- if the library is missing this module raises.

PyTorch is optional plumbing: a torch stream handle can be passed as the
jt's stream, and torch's caching allocator can serve the device memory.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfbn.so")

FBN_OK = 0
FBN_E_INVALID_ARG, FBN_E_PARSE, FBN_E_IO, FBN_E_NOMEM_HOST, FBN_E_NOMEM_DEVICE = 1, 2, 3, 4, 5
FBN_E_TOO_LARGE, FBN_E_ZERO_EVIDENCE, FBN_E_STATE, FBN_E_DEVICE, FBN_E_UNDERFLOW = 6, 7, 8, 9, 10
FBN_FP64, FBN_FP32_RESCALED = 0, 1
FBN_LAYOUT_AUTO, FBN_LAYOUT_PER_SLOT, FBN_LAYOUT_INTERLEAVED = 0, 1, 2

_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class fbn_allocator(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", C.c_void_p)]


class fbn_jt_options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("max_slots", C.c_int32), ("max_clique_entries", C.c_uint64),
                ("host_only", C.c_int32), ("tile_entries", C.c_int32), ("allocator", fbn_allocator),
                ("stream", C.c_void_p), ("layout", C.c_int32), ("shrink_evidence", C.c_int32),
                ("fp64_rerun", C.c_int32), ("slots_per_block", C.c_int32), ("fin_block", C.c_int32)]


class fbn_jt_stats_t(C.Structure):
    _fields_ = [("n_vars", C.c_int32), ("n_cliques", C.c_int32), ("n_edges", C.c_int32), ("root", C.c_int32),
                ("H", C.c_int32), ("D", C.c_int32), ("T", C.c_uint64), ("K", C.c_uint64),
                ("max_clique", C.c_uint64), ("sep_total", C.c_uint64), ("device_bytes", C.c_uint64),
                ("slot_bytes", C.c_uint64), ("n_trees", C.c_int32), ("interleaved", C.c_int32)]


class FbnError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str = ""):
        super().__init__(f"{where}: {STATUS.get(code, code)} ({detail})")
        self.code = code


STATUS = {0: "ok", 1: "invalid argument", 2: "parse error", 3: "i/o error", 4: "out of host memory",
          5: "out of device memory", 6: "clique too large", 7: "zero-probability evidence", 8: "invalid state",
          9: "device error", 10: "float32 underflow"}

_lib = None


def lib():
    """Load libfbn.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2212_04241_amd.build`")
    # torch bundles its own HIP runtime under the same soname; load it first so
    # that torch and this library share one runtime in the process
    if os.environ.get("FBN_NO_TORCH") != "1":
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    i32p, f64p, vpp = P(C.c_int32), P(C.c_double), P(C.c_void_p)
    sig = {
        "fbn_default_options": (None, [P(fbn_jt_options)]),
        "fbn_load_net": (C.c_int32, [C.c_char_p, vpp]),
        "fbn_load_net_mem": (C.c_int32, [C.c_char_p, C.c_size_t, vpp]),
        "fbn_net_from_arrays": (C.c_int32, [C.c_int32, i32p, i32p, i32p, f64p, vpp]),
        "fbn_free_net": (None, [C.c_void_p]),
        "fbn_net_n_vars": (C.c_int32, [C.c_void_p, i32p]),
        "fbn_net_var_name": (C.c_int32, [C.c_void_p, C.c_int32, C.c_char_p, C.c_size_t]),
        "fbn_net_state_name": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_char_p, C.c_size_t]),
        "fbn_net_find_var": (C.c_int32, [C.c_void_p, C.c_char_p, i32p]),
        "fbn_net_find_state": (C.c_int32, [C.c_void_p, C.c_int32, C.c_char_p, i32p]),
        "fbn_net_cpt": (C.c_int32, [C.c_void_p, C.c_int32, i32p, i32p, C.c_int32, i32p, f64p, C.c_size_t,
                                    P(C.c_size_t)]),
        "fbn_build_jt": (C.c_int32, [C.c_void_p, P(fbn_jt_options), vpp]),
        "fbn_build_forest": (C.c_int32, [P(C.c_void_p), C.c_int32, P(fbn_jt_options), vpp]),
        "fbn_free_jt": (None, [C.c_void_p]),
        "fbn_set_stream": (C.c_int32, [C.c_void_p, C.c_void_p]),
        "fbn_set_graph_mode": (C.c_int32, [C.c_void_p, C.c_int32]),
        "fbn_set_evidence": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, i32p, i32p]),
        "fbn_set_evidence_batch": (C.c_int32, [C.c_void_p, C.c_int32, i32p, i32p, i32p, i32p]),
        "fbn_calibrate": (C.c_int32, [C.c_void_p, C.c_int32, i32p, f64p, i32p]),
        "fbn_query_marginals": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, i32p, f64p, C.c_size_t]),
        "fbn_query_all": (C.c_int32, [C.c_void_p, C.c_int32, i32p, f64p, C.c_size_t, f64p, i32p]),
        "fbn_fetch_async": (C.c_int32, [C.c_void_p, C.c_int32, i32p, f64p, f64p, i32p]),
        "fbn_query_joint": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, i32p, f64p, C.c_size_t]),
        "fbn_query_joint_noalloc": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, i32p, f64p, C.c_size_t]),
        "fbn_status_str": (C.c_char_p, [C.c_int32]),
        "fbn_last_error": (C.c_char_p, []),
        "fbn_jt_stats": (C.c_int32, [C.c_void_p, P(fbn_jt_stats_t)]),
        "fbn_jt_clique": (C.c_int32, [C.c_void_p, C.c_int32, i32p, C.c_int32, i32p, i32p, i32p]),
        "fbn_jt_edge": (C.c_int32, [C.c_void_p, C.c_int32, i32p, i32p, i32p, C.c_int32, i32p]),
        "fbn_jt_index_map": (C.c_int32, [C.c_void_p, C.c_int32, i32p, C.c_size_t]),
        "fbn_jt_device_index_map": (C.c_int32, [C.c_void_p, C.c_int32, i32p, C.c_size_t]),
        "fbn_jt_profile_enable": (C.c_int32, [C.c_void_p, C.c_int32]),
        "fbn_jt_profile_read": (C.c_int32, [C.c_void_p, f64p, P(C.c_int64), f64p]),
        "fbn_jt_profile_kinds": (C.c_int32, [C.c_void_p, C.c_uint32]),
        "fbn_jt_elim_order": (C.c_int32, [C.c_void_p, i32p]),
        "fbn_jt_homes": (C.c_int32, [C.c_void_p, i32p, i32p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, (a.ctypes.data_as(C.POINTER(C.c_int32)) if a.size else None)


def _check(rc, where):
    if rc != FBN_OK:
        raise FbnError(rc, where, lib().fbn_last_error().decode(errors="replace"))


class Net:
    """An fbn_net handle."""

    def __init__(self, handle):
        self._h = handle

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.fbn_free_net(self._h)
            self._h = None


def net_n_vars(net: Net) -> int:
    n = C.c_int32()
    _check(lib().fbn_net_n_vars(net._h, C.byref(n)), "fbn_net_n_vars")
    return n.value


def net_var_name(net: Net, v: int) -> str:
    buf = C.create_string_buffer(4096)
    _check(lib().fbn_net_var_name(net._h, v, buf, len(buf)), "fbn_net_var_name")
    return buf.value.decode()


def net_state_name(net: Net, v: int, s: int) -> str:
    buf = C.create_string_buffer(4096)
    _check(lib().fbn_net_state_name(net._h, v, s, buf, len(buf)), "fbn_net_state_name")
    return buf.value.decode()


def net_find_var(net: Net, name: str) -> int:
    v = C.c_int32()
    _check(lib().fbn_net_find_var(net._h, name.encode(), C.byref(v)), "fbn_net_find_var")
    return v.value


def net_find_state(net: Net, v: int, name: str) -> int:
    s = C.c_int32()
    _check(lib().fbn_net_find_state(net._h, v, name.encode(), C.byref(s)), "fbn_net_find_state")
    return s.value


def net_cpt(net: Net, v: int):
    """(card, parents, cpt) of variable v: parents in listed order, v fastest."""
    card, npar, ln = C.c_int32(), C.c_int32(), C.c_size_t()
    _check(lib().fbn_net_cpt(net._h, v, C.byref(card), None, 0, C.byref(npar), None, 0, C.byref(ln)), "fbn_net_cpt")
    par = np.zeros(max(npar.value, 1), dtype=np.int32)
    cpt = np.zeros(max(ln.value, 1), dtype=np.float64)
    _check(lib().fbn_net_cpt(net._h, v, None, par.ctypes.data_as(C.POINTER(C.c_int32)), par.size, None,
                             cpt.ctypes.data_as(C.POINTER(C.c_double)), cpt.size, None), "fbn_net_cpt")
    return card.value, par[:npar.value].copy(), cpt[:ln.value].copy()


def load_net(path: str) -> Net:
    h = C.c_void_p()
    _check(lib().fbn_load_net(path.encode(), C.byref(h)), "fbn_load_net")
    return Net(h)


def load_net_mem(text: str) -> Net:
    b = text.encode()
    h = C.c_void_p()
    _check(lib().fbn_load_net_mem(b, len(b), C.byref(h)), "fbn_load_net_mem")
    return Net(h)


def net_from_arrays(card, n_parents, parents, cpt) -> Net:
    card, pc = _i32(card)
    npar, pn = _i32(n_parents)
    par, pp = _i32(parents)
    cpt = np.ascontiguousarray(cpt, dtype=np.float64)
    h = C.c_void_p()
    _check(lib().fbn_net_from_arrays(card.size, pc, pn, pp, cpt.ctypes.data_as(C.POINTER(C.c_double)), C.byref(h)),
           "fbn_net_from_arrays")
    return Net(h)


def net_from_spec(spec) -> Net:
    """From an object with .flat() -> (card, n_parents, parents, cpt)."""
    return net_from_arrays(*spec.flat())


def _torch_allocator(device: int):
    import torch

    def alloc(_ctx, nbytes, stream):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device, stream or 0)
        except Exception:
            return None

    def free(_ctx, ptr, _stream):
        torch.cuda.caching_allocator_delete(ptr)

    return _ALLOC_FN(alloc), _FREE_FN(free)


class JT:
    """An fbn_jt handle with its options and stats.  `net` is one Net, or a
    list of Nets for a forest (fbn_build_forest)."""

    def __init__(self, net, precision: int = FBN_FP64, max_slots: int = 1, max_clique_entries: int = 0,
                 host_only: bool = False, tile_entries: int = 0, stream=None, torch_allocator: bool = False,
                 layout: int = 0, shrink_evidence: bool = False, fp64_rerun: bool = False,
                 slots_per_block: int = 0, fin_block: int = 0):
        L = lib()
        opt = fbn_jt_options()
        L.fbn_default_options(C.byref(opt))
        opt.precision = precision
        opt.max_slots = max_slots
        if max_clique_entries:
            opt.max_clique_entries = max_clique_entries
        opt.host_only = 1 if host_only else 0
        opt.tile_entries = tile_entries
        opt.layout = layout
        opt.shrink_evidence = 1 if shrink_evidence else 0
        opt.fp64_rerun = 1 if fp64_rerun else 0
        opt.slots_per_block = slots_per_block
        opt.fin_block = fin_block
        opt.stream = C.c_void_p(stream) if stream else None
        self._cb = None
        if torch_allocator and not host_only:
            import torch
            self._cb = _torch_allocator(torch.cuda.current_device())
            opt.allocator = fbn_allocator(self._cb[0], self._cb[1], None)
        h = C.c_void_p()
        if isinstance(net, (list, tuple)):
            arr = (C.c_void_p * len(net))(*[x._h for x in net])
            _check(L.fbn_build_forest(arr, len(net), C.byref(opt), C.byref(h)), "fbn_build_forest")
        else:
            _check(L.fbn_build_jt(net._h, C.byref(opt), C.byref(h)), "fbn_build_jt")
        self._h = h
        self.precision = precision
        self.max_slots = max_slots
        st = fbn_jt_stats_t()
        _check(L.fbn_jt_stats(h, C.byref(st)), "fbn_jt_stats")
        self.stats = {k: getattr(st, k) for k, _ in fbn_jt_stats_t._fields_}
        self.n = st.n_vars
        self._card = None

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.fbn_free_jt(self._h)
            self._h = None

    def free(self):
        self.__del__()


def build_jt(net: Net, **kw) -> JT:
    return JT(net, **kw)


def build_forest(nets, **kw) -> JT:
    """One jt over several independent networks (ids offset per network)."""
    return JT(list(nets), **kw)


def set_stream(jt: JT, stream) -> None:
    _check(lib().fbn_set_stream(jt._h, C.c_void_p(stream) if stream else None), "fbn_set_stream")


def set_graph_mode(jt: JT, on: bool = True) -> None:
    """Replay each calibration as one captured HIP graph (needs a stream)."""
    _check(lib().fbn_set_graph_mode(jt._h, 1 if on else 0), "fbn_set_graph_mode")


def set_evidence(jt: JT, slot: int, vars_, states) -> None:
    v, pv = _i32(vars_)
    s, ps = _i32(states)
    if v.size != s.size:
        raise ValueError("vars and states differ in length")
    _check(lib().fbn_set_evidence(jt._h, slot, v.size, pv, ps), "fbn_set_evidence")


def set_evidence_batch(jt: JT, slots, cases) -> None:
    """cases: list of (vars, states) pairs, one per slot."""
    sl, psl = _i32(slots)
    offs = np.zeros(len(cases) + 1, dtype=np.int32)
    for i, (v, _) in enumerate(cases):
        offs[i + 1] = offs[i] + len(v)
    vv = np.concatenate([np.asarray(v, dtype=np.int32) for v, _ in cases]) if cases else np.zeros(0, np.int32)
    ss = np.concatenate([np.asarray(s, dtype=np.int32) for _, s in cases]) if cases else np.zeros(0, np.int32)
    offs, po = _i32(offs)
    vv, pv = _i32(vv)
    ss, ps = _i32(ss)
    _check(lib().fbn_set_evidence_batch(jt._h, sl.size, psl, po, pv, ps), "fbn_set_evidence_batch")


def calibrate(jt: JT, slots, want_results: bool = False):
    """Collect + distribute for the slots.  With want_results, waits and
    returns (log_pe[n], status[n])."""
    sl, psl = _i32(slots)
    if want_results:
        lp = np.zeros(sl.size, dtype=np.float64)
        st = np.zeros(sl.size, dtype=np.int32)
        _check(lib().fbn_calibrate(jt._h, sl.size, psl, lp.ctypes.data_as(C.POINTER(C.c_double)),
                                   st.ctypes.data_as(C.POINTER(C.c_int32))), "fbn_calibrate")
        return lp, st
    _check(lib().fbn_calibrate(jt._h, sl.size, psl, None, None), "fbn_calibrate")
    return None


def query_marginals(jt: JT, slot: int, vars_, card) -> np.ndarray:
    v, pv = _i32(vars_)
    n = int(sum(int(card[x]) for x in v))
    out = np.zeros(n, dtype=np.float64)
    _check(lib().fbn_query_marginals(jt._h, slot, v.size, pv, out.ctypes.data_as(C.POINTER(C.c_double)), n),
           "fbn_query_marginals")
    return out


def query_all(jt: JT, slots, marg_total: int):
    """Posteriors of all variables for each slot: (post[n, marg_total], log_pe[n], status[n])."""
    sl, psl = _i32(slots)
    out = np.zeros((sl.size, marg_total), dtype=np.float64)
    lp = np.zeros(sl.size, dtype=np.float64)
    st = np.zeros(sl.size, dtype=np.int32)
    _check(lib().fbn_query_all(jt._h, sl.size, psl, out.ctypes.data_as(C.POINTER(C.c_double)), out.size,
                               lp.ctypes.data_as(C.POINTER(C.c_double)), st.ctypes.data_as(C.POINTER(C.c_int32))),
           "fbn_query_all")
    return out, lp, st


def query_joint(jt: JT, slot: int, qvars, card, noalloc: bool = False) -> np.ndarray:
    """Joint posterior P(qvars | e) of a calibrated slot, qvars[0] slowest
    (qvars must lie together in one clique).  noalloc: the entry point that
    allocates no device memory (static scratch)."""
    q, pq = _i32(qvars)
    n = int(np.prod([int(card[x]) for x in q], dtype=np.int64)) if q.size else 0
    out = np.zeros(max(n, 1), dtype=np.float64)
    fn = lib().fbn_query_joint_noalloc if noalloc else lib().fbn_query_joint
    name = "fbn_query_joint_noalloc" if noalloc else "fbn_query_joint"
    _check(fn(jt._h, slot, q.size, pq, out.ctypes.data_as(C.POINTER(C.c_double)), n), name)
    return out[:n]


def fetch_async(jt: JT, slots, post_out, log_pe_out, flags_out) -> None:
    """Enqueue result copies into caller-owned (ideally pinned) host arrays."""
    sl, psl = _i32(slots)
    P = C.POINTER
    for a, dt in ((post_out, np.float64), (log_pe_out, np.float64), (flags_out, np.int32)):
        if a is not None and (a.dtype != dt or not a.flags.c_contiguous or a.shape[0] < sl.size):
            raise ValueError("fetch_async: output arrays must be C-contiguous float64/float64/int32 with a row per slot")
    _check(lib().fbn_fetch_async(jt._h, sl.size, psl,
                                 post_out.ctypes.data_as(P(C.c_double)) if post_out is not None else None,
                                 log_pe_out.ctypes.data_as(P(C.c_double)) if log_pe_out is not None else None,
                                 flags_out.ctypes.data_as(P(C.c_int32)) if flags_out is not None else None),
           "fbn_fetch_async")


def jt_clique(jt: JT, c: int):
    buf = np.zeros(max(jt.n, 1), dtype=np.int32)
    n, h, d = C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib().fbn_jt_clique(jt._h, c, buf.ctypes.data_as(C.POINTER(C.c_int32)), buf.size, C.byref(n), C.byref(h),
                               C.byref(d)), "fbn_jt_clique")
    return buf[:n.value].copy(), h.value, d.value


def jt_edge(jt: JT, e: int):
    buf = np.zeros(max(jt.n, 1), dtype=np.int32)
    p, ch, n = C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib().fbn_jt_edge(jt._h, e, C.byref(p), C.byref(ch), buf.ctypes.data_as(C.POINTER(C.c_int32)), buf.size,
                             C.byref(n)), "fbn_jt_edge")
    return p.value, ch.value, buf[:n.value].copy()


def _parent_size(jt: JT, e: int, card) -> int:
    p, _, _ = jt_edge(jt, e)
    vs, _, _ = jt_clique(jt, p)
    return int(np.prod([int(card[v]) for v in vs], dtype=np.int64))


def jt_index_map(jt: JT, e: int, card) -> np.ndarray:
    out = np.zeros(_parent_size(jt, e, card), dtype=np.int32)
    _check(lib().fbn_jt_index_map(jt._h, e, out.ctypes.data_as(C.POINTER(C.c_int32)), out.size), "fbn_jt_index_map")
    return out


def jt_device_index_map(jt: JT, e: int, card) -> np.ndarray:
    out = np.zeros(_parent_size(jt, e, card), dtype=np.int32)
    _check(lib().fbn_jt_device_index_map(jt._h, e, out.ctypes.data_as(C.POINTER(C.c_int32)), out.size),
           "fbn_jt_device_index_map")
    return out


PROFILE_KINDS = ("collect", "collect_finalise", "distribute", "distribute_finalise", "posteriors")


def jt_profile_enable(jt: JT, on: bool = True) -> None:
    _check(lib().fbn_jt_profile_enable(jt._h, 1 if on else 0), "fbn_jt_profile_enable")


def jt_profile_kinds(jt: JT, kinds=None) -> None:
    """Time only the named kinds (None: all) while profiling is on."""
    mask = (1 << len(PROFILE_KINDS)) - 1 if kinds is None else sum(1 << PROFILE_KINDS.index(k) for k in kinds)
    _check(lib().fbn_jt_profile_kinds(jt._h, mask), "fbn_jt_profile_kinds")


def jt_profile_read(jt: JT) -> dict:
    """{kind: (ms, launches, algorithmic bytes)} since the last read."""
    n = len(PROFILE_KINDS)
    ms = np.zeros(n, dtype=np.float64)
    cnt = np.zeros(n, dtype=np.int64)
    by = np.zeros(n, dtype=np.float64)
    _check(lib().fbn_jt_profile_read(jt._h, ms.ctypes.data_as(C.POINTER(C.c_double)),
                                     cnt.ctypes.data_as(C.POINTER(C.c_int64)),
                                     by.ctypes.data_as(C.POINTER(C.c_double))), "fbn_jt_profile_read")
    return {k: (float(ms[i]), int(cnt[i]), float(by[i])) for i, k in enumerate(PROFILE_KINDS)}


def jt_elim_order(jt: JT) -> np.ndarray:
    out = np.zeros(jt.n, dtype=np.int32)
    _check(lib().fbn_jt_elim_order(jt._h, out.ctypes.data_as(C.POINTER(C.c_int32))), "fbn_jt_elim_order")
    return out


def jt_homes(jt: JT):
    a = np.zeros(jt.n, dtype=np.int32)
    b = np.zeros(jt.n, dtype=np.int32)
    _check(lib().fbn_jt_homes(jt._h, a.ctypes.data_as(C.POINTER(C.c_int32)), b.ctypes.data_as(C.POINTER(C.c_int32))),
           "fbn_jt_homes")
    return a, b
