"""ctypes wrapper of the FP64 junction-tree oracle -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The GPU library never loads it and never falls back to it.

Each function cites the part of the paper it follows; the paper (a two-page
poster) gives no formulas, so the textbook junction-tree (Hugin) steps fill in
what it names: compiling the network into cliques and separators with potential
tables, passing messages along the tree (Section 1), and the reduction,
marginalisation and extension table operations (Section 2).

Parity pins: every function here is checked by tests that do not reuse it
(brute-force joint enumeration, hand-derived exact fractions, forward-backward
on chains, the naive-Bayes closed form, chordality / running-intersection /
maximality checks, a networkx maximum spanning tree weight, brute-force
eccentricity, re-derived index maps).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, E_INVALID, E_PARSE, E_TOO_LARGE, E_ZERO_EVIDENCE, E_NOMEM = range(6)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no vectorisation pragmas)."""
    if force or not os.path.exists(_LIB_PATH):
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared",
                               os.path.join(_HERE, "oracle.c"), "-o", _LIB_PATH, "-lm"])
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = C.CDLL(_LIB_PATH)
    P = C.POINTER
    i32p, i64p, f64p = P(C.c_int32), P(C.c_int64), P(C.c_double)
    lib.orc_net_from_text.argtypes = [C.c_char_p, C.c_size_t, P(C.c_void_p), C.c_char_p, C.c_size_t]
    lib.orc_net_from_arrays.argtypes = [C.c_int, i32p, i32p, i32p, f64p, P(C.c_void_p), C.c_char_p, C.c_size_t]
    lib.orc_net_free.argtypes = [C.c_void_p]
    lib.orc_compile.argtypes = [C.c_void_p, C.c_uint64, P(C.c_void_p)]
    lib.orc_jt_free.argtypes = [C.c_void_p]
    lib.orc_jt_stats.argtypes = [C.c_void_p, i64p]
    lib.orc_jt_clique.argtypes = [C.c_void_p, C.c_int, i32p, C.c_int, i32p, i32p]
    lib.orc_jt_edge.argtypes = [C.c_void_p, C.c_int, i32p, i32p, i32p, C.c_int]
    lib.orc_jt_map.argtypes = [C.c_void_p, C.c_int, i64p, C.c_size_t]
    lib.orc_jt_elim_order.argtypes = [C.c_void_p, i32p]
    lib.orc_jt_homes.argtypes = [C.c_void_p, i32p, i32p]
    lib.orc_jt_prior.argtypes = [C.c_void_p, f64p, C.c_size_t]
    lib.orc_query.argtypes = [C.c_void_p, C.c_int, i32p, i32p, f64p, f64p, f64p, f64p]
    lib.orc_query_joint.argtypes = [C.c_void_p, C.c_int, i32p, i32p, C.c_int, i32p, f64p]
    _lib = lib
    return lib


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct)) if a is not None else None


class OracleError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


class OracleNet:
    """A parsed and validated network (paper Section 1: a DAG over discrete
    variables with their conditional probability tables)."""

    def __init__(self, handle, n, card):
        self._h = handle
        self.n = n
        self.card = card

    @classmethod
    def from_text(cls, text: str):
        lib = _load()
        h = C.c_void_p()
        err = C.create_string_buffer(256)
        b = text.encode()
        rc = lib.orc_net_from_text(b, len(b), C.byref(h), err, 256)
        if rc:
            raise OracleError(rc, err.value.decode())
        from fbngen import net_from_text
        net = net_from_text(text)
        return cls(h, net.n, np.asarray(net.card, dtype=np.int32))

    @classmethod
    def from_net(cls, net, structure_only: bool = False):
        lib = _load()
        card, npar, par, cpt = net.flat()
        h = C.c_void_p()
        err = C.create_string_buffer(256)
        rc = lib.orc_net_from_arrays(net.n, _ptr(card, C.c_int32), _ptr(npar, C.c_int32),
                                     _ptr(par if par.size else np.zeros(1, np.int32), C.c_int32),
                                     None if structure_only else _ptr(cpt, C.c_double), C.byref(h), err, 256)
        if rc:
            raise OracleError(rc, err.value.decode())
        return cls(h, net.n, card.copy())

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_net_free(self._h)
            self._h = None


class OracleJT:
    """The compiled junction tree (paper Section 1: cliques and separators with
    potential tables; Section 2: the layer of every clique, the root chosen
    for the fewest layers, and the index mappings between tables)."""

    def __init__(self, net: OracleNet, max_entries: int = 0):
        lib = _load()
        self.net = net
        h = C.c_void_p()
        rc = lib.orc_compile(net._h, max_entries, C.byref(h))
        if rc:
            raise OracleError(rc, "compile")
        self._h = h
        st = np.zeros(8, dtype=np.int64)
        lib.orc_jt_stats(h, _ptr(st, C.c_int64))
        (self.n_cliques, self.n_edges, self.root, self.H, self.D, self.T, self.K, self.max_clique) = [int(x) for x in st]
        self.card = net.card

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_jt_free(self._h)
            self._h = None

    def clique(self, c):
        buf = np.zeros(max(1, self.net.n), dtype=np.int32)
        h = C.c_int32(); d = C.c_int32()
        k = _load().orc_jt_clique(self._h, c, _ptr(buf, C.c_int32), buf.size, C.byref(h), C.byref(d))
        return buf[:k].copy(), int(h.value), int(d.value)

    def edge(self, e):
        buf = np.zeros(max(1, self.net.n), dtype=np.int32)
        p = C.c_int32(); ch = C.c_int32()
        k = _load().orc_jt_edge(self._h, e, C.byref(p), C.byref(ch), _ptr(buf, C.c_int32), buf.size)
        return int(p.value), int(ch.value), buf[:k].copy()

    def clique_size(self, c):
        vs, _, _ = self.clique(c)
        return int(np.prod([int(self.card[v]) for v in vs], dtype=np.int64)) if len(vs) else 1

    def index_map(self, e):
        p, _, _ = self.edge(e)
        out = np.zeros(self.clique_size(p), dtype=np.int64)
        rc = _load().orc_jt_map(self._h, e, _ptr(out, C.c_int64), out.size)
        if rc:
            raise OracleError(rc, "map")
        return out

    def elim_order(self):
        out = np.zeros(self.net.n, dtype=np.int32)
        _load().orc_jt_elim_order(self._h, _ptr(out, C.c_int32))
        return out

    def homes(self):
        a = np.zeros(self.net.n, dtype=np.int32)
        b = np.zeros(self.net.n, dtype=np.int32)
        _load().orc_jt_homes(self._h, _ptr(a, C.c_int32), _ptr(b, C.c_int32))
        return a, b

    def prior(self):
        out = np.zeros(self.T, dtype=np.float64)
        _load().orc_jt_prior(self._h, _ptr(out, C.c_double), out.size)
        return out

    def sep_total(self):
        return sum(int(np.prod([int(self.card[v]) for v in self.edge(e)[2]], dtype=np.int64))
                   for e in range(self.n_edges))

    def query(self, vars_, states, tables=False, seps=False):
        """Exact inference for one evidence case (paper Section 1): returns
        (log P(e), posteriors concatenated over variables[, calibrated clique
        tables][, separator tables])."""
        lib = _load()
        v = np.ascontiguousarray(vars_, dtype=np.int32)
        s = np.ascontiguousarray(states, dtype=np.int32)
        post = np.zeros(int(np.sum(self.card)), dtype=np.float64)
        lp = C.c_double()
        tab = np.zeros(self.T, dtype=np.float64) if tables else None
        sp = np.zeros(max(1, self.sep_total()), dtype=np.float64) if seps else None
        rc = lib.orc_query(self._h, v.size, _ptr(v if v.size else np.zeros(1, np.int32), C.c_int32),
                           _ptr(s if s.size else np.zeros(1, np.int32), C.c_int32), C.byref(lp),
                           _ptr(post, C.c_double), _ptr(tab, C.c_double), _ptr(sp, C.c_double))
        if rc:
            raise OracleError(rc, "query")
        out = [float(lp.value), post]
        if tables:
            out.append(tab)
        if seps:
            out.append(sp)
        return tuple(out)


def query_joint(ojt: OracleJT, vars_, states, qvars):
    """Joint posterior P(qvars | evidence) for query variables lying together
    in one clique (paper Section 1: the conditional probability of the query
    variables given the evidence), qvars[0] slowest, qvars[-1] fastest."""
    lib = _load()
    v = np.ascontiguousarray(vars_, dtype=np.int32)
    s = np.ascontiguousarray(states, dtype=np.int32)
    q = np.ascontiguousarray(qvars, dtype=np.int32)
    out = np.zeros(int(np.prod([int(ojt.card[x]) for x in q], dtype=np.int64)) if q.size else 1, dtype=np.float64)
    rc = lib.orc_query_joint(ojt._h, v.size, _ptr(v if v.size else np.zeros(1, np.int32), C.c_int32),
                             _ptr(s if s.size else np.zeros(1, np.int32), C.c_int32), q.size,
                             _ptr(q if q.size else np.zeros(1, np.int32), C.c_int32), _ptr(out, C.c_double))
    if rc:
        raise OracleError(rc, "joint query")
    return out


def compile_net(net, max_entries: int = 0, structure_only: bool = False) -> OracleJT:
    return OracleJT(OracleNet.from_net(net, structure_only=structure_only), max_entries)


def probe_cap(net, max_entries: int):
    """0 if min-fill keeps every elimination clique within max_entries,
    else the variables of the first clique that exceeds it."""
    lib = _load()
    lib.orc_probe_cap.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(C.c_int32), C.c_int]
    on = OracleNet.from_net(net, structure_only=True)
    buf = np.zeros(net.n + 1, dtype=np.int32)
    m = lib.orc_probe_cap(on._h, max_entries, _ptr(buf, C.c_int32), buf.size)
    return None if m == 0 else buf[:m].copy()
