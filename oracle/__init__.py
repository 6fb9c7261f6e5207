"""CPU oracle for the convolution Count sketch (Heddes et al., SIGMOD 2024).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference that the GPU
library is checked against.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import it.  It shares no code with the GPU library and never
imports it; both sides receive their inputs from the `workloads` generators.

What it computes, each function citing the passage it follows:

  analyze            join-graph bookkeeping: Omega(R_k), Gamma(u), Psi(u)  (Sec. 2.6,
                     Table 1, Fig. 3; initialization paragraph of Sec. 3.2)
  draw_coefficients  per repetition, one 4-wise independent sign polynomial per join
                     and one 2-wise independent bin polynomial per graph component
                     (Sec. 3.2 initialization; Def. 2.1) over p = 2^61 - 1 (Sec. 4)
  create_sketch      Alg. 2 / Eq. 4 (C implementation in csk_oracle.c)
  estimate_eq5       the estimate X of Eq. 5 by direct enumeration of J
  estimate_alg3      Alg. 3 (GetQueryEstimate / CombineSketches) in exact integers;
                     the cross-correlation of Def. 3.1 is evaluated directly (small m)
                     or modulo primes with Chinese remaindering (through the NTT when
                     m is a power of two, term by term otherwise)
  median_lower       median of the d repetitions (Sec. 3.3; Sec. 4.1 uses l = 5)
  create_attr_sketch per-attribute Count sketches with per-component hash functions
                     (Sec. 3.4 reuse) and estimate_pairwise, the two-relation estimate
                     from two of them
  create_ams_sketch  the AMS multi-join sketch of Eq. 1 (the baseline of Sec. 2; C
                     implementation in csk_oracle.c), coefficients from
                     draw_ams_coefficients
  estimate_ams       its estimator X_t = (1/m) sum_j prod_k c_{k,t,j} (Thm. 2.3), exact
  join_size          the exact cardinality E[X] of Thm. 3.1
  variance_bound     3^(r-1)/m * prod ||F_k||_2^2 of Thm. 3.1

Every estimate is an exact Python integer.  The oracle never uses floating point for
an estimate.

Conventions the paper leaves open (the project's reading):
  * components numbered by their smallest attribute id; Omega, Gamma ascending;
  * coefficients: SplitMix64 seeded with `seed`, each draw `next() >> 3`, redrawn when
    equal to p; order: for t: for each join e: a0..a3; then for each component q: b0, b1;
  * s(x) = +1 iff (a0 + a1 x + a2 x^2 + a3 x^3 mod p) is even; h(x) = (b0 + b1 x mod p) mod m;
  * median of an even count = the lower middle element;
  * root attribute of Alg. 3 = attribute 0 unless given.
"""
from __future__ import annotations

import ctypes
import dataclasses
import types
import os
import subprocess
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

P61 = (1 << 61) - 1
_U64 = (1 << 64) - 1
_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libcsk_oracle.so")
_SRC_PATH = os.path.join(_HERE, "csk_oracle.c")


# --------------------------------------------------------------------------- build / load

def build(force: bool = False) -> str:
    """Compile the C half of the oracle with gcc (plain -O2)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", _SRC_PATH, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        L.or_poly_hash.restype = ctypes.c_uint64
        L.or_poly_hash.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32]
        L.or_sign.restype = ctypes.c_int
        L.or_sign.argtypes = [ctypes.c_void_p, ctypes.c_uint32]
        L.or_bin.restype = ctypes.c_uint64
        L.or_bin.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64]
        L.or_create_sketch.restype = None
        L.or_create_sketch.argtypes = [
            ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
            ctypes.c_int32, ctypes.c_uint64,
            ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]
        L.or_create_ams_sketch.restype = None
        L.or_create_ams_sketch.argtypes = [
            ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
            ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]
        L.or_accumulate.restype = None
        L.or_accumulate.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p]
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------- join graph (Sec. 2.6, Table 1)

class GraphError(ValueError):
    pass


@dataclasses.dataclass
class QueryInfo:
    n_rel: int
    n_attr: int
    attr_rel: List[int]
    edges: List[Tuple[int, int]]
    omega: List[List[int]]            # Omega(R_k): joined attributes of R_k, ascending
    gamma: List[List[int]]            # Gamma(u): attributes joined with u, ascending
    edge_index: Dict[Tuple[int, int], int]  # (u, v) and (v, u) -> edge position
    psi: List[int]                    # Psi(u): graph component of u
    n_comp: int

    def edge_of(self, u: int, v: int) -> int:
        return self.edge_index[(u, v)]


def analyze(graph) -> QueryInfo:
    """Omega, Gamma and Psi of a join query (Sec. 2.6, Table 1; Sec. 3.2).

    Checks that the query is acyclic (Sec. 2.6: joins are non-cyclic) and connected:
    every attribute is joined, joins link different relations, and the relations with
    the joins form a tree (|E| = r - 1, as used in the proof of Thm. 2.3)."""
    r = int(graph.n_rel)
    attr_rel = [int(x) for x in graph.attr_rel]
    w = len(attr_rel)
    edges = [(int(u), int(v)) for (u, v) in graph.edges]
    if r < 1 or w < 1:
        raise GraphError("empty query")
    if any(not (0 <= k < r) for k in attr_rel):
        raise GraphError("attribute owned by a relation out of range")
    if any(not any(a == k for a in attr_rel) for k in range(r)):
        raise GraphError("relation without joined attribute")
    gamma: List[List[int]] = [[] for _ in range(w)]
    edge_index: Dict[Tuple[int, int], int] = {}
    for e, (u, v) in enumerate(edges):
        if not (0 <= u < w and 0 <= v < w) or u == v:
            raise GraphError("bad edge")
        if attr_rel[u] == attr_rel[v]:
            raise GraphError("join inside one relation")
        if (u, v) in edge_index:
            raise GraphError("duplicate join")
        edge_index[(u, v)] = e
        edge_index[(v, u)] = e
        gamma[u].append(v)
        gamma[v].append(u)
    for u in range(w):
        if not gamma[u]:
            raise GraphError("attribute %d is not joined" % u)
        gamma[u].sort()
    if len(edges) != r - 1:
        raise GraphError("query must be a tree over its relations (|E| = r - 1)")
    # relations connected through the joins?
    parent = list(range(r))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for (u, v) in edges:
        a, b = find(attr_rel[u]), find(attr_rel[v])
        if a == b:
            raise GraphError("cyclic query")
        parent[a] = b
    if len({find(k) for k in range(r)}) != 1:
        raise GraphError("query is not connected")
    # graph components of the attribute graph, numbered by smallest attribute id
    comp = [-1] * w
    n_comp = 0
    for u in range(w):
        if comp[u] >= 0:
            continue
        stack = [u]
        comp[u] = n_comp
        while stack:
            a = stack.pop()
            for b in gamma[a]:
                if comp[b] < 0:
                    comp[b] = n_comp
                    stack.append(b)
        n_comp += 1
    omega = [[u for u in range(w) if attr_rel[u] == k] for k in range(r)]
    return QueryInfo(r, w, attr_rel, edges, omega, gamma, edge_index, comp, n_comp)


# --------------------------------------------------------------------------- hash coefficients (Sec. 3.2, Sec. 4)

def splitmix64(seed: int):
    """SplitMix64 (Steele, Lea & Flood 2014) as a generator of 64-bit integers."""
    state = seed & _U64
    while True:
        state = (state + 0x9E3779B97F4A7C15) & _U64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _U64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _U64
        yield z ^ (z >> 31)


@dataclasses.dataclass
class Coefficients:
    d: int
    n_edges: int
    n_comps: int
    sign: List[List[List[int]]]   # [d][E][4]: a0, a1, a2, a3
    bins: List[List[List[int]]]   # [d][Q][2]: b0, b1

    def sign_array(self) -> np.ndarray:
        return np.array(self.sign, dtype=np.uint64).reshape(self.d, self.n_edges, 4)

    def bin_array(self) -> np.ndarray:
        return np.array(self.bins, dtype=np.uint64).reshape(self.d, self.n_comps, 2)


def draw_coefficients(seed: int, d: int, n_edges: int, n_comps: int) -> Coefficients:
    """Sample the sign hashes (one per join, degree 3: 4-wise independent) and bin
    hashes (one per component, degree 1: 2-wise independent) of Alg. 1, for each of
    the d repetitions.  Each coefficient is uniform on [0, p)."""
    g = splitmix64(seed)

    def coef():
        while True:
            c = next(g) >> 3
            if c != P61:
                return c

    sign, bins = [], []
    for _t in range(d):
        sign.append([[coef() for _ in range(4)] for _e in range(n_edges)])
        bins.append([[coef() for _ in range(2)] for _q in range(n_comps)])
    return Coefficients(d, n_edges, n_comps, sign, bins)


def poly_value(coef: Sequence[int], x: int) -> int:
    """sum_i coef[i] * x^i mod p, written as a power sum (not Horner)."""
    return sum(int(c) * pow(int(x), i, P61) for i, c in enumerate(coef)) % P61


def sign_value(coef4: Sequence[int], x: int) -> int:
    return -1 if poly_value(coef4, x) & 1 else 1


def bin_value(coef2: Sequence[int], x: int, m: int) -> int:
    return poly_value(coef2, x) % m


# --------------------------------------------------------------------------- sketches (Alg. 2, Eq. 2-4)

def _column_plan(info: QueryInfo, k: int):
    cols = info.omega[k]
    comp = np.array([info.psi[u] for u in cols], dtype=np.int32)
    nedges = np.array([len(info.gamma[u]) for u in cols], dtype=np.int32)
    max_e = max(1, int(nedges.max()))
    edges = np.zeros((len(cols), max_e), dtype=np.int32)
    for c, u in enumerate(cols):
        for i, v in enumerate(info.gamma[u]):
            edges[c, i] = info.edge_of(u, v)
    return comp, nedges, edges, max_e


def create_sketch(info: QueryInfo, k: int, keys, weights, m: int, coeffs: Coefficients,
                  out: Optional[np.ndarray] = None) -> np.ndarray:
    """Sketch c_k of relation R_k for all repetitions: int64 [d][m] (Alg. 2).

    keys: uint32-valued array [n][|Omega(R_k)|] (tuple-major, ascending attribute id);
    weights: int64 [n] or None (= +1).  `out`, if given, is accumulated into."""
    keys = np.ascontiguousarray(np.asarray(keys).astype(np.uint32, copy=False))
    n = keys.shape[0] if keys.ndim else 0
    a = len(info.omega[k])
    if n:
        keys = keys.reshape(n, a)
    if weights is not None:
        weights = np.ascontiguousarray(np.asarray(weights, dtype=np.int64))
        assert weights.shape == (n,)
    if out is None:
        out = np.zeros((coeffs.d, m), dtype=np.int64)
    assert out.dtype == np.int64 and out.shape == (coeffs.d, m) and out.flags.c_contiguous
    comp, nedges, edges, max_e = _column_plan(info, k)
    sa, ba = coeffs.sign_array(), coeffs.bin_array()
    if n:
        lib().or_create_sketch(a, _ptr(comp), _ptr(nedges), _ptr(edges), max_e,
                               coeffs.d, m, _ptr(sa), coeffs.n_edges, _ptr(ba), coeffs.n_comps,
                               _ptr(keys), _ptr(weights), n, _ptr(out))
    return out


# --------------------------------------------------------------------------- AMS multi-join baseline (Eq. 1)

def draw_ams_coefficients(seed: int, d: int, m: int, n_edges: int) -> np.ndarray:
    """Sign polynomials of the AMS multi-join sketch (Eq. 1): one degree-3 polynomial
    (4-wise independent) per join for every counter j of every repetition t, drawn from
    the same SplitMix64 stream as Alg. 1's in the order t, j, join, a0..a3.
    Returns uint64 [d][m][n_edges][4]."""
    g = splitmix64(seed)
    out = np.empty(d * m * n_edges * 4, dtype=np.uint64)
    i = 0
    while i < out.size:
        c = next(g) >> 3
        if c != P61:
            out[i] = c
            i += 1
    return out.reshape(d, m, n_edges, 4)


def create_ams_sketch(info: QueryInfo, k: int, keys, weights, m: int, coef: np.ndarray) -> np.ndarray:
    """AMS multi-join sketch of relation R_k (Eq. 1): int64 [d][m], counter (t, j) the
    sum over tuples of Delta times the product of the signs s_{t,j,{u,v}}(i_u) of every
    join {u, v} at the relation's attributes."""
    keys = np.ascontiguousarray(np.asarray(keys).astype(np.uint32, copy=False))
    n = keys.shape[0] if keys.ndim else 0
    a = len(info.omega[k])
    d = coef.shape[0]
    out = np.zeros((d, m), dtype=np.int64)
    if n == 0:
        return out
    keys = keys.reshape(n, a)
    if weights is not None:
        weights = np.ascontiguousarray(np.asarray(weights, dtype=np.int64))
    _comp, nedges, edges, max_e = _column_plan(info, k)
    ca = np.ascontiguousarray(coef, dtype=np.uint64)
    lib().or_create_ams_sketch(a, _ptr(nedges), _ptr(edges), max_e, d, m, _ptr(ca), ca.shape[2],
                               _ptr(keys), _ptr(weights), n, _ptr(out))
    return out


def estimate_ams(sketches: Sequence[np.ndarray]):
    """The AMS multi-join estimate (Eq. 1's estimator): per repetition t,
    X_t = (1/m) sum_j prod_k c_{k,t,j}.  Returns the exact numerators S_t = m X_t (Python
    integers) and the lower median of the S_t (the median of the X_t times m)."""
    d, m = sketches[0].shape
    nums = []
    for t in range(d):
        cols = [[int(v) for v in sk[t]] for sk in sketches]
        total = 0
        for j in range(m):
            prod = 1
            for c in cols:
                prod *= c[j]
            total += prod
        nums.append(total)
    return nums, median_lower(nums)


# --------------------------------------------------------------------------- per-attribute sketches (Sec. 3.4)

def draw_attr_coefficients(seed: int, d: int, n_comps: int):
    """Hash functions shared by every join inside a graph component, for sketches kept
    per attribute (Sec. 3.4: an attribute's sketch is reused by every sub-query that
    joins it once): per repetition t and component q, a sign polynomial a0..a3 then a
    bin polynomial b0, b1, in that order from the SplitMix64 stream.
    Returns (sign uint64 [d][Q][4], bin uint64 [d][Q][2])."""
    g = splitmix64(seed)

    def coef():
        while True:
            c = next(g) >> 3
            if c != P61:
                return c

    sign = np.empty((d, n_comps, 4), dtype=np.uint64)
    bins = np.empty((d, n_comps, 2), dtype=np.uint64)
    for t in range(d):
        for q in range(n_comps):
            for i in range(4):
                sign[t, q, i] = coef()
            for i in range(2):
                bins[t, q, i] = coef()
    return sign, bins


def create_attr_sketch(keys_col, weights, m: int, sign_q: np.ndarray, bin_q: np.ndarray) -> np.ndarray:
    """Count sketch of one attribute (one key column) with its component's hash
    functions: int64 [d][m], counter (t, h_t(x) mod m) += s_t(x) Delta (Alg. 2 with one
    column and one join).  sign_q [d][4], bin_q [d][2]."""
    keys = np.ascontiguousarray(np.asarray(keys_col).astype(np.uint32, copy=False).reshape(-1, 1))
    n = keys.shape[0]
    d = sign_q.shape[0]
    out = np.zeros((d, m), dtype=np.int64)
    if n == 0:
        return out
    if weights is not None:
        weights = np.ascontiguousarray(np.asarray(weights, dtype=np.int64))
    comp = np.zeros(1, dtype=np.int32)
    nedges = np.ones(1, dtype=np.int32)
    edges = np.zeros((1, 1), dtype=np.int32)
    sa = np.ascontiguousarray(sign_q.reshape(d, 1, 4), dtype=np.uint64)
    ba = np.ascontiguousarray(bin_q.reshape(d, 1, 2), dtype=np.uint64)
    lib().or_create_sketch(1, _ptr(comp), _ptr(nedges), _ptr(edges), 1, d, m, _ptr(sa), 1, _ptr(ba), 1,
                           _ptr(keys), _ptr(weights), n, _ptr(out))
    return out


def estimate_pairwise(a: np.ndarray, b: np.ndarray):
    """Estimate of a two-relation equi-join from two attribute sketches of the same
    component: per repetition the inner product (Eq. 5 with r = 2), then the lower
    median.  Returns (per-repetition exact integers, median)."""
    reps = [sum(int(x) * int(y) for x, y in zip(a[t], b[t])) for t in range(a.shape[0])]
    return reps, median_lower(reps)


# --------------------------------------------------------------------------- sub-query sketches (Sec. 3.4)

def draw_subq_coefficients(seed: int, d: int, n_comps: int, n_joins: int):
    """Hash functions of sub-query sketches (Sec. 3.4): first, per repetition t and
    component q, a shared sign polynomial a0..a3 and a bin polynomial b0, b1 (the draw
    of `draw_attr_coefficients`); then, per repetition t and join e, a sign polynomial
    a0..a3; all from one SplitMix64 stream.
    Returns (comp_sign [d][Q][4], bins [d][Q][2], join_sign [d][E][4])."""
    g = splitmix64(seed)

    def coef():
        while True:
            c = next(g) >> 3
            if c != P61:
                return c

    comp_sign = np.empty((d, n_comps, 4), dtype=np.uint64)
    bins = np.empty((d, n_comps, 2), dtype=np.uint64)
    join_sign = np.empty((d, n_joins, 4), dtype=np.uint64)
    for t in range(d):
        for q in range(n_comps):
            for i in range(4):
                comp_sign[t, q, i] = coef()
            for i in range(2):
                bins[t, q, i] = coef()
    for t in range(d):
        for e in range(n_joins):
            for i in range(4):
                join_sign[t, e, i] = coef()
    return comp_sign, bins, join_sign


@dataclasses.dataclass
class SubQuery:
    """One sub-query of a base query: a connected set of its joins."""
    joins: List[int]                  # base join ids, ascending
    relations: List[int]              # base relations it touches, ascending
    graph: object                     # the sub-query as a join query (n_rel, attr_rel, edges), renumbered
    # per relation of the sub-query (in `relations` order): its joined columns as
    # (column index in the base relation, base component, sign functions), where a sign
    # function is ("comp", q) for component q's shared polynomial or ("join", e)
    columns: List[List[Tuple[int, int, Tuple[Tuple[str, int], ...]]]]


def subquery(base_graph, joins: Sequence[int]) -> SubQuery:
    """The sub-query of `base_graph` made of the given joins, with its hash assignment.

    The sub-query is the join query on the relations its joins touch, keeping only the
    attributes those joins name; relations, attributes and joins are renumbered in
    ascending base order.  Hash functions (Sec. 3.4: an attribute's sketch can be reused
    by every join involving it): an attribute's bin hash is that of its base component;
    inside the sub-query, a component with a single join signs both of its attributes
    with the component's shared polynomial, and a component with two or more joins signs
    each join with that join's own polynomial (independent signs, as Alg. 2 draws one
    sign hash per join)."""
    info = analyze(base_graph)
    joins = sorted(set(int(e) for e in joins))
    if not joins or any(not (0 <= e < len(info.edges)) for e in joins):
        raise GraphError("sub-query joins out of range")
    attrs = sorted({u for e in joins for u in info.edges[e]})
    rels = sorted({info.attr_rel[u] for u in attrs})
    rel_local = {k: i for i, k in enumerate(rels)}
    attr_local = {u: i for i, u in enumerate(attrs)}
    graph = types.SimpleNamespace(
        n_rel=len(rels), attr_rel=tuple(rel_local[info.attr_rel[u]] for u in attrs),
        edges=tuple((attr_local[info.edges[e][0]], attr_local[info.edges[e][1]]) for e in joins))
    sub_info = analyze(graph)  # raises when the joins are not connected
    # joins of each component of the sub-query (components of its own attribute graph)
    comp_joins: Dict[int, List[int]] = {}
    for i, e in enumerate(joins):
        comp_joins.setdefault(sub_info.psi[graph.edges[i][0]], []).append(e)
    columns = []
    for k in rels:
        cols = []
        for c, u in enumerate(info.omega[k]):
            if u not in attr_local:
                continue
            mine = [e for e in joins if u in info.edges[e]]
            in_comp = comp_joins[sub_info.psi[attr_local[u]]]
            if len(in_comp) == 1:
                signs = (("comp", info.psi[u]),)
            else:
                signs = tuple(("join", e) for e in mine)
            cols.append((c, info.psi[u], signs))
        columns.append(cols)
    return SubQuery(joins, rels, graph, columns)


def create_subq_sketch(base_info: QueryInfo, columns, keys, weights, m: int, comp_sign: np.ndarray,
                       bins: np.ndarray, join_sign: np.ndarray) -> np.ndarray:
    """Alg. 2 for one relation of a sub-query: int64 [d][m], with bucket (sum over the
    listed columns of their component's bin hash) mod m and sign the product of every
    listed sign function over the columns.  keys: the base relation's [n][a] keys;
    columns: one entry of `SubQuery.columns`."""
    keys = np.asarray(keys).astype(np.uint32, copy=False)
    n = keys.shape[0]
    d = bins.shape[0]
    Q = comp_sign.shape[1]
    out = np.zeros((d, m), dtype=np.int64)
    if n == 0:
        return out
    cols = [c for c, _, _ in columns]
    sub = np.ascontiguousarray(keys.reshape(n, -1)[:, cols])
    comp = np.array([q for _, q, _ in columns], dtype=np.int32)
    nedges = np.array([len(sg) for _, _, sg in columns], dtype=np.int32)
    max_e = int(nedges.max())
    edges = np.zeros((len(cols), max_e), dtype=np.int32)
    for i, (_, _, sg) in enumerate(columns):
        for j, (kind, idx) in enumerate(sg):
            edges[i, j] = idx if kind == "comp" else Q + idx   # the table below: shared signs, then joins
    table = np.ascontiguousarray(np.concatenate([comp_sign, join_sign], axis=1), dtype=np.uint64)
    ba = np.ascontiguousarray(bins, dtype=np.uint64)
    if weights is not None:
        weights = np.ascontiguousarray(np.asarray(weights, dtype=np.int64))
    lib().or_create_sketch(len(cols), _ptr(comp), _ptr(nedges), _ptr(edges), max_e, d, m, _ptr(table),
                           table.shape[1], _ptr(ba), base_info.n_comp, _ptr(sub), _ptr(weights), n, _ptr(out))
    return out


def filter_rows(keys, weights, attrs, predicates):
    """The tuples a query's filters keep (Sec. 4.1: filter predicates are applied while
    the relation streams in, so failing tuples never reach the sketch): rows i with
    lo <= attrs[i][col] <= hi for every (col, lo, hi).  Returns (keys, weights) of the
    kept rows in input order (weights None stays None)."""
    keys = np.asarray(keys)
    attrs = np.asarray(attrs).astype(np.uint64).reshape(keys.shape[0], -1)
    keep = np.ones(keys.shape[0], dtype=bool)
    for col, lo, hi in predicates:
        keep &= (attrs[:, col] >= lo) & (attrs[:, col] <= hi)
    return keys[keep], (None if weights is None else np.asarray(weights)[keep])


def create_sketch_py(info: QueryInfo, k: int, keys, weights, m: int, t: int,
                     sign_fn: Optional[Callable[[int, int], int]] = None,
                     bin_fn: Optional[Callable[[int, int], int]] = None,
                     coeffs: Optional[Coefficients] = None) -> List[int]:
    """Alg. 2 in pure Python for one repetition t, exact integers (no wrap).

    sign_fn(edge, x) and bin_fn(component, x) may be injected (worked examples);
    otherwise they come from `coeffs`."""
    if sign_fn is None:
        sign_fn = lambda e, x: sign_value(coeffs.sign[t][e], x)
    if bin_fn is None:
        bin_fn = lambda q, x: bin_value(coeffs.bins[t][q], x, m)
    c = [0] * m
    for i, tup in enumerate(keys):
        delta = 1 if weights is None else int(weights[i])
        x, j = 1, 0
        for col, u in enumerate(info.omega[k]):
            j = j + bin_fn(info.psi[u], int(tup[col]))
            for v in info.gamma[u]:
                x = sign_fn(info.edge_of(u, v), int(tup[col])) * x
        j = j % m
        c[j] += x * delta
    return c


def wrap_int64(v: int) -> int:
    v &= _U64
    return v - (1 << 64) if v >= (1 << 63) else v


# --------------------------------------------------------------------------- estimate (Eq. 5, Alg. 3)

def estimate_eq5(info: QueryInfo, sketches: Sequence[Sequence[int]], m: int) -> int:
    """X = sum_{j in J} prod_k c_{k, G_k(j)}, G_k(j) = (sum_{u in Omega(R_k)} j_{Psi(u)}) mod m
    (Eq. 5), by enumerating J = [m]^(number of components).  Exponential: tiny cases."""
    c = [[int(v) for v in s] for s in sketches]
    Q = info.n_comp
    total = 0
    j = [0] * Q
    while True:
        prod = 1
        for k in range(info.n_rel):
            g = sum(j[info.psi[u]] for u in info.omega[k]) % m
            prod *= c[k][g]
            if prod == 0:
                break
        total += prod
        q = 0
        while q < Q:
            j[q] += 1
            if j[q] < m:
                break
            j[q] = 0
            q += 1
        if q == Q:
            return total


class _ExactRing:
    """Vectors of Python integers; cross-correlation evaluated by Def. 3.1 directly."""

    def __init__(self, m):
        self.m = m

    def vec(self, c):
        return [int(v) for v in c]

    def ones(self):
        return [1] * self.m

    def hadamard(self, a, b):
        return [x * y for x, y in zip(a, b)]

    def correlate(self, a, x):
        # (a star x)_j = sum_i conj(a_i) x_{(j+i) mod m}; integer vectors: conj(a) = a
        m = self.m
        return [sum(a[i] * x[(j + i) % m] for i in range(m)) for j in range(m)]

    def total(self, x):
        return sum(x)


class _ModRing:
    """Vectors modulo a prime p (< 2^31) with m | p - 1; cross-correlation through the
    number-theoretic transform (a textbook radix-2 NTT) when m is a power of two, by
    its definition otherwise; exact modulo p."""

    def __init__(self, m, p, g):
        self.m, self.p, self.g = m, p, g

    def vec(self, c):
        if isinstance(c, np.ndarray) and c.dtype == np.int64:
            return (c % np.int64(self.p)).astype(np.uint64)
        return np.asarray([int(v) % self.p for v in c], dtype=np.uint64)

    def ones(self):
        return np.ones(self.m, dtype=np.uint64)

    def hadamard(self, a, b):
        return (a * b) % np.uint64(self.p)

    def correlate(self, a, x):
        m, p = self.m, self.p
        if m & (m - 1):
            # m not a power of two: Def. 3.1 term by term modulo p,
            # (a star x)_j = sum_i a_i x_{(j+i) mod m}, rows j in blocks
            out = np.empty(m, dtype=np.uint64)
            i = np.arange(m)
            for j0 in range(0, m, 256):
                j = np.arange(j0, min(m, j0 + 256))
                prod = (a[None, :] * x[(j[:, None] + i[None, :]) % m]) % np.uint64(p)
                out[j0:j0 + len(j)] = np.sum(prod, axis=1, dtype=np.uint64) % np.uint64(p)
            return out
        # a star x = (reverse a) * x, reverse(a)_i = a_{(-i) mod m} (circular convolution)
        ar = a[(-np.arange(m)) % m]
        fa = ntt(ar, p, self.g)
        fx = ntt(x, p, self.g)
        return ntt((fa * fx) % np.uint64(p), p, self.g, inverse=True)

    def total(self, x):
        return int(np.sum(x, dtype=np.uint64)) % self.p


class _SparseRing:
    """Vectors of Python integers held as {index: nonzero value}; cross-correlation by
    Def. 3.1 over the nonzero entries only: (a star x)_j collects a_i x_l at j = (l - i)
    mod m.  Exact for any m; the cost follows the supports, so it serves sketches of
    few tuples at large m (where the dense rings cost O(m^2) or O(m log m) per prime).
    The all-ones vector of CombineSketches is kept symbolic (None)."""

    def __init__(self, m):
        self.m = m

    def vec(self, c):
        return {int(j): int(v) for j, v in enumerate(c) if v != 0} if not isinstance(c, np.ndarray) else \
            {int(j): int(c[j]) for j in np.flatnonzero(c)}

    def ones(self):
        return None

    def hadamard(self, a, b):
        if a is None:
            return b
        if b is None:
            return a
        if len(a) > len(b):
            a, b = b, a
        return {j: v * b[j] for j, v in a.items() if j in b}

    def correlate(self, a, x):
        if a is None or x is None:
            raise ValueError("correlation with the all-ones vector does not occur in a valid query")
        m = self.m
        out: Dict[int, int] = {}
        for i, ai in a.items():
            for l, xl in x.items():
                j = (l - i) % m
                out[j] = out.get(j, 0) + ai * xl
        return {j: v for j, v in out.items() if v != 0}

    def total(self, x):
        return sum(x.values())


def estimate_sparse(info: QueryInfo, sketches: Sequence[Sequence[int]], m: int, root: int = 0) -> int:
    """GetQueryEstimate of Alg. 3 for one repetition in exact integers over the sketches'
    nonzero counters (_SparseRing): the same ring operations as estimate_alg3, any m."""
    ring = _SparseRing(m)
    return ring.total(_combine_sketches(root, set(), info, sketches, ring))


def _combine_sketches(u: int, V: set, info: QueryInfo, c, ring):
    """CombineSketches of Alg. 3."""
    k = info.attr_rel[u]
    x = ring.vec(c[k])
    V.add(u)
    for u2 in info.omega[k]:
        if u2 == u:
            continue
        V.add(u2)
        a = ring.ones()
        for v in info.gamma[u2]:
            a = ring.hadamard(_combine_sketches(v, V, info, c, ring), a)
        x = ring.correlate(a, x)
    for v in info.gamma[u]:
        if v in V:
            continue
        x = ring.hadamard(_combine_sketches(v, V, info, c, ring), x)
    return x


def estimate_alg3(info: QueryInfo, sketches: Sequence[Sequence[int]], m: int,
                  root: int = 0, method: str = "auto") -> int:
    """GetQueryEstimate of Alg. 3 for one repetition, exact.

    method 'direct': integer vectors, correlation by Def. 3.1 (O(m^2));
    method 'ntt':    the same sequence of ring operations modulo enough primes, then
                     the Chinese remainder theorem; |X| <= prod_k ||c_k||_1 fixes how
                     many primes are needed.  Correlations go through the NTT when m is
                     a power of two and term by term (Def. 3.1, O(m^2)) otherwise."""
    if method == "auto":
        method = "direct" if m <= 64 else "ntt"
    if method == "direct":
        return _ExactRing(m).total(_combine_sketches(root, set(), info, sketches, _ExactRing(m)))
    bound = l1_bound(sketches)
    primes = []
    modulus = 1
    for p in ntt_primes(m):
        if modulus > 2 * bound:
            break
        primes.append(p)
        modulus *= p
    if modulus <= 2 * bound:
        raise ValueError("not enough NTT primes for this bound")
    residues = []
    for p in primes:
        ring = _ModRing(m, p, primitive_root(p))
        residues.append(ring.total(_combine_sketches(root, set(), info, sketches, ring)))
    return crt_centered(residues, primes)


def estimate(info: QueryInfo, sketches, m: int, method: str = "auto", root: int = 0):
    """Per-repetition exact estimates X_t and their lower median.

    sketches: sequence over relations of int64 [d][m]."""
    d = len(sketches[0])
    reps = []
    for t in range(d):
        ct = [sketches[k][t] for k in range(info.n_rel)]
        if method == "eq5":
            reps.append(estimate_eq5(info, ct, m))
        else:
            reps.append(estimate_alg3(info, ct, m, root=root, method=method))
    return reps, median_lower(reps)


def median_lower(values: Sequence[int]) -> int:
    """Median of the repetitions (Sec. 3.3); the lower middle element for even counts."""
    s = sorted(values)
    return s[(len(s) - 1) // 2]


# --------------------------------------------------------------------------- NTT helpers

def _is_prime(n: int) -> bool:
    if n < 2:
        return False
    for q in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        if n % q == 0:
            return n == q
    dd, s = n - 1, 0
    while dd % 2 == 0:
        dd //= 2
        s += 1
    for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        x = pow(a, dd, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


_PRIME_CACHE: Dict[int, List[int]] = {}


def ntt_primes(m: int, count: int = 24) -> List[int]:
    """Primes p < 2^31 with m | p - 1, largest first."""
    step = max(2, m)
    if step not in _PRIME_CACHE:
        out = []
        c = ((1 << 31) - 1) // step
        while len(out) < count and c > 0:
            p = c * step + 1
            if p < (1 << 31) and _is_prime(p):
                out.append(p)
            c -= 1
        _PRIME_CACHE[step] = out
    return _PRIME_CACHE[step]


def _factor(n: int) -> List[int]:
    fs, q = [], 2
    while q * q <= n:
        if n % q == 0:
            fs.append(q)
            while n % q == 0:
                n //= q
        q += 1
    if n > 1:
        fs.append(n)
    return fs


def primitive_root(p: int) -> int:
    fs = _factor(p - 1)
    g = 2
    while any(pow(g, (p - 1) // q, p) == 1 for q in fs):
        g += 1
    return g


_TW: Dict[Tuple[int, int, int, bool], np.ndarray] = {}


def _twiddles(p: int, g: int, length: int, inverse: bool) -> np.ndarray:
    key = (p, g, length, inverse)
    if key not in _TW:
        w = pow(g, (p - 1) // length, p)
        if inverse:
            w = pow(w, p - 2, p)
        half = length // 2
        t = np.empty(half, dtype=np.uint64)
        acc = 1
        for i in range(half):
            t[i] = acc
            acc = acc * w % p
        _TW[key] = t
    return _TW[key]


def ntt(a: np.ndarray, p: int, g: int, inverse: bool = False) -> np.ndarray:
    """Cyclic NTT of length n = len(a) (a power of two) modulo p:
    A_f = sum_n a_n w^(n f), w a primitive n-th root of unity; inverse includes 1/n."""
    n = len(a)
    a = np.asarray(a, dtype=np.uint64) % np.uint64(p)
    if n == 1:
        return a.copy()
    bits = n.bit_length() - 1
    idx = np.arange(n)
    rev = np.zeros(n, dtype=np.int64)
    for b in range(bits):
        rev |= ((idx >> b) & 1) << (bits - 1 - b)
    a = a[rev].copy()
    P = np.uint64(p)
    length = 2
    while length <= n:
        tw = _twiddles(p, g, length, inverse)
        blk = a.reshape(-1, length)
        u = blk[:, : length // 2]
        v = (blk[:, length // 2:] * tw) % P
        a = np.concatenate(((u + v) % P, (u + P - v) % P), axis=1).reshape(-1)
        length *= 2
    if inverse:
        a = (a * np.uint64(pow(n, p - 2, p))) % P
    return a


def crt_centered(residues: Sequence[int], primes: Sequence[int]) -> int:
    """The integer X with |X| < prod(primes)/2 and X = r_i mod p_i."""
    M = 1
    for p in primes:
        M *= p
    x = 0
    for r, p in zip(residues, primes):
        Mi = M // p
        x += int(r) * Mi * pow(Mi % p, p - 2, p)
    x %= M
    return x - M if x > M // 2 else x


# --------------------------------------------------------------------------- ground truth (Thm. 3.1)

def frequency_tensor(keys, weights=None) -> Dict[Tuple[int, ...], int]:
    """F_k: tuple -> net frequency (sum of Delta)."""
    F: Dict[Tuple[int, ...], int] = {}
    for i, tup in enumerate(np.asarray(keys).tolist()):
        t = tuple(int(v) for v in (tup if isinstance(tup, list) else [tup]))
        F[t] = F.get(t, 0) + (1 if weights is None else int(weights[i]))
    return {t: f for t, f in F.items() if f != 0}


def join_size(info: QueryInfo, freqs: Sequence[Dict[Tuple[int, ...], int]]) -> int:
    """E[X] of Thm. 3.1: sum over tuple combinations of prod_k F_k(i) * prod_{joins} 1(i_u = i_v).

    Joined attributes of one graph component must carry one common value, so the sum
    runs over one value per component: relations are visited in order and each tuple
    is kept only if it agrees with the values its components already hold."""
    r = info.n_rel
    order = list(range(r))

    def rec(pos: int, assign: Dict[int, int]) -> int:
        if pos == r:
            return 1
        k = order[pos]
        total = 0
        for tup, f in freqs[k].items():
            new = dict(assign)
            ok = True
            for col, u in enumerate(info.omega[k]):
                q = info.psi[u]
                if q in new and new[q] != tup[col]:
                    ok = False
                    break
                new[q] = tup[col]
            if ok:
                total += f * rec(pos + 1, new)
        return total

    return rec(0, {})


def join_size_bruteforce(info: QueryInfo, freqs) -> int:
    """Thm. 3.1's E[X] as literally written: all combinations of one tuple per relation,
    multiplied by the indicator of every join's equality.  Exponential: tiny inputs."""
    items = [list(F.items()) for F in freqs]
    total = 0

    def rec(k, chosen):
        nonlocal total
        if k == info.n_rel:
            val = {}
            for kk, (tup, _f) in enumerate(chosen):
                for col, u in enumerate(info.omega[kk]):
                    val[u] = tup[col]
            if all(val[u] == val[v] for (u, v) in info.edges):
                prod = 1
                for _tup, f in chosen:
                    prod *= f
                total += prod
            return
        for it in items[k]:
            rec(k + 1, chosen + [it])

    rec(0, [])
    return total


def variance_bound(info: QueryInfo, freqs, m: int) -> float:
    """3^(r-1)/m * prod_k ||F_k||_2^2 (Thm. 3.1)."""
    v = 3.0 ** (info.n_rel - 1) / m
    for F in freqs:
        v *= float(sum(f * f for f in F.values()))
    return v


def l1_bound(sketches) -> int:
    """prod_k ||c_k||_1, an upper bound on |X| for a tree query."""
    b = 1
    for s in sketches:
        b *= l1_norm(s)
    return b


def l1_norm(c) -> int:
    """sum_j |c_j| as an exact integer."""
    if isinstance(c, np.ndarray) and c.dtype == np.int64:
        u = c.view(np.uint64)
        mag = np.where(c < 0, (~u) + np.uint64(1), u)
        lo = int(np.sum(mag & np.uint64(0xFFFFFFFF), dtype=np.uint64))
        hi = int(np.sum(mag >> np.uint64(32), dtype=np.uint64))
        return (hi << 32) + lo
    return sum(abs(int(v)) for v in c)
