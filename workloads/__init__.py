"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds no arithmetic of the sketching method: it only builds join-graph
descriptions and draws key / weight streams.  Both the CPU oracle and the GPU path
consume what it produces; neither imports the other.

Join graphs follow the paper's model (Sec. 2.6, Fig. 3): attributes are globally
numbered vertices, each owned by one relation; an edge {u, v} is an equi-join.

Key streams stand in for the paper's skewed real columns (Sec. 4.1, Fig. 5): a
bounded Zipf law P(rank k) proportional to k^-s over k = 1..D, key = k - 1, drawn by
inverse-CDF lookup of counter-based uniforms.  The uniforms are SplitMix64 outputs
(Steele, Lea & Flood 2014) of (seed, index), so the same (seed, index) yields the
same key on the CPU and on the GPU.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import torch

GOLDEN = 0x9E3779B97F4A7C15
_MIX1 = 0xBF58476D1CE4E5B9
_MIX2 = 0x94D049BB133111EB
DATA_SEED_BASE = 0x240215953


def _s64(v: int) -> int:
    """Reinterpret an unsigned 64-bit integer as a signed one (torch has no uint64)."""
    v &= (1 << 64) - 1
    return v - (1 << 64) if v >= (1 << 63) else v


def _lsr(z: torch.Tensor, k: int) -> torch.Tensor:
    """Logical right shift of int64 tensors holding 64-bit patterns."""
    return (z >> k) & ((1 << (64 - k)) - 1)


def splitmix64_at(seed: int, index: torch.Tensor) -> torch.Tensor:
    """The (index+1)-th output of a SplitMix64 generator seeded with `seed`.

    Returned as int64 tensors holding the unsigned 64-bit pattern.  Wrap-around
    multiplication of int64 tensors is used on purpose.
    """
    s = index.to(torch.int64) + 1
    z = s * _s64(GOLDEN) + _s64(seed)
    z = (z ^ _lsr(z, 30)) * _s64(_MIX1)
    z = (z ^ _lsr(z, 27)) * _s64(_MIX2)
    return z ^ _lsr(z, 31)


def uniform01(seed: int, n: int, device="cpu", offset: int = 0) -> torch.Tensor:
    """n float64 uniforms on [0, 1) with 53 random bits, counter-based."""
    idx = torch.arange(offset, offset + n, device=device, dtype=torch.int64)
    z = splitmix64_at(seed, idx)
    return _lsr(z, 11).to(torch.float64) * (2.0 ** -53)


_CDF_CACHE = {}


def zipf_cdf(s: float, D: int) -> torch.Tensor:
    """float64 CDF of the bounded Zipf law over ranks 1..D (built on the CPU)."""
    key = (float(s), int(D))
    if key not in _CDF_CACHE:
        k = torch.arange(1, D + 1, dtype=torch.float64)
        w = k.pow(-float(s))
        cdf = torch.cumsum(w, 0)
        cdf = cdf / cdf[-1]
        cdf[-1] = 1.0
        _CDF_CACHE[key] = cdf
    return _CDF_CACHE[key]


def zipf_keys(n: int, s: float, D: int, seed: int, device="cpu", offset: int = 0) -> torch.Tensor:
    """n uint32-valued keys (int64 tensor) from Zipf(s) over [0, D)."""
    cdf = zipf_cdf(s, D).to(device)
    u = uniform01(seed, n, device=device, offset=offset)
    k = torch.searchsorted(cdf, u, right=True)
    return k.clamp_(max=D - 1)


def uniform_keys(n: int, D: int, seed: int, device="cpu", offset: int = 0) -> torch.Tensor:
    """n keys uniform on [0, D) (int64 tensor)."""
    u = uniform01(seed, n, device=device, offset=offset)
    k = torch.floor(u * D).to(torch.int64)
    return k.clamp_(max=D - 1)


def data_seed(config: int, relation: int, column: int) -> int:
    return DATA_SEED_BASE + 1000 * config + 10 * relation + column


# --------------------------------------------------------------------------- graphs


@dataclasses.dataclass(frozen=True)
class JoinGraph:
    """A join query: attributes 0..w-1, attr_rel[u] = owning relation, edges = joins."""

    n_rel: int
    attr_rel: Tuple[int, ...]
    edges: Tuple[Tuple[int, int], ...]
    name: str = ""

    @property
    def n_attr(self) -> int:
        return len(self.attr_rel)

    def columns(self, k: int) -> List[int]:
        """Attributes of relation k in ascending id: the key-column order."""
        return [u for u, r in enumerate(self.attr_rel) if r == k]


def single_join() -> JoinGraph:
    """R0(A) join R1(A)."""
    return JoinGraph(2, (0, 1), ((0, 1),), "single")


def chain(r: int) -> JoinGraph:
    """R0(A0) - R1(A0, A1) - ... - R_{r-1}(A_{r-2}); r >= 2."""
    assert r >= 2
    attr_rel = [0]
    for k in range(1, r - 1):
        attr_rel += [k, k]
    attr_rel.append(r - 1)
    edges = tuple((2 * i, 2 * i + 1) for i in range(r - 1))
    return JoinGraph(r, tuple(attr_rel), edges, f"chain{r}")


def star(r: int) -> JoinGraph:
    """Centre R0 with r-1 attributes, each joined to a leaf relation; r >= 2."""
    assert r >= 2
    attr_rel = [0] * (r - 1) + list(range(1, r))
    edges = tuple((i, r - 1 + i) for i in range(r - 1))
    return JoinGraph(r, tuple(attr_rel), edges, f"star{r}")


def fig3_query() -> JoinGraph:
    """The example query of the paper's Fig. 3: R0(0), R1(1, 2), R2(3), R3(4);
    joins {0,1}, {1,3}, {2,4}."""
    return JoinGraph(4, (0, 1, 1, 2, 3), ((0, 1), (1, 3), (2, 4)), "fig3")


def multiway_star(r: int) -> JoinGraph:
    """All r relations joined on one value: R0.A = R1.A = ... through R0 (one component
    with r attributes)."""
    attr_rel = tuple(range(r))
    edges = tuple((0, k) for k in range(1, r))
    return JoinGraph(r, attr_rel, edges, f"mstar{r}")


def connected_subqueries(graph: JoinGraph, min_joins: int = 1) -> List[int]:
    """Every connected set of the query's joins (as a bit mask of join ids), with at
    least `min_joins` joins: the sub-queries a join-order enumeration asks about.  The
    relations and joins form a tree, so a join set is connected exactly when it touches
    one relation more than it has joins."""
    out = []
    E = len(graph.edges)
    for mask in range(1, 1 << E):
        js = [e for e in range(E) if (mask >> e) & 1]
        if len(js) < min_joins:
            continue
        rels = {graph.attr_rel[u] for e in js for u in graph.edges[e]}
        if len(rels) == len(js) + 1:
            out.append(mask)
    return out


def subquery_graph(graph: JoinGraph, mask: int):
    """The sub-query made of the joins in `mask` as a join query of its own: its
    relations, its attributes (those its joins name) and its joins, renumbered in
    ascending base order.  Returns (JoinGraph, base relations, per relation the base
    key-column indices it keeps)."""
    js = [e for e in range(len(graph.edges)) if (mask >> e) & 1]
    attrs = sorted({u for e in js for u in graph.edges[e]})
    rels = sorted({graph.attr_rel[u] for u in attrs})
    rl = {k: i for i, k in enumerate(rels)}
    al = {u: i for i, u in enumerate(attrs)}
    g = JoinGraph(len(rels), tuple(rl[graph.attr_rel[u]] for u in attrs),
                  tuple((al[graph.edges[e][0]], al[graph.edges[e][1]]) for e in js), f"{graph.name}/sub{mask}")
    cols = [[c for c, u in enumerate(graph.columns(k)) if u in al] for k in rels]
    return g, rels, cols


# --------------------------------------------------------------------------- relations


def relation_keys(graph: JoinGraph, k: int, n: int, dist: str, config: int,
                  s: float = 1.1, D: int = 10 ** 6, device="cpu", offset: int = 0) -> torch.Tensor:
    """Tuple-major keys [n, a_k] (int64 tensor holding uint32 values) for relation k.
    Columns are drawn independently; joined attributes share the rank->key map."""
    cols = []
    for c in range(len(graph.columns(k))):
        seed = data_seed(config, k, c)
        if dist == "zipf":
            cols.append(zipf_keys(n, s, D, seed, device=device, offset=offset))
        elif dist == "uniform":
            cols.append(uniform_keys(n, D, seed, device=device, offset=offset))
        else:
            raise ValueError(dist)
    return torch.stack(cols, dim=1)


def turnstile_weights(n: int, delete_frac: float, seed: int, device="cpu") -> torch.Tensor:
    """+1 / -1 weights (int64) with the given fraction of deletes."""
    u = uniform01(seed ^ 0x5DEECE66D, n, device=device)
    return torch.where(u < delete_frac, -1, 1).to(torch.int64)


def random_weights(n: int, lo: int, hi: int, seed: int) -> torch.Tensor:
    """int64 weights uniform on [lo, hi] (CPU)."""
    g = torch.Generator().manual_seed(seed)
    return torch.randint(lo, hi + 1, (n,), generator=g, dtype=torch.int64)


def random_small_relation(graph: JoinGraph, k: int, n: int, domain: int, seed: int) -> torch.Tensor:
    """Keys [n, a_k] uniform on a tiny domain (CPU), for brute-force tests."""
    g = torch.Generator().manual_seed(seed)
    a = len(graph.columns(k))
    return torch.randint(0, domain, (n, a), generator=g, dtype=torch.int64)


# --------------------------------------------------------------------------- batched / serving workloads


@dataclasses.dataclass
class QuerySpec:
    graph: JoinGraph
    m: int
    d: int
    n_per_rel: Tuple[int, ...]
    sketch_seed: int


def batched_queries(n_queries: int, seed: int, m_log2=(10, 16), d_choices=(5, 9),
                    n_range=(10 ** 3, 10 ** 6), r_range=(2, 6)) -> List[QuerySpec]:
    """Chain / star queries with uneven sizes (p = 1/2 each shape), r ~ U{r_range},
    per-relation n ~ log-uniform over n_range, m = 2^U{m_log2}, d ~ U{d_choices}."""
    g = torch.Generator().manual_seed(seed)
    out = []
    for q in range(n_queries):
        r = int(torch.randint(r_range[0], r_range[1] + 1, (1,), generator=g))
        shape = "chain" if float(torch.rand(1, generator=g)) < 0.5 else "star"
        graph = chain(r) if shape == "chain" else star(r)
        m = 1 << int(torch.randint(m_log2[0], m_log2[1] + 1, (1,), generator=g))
        d = d_choices[int(torch.randint(0, len(d_choices), (1,), generator=g))]
        lo, hi = math.log(n_range[0]), math.log(n_range[1])
        ns = tuple(int(round(math.exp(lo + (hi - lo) * float(torch.rand(1, generator=g)))))
                   for _ in range(r))
        out.append(QuerySpec(graph, m, d, ns, 7 + q))
    return out


def scaled_queries(specs: Sequence[QuerySpec], factor: float) -> List[QuerySpec]:
    """The same queries with tuple counts scaled (for reduced-size test variants)."""
    return [dataclasses.replace(s, n_per_rel=tuple(max(1, int(n * factor)) for n in s.n_per_rel))
            for s in specs]
