"""Seeded synthetic LP instances shaped like the paper's workloads.

This module only draws graphs and writes the LP relaxations of Section 2 and
Appendix B (vertex cover, independent set as set packing, multiway cut) in a
plain row-compressed form.  It holds none of the solver's arithmetic: both
the HIP path and the oracle consume what it returns.

Every draw goes through ``numpy.random.Generator(Philox(seed))`` so a seed
fixes an instance on every machine.

LP convention (the problem statement of Section 3.1 plus bounds and
inequality rows, Appendix C):

    minimise  c^T x
    subject to  A_i x  (>= | <= | =)  b_i      per row, ``sense`` +1 / -1 / 0
                0 <= x_j <= u_j                (u_j may be +inf)
                optional simplex blocks: x_B in Delta_k, some blocks fixed.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

__all__ = [
    "LPInstance", "rng_for", "er_edges", "ba_edges", "regular_edges",
    "grid_edges", "vc_lp", "mis_lp", "mc_grid_lp", "vc_er", "vc_ba",
    "mis_regular", "mc_grid", "serving_trace", "set_cover", "multicover", "kcs_packing",
    "map_lp", "map_chain_window",
]


@dataclass
class LPInstance:
    m: int                      # rows
    n: int                      # structural columns
    row_ptr: np.ndarray         # int64[m+1]
    col_idx: np.ndarray         # int32[nnz], ascending inside each row
    val: Optional[np.ndarray]   # float64[nnz] or None (all entries are 1)
    b: np.ndarray               # float64[m]
    c: np.ndarray               # float64[n]
    u: np.ndarray               # float64[n] (np.inf allowed)
    sense: np.ndarray           # int8[m]: +1 '>=', -1 '<=', 0 '='
    # simplex blocks (multiway cut): block t owns columns
    # block_first_col[t] .. block_first_col[t]+k-1
    block_first_col: Optional[np.ndarray] = None   # int64[nblocks]
    block_k: int = 0
    fixed_label: Optional[np.ndarray] = None       # int32[nblocks], -1 = free
    # pairwise factors of a MAP-inference LP: factor e joins blocks
    # pair_ends[e, 0], pair_ends[e, 1]; its k*k columns start at
    # pair_first[e], row-major in (label of the first, label of the second)
    pair_ends: Optional[np.ndarray] = None         # int32[nfactors, 2]
    pair_first: Optional[np.ndarray] = None        # int64[nfactors]
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])


def rng_for(seed: int, stream: int = 0) -> np.random.Generator:
    """Philox-backed generator; ``stream`` separates independent draws."""
    return np.random.Generator(np.random.Philox(key=np.array([seed, stream], dtype=np.uint64)))


# ----------------------------------------------------------------------------
# graphs
# ----------------------------------------------------------------------------

def er_edges(n: int, m: int, seed: int) -> np.ndarray:
    """G(n, m): m distinct unordered pairs u<v drawn without replacement.

    Returns int64[m, 2] sorted by (u, v)."""
    total = n * (n - 1) // 2
    if m > total:
        raise ValueError("m exceeds the number of vertex pairs")
    rng = rng_for(seed, 1)
    k = np.sort(rng.choice(total, size=m, replace=False))
    # pair index k enumerates (0,1),(0,2)..(0,n-1),(1,2).. ; row u starts at
    # start[u] = u*n - u*(u+1)/2
    u_all = np.arange(n, dtype=np.int64)
    start = u_all * n - u_all * (u_all + 1) // 2
    u = np.searchsorted(start, k, side="right") - 1
    v = k - start[u] + u + 1
    return np.stack([u, v], axis=1).astype(np.int64)


def _resolve_refs(val: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Pointer jumping: entries with ref>=0 copy val of the entry they point
    to (which may itself point further back)."""
    val = val.copy()
    ref = ref.copy()
    pending = np.nonzero(ref >= 0)[0]
    while pending.size:
        r = ref[pending]
        nxt = ref[r]
        done = nxt < 0
        hit = pending[done]
        val[hit] = val[r[done]]
        miss = pending[~done]
        ref[hit] = -1
        ref[miss] = nxt[~done]
        pending = miss
    return val


def ba_edges(n: int, seed: int, m_per_node: int = 3) -> np.ndarray:
    """Barabasi-Albert graph with preferential attachment.

    Start from the complete graph on m_per_node+1 vertices; every later
    vertex t attaches to m_per_node distinct earlier vertices, each picked
    proportionally to degree by drawing a uniform position in the endpoint
    list of all edges created before t (duplicates are re-drawn).  Edges are
    numbered in creation order and stored as (t, target), so the rows of a
    new vertex are contiguous.

    The endpoint-list positions are drawn up front and resolved by pointer
    jumping (a position that lands on an earlier target copies that
    target), which keeps the 2M-vertex case vectorised."""
    q = m_per_node
    s0 = q + 1
    if n < s0:
        raise ValueError("n too small")
    seed_edges = [(i, j) for i in range(s0) for j in range(i + 1, s0)]
    E0 = len(seed_edges)
    E = E0 + q * (n - s0)
    src = np.empty(E, dtype=np.int64)
    dst = np.empty(E, dtype=np.int64)
    src[:E0] = [e[0] for e in seed_edges]
    dst[:E0] = [e[1] for e in seed_edges]
    k = np.arange(E0, E, dtype=np.int64)
    t = s0 + (k - E0) // q
    src[E0:] = t
    # endpoint-list length before vertex t's edges
    avail = 2 * (E0 + q * (t - s0))
    rng = rng_for(seed, 2)
    todo = np.arange(E0, E, dtype=np.int64)
    pos = np.zeros(E, dtype=np.int64)
    while True:
        pos[todo] = np.floor(rng.random(todo.size) * avail[todo - E0]).astype(np.int64)
        val = dst.copy()
        ref = np.full(E, -1, dtype=np.int64)
        p = pos[E0:]
        even = (p & 1) == 0
        idx = np.arange(E0, E)
        val[idx[even]] = src[p[even] >> 1]
        ref[idx[~even]] = p[~even] >> 1
        dst_new = _resolve_refs(val, ref)
        d3 = dst_new[E0:].reshape(-1, q)
        # duplicates within a vertex's targets: re-draw every later copy
        bad = np.zeros_like(d3, dtype=bool)
        for a in range(q):
            for b in range(a + 1, q):
                bad[:, b] |= d3[:, a] == d3[:, b]
        if not bad.any():
            dst = dst_new
            break
        todo = E0 + np.nonzero(bad.reshape(-1))[0]
    return np.stack([src, dst], axis=1)


def regular_edges(n: int, d: int, seed: int) -> np.ndarray:
    """Random simple d-regular graph (n*d even): a random pairing of the n*d
    stubs; then, while self-loops or repeated pairs remain, the stubs of the
    defective edges together with as many uniformly chosen good edges are
    shuffled and paired again.  Returns int64[n*d/2, 2], u < v, sorted."""
    if (n * d) % 2:
        raise ValueError("n*d must be even")
    if d >= n:
        raise ValueError("d must be below n")
    rng = rng_for(seed, 3)
    stubs = np.repeat(np.arange(n, dtype=np.int64), d)
    rng.shuffle(stubs)
    e = stubs.reshape(-1, 2)
    M = e.shape[0]
    for _ in range(10000):
        e.sort(axis=1)
        key = e[:, 0] * n + e[:, 1]
        order = np.argsort(key, kind="stable")
        ks = key[order]
        bad = e[:, 0] == e[:, 1]
        rep = np.zeros(M, dtype=bool)
        rep[order[1:][ks[1:] == ks[:-1]]] = True      # every later copy of a pair
        bad |= rep
        nb = int(bad.sum())
        if nb == 0:
            break
        good = np.nonzero(~bad)[0]
        extra = rng.choice(good, size=min(len(good), max(nb, 8)), replace=False)
        idx = np.concatenate([np.nonzero(bad)[0], extra])
        st = e[idx].reshape(-1).copy()
        rng.shuffle(st)
        e[idx] = st.reshape(-1, 2)
    else:
        raise RuntimeError("regular graph repair did not converge")
    order = np.lexsort((e[:, 1], e[:, 0]))
    return e[order]


def grid_edges(side: int) -> np.ndarray:
    """4-connected side x side grid, pixel p = i*side + j.  Horizontal edges
    first (row-major), then vertical edges."""
    i, j = np.meshgrid(np.arange(side), np.arange(side - 1), indexing="ij")
    p = (i * side + j).reshape(-1)
    h = np.stack([p, p + 1], axis=1)
    i, j = np.meshgrid(np.arange(side - 1), np.arange(side), indexing="ij")
    p = (i * side + j).reshape(-1)
    v = np.stack([p, p + side], axis=1)
    return np.concatenate([h, v]).astype(np.int64)


# ----------------------------------------------------------------------------
# LP relaxations
# ----------------------------------------------------------------------------

def _edge_rows(edges: np.ndarray):
    e = np.sort(edges, axis=1)
    M = e.shape[0]
    row_ptr = np.arange(0, 2 * M + 1, 2, dtype=np.int64)
    col_idx = e.reshape(-1).astype(np.int32)
    return M, row_ptr, col_idx


def vc_lp(n: int, edges: np.ndarray, weights: np.ndarray, meta=None) -> LPInstance:
    """Vertex-cover LP relaxation (Section 2): min c^T x,
    x_u + x_v >= 1 per edge, 0 <= x <= 1."""
    M, row_ptr, col_idx = _edge_rows(edges)
    return LPInstance(m=M, n=n, row_ptr=row_ptr, col_idx=col_idx, val=None,
                      b=np.ones(M), c=np.asarray(weights, dtype=np.float64).copy(),
                      u=np.ones(n), sense=np.ones(M, dtype=np.int8),
                      meta=dict(meta or {}, kind="vc", edges=edges))


def mis_lp(n: int, edges: np.ndarray, weights: np.ndarray, meta=None) -> LPInstance:
    """Independent-set LP (set packing, Appendix B) written as a minimisation:
    min -w^T x, x_u + x_v <= 1 per edge, 0 <= x <= 1."""
    M, row_ptr, col_idx = _edge_rows(edges)
    return LPInstance(m=M, n=n, row_ptr=row_ptr, col_idx=col_idx, val=None,
                      b=np.ones(M), c=-np.asarray(weights, dtype=np.float64),
                      u=np.ones(n), sense=-np.ones(M, dtype=np.int8),
                      meta=dict(meta or {}, kind="mis", edges=edges))


def mc_grid_lp(n_vertices: int, edges: np.ndarray, edge_w: np.ndarray,
               terminals: np.ndarray, meta=None) -> LPInstance:
    """Linearised multiway-cut LP (Appendix B).

    Columns: x_v^i at v*k+i (simplex block of vertex v), then z_e^i at
    n_vertices*k + e*k + i.  Per edge e=(u,v), u<v, and label i two rows
        z - x_u^i + x_v^i >= 0      and      z + x_u^i - x_v^i >= 0,
    objective 1/2 c_e per z_e^i, z in [0,1], x_v in Delta_k, terminal
    block t_i fixed at the i-th unit vector."""
    k = len(terminals)
    E = edges.shape[0]
    e = np.sort(edges, axis=1)
    nx = n_vertices * k
    n = nx + E * k
    M = 2 * E * k
    lab = np.arange(k, dtype=np.int64)
    xu = (e[:, 0:1] * k + lab).reshape(-1)           # [E*k]
    xv = (e[:, 1:2] * k + lab).reshape(-1)
    z = nx + np.arange(E * k, dtype=np.int64)
    cols = np.empty((E * k, 2, 3), dtype=np.int64)
    vals = np.empty((E * k, 2, 3), dtype=np.float64)
    cols[:, 0] = np.stack([xu, xv, z], axis=1)
    vals[:, 0] = [-1.0, 1.0, 1.0]
    cols[:, 1] = np.stack([xu, xv, z], axis=1)
    vals[:, 1] = [1.0, -1.0, 1.0]
    row_ptr = np.arange(0, 3 * M + 1, 3, dtype=np.int64)
    c = np.zeros(n)
    c[nx:] = 0.5 * np.repeat(np.asarray(edge_w, dtype=np.float64), k)
    fixed = np.full(n_vertices, -1, dtype=np.int32)
    fixed[np.asarray(terminals)] = np.arange(k, dtype=np.int32)
    return LPInstance(m=M, n=n, row_ptr=row_ptr, col_idx=cols.reshape(-1).astype(np.int32),
                      val=vals.reshape(-1), b=np.zeros(M), c=c, u=np.ones(n),
                      sense=np.ones(M, dtype=np.int8),
                      block_first_col=np.arange(n_vertices, dtype=np.int64) * k,
                      block_k=k, fixed_label=fixed,
                      meta=dict(meta or {}, kind="mc", edges=edges, edge_w=edge_w,
                                terminals=np.asarray(terminals), n_vertices=n_vertices))


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def vc_er(n: int = 1000, m: int = 5000, seed: int = 0) -> LPInstance:
    """Vertex cover on G(n, m), weights uniform[1,10]."""
    edges = er_edges(n, m, seed)
    w = rng_for(seed, 10).uniform(1.0, 10.0, n)
    return vc_lp(n, edges, w, meta=dict(graph="er", seed=seed))


def vc_ba(n: int = 2_000_000, seed: int = 0, m_per_node: int = 3) -> LPInstance:
    """Vertex cover on a Barabasi-Albert graph, weights uniform[1,10]."""
    edges = ba_edges(n, seed, m_per_node)
    w = rng_for(seed, 10).uniform(1.0, 10.0, n)
    return vc_lp(n, edges, w, meta=dict(graph="ba", seed=seed))


def mis_regular(n: int, d: int, seed: int) -> LPInstance:
    """Weighted independent set on a random d-regular graph, weights
    uniform[1,5] (n is bumped by one when n*d is odd)."""
    if (n * d) % 2:
        n += 1
    edges = regular_edges(n, d, seed)
    w = rng_for(seed, 11).uniform(1.0, 5.0, n)
    return mis_lp(n, edges, w, meta=dict(graph="regular", d=d, seed=seed))


def mc_grid(side: int = 1024, k: int = 8, seed: int = 0) -> LPInstance:
    """Multiway cut on a side x side 4-connected grid with k terminals at
    distinct random pixels; edge weight exp(-d^2), d ~ N(0,1)."""
    edges = grid_edges(side)
    rng = rng_for(seed, 12)
    d = rng.standard_normal(edges.shape[0])
    w = np.exp(-d * d)
    terminals = rng.choice(side * side, size=k, replace=False)
    return mc_grid_lp(side * side, edges, w, terminals, meta=dict(graph="grid", side=side, seed=seed))


def _rows_from_pairs(n_rows: int, row_of: np.ndarray, col_of: np.ndarray, val=None):
    """CSR from distinct (row, column) pairs, columns ascending inside a row."""
    order = np.lexsort((col_of, row_of))
    counts = np.bincount(row_of, minlength=n_rows)
    row_ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return row_ptr, col_of[order].astype(np.int32), (None if val is None else val[order])


def _set_members(n_elements: int, n_sets: int, rng, mean_size: float):
    """Set sizes 1 + Poisson(mean_size - 1) (at most n_elements), members
    uniform (duplicates inside a set merged); every element that no set
    drew joins one set chosen uniformly.  Returns (set, element) pairs."""
    sizes = np.minimum(1 + rng.poisson(mean_size - 1.0, n_sets), n_elements)
    set_id = np.repeat(np.arange(n_sets, dtype=np.int64), sizes)
    elem = rng.integers(0, n_elements, set_id.size)
    key = np.unique(set_id * n_elements + elem)
    set_id, elem = key // n_elements, key % n_elements
    covered = np.zeros(n_elements, bool)
    covered[elem] = True
    miss = np.nonzero(~covered)[0]
    set_id = np.concatenate([set_id, rng.integers(0, n_sets, miss.size)])
    elem = np.concatenate([elem, miss])
    return set_id, elem


def set_cover(n_elements: int, n_sets: int, seed: int, mean_size: float = 8.0) -> LPInstance:
    """Weighted set cover (Appendix B): one row per element, sum over the
    sets containing it >= 1; costs U[1, 10]; x in [0, 1]."""
    rng = rng_for(seed, 20)
    set_id, elem = _set_members(n_elements, n_sets, rng, mean_size)
    row_ptr, col_idx, _ = _rows_from_pairs(n_elements, elem, set_id)
    c = rng_for(seed, 21).uniform(1.0, 10.0, n_sets)
    return LPInstance(m=n_elements, n=n_sets, row_ptr=row_ptr, col_idx=col_idx, val=None,
                      b=np.ones(n_elements), c=c, u=np.ones(n_sets), sense=np.ones(n_elements, np.int8),
                      meta=dict(kind="set_cover", seed=seed, mean_size=mean_size))


def multicover(n_elements: int, n_sets: int, seed: int, mean_size: float = 8.0,
               max_weight: int = 3, max_demand: int = 4) -> LPInstance:
    """Integer covering program (Appendix C) on a set-cover pattern: entries
    U{1..max_weight}, demands U{1..max_demand} capped at the row's total
    weight (so taking every set is feasible); costs U[1, 10]."""
    rng = rng_for(seed, 22)
    set_id, elem = _set_members(n_elements, n_sets, rng, mean_size)
    w = rng.integers(1, max_weight + 1, set_id.size).astype(np.float64)
    row_ptr, col_idx, val = _rows_from_pairs(n_elements, elem, set_id, w)
    tot = np.add.reduceat(val, row_ptr[:-1]) if val.size else np.zeros(n_elements)
    b = np.minimum(rng.integers(1, max_demand + 1, n_elements).astype(np.float64), tot)
    c = rng_for(seed, 23).uniform(1.0, 10.0, n_sets)
    return LPInstance(m=n_elements, n=n_sets, row_ptr=row_ptr, col_idx=col_idx, val=val, b=b, c=c,
                      u=np.ones(n_sets), sense=np.ones(n_elements, np.int8),
                      meta=dict(kind="multicover", seed=seed))


def kcs_packing(n_sets: int, n_elements: int, k: int, seed: int, max_weight: int = 4,
                capacity=(4, 12)) -> LPInstance:
    """k-column-sparse packing (Appendix B, Bansal et al.'s setting): every
    set holds k distinct elements with integer weights U{1..max_weight};
    element capacities U{capacity}; profits U[1, 10], written as
    min -profit^T x, A x <= b, x in [0, 1]."""
    rng = rng_for(seed, 24)
    members = rng.integers(0, n_elements, (n_sets, k))
    while True:
        srt = np.sort(members, axis=1)
        dup = np.any(srt[:, 1:] == srt[:, :-1], axis=1) if k > 1 else np.zeros(n_sets, bool)
        if not dup.any():
            break
        members[dup] = rng.integers(0, n_elements, (int(dup.sum()), k))
    set_id = np.repeat(np.arange(n_sets, dtype=np.int64), k)
    elem = members.reshape(-1).astype(np.int64)
    w = rng.integers(1, max_weight + 1, set_id.size).astype(np.float64)
    row_ptr, col_idx, val = _rows_from_pairs(n_elements, elem, set_id, w)
    b = rng.integers(capacity[0], capacity[1] + 1, n_elements).astype(np.float64)
    profit = rng_for(seed, 25).uniform(1.0, 10.0, n_sets)
    return LPInstance(m=n_elements, n=n_sets, row_ptr=row_ptr, col_idx=col_idx, val=val, b=b, c=-profit,
                      u=np.ones(n_sets), sense=-np.ones(n_elements, np.int8),
                      meta=dict(kind="kcs_packing", k=k, seed=seed))


def mixed_lp(seed: int) -> LPInstance:
    """A seeded sparse LP of mixed shape: ragged rows (a few long ones), a
    column in more than 64 rows (workgroup path), an empty column, all
    three senses, finite, zero and infinite upper bounds, and matrix values
    by seed: all 1, all +-1, or general (the three ways the sweep copies
    store entries).  Costs are non-negative where the bound is infinite, so
    the penalty problem is bounded."""
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(80, 400))
    m = int(rng.integers(200, 400))
    rows = []
    for i in range(m):
        k = int(rng.integers(1, 7)) if rng.random() > 0.03 else int(rng.integers(20, 48))
        r = set(rng.choice(np.arange(1, n - 1), size=min(k, n - 2), replace=False).tolist())
        if i % 2 == 0:
            r.add(0)                     # column 0: m/2 >= 100 entries
        rows.append(np.array(sorted(r)))  # column n-1 stays empty
    row_ptr = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    col = np.concatenate(rows).astype(np.int32)
    kind = seed % 3
    if kind == 0:
        val = None
    elif kind == 1:
        val = rng.choice([-1.0, 1.0], size=len(col))
    else:
        val = rng.uniform(-2, 3, len(col))
    sense = rng.choice([-1, 0, 1], size=m).astype(np.int8)
    u = rng.uniform(0.5, 3, n)
    u[rng.choice(n, n // 8, replace=False)] = np.inf
    u[rng.choice(n, 3, replace=False)] = 0.0
    c = rng.uniform(-1, 2, n)
    c[np.isinf(u)] = np.abs(c[np.isinf(u)])
    return LPInstance(m=m, n=n, row_ptr=row_ptr, col_idx=col, val=val, b=rng.uniform(-1, 2, m),
                      c=c, u=u, sense=sense)


def map_lp(n_vars: int, k: int, ends: np.ndarray, unary: np.ndarray, pair: np.ndarray,
           evidence=None, meta=None) -> LPInstance:
    """Local-polytope LP of MAP inference on a pairwise factor graph (the
    formulation the MAP experiments solve): node marginals mu_i in the
    k-simplex (block i, columns i*k + a), factor marginals mu_e(a, b) >= 0
    (columns n_vars*k + e*k*k + a*k + b), and per factor e = (i, j) the
    equalities sum_b mu_e(a, b) = mu_i(a) and sum_a mu_e(a, b) = mu_j(b);
    minimise sum_i unary[i] . mu_i + sum_e pair[e] . mu_e.  `pair` is
    [n_factors, k, k]; `evidence` (optional, int per variable, -1 free)
    fixes observed variables."""
    nf = ends.shape[0]
    kk = k * k
    nx = n_vars * k
    n = nx + nf * kk
    m = 2 * nf * k
    first = nx + np.arange(nf, dtype=np.int64) * kk
    lab = np.arange(k, dtype=np.int64)
    # left rows (e, a): mu_i(a) then mu_e(a, 0..k-1); right rows (e, b):
    # mu_j(b) then mu_e(0..k-1, b); node columns precede factor columns
    node_l = ends[:, 0:1].astype(np.int64) * k + lab                     # [nf, k]
    node_r = ends[:, 1:2].astype(np.int64) * k + lab
    fac_l = first[:, None, None] + lab[None, :, None] * k + lab[None, None, :]   # [nf, a, b]
    fac_r = first[:, None, None] + lab[None, None, :] * k + lab[None, :, None]   # [nf, b, a]
    cols_l = np.concatenate([node_l[:, :, None], fac_l], axis=2)          # [nf, k, k+1]
    cols_r = np.concatenate([node_r[:, :, None], fac_r], axis=2)
    cols = np.stack([cols_l, cols_r], axis=1).reshape(-1, k + 1)         # rows (e, side, label)
    vals = np.ones((cols.shape[0], k + 1))
    vals[:, 0] = -1.0
    row_ptr = np.arange(0, m * (k + 1) + 1, k + 1, dtype=np.int64)
    c = np.concatenate([np.asarray(unary, np.float64).reshape(-1), np.asarray(pair, np.float64).reshape(-1)])
    fixed = np.full(n_vars, -1, np.int32) if evidence is None else np.asarray(evidence, np.int32)
    return LPInstance(m=m, n=n, row_ptr=row_ptr, col_idx=cols.reshape(-1).astype(np.int32),
                      val=vals.reshape(-1), b=np.zeros(m), c=c, u=np.ones(n), sense=np.zeros(m, np.int8),
                      block_first_col=np.arange(n_vars, dtype=np.int64) * k, block_k=k, fixed_label=fixed,
                      pair_ends=ends.astype(np.int32), pair_first=first,
                      meta=dict(meta or {}, kind="map", n_vars=n_vars))


def map_chain_window(n_vars: int, k: int, n_factors: int, seed: int, window: int = 6) -> LPInstance:
    """A factor graph shaped like a sequence-labelling task (text chunking):
    a chain over the tokens with one transition table shared by every chain
    factor (entries N(0, 1/2)), plus n_factors - (n_vars - 1) agreement
    factors between tokens 2..window apart (-w on equal labels, w ~ U[0, 1));
    unary terms N(0, 1).  n_factors = n_vars - 1 gives a plain chain."""
    rng = rng_for(seed, 26)
    chain = np.stack([np.arange(n_vars - 1), np.arange(1, n_vars)], axis=1)
    extra = max(0, n_factors - (n_vars - 1))
    if extra:
        i = rng.integers(0, n_vars, extra * 2)
        d = rng.integers(2, window + 1, extra * 2)
        ok = i + d < n_vars
        pairs = np.unique(np.stack([i[ok], i[ok] + d[ok]], axis=1), axis=0)
        pairs = pairs[rng.permutation(len(pairs))[:extra]]
        pairs = pairs[np.lexsort((pairs[:, 1], pairs[:, 0]))]
        ends = np.concatenate([chain, pairs])
    else:
        ends = chain
    unary = rng.standard_normal((n_vars, k))
    trans = 0.5 * rng.standard_normal((k, k))
    pair = np.empty((ends.shape[0], k, k))
    pair[: n_vars - 1] = trans
    if ends.shape[0] > n_vars - 1:
        w = rng.uniform(0.0, 1.0, ends.shape[0] - (n_vars - 1))
        pair[n_vars - 1:] = -w[:, None, None] * np.eye(k)[None]
    return map_lp(n_vars, k, ends, unary, pair, meta=dict(graph="chain_window", seed=seed, window=window))


def serving_trace(n_requests: int, rate: float, seed: int,
                  min_edges: float = 1e3, max_edges: float = 1e6):
    """Poisson arrivals (exponential gaps) of mixed requests.

    Returns a list of dicts {t_arrival, kind, edges, seed}: kind uniform over
    vc / mis / mc, edge count log-uniform in [min_edges, max_edges]."""
    rng = rng_for(seed, 13)
    gaps = rng.exponential(1.0 / rate, n_requests)
    t = np.cumsum(gaps)
    kinds = rng.integers(0, 3, n_requests)
    m = np.exp(rng.uniform(np.log(min_edges), np.log(max_edges), n_requests))
    names = ["vc", "mis", "mc"]
    return [dict(t_arrival=float(t[i]), kind=names[kinds[i]], edges=int(m[i]),
                 seed=int(seed * 1_000_003 + i)) for i in range(n_requests)]


def serving_compact(req: dict) -> dict:
    """The graph of one serving request, compactly: VC on G(m/5, m),
    independent set on a 6-regular graph with n = m/3, or multiway cut
    (k = 8) on a grid of about m edges (side sqrt(m/2)); weights drawn as in
    the corresponding workloads."""
    m = req["edges"]
    sd = req["seed"]
    kind = req["kind"]
    if kind == "vc":
        n = max(10, m // 5)
        mm = min(m, n * (n - 1) // 2)
        e = er_edges(n, mm, sd).astype(np.int32)
        return dict(kind=kind, n=n, edges=e, w=rng_for(sd, 10).uniform(1.0, 10.0, n))
    if kind == "mis":
        n = max(10, m // 3)
        if (n * 6) % 2:
            n += 1
        e = regular_edges(n, 6, sd).astype(np.int32)
        return dict(kind=kind, n=n, edges=e, w=rng_for(sd, 11).uniform(1.0, 5.0, n))
    side = max(4, int(round(np.sqrt(m / 2.0))))
    rng = rng_for(sd, 12)
    E = 2 * side * (side - 1)
    d = rng.standard_normal(E)
    terminals = rng.choice(side * side, size=8, replace=False)
    return dict(kind="mc", side=side, w=np.exp(-d * d), terminals=terminals)


def serving_expand(c: dict) -> LPInstance:
    """The LP relaxation of a compact serving request."""
    if c["kind"] == "vc":
        return vc_lp(c["n"], c["edges"].astype(np.int64), c["w"])
    if c["kind"] == "mis":
        return mis_lp(c["n"], c["edges"].astype(np.int64), c["w"])
    side = c["side"]
    return mc_grid_lp(side * side, grid_edges(side), c["w"], c["terminals"], meta=dict(side=side))


def serving_instance(req: dict) -> LPInstance:
    return serving_expand(serving_compact(req))
