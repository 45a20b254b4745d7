"""Seeded synthetic graph Laplacians and sample sets.

This module builds inputs only: graphs, their Laplacians in CSR form, sample
node sets and label vectors.  It holds none of the Krylov method's arithmetic,
so both the GPU path and the CPU reference may consume what it produces.

Laplacian convention (Sec. 2.1, generalised Laplacian): L is symmetric with
L_ij < 0 exactly on edges, 0 off the edge set, and a real diagonal.  The
graphs here produce the weighted combinatorial Laplacian L = D - W with
D_ii = sum_j W_ij, which is positive semi-definite with L 1 = 0.

CSR layout handed to the library: full symmetric storage (both triangles),
the diagonal entry present in every row, column indices sorted inside each
row, int64 row pointers, int32 column indices, float64 values.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class CSRLaplacian:
    n: int
    row_ptr: np.ndarray   # int64, n+1
    col_idx: np.ndarray   # int32, nnz
    vals: np.ndarray      # float64, nnz
    name: str = ""
    unit_weights: bool = False

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.vals, self.col_idx.astype(np.int64), self.row_ptr),
                             shape=(self.n, self.n))

    def max_degree(self) -> int:
        return int(np.max(np.diff(self.row_ptr))) - 1


def laplacian_from_edges(n: int, ei, ej, w, diag_extra=None, name="",
                         unit_weights=False) -> CSRLaplacian:
    """L = D - W (+ diag(diag_extra)) from an undirected edge list.

    Each undirected edge must appear once (i != j); weights must be > 0.
    """
    ei = np.asarray(ei, dtype=np.int64)
    ej = np.asarray(ej, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    if ei.size and (np.any(ei == ej) or np.any(w <= 0)):
        raise ValueError("self loops or non-positive weights in edge list")
    rows = np.concatenate([ei, ej, np.arange(n)])
    cols = np.concatenate([ej, ei, np.arange(n)])
    deg = np.bincount(ei, weights=w, minlength=n) + np.bincount(ej, weights=w, minlength=n)
    diag = deg if diag_extra is None else deg + np.asarray(diag_extra, dtype=np.float64)
    vals = np.concatenate([-w, -w, diag])
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    A.sort_indices()
    if A.nnz != 2 * ei.size + n:
        raise ValueError("duplicate edges in edge list")
    return CSRLaplacian(n=n, row_ptr=A.indptr.astype(np.int64),
                        col_idx=A.indices.astype(np.int32), vals=A.data.astype(np.float64),
                        name=name, unit_weights=unit_weights)


def path(n: int) -> CSRLaplacian:
    i = np.arange(n - 1)
    return laplacian_from_edges(n, i, i + 1, np.ones(n - 1), name=f"path{n}", unit_weights=True)


def _grid_edges(shape):
    """Edges of a rectangular grid graph, node id = row-major index.

    Edges are listed axis by axis (axis 0 first), each in row-major order of
    the lower endpoint; weights drawn for a grid follow this order.
    """
    idx = np.arange(int(np.prod(shape))).reshape(shape)
    ei, ej = [], []
    for ax in range(len(shape)):
        lo = [slice(None)] * len(shape)
        hi = [slice(None)] * len(shape)
        lo[ax] = slice(0, shape[ax] - 1)
        hi[ax] = slice(1, shape[ax])
        ei.append(idx[tuple(lo)].ravel())
        ej.append(idx[tuple(hi)].ravel())
    return np.concatenate(ei), np.concatenate(ej)


def grid(shape, weights: str = "unit", seed: int = 0, lo: float = 0.5, hi: float = 1.5) -> CSRLaplacian:
    """2-D / 3-D grid graph (4- or 6-neighbour), unit or U[lo,hi] weights."""
    shape = tuple(int(x) for x in shape)
    n = int(np.prod(shape))
    ei, ej = _grid_edges(shape)
    if weights == "unit":
        w = np.ones(ei.size)
    elif weights == "uniform":
        w = np.random.default_rng(seed).uniform(lo, hi, size=ei.size)
    else:
        raise ValueError(weights)
    name = "grid" + "x".join(map(str, shape)) + ("" if weights == "unit" else f"_w{seed}")
    return laplacian_from_edges(n, ei, ej, w, name=name, unit_weights=(weights == "unit"))


def rgg_knn(n: int, k: int = 8, seed: int = 1) -> CSRLaplacian:
    """Random geometric graph: n points uniform in the unit square, exact
    Euclidean k-NN symmetrised by union, Gaussian weights exp(-d^2/sigma^2)
    with sigma the median (over nodes) of the distance to the k-th neighbour.
    """
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    pts = rng.random((n, 2))
    tree = cKDTree(pts)
    d, nb = tree.query(pts, k=k + 1)
    d, nb = d[:, 1:], nb[:, 1:]
    sigma = float(np.median(d[:, -1]))
    a = np.repeat(np.arange(n), k)
    b = nb.ravel()
    lo_, hi_ = np.minimum(a, b), np.maximum(a, b)
    key = np.unique(lo_ * n + hi_)
    ei, ej = key // n, key % n
    dist2 = np.sum((pts[ei] - pts[ej]) ** 2, axis=1)
    w = np.exp(-dist2 / sigma ** 2)
    L = laplacian_from_edges(n, ei, ej, w, name=f"rgg{n}_k{k}_s{seed}")
    L.sigma = sigma  # type: ignore[attr-defined]
    return L


def barabasi_albert(n: int, m_edges: int = 4, seed: int = 0) -> CSRLaplacian:
    """Barabasi-Albert preferential attachment, unit weights.

    Seed graph: the complete graph on m_edges+1 nodes.  Each later node links
    to m_edges distinct earlier nodes drawn with probability proportional to
    their current degree (sampling from the list of edge endpoints).
    """
    rng = np.random.default_rng(seed)
    m0 = m_edges + 1
    n_e = m0 * (m0 - 1) // 2 + m_edges * (n - m0)
    ei = np.empty(n_e, dtype=np.int64)
    ej = np.empty(n_e, dtype=np.int64)
    pool = np.empty(2 * n_e, dtype=np.int64)
    e = 0
    for a in range(m0):
        for b in range(a + 1, m0):
            ei[e], ej[e] = a, b
            pool[2 * e], pool[2 * e + 1] = a, b
            e += 1
    plen = 2 * e
    # draw candidate positions in bulk; redraw only on collisions
    for v in range(m0, n):
        chosen = set()
        while len(chosen) < m_edges:
            r = rng.integers(0, plen, size=m_edges)
            for x in r:
                t = int(pool[x])
                if t not in chosen:
                    chosen.add(t)
                    if len(chosen) == m_edges:
                        break
        for t in sorted(chosen):
            ei[e], ej[e] = t, v
            pool[plen], pool[plen + 1] = t, v
            plen += 2
            e += 1
    return laplacian_from_edges(n, ei, ej, np.ones(n_e), name=f"ba{n}_m{m_edges}_s{seed}",
                                unit_weights=True)


def random_weighted(n: int, p: float, seed: int = 0, lo=0.5, hi=1.5, connect=True) -> CSRLaplacian:
    """Small Erdos-Renyi graph with U[lo,hi] weights (distinct eigenvalues
    almost surely); a path through all nodes is added when `connect`."""
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.size) < p
    if connect:
        keep |= (ju == iu + 1)
    ei, ej = iu[keep], ju[keep]
    w = rng.uniform(lo, hi, size=ei.size)
    return laplacian_from_edges(n, ei, ej, w, name=f"er{n}_p{p}_s{seed}")


def disjoint_union(a: CSRLaplacian, b: CSRLaplacian) -> CSRLaplacian:
    A = sp.block_diag([a.to_scipy(), b.to_scipy()], format="csr")
    A.sort_indices()
    return CSRLaplacian(n=A.shape[0], row_ptr=A.indptr.astype(np.int64),
                        col_idx=A.indices.astype(np.int32), vals=A.data.astype(np.float64),
                        name=f"{a.name}+{b.name}")


def permute(L: CSRLaplacian, perm) -> CSRLaplacian:
    """Relabel nodes: new node i is old node perm[i]."""
    perm = np.asarray(perm)
    A = L.to_scipy()[perm][:, perm].tocsr()
    A.sort_indices()
    return CSRLaplacian(n=L.n, row_ptr=A.indptr.astype(np.int64), col_idx=A.indices.astype(np.int32),
                        vals=A.data.astype(np.float64), name=L.name + "_perm", unit_weights=L.unit_weights)


def normalized_laplacian(L: CSRLaplacian) -> CSRLaplacian:
    """Normalised Laplacian I - D^(-1/2) A D^(-1/2) of the graph whose
    combinatorial Laplacian is L = D - A (the operator of the paper's
    experiments, Sec. 8; the paper does not define it, the symmetric
    normalisation is taken).  Its off-diagonal entries stay <= 0, but rows do
    not sum to zero: the library needs GK_ASSUME_PSD for it."""
    A = L.to_scipy()
    d = np.asarray(A.diagonal()).ravel()
    if np.any(d <= 0):
        raise ValueError("isolated node: the normalised Laplacian needs degree > 0")
    adj = sp.diags(d) - A
    r = sp.diags(1.0 / np.sqrt(d))
    N = (sp.eye(L.n) - r @ adj @ r).tocsr()
    N.sort_indices()
    return CSRLaplacian(n=L.n, row_ptr=N.indptr.astype(np.int64), col_idx=N.indices.astype(np.int32),
                        vals=N.data.astype(np.float64), name=L.name + "_normalized")


def planar_radius_standin(n: int = 900, n_edges: int = 7325, seed: int = 0) -> CSRLaplacian:
    """Synthetic stand-in for the paper's 900-point planar graph (Sec. 8.2;
    its point set is not available): n points uniform in the unit square,
    unit-weight edges between the n_edges closest pairs (a radius graph whose
    radius is the n_edges-th smallest pairwise distance), combinatorial
    Laplacian."""
    from scipy.spatial.distance import pdist

    pts = np.random.default_rng(seed).random((n, 2))
    d = pdist(pts)
    order = np.argsort(d, kind="stable")[:n_edges]
    iu, ju = np.triu_indices(n, 1)
    ei, ej = iu[order], ju[order]
    o = np.lexsort((ej, ei))
    return laplacian_from_edges(n, ei[o], ej[o], np.ones(n_edges), name=f"planar{n}_e{n_edges}_s{seed}",
                                unit_weights=True)


def samples(n: int, s: int, seed: int = 0) -> np.ndarray:
    """s distinct sample nodes drawn uniformly without replacement, in draw order."""
    return np.random.default_rng(seed).choice(n, s, replace=False).astype(np.int64)


def labels(s: int, seed: int = 0) -> np.ndarray:
    """Labels y ~ N(0,1) on the s samples."""
    return np.random.default_rng(seed + 7919).standard_normal(s)


# ---------------------------------------------------------------- workloads
# Named workloads used by tests and the benchmark (sizes of the paper-derived
# configurations; the kernel parameters are those of the diffusion and
# variational spline kernels of Sec. 2.4).

def serving_pool(n_graphs: int = 8, n_min: int = 10_000, n_max: int = 500_000):
    """Resident graph pool of the serving workload: symmetrised 8-NN random
    geometric graphs with log-spaced orders N_i = n_min (n_max/n_min)^(i/7),
    seeds 100 + i."""
    out = []
    for i in range(n_graphs):
        n = int(round(n_min * (n_max / n_min) ** (i / max(n_graphs - 1, 1))))
        out.append(rgg_knn(n, 8, seed=100 + i))
    return out


def serving_requests(n_req: int, graph_sizes, seed: int = 0, s_range=(4, 128), m: int = 30,
                     gamma: float = 1e-3):
    """Request stream of the serving workload: graph uniform over the pool,
    s uniform in s_range, diffusion t ~ U[0.1, 2] or spline eps ~ U[0.001, 0.1]
    with k = 2 (each with probability 1/2), labels y ~ N(0, 1)."""
    rng = np.random.default_rng(seed)
    reqs = []
    for r in range(n_req):
        gi = int(rng.integers(len(graph_sizes)))
        s = int(rng.integers(s_range[0], s_range[1] + 1))
        if rng.random() < 0.5:
            phi = dict(kind="diffusion", t=float(rng.uniform(0.1, 2.0)))
        else:
            phi = dict(kind="spline", eps=float(rng.uniform(0.001, 0.1)), k=2.0)
        smp = rng.choice(graph_sizes[gi], s, replace=False).astype(np.int64)
        y = rng.standard_normal(s)
        reqs.append(dict(graph=gi, samples=smp, y=y, phi=phi, m=m, gamma=gamma))
    return reqs


def workload(name: str, seed: int = 0):
    """Return (L, samples, phi dict, m) for a named workload."""
    if name == "grid32_diffusion":
        L = grid((32, 32))
        return L, samples(L.n, 8, seed), dict(kind="diffusion", t=1.0), 20
    if name == "rgg100k_spline":
        L = rgg_knn(100_000, 8, seed=1)
        return L, samples(L.n, 64, seed), dict(kind="spline", eps=0.01, k=2.0), 40
    if name == "ba1m_diffusion":
        L = barabasi_albert(1_000_000, 4, seed=0)
        return L, samples(L.n, 256, seed), dict(kind="diffusion", t=0.5), 30
    if name == "grid128c_spline":
        L = grid((128, 128, 128), weights="uniform", seed=0)
        return L, samples(L.n, 512, seed), dict(kind="spline", eps=0.05, k=1.0), 30
    raise KeyError(name)
