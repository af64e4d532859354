"""Reordering by subdomains (paper Sec. 2), oracle side.

The paper labels the variables subdomain by subdomain with the interface
variables last, giving the 2x2 block system of eq. (resystem).  It uses a
vertex-based partitioner (METIS); the workloads here name their own
partitions instead:

* geometric: on a box grid, part = lexicographic index (x fastest) of
  floor(i_d * P_d / N_d) over the axes d;
* region growing: s seeds drawn from SplitMix64, multi-source FIFO BFS over
  the symmetrised pattern, first visitor wins.

Interface rule: vertex v of part i is an interface vertex iff some w != v in
another part has a stored entry A[v,w] or A[w,v].  Permutation: interiors of
part 0, 1, ..., then interfaces of part 0, 1, ...; ascending original index
inside each group.
"""
from __future__ import annotations

from collections import deque
import numpy as np
import scipy.sparse as sp

MASK64 = (1 << 64) - 1


def splitmix64(seed: int):
    """SplitMix64 generator (Steele, Lea and Flood, OOPSLA 2014)."""
    state = seed & MASK64
    while True:
        state = (state + 0x9E3779B97F4A7C15) & MASK64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        yield z ^ (z >> 31)


def geometric_labels(dims, parts) -> np.ndarray:
    """Box-grid split into prod(parts) boxes; label = px + Px*(py + Py*pz)."""
    dims = [int(d) for d in dims]
    parts = [int(p) for p in parts]
    n = int(np.prod(dims))
    v = np.arange(n, dtype=np.int64)
    label = np.zeros(n, dtype=np.int64)
    mult = 1
    for N, P in zip(dims, parts):
        i = v % N
        v = v // N
        label += mult * ((i * P) // N)
        mult *= P
    return label.astype(np.int32)


def symmetric_neighbours(A: sp.csr_matrix):
    """Adjacency lists of pattern(A) + pattern(A^T) without the diagonal, ascending."""
    P = sp.csr_matrix((np.ones(A.nnz), A.indices, A.indptr), shape=A.shape)
    P = (P + P.T).tocsr()
    P.setdiag(0)
    P.eliminate_zeros()
    P.sort_indices()
    return P.indptr, P.indices


def region_growing_labels(A: sp.csr_matrix, nparts: int, seed: int) -> np.ndarray:
    n = A.shape[0]
    gen = splitmix64(seed)
    seeds = []
    seen = set()
    while len(seeds) < min(nparts, n):
        v = next(gen) % n
        if v not in seen:
            seen.add(v)
            seeds.append(v)
    ptr, nbr = symmetric_neighbours(A)
    label = np.full(n, -1, dtype=np.int64)

    def grow(queue):
        while queue:
            v = queue.popleft()
            lv = label[v]
            for w in nbr[ptr[v]:ptr[v + 1]]:
                if label[w] < 0:
                    label[w] = lv
                    queue.append(w)

    queue = deque()
    for l, v in enumerate(seeds):
        label[v] = l
        queue.append(v)
    grow(queue)
    # vertices no seed reached: each unlabelled vertex, in ascending order,
    # starts a new region with the next label
    nxt = len(seeds)
    for v in range(n):
        if label[v] < 0:
            label[v] = nxt
            nxt += 1
            grow(deque([v]))
    return label.astype(np.int32)


def interface_mask(A: sp.csr_matrix, label: np.ndarray) -> np.ndarray:
    ptr, nbr = symmetric_neighbours(A)
    n = A.shape[0]
    rows = np.repeat(np.arange(n), np.diff(ptr))
    cut = label[rows] != label[nbr]
    mask = np.zeros(n, dtype=bool)
    mask[rows[cut]] = True
    return mask


def reorder(A: sp.csr_matrix, label: np.ndarray):
    """Return (perm, p, q, int_ptr, if_ptr) where perm[new] = old.

    int_ptr[i]..int_ptr[i+1] are the new positions of part i's interiors,
    p + if_ptr[i]..p + if_ptr[i+1] those of its interface vertices.
    """
    nparts = int(label.max()) + 1 if label.size else 0
    iface = interface_mask(A, label)
    interiors = [np.flatnonzero((label == i) & ~iface) for i in range(nparts)]
    faces = [np.flatnonzero((label == i) & iface) for i in range(nparts)]
    perm = np.concatenate(interiors + faces).astype(np.int64)
    int_ptr = np.concatenate([[0], np.cumsum([len(x) for x in interiors])]).astype(np.int64)
    if_ptr = np.concatenate([[0], np.cumsum([len(x) for x in faces])]).astype(np.int64)
    p = int(int_ptr[-1])
    q = int(if_ptr[-1])
    return perm, p, q, int_ptr, if_ptr
