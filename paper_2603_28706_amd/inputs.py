"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

Only random draws and evaluation of analytic input fields at mesh node
coordinates live here; none of the method's arithmetic does.  Vector layouts
follow the C-ABI: a spatial velocity block is d components, each over the Q2
nodes in lexicographic order (x fastest); a space-time vector is one spatial
block (velocity, then d+1 P1disc coefficients per cell) per Gauss-Radau node.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def sizes(n, k_time: int = 1):
    d = len(n)
    nn = int(np.prod([2 * m + 1 for m in n]))
    nc = int(np.prod(n))
    nv = d * nn
    ns = nv + (d + 1) * nc
    return dict(dim=d, num_nodes=nn, num_cells=nc, nv=nv, ns=ns, nt=k_time + 1,
                nst=(k_time + 1) * ns)


def uniform(seed: int, size: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """i.i.d. U[lo, hi] values."""
    return rng(seed).uniform(lo, hi, size)


def node_coordinates(n, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    """Coordinates of the Q2 nodes (spacing h/2), lexicographic with x fastest."""
    d = len(n)
    axes = [lo[k] + np.arange(2 * n[k] + 1) * (hi[k] - lo[k]) / (2 * n[k]) for k in range(d)]
    grids = np.meshgrid(*axes, indexing="ij")
    return [g.ravel(order="F") for g in grids]


def sin_series_velocity(n, seed: int, t_nodes, n_modes: int = 8, max_wave: int = 8,
                        noise: float = 0.01, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    """Smooth velocity at every time node t_mu:
    u_c(x, t_mu) = (1 + t_mu) * sum_m a_{c,m} prod_k sin(pi k_{m,k} x_k) + U[-noise, noise],
    with k_{m,k} ~ U{1..max_wave}, a ~ U[-1,1].  The modes vanish on the boundary
    of the unit box; the time variation across a slab of length tau is O(tau).
    Returns the concatenation over time nodes of d*num_nodes values."""
    g = rng(seed)
    d = len(n)
    waves = g.integers(1, max_wave + 1, size=(n_modes, d))
    amps = g.uniform(-1.0, 1.0, size=(d, n_modes))
    X = node_coordinates(n, lo, hi)
    base = []
    for c in range(d):
        f = np.zeros(X[0].size)
        for m in range(n_modes):
            term = np.full(X[0].size, amps[c, m])
            for k in range(d):
                term = term * np.sin(np.pi * waves[m, k] * X[k])
            f += term
        base.append(f)
    out = []
    for t in t_nodes:
        for c in range(d):
            out.append((1.0 + t) * base[c] + g.uniform(-noise, noise, X[0].size))
    return np.concatenate(out)


def truncation_masks(n, seed: int, choices=(1, 2, 3)):
    """Per-cell keep-masks over the 3^d local Q2 nodes.  Interior cells keep all
    nodes; a cell touching the boundary drops j of its boundary nodes (j drawn
    from `choices`, nodes chosen at random among the boundary ones), which gives
    the uneven patch sizes of the batched-smoother workload."""
    g = rng(seed)
    d = len(n)
    nb = 3 ** d
    nc = int(np.prod(n))
    masks = np.ones((nc, nb), dtype=np.uint8)
    for c in range(nc):
        ci = [(c // int(np.prod(n[:k]))) % n[k] for k in range(d)]
        bnodes = []
        for a in range(nb):
            ak = [(a // 3 ** k) % 3 for k in range(d)]
            on_b = any((ci[k] == 0 and ak[k] == 0) or (ci[k] == n[k] - 1 and ak[k] == 2)
                       for k in range(d))
            if on_b:
                bnodes.append(a)
        if bnodes:
            j = min(int(g.choice(choices)), len(bnodes))
            drop = g.choice(bnodes, size=j, replace=False)
            masks[c, drop] = 0
    return masks
