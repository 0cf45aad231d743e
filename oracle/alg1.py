"""Algorithm 1 (overlapping low-dose point sampling), integer exact.

Oracle code (test infrastructure).  Given, for each plan j, its low-dose volume
V_j (a set of voxel indices) and desired point count N_LD,j, Algorithm 1 of
Sec. 2.C.2 builds one shared point set P and the per-plan subsets p_j:

  order plans by decreasing density w_j = N_LD,j / |V_j|
  V_u <- {}, p_u <- {}
  for each plan j in that order:
      p~   <- a random selection of w_j |V_u| points of p_u       (thinning)
      p_in <- p~ intersected with V_j
      p_out<- a random selection of w_j |V_j \\ V_u| voxels of V_j \\ V_u
      p_j  <- p_in  union  p_out
      p_u  <- p~    union  p_out
      V_u  <- V_u   union  V_j
  P = union of all p_j

Readings of what the paper leaves open (each also listed in the design notes):
  * counts are fixed sizes, round-half-to-even of w_j * |X| computed in IEEE
    double as (N_LD,j / |V_j|) * |X|, clamped to |X|;
  * w_j = min(1, N_LD,j / |V_j|); a plan with an empty V_j (or N_LD,j = 0)
    gets no points and is skipped without changing V_u or p_u;
  * equal densities keep ascending plan order;
  * "randomly select K of X" = the K members of X with the smallest key
    h(seed, step, voxel), ties broken by the smaller voxel index, where step is
    2 * rank for the thinning and 2 * rank + 1 for p_out (rank = position in
    the density order) and h is built from the SplitMix64 finaliser.

The random source is a counter-based hash so the device implementation can
draw exactly the same numbers from its own code.
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


def splitmix64(z: int) -> int:
    """SplitMix64 output function (Steele, Lea and Flood, OOPSLA 2014)."""
    z = (z + GOLDEN) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def key(seed: int, step: int, voxel: int) -> int:
    """h(seed, step, voxel) = sm(sm(sm(seed) ^ step) ^ voxel), sm = splitmix64."""
    return splitmix64(splitmix64(splitmix64(seed & MASK64) ^ (step & MASK64)) ^ (voxel & MASK64))


def keys_array(seed: int, step: int, voxels: np.ndarray) -> np.ndarray:
    """The same h as `key`, for an array of voxel indices (uint64 wraps mod 2^64)."""
    def sm(z):
        z = z + np.uint64(GOLDEN)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))
    base = np.uint64(splitmix64(splitmix64(seed & MASK64) ^ (step & MASK64)))
    with np.errstate(over="ignore"):
        return sm(np.asarray(voxels, np.uint64) ^ base)


def select_smallest(members, count: int, seed: int, step: int):
    """The `count` members with the smallest (key, voxel) pairs, as a set."""
    if count <= 0:
        return set()
    vox = np.fromiter(members, dtype=np.int64, count=len(members))
    order = np.lexsort((vox, keys_array(seed, step, vox)))
    return set(vox[order[:count]].tolist())


def target_count(n_ld: int, vol_size: int, set_size: int) -> int:
    """round-half-even((N_LD / |V_j|) * |X|) in double, clamped to [0, |X|]."""
    omega = min(1.0, float(n_ld) / float(vol_size))
    return int(min(set_size, np.rint(omega * float(set_size))))


def density_order(n_ld, vol_sizes):
    """Plan indices by decreasing density, ties by ascending plan index."""
    k = len(vol_sizes)
    dens = [min(1.0, float(n_ld[j]) / float(vol_sizes[j])) if vol_sizes[j] and n_ld[j] > 0
            else -1.0 for j in range(k)]
    return sorted(range(k), key=lambda j: (-dens[j], j)), dens


def select_ld_points(volumes, n_ld, seed: int):
    """Algorithm 1.  volumes: list of k sets (or k x n bool); returns (P, p).

    P: sorted list of voxel indices; p: list of k sets (p_j subset of P).
    """
    if isinstance(volumes, np.ndarray):
        vols = [set(np.nonzero(row)[0].tolist()) for row in volumes]
    else:
        vols = [set(v) for v in volumes]
    k = len(vols)
    n_ld = [int(x) for x in np.broadcast_to(np.asarray(n_ld), (k,))]
    order, dens = density_order(n_ld, [len(v) for v in vols])
    V_u, p_u = set(), set()
    p = [set() for _ in range(k)]
    for rank, j in enumerate(order):
        if dens[j] < 0:
            continue
        Vj = vols[j]
        thin = target_count(n_ld[j], len(Vj), len(V_u))
        p_tilde = select_smallest(p_u, min(thin, len(p_u)), seed, 2 * rank)
        p_in = p_tilde & Vj
        new = Vj - V_u
        p_out = select_smallest(new, target_count(n_ld[j], len(Vj), len(new)), seed, 2 * rank + 1)
        p[j] = p_in | p_out
        p_u = p_tilde | p_out
        V_u = V_u | Vj
    P = sorted(set().union(*p)) if k else []
    return P, p


def masks_over(P, p):
    """k x |P| bool matrix: entry (j, i) is True when P[i] is in p_j."""
    index = {v: i for i, v in enumerate(P)}
    out = np.zeros((len(p), len(P)), bool)
    for j, pj in enumerate(p):
        for v in pj:
            out[j, index[v]] = True
    return out
