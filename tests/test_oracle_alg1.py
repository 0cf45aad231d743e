"""Pins of the oracle's Algorithm 1 (overlapping low-dose point sampling)."""
import os

import numpy as np
import pytest

from synth import cases
from oracle import alg1

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_reference_vectors():
    lines = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64_vectors.txt"))
             if l.strip() and not l.startswith("#")]
    for row in lines:
        state, outs = int(row[0]), [int(x) for x in row[1:]]
        got = [alg1.splitmix64((state + i * alg1.GOLDEN) & alg1.MASK64) for i in range(len(outs))]
        assert got == outs


def test_vectorised_key_matches_scalar_key():
    vox = np.array([0, 1, 2, 77, 2 ** 31 - 1, 2 ** 40 + 5], np.int64)
    for seed, step in ((0, 0), (99, 7), (2 ** 63 + 1, 12345)):
        ka = alg1.keys_array(seed, step, vox)
        assert [int(x) for x in ka] == [alg1.key(seed, step, int(v)) for v in vox]


def _check_invariants(vols, n_ld, P, p):
    k = vols.shape[0]
    assert P == sorted(set(P))
    assert set(P) == set().union(*p)
    for j in range(k):
        assert p[j] <= set(np.nonzero(vols[j])[0].tolist())


@pytest.mark.parametrize("seed", range(6))
def test_invariants_random_volumes(seed):
    vols = cases.random_volumes(7, 3000, seed)
    n_ld = np.random.default_rng(seed).integers(50, 400, 7)
    P, p = alg1.select_ld_points(vols, n_ld, seed=seed)
    _check_invariants(vols, n_ld, P, p)
    # reuse: the shared set is smaller than the sum of the per-plan sets
    assert len(P) < sum(len(x) for x in p)


def test_identical_volumes_share_one_point_set():
    v = np.zeros((5, 2000), bool)
    v[:, 300:1300] = True
    P, p = alg1.select_ld_points(v, 250, seed=3)
    assert all(x == p[0] for x in p)
    assert len(P) == 250 == len(p[0])


def test_disjoint_volumes_take_exact_counts():
    v = np.zeros((3, 3000), bool)
    v[0, :1000] = True
    v[1, 1000:1500] = True
    v[2, 1500:3000] = True
    n_ld = [100, 333, 7]
    P, p = alg1.select_ld_points(v, n_ld, seed=11)
    # no overlap: p_in is empty and p_out has round(w |V|) = N_LD points
    assert [len(x) for x in p] == n_ld
    assert len(P) == sum(n_ld)


def test_degenerate_cases():
    v = np.zeros((4, 500), bool)
    v[1, :40] = True           # N_LD >= |V|: every voxel is a point
    v[2, 100:400] = True
    v[3, 100:400] = True
    P, p = alg1.select_ld_points(v, [10, 60, 30, 0], seed=0)
    assert p[0] == set()                       # empty volume
    assert p[3] == set()                       # N_LD = 0
    assert p[1] == set(range(40))
    assert len(p[2]) == 30
    P0, p0 = alg1.select_ld_points(np.zeros((0, 10), bool), [], seed=0)
    assert P0 == [] and p0 == []


def test_nested_thinning_when_volumes_are_nested():
    """Nested volumes with equal density reduce to the 'union' construction:
    each plan's points are the union points inside its own volume."""
    v = np.zeros((3, 4000), bool)
    v[0, :1000] = True
    v[1, :2000] = True
    v[2, :4000] = True
    n_ld = [100, 200, 400]          # equal densities 0.1
    P, p = alg1.select_ld_points(v, n_ld, seed=5)
    assert p[0] <= p[1] <= p[2]
    assert set(P) == p[2]
    for j in range(3):
        assert p[j] == set(P) & set(np.nonzero(v[j])[0].tolist())


def test_selection_is_smallest_keys():
    members = set(range(0, 200, 3))
    got = alg1.select_smallest(members, 10, seed=42, step=3)
    ranked = sorted(members, key=lambda x: (alg1.key(42, 3, x), x))
    assert got == set(ranked[:10])


@pytest.mark.slow
def test_relative_std_bound():
    """Eq. after Alg. 1: std(|p_j|) / (w_j |V_j|) < 1 / sqrt(w_j |V_j|)."""
    k, n_vox, N_LD = 6, 6000, 300
    vols = cases.random_volumes(k, n_vox, 123)
    sizes = vols.sum(axis=1)
    counts = []
    for s in range(300):
        _, p = alg1.select_ld_points(vols, N_LD, seed=1000 + s)
        counts.append([len(x) for x in p])
    counts = np.array(counts, np.float64)
    want = np.minimum(N_LD, sizes).astype(np.float64)
    rel_std = counts.std(axis=0) / want
    bound = 1.0 / np.sqrt(want)
    assert np.all(rel_std < bound)
    mean_ratio = counts.mean(axis=0) / want
    assert np.all(np.abs(mean_ratio - 1.0) < 3.0 * bound / np.sqrt(300) + 2.0 / want)
