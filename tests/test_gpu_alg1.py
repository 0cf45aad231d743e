"""GPU parity of Algorithm 1 (bit-exact) and of the low-dose band."""
import sys

import numpy as np
import pytest

from synth import cases
from oracle import alg1 as oalg1
from oracle import dose as odose

pytestmark = pytest.mark.gpu

ladmm = pytest.importorskip("paper_2509_08602_amd.ladmm")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    return ladmm.Context(0)


def device_alg1(ctx, vols, n_ld, seed):
    P, words, _ = ladmm.select_ld_points(ctx, vols, n_ld, seed)
    return P, words


def check_against_oracle(ctx, vols, n_ld, seed):
    P, masks = device_alg1(ctx, vols, n_ld, seed)
    Pref, pref = oalg1.select_ld_points(vols, n_ld, seed)
    assert P.tolist() == Pref, "P differs"
    ref_masks = oalg1.masks_over(Pref, pref)
    got = cases.unpack_bits(masks, len(Pref)) if len(Pref) else np.zeros((vols.shape[0], 0), bool)
    assert np.array_equal(got, ref_masks), "masks differ"
    # words past |P| are zero
    nw = (len(Pref) + 63) // 64
    assert not masks[:, nw:].any()


@pytest.mark.parametrize("k,n_vox,seed,kind", [
    (1, 100, 0, "shells"), (5, 1000, 1, "shells"), (9, 26919, 2, "shells"),
    (30, 3001, 3, "random"), (81, 20000, 4, "shells"),
])
def test_alg1_bit_exact(ctx, k, n_vox, seed, kind):
    say("alg1", k, n_vox, seed, kind)
    vols = cases.random_volumes(k, n_vox, seed, kind=kind)
    n_ld = np.random.default_rng(seed).integers(0, 600, k)
    check_against_oracle(ctx, vols, n_ld, seed * 7919 + 1)


def test_alg1_degenerate_cases(ctx):
    say("alg1 degenerate")
    v = np.zeros((5, 777), bool)
    v[1, :40] = True
    v[2, 100:400] = True
    v[3, 100:400] = True
    v[4, 700:777] = True
    check_against_oracle(ctx, v, [10, 60, 30, 0, 500], 0)   # empty, N>=|V|, N=0, ragged tail
    check_against_oracle(ctx, np.ones((4, 64), bool), 16, 5)     # identical volumes
    check_against_oracle(ctx, np.ones((1, 1), bool), 1, 9)       # one voxel
    P, masks = device_alg1(ctx, np.zeros((0, 10), bool), [], 0)  # no plans
    assert len(P) == 0


def test_ld_band_matches_oracle_dose(ctx):
    """Band bits from the device FP64 dose equal the oracle's, except possibly
    at voxels whose dose lies within rounding of a band edge."""
    say("ld band c0")
    case = cases.make_case(0)
    w = cases.config_weights(0)
    dc = ladmm.Case.from_case(ctx, case, "f64")
    b = ladmm.Batch(dc, w, opts=ladmm.Options(rho0=1000.0, w0_bot=cases.W0_BOT))
    b.iterate(300)
    t = b.results()["t"]
    cand = case.ld_candidates
    phi = case.kernel.dose_rate(cand)
    d_ld = 0.5 * case.prescription_mean
    delta = 0.1 * case.prescription_mean
    n_vox = phi.shape[0]
    got = b.ld_band(phi, d_ld, delta)
    d = odose.dose(phi, t.T)
    ref = odose.ld_band(d, d_ld, delta)
    diff = got != ref
    assert ref.sum() > 0
    if diff.any():
        dd = d.T[diff]
        edge = np.minimum(np.abs(dd - d_ld), np.abs(dd - d_ld - delta))
        assert np.all(edge <= 1e-12 * (d_ld + delta)), edge.max()
    # the band feeds Algorithm 1 directly
    check_against_oracle(ctx, got, 200, 17)
