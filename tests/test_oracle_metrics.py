"""Oracle pins for the clinical metrics of Sec. 2.A (coverage, selectivity,
gradient index, beam-on time), against values worked out by hand."""
import numpy as np
import pytest

from oracle import metrics as om


def test_metrics_of_a_hand_built_dose():
    # ten voxels, the first four in the target (prescription 10 Gy); one shot
    # column whose dose rates are the doses, shot time 1
    doses = np.array([12.0, 10.0, 9.0, 15.0, 11.0, 4.0, 6.0, 5.0, 0.0, 20.0])
    tgt = np.array([0, 0, 0, 0, -1, -1, -1, -1, -1, -1])
    m = om.clinical_metrics(doses[:, None], np.ones((1, 1)), tgt, [10.0], 10.0, 1, 1, 1)[0]
    # covered: 12, 10, 15 -> 3 of 4; >= 10 Gy: 12, 10, 15, 11, 20 -> 5;
    # >= 5 Gy: 12, 10, 9, 15, 11, 6, 5, 20 -> 8
    assert m[0] == pytest.approx(3 / 4)
    assert m[1] == pytest.approx(3 / 5)
    assert m[2] == pytest.approx(8 / 5)
    assert m[3] == pytest.approx(1.0)


def test_beam_on_time_is_the_longest_sector_per_isocentre():
    # 2 isocentres x 2 sectors x 3 collimators
    t = np.array([1, 2, 3,   4, 0, 0,      # iso 0: sectors 6 and 4 -> 6
                  0, 0, 1,   2, 2, 2.5])   # iso 1: sectors 1 and 6.5 -> 6.5
    assert om.beam_on_time(t[:, None], 2, 2, 3)[0] == pytest.approx(12.5)
    # twice the shot times: twice the beam-on time, doses scale with them
    assert om.beam_on_time(2 * t[:, None], 2, 2, 3)[0] == pytest.approx(25.0)


def test_two_targets_use_their_own_prescriptions():
    doses = np.array([18.0, 21.0, 14.0, 16.0, 22.0, 3.0])
    tgt = np.array([0, 0, 1, 1, -1, -1])
    m = om.clinical_metrics(doses[:, None], np.ones((1, 1)), tgt, [20.0, 15.0], 15.0, 1, 1, 1)[0]
    # covered: 21 (>= 20 in target 0) and 16 (>= 15 in target 1) -> 2 of 4
    # >= 15 Gy: 18, 21, 16, 22 -> 4; >= 7.5 Gy: 18, 21, 14, 16, 22 -> 5
    assert m[0] == pytest.approx(0.5)
    assert m[1] == pytest.approx(0.5)
    assert m[2] == pytest.approx(5 / 4)


def test_no_dose_gives_undefined_ratios():
    m = om.clinical_metrics(np.zeros((4, 1)), np.ones((1, 1)), np.array([0, 0, -1, -1]), [1.0],
                            1.0, 1, 1, 1)[0]
    assert m[0] == 0.0 and np.isnan(m[1]) and np.isnan(m[2])
