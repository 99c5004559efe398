"""Pins of the oracle's detection statistics (CPU only).

SDE = (SR_max - mean) / std over the period grid (population std), the signal
detection efficiency of the box-least-squares statistic the paper cites;
peaks are taken largest first with neighbourhood and harmonic suppression.
"""
import math

import numpy as np
import pytest

import oracle
import synth


def test_closed_form_small_case():
    # mean 2, population std sqrt(3), SDE (5 - 2)/sqrt(3) = sqrt(3)
    d = oracle.detect([1, 1, 1, 5], [1.0, 2.0, 3.0, 4.0], max_peaks=4,
                      window=0.01, threshold=1.7)
    assert d["mean"] == 2.0
    assert abs(d["std"] - math.sqrt(3)) < 1e-15
    assert abs(d["sde"] - math.sqrt(3)) < 1e-15 and d["candidate"]
    # P=4 suppresses its half P=2; of the tie SR=1 at P=1 and P=3 the smaller
    # index wins, and P=1 suppresses its triple P=3: two peaks
    assert d["peak_index"].tolist() == [3, 0]
    assert d["peak_sr"].tolist() == [5.0, 1.0]
    assert abs(d["peak_sde"][1] - (1 - 2) / math.sqrt(3)) < 1e-15


def test_matches_numpy_statistics():
    rng = np.random.default_rng(4)
    sr = rng.gamma(2.0, 1e-3, 5000)
    per = np.exp(np.linspace(np.log(0.2), np.log(10), 5000))
    d = oracle.detect(sr, per, max_peaks=0)
    assert abs(d["mean"] - np.mean(sr)) < 1e-14
    assert abs(d["std"] - np.std(sr)) / np.std(sr) < 1e-12
    assert abs(d["sde"] - (sr.max() - np.mean(sr)) / np.std(sr)) < 1e-10


def test_constant_and_zero_periodograms():
    per = np.linspace(1, 2, 10)
    # 0.25 is exact in binary, so the mean is exact and the deviation 0
    d = oracle.detect(np.full(10, 0.25), per, max_peaks=3, threshold=0.5)
    assert d["std"] == 0.0 and d["sde"] == 0.0 and not d["candidate"]
    assert d["peak_index"].tolist()[0] == 0
    d0 = oracle.detect(np.zeros(10), per, max_peaks=3)
    assert d0["peak_index"].size == 0


def test_harmonic_and_neighbour_suppression():
    per = np.exp(np.linspace(np.log(0.2), np.log(10), 20001))
    sr = np.full(per.size, 1e-3)

    def bump(p0, h):
        i = int(np.argmin(np.abs(per - p0)))
        sr[i - 3:i + 4] += h * np.array([.2, .5, .8, 1., .8, .5, .2])
        return i
    i1 = bump(1.3, 10.0)
    i2 = bump(2.6, 8.0)        # the 2x harmonic of the first peak
    i3 = bump(1.7, 6.0)        # unrelated
    i4 = bump(0.65, 5.0)       # the 1/2 harmonic
    d = oracle.detect(sr, per, max_peaks=4, window=0.01)
    pk = d["peak_index"].tolist()
    assert pk[0] == i1
    assert pk[1] == i3
    assert i2 not in pk and i4 not in pk
    # neighbours of the first peak (same bump) never reappear
    assert all(abs(per[p] / per[i1] - 1) > 0.01 for p in pk[1:])


@pytest.mark.parametrize("a,c", [(3.0, 0.0), (1.0, 0.25), (0.1, -0.001)])
def test_sde_affine_invariance(a, c):
    rng = np.random.default_rng(5)
    sr = rng.gamma(2.0, 1e-2, 3000)
    per = np.exp(np.linspace(np.log(0.3), np.log(5), 3000))
    d1 = oracle.detect(sr, per, max_peaks=3)
    d2 = oracle.detect(a * sr + c, per, max_peaks=3)
    assert abs(d1["sde"] - d2["sde"]) < 1e-9
    assert d1["peak_index"].tolist() == d2["peak_index"].tolist()


def test_crafted_case_crowds_one_slice():
    """The first crafted detection case is what it claims: all 16 peaks
    (the 24 raised values, window too small to suppress) sit at indices
    3 mod 256, one thread slice of a 256-wide workgroup."""
    sr, per, mp, win = synth.detection_periodograms()[0]
    o = oracle.detect(np.asarray(sr, np.float32).astype(np.float64), per,
                      max_peaks=mp, window=win)
    assert o["peak_index"].size == 16
    assert np.all(o["peak_index"] % 256 == 3)
    # Largest first among the raised values.
    raised = np.sort(np.asarray(sr, np.float32)[3 + 256 * np.arange(24)])
    assert np.array_equal(o["peak_sr"], raised[::-1][:16].astype(np.float64))
