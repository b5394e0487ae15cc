"""Host metrics of the injection-recovery harness and its input generator.

Pins: counts and rates of hand-built cases worked out on paper; the ROC
against its definition evaluated threshold by threshold (brute force); the
area under it against the Mann-Whitney identity (AUC = P(score of a
positive > score of a negative) + P(equal) / 2, over all pairs); the
relative errors and the T0 epoch shift on cases with known answers.
"""
import itertools
import math

import numpy as np

from paper_2607_00348_amd import injection as inj
from paper_2607_00348_amd import synth


def test_confusion_precision_recall_by_hand():
    labels = [1, 1, 1, 0, 0, 0, 0]
    flags = [1, 0, 1, 1, 0, 0, 0]
    c = inj.confusion(labels, flags)
    assert c == {"tp": 2, "fp": 1, "tn": 3, "fn": 1}
    p, r = inj.precision_recall(c)
    assert p == 2 / 3 and r == 2 / 3
    p, r = inj.precision_recall({"tp": 0, "fp": 0, "tn": 4, "fn": 0})
    assert math.isnan(p) and math.isnan(r)


def test_detection_thresholds_inclusive():
    f = inj.detected([7.0, 6.999, 7.0, 12.0], [5.0, 9.0, 4.999, 5.0])
    assert f.tolist() == [True, False, False, True]


def _roc_brute(scores, labels):
    thr = sorted(set(scores), reverse=True)
    npos = sum(labels)
    nneg = len(labels) - npos
    pts = [(0.0, 0.0)]
    for h in thr:
        tp = sum(1 for s, l in zip(scores, labels) if l and s >= h)
        fp = sum(1 for s, l in zip(scores, labels) if not l and s >= h)
        pts.append((fp / nneg, tp / npos))
    return pts, thr


def test_roc_matches_its_definition():
    g = np.random.Generator(np.random.PCG64(3))
    for trial in range(20):
        n = int(g.integers(2, 40))
        scores = g.integers(0, 8, n).astype(float).tolist()     # many ties
        labels = g.integers(0, 2, n).astype(bool).tolist()
        if not any(labels) or all(labels):
            continue
        fpr, tpr, thr = inj.roc(scores, labels)
        pts, bthr = _roc_brute(scores, labels)
        assert list(zip(fpr.tolist(), tpr.tolist())) == pts
        assert thr[0] == math.inf and thr[1:].tolist() == bthr
        assert fpr[-1] == 1.0 and tpr[-1] == 1.0


def test_auc_is_the_mann_whitney_statistic():
    g = np.random.Generator(np.random.PCG64(4))
    for trial in range(20):
        n = int(g.integers(4, 30))
        scores = g.integers(0, 6, n).astype(float)
        labels = np.zeros(n, dtype=bool)
        labels[g.permutation(n)[: n // 2]] = True
        pos, neg = scores[labels], scores[~labels]
        u = sum(1.0 if a > b else 0.5 if a == b else 0.0 for a, b in itertools.product(pos, neg))
        fpr, tpr, _ = inj.roc(scores, labels)
        assert abs(inj.auc(fpr, tpr) - u / (len(pos) * len(neg))) < 1e-12
    assert inj.auc(*inj.roc([3, 2, 1, 0], [1, 1, 0, 0])[:2]) == 1.0
    assert inj.auc(*inj.roc([0, 1, 2, 3], [1, 1, 0, 0])[:2]) == 0.0


def test_relative_errors_by_hand():
    assert inj.are_ratio([2.0], [1.0]).tolist() == [0.5]
    assert inj.are_ratio([1.0], [2.0]).tolist() == [0.5]
    assert inj.are_ratio([-3e-4], [1e-4]).tolist() == [1.0]        # negative depth counts as zero
    assert inj.are_ratio([0.0], [0.0]).tolist() == [0.0]
    assert np.all(inj.are_ratio(np.linspace(0.1, 9, 50), 3.0) < 1.0)


def test_t0_error_shifts_by_whole_periods_inside_the_baseline():
    # T0_e = 1, P = 10, baseline [0, 100]: epochs 1, 11, ..., 91
    assert abs(inj.are_t0([51.5], [1.0], [10.0], 0.0, 100.0)[0] - 0.05) < 1e-15
    assert abs(inj.are_t0([-3.0], [1.0], [10.0], 0.0, 100.0)[0] - 0.4) < 1e-15    # epoch 1, not -9
    assert abs(inj.are_t0([105.0], [1.0], [10.0], 0.0, 100.0)[0] - 1.4) < 1e-15   # epoch 91, not 101
    assert abs(inj.are_t0([3.0], [1001.0], [10.0], 0.0, 100.0)[0] - 0.2) < 1e-12  # reference far outside
    # no epoch inside the baseline: the nearest over all epochs
    assert abs(inj.are_t0([4.0], [20.0], [50.0], 0.0, 10.0)[0] - 0.32) < 1e-15


def test_period_match_aliases():
    pe = np.full(6, 7.0)
    pr = np.array([7.05, 3.5, 14.0, 21.0, 7.0 / 3.0, 10.5])
    assert inj.period_match(pr, pe).tolist() == [True, True, True, True, True, False]
    assert not inj.period_match([7.2], [7.0])[0]


def test_summarize_counts():
    truths = [None, None, {"period": 5.0, "t14": 0.1, "depth": 1e-4, "t0": 1.0},
              {"period": 2.0, "t14": 0.08, "depth": 2e-4, "t0": 0.5}]
    recs = [{"sde": 8.0, "snr": 6.0, "period": 3.1, "duration": 0.1, "depth": 1e-4, "t0": 2.0},
            {"sde": 5.0, "snr": 9.0, "period": 9.0, "duration": 0.1, "depth": 1e-4, "t0": 2.0},
            {"sde": 20.0, "snr": 30.0, "period": 5.0, "duration": 0.1, "depth": 1e-4, "t0": 11.0},
            {"sde": 6.0, "snr": 30.0, "period": 4.0, "duration": 0.08, "depth": 2e-4, "t0": 0.5}]
    s = inj.summarize(recs, truths, 0.0, 100.0)
    assert (s["tp"], s["fp"], s["tn"], s["fn"]) == (1, 1, 1, 1)
    assert s["precision"] == 0.5 and s["recall"] == 0.5
    assert s["recall_period_match"] == 0.5
    assert s["are_period_matched"] == {"P": 0.0, "D": 0.0, "Dp": 0.0, "T0": 0.0}
    assert abs(s["are_all_positives"]["P"] - 0.25) < 1e-15          # (0 + |4-2|/4) / 2
    assert s["roc_auc_sde"] == 0.75


def test_injection_curves():
    n = 10
    cs = [synth.injection_curve(i, n, seed=3, days=30.0) for i in range(n)]
    assert sum(c["meta"]["transit"] is not None for c in cs) == 5
    for c in cs:
        assert len(c["t"]) == 1440 and c["t"][1] - c["t"][0] == 30.0 / 1440.0
        tr = c["meta"]["transit"]
        if tr is not None:
            assert 0.5 <= tr["period"] <= 14.0 and 0.0 <= tr["t0"] < tr["period"]
            assert 0.003 ** 2 <= tr["depth"] <= 0.012 ** 2 / (1 - 0.6 / 3 - 0.4 / 6)
    a = synth.injection_curve(4, n, seed=3, days=30.0)
    assert np.array_equal(a["y"], cs[4]["y"])
