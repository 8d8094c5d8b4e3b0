"""Set scores of the composition study (host arithmetic only)."""
import pytest

pytest.importorskip("torch")
from paper_2207_11662_amd.composition import set_metrics  # noqa: E402


def test_set_metrics_values():
    m = set_metrics([1, 2, 3, 4], [3, 4, 5])
    assert m["jaccard"] == pytest.approx(2 / 5)
    assert m["precision"] == pytest.approx(2 / 4)
    assert m["recall"] == pytest.approx(2 / 3)
    assert m["f1"] == pytest.approx(2 * (1 / 2) * (2 / 3) / (1 / 2 + 2 / 3))
    assert (m["pred"], m["true"]) == (4, 3)


def test_set_metrics_edges():
    assert set_metrics([], [])["jaccard"] == 1.0
    m = set_metrics([], [1])
    assert m["recall"] == 0.0 and m["precision"] == 0.0 and m["f1"] == 0.0
    m = set_metrics([7, 7, 8], [8, 7])                  # duplicates count once
    assert m["jaccard"] == 1.0 and m["f1"] == 1.0
    assert set_metrics([1], [2])["jaccard"] == 0.0
