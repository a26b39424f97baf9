"""Host logic of the differentiable eigenvalue wrapper (no device needed)."""
import numpy as np
import pytest

pytest.importorskip("torch")
from paper_1402_6297_amd import autograd  # noqa: E402


def test_clusters_split_on_relative_gap():
    om = np.array([1.0, 1.0 + 1e-12, 1.5, 2.0, 2.0 * (1 + 5e-9), 2.0 * (1 + 1e-8) + 1e-6])
    assert autograd.clusters(om, 1e-8) == [[0, 1], [2], [3, 4], [5]]


def test_equal_weights_in_a_cluster_pass_unchanged():
    om = np.array([1.0, 1.0, 3.0])
    w = np.array([0.25, 0.25, -1.0])
    assert np.array_equal(autograd.cluster_weights(om, w, 1e-8), w)


def test_unequal_weights_in_a_cluster_are_averaged_with_a_warning():
    om = np.array([1.0, 1.0 + 1e-13, 3.0])
    with pytest.warns(RuntimeWarning, match="degenerate"):
        w = autograd.cluster_weights(om, np.array([1.0, 0.0, 2.0]), 1e-8)
    assert np.allclose(w, [0.5, 0.5, 2.0])


def test_cut_inside_a_cluster_is_detected():
    om = np.array([1.0, 2.0, 2.0 * (1 + 1e-12), 3.0])
    assert autograd.cut_in_cluster(om, 2, 1e-8)
    assert not autograd.cut_in_cluster(om, 1, 1e-8)
    assert not autograd.cut_in_cluster(om, 3, 1e-8)
    assert not autograd.cut_in_cluster(om, 4, 1e-8)
