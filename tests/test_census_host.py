"""Host-side mode census of the mixture posterior's k! symmetric modes."""

import itertools
import math

import numpy as np

from paper_0905_2441_amd.samplers import mode_census


def test_census_recovers_relabelled_modes():
    mu = np.array([-3.0, 0.0, 3.0, 6.0])
    perms = list(itertools.permutations(range(4)))
    rng = np.random.default_rng(3)
    counts = rng.integers(1, 50, size=len(perms))
    cols = []
    for p, c in zip(perms, counts):
        cols.append(mu[list(p)][:, None] + 0.05 * rng.standard_normal((4, c)))
    theta = np.hstack(cols)
    census = mode_census(theta)
    assert len(census) == math.factorial(4) == 24
    for p, c in zip(perms, counts):
        ranks = tuple(int(r) for r in np.argsort(np.argsort(mu[list(p)])))
        assert abs(census[ranks] - c / counts.sum()) < 1e-12
    assert abs(sum(census.values()) - 1.0) < 1e-12


def test_census_uses_weights():
    theta = np.array([[0.0, 1.0, 2.0], [1.0, 0.0, 3.0]])      # k = 2, three particles
    census = mode_census(theta, W=np.array([0.5, 0.2, 0.3]))
    assert abs(census[(0, 1)] - 0.8) < 1e-15 and abs(census[(1, 0)] - 0.2) < 1e-15


def test_traversal_time_counts_iterations_to_all_modes():
    from paper_0905_2441_amd.samplers import traversal_time
    mu = np.array([-3.0, 0.0, 3.0, 6.0])
    perms = list(itertools.permutations(range(4)))
    rows = [mu[list(p)] for p in perms[:23]] * 3 + [mu[list(perms[23])]]
    assert traversal_time(np.array(rows)) == 70
    assert traversal_time(np.array(rows[:-1])) is None
