"""The quality measures reported for the edge-preservation workload, pinned
against the oracle's PSNR and hand-computed cases, and the workload's
generator (deterministic, piecewise constant, edge-dense)."""
import math

import numpy as np

import oracle
from paper_2311_03010_amd import metrics, synth


def test_psnr_matches_oracle_and_closed_form():
    rng = np.random.Generator(np.random.PCG64(7))
    a = rng.uniform(0, 255, size=(37, 53))
    b = a + rng.standard_normal(a.shape)
    assert abs(metrics.psnr(a, b) - oracle.psnr(a, b)) < 1e-12
    # constant offset d: RMS error d, PSNR = 20 log10(255 / d)
    assert abs(metrics.psnr(a, a + 3.0) - 20 * math.log10(255 / 3.0)) < 1e-12
    assert metrics.psnr(a, a) == float("inf")


def test_edge_map_of_a_step():
    # vertical step of height 100 between columns 9 and 10: the Sobel x
    # response is 4 * 100 on the two columns next to the step, 0 elsewhere
    u = np.zeros((12, 20))
    u[:, 10:] = 100.0
    e = metrics.edge_map(u, threshold=60.0)
    cols = np.flatnonzero(e.any(axis=0))
    assert list(cols) == [9, 10] and e[:, 9].all() and e[:, 10].all()
    assert not metrics.edge_map(u, threshold=400.0).any()
    assert metrics.edge_error(u, u) == 0.0 and metrics.edge_recall(u, u) == 1.0
    assert metrics.edge_recall(u, np.zeros_like(u)) == 0.0
    assert abs(metrics.edge_error(u, np.zeros_like(u)) - 24 / 240) < 1e-15


def test_edge_workload_is_deterministic_and_edge_dense():
    p = synth.edge_workload(H=128, n_levels=4)
    q = synth.edge_workload(H=128, n_levels=4)
    np.testing.assert_array_equal(p.g_delta, q.g_delta)
    assert p.psf.shape == (23, 23) and abs(p.psf.sum() - 1.0) < 1e-12
    # piecewise constant with many regions and a large share of edge pixels
    assert len(np.unique(p.u_true)) > 20
    assert metrics.edge_map(p.u_true).mean() > 0.1
    assert abs(p.delta - 1.0) < 0.05
