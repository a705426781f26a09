"""Marker geometries drawn by the seeded input module (no method arithmetic)."""
import numpy as np
import pytest

from synthetic import icosphere_spacing, icosphere_unit, shell_problem


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_icosphere_counts_and_regularity(level):
    v = icosphere_unit(level)
    assert len(v) == 10 * 4 ** level + 2                       # V = 10 * 4^l + 2 (Euler: V - E + F = 2)
    assert np.allclose(np.linalg.norm(v, axis=1), 1.0, atol=1e-14)
    assert np.abs(v.mean(axis=0)).max() < 1e-12               # centrally symmetric point set
    assert len(np.unique(np.round(v, 12), axis=0)) == len(v)  # no duplicate vertices
    d = np.sqrt(((v[:, None, :] - v[None, :, :]) ** 2).sum(axis=2))
    np.fill_diagonal(d, np.inf)
    nn = d.min(axis=1)
    assert nn.min() > 0.8 * nn.mean()                          # near-uniform spacing
    assert abs(nn.mean() - icosphere_spacing(level)) < 1e-14


def test_icosahedron_edge_length():
    # the 12 vertices of the regular icosahedron: edge / circumradius = 4 / sqrt(10 + 2 sqrt 5)
    assert abs(icosphere_spacing(0) - 4.0 / np.sqrt(10.0 + 2.0 * np.sqrt(5.0))) < 1e-14


@pytest.mark.parametrize("filled", [False, True])
def test_shell_problem_spacing(filled):
    p = shell_problem(3, 32, 2, filled=filled)
    R = p.meta["radius_h"] * p.h
    rel = (p.R - p.centres[0] + 0.5) % 1.0 - 0.5               # minimum image around the centre
    r = np.linalg.norm(rel, axis=1)
    assert np.abs(r[:162] - R).max() < 1e-12
    assert r.max() <= R + 1e-12
    d = np.sqrt(((rel[:, None, :] - rel[None, :, :]) ** 2).sum(axis=2))
    np.fill_diagonal(d, np.inf)
    assert abs(d[:162, :162].min(axis=1).mean() / p.h - 2.0) < 1e-9
    assert (p.nmarkers > 162) == filled


def test_sedimentation_problem_shapes():
    from synthetic import sedimentation_problem
    prob, F, T = sedimentation_problem(0)
    assert prob.steady and prob.n == 128 and prob.nbodies == 16 and prob.nmarkers == 16 * 110
    assert F.shape == (16, 3) and np.all(F[:, 2] == -1.0) and not np.any(F[:, :2]) and not np.any(T)
    # surface gap of at least 4h between spheres (periodic distance)
    c = prob.centres
    dc = c[:, None, :] - c[None, :, :]
    dc -= np.round(dc)
    dist = np.sqrt((dc ** 2).sum(-1)) + np.eye(16) * 10
    assert dist.min() >= 2 * 6 * prob.h + 4 * prob.h - 1e-12
