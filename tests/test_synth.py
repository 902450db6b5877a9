"""The seeded input generator: SU(3) links, moments, reproducibility."""
import numpy as np

from paper_1612_06556_amd import synth


def test_su3_properties_and_moments():
    U = synth.su3_field((8, 8, 8, 8), 1001)
    I3 = np.eye(3)
    UU = U @ np.conj(np.swapaxes(U, -1, -2))
    assert np.abs(UU - I3).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14
    # near-unit field: <Re tr U>/3 about 0.94 for eps = 0.3
    m = np.trace(U, axis1=-2, axis2=-1).real.mean() / 3
    assert 0.93 < m < 0.95


def test_reproducible_and_chunk_invariant(monkeypatch):
    a = synth.su3_field((4, 4, 4, 8), 5)
    monkeypatch.setattr(synth, "_CHUNK_SITES", 37)
    b = synth.su3_field((4, 4, 4, 8), 5)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, synth.su3_field((4, 4, 4, 8), 6))


def test_spinor_moments_and_point_sources():
    s = synth.gaussian_spinor((8, 8, 8, 8), 3)
    assert abs(np.mean(np.abs(s) ** 2) - 1.0) < 0.01
    b = synth.point_sources((4, 4, 4, 4))
    assert b.shape == (12, 256, 4, 3)
    assert np.array_equal(b.reshape(12, -1)[:, :12], np.eye(12))
