"""The seeded input generators: exactness of the link exponential and the recipe."""
import numpy as np

import synth


def test_expi_matches_eigendecomposition():
    g = synth.rng(5)
    h = synth.random_hermitian_traceless((4000,), g)
    for eps in (1e-4, 0.3, 1.0, 3.0):
        q = eps * h
        w, v = np.linalg.eigh(q)
        ref = (v * np.exp(1j * w)[..., None, :]) @ np.conj(np.swapaxes(v, -1, -2))
        assert np.abs(synth.expi_hermitian(q) - ref).max() < 1e-13
        assert np.abs(synth.expi_hermitian(-q) - np.conj(np.swapaxes(ref, -1, -2))).max() < 1e-13


def test_random_links_su3_and_chunk_invariant():
    dims = (4, 4, 4, 8)
    u = synth.random_links(dims, 0.3, 1000, chunk_sites=100)
    u2 = synth.random_links(dims, 0.3, 1000, chunk_sites=1 << 30)
    assert np.array_equal(u, u2)
    m = u.reshape(-1, 3, 3)
    assert np.abs(m @ np.conj(np.swapaxes(m, -1, -2)) - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(m) - 1).max() < 1e-14
    # third column = conj(col0 x col1) for SU(3) (what SU(3) reconstruction relies on)
    c = np.conj(np.cross(m[:, :, 0], m[:, :, 1]))
    assert np.abs(c - m[:, :, 2]).max() < 1e-14


def test_hermitian_recipe_normalisation():
    h = synth.random_hermitian_traceless((200000,), synth.rng(9))
    assert np.abs(np.trace(h, axis1=-2, axis2=-1)).max() < 1e-14
    # entrywise Gaussian recipe: E tr H^2 = 8
    assert abs(np.mean(np.einsum("nij,nji->n", h, h).real) - 8.0) < 0.1


def test_haar_su3_and_sources():
    om = synth.haar_su3((1000,), synth.rng(3))
    assert np.abs(om @ np.conj(np.swapaxes(om, -1, -2)) - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(om) - 1).max() < 1e-14
    dims = (4, 4, 4, 6)
    z = synth.z2_source(dims, 1)
    assert set(np.unique(z.real)) == {-1.0, 1.0} and np.all(z.imag == 0)
    p = synth.point_source(dims, 2, 1)
    assert p.sum() == 1 and p[0, 0, 0, 0, 2, 1] == 1
    assert np.array_equal(synth.gaussian_source(dims, 4), synth.gaussian_source(dims, 4))
