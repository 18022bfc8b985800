"""Host side of the seeded input generator (CPU only)."""
import numpy as np

import ssegen


def setup_module(module):
    ssegen.build_host()


def test_philox_known_answers():
    # Known-answer vectors published with Philox4x32-10 (Random123 distribution).
    kat = [
        ([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
        ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
        ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
         [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
    ]
    for ctr, key, want in kat:
        assert list(ssegen.philox4x32_10(ctr, key)) == want


def test_normal_moments_and_exactness():
    x = np.array([ssegen.normal(7, i, ssegen.S_DH) for i in range(20000)])
    assert abs(x.mean()) < 0.03 and abs(x.std() - 1.0) < 0.03
    assert np.all(np.abs(x) < 6.0)
    # every value is a multiple of 2^-32 (the twelve-uniform sum is exact)
    assert np.all(np.ldexp(x, 32) == np.round(np.ldexp(x, 32)))


def test_neigh_table():
    n = ssegen.neigh(1912, 64, 6)
    for a in range(64):
        row = n[a]
        assert len(set(row.tolist())) == 6 and a not in row
        assert row.min() >= 0 and row.max() < 64
    assert np.array_equal(n, ssegen.neigh(1912, 64, 6))
    assert not np.array_equal(n, ssegen.neigh(1913, 64, 6))


def test_blocks_antihermitian_and_consistent():
    G = ssegen.G(5, 1, 2, 5, 3, 4)
    assert np.array_equal(G, -np.conj(np.swapaxes(G, -1, -2)))
    # block list generation agrees with the full tensor
    blocks = np.array([[1, 4, 2], [0, 0, 0], [1, 2, 1]])
    Gb = ssegen.G_blocks(5, 1, 5, 3, 4, blocks)
    for t, (k, e, a) in enumerate(blocks):
        assert np.array_equal(Gb[t], G[k, e, a])
    D = ssegen.D(5, 0, 2, 3, 3, 2)
    assert np.array_equal(D, -np.conj(np.swapaxes(D, -1, -2)))
    # the two components differ
    assert not np.array_equal(ssegen.G(5, 0, 2, 5, 3, 4), G)


def test_scaled_blocks_span_decades():
    G = ssegen.G(3, 0, 1, 400, 8, 2, scaled=True)
    norms = np.linalg.norm(G.reshape(-1, 4), axis=1)
    assert norms.min() < 1e-4 and norms.max() > 10.0
    assert np.array_equal(G, -np.conj(np.swapaxes(G, -1, -2)))


def test_perturbation_moves_one_percent_and_keeps_symmetry():
    G = ssegen.G(9, 0, 1, 6, 5, 4).reshape(-1, 4, 4).copy()
    G0 = G.copy()
    flat = np.arange(G.shape[0])
    ssegen.perturb(77, 0, ssegen.S_PERT_G, G, flat)
    rel = np.linalg.norm((G - G0).reshape(len(G), -1), axis=1) / np.linalg.norm(
        G0.reshape(len(G), -1), axis=1)
    assert np.allclose(rel, 0.01, rtol=1e-12)
    assert np.allclose(G, -np.conj(np.swapaxes(G, -1, -2)), atol=1e-15)
    G1 = G0.copy()
    ssegen.perturb(77, 1, ssegen.S_PERT_G, G1, flat)
    assert not np.array_equal(G1, G)  # iterations draw fresh noise
