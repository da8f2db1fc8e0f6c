"""The host regenerator of the device-drawn Cholesky vectors (CPU only):
Philox4x32-10 against the published known-answer vectors of its authors'
Random123 distribution, and the properties of the drawn blocks."""
import numpy as np

from paper_2006_05226_amd.synth import device_cholesky_block, philox4x32_10

# Philox4x32-10 known-answer vectors (Random123 kat_vectors): counter, key -> output
KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


def test_philox_known_answers():
    for ctr, key, want in KAT:
        got = philox4x32_10(*[np.array([c]) for c in ctr], *key)
        assert tuple(int(g[0]) for g in got) == want


def test_philox_vectorised_equals_elementwise():
    c0 = np.arange(1000, dtype=np.uint64) * np.uint64(2654435761) % np.uint64(1 << 32)
    c1 = np.arange(1000, dtype=np.uint64) % np.uint64(37)
    x = philox4x32_10(c0, c1, 0, 0, 12345, 678)
    for i in (0, 17, 999):
        y = philox4x32_10(np.array([c0[i]]), np.array([c1[i]]), 0, 0, 12345, 678)
        assert all(int(a[i]) == int(b[0]) for a, b in zip(x, y))


def test_device_block_symmetry_scale_and_distribution():
    O, V, seed = 7, 23, 99
    n = O + V
    full = device_cholesky_block(np.arange(30), np.arange(n), np.arange(n), O, V, seed)
    assert np.array_equal(full, full.transpose(0, 2, 1))        # L[K][p][q] = L[K][q][p]
    sub = device_cholesky_block([3, 11], [5, 20, 1], [29, 0], O, V, seed)
    assert np.array_equal(sub, full[[3, 11]][:, [5, 20, 1]][:, :, [29, 0]])
    z = full / (0.5 / np.sqrt(O * V) * np.exp(-np.arange(30) / 10.0))[:, None, None]
    iu = np.triu_indices(n)
    zz = z[:, iu[0], iu[1]].ravel()
    assert abs(zz.mean()) < 0.05 and abs(zz.std() - 1.0) < 0.05   # standard normal draws
    other = device_cholesky_block([0], [0], [1], O, V, seed + 1)
    assert other[0, 0, 0] != full[0, 0, 1]
