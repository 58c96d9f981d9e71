"""The seeded input generators: reproducible, S^z = 0, chains move by exchanges only."""
import numpy as np

from paper_1611_09467_amd import workloads as wl


def test_peps_reproducible_and_shapes():
    a = wl.make_peps(4, 5, 3, seed=7)
    b = wl.make_peps(4, 5, 3, seed=7)
    flat = wl.pack_peps(a)
    assert np.array_equal(flat, wl.pack_peps(b))
    assert flat.size == sum(wl.site_sizes(4, 5, 3))
    back = wl.unpack_peps(flat, 4, 5, 3)
    for i in range(4):
        for j in range(5):
            assert back[i][j].shape == (2,) + wl.site_dims(4, 5, 3, i, j)
            assert np.array_equal(back[i][j], a[i][j])
    assert a[0][0].shape == (2, 1, 3, 1, 3) and a[3][4].shape == (2, 3, 1, 3, 1)


def test_bias_is_identity_like():
    a = wl.make_peps(3, 3, 2, seed=1)
    b = wl.make_peps(3, 3, 2, seed=1, bias=0.1)
    diff = b[1][1] - a[1][1]
    want = np.zeros_like(diff)
    for x in range(2):
        for y in range(2):
            want[:, x, x, y, y] = 0.1
    np.testing.assert_allclose(diff, want, atol=1e-15)


def test_sz0_configs():
    S = wl.random_sz0_configs(4, 4, 100, 3)
    assert S.dtype == np.uint8 and S.shape == (100, 16)
    assert np.all(S.sum(axis=1) == 8)
    assert np.array_equal(S, wl.random_sz0_configs(4, 4, 100, 3))


def test_chains_move_by_nn_exchanges():
    N, M = 6, 6
    S = wl.chain_configs(N, M, 8, 16, 5)
    assert S.shape == (128, 36) and np.all(S.sum(axis=1) == 18)
    bonds = {tuple(b) for b in wl.nn_bonds(N, M)}
    starts = wl.random_sz0_configs(N, M, 8, 1005)
    for c in range(8):
        prev = starts[c]
        for t in range(16):
            cur = S[c * 16 + t]
            d = np.nonzero(cur != prev)[0]
            assert d.size in (0, 2)
            if d.size == 2:
                assert tuple(d) in bonds
            prev = cur
