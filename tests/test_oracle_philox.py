"""Pin of the oracle's Philox4x64-10 against numpy's implementation of the
published generator (Salmon et al., SC'11); numpy advances the counter by
one before producing a block."""
import numpy as np
import pytest

import oracle as O


@pytest.mark.parametrize("key,ctr", [((0, 0), (0, 0, 0, 0)), ((0x1234, 0x5678), (5, 7, 0, 0)),
                                      ((2**64 - 1, 3), (2**63 + 11, 1, 2, 3)),
                                      ((1, 0), (0, 1, 0, 0))])
def test_philox_matches_numpy(key, ctr):
    bg = np.random.Philox(counter=np.array(ctr, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    ref = [int(v) for v in bg.random_raw(4)]
    nxt = list(ctr)
    nxt[0] = (nxt[0] + 1) % 2**64
    if nxt[0] == 0:
        nxt[1] += 1
    assert O.philox4x64_10(nxt, key) == ref


def test_draw_ranges_and_layout():
    n, D = 1000, 0.05
    idxs = []
    for t in range(2000):
        i, d, u = O.draw(7, 3, t, n, D)
        assert 0 <= i < n
        assert np.all(d >= -D) and np.all(d < D)
        assert 0.0 <= u < 1.0
        idxs.append(i)
    assert len(set(idxs)) > 800
    # stream 0 word 0 gives the index by a 64x64 high multiply
    w = O.philox4x64_10((5, 0, 0, 0), (7, 3))
    assert O.draw(7, 3, 5, n, D)[0] == (w[0] * n) >> 64
    v = O.philox4x64_10((5, 1, 0, 0), (7, 3))
    assert O.draw(7, 3, 5, n, D)[2] == (v[0] >> 11) * 2.0 ** -53
