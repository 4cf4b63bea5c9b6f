"""The GPU's generator against the oracle's, word for word (runs on an MI355X).

Both sides implement Philox4x64-10 from its published description, and the
oracle's is pinned to numpy's own Philox.  Here 1e6 counters spread over every
purpose tag of the method (loading, waits, collisions, ion partners, births,
the atoms' source and events, the yield rule) and over extreme counter and key
words must give the same four 64-bit words on both sides.
"""
import numpy as np
import pytest

from oracle import philox as R

pytestmark = pytest.mark.gpu

TAGS = [R.tag(s, pu) for s in (R.SP_E, R.SP_I) for pu in (R.INIT, R.SKIP, R.COLL, R.ION, R.CHILD)] + \
       [R.tag(R.SP_AL, R.TP_SRC), R.tag(R.SP_AL, R.TP_EVT), R.tag(R.SP_YIELD, R.YIELD)]


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1607_04069_amd as mod
    return mod


def test_generator_words_match_the_oracle(pm):
    rng = np.random.default_rng(1607)
    n = 1_000_000 // len(TAGS)
    total = 0
    for j, tag in enumerate(TAGS):
        # counter and key words from small to the top of their range
        id0 = [0, 2 ** 64 - n, int(rng.integers(0, 2 ** 63))][j % 3]
        index = [0, 2 ** 64 - 1, int(rng.integers(0, 2 ** 40))][(j + 1) % 3]
        aux = [0, 1, 2 ** 63 + 5][j % 3]
        seed, key = [(1607, 0), (2 ** 64 - 1, 2 ** 32 - 1), (int(rng.integers(0, 2 ** 63)), 12345)][(j + 2) % 3]
        got = pm.philox_words(id0, index, tag, aux, seed, key, n)
        ids = (np.uint64(id0) + np.arange(n, dtype=np.uint64))
        want = np.stack(R.philox4x64(ids, np.uint64(index), np.uint64(tag), np.uint64(aux),
                                     np.uint64(seed), np.uint64(key)), axis=1)
        assert got.shape == want.shape
        assert np.array_equal(got, want), (tag, int(np.count_nonzero(np.any(got != want, axis=1))))
        total += n
    assert total >= 999_000
