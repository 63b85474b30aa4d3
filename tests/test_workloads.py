"""Input generators (no part of the method): the C helper of the electrolyte
generator accepts exactly the candidates the NumPy loop accepts, and the
result is a valid random sequential addition."""
import os

import numpy as np
import pytest

from paper_1708_01135_amd import workloads as wl


@pytest.mark.skipif(not os.path.exists(wl._RSA_LIB), reason="input helper not built")
@pytest.mark.parametrize("n, seed", [(4000, 1), (30000, 2)])
def test_electrolyte_helper_matches_numpy(n, seed):
    a_pos, a_q, a_L = wl.electrolyte(n, 0.8, seed)
    b_pos, b_q, b_L = wl.electrolyte(n, 0.8, seed, use_helper=False)
    assert a_L == b_L
    assert np.array_equal(a_pos, b_pos) and np.array_equal(a_q, b_q)


def test_electrolyte_is_a_valid_packing():
    pos, q, L = wl.electrolyte(3000, 0.8, 7)
    assert pos.shape == (3000, 3) and np.all((pos >= 0) & (pos < L))
    assert q.sum() == 0 and set(np.unique(q)) == {-1.0, 1.0}
    d = pos[:, None, :] - pos[None, :, :]
    d -= L * np.round(d / L)
    r2 = np.einsum("ijk,ijk->ij", d, d)
    np.fill_diagonal(r2, np.inf)
    assert r2.min() >= 0.8 ** 2
