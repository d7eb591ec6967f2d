"""The allocation-free update call, mf_apply_updates_noalloc, against
mf_apply_updates through the C-ABI: two handles of one graph take the same
batches, the first through the existing entry point, the second through the
allocation-free one, two calls in a row with the second batch smaller.
Values and canonical cuts must be equal, and the allocation-free handle's
state must pass the oracle's full check (value, cut, layout, validator,
exact heights)."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import check_solved, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mf():
    import torch
    assert torch.cuda.is_available()
    from paper_2511_05895_amd import mf as m
    return m


def _graph(which):
    if which == "c1":
        return W.c1_random_1k(), 100
    if which == "grid":
        return W.seg_grid(96, seed=7), 100
    return W.rmat(14, 16, seed=11), 1000


@pytest.mark.parametrize("flags", [0, 2])
@pytest.mark.parametrize("which", ["c1", "grid", "rmat"])
def test_noalloc_matches_apply_updates(mf, which, flags):
    g, inc = _graph(which)
    log(f"noalloc {which} flags={flags}: n={g.n} m={g.m}")
    rng = np.random.default_rng(17)
    with mf.MaxFlow(g, flags=flags) as A, mf.MaxFlow(g, flags=flags) as B:
        assert A.solve() == B.solve()
        cap = g.cap.copy()
        for k in (max(2, g.m // 20), max(1, g.m // 200)):
            ids, new = W.mixed_batch(cap, k, inc, rng)
            cap[ids] = new
            va = A.update(ids, new)
            vb = B.update_noalloc(ids, new)
            assert va == vb
            sa, ca = A.min_cut()
            sb, cb = B.min_cut()
            assert ca == cb == vb
            assert np.array_equal(sa, sb)
            check_solved(B, g, cap, exact_heights=(flags == 0))


def test_noalloc_limit(mf):
    """A batch above MF_NOALLOC_MAX_UPDATES is refused and leaves the handle
    as it was; the next call goes on from the same state."""
    g = W.c2_grid_512()
    assert g.m > mf.MF_NOALLOC_MAX_UPDATES
    rng = np.random.default_rng(3)
    with mf.MaxFlow(g) as F:
        v = F.solve()
        ids, new = W.mixed_batch(g.cap, mf.MF_NOALLOC_MAX_UPDATES + 1, 100, rng)
        with pytest.raises(mf.MfError) as ei:
            F.update_noalloc(ids, new)
        assert ei.value.code == mf.MF_EINVAL
        assert F.value() == v
        cap = g.cap.copy()
        ids, new = W.mixed_batch(cap, 2000, 100, rng)
        cap[ids] = new
        F.update_noalloc(ids, new)
        check_solved(F, g, cap)
