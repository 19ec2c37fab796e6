"""pic_rate_eval_noalloc (the entry point that allocates nothing) against
pic_rate_eval, through the C ABI: identical ln nu for every rate mode, on two
calls in a row (the second smaller, so it reads the static staging buffer
after a larger call), with no allocation through the handle's allocator."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1606_02862_amd as pkg
    pkg.load()
    return pkg


class _CountingAllocator:
    """torch device memory, counting the requests."""

    def __init__(self):
        from paper_1606_02862_amd import _capi as A
        self.calls, self.live = 0, {}
        self._alloc = A.ALLOC_FN(self._do_alloc)
        self._free = A.FREE_FN(self._do_free)
        self.struct = A.AllocT(self._alloc, self._free, None)

    def _do_alloc(self, nbytes, user):
        self.calls += 1
        t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
        self.live[t.data_ptr()] = t
        return t.data_ptr()

    def _do_free(self, ptr, user):
        self.live.pop(ptr, None)


def test_noalloc_rate_eval_matches_rate_eval(P):
    from paper_1606_02862_amd import _capi as A
    cfg = workloads.reduced(3, 16, 16, 8)
    alloc = _CountingAllocator()
    T, ne, Z = workloads.loguniform_rate_inputs(31, A.PIC_RATE_EVAL_NOALLOC_MAX, t_range=(0.5, 3e4),
                                                n_range=(1e18, 1e24))
    with P.Pic(cfg, allocator=alloc) as pic:
        pic.mlp_train(1, n_train=65536, batch=1024, steps=200, seed=5)
        pic.rate_eval("table", 1, T[:8], ne[:8], Z[:8])           # builds the table
        for mode in ("exact", "mlp", "table"):
            for n in (A.PIC_RATE_EVAL_NOALLOC_MAX, 7777):          # full buffer, then a smaller call
                want = pic.rate_eval(mode, 1, T[:n], ne[:n], Z[:n])
                before = alloc.calls
                got = pic.rate_eval(mode, 1, T[:n], ne[:n], Z[:n], noalloc=True)
                assert alloc.calls == before, "the no-alloc entry point allocated"
                print(mode, n, "finite", int(np.isfinite(want).sum()), flush=True)
                assert np.array_equal(np.isfinite(got), np.isfinite(want))
                assert np.array_equal(got, want), mode
        with pytest.raises(P.PicError) as e:
            n = A.PIC_RATE_EVAL_NOALLOC_MAX + 1
            pic.rate_eval("exact", 1, np.full(n, 100.0), np.full(n, 1e21), np.zeros(n, dtype=np.int32), noalloc=True)
        assert e.value.code == A.PIC_ERR_ARG
