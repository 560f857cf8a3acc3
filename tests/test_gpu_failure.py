"""Allocator failure: when the caller's allocator returns NULL at its n-th
call, the entry point reports MASK_ERR_NOMEM and has handed every block it
obtained back to the allocator (counted by the callbacks), for every n up
to the number of allocations the call makes; a later call with a working
allocator succeeds."""
import ctypes

import numpy as np
import pytest

import datagen
from tests.gpu_helpers import dev

pytestmark = pytest.mark.gpu

NOMEM = 2


class CountingAllocator:
    """mask_allocator over PyTorch's caching allocator that fails its
    `fail_at`-th call (1-based; None: never) and tracks the live blocks."""

    def __init__(self, pk, fail_at=None):
        import torch
        self.calls = 0
        self.fail_at = fail_at
        self.live = {}
        self.freed = 0
        self.errors = []

        def _alloc(ctx, nbytes, stream):
            self.calls += 1
            if self.fail_at is not None and self.calls == self.fail_at:
                return None
            p = torch.cuda.caching_allocator_alloc(int(nbytes), 0, stream or 0)
            self.live[p] = int(nbytes)
            return p

        def _free(ctx, ptr, nbytes, stream):
            # (an exception cannot cross the C callback: errors are recorded)
            if ptr not in self.live:
                self.errors.append(f"freed {ptr:#x}, a block it was not given")
                return
            if self.live.pop(ptr) != int(nbytes):
                self.errors.append(f"freed {ptr:#x} with another size")
            self.freed += 1
            torch.cuda.caching_allocator_delete(ptr)

        self._a = pk._ALLOC_FN(_alloc)
        self._f = pk._FREE_FN(_free)
        self.struct = pk.mask_allocator(None, self._a, self._f)


@pytest.fixture(scope="module")
def pk():
    import torch
    assert torch.cuda.is_available()
    import paper_2208_02734_amd as pk
    pk.lib()
    return pk


def _data(n=4000, d=16, seed=700):
    mix = datagen.mixture_params(seed, 20, d)
    return datagen.sample_mixture(mix, n, seed + 1)


def _build(pk, X, alloc, precision="fp32", init="first"):
    import torch
    m = pk._matrix(X)
    p, lv = pk._params([(4, 50), (1, 10)], 3, 1, "l2", precision, 0, None, None, init)
    h = ctypes.c_void_p()
    st = pk.lib().mask_build(ctypes.byref(m), ctypes.byref(p), ctypes.byref(alloc.struct),
                             None, ctypes.byref(h))
    torch.cuda.synchronize()
    return st, h


@pytest.mark.parametrize("precision,init", [("fp32", "first"), ("bf16", "kmeans++")])
def test_build_frees_everything_when_an_allocation_fails(pk, precision, init):
    Xd = dev(_data())
    ok = CountingAllocator(pk)
    st, h = _build(pk, Xd, ok, precision, init)
    assert st == 0
    n_calls = ok.calls
    assert n_calls >= 5 and ok.live  # the index keeps blocks until it is freed
    pk.lib().mask_free(h)
    assert not ok.live
    for fail_at in range(1, n_calls + 1):
        a = CountingAllocator(pk, fail_at)
        st, h = _build(pk, Xd, a, precision, init)
        assert st == NOMEM, (fail_at, st)
        assert not h.value
        assert not a.live and not a.errors, (fail_at, len(a.live), a.errors[:2])
        assert a.calls == fail_at  # nothing is allocated after the failure
    again = CountingAllocator(pk)
    st, h = _build(pk, Xd, again, precision, init)
    assert st == 0
    pk.lib().mask_free(h)
    assert not again.live and not again.errors and not ok.errors


def test_kmeans_and_server_report_nomem_and_free(pk):
    import torch
    X = _data(3000, 8, seed=710)
    Xd = dev(X)
    m = pk._matrix(Xd)
    cent = torch.empty((3 * 20, 8), dtype=torch.float32, device="cuda")
    labels = torch.empty(3000, dtype=torch.int32, device="cuda")

    def kmeans(alloc):
        st = pk.lib().mask_kmeans(ctypes.byref(m), 3, 20, 4, 0, None, cent.data_ptr(),
                                  labels.data_ptr(), None, ctypes.byref(alloc.struct), None)
        torch.cuda.synchronize()
        return st

    ok = CountingAllocator(pk)
    assert kmeans(ok) == 0 and not ok.live
    for fail_at in range(1, ok.calls + 1):
        a = CountingAllocator(pk, fail_at)
        assert kmeans(a) == NOMEM
        assert not a.live and not a.errors
    # the server's arena comes from the allocator too
    ix = pk.mask_build(Xd, [(3, 20)], iters=2, seed=1)
    a = CountingAllocator(pk, 1)
    p = pk.mask_server_params(1 << 20, 256, 2, 0)
    h = ctypes.c_void_p()
    st = pk.lib().mask_server_create(ix.handle, ctypes.byref(p), ctypes.byref(a.struct),
                                     ctypes.byref(h))
    assert st == NOMEM and not h.value and not a.live
    ok = CountingAllocator(pk)
    st = pk.lib().mask_server_create(ix.handle, ctypes.byref(p), ctypes.byref(ok.struct),
                                     ctypes.byref(h))
    assert st == 0 and ok.live
    pk.lib().mask_server_destroy(h)
    assert not ok.live and not ok.errors
    ix.free()
