"""mask_query_screened_noalloc: the screened descent on the library's static
per-GPU scratch (no workspace, no allocation) returns what
mask_query_screened returns with a caller's workspace, bit for bit, on two
calls in a row (the second smaller, so the scratch still holds the first
call's rows), across several slices of the static scratch."""
import numpy as np
import pytest

import datagen
from tests.gpu_helpers import dev, host

pytestmark = pytest.mark.gpu

SCRATCH = 64 << 20  # MASK_NOALLOC_SCRATCH_BYTES


@pytest.fixture(scope="module")
def pk():
    import torch
    assert torch.cuda.is_available()
    import paper_2208_02734_amd as pk
    pk.lib()
    return pk


def _mixture(n, d, n_comp, seed, nq):
    mix = datagen.mixture_params(seed, n_comp, d, sigma_mode="loguniform", sigma_low=0.1,
                                 sigma_high=3.0)
    return datagen.sample_mixture(mix, n, seed + 1), datagen.sample_mixture(mix, nq, seed + 2)


def test_noalloc_equals_the_workspace_entry_point(pk):
    import torch
    X, Q = _mixture(60_000, 32, 120, seed=1500, nq=4000)
    # 10,000 / 200 / 10 prototypes: every level screened, 41,096 bytes per
    # query, so 4,000 queries take three slices of the 64 MiB scratch
    ix = pk.mask_build(dev(X), [(20, 500), (1, 200), (1, 10)], iters=4, seed=5,
                       precision="bf16")
    per = pk.mask_screen_bytes(ix)
    assert per == 4 * (10016 + 224 + 32) + 8
    assert SCRATCH // per < Q.shape[0]
    beams = [4, 24, 64]
    for nq, k in ((Q.shape[0], 10), (517, 7)):
        q = dev(Q[:nq])
        ws = torch.empty(per * nq + 256, dtype=torch.uint8, device="cuda")
        want = [host(t) for t in pk.mask_query_screened(ix, q, k, beams, workspace=ws)]
        got = [host(t) for t in pk.mask_query_screened_noalloc(ix, q, k, beams)]
        torch.cuda.synchronize()
        assert got[0].shape == (nq, k)
        assert np.array_equal(got[0], want[0]), f"ids differ for {nq} queries"
        assert np.array_equal(got[1].view(np.uint32), want[1].view(np.uint32)), \
            f"distances differ for {nq} queries"
        assert (got[0] >= 0).all()
    ix.free()


def test_noalloc_writes_into_given_outputs_and_checks_arguments(pk):
    import torch
    X, Q = _mixture(3000, 16, 10, seed=1510, nq=33)
    f32 = pk.mask_build(dev(X), [(2, 20)], iters=2, seed=1)
    with pytest.raises(pk.MaskError) as e:
        pk.mask_query_screened_noalloc(f32, dev(Q), 5, [4])
    assert e.value.status == 4  # only the BF16 form is screened
    f32.free()
    g = pk.mask_build(dev(X), [(2, 20)], iters=2, seed=1, precision="bf16")
    with pytest.raises(pk.MaskError) as e:
        pk.mask_query_screened_noalloc(g, dev(Q), 5, [0])
    assert e.value.status == 1
    ids = torch.full((33, 5), -7, dtype=torch.int32, device="cuda")
    dist = torch.zeros((33, 5), dtype=torch.float32, device="cuda")
    pk.mask_query_screened_noalloc(g, dev(Q), 5, [4], out=(ids, dist))
    want = [host(t) for t in pk.mask_query_screened(g, dev(Q), 5, [4])]
    assert np.array_equal(host(ids), want[0])
    assert np.array_equal(host(dist).view(np.uint32), want[1].view(np.uint32))
    g.free()
