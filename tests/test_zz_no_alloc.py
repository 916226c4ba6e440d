"""lbfd_read_field_noalloc, the read entry point that allocates nothing (it
stages through the library's fixed device array), against lbfd_read_field on
the same states: two calls in a row, the second on a smaller input, every
field identical to the last bit, and requests above the array's capacity
refused with LBFD_ESCRATCH."""
import numpy as np
import pytest

import workloads as W
from tests.parity import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbfd():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_15242_amd import lbfd as L

    L.load()
    return L


FIELDS_2D = ("f", "rhoR", "rhoB", "rhoN", "u", "psi", "phi", "force", "G", "Sprev", "Bprev")


def _same(a, b):
    return a.shape == b.shape and np.array_equal(a.view(np.uint64), b.view(np.uint64))


def test_noalloc_read_matches_read_field_twice(lbfd):
    # first call: a 3-D walled column in BF16 deviations (every field, the
    # populations included); second call: a smaller 2-D droplet in FP64
    big_p, big_q = W.bubble_rise(nx=40, ny=36, nz=70, radius=7.0, precision="bf16dev")
    small_p, small_q = W.droplet_adsorption(n=48, radius=10.0, ny=40)
    say(f"[noalloc] big {big_p['nx']}x{big_p['ny']}x{big_p['nz']} bf16dev, small 48x40 fp64")
    big = lbfd.Solver(big_p).init_fields(big_q).step(7)
    small = lbfd.Solver(small_p).init_fields(small_q).step(5)
    for s in (big, small):
        for name in FIELDS_2D:
            a = s.field_noalloc(name)
            b = s.field(name)
            assert _same(a, b), name
            assert np.isfinite(a).all(), name
        # a second read after more steps: the array keeps the last call's
        # contents, which must not leak into the next result
        s.step(3)
        assert _same(s.field_noalloc("psi"), s.field("psi"))
        assert _same(s.field_noalloc("u"), s.field("u"))
    say("[noalloc] identical to lbfd_read_field on both")


def test_noalloc_rejects_requests_beyond_capacity(lbfd):
    # D3Q19 populations of 128 x 128 x 32 nodes: 19 * 524288 = 9.96 M doubles,
    # above the 8 Mi of the fixed array; a scalar field of the same grid fits
    p, q = W.bubble_rise(nx=128, ny=128, nz=32, radius=8.0, precision="bf16dev")
    s = lbfd.Solver(p).init_fields(q)
    assert 19 * s.N > lbfd.SCRATCH_DOUBLES >= s.N
    with pytest.raises(lbfd.LbfdError) as e:
        s.field_noalloc("f")
    assert e.value.status == lbfd.LBFD_ESCRATCH
    assert _same(s.field_noalloc("rhoN"), s.field("rhoN"))
    # a wrong count is still EINVAL, checked before anything runs
    import ctypes as C
    out = np.zeros(5)
    st = lbfd.load().lbfd_read_field_noalloc(s.h, lbfd.FIELDS["psi"], out.ctypes.data_as(C.POINTER(C.c_double)), 5)
    assert st == lbfd.LBFD_EINVAL
