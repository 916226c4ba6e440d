"""The C ABI library loads on a host without a GPU and exports every entry
point declared in include/lbfd.h; parameter validation runs on the host."""
import ctypes as C
import os
import re

import pytest

import workloads as W
from paper_2311_15242_amd import build as B
from paper_2311_15242_amd import lbfd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in sorted(os.listdir(inc)):
        if fn.endswith(".h"):
            txt = open(os.path.join(inc, fn)).read()
            names |= set(re.findall(r"^\s*(?:int|int64_t|void|const char \*|lbfd_\w+ \*)\s*(lbfd_\w+)\s*\(",
                                    txt, re.M))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB):
        pytest.skip("liblbfd.so not built (run __graft_entry__.build())")
    return lbfd.load()


def test_exports_match_header(lib):
    names = declared()
    assert len(names) >= 11
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(lbfd.EXPORTED) == names


def test_structs_match_header_sizes(lib):
    # the C structs are plain and naturally aligned; ctypes computes the same layout
    assert C.sizeof(lbfd.Params) % 8 == 0
    assert C.sizeof(lbfd.Obs) % 8 == 0
    assert lbfd.Obs.status.offset + 4 <= C.sizeof(lbfd.Obs)


def test_workspace_size_and_validation(lib):
    p = W.finalize(dict(lattice=W.D3Q19, nx=128, ny=128, nz=384, precision="bf16dev"))
    n = lbfd.workspace_bytes(p)
    N = 128 * 128 * 384
    # two 16-bit population buffers dominate; total stays well under 288 GB
    assert 2 * 19 * 2 * N < n < 400 * N
    with pytest.raises(lbfd.LbfdError) as e:
        lbfd.workspace_bytes(dict(p, nx=2))
    assert e.value.status == lbfd.LBFD_EINVAL
    with pytest.raises(lbfd.LbfdError):
        lbfd.workspace_bytes(dict(p, rhoR0=-1.0))
    with pytest.raises(lbfd.LbfdError):
        lbfd.workspace_bytes(dict(p, sor_max_sweeps=10_000))
    # 32-bit byte offsets: the largest grids, 16-byte elements (FP64: 32-byte)
    big = dict(p, nx=512, ny=512)
    assert lbfd.workspace_bytes(dict(big, nz=1023)) < 70 * 2**30
    for prec, nz in (("bf16dev", 1024), ("fp64", 512)):
        with pytest.raises(lbfd.LbfdError):
            lbfd.workspace_bytes(W.finalize(dict(big, nz=nz, precision=prec)))
    lbfd.workspace_bytes(W.finalize(dict(big, nz=511, precision="fp64")))
    # alphaB from eq 42 must stay in (0, 1)
    with pytest.raises(lbfd.LbfdError):
        lbfd.workspace_bytes(dict(p, rhoR0=10.0, rhoB0=1.0))


def test_create_rejects_missing_workspace(lib):
    p = W.finalize(dict(lattice=W.D2Q9, nx=16, ny=16))
    h = C.c_void_p()
    st = lib.lbfd_create(C.byref(lbfd.params_struct(p)), None, 0, None, C.byref(h))
    assert st == lbfd.LBFD_EWORKSPACE and not h.value
    assert lib.lbfd_strerror(st).decode().startswith("device workspace")


def test_precision_sizes(lib):
    sizes = {}
    for prec in W.PRECISIONS:
        p = W.finalize(dict(lattice=W.D3Q19, nx=64, ny=64, nz=64, precision=prec))
        sizes[prec] = lbfd.workspace_bytes(p)
    assert sizes["fp64"] > sizes["fp32"] > sizes["bf16dev"]
    assert sizes["fp16dev"] == sizes["bf16dev"]


def _batch_bytes(lib, plist):
    arr = (lbfd.Params * len(plist))(*[lbfd.params_struct(p) for p in plist])
    nb = C.c_size_t()
    st = lib.lbfd_batch_workspace_bytes(arr, len(plist), C.byref(nb))
    return st, int(nb.value)


def test_batch_workspace_and_validation(lib):
    plist = [p for p, _ in W.batch_instances(W.load_manifest()[:5])]
    st, nb = _batch_bytes(lib, plist)
    assert st == lbfd.LBFD_OK
    # instance slices (each 256-aligned) plus the parameter table and tile prefixes
    singles = sum(-(-lbfd.workspace_bytes(p) // 256) * 256 for p in plist)
    assert singles < nb < singles + 5 * 4096 + 4096
    # lattice, precision, fd_enable and sor_max_sweeps are common to a batch
    for key, val in (("lattice", W.D3Q19), ("precision", "fp32"), ("fd_enable", 0), ("sor_max_sweeps", 7)):
        bad = list(plist)
        bad[3] = W.finalize(dict(plist[3], **{key: val}))
        assert _batch_bytes(lib, bad)[0] == lbfd.LBFD_EINVAL, key
    # an invalid instance fails the batch; grids and physics may differ freely
    assert _batch_bytes(lib, plist[:2] + [dict(plist[2], nx=2)])[0] == lbfd.LBFD_EINVAL
    assert _batch_bytes(lib, [plist[0], dict(plist[0], gravity=[0.0, 0.0, 0.0], nx=40)])[0] == lbfd.LBFD_OK
    # empty batch
    nb = C.c_size_t()
    assert lib.lbfd_batch_workspace_bytes(None, 0, C.byref(nb)) == lbfd.LBFD_EINVAL
    h = C.c_void_p()
    arr = (lbfd.Params * 1)(lbfd.params_struct(plist[0]))
    assert lib.lbfd_batch_create(arr, 1, None, 0, None, C.byref(h)) == lbfd.LBFD_EWORKSPACE and not h.value
    assert lib.lbfd_batch_instance(None, 0) is None


def test_batch_manifest_is_the_seeded_draw():
    m = W.load_manifest()
    assert m == W.batch_manifest(64, 0)
    assert all(128 <= x["W"] <= 256 and 256 <= x["H"] <= 768 for x in m)
    assert all(1.0 <= x["Eo"] <= 50.0 and 0.01 <= x["Bi"] <= 10.0 for x in m)
