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
    txt = open(os.path.join(ROOT, "include", "lbfd.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*(lbfd_\w+)\s*\(", txt, re.M)))


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
