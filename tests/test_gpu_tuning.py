"""The launch shapes the autotuner chooses from leave every result unchanged:
the same workload stepped with different node-tile rows and SOR grids gives
identical fields (to the last bit), alone and in a batch, and out-of-range
shapes are refused."""
import numpy as np
import pytest

import workloads as W
from tests.parity import say

pytestmark = pytest.mark.gpu

SHAPES = [dict(rows=4, sor_wg_per_cu=8, sor_narrow=256), dict(rows=1, sor_wg_per_cu=2, sor_narrow=8),
          dict(rows=2, sor_wg_per_cu=16, sor_narrow=1024)]


@pytest.fixture(scope="module")
def lbfd():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_15242_amd import lbfd as L

    L.load()
    return L


def _fields(s):
    return {n: s.field(n) for n in ("f", "rhoN", "u", "psi", "phi", "G", "force")}


def _same(a, b):
    return all(np.array_equal(a[k].view(np.uint64), b[k].view(np.uint64)) for k in a)


@pytest.mark.parametrize("case", ["box3d_bf16", "bubble2d_fp64_odd"])
def test_results_do_not_depend_on_the_launch_shape(lbfd, case):
    if case == "box3d_bf16":
        # ragged in x and y, walls on two axes, periodic z
        p, q = W.bubble_rise(nx=70, ny=37, nz=40, radius=7.0, precision="bf16dev")
    else:
        # odd periodic height (seam classes of the SOR), FP64
        p, q = W.bubble_rise(nx=48, ny=81, nz=1, radius=8.0, lattice=W.D2Q9, precision="fp64")
    say(f"[tuning] {case}")
    ref = None
    for t in SHAPES:
        s = lbfd.Solver(p, tuning=t).init_fields(q)
        assert s.get_tuning() == t
        s.step(9)
        f = _fields(s)
        ob = s.observables()
        assert ob["status"] == 0
        if ref is None:
            ref, ob0 = f, ob
        else:
            assert _same(f, ref), t
            for k in ("total_surf", "mass_R", "psi_av", "deformation"):
                assert ob[k] == ob0[k], (k, t)
        s.close()


def test_batch_shapes_match_single_runs(lbfd):
    manifest = W.load_manifest()[:6]
    inst = W.batch_instances(manifest, precision="bf16dev", scale=0.25)
    say(f"[tuning] batch of {len(inst)}")
    singles = []
    for p, q in inst:
        s = lbfd.Solver(p, tuning=None).init_fields(q).step(7)
        singles.append((s.field("u"), s.field("psi")))
        s.close()
    for rows in (1, 2, 4):
        b = lbfd.Batch([p for p, _ in inst], tuning=dict(rows=rows))
        for m, (_, q) in zip(b.members, inst):
            m.init_fields(q)
        b.step(7)
        for m, (u, ps) in zip(b.members, singles):
            assert np.array_equal(m.field("u"), u) and np.array_equal(m.field("psi"), ps), rows
        b.close()


def test_out_of_range_shapes_are_refused(lbfd):
    p, q = W.droplet_adsorption(n=32, radius=8.0)
    s = lbfd.Solver(p, tuning=None)
    for bad in (dict(rows=3), dict(rows=8), dict(sor_wg_per_cu=0), dict(sor_wg_per_cu=33), dict(sor_narrow=12),
                dict(sor_narrow=4)):
        with pytest.raises(lbfd.LbfdError) as e:
            s.set_tuning(bad)
        assert e.value.status == lbfd.LBFD_EINVAL
    assert s.get_tuning() == lbfd.DEFAULT_TUNING
