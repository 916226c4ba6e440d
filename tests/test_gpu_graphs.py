"""Graph replay of steps (lbfd_set_graphs, lbfd_batch_set_graphs).

A call that advances four or more steps replays a captured two-step HIP graph.
The replayed steps must be bit-identical to the same steps launched one kernel
at a time, after every call, with the caller's own eager work and
synchronisations between the replays (the graph is replayed many times, from
both buffer-role states).
"""
import numpy as np
import pytest

import workloads as W
from tests.parity import say

pytestmark = pytest.mark.gpu

FIELDS = ("f", "rhoR", "rhoB", "u", "psi", "phi", "force", "G", "Sprev", "Bprev")
# step counts per call: short calls run eagerly, long ones replay from either parity
CALLS = (1, 6, 3, 9, 4, 1, 12)


@pytest.fixture(scope="module")
def lbfd():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_15242_amd import lbfd as L

    L.load()
    return L


def same(a, b, what):
    for name in FIELDS:
        x, y = a.field(name), b.field(name)
        assert np.array_equal(x, y), f"{what}: {name} differs (max {float(np.abs(x - y).max()):.3e})"
    oa, ob = a.observables(), b.observables()
    for k in ("total_surf", "sor_sweeps", "status", "step", "mass_R"):
        assert oa[k] == ob[k], (what, k)


def churn():
    """Unrelated eager work on the caller's stream between replays."""
    import torch

    x = torch.randn(1 << 20, device="cuda")
    return float((x * x).sum().item())


@pytest.mark.parametrize("case,prec", [("walled3d", "fp64"), ("walled3d", "bf16dev"), ("odd2d", "fp32"),
                                       ("nofd2d", "fp16dev")])
def test_single_graph_replay_identical(lbfd, case, prec):
    if case == "walled3d":
        p, q = W.make(dict(lattice=W.D3Q19, nx=23, ny=21, nz=19, bc=[W.WALL, W.WALL, W.WALL],
                           wall_u=[[0, 0, 0], [0, 0, 0], [0.01, 0, 0], [-0.01, 0, 0], [0, 0.008, 0], [0, 0, 0]],
                           rhoR0=0.3, muR0=0.05, muB0=0.12, sigma0=0.01, Ds=0.05, Db=0.08, gravity=[0, 2e-6, -1e-5],
                           precision=prec),
                      dict(drops=[(10.0, 9.5, 8.0, 5.5)], width=3.0, psi0=0.2, phi0_out=0.06, phi0_in=0.01))
    elif case == "odd2d":
        p, q = W.droplet_adsorption(n=70, radius=11.0, precision=prec, ny=37)
    else:
        p, q = W.droplet_adsorption(n=48, radius=10.0, precision=prec, fd_enable=0)
    say(f"[graph replay] {case} {prec}")
    a = lbfd.Solver(p).init_fields(q).graphs(False)
    b = lbfd.Solver(p).init_fields(q)
    for i, n in enumerate(CALLS):
        a.step(n)
        b.step(n)
        churn()
        same(a, b, f"{case} call {i} ({n} steps)")
    assert b.observables()["status"] == 0
    a.close()
    b.close()


def test_batch_graph_replay_identical(lbfd):
    inst = W.batch_instances(W.load_manifest()[:6], precision="bf16dev", scale=0.5)
    say(f"[batch graph replay] {len(inst)} instances")

    def make():
        bt = lbfd.Batch([p for p, _ in inst])
        for m, (_, q) in zip(bt.members, inst):
            m.init_fields(q)
        return bt

    a, b = make().graphs(False), make()
    for i, n in enumerate(CALLS):
        a.step(n)
        b.step(n)
        churn()
        for j in range(len(inst)):
            same(a[j], b[j], f"batch call {i} instance {j}")
    a.close()
    b.close()
