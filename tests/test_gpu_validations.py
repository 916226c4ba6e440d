"""The physics validations of bench.py run end to end on small grids (the
published comparisons use the sizes in their docstrings); each must finish with
a clean status and values of the right sign and size."""
import numpy as np
import pytest

import bench

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_15242_amd import lbfd

    lbfd.load()


def test_ygb_small(gpu):
    r = bench.ygb_validation(4, "bf16dev", max_steps=2000, chunk=200, tol=1e-3, widths=(5,))
    c = r["cases"][0]
    print(c)
    assert c["grid"] == [20, 20, 40]
    assert c["steps"] >= 2000 or c["converged"]
    assert 0.3 < c["u_over_uygb"] < 2.0 and abs(c["radius_end"] - 4.0) < 1.0


def test_adsorption_small(gpu):
    r = bench.adsorption_validation(4, "fp64", taus=(0.5, 1.0), samples=4)
    print(r["psi"])
    assert r["status"] == 0
    sims = [x["sim"] for x in r["psi"]]
    assert all(v > 0 for v in sims) and sims == sorted(sims)


def test_uptake_early(gpu):
    r = bench.uptake_validation(times=(50, 100))
    print(r)
    assert r["status"] == 0
    assert all(abs(d) < 0.2 for d in r["rel_diff"])


def test_retardation_small(gpu):
    r = bench.retardation_study(4, "fp32", tau_eo1=1.0, tau_eo10=1.0)
    print(r["checks"])
    for name, c in r["cases"].items():
        assert np.isfinite(c["re"]) and c["re"] > 0, name
    assert r["cases"]["Eo10 Bi1"]["psi_av"] > 0 and r["cases"]["Eo1 clean"]["psi_av"] == 0


def test_shear_small(gpu):
    r = bench.shear_study(R=10)
    print(r["checks"], {k: v["tau8"] for k, v in r["cases"].items()})
    assert set(r["cases"]) == {"Pe_b 0.1", "Pe_b 1", "Pe_b 10", "insoluble"}
    for name, c in r["cases"].items():
        assert c["status"] == 0, name
        assert 0.0 < c["tau4"]["deformation"] < 1.0 and 0.0 < c["tau8"]["deformation"] < 1.0, name
