"""Parity of the finite-chaos benchmark path (non-affine coefficient, forcing assembly, time marching,
error sums) with the FP64 CPU oracle, on an MI355X.

Tolerances:
  * spatial load vectors, chaos projection weights, error sums of a given slab vector (quadrature
    sums in FP64, different summation order): 1e-12 relative;
  * non-affine operator apply: 1e-12 relative;
  * marched errors and the last slab (slab solves to rtol 1e-12): 1e-8 relative;
  * 128^2-cell Q3 / dG(3) / 64-slab runs: properties that hold at any size (the p = 0 variance errors
    are the printed values of Table tab:finite-errors-rates, since the discrete variance is then 0;
    the mean error does not change from p = 0 to p = 1).
"""
import numpy as np
import pytest

import sg_inputs
from oracle import finitechaos as fc
from oracle.slab import from_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rel_inf(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def test_setup_pieces_match_oracle(torch_cuda):
    from paper_2605_21046_amd.finitechaos import FiniteChaosRun
    fw = sg_inputs.finite_chaos_workload(4, 3, 3, 8, 2, 1)
    print("finite-chaos set-up 4x4 Q3 p=2", flush=True)
    R = FiniteChaosRun(fw)
    P = from_workload(fw.base)
    m, k = fc.spatial_loads(P)
    V = R.V.cpu().numpy()
    assert _rel_inf(V[0], m) <= 1e-12
    for i in range(k.shape[0]):
        assert _rel_inf(V[1 + i], k[i]) <= 1e-12
    assert _rel_inf(R.D, fc.forcing_chaos_weights(P, fw)) <= 1e-13
    assert [tuple(a) for a in R.P.index_set()] == P.index_set
    R.close()


def test_nonaffine_apply_matches_oracle(torch_cuda):
    from paper_2605_21046_amd import sgheat
    torch = torch_cuda
    fw = sg_inputs.finite_chaos_workload(4, 3, 3, 8, 2, 1)
    G = sgheat.problem_from_workload(fw.base)
    P = from_workload(fw.base)
    x = sg_inputs.uniform_vector(P.n, 41)
    y = G.apply(torch.from_numpy(x).to("cuda")).cpu().numpy()
    G.close()
    assert _rel_inf(y, P.assemble_full() @ x) <= 1e-12


def test_error_sums_of_a_given_slab_match_oracle(torch_cuda):
    from paper_2605_21046_amd.finitechaos import FiniteChaosRun
    torch = torch_cuda
    fw = sg_inputs.finite_chaos_workload(4, 3, 3, 8, 1, 1)
    R = FiniteChaosRun(fw)
    P = from_workload(fw.base)
    u = 0.05 * sg_inputs.uniform_vector(P.n, 42)
    u[P.full_boundary_mask()] = 0.0
    acc = R.P.separable_error(torch.from_numpy(u).to("cuda"), R.nq1, R.s_qp, R.gs_qp, (fw.base.tau * R.st) ** 4,
                              R.c, R.C2)
    R.close()
    ref = fc.errors(P, fw, [u])
    got = {"E_full_L2": np.sqrt(acc[0] + R.tail * acc[6]), "E_full_H1": np.sqrt(acc[1] + R.tail * acc[7]),
           "E_mean_L2": np.sqrt(acc[2]), "E_mean_H1": np.sqrt(acc[3]), "E_var_L2": np.sqrt(acc[4]),
           "E_var_H1": np.sqrt(acc[5])}
    for key, v in ref.items():
        assert _rel(got[key], v) <= 1e-12, key


@pytest.mark.parametrize("p", [1, 2])
def test_marched_errors_match_oracle(torch_cuda, p):
    from paper_2605_21046_amd.finitechaos import FiniteChaosRun
    fw = sg_inputs.finite_chaos_workload(4, 3, 3, 8, p, 2)
    print(f"finite-chaos march 4x4 Q3 dG(3) 8 slabs p={p}", flush=True)
    R = FiniteChaosRun(fw, rtol=1e-12)
    errs, u = R.run()
    its = [i["iterations"] for i in R.info]
    R.close()
    P = from_workload(fw.base)
    U = fc.march(fw, P)
    ref = fc.errors(P, fw, U)
    print(f"iterations per slab {min(its)}..{max(its)}; {errs}", flush=True)
    assert _rel_inf(u.cpu().numpy(), U[-1]) <= 1e-8
    for key, v in ref.items():
        assert _rel(errs[key], v) <= 1e-8, key


def test_full_resolution_properties(torch_cuda):
    """128^2 Q3 cells, dG(3), 64 slabs (the paper's discretisation) at p = 0 and p = 1."""
    from paper_2605_21046_amd.finitechaos import FiniteChaosRun
    table = {}
    for line in open(__file__.replace("test_gpu_finitechaos.py", "golden/finite_chaos_table.txt")):
        if not line.startswith("#") and line.strip():
            v = line.split()
            table[int(v[0])] = [float(x) for x in v[2:]]
    out = {}
    for p in [0, 1]:
        print(f"finite-chaos 128^2 Q3 dG(3) 64 slabs p={p}", flush=True)
        R = FiniteChaosRun(sg_inputs.finite_chaos_workload(128, 3, 3, 64, p, 5), rtol=1e-10)
        out[p], _ = R.run()
        R.close()
        print(out[p], flush=True)
    assert f"{out[0]['E_var_L2']:.5e}" == f"{table[0][4]:.5e}"
    assert f"{out[0]['E_var_H1']:.5e}" == f"{table[0][5]:.5e}"
    assert out[1]["E_mean_L2"] == pytest.approx(out[0]["E_mean_L2"], rel=1e-6)
