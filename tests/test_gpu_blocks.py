"""Per-mode diagonal blocks in the block-Jacobi preconditioner (desc.diag_blocks = 1) against the FP64
CPU oracle's per-mode hierarchies, on an MI355X.

Tolerances: one V-cycle in FP64, 1e-10 relative (Gauss-Jordan patch inverses against LU solves,
different summation orders through three levels); mixed precision 1e-5; solves by their true
residual recomputed by the oracle.
"""
import numpy as np
import pytest

import sg_inputs
from oracle import multigrid
from oracle import montecarlo as mc
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


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-5)])
def test_per_mode_vcycle_matches_oracle(torch_cuda, precision, tol):
    from paper_2605_21046_amd import sgheat
    torch = torch_cuda
    w = sg_inputs.finite_chaos_workload(4, 3, 3, 8, 2, 2).base      # non-affine, 15 modes, 2 levels
    print(f"per-mode V-cycle, precision {precision}", flush=True)
    G = sgheat.problem_from_workload(w, precision, diag_blocks=1)
    P = from_workload(w)
    r = sg_inputs.uniform_vector(P.n, 81)
    z = G.vcycle(torch.from_numpy(r).to("cuda")).cpu().numpy()
    G.close()
    ref = multigrid.block_hierarchies_from_workload(w).vcycle(r, P.n_xi)
    assert _rel_inf(z, ref) <= tol
    # and it differs from the mean-block cycle (the blocks really differ here)
    ref0 = multigrid.hierarchy_from_workload(w).vcycle(r, P.n_xi)
    assert _rel_inf(ref0, ref) > 1e-3


def test_per_mode_blocks_of_an_affine_coefficient_equal_the_mean_block(torch_cuda):
    from paper_2605_21046_amd import sgheat
    torch = torch_cuda
    w = sg_inputs.WORKLOADS["t2q2"]
    G0 = sgheat.problem_from_workload(w)
    G1 = sgheat.problem_from_workload(w, diag_blocks=1)
    r = torch.from_numpy(sg_inputs.uniform_vector(G0.n(0), 82)).to("cuda")
    z0, z1 = G0.vcycle(r).cpu().numpy(), G1.vcycle(r).cpu().numpy()
    G0.close()
    G1.close()
    assert _rel_inf(z1, z0) <= 1e-12


def test_per_mode_blocks_cut_the_iterations_of_the_nonaffine_solve(torch_cuda):
    from paper_2605_21046_amd import sgheat
    torch = torch_cuda
    w = sg_inputs.finite_chaos_workload(8, 3, 3, 16, 3, 3).base      # 35 modes, 3 levels
    print("per-mode blocks: non-affine solve", flush=True)
    P = from_workload(w)
    b = 0.1 * sg_inputs.uniform_vector(P.n, 83)
    b[P.full_boundary_mask()] = 0.0
    its = {}
    for diag in (0, 1):
        G = sgheat.problem_from_workload(w, diag_blocks=diag)
        x, info = G.solve(torch.from_numpy(b).to("cuda"), rtol=1e-10, max_iter=1000)
        G.close()
        assert info["converged"]
        r = b - P.apply_route2(x.cpu().numpy())
        assert np.linalg.norm(r) <= 1.0001e-10 * np.linalg.norm(b)
        its[diag] = info["iterations"]
    print(its, flush=True)
    assert its[1] < its[0]


def test_per_sample_vcycle_matches_pathwise_hierarchies(torch_cuda):
    """A sample batch with per-sample blocks: every sample's V-cycle is the pathwise problem's own."""
    from paper_2605_21046_amd.montecarlo import SampleBatch
    torch = torch_cuda
    ew = sg_inputs.MC_ERROR_WORKLOADS["e2"]                        # finite-chaos coefficient, 2 levels
    sw = sg_inputs.SampleWorkload(ew.base, ew.n_samples, ew.n_slabs, ew.seed)
    xs = ew.samples()
    B = SampleBatch(sw, samples=xs, diag_blocks=1)
    r = sg_inputs.uniform_vector(B.P.n(0), 84)
    z = B.P.vcycle(torch.from_numpy(r).to("cuda")).cpu().numpy().reshape(len(xs), -1)
    B.close()
    R = r.reshape(len(xs), -1)
    for s, xi in enumerate(xs):
        probs = [mc.pathwise_problem(ew.base, xi, l) for l in range(ew.base.n_levels)]
        H = multigrid.Hierarchy(probs, ew.base.pre_smooth, ew.base.post_smooth, ew.base.vanka_omega)
        assert _rel_inf(z[s], H.vcycle_mode(R[s])) <= 1e-10


def test_error_split_with_per_sample_blocks(torch_cuda):
    from oracle import mcerrors as me
    from paper_2605_21046_amd.mcerrors import MCErrorStudy
    ew = sg_inputs.MC_ERROR_WORKLOADS["e2"]
    its = {}
    for diag in (0, 1):
        S = MCErrorStudy(ew, rtol=1e-12, diag_blocks=diag)
        got = S.run()
        its[diag] = max(i["iterations"] for i in S.info)
        S.close()
    print(its, flush=True)
    ref = me.error_split(ew)
    for key in ["tot_mean", "disc_mean", "tot_var", "disc_var"]:
        assert got[key] == pytest.approx(ref[key], rel=1e-8), key
    assert its[1] < its[0]
