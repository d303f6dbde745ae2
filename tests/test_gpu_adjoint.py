"""Parity of the adjoint building blocks and of the adjoint gradient (HIP path through the C ABI)
with the FP64 CPU oracle, on an MI355X.

Tolerances:
  * AA^T apply, slab transfer, cell-wise forms, QoI and its gradient (one kernel pass each, FP64):
    1e-12 relative (summation order only);
  * adjoint-handle FGMRES: true relative residual <= rtol recomputed by the oracle with AA^T;
  * gradient of J over a slab sequence: 1e-7 relative to the oracle's (direct solves) with the
    GPU slab solves at rtol 1e-12 (the error of the iterative solves enters linearly);
  * full-size (16^3 cells, 10 slabs) gradient against central differences of the GPU forward sweep:
    1e-4 relative (difference step 1e-5; the solver tolerance 1e-11 and the O(h^2) truncation set it).
"""
import numpy as np
import pytest

import sg_inputs
from oracle import adjoint as adj
from oracle import chaos
from oracle.slab import from_workload

pytestmark = pytest.mark.gpu

SMALL = ["c1", "t2q3", "t3q2"]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _to_gpu(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _rel_inf(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _interior_vector(P, seed):
    x = sg_inputs.uniform_vector(P.n, seed)
    x[P.full_boundary_mask()] = 0.0
    return x


@pytest.mark.parametrize("name", SMALL)
def test_apply_transpose_matches_oracle(torch_cuda, name):
    from paper_2605_21046_amd import sgheat
    torch = torch_cuda
    w = sg_inputs.WORKLOADS[name]
    print(f"apply_T parity {name}", flush=True)
    P = from_workload(w)
    AT = P.assemble_full().T.tocsr()
    x = sg_inputs.uniform_vector(P.n, 11)
    G = sgheat.problem_from_workload(w)
    y = G.apply_T(_to_gpu(torch, x)).cpu().numpy()
    assert _rel_inf(y, AT @ x) <= 1e-12
    GT = sgheat.problem_from_workload(w, transpose=1)
    y2 = GT.apply(_to_gpu(torch, x)).cpu().numpy()
    assert _rel_inf(y2, AT @ x) <= 1e-12
    y3 = GT.apply_T(_to_gpu(torch, x)).cpu().numpy()          # back to AA
    assert _rel_inf(y3, P.apply_route1(x)) <= 1e-12


@pytest.mark.parametrize("name", ["c1", "t3q2"])
def test_adjoint_handle_solve(torch_cuda, name):
    from paper_2605_21046_amd import sgheat
    torch = torch_cuda
    w = sg_inputs.WORKLOADS[name]
    print(f"adjoint solve {name}", flush=True)
    P = from_workload(w)
    AT = P.assemble_full().T.tocsr()
    b = _interior_vector(P, 12)
    GT = sgheat.problem_from_workload(w, transpose=1)
    x, info = GT.solve(_to_gpu(torch, b), rtol=1e-10)
    xh = x.cpu().numpy()
    assert np.linalg.norm(b - AT @ xh) / np.linalg.norm(b) <= 1.0001e-10
    assert info["iterations"] <= 30


@pytest.mark.parametrize("name", SMALL)
@pytest.mark.parametrize("transpose", [False, True])
def test_slab_transfer_matches_oracle(torch_cuda, name, transpose):
    from paper_2605_21046_amd import sgheat
    torch = torch_cuda
    w = sg_inputs.WORKLOADS[name]
    P = from_workload(w)
    JJ = adj.transfer_matrix(P)
    if transpose:
        JJ = JJ.T.tocsr()
    x = _interior_vector(P, 13)
    G = sgheat.problem_from_workload(w)
    y = G.slab_transfer(_to_gpu(torch, x), transpose=transpose).cpu().numpy()
    assert _rel_inf(y, JJ @ x) <= 1e-12


@pytest.mark.parametrize("name", ["c1", "t3q2"])
def test_stiffness_forms_match_oracle(torch_cuda, name):
    from paper_2605_21046_amd import sgheat
    torch = torch_cuda
    w = sg_inputs.WORKLOADS[name]
    P = from_workload(w)
    G = sgheat.problem_from_workload(w)
    lam, u = _interior_vector(P, 14), _interior_vector(P, 15)
    pts = P.mesh.qp_coords()
    fields = [np.ones((P.mesh.n_cells, P.mesh.nq))] + [sg_inputs.sine_shape_at(m, pts) for m in range(1, w.n_vars + 1)]
    for mu_index, mu in enumerate(P.coef_mu):
        Gm = chaos.galerkin_tensor(mu, P.index_set)
        ref = adj.cell_forms(P, lam, u, Gm, fields[mu_index])
        got = G.stiffness_form_cells(mu_index, fields[mu_index], _to_gpu(torch, lam), _to_gpu(torch, u))
        assert _rel_inf(got.cpu().numpy(), ref) <= 1e-12


@pytest.mark.parametrize("name", ["c1", "t3q2"])
def test_stiffness_form_accumulate_and_field_cache(torch_cuda, name):
    """Device accumulation of the forms over a sequence of calls that revisit modes, change a field and
    give it back: every per-cell result against the oracle (1e-12), the accumulated cells and total
    against the oracle's sums (1e-12 of the summed magnitudes)."""
    from paper_2605_21046_amd import sgheat
    torch = torch_cuda
    w = sg_inputs.WORKLOADS[name]
    P = from_workload(w)
    G = sgheat.problem_from_workload(w)
    lam, u = _interior_vector(P, 24), _interior_vector(P, 25)
    lg, ug = _to_gpu(torch, lam), _to_gpu(torch, u)
    pts = P.mesh.qp_coords()
    fields = [np.ones((P.mesh.n_cells, P.mesh.nq))] + [sg_inputs.sine_shape_at(m, pts) for m in range(1, w.n_vars + 1)]
    calls = [(i, fields[i]) for i in range(len(P.coef_mu))]
    calls += [(1, 2.0 * fields[1]), (0, 0.5 * fields[0] + 1.0), (1, fields[1]), (len(P.coef_mu) - 1, fields[-1])]
    cells = torch.zeros(P.mesh.n_cells, dtype=torch.float64, device="cuda")
    total = torch.zeros(1, dtype=torch.float64, device="cuda")
    exp_cells = np.zeros(P.mesh.n_cells)
    mag = np.zeros(P.mesh.n_cells)
    for k, (i, f) in enumerate(calls):
        print(f"form accumulate {name} call {k} mode {i}", flush=True)
        ref = adj.cell_forms(P, lam, u, chaos.galerkin_tensor(P.coef_mu[i], P.index_set), f)
        got = G.stiffness_form_cells(i, f, lg, ug).cpu().numpy()
        assert _rel_inf(got, ref) <= 1e-12
        scale = (-1.0) ** k * (1.0 + 0.25 * k)
        G.stiffness_form_accumulate(i, f, lg, ug, scale, cells=cells, total=total)
        exp_cells += scale * ref
        mag += np.abs(scale * ref)
    assert np.abs(cells.cpu().numpy() - exp_cells).max() <= 1e-12 * mag.max()
    assert abs(total.item() - exp_cells.sum()) <= 1e-12 * mag.sum()
    with pytest.raises(sgheat.SgError):
        G.stiffness_form_accumulate(0, fields[0], lg, ug, 1.0)


@pytest.mark.parametrize("name", ["c1", "t3q2"])
def test_qoi_and_gradient_match_oracle(torch_cuda, name):
    from paper_2605_21046_amd import sgheat
    torch = torch_cuda
    w = sg_inputs.WORKLOADS[name]
    P = from_workload(w)
    G = sgheat.problem_from_workload(w)
    u = _interior_vector(P, 16)
    EQ, VQ, g = adj.qoi(P, u, w.n_vars, w.chaos_degree, 0.7, 1.3)
    gg = torch.zeros(P.n, dtype=torch.float64, device="cuda")
    e, v = G.qoi_mean_var(_to_gpu(torch, u), 0.7, 1.3, grad=gg)
    assert e == pytest.approx(EQ, rel=1e-12)
    assert v == pytest.approx(VQ, rel=1e-11)
    assert _rel_inf(gg.cpu().numpy(), g) <= 1e-12


@pytest.mark.parametrize("name", ["a2", "a3"])
def test_adjoint_gradient_matches_oracle(torch_cuda, name):
    from paper_2605_21046_amd.adjoint import SlabSequence
    aw = sg_inputs.ADJOINT_WORKLOADS[name]
    print(f"adjoint gradient {name}", flush=True)
    th, a0 = aw.theta0(), aw.a0_cells0()
    J0, (E0, V0), dth0, da00 = adj.gradient(aw, th, a0)
    seq = SlabSequence(aw, rtol=1e-12)
    J, (E, V), dth, da0 = seq.gradient(th, a0)
    seq.close()
    assert J == pytest.approx(J0, rel=1e-9)
    assert V == pytest.approx(V0, rel=1e-7)
    assert np.max(np.abs(dth - dth0)) <= 1e-7 * np.max(np.abs(dth0))
    assert np.max(np.abs(da0 - da00)) <= 1e-7 * np.max(np.abs(da00))


def test_autograd_function_returns_the_adjoint_gradient(torch_cuda):
    from paper_2605_21046_amd.adjoint import SlabSequence, make_function
    torch = torch_cuda
    aw = sg_inputs.ADJOINT_WORKLOADS["a2"]
    seq = SlabSequence(aw, rtol=1e-12)
    th = torch.tensor(aw.theta0(), dtype=torch.float64, requires_grad=True)
    a0 = torch.tensor(aw.a0_cells0(), dtype=torch.float64, requires_grad=True)
    J = make_function().apply(th, a0, seq)
    J.backward()
    _, _, dth, da0 = adj.gradient(aw, aw.theta0(), aw.a0_cells0())
    seq.close()
    assert np.max(np.abs(th.grad.numpy() - dth)) <= 1e-7 * np.max(np.abs(dth))
    assert np.max(np.abs(a0.grad.numpy() - da0)) <= 1e-7 * np.max(np.abs(da0))


def test_autograd_backward_after_a_second_forward(torch_cuda):
    """Two evaluations of J before backward: each backward returns the gradient at its own
    parameters (the second forward moved the handles' coefficients and checkpoints)."""
    from paper_2605_21046_amd.adjoint import SlabSequence, make_function
    torch = torch_cuda
    aw = sg_inputs.ADJOINT_WORKLOADS["a2"]
    seq = SlabSequence(aw, rtol=1e-12)
    f = make_function()
    th1 = torch.tensor(aw.theta0(), dtype=torch.float64, requires_grad=True)
    a01 = torch.tensor(aw.a0_cells0(), dtype=torch.float64, requires_grad=True)
    th2 = torch.tensor(1.7 * aw.theta0(), dtype=torch.float64, requires_grad=True)
    a02 = torch.tensor(aw.a0_cells0() + 0.1, dtype=torch.float64, requires_grad=True)
    J1 = f.apply(th1, a01, seq)
    J2 = f.apply(th2, a02, seq)
    J1.backward()
    J2.backward()
    seq.close()
    for th, a0, J in ((th1, a01, J1), (th2, a02, J2)):
        Jo, _, dth, da0 = adj.gradient(aw, th.detach().numpy(), a0.detach().numpy())
        assert float(J.detach()) == pytest.approx(Jo, rel=1e-9)
        assert np.max(np.abs(th.grad.numpy() - dth)) <= 1e-7 * np.max(np.abs(dth))
        assert np.max(np.abs(a0.grad.numpy() - da0)) <= 1e-7 * np.max(np.abs(da0))


def test_full_size_gradient_against_central_differences(torch_cuda):
    """16^3 cells, 10 slabs, 20 modes: the adjoint gradient against central differences of J."""
    from paper_2605_21046_amd.adjoint import SlabSequence
    aw = sg_inputs.ADJOINT_WORKLOADS["c5"]
    print("adjoint full size c5", flush=True)
    th, a0 = aw.theta0(), aw.a0_cells0()
    seq = SlabSequence(aw, rtol=1e-11)
    J, _, dth, da0 = seq.gradient(th, a0)
    h = 1e-5
    tp, tm = th.copy(), th.copy()
    tp[0] += h
    tm[0] -= h
    fd = (seq.forward(tp, a0)[0] - seq.forward(tm, a0)[0]) / (2 * h)
    assert dth[0] == pytest.approx(fd, rel=1e-4)
    c = int(np.argmax(np.abs(da0)))
    ap, am = a0.copy(), a0.copy()
    ap[c] += h
    am[c] -= h
    fd = (seq.forward(th, ap)[0] - seq.forward(th, am)[0]) / (2 * h)
    seq.close()
    assert da0[c] == pytest.approx(fd, rel=1e-4)
