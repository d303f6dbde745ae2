"""Parity of the member-batch path (independent SG problems of mixed chaos degree in one handle) and
of the chaos-moment kernel with the FP64 CPU oracle, on an MI355X.

Tolerances:
  * batch operator apply (one kernel pass, FP64): 1e-12 relative to each member's oracle block;
  * chaos moments (copy and a sum of squares, FP64): 1e-12 relative;
  * slab sequence (rtol 1e-12 per slab solve): 1e-9 relative per member on the small cases;
  * 64 members on 64^2 cells, 20 slabs (rtol 1e-10 on each handle's whole residual): the last slab
    of sampled members satisfies the oracle's slab equation AA U^(20) = JJ U^(19) to a relative
    residual of 1e-9 (a member's share of the handle's residual, relative to its own right-hand side,
    is at most 1e-10 * ||b_handle|| / ||b_member||, about 1e-10 * sqrt(members per handle) here).
"""
import math

import numpy as np
import pytest

import sg_inputs
from oracle import adjoint as adj
from oracle import members as mb

pytestmark = pytest.mark.gpu


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


def _one_handle(mw, precision=0):
    """All members of a small workload in a single handle."""
    from paper_2605_21046_amd import sgheat
    w = mw.base
    spec = sgheat.Spec(w.dim, w.n_cells_1d, w.fe_degree, w.time_degree, w.tau, w.n_vars, 0, w.n_levels, w.lo, w.hi)
    mus, coef = sg_inputs.coef_qp_levels(w, lambda lvl: sgheat.quadrature_points(spec, lvl))
    return sgheat.Problem(spec, mus, coef, precision, members=(list(mw.degrees), mw.scales(mus)))


def _split(mw, x):
    modes = [math.comb(mw.base.n_vars + p, p) for p in mw.degrees]
    per = x.size // sum(modes)
    out, off = [], 0
    for m in modes:
        out.append(x[off * per:(off + m) * per])
        off += m
    return out


@pytest.mark.parametrize("name", ["b2", "b3"])
def test_member_batch_apply_matches_oracle(torch_cuda, name):
    torch = torch_cuda
    mw = sg_inputs.MEMBER_WORKLOADS[name]
    print(f"member-batch apply {name}", flush=True)
    G = _one_handle(mw)
    x = sg_inputs.uniform_vector(G.n(0), 31)
    y = G.apply(_to_gpu(torch, x)).cpu().numpy()
    G.close()
    for j, (xj, yj) in enumerate(zip(_split(mw, x), _split(mw, y))):
        P = mb.member_problem(mw, j)
        assert _rel_inf(yj, P.assemble_full() @ xj) <= 1e-12


@pytest.mark.parametrize("name", ["b2", "b3"])
def test_chaos_moments_match_oracle(torch_cuda, name):
    torch = torch_cuda
    mw = sg_inputs.MEMBER_WORKLOADS[name]
    G = _one_handle(mw)
    u = sg_inputs.uniform_vector(G.n(0), 32)
    J = len(mw.degrees)
    m = J * G.shape[1] * G.shape[2]
    mean, var = G.chaos_moments(_to_gpu(torch, u), var=torch.empty(m, dtype=torch.float64, device="cuda"))
    G.close()
    mean = mean.cpu().numpy().reshape(J, -1)
    var = var.cpu().numpy().reshape(J, -1)
    for j, uj in enumerate(_split(mw, u)):
        e, v = mb.chaos_moments(uj, math.comb(mw.base.n_vars + mw.degrees[j], mw.degrees[j]))
        assert _rel_inf(mean[j], e) <= 1e-12
        if mw.degrees[j] == 0:
            assert np.all(var[j] == 0.0)
        else:
            assert _rel_inf(var[j], v) <= 1e-12


def test_chaos_moments_of_a_plain_handle(torch_cuda):
    from paper_2605_21046_amd import sgheat
    from oracle.slab import from_workload
    torch = torch_cuda
    w = sg_inputs.WORKLOADS["t2q2"]
    G = sgheat.problem_from_workload(w)
    u = sg_inputs.uniform_vector(G.n(0), 33)
    m = G.shape[1] * G.shape[2]
    mean, var = G.chaos_moments(_to_gpu(torch, u), var=torch.empty(m, dtype=torch.float64, device="cuda"))
    G.close()
    e, v = mb.chaos_moments(u, from_workload(w).n_xi)
    assert _rel_inf(mean.cpu().numpy(), e) <= 1e-12
    assert _rel_inf(var.cpu().numpy(), v) <= 1e-12


@pytest.mark.parametrize("name", ["b2", "b3"])
def test_member_sequences_match_oracle(torch_cuda, name):
    from paper_2605_21046_amd.sgbatch import MemberBatch
    mw = sg_inputs.MEMBER_WORKLOADS[name]
    print(f"member-batch sequence {name}", flush=True)
    B = MemberBatch(mw, rtol=1e-12)
    us = B.run()
    mean, var = B.moments(us)
    got = [B.member_vector(us, j).cpu().numpy() for j in range(len(mw.degrees))]
    mean, var = mean.cpu().numpy(), var.cpu().numpy()
    B.close()
    for j in range(len(mw.degrees)):
        ref = mb.member_sequence(mw, j)[-1]
        assert _rel_inf(got[j], ref) <= 1e-9
        e, v = mb.chaos_moments(ref, B.modes[j])
        assert _rel_inf(mean[j].reshape(-1), e) <= 1e-9
        if mw.degrees[j] > 0:
            assert _rel_inf(var[j].reshape(-1), v) <= 1e-8


def test_member_scale_of_the_mean_mode_must_be_one(torch_cuda):
    from paper_2605_21046_amd import sgheat
    mw = sg_inputs.MEMBER_WORKLOADS["b2"]
    w = mw.base
    spec = sgheat.Spec(w.dim, w.n_cells_1d, w.fe_degree, w.time_degree, w.tau, w.n_vars, 0, w.n_levels, w.lo, w.hi)
    mus, coef = sg_inputs.coef_qp_levels(w, lambda lvl: sgheat.quadrature_points(spec, lvl))
    sc = mw.scales(mus)
    sc[1, 0] = 1.5
    with pytest.raises(sgheat.SgError, match="SG_EINVAL"):
        sgheat.Problem(spec, mus, coef, members=(list(mw.degrees), sc))


def test_full_size_member_batch_satisfies_the_oracle_slab_equation(torch_cuda):
    """64 members (16 each of degree 1..4) on 64^2 Q2 cells, 20 slabs: the last slab of one member
    of each degree against the oracle's assembled AA and JJ."""
    from paper_2605_21046_amd.sgbatch import MemberBatch
    mw = sg_inputs.MEMBER_WORKLOADS["c4"]
    print("member-batch full size c4", flush=True)
    B = MemberBatch(mw, rtol=1e-10)
    assert len(B.handles) == 3
    us = B.run(keep_previous=True)
    for j in [0, 17, 34, 51]:                  # degrees 1, 2, 3, 4
        u = B.member_vector(us, j).cpu().numpy()
        up = B.member_vector(B.previous, j).cpu().numpy()
        P = mb.member_problem(mw, j)
        rhs = adj.transfer_matrix(P) @ up
        r = P.assemble_full() @ u - rhs
        print(f"member {j} (degree {mw.degrees[j]}): relative residual {np.linalg.norm(r) / np.linalg.norm(rhs):.2e}",
              flush=True)
        assert np.linalg.norm(r) <= 1e-9 * np.linalg.norm(rhs)
    B.close()
