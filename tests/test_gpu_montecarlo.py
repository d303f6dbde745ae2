"""Parity of the sample-batch (Monte-Carlo pathwise) path with the FP64 CPU oracle, on an MI355X.

The batch handle holds every sample's slab system as one row block; the oracle solves each sample
on its own (one chaos mode, the sampled coefficient).

Tolerances:
  * batch operator apply (one kernel pass, FP64): 1e-12 relative to the oracle's block of each sample;
  * batch FGMRES: true relative residual <= rtol, recomputed by the oracle per block;
  * sample mean and unbiased variance (FP64, two passes over the samples): 1e-12 relative;
  * slab sequence (rtol 1e-12 per slab solve): 1e-9 relative per sample on the small cases; 1e-8 on
    the 64^2-cell, 20-slab batch (one sample checked against the oracle's solve, the error of the
    iterative solves enters linearly and is damped slab to slab).
"""
import numpy as np
import pytest

import sg_inputs
from oracle import montecarlo as mc

pytestmark = pytest.mark.gpu

SMALL = ["m2", "m3", "m2q3"]


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


def _blocks(sw):
    return [mc.pathwise_problem(sw.base, xi) for xi in sw.samples()]


@pytest.mark.parametrize("name", SMALL)
def test_batch_apply_matches_per_sample_oracle(torch_cuda, name):
    from paper_2605_21046_amd.montecarlo import SampleBatch
    torch = torch_cuda
    sw = sg_inputs.SAMPLE_WORKLOADS[name]
    print(f"sample-batch apply {name}", flush=True)
    B = SampleBatch(sw)
    x = sg_inputs.uniform_vector(B.P.n(0), 21)
    y = B.P.apply(_to_gpu(torch, x)).cpu().numpy().reshape(B.n_s, -1)
    xs = x.reshape(B.n_s, -1)
    for s, P in enumerate(_blocks(sw)):
        assert _rel_inf(y[s], P.assemble_full() @ xs[s]) <= 1e-12
    B.close()


@pytest.mark.parametrize("name", ["m2", "m3"])
@pytest.mark.parametrize("precision", [0, 1])
def test_batch_solve_residual(torch_cuda, name, precision):
    from paper_2605_21046_amd.montecarlo import SampleBatch
    torch = torch_cuda
    sw = sg_inputs.SAMPLE_WORKLOADS[name]
    print(f"sample-batch solve {name} precision {precision}", flush=True)
    B = SampleBatch(sw, precision=precision)
    blocks = _blocks(sw)
    b = sg_inputs.uniform_vector(B.P.n(0), 22).reshape(B.n_s, -1)
    for s, P in enumerate(blocks):
        b[s][P.full_boundary_mask()] = 0.0
    x, info = B.P.solve(_to_gpu(torch, b.reshape(-1)), rtol=1e-10)
    assert info["converged"]
    xh = x.cpu().numpy().reshape(B.n_s, -1)
    r2 = sum(np.sum((b[s] - P.assemble_full() @ xh[s]) ** 2) for s, P in enumerate(blocks))
    assert np.sqrt(r2) / np.linalg.norm(b) <= 1.0001e-10
    B.close()


@pytest.mark.parametrize("name", SMALL)
def test_sample_statistics_match_the_estimators(torch_cuda, name):
    from paper_2605_21046_amd.montecarlo import SampleBatch
    torch = torch_cuda
    sw = sg_inputs.SAMPLE_WORKLOADS[name]
    B = SampleBatch(sw)
    u = sg_inputs.uniform_vector(B.P.n(0), 23)
    mean, var = B.statistics(_to_gpu(torch, u))
    U = u.reshape(B.n_s, -1)
    assert _rel_inf(mean.cpu().numpy().reshape(-1), mc.sample_mean(U)) <= 1e-12
    assert _rel_inf(var.cpu().numpy().reshape(-1), mc.sample_variance(U)) <= 1e-12
    B.close()


@pytest.mark.parametrize("name", SMALL)
def test_slab_sequence_matches_pathwise_oracle(torch_cuda, name):
    from paper_2605_21046_amd.montecarlo import SampleBatch
    sw = sg_inputs.SAMPLE_WORKLOADS[name]
    print(f"sample-batch sequence {name}", flush=True)
    B = SampleBatch(sw, rtol=1e-12)
    u = B.run()
    got = u.cpu().numpy().reshape(B.n_s, -1)
    mean, var = B.statistics(u)
    B.close()
    ref = mc.batch_final_slabs(sw)
    for s in range(sw.n_samples):
        assert _rel_inf(got[s], ref[s]) <= 1e-9
    assert _rel_inf(mean.cpu().numpy().reshape(-1), mc.sample_mean(ref)) <= 1e-9
    assert _rel_inf(var.cpu().numpy().reshape(-1), mc.sample_variance(ref)) <= 1e-7


def test_nonpositive_sample_is_rejected(torch_cuda):
    from paper_2605_21046_amd import sgheat
    from paper_2605_21046_amd.montecarlo import SampleBatch
    sw = sg_inputs.SAMPLE_WORKLOADS["m2"]
    xs = sw.samples().copy()
    xs[3, 0] = -40.0                      # a = 1 - 4 sin(pi x) sin(pi y) + ... < 0 near the centre
    with pytest.raises(sgheat.SgError, match="SG_EINVAL"):
        SampleBatch(sw, samples=xs)


def test_full_size_batch_one_sample_against_oracle(torch_cuda):
    """256 samples, 2D Q2 64^2 cells, dG(1), 20 slabs: the sample with the largest |xi| vs the oracle."""
    from paper_2605_21046_amd.montecarlo import SampleBatch
    torch = torch_cuda
    sw = sg_inputs.SAMPLE_WORKLOADS["c4"]
    print("sample-batch full size c4", flush=True)
    B = SampleBatch(sw, rtol=1e-12)
    u = B.run()
    got = u.view(B.n_s, -1)
    mean, var = B.statistics(u)
    assert torch.allclose(mean.view(-1), got.mean(dim=0), rtol=1e-12, atol=1e-15)
    assert torch.allclose(var.view(-1), got.var(dim=0, unbiased=True), rtol=1e-10, atol=1e-18)
    s = int(np.argmax(np.linalg.norm(B.samples, axis=1)))
    B.close()
    ref = mc.pathwise_sequence(sw, sw.samples()[s])[-1]
    assert _rel_inf(got[s].cpu().numpy(), ref) <= 1e-8
