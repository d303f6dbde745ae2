"""The allocation-free operator apply (sg_operator_apply_noalloc) against sg_operator_apply, through the
C ABI, on an MI355X: two calls in a row, the second on a smaller problem than the first (the shared
scratch still holds the first call's cell-local results), each bitwise equal to the regular apply of the
same handle (the same kernels write the same layout, so the rounding is the same) and within 1e-12 of
the oracle's operator; a problem whose cell-local results exceed the 64 MiB scratch is rejected before
anything is enqueued."""
import numpy as np
import pytest

import sg_inputs
from oracle.slab import from_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_noalloc_apply_matches_the_regular_apply_on_two_calls(torch_cuda):
    torch = torch_cuda
    from paper_2605_21046_amd import sgheat
    # 3D Q2 dG(1) with the 35-mode index set on 10^3 cells, then the smaller 2D Q3 workload
    for name in ("t3c2", "t2q3"):
        w = sg_inputs.WORKLOADS[name]
        print(f"no-alloc apply {name}", flush=True)
        G = sgheat.problem_from_workload(w)
        P = from_workload(w)
        x = sg_inputs.uniform_vector(P.n, sg_inputs.SEED_APPLY_INPUT)
        xg = torch.from_numpy(x).to("cuda")
        y_ref = G.apply(xg)
        y = torch.full_like(xg, float("nan"))
        G.apply_noalloc(xg, y)
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref)
        yo = P.apply_route2(x)
        assert np.abs(y.cpu().numpy() - yo).max() <= 1e-12 * np.abs(yo).max()
        G.close()


def test_noalloc_apply_rejects_problems_beyond_the_scratch(torch_cuda):
    torch = torch_cuda
    from paper_2605_21046_amd import sgheat
    # 35 modes x 2 time DoFs x 20^3 cells x 27 points x 8 B = 121 MB of cell-local results > 64 MiB
    w = sg_inputs.WORKLOADS["t3c2"].with_(name="t3c2big", n_cells_1d=20, n_levels=3, tau=1.0 / 20)
    G = sgheat.problem_from_workload(w)
    x = torch.zeros(G.n(0), dtype=torch.float64, device="cuda")
    y = torch.full_like(x, 7.0)
    with pytest.raises(sgheat.SgError) as e:
        G.apply_noalloc(x, y)
    assert "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((y == 7.0).all())
    G.close()
