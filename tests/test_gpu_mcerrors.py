"""Parity of the Monte-Carlo error split (pathwise forcing, quadrature-point estimators, total /
discretisation / sampling errors) with the FP64 CPU oracle, on an MI355X.

Tolerances: slab solves to rtol 1e-12, so the six errors agree with the oracle's (direct solves) to
1e-8 relative; the pure sampling errors involve no solve (1e-12).  Several handles feed one estimate
(e2: 6 samples in two handles of 3).  At full size (c6: 512 samples on 32^2 Q3 cells, dG(3), 16 slabs,
four handles) the split's triangle inequalities and the closed-form sampling errors are checked.
"""
import math

import numpy as np
import pytest

import sg_inputs
from oracle import mcerrors as me

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("name", ["e2", "e3"])
def test_error_split_matches_oracle(torch_cuda, name):
    from paper_2605_21046_amd.mcerrors import MCErrorStudy
    ew = sg_inputs.MC_ERROR_WORKLOADS[name]
    print(f"MC error split {name}", flush=True)
    S = MCErrorStudy(ew, rtol=1e-12)
    assert len(S.handles) == math.ceil(ew.n_samples / ew.batch)
    got = S.run()
    S.close()
    ref = me.error_split(ew)
    for key in ["tot_mean", "disc_mean", "tot_var", "disc_var"]:
        assert got[key] == pytest.approx(ref[key], rel=1e-8), key
    for key in ["mc_mean", "mc_var"]:
        assert got[key] == pytest.approx(ref[key], rel=1e-10), key


def test_cumulative_windows_match_oracle(torch_cuda):
    """Every window of the first k handles equals the oracle's split over those samples."""
    from paper_2605_21046_amd.mcerrors import MCErrorStudy
    ew = sg_inputs.MC_ERROR_WORKLOADS["e2"]
    S = MCErrorStudy(ew, rtol=1e-12)
    rows = S.run(windows=True)
    S.close()
    xs = ew.samples()
    assert [r["N"] for r in rows] == [3, 6]
    for r in rows:
        ref = me.error_split(ew, xs[: r["N"]])
        for key in ["tot_mean", "disc_mean", "tot_var", "disc_var"]:
            assert r[key] == pytest.approx(ref[key], rel=1e-8), (r["N"], key)
        for key in ["mc_mean", "mc_var"]:
            assert r[key] == pytest.approx(ref[key], rel=1e-10), (r["N"], key)


def test_full_size_error_split_properties(torch_cuda):
    from paper_2605_21046_amd.mcerrors import MCErrorStudy
    ew = sg_inputs.MC_ERROR_WORKLOADS["c6"]
    print("MC error split full size c6", flush=True)
    S = MCErrorStudy(ew, rtol=1e-10)
    got = S.run()
    its = [i["iterations"] for i in S.info]
    g = me.g_q_many(ew.samples())
    S.close()
    print(got, f"iterations per slab {min(its)}..{max(its)}", flush=True)
    assert got["tot_mean"] <= got["disc_mean"] + got["mc_mean"] + 1e-15
    assert got["tot_var"] <= got["disc_var"] + got["mc_var"] + 1e-15
    assert got["mc_mean"] == pytest.approx(abs(np.mean(g) - 1.0) / 3.0, rel=1e-8)
    assert got["disc_mean"] < 1e-3 * got["mc_mean"]
