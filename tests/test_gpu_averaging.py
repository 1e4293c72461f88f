"""The two alignment averages of the averaging workload (Eq. 5 with ten
fixed angles, Eq. 6 with the axis sampled per trajectory) against the
oracle, through one batched plan and the step-wise path."""
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
NTHREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def sf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2608_13686_amd as sf
    return sf


def rel(a, b):
    r = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    print(f"relative L2 {r:.3e}", flush=True)
    return r


def test_joint_isotropic_average_matches_oracle(sf, orc):
    import torch
    p = W.workload_averaging("H2")["joint"]
    out = sf.run([p], [3000], [55], h_max=10.0)
    torch.cuda.synchronize()
    vo, _, _ = orc.dipole(p, 55, 0, 3000, NTHREADS)
    assert rel(out["v"][0].cpu().numpy(), vo) < 1e-10


def test_standard_ten_angle_average_matches_oracle(sf, orc):
    import torch
    probs, wts = W.workload_averaging("H2")["standard"]
    n, seeds = [300] * len(probs), [400 + i for i in range(len(probs))]
    plan = sf.Plan(probs, n, seeds, tuning=(1, 8, 1, 1), h_max=10.0)
    plan.run()
    torch.cuda.synchronize()
    v = sum(w * plan.v_of(i).cpu().numpy() for i, w in enumerate(wts))
    vo = sum(w * orc.dipole(p, s, 0, 300, NTHREADS)[0] for p, s, w in zip(probs, seeds, wts))
    assert rel(v, vo) < 1e-10
    plan.close()
