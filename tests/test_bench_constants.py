"""The algorithmic flop counts that bench.py prices its roofline with are the
oracle's operation tally (each +, -, x, /, sqrt and tanh once) of one
residual per node of a 512-node Sod tube, plus 15 for the stage combine."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.mark.parametrize("weights", ["fe", "js", "z", "pfe", "linear"])
def test_flops_per_point_stage_match_oracle_tally(ora, W, weights):
    import bench
    _, U, _ = W.shock_tube(1.0, 0.75, 1.0, 0.125, 0.0, 0.1, 512)
    P = ora.Problem(system="euler", ndim=1, n=(512,), h=(1.0 / 511,), weights=weights, xi=100.0,
                    kappa=0.5, zpow=2, eps=1e-40, diff="mnd6", charproj=True, gamma=1.4,
                    bc="transmissive")
    c = P.count_residual_ops(U)
    assert sum(c.values()) / 512 + 15 == bench.FLOPS_PER_POINT_STAGE[weights]


@pytest.mark.parametrize("gpus", ["2", "8"])
def test_bench_refuses_more_than_one_gpu(gpus):
    """bench.py measures one GPU: --gpus N > 1 exits with status 2 and says
    so, before anything touches a device."""
    import subprocess
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", gpus],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout.strip()
