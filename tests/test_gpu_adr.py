"""The GPU ADR tool (paper_2306_09760_amd.adr) against the same analysis of
the oracle's residuals."""
import numpy as np
import pytest
import torch

from gpu_util import say
from test_oracle_adr import adr_oracle

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [64, 256])
@pytest.mark.parametrize("weights,xi,kappa", [("fe", 1e6, 0.5), ("fe", 100.0, 0.5), ("fe", 1e6, 0.3),
                                              ("fe", 10.0, 0.5), ("z", 1e6, 0.5), ("linear", 1e6, 0.5)])
def test_adr_matches_oracle(ora, n, weights, xi, kappa):
    from paper_2306_09760_amd import adr
    assert torch.cuda.is_available()
    a, kr, ki = adr.adr(n, weights=weights, xi=xi, kappa=kappa)
    ao, ko = adr_oracle(ora, n, weights=weights, xi=xi, kappa=kappa)
    err = np.max(np.abs(kr + 1j * ki - ko))
    say("adr", n, weights, xi, kappa, "max |k_gpu - k_oracle|", err, adr.summary(a, kr, ki))
    assert np.array_equal(a, ao) and err < 1e-12
