"""Approximate dispersion relation (Sec. 3.2, eq. 22-28) of the oracle's
scheme: the modified wavenumber k(alpha) = FT(h u')/FT(u) of a cosine wave on
a periodic grid, u' = -R for c = 1.  Pins: the linear scheme's ADR is its
Fourier symbol; at xi = 1e6 the FE map returns the ideal weights on smooth
waves, so the ADR equals the linear symbol exactly at low wavenumbers (and
further than the Z weights do); and the paper's Fig. 5-6 observations:
overshoot of the dispersion at kappa = 0.3 (xi = 1e6) and at xi = 10, none
to speak of for xi >= 100 at kappa = 0.5."""
import numpy as np
import pytest

from test_oracle_scheme import _symbol


def adr_oracle(ora, n, **kw):
    modes = np.arange(1, n // 2 + 1)
    rows = max(len(modes), 9)
    m_rows = np.resize(modes, rows)
    j = np.arange(n)
    U = np.cos((2 * np.pi * m_rows / n)[:, None] * j[None, :])[None].copy()
    P = ora.Problem(system="advection", ndim=2, n=(n, rows), h=(1.0, 1.0), adv=(1.0, 0.0),
                    bc="periodic", **kw)
    R = P.residual(U)[0]
    idx = np.arange(rows)
    k = np.fft.fft(-R, axis=1)[idx, m_rows] / np.fft.fft(U[0], axis=1)[idx, m_rows]
    return 2 * np.pi * modes / n, k[: len(modes)]


def test_linear_adr_is_the_symbol(ora):
    a, k = adr_oracle(ora, 64, weights="linear")
    assert np.abs(k - _symbol(a)).max() < 1e-13


def test_fe_adr_equals_linear_symbol_at_low_wavenumbers(ora):
    a, kfe = adr_oracle(ora, 64, weights="fe", xi=1e6, kappa=0.5)
    _, kz = adr_oracle(ora, 64, weights="z", xi=1e6)
    low = a <= 0.49
    assert np.abs(kfe[low] - _symbol(a[low])).max() < 1e-13
    assert np.abs(kz[low] - _symbol(a[low])).max() > 1e-10   # Z leaves the ideal weights earlier


@pytest.mark.parametrize("kappa,xi,overshoot", [(0.3, 1e6, True), (0.4, 1e6, True), (0.5, 10.0, True),
                                                (0.5, 100.0, False), (0.5, 1e6, False)])
def test_dispersion_overshoot_of_fig5_fig6(ora, kappa, xi, overshoot):
    a, k = adr_oracle(ora, 64, weights="fe", xi=xi, kappa=kappa)
    over = float(np.max(k.imag - a))
    assert (over > 5e-3) if overshoot else (over < 1e-4), over
