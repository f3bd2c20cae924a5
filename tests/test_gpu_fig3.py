"""Synthetic analogue of the paper's Fig. 3 (Sec. 4) on the device: one macro-particle
with a single electron (N = 1), all-coherent (point shape, N^2), all-incoherent (g = 0, N)
and Gaussian form-factor (Eq. 12) weightings.  Each device spectrum is checked against the
oracle on the same inputs (parity gate, per frequency); then the ratios to the one-electron
spectrum against N^2, N and Eq. 12, and the coherent -> incoherent transition frequency
against its closed form."""
import numpy as np
import pytest

import oracle
from workloads import Fig3Analogue, flatten
from tests.helpers import assert_parity, to_device

pytestmark = pytest.mark.gpu

C = 299792458.0


@pytest.fixture(scope="module")
def rad():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1802_03972_amd as rad
    from paper_1802_03972_amd.build import ensure_built
    ensure_built()    # a built library is used as is
    rad._lib.lib()
    return rad


def test_fig3_analogue_against_oracle_and_scalings(rad):
    f = Fig3Analogue()
    w = f.workload
    dirs, om = f.directions(), f.omegas()
    N, sigma = f.electrons, f.sigma
    runs = {"single electron": ("point", 0.0, 1.0), "coherent": ("point", 0.0, N),
            "incoherent": ("gauss", 1.0, N), "form factor": ("gauss", sigma, N)}
    I = {}
    for name, (shape, length, weight) in runs.items():
        st = f.trajectory(weight)
        g = rad.Grid(dirs, 0.0, 0.0, 0, shape=shape, shape_len=length, dt=w.dt, omegas=om)
        g.push_steps(w.t0, w.n_steps, to_device(st, "f64"))
        I[name] = g.spectrum()
        Iref = oracle.spectrum(flatten(st, w.times()), dirs, om, shape, length, w.dt)
        assert_parity(I[name], Iref, f"Fig. 3 analogue, {name}")
    I1 = I["single electron"]
    g_ref = np.exp(-(om * sigma / C) ** 2)
    F2 = N + (N * N - N) * g_ref
    assert np.max(np.abs(I["coherent"] / I1 / N ** 2 - 1)) <= 1e-4
    assert np.max(np.abs(I["incoherent"] / I1 / N - 1)) <= 1e-4
    ratio = I["form factor"] / I1
    assert np.max(np.abs(ratio / F2 - 1)) <= 1e-4
    # transition F^2 = 2N, interpolated in log(omega) on the on-axis spectrum
    y = np.log(ratio[0] / (2 * N))
    k = int(np.argmax(y < 0))
    t = y[k - 1] / (y[k - 1] - y[k])
    om_t = float(np.exp(np.log(om[k - 1]) + t * (np.log(om[k]) - np.log(om[k - 1]))))
    om_t_ref = C / sigma * np.sqrt(np.log(N - 1))
    print(f"transition omega {om_t:.4e}, closed form {om_t_ref:.4e}")
    assert abs(om_t / om_t_ref - 1) <= 0.01
