"""A push of more than 2^31 particles (86 GB of FP32 particle data resident in HBM): particle
indices, chunk ranges and launch cutting are 64-bit throughout.  The particles repeat one
seeded period of 1000 at one time step, so the exact spectrum is (n / 1000)^2 times the
oracle's spectrum of the period; the same data pushed as two halves (each below 2^31
elements) must agree with the single push to FP32 rounding."""
import numpy as np
import pytest

import oracle
from workloads import SINGLE, FIELDS, flatten
from tests.helpers import assert_close, assert_parity

pytestmark = pytest.mark.gpu

PERIOD = 1000
COPIES = 2147484          # 2,147,484,000 particles > 2^31


@pytest.fixture(scope="module")
def rad():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1802_03972_amd as rad
    from paper_1802_03972_amd.build import ensure_built
    ensure_built()    # a built library is used as is
    rad._lib.lib()
    return rad


def test_push_beyond_two_to_the_31_particles(rad):
    import torch
    n = PERIOD * COPIES
    assert n > 2 ** 31
    w = SINGLE.scaled(n_particles=PERIOD, n_steps=1, nx_dir=2, ny_dir=2, n_omega=16, seed=81)
    st = w.steps()
    t = float(w.times()[0])

    def grid():
        return rad.Grid(w.directions(), w.omega0, w.domega, w.n_omega, shape=w.shape, shape_len=w.shape_len,
                        dt=w.dt)

    big = {k: torch.as_tensor(np.ascontiguousarray(st[k][0]), dtype=torch.float32, device="cuda:0").repeat(COPIES)
           for k in FIELDS}
    g = grid()
    g.push_step(t, big)
    I = g.spectrum()
    h = PERIOD * (COPIES // 2)
    g2 = grid()
    g2.push_step(t, {k: v[:h] for k, v in big.items()})
    g2.push_step(t, {k: v[h:] for k, v in big.items()})
    I2 = g2.spectrum()            # synchronises: the pushes have read the particles
    del big
    torch.cuda.empty_cache()
    assert_close(I, I2, f"{n} particles in one push vs two halves", tol_inf=1e-5, tol_freq=1e-5)
    # st holds the FP32-rounded values the device ingests (FP32-input workload)
    Iref = oracle.spectrum(flatten(st, w.times()), w.directions(), w.omegas(), w.shape, w.shape_len, w.dt)
    assert_parity(I, Iref * float(COPIES) ** 2, f"{n} particles (periodic) vs oracle x copies^2")
