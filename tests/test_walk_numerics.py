"""FP32 accuracy of the two frequency walks of the kernels (FP32 emulation on the CPU, no
GPU).  A lane of the accumulate kernel reaches exp(i(s + k) theta), k = 0..15, theta the
per-frequency phase step, from an FP32 seed at k = 8 (the middle of its block) and the
rotation w = exp(i theta) rounded once to FP32; a thread of the tracked-particle kernel does
the same over k = 0..7 from k = 4.

* Complex-product walk (z <- z w forward, z <- z conj(w) backward): about one rounding of w
  per product, so a few ulps after at most 8 products, whatever theta is.
* Three-term walk (z_{k+1} = 2 cos(theta) z_k - z_{k-1}), written as the kernel writes it:
  y_k = sigma_k z_k with sigma = (+, +, -, -) by k mod 4, so that every step is one
  multiply-add per component.  A perturbation of one step reaches m steps later multiplied by
  sin(m theta) / sin(theta), which is at most m in size: the error after m steps is bounded by
  about m^2 roundings, also for theta near 0 or pi where 1 / sin(theta) is huge.  With the seed
  in the middle (m <= 7) that is a few 1e-6; the same recurrence walked 15 steps from one end
  of the block is several times worse.

A mistake in the sign factors or in the sign of the recurrence coefficient (a plausible slip in
the kernel's algebra) gives errors of order 1 and fails the bound test."""
import numpy as np

f32 = np.float32
ULP = 2.0 ** -23


def fma(a, b, c):
    """FP32 fused multiply-add: exact FP64 product of two FP32 values, one final rounding."""
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(f32)


def mul(a, b):
    return (a.astype(np.float64) * b.astype(np.float64)).astype(f32)


def steps_near_degenerate(n, rng):
    """Phase steps within 1e-7..1e-2 rad of 0 or pi, plus uniformly random ones."""
    eps = 10.0 ** rng.uniform(-7, -2, n) * rng.choice([-1.0, 1.0], n)
    near = np.pi * rng.integers(0, 2, n) + eps
    return np.concatenate([near, rng.uniform(0, 2 * np.pi, n)])


def seed_and_w(theta, phase0, ks):
    zr = np.cos(phase0 + ks * theta).astype(f32)
    zi = np.sin(phase0 + ks * theta).astype(f32)
    return zr, zi, np.cos(theta).astype(f32), np.sin(theta).astype(f32)


def cplx(r, i):
    return r.astype(np.float64) + 1j * i.astype(np.float64)


def walk_product(theta, phase0):
    """z <- z w forward (indices 9..15) and z <- z conj(w) backward (7..0) from the seed at 8."""
    zr, zi, wr, wi = seed_and_w(theta, phase0, 8)
    out = np.zeros((16, theta.size), np.complex128)
    out[8] = cplx(zr, zi)
    fr, fi = zr, zi
    for k in range(9, 16):
        fr, fi = fma(fr, wr, mul(fi, -wi)), fma(fr, wi, mul(fi, wr))
        out[k] = cplx(fr, fi)
    br, bi = zr, zi
    for k in range(7, -1, -1):
        br, bi = fma(br, wr, mul(bi, wi)), fma(bi, wr, mul(br, -wi))
        out[k] = cplx(br, bi)
    return out


def sigma(k):
    return -1.0 if k & 2 else 1.0


def walk_three_term_mid(theta, phase0, flip_sigma=False, W=16):
    """The kernels' three-term walk on y_k = sigma_k z_k over W frequencies (16 in the
    accumulate kernel, 8 in the tracked-particle kernel) from the seed at s = W/2: forward
    from (y_s, y_s+1 = z w), backward from (y_s, y_s-1 = -c y_s + y_s+1, i.e.
    -(c z_s - z_s+1)); returns z_k = sigma_k y_k."""
    ks = W // 2
    zr, zi, wr, wi = seed_and_w(theta, phase0, ks)
    pc = (f32(2) * wr).astype(f32)          # exact doubling
    nc = -pc
    y = [None] * W
    pr, pi = zr, zi
    cr, ci = fma(zr, wr, mul(zi, -wi)), fma(zr, wi, mul(zi, wr))
    y[ks], y[ks + 1] = (pr, pi), (cr, ci)
    y[ks - 1] = (fma(nc, zr, cr), fma(nc, zi, ci))
    for k in range(ks + 1, W - 1):
        ck = nc if k & 1 else pc
        nr, ni = fma(ck, cr, pr), fma(ck, ci, pi)
        pr, pi, cr, ci = cr, ci, nr, ni
        y[k + 1] = (cr, ci)
    pr, pi = zr, zi
    cr, ci = y[ks - 1]
    for k in range(ks - 1, 0, -1):
        ck = pc if k & 1 else nc
        nr, ni = fma(ck, cr, pr), fma(ck, ci, pi)
        pr, pi, cr, ci = cr, ci, nr, ni
        y[k - 1] = (cr, ci)
    s = (lambda k: 1.0 if (k & 1) else sigma(k)) if flip_sigma else sigma
    return np.stack([s(k) * cplx(*y[k]) for k in range(W)])


def walk_three_term_from_start(theta, phase0):
    """The plain recurrence z_{k+1} = 2 cos(theta) z_k - z_{k-1} from FP32 values at indices 0
    and 1 (up to 15 steps)."""
    zr, zi, wr, wi = seed_and_w(theta, phase0, 0)
    c = (f32(2) * wr).astype(f32)
    out = np.zeros((16, theta.size), np.complex128)
    pr, pi = zr, zi
    cr, ci = fma(zr, wr, mul(zi, -wi)), fma(zr, wi, mul(zi, wr))
    out[0], out[1] = cplx(pr, pi), cplx(cr, ci)
    for k in range(1, 15):
        nr, ni = fma(c, cr, -pr), fma(c, ci, -pi)
        pr, pi, cr, ci = cr, ci, nr, ni
        out[k + 1] = cplx(cr, ci)
    return out


def exact(theta, phase0, W=16):
    k = np.arange(W)[:, None]
    return np.exp(1j * (phase0 + k * theta))


def inputs(seed, n=20000):
    rng = np.random.default_rng(seed)
    theta = steps_near_degenerate(n, rng)
    return theta, rng.uniform(0, 2 * np.pi, theta.size)


def test_complex_product_walk_stays_within_a_few_ulps():
    theta, phase0 = inputs(5)
    err = np.abs(walk_product(theta, phase0) - exact(theta, phase0)).max()
    assert err < 2e-6, err          # |z| = 1: at most 8 products of a few ulps each


def test_mid_seeded_three_term_walk_within_its_m_squared_bound():
    theta, phase0 = inputs(6)
    err = np.abs(walk_three_term_mid(theta, phase0) - exact(theta, phase0))
    m = np.abs(np.arange(16) - 8)[:, None]
    # seed and w rounding (a few ulps) plus ~m^2 roundings of 2 cos(theta) and of the steps;
    # the same bound near 0 and pi (first half of the inputs) as for random steps
    bound = (4 + 2 * m + m * m) * ULP
    assert (err <= bound).all(), (err / bound).max()
    assert err.max() < 6e-6, err.max()


def test_tracked_kernel_three_term_walk_over_8_frequencies():
    theta, phase0 = inputs(10)
    err = np.abs(walk_three_term_mid(theta, phase0, W=8) - exact(theta, phase0, W=8))
    m = np.abs(np.arange(8) - 4)[:, None]
    assert (err <= (4 + 2 * m + m * m) * ULP).all()
    assert err.max() < 2e-6, err.max()


def test_three_term_walk_is_not_amplified_near_zero_and_pi():
    theta, phase0 = inputs(7)
    err = np.abs(walk_three_term_mid(theta, phase0) - exact(theta, phase0)).max(axis=0)
    near = np.arange(theta.size) < theta.size // 2
    tiny = near & (np.abs(np.sin(theta)) < 1e-5)      # 1 / sin(theta) > 1e5
    assert tiny.sum() > 1000
    assert err[tiny].max() < 2 * err[~near].max() + 1e-6, (err[tiny].max(), err[~near].max())


def test_long_three_term_walk_is_worse_than_the_mid_seeded_one():
    theta, phase0 = inputs(8)
    ex = exact(theta, phase0)
    long_err = np.abs(walk_three_term_from_start(theta, phase0) - ex).max()
    mid_err = np.abs(walk_three_term_mid(theta, phase0) - ex).max()
    assert long_err > 2.5 * mid_err, (long_err, mid_err)
    assert long_err < (4 + 2 * 15 + 15 * 15) * ULP    # still bounded by m^2 (m = 15)


def test_wrong_sign_factors_break_the_three_term_walk():
    theta, phase0 = inputs(9, 2000)
    err = np.abs(walk_three_term_mid(theta, phase0, flip_sigma=True) - exact(theta, phase0)).max()
    assert err > 1.0, err
