/*
 * FP64 CPU oracle for the in-situ macro-particle radiation sum.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the bench's
 * CPU-baseline leg may load this library.  It shares no code, header, table or
 * constant with the device path.
 *
 * Paper: Pausch et al., "Quantitatively consistent computation of coherent and
 * incoherent radiation in particle-in-cell codes - a general form factor formalism
 * for macro-particles" (arXiv:1802.03972).
 *
 * What is computed, for every observation direction n and frequency omega:
 *
 *   S(n, omega) = sum over samples i of  F_i(omega) * A_i(n) * exp(i omega (t_i - n.r_i / c))
 *   I(n, omega) = C * (|S_x|^2 + |S_y|^2 + |S_z|^2),   C = (q_e dt)^2 / (16 pi^3 eps0 c)
 *
 * where a "sample" is one macro-particle at one time step (the double sum over
 * steps j and macro-particles m of Eq. 13), A is the radiation amplitude of Eq. 1
 * evaluated with plain cross products, the phase is the complex phase of Eq. 1, and
 * F_i = sqrt(F^2) with F^2 = N + (N^2 - N) |F[rho]|^2 the closed-form form factor of
 * Eqs. 11-12 for a macro-particle of weighting N.
 *
 * Readings where the text is garbled or silent:
 *  - Eq. 13 prints the prefactor as dt q_e / (16 pi^3 eps0 c) outside |.|^2, which
 *    does not match the units of Eq. 1.  The time integral of Eq. 1 discretised by
 *    the rectangle rule puts dt inside the square, so C = (q_e dt)^2/(16 pi^3 eps0 c).
 *  - Table 1 lists |F[rho]|^2 for un-normalised shapes.  Eqs. 10-12 need a
 *    normalised density (F^2(0) = N^2), so the shape factor used is
 *    g(omega) = |F~(omega)|^2 with F~(0) = 1:
 *      CIC sinc^2(omega D / 2c), TSC sinc^4, QSC sinc^6 (sinc(x) = sin(x)/x),
 *      Gauss exp(-omega^2 sigma^2 / c^2) for rho ~ exp(-x^2 / 2 sigma^2).
 *    For the 1-D shapes the factor is applied along n independently of the direction
 *    (the paper takes n = e_x without loss of generality when deriving it).
 *  - Shapes 5-7 are the cubic-cell versions (side D): the density is the product of the
 *    1-D density along x, y and z, so its transform at wave vector omega n / c is the
 *    product of the 1-D transforms at omega n_c / c:
 *      g(n, omega) = prod_c sinc^(2p)(omega n_c D / 2c),  p = 1 (CIC), 2 (TSC), 3 (QSC).
 *  - c in Eq. 1 is the speed of light (the text calls it a mass).
 *  - Sums are accumulated with Neumaier compensation so that the reference value does
 *    not drift over ~1e8 terms; this does not change which terms are summed.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* CODATA 2018 SI values. */
static const double ORC_C = 299792458.0;          /* speed of light [m/s], exact      */
static const double ORC_QE = 1.602176634e-19;     /* elementary charge [C], exact     */
static const double ORC_EPS0 = 8.8541878128e-12;  /* vacuum permittivity [F/m]        */
static const double ORC_PI = 3.14159265358979323846;

enum { ORC_SHAPE_POINT = 0, ORC_SHAPE_CIC = 1, ORC_SHAPE_TSC = 2, ORC_SHAPE_QSC = 3,
       ORC_SHAPE_GAUSS = 4, ORC_SHAPE_CIC3D = 5, ORC_SHAPE_TSC3D = 6, ORC_SHAPE_QSC3D = 7 };

/* Table 1, normalised: squared Fourier transform of the unit-charge shape. */
double oracle_shape_g(int shape, double len, double omega)
{
    if (shape == ORC_SHAPE_POINT) return 1.0;
    if (shape == ORC_SHAPE_GAUSS) {
        double a = omega * len / ORC_C;
        return exp(-a * a);
    }
    double x = omega * len / (2.0 * ORC_C);
    double s = (x == 0.0) ? 1.0 : sin(x) / x;
    double s2 = s * s;
    if (shape == ORC_SHAPE_CIC) return s2;
    if (shape == ORC_SHAPE_TSC) return s2 * s2;
    if (shape == ORC_SHAPE_QSC) return s2 * s2 * s2;
    return NAN;
}

/* Cubic-cell shapes: product of the 1-D factor over the three axes at omega * |n_c|. */
double oracle_shape_g3(int shape, double len, const double n[3], double omega)
{
    int base = shape - ORC_SHAPE_CIC3D + ORC_SHAPE_CIC;
    return oracle_shape_g(base, len, omega * fabs(n[0])) *
           oracle_shape_g(base, len, omega * fabs(n[1])) *
           oracle_shape_g(base, len, omega * fabs(n[2]));
}

/* Eq. 12: F^2 = N + (N^2 - N) g  (incoherent + coherent part). */
double oracle_form_factor_sq(double N, double g)
{
    return N + (N * N - N) * g;
}

static void cross3(const double a[3], const double b[3], double out[3])
{
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

/* Eq. 1: A = n x [(n - beta) x dbeta] / (1 - beta.n)^2. */
void oracle_amplitude(const double n[3], const double beta[3], const double dbeta[3],
                      double A[3])
{
    double nmb[3] = { n[0] - beta[0], n[1] - beta[1], n[2] - beta[2] };
    double inner[3], outer[3];
    cross3(nmb, dbeta, inner);
    cross3(n, inner, outer);
    double D = 1.0 - (beta[0] * n[0] + beta[1] * n[1] + beta[2] * n[2]);
    double D2 = D * D;
    A[0] = outer[0] / D2;
    A[1] = outer[1] / D2;
    A[2] = outer[2] / D2;
}

/* Prefactor of Eq. 13 with the rectangle-rule dt inside the square. */
double oracle_prefactor(double dt)
{
    double q = ORC_QE * dt;
    return q * q / (16.0 * ORC_PI * ORC_PI * ORC_PI * ORC_EPS0 * ORC_C);
}

typedef struct { double sum, comp; } nsum;

static void nsum_add(nsum* s, double v)
{
    double t = s->sum + v;
    if (fabs(s->sum) >= fabs(v)) s->comp += (s->sum - t) + v;
    else s->comp += (v - t) + s->sum;
    s->sum = t;
}

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Complex spectrum.  Samples are flat arrays of length n_samples (one entry per
 * macro-particle per step, with its own time t).  dirs: n_dir x 3 unit vectors.
 * omegas: n_omega angular frequencies [rad/s].  S_out: n_dir x n_omega x 3 complex,
 * interleaved (re, im), i.e. S_out[((d * n_omega + k) * 3 + c) * 2 + {0,1}].
 * Returns 0, or -1 on a bad argument.
 */
int oracle_spectrum_complex(int64_t n_samples, const double* t,
                            const double* x, const double* y, const double* z,
                            const double* bx, const double* by, const double* bz,
                            const double* dbx, const double* dby, const double* dbz,
                            const double* weight,
                            int n_dir, const double* dirs, int n_omega, const double* omegas,
                            int shape, double shape_len, double* S_out)
{
    if (n_samples < 0 || n_dir < 0 || n_omega < 0 || !S_out) return -1;
    if (shape < ORC_SHAPE_POINT || shape > ORC_SHAPE_QSC3D) return -1;
    int64_t n_points = (int64_t)n_dir * n_omega;

#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < n_points; ++p) {
        int d = (int)(p / n_omega);
        int k = (int)(p % n_omega);
        const double* n = dirs + 3 * d;
        double omega = omegas[k];
        double g = shape >= ORC_SHAPE_CIC3D ? oracle_shape_g3(shape, shape_len, n, omega)
                                            : oracle_shape_g(shape, shape_len, omega);
        nsum acc[6] = { { 0, 0 }, { 0, 0 }, { 0, 0 }, { 0, 0 }, { 0, 0 }, { 0, 0 } };
        for (int64_t i = 0; i < n_samples; ++i) {
            double beta[3] = { bx[i], by[i], bz[i] };
            double dbeta[3] = { dbx[i], dby[i], dbz[i] };
            double A[3];
            oracle_amplitude(n, beta, dbeta, A);
            double F = sqrt(oracle_form_factor_sq(weight[i], g));
            double ndotr = n[0] * x[i] + n[1] * y[i] + n[2] * z[i];
            double phase = omega * (t[i] - ndotr / ORC_C);
            double cr = cos(phase), ci = sin(phase);
            for (int c = 0; c < 3; ++c) {
                nsum_add(&acc[2 * c], F * A[c] * cr);
                nsum_add(&acc[2 * c + 1], F * A[c] * ci);
            }
        }
        double* out = S_out + p * 6;
        for (int c = 0; c < 6; ++c) out[c] = acc[c].sum + acc[c].comp;
    }
    return 0;
}

/* Intensity d^2I/(dOmega domega) [J s / sr] on the same grid: n_dir x n_omega. */
int oracle_spectrum(int64_t n_samples, const double* t,
                    const double* x, const double* y, const double* z,
                    const double* bx, const double* by, const double* bz,
                    const double* dbx, const double* dby, const double* dbz,
                    const double* weight,
                    int n_dir, const double* dirs, int n_omega, const double* omegas,
                    int shape, double shape_len, double dt, double* I_out)
{
    int64_t n_points = (int64_t)n_dir * n_omega;
    double* S = (double*)malloc(sizeof(double) * 6 * (size_t)(n_points > 0 ? n_points : 1));
    if (!S) return -2;
    int rc = oracle_spectrum_complex(n_samples, t, x, y, z, bx, by, bz, dbx, dby, dbz, weight,
                                     n_dir, dirs, n_omega, omegas, shape, shape_len, S);
    if (rc == 0) {
        double C = oracle_prefactor(dt);
        for (int64_t p = 0; p < n_points; ++p) {
            double s = 0.0;
            for (int c = 0; c < 6; ++c) s += S[p * 6 + c] * S[p * 6 + c];
            I_out[p] = C * s;
        }
    }
    free(S);
    return rc;
}
