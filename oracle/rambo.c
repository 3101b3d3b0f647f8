/* oracle/rambo.c -- CPU reference for the random numbers and the phase-space points.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call this
 * file; only tests/, the smoke check and the bench's cpu_baseline leg use it.  It shares
 * no code with the HIP library.
 *
 * The paper's "standalone" application draws random numbers and samples phase space on
 * the GPU before the matrix-element step (Sec. 1, description of the standalone and
 * madevent applications).  The paper names neither the generator nor the sampler; the
 * readings followed here are:
 *   - random numbers: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
 *     as easy as 1, 2, 3", SC'11), key = (seed, 0), one 4x64-bit block per final-state
 *     particle, counter = (event * n_final + particle, 0, 0, 0);
 *     uniform r = ((u >> 11) + 0.5) * 2^-53, so 0 < r < 1;
 *   - phase space: RAMBO (Kleiss, Stirling, Ellis, Comput. Phys. Commun. 40 (1986) 359):
 *     isotropic massless momenta with an exponential energy spectrum, a conformal boost
 *     and scale to sqrt(s), then the massive rescaling by a common factor xi solved by
 *     Newton's method.
 * All arithmetic is double precision and the algorithm is written out step by step,
 * with no blocking or fusion.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>

/* Philox4x64 constants from the SC'11 paper: the two round multipliers and the two
 * Weyl-sequence key increments (golden ratio and sqrt(3)-1 in 64-bit fixed point). */
static const uint64_t PHILOX_M0 = 0xD2E7470EE14C6C93ULL;
static const uint64_t PHILOX_M1 = 0xCA5A826395121157ULL;
static const uint64_t PHILOX_W0 = 0x9E3779B97F4A7C15ULL;
static const uint64_t PHILOX_W1 = 0xBB67AE8584CAA73BULL;

static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

/* One Philox4x64 block with 10 rounds.  Each round: two 64x64->128 products of the
 * even words with the multipliers; the high halves are xored with the odd words and the
 * key, and the words are permuted.  The key is bumped by the Weyl increments before
 * every round but the first. */
void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(PHILOX_M0, x0, &hi0, &lo0);
        mulhilo64(PHILOX_M1, x2, &hi1, &lo1);
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

double or_u01(uint64_t u)
{
    return ((double)(u >> 11) + 0.5) * 0x1.0p-53;
}

/* Four uniforms for final-state particle `i` of event `evt`. */
void or_uniforms(uint64_t seed, int64_t evt, int n_final, int i, double r[4])
{
    uint64_t ctr[4] = {(uint64_t)evt * (uint64_t)n_final + (uint64_t)i, 0, 0, 0};
    uint64_t key[2] = {seed, 0};
    uint64_t u[4];
    or_philox4x64_10(ctr, key, u);
    for (int k = 0; k < 4; ++k) r[k] = or_u01(u[k]);
}

/* RAMBO for one event.  out = [2 + n_final][4] with (E, px, py, pz) in GeV: the two
 * massless beams along +z and -z first, then the final-state particles in order.
 * Returns the number of Newton iterations used by the massive step (0 if massless). */
int or_rambo_event(uint64_t seed, double sqrt_s, int n_final, const double *masses,
                   int64_t evt, double *out)
{
    double q[16][4];
    double p[16][4];
    const double two_pi = 6.283185307179586476925286766559;

    /* step 1: isotropic massless vectors with energy density q0 * exp(-q0) */
    for (int i = 0; i < n_final; ++i) {
        double r[4];
        or_uniforms(seed, evt, n_final, i, r);
        double c = 2.0 * r[0] - 1.0;
        double s = sqrt(1.0 - c * c);
        double phi = two_pi * r[1];
        double q0 = -log(r[2] * r[3]);
        q[i][0] = q0;
        q[i][1] = q0 * s * cos(phi);
        q[i][2] = q0 * s * sin(phi);
        q[i][3] = q0 * c;
    }

    /* step 2: conformal transformation to the centre-of-mass frame at energy sqrt(s) */
    double Q[4] = {0, 0, 0, 0};
    for (int i = 0; i < n_final; ++i)
        for (int mu = 0; mu < 4; ++mu) Q[mu] += q[i][mu];
    double M = sqrt(Q[0] * Q[0] - Q[1] * Q[1] - Q[2] * Q[2] - Q[3] * Q[3]);
    double b[3] = {-Q[1] / M, -Q[2] / M, -Q[3] / M};
    double gamma = Q[0] / M;
    double a = 1.0 / (1.0 + gamma);
    double x = sqrt_s / M;
    for (int i = 0; i < n_final; ++i) {
        double bq = b[0] * q[i][1] + b[1] * q[i][2] + b[2] * q[i][3];
        p[i][0] = x * (gamma * q[i][0] + bq);
        for (int k = 0; k < 3; ++k)
            p[i][k + 1] = x * (q[i][k + 1] + b[k] * q[i][0] + a * bq * b[k]);
    }

    /* step 3: massive particles.  Solve sum_i sqrt(m_i^2 + xi^2 E_i^2) = sqrt(s) for xi
     * (E_i = |p_i| of the massless momenta) by Newton's method, starting from the value given
     * in the RAMBO paper, xi0 = sqrt(1 - (sum m / sqrt s)^2), until the residual stops
     * decreasing (its rounding floor: energy then balances to a few ulp of sqrt(s)) or after
     * 50 steps; the xi of the smallest residual is used. */
    double msum = 0.0;
    int massive = 0;
    for (int i = 0; i < n_final; ++i) {
        msum += masses[i];
        if (masses[i] > 0.0) massive = 1;
    }
    int iters = 0;
    if (massive) {
        double xi = sqrt(1.0 - (msum / sqrt_s) * (msum / sqrt_s));
        double xi_best = xi, r_best = INFINITY;
        for (iters = 0; iters < 50; ++iters) {
            double f = -sqrt_s, fp = 0.0;
            for (int i = 0; i < n_final; ++i) {
                double e = sqrt(masses[i] * masses[i] + xi * xi * p[i][0] * p[i][0]);
                f += e;
                fp += xi * p[i][0] * p[i][0] / e;
            }
            if (!(fabs(f) < r_best)) break;
            r_best = fabs(f);
            xi_best = xi;
            if (f == 0.0) break;
            xi -= f / fp;
        }
        xi = xi_best;
        for (int i = 0; i < n_final; ++i) {
            double e = sqrt(masses[i] * masses[i] + xi * xi * p[i][0] * p[i][0]);
            p[i][0] = e;
            for (int k = 1; k < 4; ++k) p[i][k] *= xi;
        }
    }

    double h = 0.5 * sqrt_s;
    out[0] = h; out[1] = 0.0; out[2] = 0.0; out[3] = h;
    out[4] = h; out[5] = 0.0; out[6] = 0.0; out[7] = -h;
    for (int i = 0; i < n_final; ++i)
        for (int mu = 0; mu < 4; ++mu) out[4 * (i + 2) + mu] = p[i][mu];
    return iters;
}

/* Events evt0 .. evt0+n_evt-1 into out[n_evt][2+n_final][4]. Returns 0, or -1 on bad
 * arguments (n_final outside 2..16, n_evt < 0, sqrt_s <= sum of masses). */
int or_rambo(uint64_t seed, double sqrt_s, int n_final, const double *masses,
             int64_t evt0, int64_t n_evt, double *out)
{
    if (n_final < 2 || n_final > 16 || n_evt < 0) return -1;
    double msum = 0.0;
    for (int i = 0; i < n_final; ++i) msum += masses[i];
    if (!(sqrt_s > msum)) return -1;
    int n_par = n_final + 2;
    for (int64_t e = 0; e < n_evt; ++e)
        or_rambo_event(seed, sqrt_s, n_final, masses, evt0 + e, out + (size_t)e * n_par * 4);
    return 0;
}
