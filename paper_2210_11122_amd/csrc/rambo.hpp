// rambo.hpp -- phase-space points on the GPU, one lane per event.
//
// Random numbers: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): key (seed, 0), one
// block per final-state particle with counter (event * n_final + particle, 0, 0, 0);
// uniform r = ((u >> 11) + 0.5) 2^-53 in (0, 1).
// Momenta: RAMBO (Kleiss, Stirling, Ellis, Comput. Phys. Commun. 40 (1986) 359) --
// isotropic massless vectors with energy density q0 exp(-q0), conformal transformation to
// the centre-of-mass frame at sqrt(s), then the common rescaling xi that puts massive
// particles on shell (Newton's method from the paper's starting value until the residual
// stops decreasing, at most 50 steps).  Output layout [event][particle][E, px, py, pz] with the two
// beams along +z and -z first.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace me {

struct Philox4x64 {
    uint64_t v[4];
};

__device__ __forceinline__ Philox4x64 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                                    uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += W0; k1 += W1; }
        const uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
        const uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
        const uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    return {{c0, c1, c2, c3}};
}

__device__ __forceinline__ double u01(uint64_t u) { return ((double)(u >> 11) + 0.5) * 0x1.0p-53; }

struct FinalMasses {
    double m[8];
};

template <int NF>
__global__ __launch_bounds__(256) void rambo_kernel(uint64_t seed, double sqrt_s, FinalMasses fm,
                                                    int64_t evt0, int64_t n_evt, double* __restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_evt) return;
    const int64_t evt = evt0 + t;
    const double* mass = fm.m;
    double q[NF][4], p[NF][4];
    const double two_pi = 6.283185307179586476925286766559;
#pragma unroll
    for (int i = 0; i < NF; ++i) {
        Philox4x64 u = philox4x64_10((uint64_t)evt * NF + i, 0, 0, 0, seed, 0);
        const double c = 2.0 * u01(u.v[0]) - 1.0;
        const double s = sqrt(1.0 - c * c);
        const double phi = two_pi * u01(u.v[1]);
        const double q0 = -log(u01(u.v[2]) * u01(u.v[3]));
        q[i][0] = q0;
        q[i][1] = q0 * s * cos(phi);
        q[i][2] = q0 * s * sin(phi);
        q[i][3] = q0 * c;
    }
    double Q[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < NF; ++i)
#pragma unroll
        for (int m = 0; m < 4; ++m) Q[m] += q[i][m];
    const double M = sqrt(Q[0] * Q[0] - Q[1] * Q[1] - Q[2] * Q[2] - Q[3] * Q[3]);
    const double b[3] = {-Q[1] / M, -Q[2] / M, -Q[3] / M};
    const double gam = Q[0] / M, a = 1.0 / (1.0 + gam), x = sqrt_s / M;
#pragma unroll
    for (int i = 0; i < NF; ++i) {
        const double bq = b[0] * q[i][1] + b[1] * q[i][2] + b[2] * q[i][3];
        p[i][0] = x * (gam * q[i][0] + bq);
#pragma unroll
        for (int k = 0; k < 3; ++k) p[i][k + 1] = x * (q[i][k + 1] + b[k] * q[i][0] + a * bq * b[k]);
    }
    double msum = 0.0;
    bool massive = false;
#pragma unroll
    for (int i = 0; i < NF; ++i) {
        msum += mass[i];
        massive |= mass[i] > 0.0;
    }
    if (massive) {
        double xi = sqrt(1.0 - (msum / sqrt_s) * (msum / sqrt_s));
        double xi_best = xi, r_best = INFINITY;
        for (int it = 0; it < 50; ++it) {
            double f = -sqrt_s, fp = 0.0;
#pragma unroll
            for (int i = 0; i < NF; ++i) {
                const double e = sqrt(mass[i] * mass[i] + xi * xi * p[i][0] * p[i][0]);
                f += e;
                fp += xi * p[i][0] * p[i][0] / e;
            }
            // Newton until the residual stops decreasing (its rounding floor), keeping the best xi
            if (!(fabs(f) < r_best)) break;
            r_best = fabs(f);
            xi_best = xi;
            if (f == 0.0) break;
            xi -= f / fp;
        }
        xi = xi_best;
#pragma unroll
        for (int i = 0; i < NF; ++i) {
            p[i][0] = sqrt(mass[i] * mass[i] + xi * xi * p[i][0] * p[i][0]);
#pragma unroll
            for (int k = 1; k < 4; ++k) p[i][k] *= xi;
        }
    }
    double* o = out + t * (NF + 2) * 4;
    const double hs = 0.5 * sqrt_s;
    o[0] = hs; o[1] = 0.0; o[2] = 0.0; o[3] = hs;
    o[4] = hs; o[5] = 0.0; o[6] = 0.0; o[7] = -hs;
#pragma unroll
    for (int i = 0; i < NF; ++i)
#pragma unroll
        for (int m = 0; m < 4; ++m) o[4 * (i + 2) + m] = p[i][m];
}

}  // namespace me
