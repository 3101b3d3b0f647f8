// colorsum.hpp -- the colour-matrix contraction on the matrix cores, batched over events.
//
// For every (event, helicity) column the amplitude kernel leaves the colour-flow
// amplitudes J_c (c < NC, real and imaginary rows) in HBM, layout
// jamp[h][2c + re/im][column], column = event within the chunk, row stride ld.  Here
//     ME_h = (1/D) sum_{c,c'} (Re J_c Chat_{cc'} Re J_c' + Im J_c Chat_{cc'} Im J_c')
// with Chat = D * C the integer colour matrix, as the matrix product Chat x J over 16
// event columns per wavefront, followed by the column dot product and the sum over the
// filtered helicities in FP64.
//
// FP64 form: v_mfma_f64_16x16x4f64 (A = Chat tile 16x4, B = J tile 4x16, D 16x16 in FP64).
// Mixed form: the FP32 jamps of one (event, helicity) are scaled by a power of two so that
// the largest |J| lies in [1/2, 1), split exactly into two FP16 terms hi + lo * 2^-11, and
// contracted with v_mfma_f32_16x16x16f16 (FP32 accumulation); the dot product is formed in
// FP32 from the scaled FP32 jamps, unscaled exactly, and summed over helicities in FP64.
//
// MFMA operand layouts (lane l, i = l % 16, g = l / 16):
//   f64 16x16x4:  A[i][g], B[g][i], D[g + 4r][i] (r = 0..3)
//   f16 16x16x16: A[i][4g + t], B[4g + t][i] (t = 0..3), D[4g + r][i]
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace me {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef _Float16 v4h __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double sum_lane_groups(double x)
{
    x += __shfl_xor(x, 16, 64);
    x += __shfl_xor(x, 32, 64);
    return x;
}
__device__ __forceinline__ float max_lane_groups(float x)
{
    x = fmaxf(x, __shfl_xor(x, 16, 64));
    x = fmaxf(x, __shfl_xor(x, 32, 64));
    return x;
}

// A operands of Chat for the f64 MFMA, pre-arranged per lane: aop[(mt * KT + kt) * 64 + l]
// = Chat[16 mt + l % 16][4 kt + l / 16] (zero outside NC).
template <int NC>
__global__ __launch_bounds__(256) void colour_sum_f64(const double* __restrict__ J, int64_t ld, int n_good,
                                                      int64_t n_evt, const double* __restrict__ aop,
                                                      double scale_hel, double scale_avg,
                                                      double* __restrict__ out, double* __restrict__ out_hel)
{
    constexpr int MT = (NC + 15) / 16, KT = (NC + 3) / 4;
    constexpr bool AREG = MT * KT <= 24;
    const int lane = threadIdx.x & 63;
    const int64_t e0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
    if (e0 >= n_evt) return;
    const int i = lane & 15, g = lane >> 4;
    const int64_t e = e0 + i;
    const bool valid = e < n_evt;
    const int64_t ec = valid ? e : n_evt - 1;
    double A[AREG ? MT * KT : 1];
    if (AREG) {
#pragma unroll
        for (int q = 0; q < MT * KT; ++q) A[q] = aop[q * 64 + lane];
    }
    double me = 0.0;
    for (int h = 0; h < n_good; ++h) {
        const double* Jh = J + (int64_t)h * (2 * NC) * ld;
        double part = 0.0;
#pragma unroll
        for (int ri = 0; ri < 2; ++ri) {
            v4d d[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) d[mt] = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kt = 0; kt < KT; ++kt) {
                const int c = 4 * kt + g;
                const double b = (c < NC) ? Jh[(int64_t)(2 * c + ri) * ld + ec] : 0.0;
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const double a = AREG ? A[mt * KT + kt] : aop[(mt * KT + kt) * 64 + lane];
                    d[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, d[mt], 0, 0, 0);
                }
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int c = 16 * mt + g + 4 * r;
                    if (c < NC) part += Jh[(int64_t)(2 * c + ri) * ld + ec] * d[mt][r];
                }
        }
        part = sum_lane_groups(part);
        if (out_hel && g == 0 && valid) out_hel[e * n_good + h] = part * scale_hel;
        me += part;
    }
    if (g == 0 && valid) out[e] = me * scale_avg;
}

// A operands of Chat for the f16 MFMA: aop[((mt * KB + kb) * 64 + l) * 4 + t]
// = Chat[16 mt + l % 16][16 kb + 4 (l / 16) + t].
template <int NC>
__global__ __launch_bounds__(256) void colour_sum_f16(const float* __restrict__ J, int64_t ld, int n_good,
                                                      int64_t n_evt, const _Float16* __restrict__ aop,
                                                      double scale_hel, double scale_avg,
                                                      double* __restrict__ out, double* __restrict__ out_hel)
{
    constexpr int MT = (NC + 15) / 16, KB = MT;
    constexpr bool AREG = MT * KB <= 16;
    const int lane = threadIdx.x & 63;
    const int64_t e0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
    if (e0 >= n_evt) return;
    const int i = lane & 15, g = lane >> 4;
    const int64_t e = e0 + i;
    const bool valid = e < n_evt;
    const int64_t ec = valid ? e : n_evt - 1;
    v4h A[AREG ? MT * KB : 1];
    if (AREG) {
#pragma unroll
        for (int q = 0; q < MT * KB; ++q) A[q] = *reinterpret_cast<const v4h*>(aop + (q * 64 + lane) * 4);
    }
    double me = 0.0;
    for (int h = 0; h < n_good; ++h) {
        const float* Jh = J + (int64_t)h * (2 * NC) * ld;
        // this lane's rows of column i: c = 16 kb + 4 g + t
        float x[2][KB][4];
        float mx = 0.0f;
#pragma unroll
        for (int ri = 0; ri < 2; ++ri)
#pragma unroll
            for (int kb = 0; kb < KB; ++kb)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int c = 16 * kb + 4 * g + t;
                    const float v = (c < NC) ? Jh[(int64_t)(2 * c + ri) * ld + ec] : 0.0f;
                    x[ri][kb][t] = v;
                    mx = fmaxf(mx, fabsf(v));
                }
        mx = max_lane_groups(mx);
        // power-of-two scale: largest |J| of the column into [1/2, 1)
        int ex = 0;
        if (mx > 0.0f) frexpf(mx, &ex);
        const float s = ldexpf(1.0f, -ex);
        float part = 0.0f;
#pragma unroll
        for (int ri = 0; ri < 2; ++ri) {
            v4h bh[KB], bl[KB];
#pragma unroll
            for (int kb = 0; kb < KB; ++kb)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const float v = x[ri][kb][t] * s;
                    const _Float16 hi = (_Float16)v;
                    bh[kb][t] = hi;
                    bl[kb][t] = (_Float16)((v - (float)hi) * 2048.0f);
                    x[ri][kb][t] = v;
                }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                v4f dh = {0.f, 0.f, 0.f, 0.f}, dl = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kb = 0; kb < KB; ++kb) {
                    const v4h a = AREG ? A[mt * KB + kb] : *reinterpret_cast<const v4h*>(aop + ((mt * KB + kb) * 64 + lane) * 4);
                    dh = __builtin_amdgcn_mfma_f32_16x16x16f16(a, bh[kb], dh, 0, 0, 0);
                    dl = __builtin_amdgcn_mfma_f32_16x16x16f16(a, bl[kb], dl, 0, 0, 0);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) part += x[ri][mt][r] * (dh[r] + dl[r] * (1.0f / 2048.0f));
            }
        }
        double p = sum_lane_groups((double)part) / ((double)s * (double)s);
        if (out_hel && g == 0 && valid) out_hel[e * n_good + h] = p * scale_hel;
        me += p;
    }
    if (g == 0 && valid) out[e] = me * scale_avg;
}

}  // namespace me
