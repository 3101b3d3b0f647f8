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
// Symmetry: Chat is symmetric, so with the colour index cut into blocks of 16 the
// contraction equals J^T A J for the block upper-triangular A with A = Chat on diagonal
// blocks, 2 Chat above them and 0 below; only the tiles of A that touch the upper triangle
// are multiplied (36 of 64 blocks for 120 flows).  The host prepares A in that form.
//
// Helicity groups: blockIdx.y selects a group of consecutive filtered helicities.  With one
// group the kernel writes the averaged result; with several, each group writes its partial
// sum to part[group][event] and hel_reduce adds the groups in a fixed order, so every
// event's result is independent of the batch it came in.
//
// FP64 form: v_mfma_f64_16x16x4f64 (A tile 16x4, B tile 4x16, D 16x16, all FP64).
// Mixed forms: the FP32 real (imaginary) rows of one (event, helicity) column are scaled by
// a power of two so that their largest |J| lies in [1/2, 1), split exactly into two 16-bit
// terms hi + lo * 2^-p (p = 11 for FP16, 8 for BF16), and contracted with
// v_mfma_f32_16x16x32_{f16,bf16} (FP32 accumulation); the dot product with the scaled FP32
// jamps is formed in FP64, unscaled exactly, and summed over helicities in FP64.  Colour
// numerators that a 16-bit type cannot hold exactly (BF16 keeps 8 significant bits) are
// split the same way on the host into A_hi + A_lo, both exact; tiles whose A_lo vanishes
// are skipped by a per-tile mask.
//
// MFMA operand layouts (lane l, i = l % 16, g = l / 16):
//   f64 16x16x4:   A[i][g], B[g][i], D[g + 4r][i] (r = 0..3)
//   16x16x32:      A[i][8g + t], B[8g + t][i] (t = 0..7), D[4g + r][i]
// In the 16x16x32 form the k slot (kb, 8g + t) carries colour 16 (2 kb + t / 4) + 4 g + t % 4,
// so that the B elements a lane holds are exactly the D rows it receives (the dot product
// then needs no data exchange between lanes).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace me {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

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

// tile counts of the block upper-triangular colour matrix
__host__ __device__ constexpr int cs64_tiles(int nc)
{
    int n = 0;
    for (int mt = 0; mt < (nc + 15) / 16; ++mt)
        for (int kt = 4 * mt; kt < (nc + 3) / 4; ++kt) ++n;
    return n;
}
__host__ __device__ constexpr int cs16_tiles(int nc)
{
    int n = 0;
    for (int mt = 0; mt < (nc + 15) / 16; ++mt)
        for (int kb = mt / 2; kb < ((nc + 15) / 16 + 1) / 2; ++kb) ++n;
    return n;
}

// the colour-matrix operands are re-read from the cache for every helicity: hiding the table
// pointer from loop-invariant code motion keeps the compiler from hoisting all of them into
// registers (which would leave one wave per SIMD for the large matrix)
template <class P>
__device__ __forceinline__ const P* opaque(const P* p)
{
    __asm__ volatile("" : "+s"(p));
    return p;
}

// store or accumulate the helicity-group result of one event
__device__ __forceinline__ void cs_store(double me, int64_t e, int64_t n_evt, double scale_avg, double* out,
                                         double* part)
{
    if (gridDim.y == 1)
        out[e] = me * scale_avg;
    else
        part[(int64_t)blockIdx.y * n_evt + e] = me;
}

// One colour flow (the e+e- processes): D |M_h|^2 = Chat_00 (Re J^2 + Im J^2), a scalar, with
// one rounding sequence wherever it is formed (the colour-sum kernel, the amplitude kernels
// that do the colour sum themselves); the empty asm keeps the compiler from fusing the last
// multiply into a later addition.  c00 = aop[0], the one operand of the 1x1 table.
__device__ __forceinline__ double cs1(double jr, double ji, double c00)
{
    double v = c00 * __builtin_fma(jr, jr, ji * ji);
    asm volatile("" : "+v"(v));
    return v;
}

// One colour flow in a mixed form, as the 16-bit tile computes it for that column: the jamp
// scaled by a power of two into [1/2, 1), split into hi + lo * 2^-p, both multiplied by the one
// operand (exact in FP32, the only non-zero products the tile adds), and the dot product formed
// in FP64 and unscaled.  Bitwise the tile's value (16-bit element types below).
template <class T>
__device__ __forceinline__ double cs1_h16_part(float x, float a00)
{
    float mx = fabsf(x);
    int ex = 0;
    if (mx > 0.0f) frexpf(mx, &ex);
    const float s = ldexpf(1.0f, -ex);
    const float v = x * s;
    const typename T::elem hi = T::round(v);
    const typename T::elem lo = T::round((v - T::value(hi)) * T::LO);
    const float dh = a00 * T::value(hi), dl = a00 * T::value(lo);
    double acc = 0.0;
    acc += (double)v * ((double)dh + (double)dl * (1.0 / T::LO));
    return acc / ((double)s * (double)s);
}
template <class T>
__device__ __forceinline__ double cs1_h16(float jr, float ji, const typename T::elem* aop)
{
    const float a00 = T::value(aop[0]);
    double part = 0.0;
    part += cs1_h16_part<T>(jr, a00);
    part += cs1_h16_part<T>(ji, a00);
    asm volatile("" : "+v"(part));
    return part;
}

// Two colour flows (gg -> tt~): D |M_h|^2 = sum over re/im of J^T Chat J with the 2x2 integer
// matrix, as a scalar in one fixed rounding sequence (rows of Chat J by fused multiply-adds, then
// the dot product); Chat_rc = aop[r + 16 c], the diagonal tile of the 16x4 table.
__device__ __forceinline__ double cs2_part(double a, double b, double c00, double c01, double c10, double c11)
{
    const double r0 = __builtin_fma(c01, b, c00 * a), r1 = __builtin_fma(c11, b, c10 * a);
    return __builtin_fma(b, r1, a * r0);
}
__device__ __forceinline__ double cs2(double j0r, double j0i, double j1r, double j1i, const double* aop)
{
    const double c00 = aop[0], c10 = aop[1], c01 = aop[16], c11 = aop[17];
    double v = cs2_part(j0r, j1r, c00, c01, c10, c11) + cs2_part(j0i, j1i, c00, c01, c10, c11);
    asm volatile("" : "+v"(v));
    return v;
}
// Up to 16 flows as a scalar (gg -> tt~g: 6): for re and im, each row of Chat J as a chain of
// fused multiply-adds over c, then the dot product with J as another; Chat_rc is
// aop[(c / 4) * 64 + r + 16 (c % 4)], the diagonal 16-block of the table (A = Chat there).
// j(c, ri) gives the jamps.
template <int NC, class Jget>
__device__ __forceinline__ double csn(const Jget& j, const double* aop)
{
    static_assert(NC <= 16, "one diagonal tile");
    double v = 0.0;
#pragma unroll
    for (int ri = 0; ri < 2; ++ri) {
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < NC; ++r) {
            double row = aop[r] * j(0, ri);
#pragma unroll
            for (int c = 1; c < NC; ++c) row = __builtin_fma(aop[(c / 4) * 64 + r + 16 * (c % 4)], j(c, ri), row);
            s = __builtin_fma(j(r, ri), row, s);
        }
        v += s;
    }
    asm volatile("" : "+v"(v));
    return v;
}
// the scalar forms from a lane's own jamps Jr[2 c + re/im] (amplitude kernels with register jamps)
template <int NC>
__device__ __forceinline__ double colour_sum_regs(const double* Jr, const double* __restrict__ aop)
{
    static_assert(NC <= 6, "scalar colour sums up to six flows");
    if constexpr (NC == 1)
        return cs1(Jr[0], Jr[1], aop[0]);
    else if constexpr (NC == 2)
        return cs2(Jr[0], Jr[1], Jr[2], Jr[3], aop);
    else
        return csn<NC>([&](int c, int ri) { return Jr[2 * c + ri]; }, aop);
}

// One (16-event tile, helicity) column block of the FP64 form: returns this lane's share of
// D * |M_h|^2 for event column i (the four lane groups' shares add up to it).  load(c, ri) gives
// the jamp of colour c (re/im) of this lane's column.  A: the tile operands in registers when
// AREG, else read from aop.
template <int NC, bool AREG, class Load, bool ALDS = false>
__device__ __forceinline__ double cs64_column(const Load& load, const double* A, const double* aop, int lane)
{
    if constexpr (NC == 1) {
        // no tile for a 1x1 matrix: lane group 0 holds the whole value
        return (lane >> 4) == 0 ? cs1((double)load(0, 0), (double)load(0, 1), aop[0]) : 0.0;
    }
    if constexpr (NC == 2) {
        return (lane >> 4) == 0 ? cs2((double)load(0, 0), (double)load(0, 1), (double)load(1, 0), (double)load(1, 1), aop)
                                : 0.0;
    }
    if constexpr (NC > 2 && NC <= 6) {
        return (lane >> 4) == 0 ? csn<NC>([&](int c, int ri) { return (double)load(c, ri); }, aop) : 0.0;
    }
    constexpr int MT = (NC + 15) / 16, KT = (NC + 3) / 4;
    // the real/imaginary loop stays rolled for the large matrices (register pressure)
    constexpr int RI_UNROLL = NC > 24 ? 1 : 2;
    const int g = lane >> 4;
    double part_h = 0.0;
#pragma unroll RI_UNROLL
    for (int ri = 0; ri < 2; ++ri) {
        // this lane's B elements: colours c = 4 kt + g, which are also its D rows
        double b[KT];
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
            const int c = 4 * kt + g;
            b[kt] = (c < NC) ? (double)load(c, ri) : 0.0;
        }
        int q = 0;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            // operands from LDS (ALDS): read tile row by tile row, not all at once
            if constexpr (ALDS) __asm__ volatile("" ::: "memory");
            const double* ap = ALDS ? aop : opaque(aop);
            v4d d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kt = 4 * mt; kt < KT; ++kt, ++q) {
                const double a = AREG ? A[q] : ap[q * 64 + lane];
                d = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[kt], d, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (4 * mt + r < KT) part_h += b[4 * mt + r] * d[r];
        }
    }
    return part_h;
}

#ifndef CS64_A_IN_LDS
#define CS64_A_IN_LDS 1
#endif
// A operands, per lane, in the kernel's tile order (mt ascending, then kt >= 4 mt):
// aop[q * 64 + l] = A[16 mt + l % 16][4 kt + l / 16].
template <int NC>
__global__ __launch_bounds__(256) void colour_sum_f64(const double* __restrict__ J, int64_t ld, int n_good,
                                                      int hel_per_group, int64_t n_evt,
                                                      const double* __restrict__ aop, double scale_hel,
                                                      double scale_avg, double* __restrict__ out,
                                                      double* __restrict__ out_hel, double* __restrict__ part)
{
    constexpr int NT = cs64_tiles(NC);
    constexpr bool AREG = NT <= 24;
    // the large matrix: its operands staged in LDS once per workgroup (NT * 512 B), instead of
    // each wave reading them through the caches for every tile
    constexpr bool ALDS = !AREG && CS64_A_IN_LDS;
    __shared__ double As[ALDS ? NT * 64 : 1];
    if constexpr (ALDS) {
        for (int k = threadIdx.x; k < NT * 64; k += 256) As[k] = aop[k];
        __syncthreads();
    }
    const int lane = threadIdx.x & 63;
    const int64_t e0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
    if (e0 >= n_evt) return;
    const int i = lane & 15, g = lane >> 4;
    const int64_t e = e0 + i;
    const bool valid = e < n_evt;
    const int64_t ec = valid ? e : n_evt - 1;
    const int h0 = blockIdx.y * hel_per_group, h1 = min(n_good, h0 + hel_per_group);
    double A[AREG ? NT : 1];
    if (AREG) {
#pragma unroll
        for (int q = 0; q < NT; ++q) A[q] = aop[q * 64 + lane];
    }
    double me = 0.0;
    for (int h = h0; h < h1; ++h) {
        const double* Jh = J + (int64_t)h * (2 * NC) * ld;
        const auto load = [&](int c, int ri) { return Jh[(int64_t)(2 * c + ri) * ld + ec]; };
        double part_h = sum_lane_groups(cs64_column<NC, AREG, decltype(load), ALDS>(load, A, ALDS ? As : aop, lane));
        if (out_hel && g == 0 && valid) out_hel[e * n_good + h] = part_h * scale_hel;
        me += part_h;
    }
    if (g == 0 && valid) cs_store(me, e, n_evt, scale_avg, out, part);
}

// 16-bit element types of the mixed colour sum
struct Fp16Terms {
    typedef _Float16 elem;
    typedef v8h vec;
    static constexpr float LO = 2048.0f;  // hi keeps 11 significant bits
    static __device__ __forceinline__ elem round(float v) { return (_Float16)v; }
    static __device__ __forceinline__ float value(elem x) { return (float)x; }
    static __device__ __forceinline__ v4f mfma(vec a, vec b, v4f c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};
struct Bf16Terms {
    typedef __bf16 elem;
    typedef v8bf vec;
    static constexpr float LO = 256.0f;  // hi keeps 8 significant bits
    static __device__ __forceinline__ elem round(float v) { return (__bf16)v; }
    static __device__ __forceinline__ float value(elem x) { return (float)x; }
    static __device__ __forceinline__ v4f mfma(vec a, vec b, v4f c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};

// One (16-event tile, helicity) column block of the mixed forms: this lane's share of
// D * |M_h|^2 for event column i, from the FP32 jamps load(c, ri) of its column.
template <int NC, class T, bool AREG, class Load>
__device__ __forceinline__ double cs16_column(const Load& load, const typename T::vec* A,
                                              const typename T::elem* aop, const typename T::elem* aop_lo,
                                              uint64_t lo_mask, int lane)
{
    typedef typename T::vec vec;
    typedef typename T::elem elem;
    constexpr int MT = (NC + 15) / 16, KB = (MT + 1) / 2;
    const int g = lane >> 4;
    double part_h = 0.0;
#pragma unroll 1
    for (int ri = 0; ri < 2; ++ri) {
        // x[kb][t]: colour 16 (2 kb + t / 4) + 4 g + t % 4 of column i
        float x[KB][8];
        float mx = 0.0f;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int c = 16 * (2 * kb + t / 4) + 4 * g + t % 4;
                const float v = (c < NC) ? (float)load(c, ri) : 0.0f;
                x[kb][t] = v;
                mx = fmaxf(mx, fabsf(v));
            }
        mx = max_lane_groups(mx);
        // power-of-two scale: largest |J| of the column into [1/2, 1)
        int ex = 0;
        if (mx > 0.0f) frexpf(mx, &ex);
        const float s = ldexpf(1.0f, -ex);
        vec bh[KB], bl[KB];
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const float v = x[kb][t] * s;
                const elem hi = T::round(v);
                bh[kb][t] = hi;
                bl[kb][t] = T::round((v - T::value(hi)) * T::LO);
                x[kb][t] = v;
            }
        double acc = 0.0;  // the column dot product, in FP64 (colour sums can cancel)
        int q = 0;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const elem* ap = opaque(aop);
            const elem* ap_lo = opaque(aop_lo);
            v4f dh = {0.f, 0.f, 0.f, 0.f}, dl = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = mt / 2; kb < KB; ++kb, ++q) {
                const vec a = AREG ? A[q] : *reinterpret_cast<const vec*>(ap + (q * 64 + lane) * 8);
                dh = T::mfma(a, bh[kb], dh);
                dl = T::mfma(a, bl[kb], dl);
                if ((lo_mask >> q) & 1) {
                    const vec alo = *reinterpret_cast<const vec*>(ap_lo + (q * 64 + lane) * 8);
                    dh = T::mfma(alo, bh[kb], dh);
                }
            }
            // D rows 16 mt + 4 g + r are this lane's x[mt / 2][4 (mt % 2) + r]
#pragma unroll
            for (int r = 0; r < 4; ++r)
                acc += (double)x[mt / 2][4 * (mt % 2) + r] * ((double)dh[r] + (double)dl[r] * (1.0 / T::LO));
        }
        part_h += acc / ((double)s * (double)s);
    }
    return part_h;
}

// A operands, per lane, in the kernel's tile order (mt ascending, then kb >= mt / 2):
// aop[(q * 64 + l) * 8 + t] = A[16 mt + l % 16][colour of k slot (kb, 8 (l / 16) + t)].
// aop_lo (A_lo, same layout) is read for the tiles whose bit is set in lo_mask.
template <int NC, class T>
__global__ __launch_bounds__(256) void colour_sum_h16(const float* __restrict__ J, int64_t ld, int n_good,
                                                      int hel_per_group, int64_t n_evt,
                                                      const typename T::elem* __restrict__ aop,
                                                      const typename T::elem* __restrict__ aop_lo, uint64_t lo_mask,
                                                      double scale_hel, double scale_avg, double* __restrict__ out,
                                                      double* __restrict__ out_hel, double* __restrict__ part)
{
    typedef typename T::vec vec;
    constexpr int NT = cs16_tiles(NC);
    constexpr bool AREG = NT <= 8;
    const int lane = threadIdx.x & 63;
    const int64_t e0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
    if (e0 >= n_evt) return;
    const int i = lane & 15, g = lane >> 4;
    const int64_t e = e0 + i;
    const bool valid = e < n_evt;
    const int64_t ec = valid ? e : n_evt - 1;
    const int h0 = blockIdx.y * hel_per_group, h1 = min(n_good, h0 + hel_per_group);
    vec A[AREG ? NT : 1];
    if (AREG) {
#pragma unroll
        for (int q = 0; q < NT; ++q) A[q] = *reinterpret_cast<const vec*>(aop + (q * 64 + lane) * 8);
    }
    double me = 0.0;
    for (int h = h0; h < h1; ++h) {
        const float* Jh = J + (int64_t)h * (2 * NC) * ld;
        const auto load = [&](int c, int ri) { return Jh[(int64_t)(2 * c + ri) * ld + ec]; };
        double part_h = sum_lane_groups(cs16_column<NC, T, AREG>(load, A, aop, aop_lo, lo_mask, lane));
        if (out_hel && g == 0 && valid) out_hel[e * n_good + h] = part_h * scale_hel;
        me += part_h;
    }
    if (g == 0 && valid) cs_store(me, e, n_evt, scale_avg, out, part);
}

// The same contractions inside an amplitude kernel whose wave (64 events of one helicity) holds
// its jamps in LDS, Jl[(2c + re/im) * 64 + event]: for each of the four 16-event tiles the lanes
// load the B operands from the other lanes' slots and run the same column body as the separate
// kernels (so each |M_h|^2 is bitwise the same).  Returns this lane's event's D * |M_h|^2.  The
// caller must have completed all jamp updates of the wave (a barrier) before the call.
template <int NC, class JT>
__device__ __forceinline__ double colour_sum_lds(const JT* Jl, const double* __restrict__ aop, int lane)
{
    constexpr int NT = cs64_tiles(NC);
    static_assert(NT <= 24, "operands held in registers");
    const int i = lane & 15, g = lane >> 4;
    double A[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) A[q] = aop[q * 64 + lane];
    double mine = 0.0;
#pragma unroll 1
    for (int j = 0; j < 4; ++j) {  // events 16 j .. 16 j + 15
        const auto load = [&](int c, int ri) { return Jl[(2 * c + ri) * 64 + 16 * j + i]; };
        const double part_h = sum_lane_groups(cs64_column<NC, true>(load, A, aop, lane));
        if (g == j) mine = part_h;  // lane 16 g + i is event 16 g + i
    }
    return mine;
}
template <int NC, class T>
__device__ __forceinline__ double colour_sum_lds_h16(const float* Jl, const typename T::elem* __restrict__ aop,
                                                     const typename T::elem* __restrict__ aop_lo, uint64_t lo_mask,
                                                     int lane)
{
    typedef typename T::vec vec;
    constexpr int NT = cs16_tiles(NC);
    static_assert(NT <= 8, "operands held in registers");
    const int i = lane & 15, g = lane >> 4;
    vec A[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) A[q] = *reinterpret_cast<const vec*>(aop + (q * 64 + lane) * 8);
    double mine = 0.0;
#pragma unroll 1
    for (int j = 0; j < 4; ++j) {
        const auto load = [&](int c, int ri) { return Jl[(2 * c + ri) * 64 + 16 * j + i]; };
        const double part_h = sum_lane_groups(cs16_column<NC, T, true>(load, A, aop, aop_lo, lo_mask, lane));
        if (g == j) mine = part_h;
    }
    return mine;
}

// The helicity sum after the fused colour sum, in the order of the separate colour-sum kernel
// with the same helicity groups: within each group of hel_per_group consecutive helicities from
// zero, then the groups in order (so the result is bitwise that of the separate kernels).
// part_h[h][e] = D |M_h|^2.
static __global__ __launch_bounds__(256) void hel_reduce_grouped(const double* __restrict__ part_h, int n_good,
                                                                 int hel_per_group, int64_t n_evt, double scale,
                                                                 double* __restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n_evt) return;
    double s = 0.0;
    for (int h0 = 0; h0 < n_good; h0 += hel_per_group) {
        const int h1 = min(n_good, h0 + hel_per_group);
        double m = 0.0;
        for (int h = h0; h < h1; ++h) m += part_h[(int64_t)h * n_evt + e];
        s += m;
    }
    out[e] = s * scale;
}

// out[e] = scale * sum over helicity groups of part[group][e], groups in order
static __global__ __launch_bounds__(256) void hel_reduce(const double* __restrict__ part, int groups, int64_t n_evt,
                                                  double scale, double* __restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n_evt) return;
    double s = 0.0;
    for (int k = 0; k < groups; ++k) s += part[(int64_t)k * n_evt + e];
    out[e] = s * scale;
}

}  // namespace me
