// select.hpp -- event-by-event helicity and leading-colour choice.
//
// An unweighted event records one helicity configuration and one colour flow (the per-event
// choices that the paper, Sec. 4, lists as still missing from its event files).  For event e
// the helicity is drawn among the filtered helicities with probability |M_h|^2 / sum_h |M_h|^2
// (colour-summed, from the colour sum), and the colour flow k with probability
// w_k / sum_k w_k, w_k = sum_h |J_k,h|^2 the leading-colour weight of flow k (the diagonal
// of the colour sum, summed over the same helicities).  Each draw takes the smallest index j
// with r * W < sum_{i <= j} w_i, with the caller's uniform r in [0, 1) and the sums formed in
// FP64 in index order; if rounding leaves no such j, the last index of positive weight.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace me {

// w[k][e] = sum over helicities of |J_k|^2, for the jamps jamp[h][2k + re/im][column] of one chunk
template <class R>
__global__ __launch_bounds__(256) void lc_weights(const R* __restrict__ J, int64_t ld, int nc, int n_good,
                                                  int64_t n_evt, double* __restrict__ w)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int k = blockIdx.y;
    if (e >= n_evt) return;
    double s = 0.0;
    for (int h = 0; h < n_good; ++h) {
        const R* Jh = J + (int64_t)h * (2 * nc) * ld;
        const double re = (double)Jh[(int64_t)(2 * k) * ld + e], im = (double)Jh[(int64_t)(2 * k + 1) * ld + e];
        s += re * re + im * im;
    }
    w[(int64_t)k * n_evt + e] = s;
}

// index drawn from the weights x[0..n) (stride `stride` between consecutive weights) with uniform r
__device__ __forceinline__ int draw(const double* x, int n, int64_t stride, double r)
{
    double tot = 0.0;
    for (int j = 0; j < n; ++j) tot += x[j * stride];
    const double target = r * tot;
    double cum = 0.0;
    int last = 0;
    for (int j = 0; j < n; ++j) {
        const double v = x[j * stride];
        cum += v;
        if (v > 0.0) last = j;
        if (target < cum) return j;
    }
    return last;
}

// hel_me[e * n_good + h]: colour-summed |M_h|^2; w[k * n_evt + e]: leading-colour weights;
// hel_index[h]: the helicity-combination index of the h-th filtered helicity
__global__ __launch_bounds__(256) void select_events(const double* __restrict__ hel_me, int n_good,
                                                     const double* __restrict__ w, int nc, int64_t n_evt,
                                                     const int* __restrict__ hel_index,
                                                     const double* __restrict__ r_hel, const double* __restrict__ r_col,
                                                     int* __restrict__ out_hel, int* __restrict__ out_col)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n_evt) return;
    out_hel[e] = hel_index[draw(hel_me + e * n_good, n_good, 1, r_hel[e])];
    out_col[e] = draw(w + e, nc, n_evt, r_col[e]);
}

}  // namespace me
