// me_abi.cpp -- the C ABI of libme.so (declared in include/me.h).
//
// A handle owns the resident tables of one process: the colour matrix as matrix-core
// operands, the list of helicities that contribute, and one jamp scratch buffer per
// stream.  me_sigma runs, chunk by chunk, the generated amplitude kernel (one lane per
// (event, helicity)) and the colour-sum kernel (matrix cores, helicity sum in FP64).
#include "me.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "colorsum.hpp"
#include "process.hpp"
#include "rambo.hpp"
#include "select.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

const me::ProcessDesc* find_process(const char* name)
{
    const me::ProcessDesc* all[] = {me::process_ee_mumu(), me::process_gg_tt(),    me::process_gg_ttg(),
                                    me::process_gg_ttgg(), me::process_gg_ttggg(), me::process_gg_gg(),
                                    me::process_ee_mumu_z()};
    for (auto* p : all)
        if (p && std::strcmp(p->name, name) == 0) return p;
    return nullptr;
}

struct Scratch {
    void* ptr = nullptr;
    size_t bytes = 0;
};

// Two internal streams per (device, caller stream): the chunks of a process with segment
// kernels alternate between them, so that the reduction of one chunk (bound by HBM) runs beside
// the segment kernels of the next (bound by the VALU).  One pair serves every handle and lives
// until the process ends: a pair per handle would crowd the device's few hardware queues, and
// streams that share a queue run one after the other.
struct Helpers {
    std::mutex mu;   // one call's record/launch/wait sequence at a time
    hipStream_t s[2] = {nullptr, nullptr};
    hipEvent_t start = nullptr, done[2] = {nullptr, nullptr};
};
std::mutex g_helpers_mu;
std::map<std::pair<int, hipStream_t>, Helpers> g_helpers;

// the helper pair of caller stream st on the current device (created on first use); null on failure
Helpers* helpers_for(hipStream_t st)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_helpers_mu);
    Helpers& x = g_helpers[{dev, st}];
    if (!x.start) {
        bool ok = true;
        for (int i = 0; i < 2 && ok; ++i)
            ok = (x.s[i] || hipStreamCreateWithFlags(&x.s[i], hipStreamNonBlocking) == hipSuccess) &&
                 (x.done[i] || hipEventCreateWithFlags(&x.done[i], hipEventDisableTiming) == hipSuccess);
        if (!ok || hipEventCreateWithFlags(&x.start, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    return &x;
}

// Scratch of me_sigma_noalloc: one array per GPU, part of the library's code object, so it is
// allocated when the library is loaded onto a device and held until the process ends.  In host
// code its name is only a stand-in for the symbol: the device address comes from
// hipGetSymbolAddress, per device (each GPU holds its own copy at its own address).
static __device__ __align__(256) unsigned char static_scratch[ME_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_static_mu;
void* g_static_ptr[MAX_DEVICES] = {};

// device address of the current device's static scratch (resolved once per device); null on failure
void* static_scratch_ptr()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
        (void)hipGetLastError();
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(static_scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_static_ptr[dev] = p;
    }
    return g_static_ptr[dev];
}

constexpr double PI = 3.141592653589793238462643383279502884;
constexpr size_t SCRATCH_MIN = size_t(1) << 30;   // jamp scratch per stream: at least 1 GiB,
constexpr int64_t SCRATCH_EVENTS = 4096;          // room for 4096 events, at most 1/8 of the device
constexpr int PREPASS_EVENTS = 1024;
constexpr uint64_t PREPASS_SEED = 0x5EED;
constexpr double PREPASS_THRESHOLD = 1e-20;
constexpr int64_t COLOUR_TARGET_WAVES = 8192;   // colour-sum waves per launch the helicity split aims for

bool is_device_pointer(const void* p)
{
    if (!p) return false;
    hipPointerAttribute_t a;
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

}  // namespace

struct me_handle {
    const me::ProcessDesc* P = nullptr;
    int precision = ME_FP64;
    double mt = 173.0, alpha_em = 1.0 / 132.507, alpha_s = 0.118, g = 0.0;
    int n_good = 0;
    signed char* d_hel_good = nullptr;
    int* d_hel_index = nullptr;  // helicity-combination index of each good helicity
    std::vector<signed char> h_hel_good;
    std::vector<double> hel_ratio;
    double* d_aop64 = nullptr;
    _Float16* d_aop16 = nullptr;
    __bf16* d_aopb = nullptr;      // BF16 A_hi
    __bf16* d_aopb_lo = nullptr;   // BF16 A_lo (exact remainder of numerators BF16 cannot hold)
    uint64_t lo_mask_b16 = 0;      // tiles with a non-zero A_lo
    int groups = 1, hel_per_group = 1;  // helicity split of the colour sum
    bool fuse_colour = true;            // use the amplitude kernel's own colour sum where it has one
    size_t jamp_bytes_per_event = 0;
    size_t bytes_resident = 0;
    int64_t chunk = 0;
    size_t bytes_per_event = 0;
    size_t scratch_cap = 0;
    std::mutex mu;
    std::unordered_map<hipStream_t, Scratch> scratch;
    // optional launch timing: HIP events recorded around every kernel launch on its stream
    bool profiling = false;
    struct Mark {
        hipEvent_t a, b;
        int kind;  // 0 amplitude kernel, 1 colour-sum kernel
    };
    std::vector<Mark> marks;
};

namespace {

// ---------------------------------------------------------------------------------------
// kernel dispatch over the compile-time colour-flow count

struct ColourArgs {
    int64_t ld;
    int n_good, hel_per_group, groups;
    int64_t n;
    double scale_hel, scale_avg;
    double *out, *out_hel, *part;
};

template <int NC>
hipError_t launch_cs64(const double* J, const double* aop, const ColourArgs& a, hipStream_t st)
{
    hipLaunchKernelGGL((me::colour_sum_f64<NC>), dim3((unsigned)((a.n + 63) / 64), (unsigned)a.groups), dim3(256),
                       0, st, J, a.ld, a.n_good, a.hel_per_group, a.n, aop, a.scale_hel, a.scale_avg, a.out, a.out_hel,
                       a.part);
    return hipGetLastError();
}
template <int NC, class T>
hipError_t launch_cs16(const float* J, const typename T::elem* aop, const typename T::elem* aop_lo, uint64_t lo_mask,
                       const ColourArgs& a, hipStream_t st)
{
    hipLaunchKernelGGL((me::colour_sum_h16<NC, T>), dim3((unsigned)((a.n + 63) / 64), (unsigned)a.groups), dim3(256),
                       0, st, J, a.ld, a.n_good, a.hel_per_group, a.n, aop, aop_lo, lo_mask, a.scale_hel, a.scale_avg,
                       a.out, a.out_hel, a.part);
    return hipGetLastError();
}
template <class T>
hipError_t dispatch_cs16(int nc, const float* j, const typename T::elem* aop, const typename T::elem* aop_lo,
                         uint64_t lo_mask, const ColourArgs& a, hipStream_t st)
{
    switch (nc) {
    case 1: return launch_cs16<1, T>(j, aop, aop_lo, lo_mask, a, st);
    case 2: return launch_cs16<2, T>(j, aop, aop_lo, lo_mask, a, st);
    case 6: return launch_cs16<6, T>(j, aop, aop_lo, lo_mask, a, st);
    case 24: return launch_cs16<24, T>(j, aop, aop_lo, lo_mask, a, st);
    case 120: return launch_cs16<120, T>(j, aop, aop_lo, lo_mask, a, st);
    }
    return hipErrorInvalidValue;
}

// colour sum of one chunk; with several helicity groups the partial sums go through `part`
// (groups x n doubles) and a fixed-order reduction
hipError_t colour_sum(const me_handle* h, int precision, const void* J, int64_t ld, int n_good, int hel_per_group,
                      int groups, int64_t n, double* out, double* out_hel, double* part, hipStream_t st)
{
    const double sh = 1.0 / h->P->colour_den, sa = 1.0 / ((double)h->P->colour_den * h->P->avg);
    const ColourArgs a{ld, n_good, hel_per_group, groups, n, sh, sa, out, out_hel, part};
    hipError_t e = hipErrorInvalidValue;
    if (precision == ME_FP64) {
        const double* j = static_cast<const double*>(J);
        switch (h->P->nc) {
        case 1: e = launch_cs64<1>(j, h->d_aop64, a, st); break;
        case 2: e = launch_cs64<2>(j, h->d_aop64, a, st); break;
        case 6: e = launch_cs64<6>(j, h->d_aop64, a, st); break;
        case 24: e = launch_cs64<24>(j, h->d_aop64, a, st); break;
        case 120: e = launch_cs64<120>(j, h->d_aop64, a, st); break;
        }
    } else if (precision == ME_MIXED_FP16) {
        e = dispatch_cs16<me::Fp16Terms>(h->P->nc, static_cast<const float*>(J), h->d_aop16, h->d_aop16, 0, a, st);
    } else {
        e = dispatch_cs16<me::Bf16Terms>(h->P->nc, static_cast<const float*>(J), h->d_aopb, h->d_aopb_lo,
                                         h->lo_mask_b16, a, st);
    }
    if (e != hipSuccess || groups == 1) return e;
    hipLaunchKernelGGL(me::hel_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, part, groups, n, sa, out);
    return hipGetLastError();
}

// helicity groups of the colour sum for launches of up to `chunk` events: enough
// (event tile, group) waves to fill the device when a chunk alone does not
void helicity_groups(const me::ProcessDesc* P, int n_good, int64_t chunk, int* groups, int* hel_per_group)
{
    int64_t G = 1;
    if (P->nc > 6) {
        const int64_t waves = (chunk + 15) / 16;
        G = std::min<int64_t>(std::max<int64_t>((COLOUR_TARGET_WAVES + waves - 1) / waves, 1), n_good);
    }
    *hel_per_group = (int)((n_good + G - 1) / G);
    *groups = (n_good + *hel_per_group - 1) / *hel_per_group;
}

template <int NF>
hipError_t launch_rambo(uint64_t seed, double sqrt_s, const me::FinalMasses& fm, int64_t evt0, int64_t n, double* out,
                        hipStream_t st)
{
    hipLaunchKernelGGL(me::rambo_kernel<NF>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, seed, sqrt_s, fm,
                       evt0, n, out);
    return hipGetLastError();
}

hipError_t rambo(const me_handle* h, uint64_t seed, double sqrt_s, int64_t evt0, int64_t n, double* out, hipStream_t st)
{
    me::FinalMasses fm{};
    const int nf = h->P->npar - 2;
    for (int i = 0; i < nf; ++i) fm.m[i] = h->P->final_massive[i] ? h->mt : 0.0;
    switch (nf) {
    case 2: return launch_rambo<2>(seed, sqrt_s, fm, evt0, n, out, st);
    case 3: return launch_rambo<3>(seed, sqrt_s, fm, evt0, n, out, st);
    case 4: return launch_rambo<4>(seed, sqrt_s, fm, evt0, n, out, st);
    case 5: return launch_rambo<5>(seed, sqrt_s, fm, evt0, n, out, st);
    }
    return hipErrorInvalidValue;
}

double final_mass_sum(const me_handle* h)
{
    double s = 0.0;
    for (int i = 0; i < h->P->npar - 2; ++i) s += h->P->final_massive[i] ? h->mt : 0.0;
    return s;
}

// start/stop a timed launch when profiling is on (events on the launch stream)
struct TimedLaunch {
    me_handle* h;
    hipStream_t st;
    int kind;
    hipEvent_t a = nullptr, b = nullptr;
    TimedLaunch(me_handle* hh, hipStream_t s, int k, bool on) : h(hh), st(s), kind(k)
    {
        if (on && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess) (void)hipEventRecord(a, st);
    }
    void done()
    {
        if (!b) return;
        (void)hipEventRecord(b, st);
        std::lock_guard<std::mutex> lk(h->mu);
        h->marks.push_back({a, b, kind});
        a = b = nullptr;
    }
};

// per-event strong coupling: every tree amplitude of a pure-QCD process carries g_s^(n_par - 2)
// (a three-gluon or quark-gluon vertex one power, the four-gluon vertex two), so |M|^2 computed
// at the handle's alpha_s becomes the per-event value through the factor (a_e / a_0)^(n_par - 2)
__global__ __launch_bounds__(256) void scale_alphas(double* __restrict__ out, const double* __restrict__ alphas,
                                                    double inv_alpha0, int power, int64_t n)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const double r = alphas[e] * inv_alpha0;
    double f = 1.0;
    for (int k = 0; k < power; ++k) f *= r;
    out[e] *= f;
}

// single-diagram enhancement: out[e] *= (sum_h W_chan,h) / (sum_h sum_d W_d,h) from the
// per-lane sums sde[h][0: channel, 1: all][column] of the amplitude kernel; chan[e] < 0: no factor
__global__ __launch_bounds__(256) void sde_apply(double* __restrict__ out, const double* __restrict__ sde,
                                                 const int* __restrict__ chan, int n_good, int64_t ld, int64_t n)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n || chan[e] < 0) return;
    double num = 0.0, den = 0.0;
    for (int h = 0; h < n_good; ++h) {
        num += sde[(int64_t)(2 * h) * ld + e];
        den += sde[(int64_t)(2 * h + 1) * ld + e];
    }
    out[e] *= num / den;
}

// per-event helicity and colour-flow draws (select.hpp); hel_me and w are chunk scratch
struct Selection {
    const double *r_hel, *r_col;
    int *out_hel, *out_col;
    double *hel_me, *w;
};

// amplitude kernel + colour sum (+ the optional per-event kernels) for events [0, n) of `mom`, in
// chunks; scratch: jamps of `chunk` events (jamp_bytes_per_event each), then the helicity-group
// partial sums
int run_chunks(me_handle* h, int precision, const signed char* hel, int n_good, int hel_per_group, int groups,
               int64_t chunk, size_t jamp_bytes_per_event, const double* mom, int64_t n, double* out, double* out_hel,
               void* scratch, hipStream_t st, bool timed = false, const Selection* sel = nullptr,
               const double* alphas = nullptr, const int* chan = nullptr, double* sde = nullptr)
{
    const me::ProcessDesc* P = h->P;
    const bool fp64 = precision == ME_FP64;
    // the colour sum inside the amplitude kernel: plain |M|^2 only (the selection, the
    // per-helicity output and the channel weights read the jamps)
    const bool fused = P->fused_colour && h->fuse_colour && !sel && !out_hel && !chan;
    // the operand tables of the separate colour sum of this precision
    me::FusedColour fcol{nullptr, nullptr, 0, precision, nullptr, 0.0, hel_per_group};
    if (precision == ME_FP64) fcol.aop = h->d_aop64, fcol.form = ME_FP64;
    else if (precision == ME_MIXED_FP16) fcol.aop = h->d_aop16;
    else fcol.aop = h->d_aopb, fcol.aop_lo = h->d_aopb_lo, fcol.lo_mask = h->lo_mask_b16;
    // small processes: the amplitude kernel also sums the helicities (one launch), in a workgroup
    // of all good helicities, or with one lane per event for large enough chunks (FP64, and the
    // mixed forms of one flow whose colour operand the 16-bit type holds exactly)
    const bool hsum_waves = fused && P->hel_sum_in_kernel && n_good <= 16;
    const bool lane_form = fused && P->lane_min_events > 0 &&
                           (precision == ME_FP64 || (P->nc == 1 && !(fcol.lo_mask & 1)));
    void* jamp = scratch;
    double* part = reinterpret_cast<double*>(static_cast<char*>(scratch) + (size_t)chunk * jamp_bytes_per_event);
    for (int64_t c0 = 0; c0 < n; c0 += chunk) {
        const int64_t nc = std::min(chunk, n - c0);
        const int64_t ld = (nc + 63) / 64 * 64;
        const double* m = mom + c0 * P->npar * 4;
        TimedLaunch ta(h, st, 0, timed);
        const int* ch = chan ? chan + c0 : nullptr;
        const bool hsum = hsum_waves || (lane_form && nc >= P->lane_min_events);
        hipError_t e;
        if (fused && hsum) {
            // the amplitude kernel ends with the colour sum and the helicity sum
            fcol.hsum_out = out + c0;
            fcol.hsum_scale = 1.0 / ((double)P->colour_den * P->avg);
            e = fp64 ? P->launch_f64(m, nc, ld, hel, n_good, h->mt, h->g, static_cast<double*>(jamp), nullptr,
                                     nullptr, &fcol, st)
                     : P->launch_f32(m, nc, ld, hel, n_good, h->mt, h->g, static_cast<float*>(jamp), nullptr,
                                     nullptr, &fcol, st);
            ta.done();
            if (e != hipSuccess) return fail(ME_EHIP, std::string("amplitude kernel: ") + hipGetErrorString(e));
        } else if (fused) {
            // the amplitude kernel ends with the colour sum: D |M_h|^2 per (helicity, event) in the
            // jamp scratch, then the helicity sum in the separate kernels' order (same groups)
            e = fp64 ? P->launch_f64(m, nc, ld, hel, n_good, h->mt, h->g, static_cast<double*>(jamp), nullptr,
                                     nullptr, &fcol, st)
                     : P->launch_f32(m, nc, ld, hel, n_good, h->mt, h->g, static_cast<float*>(jamp), nullptr,
                                     nullptr, &fcol, st);
            ta.done();
            if (e != hipSuccess) return fail(ME_EHIP, std::string("amplitude kernel: ") + hipGetErrorString(e));
            TimedLaunch tc(h, st, 1, timed);
            hipLaunchKernelGGL(me::hel_reduce_grouped, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st,
                               static_cast<const double*>(jamp), n_good, hel_per_group, nc,
                               1.0 / ((double)P->colour_den * P->avg), out + c0);
            e = hipGetLastError();
            tc.done();
            if (e != hipSuccess) return fail(ME_EHIP, std::string("helicity-sum kernel: ") + hipGetErrorString(e));
        } else {
            e = fp64 ? P->launch_f64(m, nc, ld, hel, n_good, h->mt, h->g, static_cast<double*>(jamp), ch, sde, nullptr, st)
                     : P->launch_f32(m, nc, ld, hel, n_good, h->mt, h->g, static_cast<float*>(jamp), ch, sde, nullptr, st);
            ta.done();
            if (e != hipSuccess) return fail(ME_EHIP, std::string("amplitude kernel: ") + hipGetErrorString(e));
            TimedLaunch tc(h, st, 1, timed);
            double* oh = sel ? sel->hel_me : (out_hel ? out_hel + c0 * n_good : nullptr);
            e = colour_sum(h, precision, jamp, ld, n_good, hel_per_group, groups, nc, out + c0, oh, part, st);
            tc.done();
            if (e != hipSuccess) return fail(ME_EHIP, std::string("colour-sum kernel: ") + hipGetErrorString(e));
        }
        if (chan) {
            hipLaunchKernelGGL(sde_apply, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, out + c0, sde, ch,
                               n_good, ld, nc);
            e = hipGetLastError();
            if (e != hipSuccess) return fail(ME_EHIP, std::string("channel-weight kernel: ") + hipGetErrorString(e));
        }
        if (alphas && P->coupling == 1) {
            hipLaunchKernelGGL(scale_alphas, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, out + c0,
                               alphas + c0, 1.0 / h->alpha_s, P->npar - 2, nc);
            e = hipGetLastError();
            if (e != hipSuccess) return fail(ME_EHIP, std::string("coupling kernel: ") + hipGetErrorString(e));
        }
        if (sel) {
            const dim3 grid((unsigned)((nc + 255) / 256), (unsigned)P->nc);
            if (fp64)
                hipLaunchKernelGGL(me::lc_weights<double>, grid, dim3(256), 0, st, static_cast<const double*>(jamp), ld,
                                   P->nc, n_good, nc, sel->w);
            else
                hipLaunchKernelGGL(me::lc_weights<float>, grid, dim3(256), 0, st, static_cast<const float*>(jamp), ld,
                                   P->nc, n_good, nc, sel->w);
            hipLaunchKernelGGL(me::select_events, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, sel->hel_me,
                               n_good, sel->w, P->nc, nc, h->d_hel_index, sel->r_hel + c0, sel->r_col + c0,
                               sel->out_hel + c0, sel->out_col + c0);
            e = hipGetLastError();
            if (e != hipSuccess) return fail(ME_EHIP, std::string("selection kernels: ") + hipGetErrorString(e));
        }
    }
    return ME_OK;
}

void free_handle(me_handle* h)
{
    if (!h) return;
    // the caller's streams may be gone by now: wait for the whole device before freeing the
    // scratch that queued work may still use
    bool any = false;
    for (auto& kv : h->scratch) any |= kv.second.ptr != nullptr;
    if (any) (void)hipDeviceSynchronize();
    for (auto& kv : h->scratch)
        if (kv.second.ptr) (void)hipFree(kv.second.ptr);
    for (auto& m : h->marks) {
        (void)hipEventDestroy(m.a);
        (void)hipEventDestroy(m.b);
    }
    if (h->d_hel_good) (void)hipFree(h->d_hel_good);
    if (h->d_hel_index) (void)hipFree(h->d_hel_index);
    if (h->d_aop64) (void)hipFree(h->d_aop64);
    if (h->d_aop16) (void)hipFree(h->d_aop16);
    if (h->d_aopb) (void)hipFree(h->d_aopb);
    if (h->d_aopb_lo) (void)hipFree(h->d_aopb_lo);
    delete h;
}

// colour matrix as matrix-core A operands, block upper-triangular (see colorsum.hpp for the
// layouts and the tile order)
int upload_colour(me_handle* h)
{
    const me::ProcessDesc* P = h->P;
    const int NC = P->nc;
    const int MT = (NC + 15) / 16, KT = (NC + 3) / 4, KB = (MT + 1) / 2;
    // A[r][c] = w * Chat[r][c], w = 1 on diagonal 16-blocks, 2 above, 0 below
    auto A = [&](int r, int c) -> double {
        if (r >= NC || c >= NC || c / 16 < r / 16) return 0.0;
        return (c / 16 == r / 16 ? 1.0 : 2.0) * P->colour_num[r * NC + c];
    };
    std::vector<double> a64;
    for (int mt = 0; mt < MT; ++mt)
        for (int kt = 4 * mt; kt < KT; ++kt)
            for (int l = 0; l < 64; ++l) a64.push_back(A(16 * mt + l % 16, 4 * kt + l / 16));
    std::vector<_Float16> a16;
    std::vector<__bf16> ab, ablo;
    uint64_t lo_mask = 0;
    int q = 0;
    for (int mt = 0; mt < MT; ++mt)
        for (int kb = mt / 2; kb < KB; ++kb, ++q) {
            bool lo_used = false;
            for (int l = 0; l < 64; ++l)
                for (int t = 0; t < 8; ++t) {
                    const int c = 16 * (2 * kb + t / 4) + 4 * (l / 16) + t % 4;
                    const double v = A(16 * mt + l % 16, c);
                    const _Float16 x = (_Float16)v;
                    if ((double)x != v) return fail(ME_EINVAL, "colour matrix numerator not exact in FP16");
                    a16.push_back(x);
                    const __bf16 hi = (__bf16)(float)v;
                    const double rest = v - (double)(float)hi;
                    const __bf16 lo = (__bf16)(float)rest;
                    if ((double)(float)lo != rest) return fail(ME_EINVAL, "colour matrix numerator not exact in two BF16 terms");
                    ab.push_back(hi);
                    ablo.push_back(lo);
                    lo_used |= rest != 0.0;
                }
            if (lo_used) {
                if (q >= 64) return fail(ME_EINVAL, "colour matrix too large for the BF16 tile mask");
                lo_mask |= uint64_t(1) << q;
            }
        }
    h->lo_mask_b16 = lo_mask;
    const size_t b64 = a64.size() * sizeof(double), b16 = a16.size() * sizeof(_Float16), bb = ab.size() * sizeof(__bf16);
    if (hipMalloc(&h->d_aop64, b64) != hipSuccess || hipMalloc(&h->d_aop16, b16) != hipSuccess ||
        hipMalloc(&h->d_aopb, bb) != hipSuccess || hipMalloc(&h->d_aopb_lo, bb) != hipSuccess)
        return fail(ME_ENOMEM, "hipMalloc of the colour tables failed");
    if (hipMemcpy(h->d_aop64, a64.data(), b64, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->d_aop16, a16.data(), b16, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->d_aopb, ab.data(), bb, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->d_aopb_lo, ablo.data(), bb, hipMemcpyHostToDevice) != hipSuccess)
        return fail(ME_EHIP, "upload of the colour tables failed");
    h->bytes_resident += b64 + b16 + 2 * bb;
    return ME_OK;
}

// helicity-filter pre-pass: every helicity on PREPASS_EVENTS fixed RAMBO events, in FP64
int helicity_prepass(me_handle* h, hipStream_t st)
{
    const me::ProcessDesc* P = h->P;
    const int nhel = P->nhel, npar = P->npar;
    std::vector<signed char> all((size_t)nhel * npar);
    for (int hh = 0; hh < nhel; ++hh)
        for (int i = 0; i < npar; ++i) all[(size_t)hh * npar + i] = ((hh >> (npar - 1 - i)) & 1) ? 1 : -1;
    const int64_t n = PREPASS_EVENTS;
    const double sqrt_s = P->coupling ? 1500.0 : 500.0;
    signed char* d_all = nullptr;
    double *d_mom = nullptr, *d_out = nullptr, *d_hel = nullptr, *d_jamp = nullptr;
    const size_t jamp_per_event = (size_t)nhel * 2 * (P->nc + P->nslot) * sizeof(double);
    const int64_t pchunk =
        std::min<int64_t>(n, std::max<int64_t>(64, (int64_t)((size_t(512) << 20) / jamp_per_event) / 64 * 64));
    int groups = 1, hpg = 1;
    helicity_groups(P, nhel, pchunk, &groups, &hpg);
    const size_t jbytes = (jamp_per_event + groups * sizeof(double)) * pchunk;
    int rc = ME_OK;
    if (hipMalloc(&d_all, all.size()) != hipSuccess || hipMalloc(&d_mom, n * npar * 4 * sizeof(double)) != hipSuccess ||
        hipMalloc(&d_out, n * sizeof(double)) != hipSuccess ||
        hipMalloc(&d_hel, (size_t)n * nhel * sizeof(double)) != hipSuccess || hipMalloc(&d_jamp, jbytes) != hipSuccess) {
        rc = fail(ME_ENOMEM, "hipMalloc for the helicity pre-pass failed");
    }
    std::vector<double> out(n), hel((size_t)n * nhel);
    if (rc == ME_OK && hipMemcpyAsync(d_all, all.data(), all.size(), hipMemcpyHostToDevice, st) != hipSuccess)
        rc = fail(ME_EHIP, "upload of the helicity table failed");
    if (rc == ME_OK && rambo(h, PREPASS_SEED, std::max(sqrt_s, 2.0 * final_mass_sum(h) + 1.0), 0, n, d_mom, st) != hipSuccess)
        rc = fail(ME_EHIP, "pre-pass RAMBO launch failed");
    if (rc == ME_OK)
        rc = run_chunks(h, ME_FP64, d_all, nhel, hpg, groups, pchunk, jamp_per_event, d_mom, n, d_out, d_hel, d_jamp, st);
    if (rc == ME_OK) {
        if (hipMemcpyAsync(out.data(), d_out, n * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(hel.data(), d_hel, hel.size() * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            rc = fail(ME_EHIP, "pre-pass copy-back failed");
    }
    if (d_all) (void)hipFree(d_all);
    if (d_mom) (void)hipFree(d_mom);
    if (d_out) (void)hipFree(d_out);
    if (d_hel) (void)hipFree(d_hel);
    if (d_jamp) (void)hipFree(d_jamp);
    if (rc != ME_OK) return rc;
    h->hel_ratio.assign(nhel, 0.0);
    for (int64_t e = 0; e < n; ++e) {
        const double tot = out[e] * P->avg;
        if (!(tot > 0.0)) continue;
        for (int hh = 0; hh < nhel; ++hh) h->hel_ratio[hh] = std::max(h->hel_ratio[hh], hel[e * nhel + hh] / tot);
    }
    h->h_hel_good.clear();
    for (int hh = 0; hh < nhel; ++hh)
        if (h->hel_ratio[hh] > PREPASS_THRESHOLD)
            h->h_hel_good.insert(h->h_hel_good.end(), all.begin() + (size_t)hh * npar, all.begin() + (size_t)(hh + 1) * npar);
    h->n_good = (int)(h->h_hel_good.size() / npar);
    if (h->n_good == 0) return fail(ME_EINVAL, "helicity pre-pass found no contributing helicity");
    std::vector<int> index;
    for (int hh = 0; hh < nhel; ++hh)
        if (h->hel_ratio[hh] > PREPASS_THRESHOLD) index.push_back(hh);
    if (hipMalloc(&h->d_hel_good, h->h_hel_good.size()) != hipSuccess ||
        hipMalloc(&h->d_hel_index, index.size() * sizeof(int)) != hipSuccess)
        return fail(ME_ENOMEM, "hipMalloc of the helicity list failed");
    if (hipMemcpy(h->d_hel_good, h->h_hel_good.data(), h->h_hel_good.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->d_hel_index, index.data(), index.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
        return fail(ME_EHIP, "upload of the helicity list failed");
    h->bytes_resident += h->h_hel_good.size() + index.size() * sizeof(int);
    return ME_OK;
}

}  // namespace

extern "C" {

const char* me_last_error(void) { return g_err.c_str(); }

me_handle* me_create(const char* process, const double* masses, int n_masses, const double* couplings,
                     int n_couplings, int precision, void* stream)
{
    g_err.clear();
    if (!process) { fail(ME_EINVAL, "process is NULL"); return nullptr; }
    const me::ProcessDesc* P = find_process(process);
    if (!P) { fail(ME_ENOPROC, std::string("unknown process: ") + process); return nullptr; }
    if (precision != ME_FP64 && precision != ME_MIXED_FP16 && precision != ME_MIXED_BF16) {
        fail(ME_EINVAL, "unknown precision");
        return nullptr;
    }
    if ((masses && (n_masses < 1 || n_masses > 2)) || (couplings && n_couplings != 2)) {
        fail(ME_EINVAL, "masses: {m_t} or {m_t, w_t}; couplings: {alpha_em, alpha_s}");
        return nullptr;
    }
    me_handle* h = new me_handle();
    h->P = P;
    h->precision = precision;
    if (masses) {
        h->mt = masses[0];
        if (n_masses == 2 && masses[1] != 0.0) {
            fail(ME_EINVAL, "non-zero top width is not supported");
            delete h;
            return nullptr;
        }
    }
    if (couplings) {
        h->alpha_em = couplings[0];
        h->alpha_s = couplings[1];
    }
    if (!(h->mt >= 0.0) || !(h->alpha_em > 0.0) || !(h->alpha_s > 0.0)) {
        fail(ME_EINVAL, "the top mass must be >= 0 and the couplings positive");
        delete h;
        return nullptr;
    }
    h->g = std::sqrt(4.0 * PI * (P->coupling ? h->alpha_s : h->alpha_em));
    // set-up of me_sigma_noalloc: the device address of this GPU's static scratch (a failure
    // here is reported by that entry point, which tries again)
    (void)static_scratch_ptr();
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (upload_colour(h) != ME_OK || helicity_prepass(h, st) != ME_OK) {
        std::string msg = g_err;
        free_handle(h);
        g_err = msg;
        return nullptr;
    }
    const size_t rsize = (precision == ME_FP64) ? sizeof(double) : sizeof(float);
    h->jamp_bytes_per_event = (size_t)h->n_good * 2 * (P->nc + P->nslot) * rsize;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) total_b = size_t(64) << 30;
    h->scratch_cap = std::max(SCRATCH_MIN, std::min<size_t>(SCRATCH_EVENTS * h->jamp_bytes_per_event, total_b / 8));
    int64_t chunk = (int64_t)(h->scratch_cap / h->jamp_bytes_per_event) / 64 * 64;
    h->chunk = std::max<int64_t>(64, chunk);
    // the helicity split is fixed per handle, so an event's result does not depend on the batch
    helicity_groups(P, h->n_good, h->chunk, &h->groups, &h->hel_per_group);
    h->bytes_per_event = h->jamp_bytes_per_event + (h->groups > 1 ? h->groups * sizeof(double) : 0);
    return h;
}

void me_destroy(me_handle* h) { free_handle(h); }

int me_set_option(me_handle* h, int option, int value)
{
    if (!h) return fail(ME_EINVAL, "handle is NULL");
    if (option != ME_OPT_FUSED_COLOUR) return fail(ME_EINVAL, "unknown option");
    if (value != 0 && value != 1) return fail(ME_EINVAL, "option value must be 0 or 1");
    h->fuse_colour = value != 0;
    return ME_OK;
}

int me_info(const me_handle* h, me_info_t* out)
{
    if (!h || !out) return fail(ME_EINVAL, "NULL argument");
    const me::ProcessDesc* P = h->P;
    out->n_par = P->npar;
    out->n_diagrams = P->n_diagrams;
    out->n_amplitudes = P->n_amplitudes;
    out->n_colors = P->nc;
    out->n_hel = P->nhel;
    out->n_good_hel = h->n_good;
    out->precision = h->precision;
    out->avg_factor = P->avg;
    out->sym_factor = P->sym;
    out->flops_amp_lane = P->flops_lane;
    out->flops_amp_exec_lane = P->flops_exec_lane;
    out->n_partial_slots = P->nslot;
    out->flops_colour_lane = 4.0 * P->nc * P->nc + 4.0 * P->nc + 1.0;
    out->bytes_resident = (int64_t)h->bytes_resident;
    out->bytes_per_event_scratch = (int64_t)h->bytes_per_event;
    out->chunk_events = h->chunk;
    out->n_order = P->n_order;
    out->helicity_groups = h->groups;
    out->lines_per_diagram = P->lines_per_diagram;
    out->fused_colour = (P->fused_colour && h->fuse_colour) ? 1 : 0;
    return ME_OK;
}

int me_good_helicities(const me_handle* h, signed char* out)
{
    if (!h || !out) return fail(ME_EINVAL, "NULL argument");
    std::memcpy(out, h->h_hel_good.data(), h->h_hel_good.size());
    return h->n_good;
}

int me_helicity_ratios(const me_handle* h, double* out)
{
    if (!h || !out) return fail(ME_EINVAL, "NULL argument");
    std::memcpy(out, h->hel_ratio.data(), h->hel_ratio.size() * sizeof(double));
    return (int)h->hel_ratio.size();
}

int rambo_momenta(const me_handle* h, uint64_t seed, double sqrt_s, int64_t evt0, int64_t n_evt, double* out,
                  void* stream)
{
    if (!h) return fail(ME_EINVAL, "handle is NULL");
    if (n_evt < 0 || evt0 < 0) return fail(ME_EINVAL, "negative event count or offset");
    if (n_evt == 0) return ME_OK;
    if (!(sqrt_s > final_mass_sum(h))) return fail(ME_EINVAL, "sqrt_s must exceed the sum of final-state masses");
    if (!is_device_pointer(out)) return fail(ME_EINVAL, "out must be a device pointer");
    hipError_t e = rambo(h, seed, sqrt_s, evt0, n_evt, out, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(ME_EHIP, std::string("RAMBO kernel: ") + hipGetErrorString(e));
    return ME_OK;
}

namespace {

// scratch of `need` bytes for stream st (grown when too small); null on failure
void* stream_scratch(me_handle* h, hipStream_t st, size_t need)
{
    std::lock_guard<std::mutex> lk(h->mu);
    Scratch& s = h->scratch[st];
    if (s.bytes < need) {
        if (s.ptr) {
            (void)hipStreamSynchronize(st);
            (void)hipFree(s.ptr);
            s.ptr = nullptr;
            s.bytes = 0;
        }
        size_t want = std::max(need, std::min<size_t>(h->scratch_cap, 2 * s.bytes));
        if (hipMalloc(&s.ptr, want) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        s.bytes = want;
    }
    return s.ptr;
}

// the plain |M|^2 in chunks that alternate between the two internal streams of the caller's
// stream st; st waits for both at the end
int sigma_piped(me_handle* h, const double* momenta, int64_t n_evt, double* out, const double* alphas,
                hipStream_t st, int64_t chunk)
{
    Helpers* hp = helpers_for(st);
    if (!hp) return fail(ME_EHIP, "creating the internal streams failed");
    std::lock_guard<std::mutex> lk(hp->mu);
    const size_t need = (size_t)chunk * h->bytes_per_event;
    void* scr[2];
    for (int i = 0; i < 2; ++i)
        if (!(scr[i] = stream_scratch(h, hp->s[i], need))) return fail(ME_ENOMEM, "hipMalloc of the jamp scratch failed");
    // the inputs are ready once the caller's stream reaches this point
    if (hipEventRecord(hp->start, st) != hipSuccess) return fail(ME_EHIP, "event record failed");
    for (int i = 0; i < 2; ++i)
        if (hipStreamWaitEvent(hp->s[i], hp->start, 0) != hipSuccess)
            return fail(ME_EHIP, "ordering the internal streams after the caller's stream failed");
    const int npar = h->P->npar;
    int64_t k = 0;
    int rc = ME_OK;
    for (int64_t c0 = 0; c0 < n_evt && rc == ME_OK; c0 += chunk, ++k) {
        const int64_t nc = std::min(chunk, n_evt - c0);
        const int i = (int)(k & 1);
        rc = run_chunks(h, h->precision, h->d_hel_good, h->n_good, h->hel_per_group, h->groups, chunk,
                        h->jamp_bytes_per_event, momenta + c0 * npar * 4, nc, out + c0, nullptr, scr[i], hp->s[i],
                        h->profiling, nullptr, alphas ? alphas + c0 : nullptr);
    }
    // joined also after an error, so that no queued chunk outlives the caller's view of the call
    for (int i = 0; i < 2; ++i) {
        const bool joined = hipEventRecord(hp->done[i], hp->s[i]) == hipSuccess &&
                            hipStreamWaitEvent(st, hp->done[i], 0) == hipSuccess;
        if (!joined && rc == ME_OK) rc = fail(ME_EHIP, "joining the internal streams to the caller's stream failed");
    }
    return rc;
}

// How a call of n_evt events runs: equal chunks no larger than the handle's chunk; for processes
// with segment kernels, the plain |M|^2 of more than one chunk alternates its chunks between two
// internal streams, each with a scratch buffer of its own (full-size chunks keep the short segment
// launches several rounds of waves deep).  Scratch per event of a chunk: the plain |M|^2 of a
// kernel with the colour sum inside keeps one double per (event, helicity); otherwise the jamps
// (and partial slots) of every helicity plus the helicity-group sums, and `extra` bytes.
struct CallPlan {
    int64_t chunk;
    bool piped;
    size_t per_event;
};
CallPlan plan_call(const me_handle* h, int64_t n_evt, bool plain, size_t extra)
{
    CallPlan c;
    const int64_t n_chunks = (n_evt + h->chunk - 1) / h->chunk;
    c.chunk = ((n_evt + n_chunks - 1) / n_chunks + 63) / 64 * 64;
    c.piped = plain && h->P->nslot > 0 && n_evt > h->chunk;
    const bool fused = plain && h->P->fused_colour && h->fuse_colour;
    c.per_event = fused ? (size_t)h->n_good * sizeof(double) : h->bytes_per_event + extra;
    return c;
}

// me_sigma and its variants: equal chunks through the stream's scratch
int sigma_impl(me_handle* h, const double* momenta, int64_t n_evt, double* out_me2, double* out_hel,
               const Selection* sel_in, void* stream, const double* alphas = nullptr, const int* chan = nullptr)
{
    if (!h) return fail(ME_EINVAL, "handle is NULL");
    if (n_evt < 0) return fail(ME_EINVAL, "negative event count");
    if (n_evt == 0) return ME_OK;
    if (!is_device_pointer(momenta) || !is_device_pointer(out_me2) || (out_hel && !is_device_pointer(out_hel)))
        return fail(ME_EINVAL, "momenta and outputs must be device pointers");
    if (sel_in && (!is_device_pointer(sel_in->r_hel) || !is_device_pointer(sel_in->r_col) ||
                   !is_device_pointer(sel_in->out_hel) || !is_device_pointer(sel_in->out_col)))
        return fail(ME_EINVAL, "random numbers and choices must be device pointers");
    if (alphas && !is_device_pointer(alphas)) return fail(ME_EINVAL, "alpha_s must be a device pointer");
    if (chan && !is_device_pointer(chan)) return fail(ME_EINVAL, "channel ids must be a device pointer");
    if (chan && !h->P->sde_supported) return fail(ME_EINVAL, "no single-diagram channel weights for this process");
    if (reinterpret_cast<uintptr_t>(momenta) % 16 != 0) return fail(ME_EINVAL, "momenta must be 16-byte aligned");
    hipStream_t st = static_cast<hipStream_t>(stream);
    // selection adds |M_h|^2 and the leading-colour weights of one chunk
    const size_t sel_bytes = sel_in ? (size_t)(h->n_good + h->P->nc) * sizeof(double) : 0;
    // channel weights add two sums per (event, helicity)
    const size_t sde_bytes = chan ? (size_t)2 * h->n_good * sizeof(double) : 0;
    const CallPlan plan = plan_call(h, n_evt, !sel_in && !out_hel && !chan, sel_bytes + sde_bytes);
    const int64_t chunk = plan.chunk;
    if (plan.piped) return sigma_piped(h, momenta, n_evt, out_me2, alphas, st, chunk);
    void* scratch = stream_scratch(h, st, (size_t)chunk * plan.per_event);
    if (!scratch) return fail(ME_ENOMEM, "hipMalloc of the jamp scratch failed");
    Selection sel{};
    if (sel_in) {
        sel = *sel_in;
        sel.hel_me = reinterpret_cast<double*>(static_cast<char*>(scratch) + (size_t)chunk * h->bytes_per_event);
        sel.w = sel.hel_me + (size_t)chunk * h->n_good;
    }
    double* sde = chan ? reinterpret_cast<double*>(static_cast<char*>(scratch) +
                                                   (size_t)chunk * (h->bytes_per_event + sel_bytes))
                       : nullptr;
    return run_chunks(h, h->precision, h->d_hel_good, h->n_good, h->hel_per_group, h->groups, chunk,
                      h->jamp_bytes_per_event, momenta, n_evt, out_me2, out_hel, scratch, st, h->profiling,
                      sel_in ? &sel : nullptr, alphas, chan, sde);
}

}  // namespace

int me_reserve_scratch(me_handle* h, int64_t n_evt, void* stream)
{
    if (!h) return fail(ME_EINVAL, "handle is NULL");
    if (n_evt < 0) return fail(ME_EINVAL, "negative event count");
    if (n_evt == 0) return ME_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // every plain call of at most n_evt events: chunks of at most min(n_evt rounded up, chunk) on
    // `stream`, and full chunks on both internal streams where such a call is piped
    const CallPlan one = plan_call(h, std::min<int64_t>(n_evt, h->chunk), true, 0);
    if (!stream_scratch(h, st, (size_t)one.chunk * one.per_event))
        return fail(ME_ENOMEM, "hipMalloc of the jamp scratch failed");
    if (plan_call(h, n_evt, true, 0).piped) {
        Helpers* hp = helpers_for(st);
        if (!hp) return fail(ME_EHIP, "creating the internal streams failed");
        for (int i = 0; i < 2; ++i)
            if (!stream_scratch(h, hp->s[i], (size_t)h->chunk * h->bytes_per_event))
                return fail(ME_ENOMEM, "hipMalloc of the jamp scratch failed");
    }
    return ME_OK;
}

int me_release_scratch(me_handle* h, void* stream)
{
    if (!h) return fail(ME_EINVAL, "handle is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<hipStream_t> ss{st};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(ME_EHIP, "hipGetDevice failed");
    {
        std::lock_guard<std::mutex> lk(g_helpers_mu);
        auto it = g_helpers.find({dev, st});
        if (it != g_helpers.end())
            for (int i = 0; i < 2; ++i)
                if (it->second.s[i]) ss.push_back(it->second.s[i]);
    }
    std::lock_guard<std::mutex> lk(h->mu);
    int rc = ME_OK;
    for (hipStream_t x : ss) {
        auto it = h->scratch.find(x);
        if (it == h->scratch.end()) continue;
        if (it->second.ptr && (hipStreamSynchronize(x) != hipSuccess || hipFree(it->second.ptr) != hipSuccess))
            rc = fail(ME_EHIP, "freeing the jamp scratch failed");
        h->scratch.erase(it);
    }
    return rc;
}

int64_t me_scratch_bytes(const me_handle* h)
{
    if (!h) return fail(ME_EINVAL, "handle is NULL");
    std::lock_guard<std::mutex> lk(const_cast<me_handle*>(h)->mu);
    int64_t n = 0;
    for (auto& kv : h->scratch) n += (int64_t)kv.second.bytes;
    return n;
}

int me_sigma_hel(me_handle* h, const double* momenta, int64_t n_evt, double* out_me2, double* out_hel, void* stream)
{
    return sigma_impl(h, momenta, n_evt, out_me2, out_hel, nullptr, stream);
}

int me_sigma_select(me_handle* h, const double* momenta, int64_t n_evt, const double* rnd_hel, const double* rnd_col,
                    double* out_me2, int* out_hel, int* out_col, void* stream)
{
    if (n_evt > 0 && (!rnd_hel || !rnd_col || !out_hel || !out_col))
        return fail(ME_EINVAL, "random numbers and choices must be given");
    const Selection sel{rnd_hel, rnd_col, out_hel, out_col, nullptr, nullptr};
    return sigma_impl(h, momenta, n_evt, out_me2, nullptr, &sel, stream);
}

int me_sigma_alphas(me_handle* h, const double* momenta, int64_t n_evt, const double* alpha_s_evt, double* out_me2,
                    void* stream)
{
    if (n_evt > 0 && !alpha_s_evt) return fail(ME_EINVAL, "alpha_s_evt must be given");
    return sigma_impl(h, momenta, n_evt, out_me2, nullptr, nullptr, stream, alpha_s_evt);
}

int me_sigma_channel(me_handle* h, const double* momenta, int64_t n_evt, const int* channel, double* out_me2,
                     void* stream)
{
    if (n_evt > 0 && !channel) return fail(ME_EINVAL, "channel ids must be given");
    return sigma_impl(h, momenta, n_evt, out_me2, nullptr, nullptr, stream, nullptr, channel);
}

int me_diagrams(const me_handle* h, int* out)
{
    if (!h || !out) return fail(ME_EINVAL, "NULL argument");
    if (!h->P->sde_supported) return fail(ME_EINVAL, "no single-diagram channel weights for this process");
    std::memcpy(out, h->P->diagram_lines, sizeof(int) * h->P->n_diagrams * h->P->lines_per_diagram);
    return h->P->n_diagrams;
}

int me_colour_flows(const me_handle* h, int* out)
{
    if (!h || !out) return fail(ME_EINVAL, "NULL argument");
    const int no = h->P->n_order;
    if (no > 0) std::memcpy(out, h->P->orderings, sizeof(int) * h->P->nc * no);
    return h->P->nc;
}

int me_profile(me_handle* h, int enable, double* ms_amp, double* ms_colour, int64_t* n_amp, int64_t* n_colour)
{
    if (!h) return fail(ME_EINVAL, "handle is NULL");
    std::vector<me_handle::Mark> marks;
    {
        std::lock_guard<std::mutex> lk(h->mu);
        marks.swap(h->marks);
        h->profiling = enable != 0;
    }
    double t[2] = {0.0, 0.0};
    int64_t c[2] = {0, 0};
    int rc = ME_OK;
    for (auto& m : marks) {
        float ms = 0.0f;
        if (hipEventSynchronize(m.b) != hipSuccess || hipEventElapsedTime(&ms, m.a, m.b) != hipSuccess)
            rc = fail(ME_EHIP, "reading launch timers failed");
        t[m.kind] += ms;
        c[m.kind] += 1;
        (void)hipEventDestroy(m.a);
        (void)hipEventDestroy(m.b);
    }
    if (ms_amp) *ms_amp = t[0];
    if (ms_colour) *ms_colour = t[1];
    if (n_amp) *n_amp = c[0];
    if (n_colour) *n_colour = c[1];
    return rc;
}

int me_sigma(me_handle* h, const double* momenta, int64_t n_evt, double* out_me2, void* stream)
{
    return me_sigma_hel(h, momenta, n_evt, out_me2, nullptr, stream);
}

int me_sigma_noalloc(me_handle* h, const double* momenta, int64_t n_evt, double* out_me2, void* stream)
{
    if (!h) return fail(ME_EINVAL, "handle is NULL");
    if (n_evt < 0) return fail(ME_EINVAL, "negative event count");
    if (n_evt == 0) return ME_OK;
    if (!is_device_pointer(momenta) || !is_device_pointer(out_me2))
        return fail(ME_EINVAL, "momenta and out_me2 must be device pointers");
    if (reinterpret_cast<uintptr_t>(momenta) % 16 != 0) return fail(ME_EINVAL, "momenta must be 16-byte aligned");
    void* scr = static_scratch_ptr();
    if (!scr) return fail(ME_EHIP, "hipGetSymbolAddress of the static scratch failed");
    const me::ProcessDesc* P = h->P;
    // scratch per event: D |M_h|^2 per good helicity where the amplitude kernel does the colour sum,
    // else the jamps (and partial slots) of every good helicity plus the helicity-group sums
    const bool fused = P->fused_colour && h->fuse_colour;
    const size_t per_event = fused ? (size_t)h->n_good * sizeof(double) : h->bytes_per_event;
    const int64_t fit = (int64_t)(ME_NOALLOC_SCRATCH_BYTES / per_event) / 64 * 64;
    if (fit < 64)
        return fail(ME_ENOMEM, std::string("me_sigma_noalloc: ") + P->name + " needs " +
                                   std::to_string(64 * per_event) + " bytes of scratch for one 64-event chunk; the "
                                   "static scratch holds " + std::to_string((size_t)ME_NOALLOC_SCRATCH_BYTES));
    // the handle's own chunk where it fits (the launches of me_sigma), else the largest that does;
    // the helicity groups are the handle's, so every event's result is bitwise that of me_sigma
    const int64_t cap = std::min<int64_t>(h->chunk, fit);
    const int64_t n_chunks = (n_evt + cap - 1) / cap;
    const int64_t chunk = ((n_evt + n_chunks - 1) / n_chunks + 63) / 64 * 64;
    const size_t jamp_per_event = fused ? per_event : h->jamp_bytes_per_event;
    return run_chunks(h, h->precision, h->d_hel_good, h->n_good, h->hel_per_group, h->groups, chunk, jamp_per_event,
                      momenta, n_evt, out_me2, nullptr, scr, static_cast<hipStream_t>(stream));
}

}  // extern "C"
