// process.hpp -- descriptor of a generated process, shared by the generated kernels and the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace me {

// chan == nullptr: plain kernels; otherwise chan[n_evt] channel ids and sde[n_good][2][ld] the
// per-lane single-diagram sums (channel, all)
// The colour sum inside the amplitude kernel (processes with fused_colour): the operand tables
// of the separate colour-sum kernel of the same form.  With a FusedColour the kernel writes
// D |M_h|^2 as doubles to ((double*)jamp)[h * n_evt + event] instead of the jamps.
struct FusedColour {
    const void* aop;     // FP64 tiles (FP64 kernel) or FP16 / BF16 hi tiles (FP32 kernel)
    const void* aop_lo;  // BF16 lo tiles (BF16 form)
    uint64_t lo_mask;    // tiles with a non-zero lo part (BF16 form)
    int form;            // ME_FP64, ME_MIXED_FP16 or ME_MIXED_BF16 (me.h)
    // processes with hel_sum_in_kernel or lane_min_events: if hsum_out is set, the kernel also
    // sums the good helicities (one workgroup holding all of an event block's, or one lane per
    // event for batches of at least lane_min_events), in groups of hel_per_group from the first
    // (the order of the separate helicity-sum kernel), times hsum_scale, into hsum_out[event];
    // nothing goes to the jamp scratch
    double* hsum_out;
    double hsum_scale;
    int hel_per_group;
};

// fc: null, or the fused colour sum (then chan must be null)
typedef hipError_t (*amp_launch_f64)(const double* mom, int64_t n_evt, int64_t ld, const signed char* hel,
                                     int n_good, double mt, double g, double* jamp, const int* chan, double* sde,
                                     const FusedColour* fc, hipStream_t st);
typedef hipError_t (*amp_launch_f32)(const double* mom, int64_t n_evt, int64_t ld, const signed char* hel,
                                     int n_good, double mt, double g, float* jamp, const int* chan, double* sde,
                                     const FusedColour* fc, hipStream_t st);

struct ProcessDesc {
    const char* name;
    int npar;          // particles, incoming first
    int nc;            // colour flows (jamps)
    int nhel;          // helicity combinations, 2^npar
    int avg;           // initial-state spin x colour average
    int sym;           // identical final-state particle factor (reported, not applied)
    int coupling;      // 0: alpha_em (QED), 1: alpha_s (QCD)
    const int* colour_num;     // nc x nc integer numerators of the colour matrix
    int colour_den;            // their common denominator
    const int* final_massive;  // npar-2 flags: final-state particle carries the top mass
    const int* orderings;      // nc x n_order: the gluon order of each colour flow
    int n_order;               // entries per flow (gluons of the quark line; for gg->gg the three non-root gluons)
    int n_diagrams;            // Feynman diagrams
    int n_amplitudes;          // vertex contractions (four-gluon vertices count 3)
    double flops_lane;         // algorithmic flops of the amplitude kernel per (event, helicity)
    double flops_exec_lane;    // flops it executes (more when segments recompute currents)
    int nslot;                 // partial jamp slots per (event, helicity); 0: jamps written directly
    const int* diagram_lines;  // n_diagrams x lines_per_diagram internal-line masks (0-padded)
    int lines_per_diagram;
    int sde_supported;         // single-diagram channel weights available
    int fused_colour;          // the amplitude kernels can do the colour sum themselves (FusedColour)
    int hel_sum_in_kernel;     // ... and the helicity sum (FusedColour.hsum_out; at most 16 good helicities)
    int64_t lane_min_events;   // batches from this size can take the kernel with one lane per event, which
                               // also sums the helicities: FP64, and mixed forms of one flow (0: none)
    amp_launch_f64 launch_f64;
    amp_launch_f32 launch_f32;
};

const ProcessDesc* process_ee_mumu();
const ProcessDesc* process_gg_tt();
const ProcessDesc* process_gg_ttg();
const ProcessDesc* process_gg_ttgg();
const ProcessDesc* process_gg_ttggg();
const ProcessDesc* process_gg_gg();
const ProcessDesc* process_ee_mumu_z();

}  // namespace me
