/* me.h -- C ABI of the MI355X leading-order matrix-element library (libme.so).
 *
 * The library computes, for every phase-space event independently, the tree-level
 * matrix element of a fixed process, summed over helicities and colours and averaged
 * over the initial states (the per-event ME calculation of the paper, Sec. 1 and 2; the
 * process set ee->mumu, gg->tt~ + 0..3 gluons of Sec. 2).  The GPU path evaluates every
 * Feynman diagram with HELAS-style wavefunctions, accumulates the colour-flow amplitudes,
 * contracts them with the colour matrix (on the matrix cores; in FP64 with up to six flows,
 * as scalar fused multiply-adds in each lane) and sums the helicities that a pre-pass found
 * to contribute.
 *
 * Conventions.  Units GeV; momenta (E, px, py, pz), metric (+,-,-,-).  Particle order:
 *   ee_mumu  (e+, e-, mu+, mu-)
 *   gg_tt    (g, g, t, t~)          gg_ttg  (g, g, t, t~, g)
 *   gg_ttgg  (g, g, t, t~, g, g)    gg_ttggg (g, g, t, t~, g, g, g)
 *   gg_gg    (g, g, g, g)           (test process)
 *   ee_mumu_z (e+, e-, mu+, mu-)     photon and Z exchange (M_Z = 91.188, Gamma_Z = 2.441404,
 *                                    M_W = 80.419 GeV, sin^2 theta_W = 1 - M_W^2/M_Z^2)
 * The returned value is the spin- and colour-averaged |M|^2 WITHOUT the identical-
 * particle factor (me_info reports that factor as sym_factor).
 *
 * Memory.  Event buffers are DEVICE memory owned by the caller and must stay alive until
 * the work enqueued on `stream` has completed.  `stream` is a hipStream_t (NULL: the null
 * stream).  Calls enqueue work and return without synchronising, except me_create, which
 * runs the helicity pre-pass and synchronises on `stream` once.
 *
 * Errors.  Functions return ME_OK (0) or a negative code; me_create returns NULL on
 * error.  me_last_error() gives a message for the calling thread's last error.  No
 * exception crosses the ABI.  HIP errors of asynchronous work surface at a later call.
 */
#ifndef ME_H
#define ME_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ME_FP64 = 0, ME_MIXED_FP16 = 1, ME_MIXED_BF16 = 2 };
enum { ME_OK = 0, ME_EINVAL = -1, ME_ENOPROC = -2, ME_ENOMEM = -3, ME_EHIP = -4 };

typedef struct me_handle me_handle; /* opaque, owned by the library */

/* Create a handle for `process` (see the list above).
 * masses:    {m_t} or {m_t, w_t}; the top width must be 0 (no width in propagators).
 *            m_t >= 0 (0: the massless-quark limit).  Ignored by ee_mumu and gg_gg.
 *            NULL: m_t = 173.
 * couplings: {alpha_em, alpha_s}; NULL: {1/132.507, 0.118}.  Fixed couplings.
 * precision: ME_FP64 (all FP64), ME_MIXED_FP16 (FP32 wavefunctions and amplitudes,
 *            FP16 matrix-core colour sum with FP32 accumulation, FP64 momenta,
 *            propagator denominators and helicity sum) or ME_MIXED_BF16 (as ME_MIXED_FP16
 *            with BF16 matrix-core operands).  In both mixed forms each jamp column is
 *            scaled by a power of two and split exactly into two 16-bit terms.  (The
 *            paper's reduced-precision variant is all-single; Sec. 2, Tables 1 and 2.)
 * Copies the arrays, uploads the colour matrix and helicity table, and runs the
 * helicity-filter pre-pass: 1024 RAMBO events from the fixed seed 0x5EED, every helicity
 * evaluated, helicity h kept iff max_e |M_h(e)|^2 / |M(e)|^2 > 1e-20.  The mask does not
 * depend on later inputs.  Returns NULL on error. */
me_handle *me_create(const char *process, const double *masses, int n_masses,
                     const double *couplings, int n_couplings, int precision, void *stream);

/* RAMBO phase-space points for the handle's process at energy sqrt_s.  In the paper's standalone
 * application the random numbers and the phase-space sampling are simple components that can run
 * entirely on the GPU beside the matrix element (Sec. 1); the generator (RAMBO) and the RNG are
 * readings, as the paper names neither.  The handle argument (for the final-state masses) and
 * evt0 (the first event of the stream, so that a batch can be made in pieces) are additions:
 * out = DEVICE double[n_evt][n_par][4], events evt0 .. evt0+n_evt-1 of the stream `seed`
 * (Philox4x64-10, key (seed, 0), counter (event * n_final + particle, 0, 0, 0)).  Beams are
 * particles 0 and 1 along +z and -z.  n_evt == 0 is a no-op.  ME_EINVAL for a NULL or host
 * pointer, n_evt < 0, evt0 < 0, or sqrt_s not above the sum of final-state masses. */
int rambo_momenta(const me_handle *h, uint64_t seed, double sqrt_s, int64_t evt0, int64_t n_evt,
                  double *out, void *stream);

/* The matrix element of every event: the per-event, leading-order calculation the paper moves to
 * the GPU with one lane of data parallelism per event (Sec. 1 and 2), here summed over helicities
 * and colours and averaged over the initial states.
 * out_me2[e] = averaged |M|^2 of event e for momenta = DEVICE double[n_evt][n_par][4]
 * (16-byte aligned).  n_evt == 0 is a no-op.  ME_EINVAL for NULL or host pointers,
 * misalignment or n_evt < 0.  Unphysical momenta are not checked (they give NaN/inf).
 * Work is split into chunks that bound the handle's per-stream scratch; calls on
 * different streams may overlap.  For processes with segment kernels (gg_ttggg) and
 * batches of more than one chunk, the chunks alternate between two internal streams, each
 * with its own scratch (twice the per-stream scratch), of the caller's stream (default priority; one pair per device and caller stream, shared
 * by all handles, created on first use and kept until the process ends); they start
 * after the work queued on `stream` before the call, and `stream` waits for both, so work
 * queued on `stream` after the call sees the finished output. */
int me_sigma(me_handle *h, const double *momenta, int64_t n_evt, double *out_me2, void *stream);

/* me_sigma for callers that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same arguments, same results: every event's
 * out_me2 is bitwise that of me_sigma on the same handle.  It calls no hipMalloc, hipFree or other
 * allocating routine.  Its scratch is a static device array of ME_NOALLOC_SCRATCH_BYTES (256 MiB)
 * that belongs to the library: one per GPU, held from the library's first use on that GPU until
 * the process ends.  Its address is resolved when a handle is created on the GPU (or at the
 * first call there).  The batch runs on `stream` alone, with no internal streams, in chunks of at
 * most the handle's chunk_events (me_info) that fit the array; no kernel reads a part of the
 * array that the same call has not written, so nothing needs clearing between calls.
 * Every call on one GPU shares that GPU's array, whichever handle or stream it uses, and the
 * array keeps the last call's contents: calls that overlap in time on one GPU (other host
 * threads, or other streams whose work has not completed) race and give wrong results.
 * Errors as me_sigma; ME_ENOMEM if one 64-event chunk of the handle's process and precision needs
 * more scratch than the array holds (none of the processes in the list above does), ME_EHIP if
 * the array's device address cannot be resolved. */
#define ME_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int me_sigma_noalloc(me_handle *h, const double *momenta, int64_t n_evt, double *out_me2, void *stream);

/* Scratch of a handle (a reading: the paper has no memory interface; a server that admits
 * requests by device-memory footprint needs to know and bound what the library holds).  The
 * scratch of calls on a stream is kept per (handle, stream), and per internal stream where a call
 * uses them, and grows when a call needs more; it lives until me_release_scratch or me_destroy.
 * The streams a handle was used on need not outlive it: me_destroy waits for the device.
 * me_reserve_scratch: allocates now what every me_sigma / me_sigma_alphas call of at most n_evt
 * events on `stream` needs, so that such calls allocate nothing more.  Synchronises `stream`
 * only if an existing smaller buffer must be replaced.  ME_ENOMEM if the allocation fails.
 * me_release_scratch: waits for `stream` (and its internal streams) and frees what the handle
 * holds for calls on it.
 * me_scratch_bytes: the bytes of scratch the handle holds now over all streams (< 0 on error). */
int me_reserve_scratch(me_handle *h, int64_t n_evt, void *stream);
int me_release_scratch(me_handle *h, void *stream);
int64_t me_scratch_bytes(const me_handle *h);

/* As me_sigma, and also out_hel[e * n_good + k] = colour-summed |M_h|^2 (not averaged) of
 * the k-th good helicity of event e (DEVICE double[n_evt][n_good], may be NULL). */
int me_sigma_hel(me_handle *h, const double *momenta, int64_t n_evt, double *out_me2, double *out_hel,
                 void *stream);

/* As me_sigma, and also one helicity configuration and one colour flow per event, drawn
 * from the event's own weights, as an unweighted event file records them (the two per-event
 * choices the paper names as still missing from its event files, Sec. 4).
 * rnd_hel, rnd_col: DEVICE double[n_evt], caller's uniforms in [0, 1).
 * out_hel[e]: helicity-combination index (the numbering of me_helicity_ratios) drawn among
 *             the good helicities with probability |M_h|^2 / sum_h |M_h|^2 (colour-summed);
 * out_col[e]: colour-flow index k (the order of me_colour_flows) drawn with probability
 *             w_k / sum_k w_k, w_k = sum_h |J_k,h|^2 the leading-colour weight of flow k.
 * A draw takes the smallest index j with r * sum_i w_i < sum_{i<=j} w_i (FP64, index order).
 * DEVICE int32 outputs of n_evt entries.  ME_EINVAL for NULL or host pointers. */
int me_sigma_select(me_handle *h, const double *momenta, int64_t n_evt, const double *rnd_hel,
                    const double *rnd_col, double *out_me2, int *out_hel, int *out_col, void *stream);

/* As me_sigma with a strong coupling per event (the "running" alpha_s of the paper, Sec. 2):
 * alpha_s_evt = DEVICE double[n_evt], alpha_s at each event's renormalisation scale, chosen and
 * evaluated by the caller.  Exact for these tree-level QCD processes: |M|^2 is homogeneous of
 * degree n_par - 2 in alpha_s, so the library evaluates the amplitudes at the handle's alpha_s
 * and multiplies by (alpha_s_evt[e] / alpha_s)^(n_par - 2).  No effect for ee_mumu and ee_mumu_z.
 * ME_EINVAL for NULL or host pointers. */
int me_sigma_alphas(me_handle *h, const double *momenta, int64_t n_evt, const double *alpha_s_evt,
                    double *out_me2, void *stream);

/* As me_sigma, multiplied by the single-diagram-enhancement weight of each event's channel
 * (MadEvent's multichannel algorithm, which the paper, Sec. 2, lists among the features of
 * its ME engine): channel = DEVICE int32[n_evt], a Feynman-diagram index in [0, n_diagrams)
 * (me_diagrams gives each diagram's internal lines), or -1 for no weight.
 *   out_me2[e] = |M|^2 * W_c / sum_d W_d,  W_d = sum over good helicities and over the diagram's
 *   four-gluon colour structures of the colour-summed square of that single diagram.
 * The weights of all channels of an event sum to 1.  An id >= n_diagrams gives 0.
 * ME_EINVAL for NULL or host pointers, or gg_gg (no channel weights). */
int me_sigma_channel(me_handle *h, const double *momenta, int64_t n_evt, const int *channel,
                     double *out_me2, void *stream);

/* The Feynman diagrams: out[d * lines_per_diagram + j] = j-th internal line of diagram d as a
 * mask of external particles (bit i = particle i, the side without particle 0), ascending,
 * 0-padded (me_info: lines_per_diagram).  out must hold n_diagrams * lines_per_diagram ints.
 * Returns n_diagrams, or ME_EINVAL for gg_gg. */
int me_diagrams(const me_handle *h, int *out);

/* colour flows: out[k * n_order + j] = the j-th gluon (0 = first gluon of the process) in
 * the ordering of flow k, n_order = gluons on the quark line (gg_gg: the three gluons after
 * gluon 3, which closes the trace; ee_mumu: 0).  out must hold n_colors * n_order ints.
 * Returns n_colors. */
int me_colour_flows(const me_handle *h, int *out);

typedef struct {
    int n_par, n_diagrams, n_amplitudes, n_colors, n_hel, n_good_hel, precision;
    double avg_factor, sym_factor;
    double flops_amp_lane;     /* algorithmic flops of the amplitude kernel per (event, helicity) */
    double flops_amp_exec_lane;/* flops it executes (above when segment kernels recompute currents) */
    int n_partial_slots;       /* partial jamp slots per (event, helicity) (0: jamps written directly) */
    double flops_colour_lane;  /* algorithmic flops of the colour sum per (event, helicity) */
    int64_t bytes_resident;    /* device bytes held by the handle (tables) */
    int64_t bytes_per_event_scratch; /* jamp scratch per event (per stream in use) */
    int64_t chunk_events;      /* events per amplitude/colour-sum launch pair */
    int n_order;               /* entries per colour flow in me_colour_flows */
    int helicity_groups;       /* colour-sum launches split the good helicities into this many groups */
    int lines_per_diagram;     /* entries per diagram in me_diagrams */
    int fused_colour;          /* 1: me_sigma / me_sigma_alphas contract the colour matrix inside the
                                  amplitude kernel (every process but gg_ttggg) */
} me_info_t;

/* Reading (the paper defines no such call): sizes, counts and factors of a handle, for callers
 * that size buffers, and for measurement (flop counts per lane). */
int me_info(const me_handle *h, me_info_t *out);

/* good helicities: out[k * n_par + i] = helicity (+1/-1) of particle i in the k-th good
 * combination; out must hold n_good_hel * n_par bytes.  Returns n_good_hel. */
int me_good_helicities(const me_handle *h, signed char *out);

/* the pre-pass statistic: out[hh] = max over its events of |M_hh|^2 / |M|^2, for all
 * n_hel helicity combinations (index: particle i's bit (l+1)/2 at 2^(n_par-1-i)). */
int me_helicity_ratios(const me_handle *h, double *out);

/* Launch timing, for measurement: with enable != 0, every later me_sigma call records a
 * HIP event pair around each kernel launch on its stream.  Each call returns (and clears)
 * what was recorded since the previous call: total milliseconds and launch counts of the
 * amplitude kernel and of the colour-sum kernel (it waits for those events).  With the
 * fused colour sum (me_info_t.fused_colour) the amplitude figures include the colour
 * contraction and the colour-sum figures are those of the helicity-sum kernel.  On the
 * two-stream path of me_sigma (gg_ttggg) the launches of the two internal streams overlap,
 * so the totals can exceed the wall time.  Any pointer may be NULL.  Not for use while
 * another thread calls me_sigma on the same handle. */
int me_profile(me_handle *h, int enable, double *ms_amp, double *ms_colour, int64_t *n_amp,
               int64_t *n_colour);

/* Options of a handle, set between calls (not while work of the handle is being enqueued).
 * ME_OPT_FUSED_COLOUR (default 1): for the plain |M|^2 (me_sigma, me_sigma_alphas) of a
 * process whose amplitude kernel ends holding all jamps of its lanes (every process but
 * gg_ttggg, whose jamps come out of a window of partial sums), in every precision, the
 * kernel contracts them with the colour matrix itself (the same matrix-core tiles, or scalar
 * forms, operand splits, sums and order as the separate colour-sum kernel of that precision,
 * so each helicity's |M_h|^2 is bitwise the same) and writes one FP64 value per (event,
 * helicity) instead of the jamps; a second kernel sums the helicities in the separate
 * kernel's groups and order (the e+e- processes sum them in the same kernel).  0: always the separate colour-sum kernel.  Both settings, and the calls that
 * need the jamps (me_sigma_hel, me_sigma_select), give bitwise the same |M|^2.
 * ME_EINVAL for an unknown option or a value other than 0 or 1. */
enum { ME_OPT_FUSED_COLOUR = 1 };
int me_set_option(me_handle *h, int option, int value);

/* Reading (the paper defines no error interface): the message of the calling thread's last
 * failed call; thread-local, valid until the thread's next call. */
const char *me_last_error(void);

/* Frees the handle and its device memory (the colour tables, helicity list and per-stream
 * scratch), after waiting for the device; NULL-safe.  Its place in the call sequence is the
 * target's; that it waits for the device, not only for the streams the handle used, is a
 * reading: those streams may be gone. */
void me_destroy(me_handle *h);

#ifdef __cplusplus
}
#endif
#endif
