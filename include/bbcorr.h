/*
 * bbcorr.h -- C ABI of the MI355X (gfx950) effective-block baryon-baryon correlator.
 *
 * The library computes the four-point correlators of Sec. 2, Eq. (2) of
 * H. Nemura, "Instructive discussion of an effective block algorithm for
 * baryon-baryon correlators" (arXiv:1510.00903):
 *
 *   C_ch(r, t)_{a b a' b'} = exp(E_ch (t - t0)) *
 *        sum_X < B1_a(X + r, t) B2_b(X, t)  Bbar4_b'  Bbar3_a' >
 *
 * for the 52 isospin-symmetric octet-octet channels of Sec. 4, Eqs.
 * (GeneralBB_NN)-(GeneralBB_XX), from light (u = d) and strange wall-source
 * propagators, with the effective block algorithm of Sec. 3: site-local block
 * construction, 3-D FFT of every block component, contraction of the open
 * source indices in momentum space (Eq. (LN.pLLp.FFT)) and inverse FFT.
 *
 * Conventions (all fixed by the paper unless marked "reading"):
 *  - Propagator of flavour f on one time slice: S_f(x)[i][j], i = 3*mu + c the
 *    sink spin-colour, j = 3*mu' + c' the source spin-colour (reading: the
 *    paper does not fix the flattening), complex interleaved (re, im).
 *    Sites are ordered x fastest, then y, then z (Sec. 6, index xi).
 *  - Baryon fields of Sec. 2 with C = gamma_4 gamma_2 in the Dirac
 *    representation; the source operator is the sink operator with primed
 *    indices and the quark fields in mirrored order (Sec. 3, Eq. (LN.pLLp.ududsu)).
 *  - Spatial boundary periodic; B1 sits at X + r (Sec. 3).
 *  - Spin components: BBC_SPIN_UPPER computes alpha, beta, alpha', beta' in
 *    {0, 1} (Dirac upper components, positive parity forward in time, Sec. 6),
 *    BBC_SPIN_LOWER the lower pair {2, 3} of every index (backward in time),
 *    BBC_SPIN_FULL all four components of every index (256 values, bbc_correlate
 *    only, layout below).
 *  - Output element (t-index n, channel-index m, site r, spin s) with
 *    s = a + 2*(b + 2*(a' + 2*b')) is at
 *        C_out[((n * n_ch + m) * V + r) * 16 + s]
 *    i.e. the paper's linear index xi of Sec. 6 with the channel and time
 *    running over the requested lists.
 *
 * Errors: every call returns a bbc_status; on failure a message is kept per
 * thread (bbc_last_error).  Arguments are validated before any device work.
 * On failure the contents of output buffers are unspecified.  No C++
 * exception crosses this interface.
 *
 * Ownership: the caller owns every input and output buffer; the library never
 * frees them.  A context owns its device workspace, which it allocates on the
 * first call that needs it and keeps within the budget given to bbc_create.
 */
#ifndef BBCORR_H
#define BBCORR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BBC_OK = 0,
    BBC_EINVAL = -1,       /* bad argument (null pointer, size, channel, lattice) */
    BBC_ENOMEM = -2,       /* workspace would exceed the budget, or allocation failed */
    BBC_EDEVICE = -3,      /* HIP runtime error */
    BBC_EUNSUPPORTED = -4, /* valid request the library does not handle (e.g. lattice extent) */
    BBC_ETIMEOUT = -5,     /* bbc_wait: job not finished within the timeout */
    BBC_ECANCELLED = -6,   /* bbc_wait: job was cancelled */
    BBC_ESTATE = -7        /* call not valid in the current state (server not started, job running) */
} bbc_status;

typedef enum { BBC_F64 = 0, BBC_F32 = 1 } bbc_precision;
typedef enum { BBC_SPIN_UPPER = 0, BBC_SPIN_LOWER = 1, BBC_SPIN_FULL = 2 } bbc_spin;

typedef struct bbc_context bbc_context;

/* Number of channels: the 52 channels of Sec. 4 in printed order (indices 0..51),
   followed by the four off-diagonal channels the paper omits because they vanish
   in the isospin limit (indices 52..55; computed for verification only). */
int bbc_num_channels(void);          /* 52 */
int bbc_num_channels_all(void);      /* 56 */

/* Other charge states (Sec. 4 notes that the extension is direct): any
   quadruple of the octet fields B1 B2 > B3 B4 whose sink and source hold the
   same numbers of u, d and s quarks is a channel too.  Baryon indices 0..7 name
   the fields p, n, S+, S-, X0, X-, L, S0 (bbc_baryon_name); bbc_channel_id
   returns the index of a quadruple in the list above when it is listed, else
   56 + ((b1 * 8 + b2) * 8 + b3) * 8 + b4, or BBC_EINVAL if an index is out of
   range or the quark content differs.  Every call taking a channel index
   accepts these ids.

   General fields (Sec. 2, Eq. (FieldOperator_B): B = eps((q1 Gamma_1 q2) Gamma_2 q3)):
   baryon indices 8..39 name
     8, 9    p2, n2: the nucleon with {Gamma_1, Gamma_2} = {C, gamma_5}, flavour
             terms as p and n;
     10..39  decuplet fields with {C gamma_l, 1} (Sec. 4 footnote), l = 1, 2, 3:
             index 10 + 3 f + l - 1 for f = 0 D++ (uuu), 1 D- (ddd), 2 O- (sss),
             3 D+, 4 D0, 5 S*+, 6 S*0, 7 S*-, 8 X*0, 9 X*-; names "D++(1)" etc.
             The members of mixed flavour are the symmetric flavour
             combinations (a reading), e.g. D+ = (2 eps (u G d) u + eps (u G u) d) / sqrt3,
             S*0 = sqrt(2/3) (eps (u G d) s + eps (d G s) u + eps (s G u) d).
   A quadruple holding at least one of them has the id
     4152 + ((b1 * 40 + b2) * 40 + b3) * 40 + b4     (4152 = 56 + 8^4),
   valid when the quark content matches.  Sink and source fields may differ in
   their spin structures (e.g. p2 n > p n2).  Reading: the source tensor is the
   sink tensor with primed indices for every field (as for the octet). */
int bbc_num_baryons(void);           /* 40 */
const char *bbc_baryon_name(int b);  /* NULL for an invalid index */
int bbc_channel_id(int b1, int b2, int b3, int b4);

/* Channel name "B1 B2 > B3 B4" with baryon names p n L S+ S0 S- X0 X-
   (L = Lambda, S = Sigma, X = Xi).  Returns NULL for an invalid index. */
const char *bbc_channel_name(int channel);

/* Number of light and strange quark propagators in every term of a channel
   (n_light + n_strange = 6).  Sec. 2 field content. */
bbc_status bbc_channel_content(int channel, int *n_light, int *n_strange);

/* Source terms of a channel: the number of terms of source baryons B3 and B4
   (3 for Lambda = X_u, X_d, X_s; 2 for Sigma0 = X_u, X_d; 1 otherwise), Sec. 2. */
bbc_status bbc_source_terms(int channel, int *n_terms3, int *n_terms4);

/* Diagram classification of Sec. 3 and Tables 1-4 for one channel and one
   combination of source terms (term3 of B3, term4 of B4): the number of
   diagrams and, for each, the number of iterations of its open-index sum (K)
   and the parity of its permutation (+1 / -1).  K and sign must hold room for
   max_diagrams entries. */
bbc_status bbc_diagram_table(int channel, int term3, int term4, int max_diagrams,
                             int *n_diagrams, int32_t *K, int32_t *sign);

/* Plan statistics for a channel set: number of distinct block intermediates,
   complex components per site (both sink spins), contraction terms, and the
   total open-index iterations (sum of K over diagrams and source terms). */
bbc_status bbc_plan_stats(int n_ch, const int32_t *ch_list, int64_t *n_intermediates,
                          int64_t *n_components, int64_t *n_terms, int64_t *n_iterations);

/* Pair form of the contraction for a channel set (Sec. 3 Eq. (LN.pLLp.FFT)):
   each channel is a weighted sum of products of two intermediate views with the
   open source indices summed.  Outputs: the number of distinct pair products,
   of contraction tasks (one wave each: a row view and its partners), the sum
   over pairs of the open-index extent K, and the number of (channel, pair)
   weights.  Host only; any output may be NULL. */
bbc_status bbc_pair_stats(int n_ch, const int32_t *ch_list, int64_t *n_pairs, int64_t *n_tasks,
                          int64_t *pair_items, int64_t *n_weights);

/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the
   workspace (0: no bound beyond free memory). */
bbc_status bbc_create(int device, uint64_t hbm_budget_bytes, bbc_context **out);
void bbc_destroy(bbc_context *ctx);

/* Thread-local message of the last failure in this thread ("" if none). */
const char *bbc_last_error(void);

/* Device workspace needed by bbc_correlate for the given request, in bytes. */
bbc_status bbc_footprint(const int32_t lattice[3], bbc_precision prec, int n_ch,
                         const int32_t *ch_list, uint64_t *bytes);

/*
 * Correlators for n_t time slices and n_ch channels (Sec. 2 Eq. (2), Sec. 3).
 *
 *   lattice[3]    Lx, Ly, Lz; each in {1,2,3,4,6,8,12,16,24,32,48,64,96}.
 *   prec          BBC_F64: propagators and output are complex double.
 *                 BBC_F32: complex float (blocks, FFT and contraction in FP32).
 *   S_light, S_strange  device pointers, [n_t][Lz][Ly][Lx][12][12] complex of
 *                 the precision's type: the slices for the times in t_list.
 *   t_list[n_t]   time of each slice (used for exp(E (t - t0)) only).
 *   t0            source time.
 *   ch_list[n_ch] channel ids (0..55, extended ids and general-field ids as
 *                 above), any order, repeats allowed.
 *   spin          BBC_SPIN_UPPER or BBC_SPIN_LOWER (components 2,3 mapped to 0,1),
 *                 or BBC_SPIN_FULL: every component of alpha, beta, alpha', beta'
 *                 over 0..3, 256 values per site, at
 *                     C_out[((n * n_ch + m) * V + r) * 256 + s],
 *                     s = alpha + 4 * (beta + 4 * (alpha' + 4 * beta')),
 *                 computed as 16 upper-pair evaluations, one per choice of upper
 *                 or lower pair for each of the four baryons (a baryon's lower
 *                 pair is the upper pair of its field with the rows of Gamma_2
 *                 moved up by two).  C_out (device memory only in this mode) then
 *                 holds n_t * n_ch * V * 256 values; C_scale is as below (the same
 *                 for every component).  The serving calls, the CPT average and
 *                 bbc_correlate_noalloc take UPPER or LOWER only.
 *   energy[n_ch]  E_ch of the normalisation factor exp(E_ch (t - t0)) of Sec. 2
 *                 Eq. (2); NULL means 0 for every channel (unnormalised).
 *   C_out         device pointer, n_t * n_ch * V * 16 complex of the
 *                 precision's type, layout given above.
 *   C_scale       BBC_F32 only (NULL for BBC_F64): device pointer to n_t * n_ch
 *                 doubles.  The correlator is C_scale[n * n_ch + m] times the
 *                 FP32 field of (n, m); the FP64 factor carries the power-of-two
 *                 rescaling of the propagators and exp(E (t - t0)), so that
 *                 six-propagator products do not leave the FP32 range.
 *   stream        hipStream_t (as void*) on which all work is ordered; NULL = default.
 * n_t = 0 is a valid empty request: the arguments are checked, nothing is
 * enqueued, and the slice-sized buffers (S_*, t_list, C_out, C_scale) may be NULL.
 * Stream-ordered: returns after enqueueing; synchronise the stream before reading C_out.
 * Calls on one context share its workspace: each bbc_correlate or
 * bbc_correlate_cpt call's stream first waits for the work of the previous such
 * call on the context (an event), so calls on different streams run one after
 * the other on the device and never overwrite each other's intermediates.
 */
bbc_status bbc_correlate(bbc_context *ctx, const int32_t lattice[3], bbc_precision prec,
                         const void *S_light, const void *S_strange,
                         int n_t, const int32_t *t_list, int t0,
                         int n_ch, const int32_t *ch_list, bbc_spin spin,
                         const double *energy, void *C_out, double *C_scale, void *stream);

/*
 * bbc_correlate without any device allocation, for callers that cannot call
 * hipMalloc: code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation.  Same arguments, results and layouts as
 * bbc_correlate (the same kernels run, so the results are bit-identical), with
 * S_light, S_strange, C_out and C_scale in device memory only (BBC_EINVAL
 * otherwise).  The plan tables, the momentum-group table, the energies and the
 * slice workspace live in a fixed scratch array of 192 MiB (201326592 bytes)
 * that the library holds on every GPU it runs on until the process ends; a
 * request that needs more (bbc_footprint plus a few hundred KB of tables)
 * fails with BBC_ENOMEM before anything is enqueued.  192 MiB holds, e.g.,
 * 8^3 with channel 1 (p Lambda) in FP64, 6^3 with all 52 channels in FP64, or
 * 8^3 with all 52 channels in FP32.  Host-side planning may allocate host
 * memory; the tables are copied to the scratch with hipMemcpyAsync on `stream`.
 * Every call on one GPU -- from any context or stream -- shares that GPU's
 * scratch, which keeps the last call's contents: calls that overlap on one
 * GPU race, so the caller must order them (e.g. one stream).  Profiling and
 * graph mode do not apply (ordinary stream-ordered launches).
 */
bbc_status bbc_correlate_noalloc(bbc_context *ctx, const int32_t lattice[3], bbc_precision prec,
                                 const void *S_light, const void *S_strange,
                                 int n_t, const int32_t *t_list, int t0,
                                 int n_ch, const int32_t *ch_list, bbc_spin spin,
                                 const double *energy, void *C_out, double *C_scale, void *stream);

/*
 * Kernel variants (tile and launch shapes) of one request shape: the lattice,
 * the precision, the spin selection and the channel list (in its order).  The
 * steps of Sec. 3 and Sec. 5 (blocks, forward FFT, open-index contraction) each
 * have variants that form the same values in the same order, so every choice
 * gives bit-identical results and only the speed differs:
 *   pairs   open-index contraction on the matrix cores: FP64 0 = a whole
 *           momentum group per wave, 1 = the same with the loads of the next
 *           open-index step issued ahead, 2 = half a group per wave, 3 = half a
 *           group, loads ahead, 4 = operands staged through LDS (whole group
 *           lines), 5 = staged, double-buffered, 6 = staged per set of 4
 *           momenta (half lines), 7 = the same, double-buffered, 8 = row
 *           tiles staged per set of 4 momenta (up to three row views share
 *           their column views' loads); FP32 0 = plain,
 *           1 = loads ahead, 2 = staged through LDS, 3 = staged, double-buffered,
 *           4 = staged, 4 open indices per round, 5 = row tiles (three rows);
 *   blocks  block construction, sites per workgroup x component shares:
 *           0 = 4 x 2, 1 = 4 x 4, 2 = 8 x 2;
 *   planes  x-y plane pass of the forward FFT (square 24- and 32-point planes):
 *           0 = as many planes per workgroup as 80 KB of LDS hold, 1 = half;
 *   slices  time slices of one device-resident request run at once, 2^slices
 *           (0..3): slice i runs on library stream i mod 2^slices with its own
 *           workspace, the streams forked from and joined back into the
 *           caller's stream (in graph mode: parallel branches of one graph);
 *           the workspace grows accordingly, and fewer run at once where the
 *           context budget would be exceeded.  Profiled calls run one at a time;
 *   combine channel sums from the pair products: 0 = batches of 8 entries whose
 *           loads are issued together, 1 = batches of 16, 2 = the pair products
 *           staged through LDS a chunk at a time (each read once per momentum
 *           group).
 * A context keeps one choice per request shape; shapes without one take the
 * library's built-in choice.  Graphs captured in graph mode keep the variants
 * of their capture (same results).
 */
typedef struct {
    int32_t pairs;
    int32_t blocks;
    int32_t planes;
    int32_t slices;
    int32_t combine;
} bbc_tuning;

/* The variants a request shape runs with; *tuned (may be NULL) = 1 if the
   context holds a choice for it (set, tuned or loaded), 0 if built-in. */
bbc_status bbc_tuning_get(bbc_context *ctx, const int32_t lattice[3], bbc_precision prec, int n_ch,
                          const int32_t *ch_list, bbc_spin spin, bbc_tuning *out, int *tuned);

/* Sets the variants of a request shape (t = NULL: back to the built-in choice).
   BBC_EINVAL for a variant out of range. */
bbc_status bbc_tuning_set(bbc_context *ctx, const int32_t lattice[3], bbc_precision prec, int n_ch,
                          const int32_t *ch_list, bbc_spin spin, const bbc_tuning *t);

/*
 * Autotuner: times whole time slices (blocks through finalisation) of the
 * request shape on one device-resident slice S_light, S_strange
 * ([Lz][Ly][Lx][12][12] of the precision's type) and keeps the fastest
 * variants: a coordinate search from the current choice over the contraction
 * kernel, the plane pass (lattices that take one), the block kernel, the
 * channel sums and the number of concurrent slices (those whose workspaces fit in 16 GB and the
 * context budget), each candidate timed over `reps` rounds (1..1000) of up to
 * 8 slices after one untimed round, with HIP events on `stream`.  The choice is stored in the context
 * (and written to the tuning file, see below); out and ms_per_slice (the best
 * time per slice, milliseconds) may be NULL.  Allocates a scratch output
 * buffer and grows the context workspace as bbc_correlate does; synchronises
 * `stream` before returning.
 */
bbc_status bbc_autotune(bbc_context *ctx, const int32_t lattice[3], bbc_precision prec,
                        const void *S_light, const void *S_strange, int n_ch, const int32_t *ch_list,
                        bbc_spin spin, int reps, void *stream, bbc_tuning *out, double *ms_per_slice);

/*
 * Tuning file (JSON): {"bbc_tuning": 1, "entries": [{"lattice": [Lx, Ly, Lz],
 * "precision": 0|1, "spin_offset": 0|2, "channel_hash": "<FNV-1a of the
 * channel list, 16 hex digits>", "pairs": p, "blocks": b, "planes": l,
 * "slices": s, "combine": c}, ...]}.
 * bbc_tuning_save writes every choice the context holds (replacing the file
 * atomically); bbc_tuning_load merges a file's entries into the context
 * (BBC_EINVAL on a malformed file or a value out of range).  If the environment
 * variable BBC_TUNING_CACHE names a file, bbc_create loads it when it exists
 * and bbc_autotune rewrites it after each tuning.
 */
bbc_status bbc_tuning_save(bbc_context *ctx, const char *path);
bbc_status bbc_tuning_load(bbc_context *ctx, const char *path);

/*
 * Forward/backward (CPT) average of Sec. 6.  The baryon pair propagating
 * forward in time (upper spinor components) and the antibaryon pair
 * propagating backward (lower components) are related by charge conjugation,
 * parity and time reversal; the paper averages the two to double its samples.
 * For each tau in tau_list:
 *
 *   R(r, tau) = 1/2 exp(E tau) [ C_upper(r; slice (t0 + tau) mod Lt)
 *                                + sign * C_lower(r; slice (t0 - tau) mod Lt) ]
 *
 * with the lower component 2 + s re-indexed to s (no spin flip), as the paper
 * describes.  Readings: the slice map mod Lt, the common factor exp(E tau), and
 * sign (+1 or -1; +1 when each baryon's backward part carries the same factor,
 * which enters the pair squared).
 *
 *   lattice[3], prec, ch_list, energy   as for bbc_correlate.
 *   Lt            number of time slices held in S_light / S_strange (>= 1).
 *   S_light, S_strange  device pointers, [Lt][Lz][Ly][Lx][12][12]: every slice.
 *   t0            source slice, 0 <= t0 < Lt.
 *   tau_list[n_tau]  distances from t0, 0 <= tau < Lt (tau >= Lt/2 is accepted
 *                 and simply reads the slices the map gives).
 *   R_out         device pointer, n_tau * n_ch * V * 16 complex, the
 *                 bbc_correlate layout with tau in place of t.
 *   R_scale       BBC_F32 only: device pointer to n_tau * n_ch doubles; R is
 *                 R_scale times the FP32 field (the larger of the two parts'
 *                 factors; the parts are combined in FP64 and rounded once).
 * Device memory only (BBC_EINVAL otherwise).  Uses the context workspace of one
 * slice plus one output slice; stream-ordered like bbc_correlate; graph mode
 * does not apply (the calls run as ordinary launches).
 */
bbc_status bbc_correlate_cpt(bbc_context *ctx, const int32_t lattice[3], int Lt, bbc_precision prec,
                             const void *S_light, const void *S_strange, int t0, int n_tau,
                             const int32_t *tau_list, int n_ch, const int32_t *ch_list, int sign,
                             const double *energy, void *R_out, double *R_scale, void *stream);

/*
 * Serving: continuous batching of correlator jobs on one device.
 *
 * A job is (resident propagator set, list of its time slices, channel list).
 * bbc_server_start starts n_slots slots, each with its own HIP stream and
 * workspace.  Queued jobs are admitted in arrival order as soon as a slot is
 * free and the job's workspace fits the context's HBM budget (together with
 * the resident propagators and the other slots' workspaces).  When the job at
 * the head of the queue does not fit, one of the next 8 queued jobs that fits
 * may start instead, at most 16 times per head job (so the head job is delayed,
 * never starved); slot workspaces are kept and reused between jobs, and the
 * workspaces of idle slots are released when the head job needs the room.  A
 * job whose workspace cannot fit beside its own propagator set is refused by
 * bbc_submit (BBC_ENOMEM); one that cannot fit beside the other resident
 * propagator sets while no job runs fails with BBC_ENOMEM.  An admitted job
 * advances one time slice at a time, so jobs that arrive while others run are
 * started between slices and their work overlaps on the device.  A job's
 * result does not depend on what runs beside it (same kernels, own workspace,
 * fixed reduction order).  Output buffers are caller-owned device memory
 * (layout as for bbc_correlate) and must stay valid until the job finishes.
 *
 * bbc_prop_upload copies n_t slices of both flavours (host or device memory,
 * [n_t][Lz][Ly][Lx][12][12] complex of the precision's type) into memory owned
 * by the context and returns a handle; bbc_prop_release frees it once no queued
 * or running job uses it.  bbc_submit queues a job over slices slice_idx[] of a
 * propagator set (t_list gives their times for exp(E (t - t0))).  Job states:
 * 0 queued, 1 running, 2 done, 3 cancelled, 4 failed.  bbc_wait blocks until the
 * job ends (timeout_ms < 0: no limit) and returns BBC_OK, BBC_ECANCELLED, the
 * job's error, or BBC_ETIMEOUT.  bbc_cancel removes a queued job or stops a
 * running one after its slices in flight (its output is then incomplete).
 * bbc_job_times reports submit-to-start, start-to-end and total wall time in ms.
 * bbc_job_forget drops a finished job's record.  bbc_server_stop cancels queued
 * jobs, waits for running ones, and frees the slots.
 */
bbc_status bbc_server_start(bbc_context *ctx, int n_slots);
bbc_status bbc_server_stop(bbc_context *ctx);
bbc_status bbc_prop_upload(bbc_context *ctx, const int32_t lattice[3], bbc_precision prec, const void *S_light,
                           const void *S_strange, int n_t, uint64_t *handle);
bbc_status bbc_prop_release(bbc_context *ctx, uint64_t handle);
bbc_status bbc_submit(bbc_context *ctx, uint64_t prop, int n_t, const int32_t *slice_idx, const int32_t *t_list,
                      int t0, int n_ch, const int32_t *ch_list, bbc_spin spin, const double *energy, void *C_out,
                      double *C_scale, uint64_t *job);
bbc_status bbc_poll(bbc_context *ctx, uint64_t job, int *state);
bbc_status bbc_wait(bbc_context *ctx, uint64_t job, int timeout_ms);
bbc_status bbc_cancel(bbc_context *ctx, uint64_t job);
bbc_status bbc_job_times(bbc_context *ctx, uint64_t job, double *queue_ms, double *run_ms, double *total_ms);
bbc_status bbc_job_forget(bbc_context *ctx, uint64_t job);

/*
 * Measurement.  With profiling on, bbc_correlate records a HIP event pair on
 * its stream around every kernel stage of every time slice:
 *   0 block construction (step 1a)
 *   1 forward FFT (step 1b): one pass per axis, or on small cubic lattices one
 *     fused pass that also writes the momentum groups
 *   2 copy into the momentum groups (no kernel when stage 1 was fused)
 *   3 open-index contraction of every pair of intermediates (step 2a, matrix cores)
 *   4 inverse FFT (step 2b), one pass per axis
 *   5 normalisation / output layout
 *   6 channels as weighted sums of the pair products (step 2a)
 * bbc_profile_read waits for the recorded events, adds their elapsed times to
 * ms[stage] (milliseconds) and the number of kernels launched inside them to
 * launches[stage] (both arrays of n_stages <= BBC_NUM_STAGES entries,
 * overwritten), then clears the record.  Timing adds two events per stage and
 * slice; it does not change results.
 */
#define BBC_NUM_STAGES 7

/*
 * Graph mode.  With it on, a bbc_correlate call whose propagators, output and
 * scale are device memory is captured once (all its time slices, on an
 * internal stream) into a HIP graph, cached under the call's arguments
 * (buffers, lattice, channels, slices, t0, precision), and replayed on the
 * caller's stream; later calls with the same arguments replay it and read the
 * buffers' current contents.  Host-memory calls and profiled calls run as
 * ordinary stream-ordered launches.  At most 16 graphs are kept; turning the
 * mode off (or a workspace reallocation) waits for the device and frees them.
 * The captured sequence holds kernel launches only.
 *
 * The serving loop follows the same switch: with it on, each slot captures one
 * time slice per request shape (plan, lattice, precision, with or without
 * energies, the slot's workspace, kernel variants) and replays it for every
 * slice of every job of that shape on the slot, after a one-thread kernel has
 * written the slice's propagator, output and scale addresses and t - t0 to the
 * slot's argument record in device memory (the captured block, rescale and
 * output kernels read them there).  Per slice the host then issues two
 * launches instead of one per kernel.  A slot keeps at most 16 graphs; they
 * are freed when its workspace changes and when the server stops.  Results
 * are the same bits with the mode on or off.
 */
bbc_status bbc_graph_mode(bbc_context *ctx, int enable);
bbc_status bbc_profile_enable(bbc_context *ctx, int enable);
bbc_status bbc_profile_read(bbc_context *ctx, int n_stages, double *ms, int64_t *launches);

/*
 * Post-processing of C(r, t) (Sec. 2).  All buffers are device memory on the
 * context's GPU, complex interleaved (re, im); calls are stream-ordered on
 * `stream` and do not allocate.  `in` and `out` must not overlap.
 *
 * bbc_spin_project: projection of the 16 spin values of each site (the
 *   bbc_correlate layout, spin index s = a + 2 (b + 2 (a' + 2 b')) for sink spins
 *   a, b and source spins a', b' of the selected upper or lower components,
 *   component 0 = spin up, 1 = down in the Dirac representation) onto n_out
 *   combinations: out[f][site][m] = sum_s W[m][s] in[f][site][s] for n_fields
 *   fields of V sites.  W: host array of n_out x 16 complex doubles; with
 *   W[m][s] = P^(J,M)(a,b)* P^(J,M)(a',b') (Clebsch-Gordan coefficients) it forms
 *   the source operator J^(J,M) of Sec. 2 and the same projection at the sink.
 *   1 <= n_out <= 16; the FP32 form's per-(t, channel) scale factors pass through
 *   unchanged (the projection is linear).
 */
bbc_status bbc_spin_project(bbc_context *ctx, const int32_t lattice[3], bbc_precision prec, int n_fields,
                            const void *in, int n_out, const double *W, void *out, void *stream);

/*
 * bbc_cubic_project: projection of the relative coordinate onto the A1+
 *   representation of the cubic group, P f(r) = (1/24) sum_{R in O} f(R r) over the
 *   24 proper rotations, r taken mod L (Sec. 2, separation of 3S1 from 3D1); with
 *   mode BBC_CUBIC_A1_COMPLEMENT the output is Q f = f - P f.  Layout
 *   [n_fields][z][y][x][n_comp]; the lattice must be cubic (else BBC_EUNSUPPORTED).
 */
#define BBC_CUBIC_A1 0
#define BBC_CUBIC_A1_COMPLEMENT 1
bbc_status bbc_cubic_project(bbc_context *ctx, const int32_t lattice[3], bbc_precision prec, int n_fields, int n_comp,
                             const void *in, int mode, void *out, void *stream);

/*
 * bbc_central_potential: leading-order central potential of the HAL QCD method
 *   (Sec. 2), V(r, t) = (lap R(r, t) / (2 mu) - dR/dt) / R(r, t), with the six-point
 *   periodic lattice Laplacian and the symmetric difference (R(t+1) - R(t-1)) / 2,
 *   for the n_t - 2 inner slices of each of n_fields independent sequences of n_t
 *   consecutive slices, R[f][t][z][y][x] (complex FP64; e.g. a spin-projected C
 *   per channel with the e^{(m1+m2)(t-t0)} normalisation).  inv_2mu = 1 / (2 mu),
 *   mu the reduced mass in lattice units.  V_out: [f][n_t - 2][z][y][x] complex
 *   FP64.  Sites where R = 0 give non-finite values.
 */
bbc_status bbc_central_potential(bbc_context *ctx, const int32_t lattice[3], int n_fields, int n_t, const void *R,
                                 double inv_2mu, void *V_out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* BBCORR_H */
