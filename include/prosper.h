/*
 * prosper.h -- C ABI of the MI355X truncated-EM sparse-coding library.
 *
 * The library computes the truncated E-step (and the M-step it feeds) of the
 * probabilistic sparse-coding learners described in ProSper (Exarchakis et
 * al.), section "Learning Algorithm and Data Models":
 *
 *   prior          p(s | Theta)          (Eq. 1)
 *   noise model    p(y | s, Theta) = N(y; f(Theta, s), sigma^2 I)   (Eq. 2)
 *
 * with the model family of Table 1:
 *   PROSPER_BSC  s in {0,1}^H,    Bernoulli(pi),           f = W s
 *   PROSPER_TSC  s in {-1,0,1}^H, P(+-1) = pi/2 each,      f = W s
 *   PROSPER_MCA  s in {0,1}^H,    Bernoulli(pi),           f_d = max_h s_h W_dh
 *   PROSPER_MMCA s in {0,1}^H,    Bernoulli(pi),           f_d = the s_h W_dh of largest
 *                magnitude (lower h on a tie); statistics and M-step as MCA
 *   PROSPER_DSC  s_h in {phi_0 = 0, phi_1, ..., phi_{V-1}} (a given value set),
 *                categorical prior p(s_h = phi_v) = pv_v,   f = W s
 *                (discrete sparse coding; V = 2, phi = {0, 1} is BSC, and V = 3,
 *                phi = {0, 1, -1} with pv_1 = pv_2 is TSC)
 *
 * Truncated posteriors (same section): for each data point y_n the library
 * preselects H' latents I_n (the "Hprime" argument of the API section) and
 * renormalises the exact posterior on
 *   K_n = { s : s_h = 0 for h not in I_n, and #nonzero(s) <= gamma }
 * ("gamma" of the API section).  |K_n| = sum_{k<=gamma} C(H',k) (V-1)^k with
 * V = 2 (BSC, MCA, MMCA), 3 (TSC) or the DSC value count.
 *
 * Conventions (all entry points)
 *  - Every device pointer is owned by the caller; the library never frees one.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls are asynchronous on it; outputs are valid once it is synchronised.
 *  - Every call returns a prosper_status (0 = success).  No C++ exception
 *    crosses the ABI.  On failure nothing has been enqueued and the text of
 *    the error is available from prosper_last_error().
 *  - Matrices are row-major, float32 unless stated:
 *      Y  N x D   data, row n is y_n
 *      W  D x H   dictionary, column h is component W_h  (f = W s)
 *  - A context is not thread-safe; use one per host thread.  Its calls share
 *    one device workspace: calls on different streams of one context must not
 *    overlap on the device (order them, e.g. with an event, or use one context
 *    per stream).
 */
#ifndef PROSPER_H
#define PROSPER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PROSPER_OK = 0,
    PROSPER_EINVAL = -1,    /* an argument is outside its documented range      */
    PROSPER_ENOMEM = -2,    /* device memory for the context could not be had   */
    PROSPER_EDEVICE = -3,   /* a HIP runtime error (no GPU, launch failure, ...) */
    PROSPER_EBUSY = -4,     /* serving queue full; nothing was queued           */
    PROSPER_ENOTFOUND = -5, /* unknown serving request id                       */
    PROSPER_ETIMEDOUT = -6  /* serving wait ran out of time; request still live */
} prosper_status;

typedef enum {
    PROSPER_BSC = 0, PROSPER_TSC = 1, PROSPER_MCA = 2, PROSPER_MMCA = 3, PROSPER_DSC = 4
} prosper_model;

/* Precision of the N x D x H projection contraction (W^T y for all latents).
 *  PROSPER_FP32:   FP32 MFMA (v_mfma_f32_16x16x4_f32), FP32 accumulation.
 *  PROSPER_BF16:   BF16 MFMA with FP32 accumulation; each operand is split into
 *                  a BF16 head and a BF16 tail and three products are summed
 *                  (head*head + head*tail + tail*head).
 *  PROSPER_BF16X1: one BF16 product (the heads) with FP32 accumulation for the
 *                  ranking, then b of the H' selected candidates recomputed in
 *                  FP32 from y and W (the FP32 fix-up the state walk uses).  The
 *                  wider error band of the single product sends more points
 *                  through the exact re-scoring; the selection stays exact.
 *                  E-step only (EINVAL in prosper_serve).
 * Everything after the projection (state log-joints, normalisation, moments)
 * runs in FP32; M-step solve and the sigma/pi reductions run in FP64. */
typedef enum { PROSPER_FP32 = 0, PROSPER_BF16 = 1, PROSPER_BF16X1 = 2 } prosper_precision;

/* Flags for prosper_args.flags */
#define PROSPER_FLAG_NONE          0u
/* PROSPER_FLAG_FACTOR_B (BSC/TSC, accumulate = 1 only; EINVAL otherwise):
 * this call completes the accumulation of acc for the next M-step.  After
 * adding its own <s s^T> into acc->B, the library factors B (the Cholesky
 * factor prosper_mstep needs, see there) in the context's workspace on
 * `stream`, while the A statistics of the same call run on a second stream of
 * the context; the call completes on `stream` once both are done.  A following
 * prosper_mstep on the same context with the same acc->B pointer, D, H and
 * model reuses that factor and only solves.  Any later accumulating E-step,
 * or any prosper_mstep, on the context discards it; the caller must not
 * modify acc->B in between. */
#define PROSPER_FLAG_FACTOR_B      1u
/* PROSPER_FLAG_ZERO_ACC (accumulate = 1 only): the call overwrites acc (A, B,
 * scal and, for DSC, vcount) with this call's statistics instead of adding
 * into them; the clearing rides on the parameter-preparation kernels, so an
 * EM loop needs no separate fill of the accumulators. */
#define PROSPER_FLAG_ZERO_ACC      2u

/* Limits of this build */
#define PROSPER_MAX_HPRIME   32
#define PROSPER_MAX_D        1024
#define PROSPER_MAX_H        1024
#define PROSPER_MAX_TOPK     8
#define PROSPER_MAX_STATES   (1 << 20)
#define PROSPER_MAX_VALUES   8   /* DSC: V <= 8 */
#define PROSPER_DSC_MAX_GAMMA 10 /* DSC: gamma <= 10 (3-bit value codes of the actives) */

typedef struct {
    int32_t model;          /* prosper_model */
    int32_t precision;      /* prosper_precision */
    int64_t N;              /* data points, >= 0 (0 = no-op) */
    int32_t D, H;           /* observed / latent dimensions, 1..PROSPER_MAX_D / _H */
    int32_t Hprime;         /* 1 <= H' <= min(H, PROSPER_MAX_HPRIME) */
    int32_t gamma;          /* 0 <= gamma <= H'; |K| <= PROSPER_MAX_STATES */
    double  pi;             /* prior sparsity, 0 < pi < 1 (Eq. 1) */
    double  sigma;          /* noise standard deviation, > 0 and finite (Eq. 2) */
    const double* theta_dev;/* optional device pointer to {pi, sigma}; when set the
                               kernels read pi and sigma from it (no host sync in an
                               EM loop) and the host values above are ignored */
    int32_t topk;           /* 0..PROSPER_MAX_TOPK most probable states per point;
                               topk <= |K| */
    int32_t accumulate;     /* 1: add the M-step sufficient statistics into acc */
    uint32_t flags;         /* PROSPER_FLAG_NONE, or PROSPER_FLAG_FACTOR_B and/or
                               PROSPER_FLAG_ZERO_ACC */
    float   beta;           /* posterior temperature of deterministic annealing (the
                               schedule object of the paper's user-interface section):
                               q_n(s) proportional to p(y_n, s | Theta)^beta on K_n, in
                               (0, 1]; 0 stands for 1 (no annealing).  Moments, top-k
                               and statistics use the tempered q; logL stays
                               untempered.  beta != 1 runs the table-driven state walk. */
    /* DSC only (ignored by the other models): */
    int32_t nvalues;        /* V, 2..PROSPER_MAX_VALUES */
    float   phi[PROSPER_MAX_VALUES];  /* phi[0] = 0; phi[1..V-1] finite, non-zero, distinct */
    double  pv[PROSPER_MAX_VALUES];   /* prior pv[0..V-1], each > 0, summing to 1 (within
                               1e-9).  With theta_dev set they are read from the device
                               instead: theta_dev = {pi, sigma, pv_0, ..., pv_{V-1}}
                               (pi unused), the layout prosper_mstep writes for DSC. */
} prosper_args;

/* Per-point outputs of the E-step; any pointer may be NULL to skip it.
 * All device pointers. */
typedef struct {
    int32_t*  sel;      /* N x H'   preselected latent indices I_n, ascending */
    float*    s_mean;   /* N x H'   <s_h> under q_n, aligned with sel */
    float*    logL;     /* N        log sum_{s in K_n} p(y_n, s | Theta)
                                    (natural log, all constants included) */
    uint32_t* top_mask; /* N x topk slot masks of the most probable states
                           (bit j = slot j, i.e. latent sel[n][j], is non-zero);
                           TSC: N x topk x 2 = {active mask, minus-sign mask};
                           DSC: N x topk x 4 = {active mask, then three bit planes of
                           the value codes: bit j of plane p is bit p of the code
                           v (s = phi_v) of slot j} */
    float*    top_q;    /* N x topk their posterior probabilities q_n(s),
                           descending; equal q ordered by canonical state order */
    uint8_t*  flagged;  /* N        1 if the H'-th and (H'+1)-th selection scores
                                    are within 1e-6 relative (max(1,|r|)) */
    /* BSC/TSC only (EINVAL for the other models); either one present runs the
     * table-driven state walk.  They feed prosper_mstep_et. */
    float*    k_mean;   /* N        <number of non-zero latents> under q_n */
    float*    res;      /* N        <||y_n - W s||^2> under q_n, with the W of this call */
} prosper_point_out;

/* Sufficient statistics for the M-step, accumulated (added) by prosper_estep
 * when args.accumulate = 1.  The caller zeroes them before the first E-step
 * of an iteration.  Device pointers.
 *   BSC/TSC/DSC: A (D x H) += y_n <s>_n^T ;  B (H x H, upper triangle incl.
 *             diagonal in row-major h <= h') += <s s^T>_n
 *   MCA:      A (D x H) += R_n o y_n  (numerator);  B (D x H) += R_n
 *             (denominator), R_n[d,h] = posterior mass of the states whose max
 *             over active components at pixel d is attained first by h and is > 0
 *   scal (5 doubles): [0] sum_n <#nonzero(s)>  [1] sum_n logL_n
 *             [2] sum_n ||y_n||^2  [3] sum_n <||y_n - f(s)||^2> (MCA only)
 *             [4] N
 *   vcount (DSC only, V doubles): [v] += sum_n <number of latents at phi_v>
 *             for v = 1..V-1 ([0] is not touched) */
typedef struct {
    float*  A;
    float*  B;
    double* scal;
    double* vcount;
} prosper_acc;

typedef struct prosper_ctx prosper_ctx;

/* Create a context on HIP device `device`.  `workspace_bytes` is an initial
 * reservation (0 = grow on demand).  Returns EDEVICE when no GPU is usable. */
prosper_status prosper_ctx_create(int device, size_t workspace_bytes, prosper_ctx** out);
void           prosper_ctx_destroy(prosper_ctx* ctx);
/* Text of the last failure on this context (or of the last context-less call
 * on this thread when ctx is NULL).  Never NULL. */
const char*    prosper_last_error(const prosper_ctx* ctx);

/* Per-kernel timing ------------------------------------------------------
 * When enabled, every kernel group the context launches (parameter prep,
 * projection + preselection, state walk, A accumulation, M-step) is
 * bracketed by HIP events recorded on the stream it runs on.
 * prosper_profile(ctx, 1) enables and clears the counters, (ctx, 0) disables.
 * prosper_profile_read waits for the recorded events, and fills up to `cap`
 * entries: group name (static string), total elapsed ms and launch count.
 * Returns the number of groups (may exceed cap), or a negative status. */
prosper_status prosper_profile(prosper_ctx* ctx, int32_t enable);
/* Restrict the timing to the group named `group` (one of the names
 * prosper_profile_read returns); NULL or "" times every group again.  Fewer
 * events keep the timed work closer to the untimed one. */
prosper_status prosper_profile_only(prosper_ctx* ctx, const char* group);
int32_t        prosper_profile_read(prosper_ctx* ctx, int32_t cap, const char** names,
                                    double* total_ms, int64_t* launches);

/* Host-only helpers (no GPU needed) ------------------------------------ */

/* Validate an argument block exactly as prosper_estep does (shape, range,
 * enum and state-count checks; pointers are not inspected). */
prosper_status prosper_validate_args(const prosper_args* args);

/* |K| for (model, H', gamma); EINVAL for out-of-range input. */
prosper_status prosper_state_count(int32_t model, int32_t Hprime, int32_t gamma, int64_t* count);

/* The canonical state table: k ascending, slot tuples lexicographically,
 * TSC sign patterns of one support in binary counting order (bit i of the
 * counter is the sign of the i-th active slot, 0 -> +1).  Host buffers of
 * `capacity` entries; act[k] = active-slot mask, sgn[k] = minus-sign mask
 * (zero for BSC/MCA; sgn may be NULL). */
prosper_status prosper_state_table(int32_t model, int32_t Hprime, int32_t gamma,
                                   uint32_t* act, uint32_t* sgn, int64_t capacity);

/* DSC counterparts of the two calls above: |K| for V values, and the table
 * in the same order with codes[k] = the value codes (1..V-1) of the active
 * slots, 3 bits each, the lowest active slot in bits 0-2; the codes of one
 * support run in mixed-radix counting order (base V-1), the digit of the
 * lowest active slot least significant.  gamma <= PROSPER_DSC_MAX_GAMMA. */
prosper_status prosper_dsc_state_count(int32_t nvalues, int32_t Hprime, int32_t gamma,
                                       int64_t* count);
prosper_status prosper_dsc_state_table(int32_t nvalues, int32_t Hprime, int32_t gamma,
                                       uint32_t* act, uint32_t* codes, int64_t capacity);

/* E-step ---------------------------------------------------------------- */

/* Truncated E-step over N points.
 * Y: N x D FP32 (device), W: D x H FP32 (device).  For each point: ranking of
 * all H latents by the singleton log-joint (ties to the lower index), the H'
 * best as I_n, every state of K_n scored with its log-joint (Eq. 1 + Eq. 2),
 * log-sum-exp normalisation to q_n, and the moments / statistics requested in
 * `out` and `acc` (acc may be NULL when args.accumulate = 0).
 * NaN in Y is not checked and propagates into logL. */
prosper_status prosper_estep(prosper_ctx* ctx, const prosper_args* args,
                             const float* Y, const float* W,
                             const prosper_point_out* out, const prosper_acc* acc,
                             void* stream);

/* E-step without allocation ---------------------------------------------
 * For callers that cannot allocate device memory: code recorded into a HIP
 * graph, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, outputs and errors as prosper_estep (accumulation and topk
 * included), on the current HIP device, with no context: every intermediate
 * (state table, parameter preparation, per-point workspace, statistics
 * partials) lives in one file-scope device array of 64 MiB per GPU, held from
 * library load until the process ends.  The call allocates and frees
 * nothing; inputs and outputs are still the caller's.
 *  - Returns EINVAL when the call's intermediates do not fit in 64 MiB (at
 *    D = H = 256 and H' = 12 about 56 bytes per point plus 1 MB, and 13 MB
 *    more with statistics, when sel and s_mean are supplied: N up to about
 *    1.1 million, or 0.9 million with statistics), and for
 *    PROSPER_FLAG_FACTOR_B (it needs a context's second stream).
 *  - The array is shared by every call on that GPU and keeps the last call's
 *    contents; each call clears what it needs cleared with kernels (no
 *    memset).  Calls that overlap on one GPU (different streams or host
 *    threads) race on it and must be serialised by the caller.
 *  - Per-point outputs are bit-identical to prosper_estep's; the statistics
 *    are summed over fewer partials (at most 32), so A, B and scal agree with
 *    prosper_estep's up to FP32 summation order. */
prosper_status prosper_estep_static(const prosper_args* args, const float* Y, const float* W,
                                    const prosper_point_out* out, const prosper_acc* acc,
                                    void* stream);

/* M-step ----------------------------------------------------------------- */

/* The M-step of truncated EM (section "Learning Algorithm and Data Models":
 * the parameters that maximise the free energy under the truncated
 * posteriors of the E-step, for the data models of Table 1): new parameters
 * from one E-step's statistics, in FP64 on the device.
 *   BSC/TSC: W_new = A B^-1 on the latents with B_hh > 0 (Cholesky of that
 *            block; other columns keep W_old), pi = scal[0]/(N H),
 *            sigma^2 = (scal[2] - 2 tr(W_new^T A) + tr(W_new^T W_new B))/(N D)
 *   MCA:     W_new[d,h] = A[d,h]/B[d,h] where B[d,h] > 0 (else W_old),
 *            pi as above, sigma^2 = scal[3]/(N D)
 *   DSC:     W and sigma as BSC; pv_v = vcount[v]/(N H) for v >= 1,
 *            pv_0 = 1 - sum_{v>=1} pv_v (the expected share of latents at each
 *            value); needs acc->vcount and args->nvalues
 * W_old and W_new (D x H FP32) may alias.  theta_new (device) gets {pi, sigma}
 * (2 doubles), for DSC {pi, sigma, pv_0, ..., pv_{V-1}} (2 + V doubles); it
 * may equal args->theta_dev.  args supplies model, D, H (and nvalues).
 * Errors: EINVAL for a NULL pointer, an unknown model or D, H out of range;
 * EDEVICE for a HIP failure (message in prosper_last_error). */
prosper_status prosper_mstep(prosper_ctx* ctx, const prosper_args* args,
                             const prosper_acc* acc, const float* W_old, float* W_new,
                             double* theta_new, void* stream);

/* M-step variant with pi and sigma from the selected points ---------------
 * The deterministic-annealing section names M-step variants without a
 * formula; this is the reading taken (BSC/TSC).  W_new as prosper_mstep,
 * from all points.  The points kept are the N_cut = clamp(round(N A), 1, N)
 * with the largest logL_n (ties to the lower index), A = P(#non-zero <= gamma)
 * under the prior with the E-step's pi; with B = E[#non-zero; #non-zero <=
 * gamma] under the same prior:
 *   pi_new    = pi * mean_kept <k>_n * A / B      (pi when B = 0)
 *   sigma_new = sqrt(sum_kept res_n / (N_cut D))  (res of the E-step's W)
 * logL, k_mean, res: device, N each, as written by prosper_estep (N = args->N).
 * The E-step's pi is args->theta_dev[0] when set, else args->pi; args supplies
 * model, N, D, H, gamma.  theta_new (device, 2 doubles) may equal theta_dev.
 * Errors as prosper_mstep, plus EINVAL for another model or N < 1. */
prosper_status prosper_mstep_et(prosper_ctx* ctx, const prosper_args* args,
                                const prosper_acc* acc, const float* logL,
                                const float* k_mean, const float* res, const float* W_old,
                                float* W_new, double* theta_new, void* stream);

/* Serving: E-step-only posterior inference with continuous batching ------
 * The `inference` method of the user-interface section: for each data point
 * of a request, the most likely latent states of its truncated posterior and
 * their probabilities (top_mask / top_q), with the preselection, posterior
 * means and logL of prosper_point_out, for a dictionary the server keeps
 * resident. */

typedef struct prosper_server prosper_server;

/* Start a server.  It copies W (device or host pointer, D x H FP32) once and
 * keeps it, its derived tables and the state tables resident.  Queued
 * requests with the same (Hprime, gamma, topk) are batched into one launch;
 * batches are admitted while the device memory they need fits in
 * mem_budget_bytes and fewer than max_inflight are on the GPU, and run
 * concurrently on `n_streams` HIP streams (1..8).  queue_capacity bounds
 * pending requests.  The server holds mem_budget_bytes of device memory and
 * twice that of pinned host memory (output staging, and an ingress area into
 * which submit copies request inputs).  Models: BSC, TSC, MCA, MMCA (EINVAL
 * for DSC, whose prior has no place in this call). */
prosper_status prosper_serve(prosper_ctx* ctx, const float* W, int32_t W_on_device,
                             int32_t model, int32_t D, int32_t H, double pi,
                             double sigma, int32_t precision, size_t mem_budget_bytes,
                             int32_t max_inflight, int32_t n_streams,
                             int32_t queue_capacity, prosper_server** out);

/* Queue one request of `npatches` points (host buffer Y_host, npatches x D).
 * Y_host is copied into the ingress area during the call when it has room;
 * otherwise the server thread reads Y_host when it launches the request, so
 * the buffer must stay valid until prosper_serve_wait returns for this id.  The per-point
 * outputs in out_host are host buffers with the layouts of prosper_point_out
 * (NULL to skip) and are filled when the request completes.  Returns EBUSY
 * when the queue is full and EINVAL for a request larger than the budget. */
prosper_status prosper_serve_submit(prosper_server* srv, const float* Y_host, int64_t npatches,
                                    int32_t Hprime, int32_t gamma, int32_t topk,
                                    const prosper_point_out* out_host, uint64_t* req_id);

/* Wait for a request (timeout_us < 0: forever).  On success the outputs are
 * in place, *latency_ms (may be NULL) is submit-to-completion wall time and
 * the id is retired.  The request's own status is returned (a failed request
 * does not stop the server). */
prosper_status prosper_serve_wait(prosper_server* srv, uint64_t req_id, int64_t timeout_us,
                                  double* latency_ms);

/* prosper_serve_wait with the request's time split into stages (ms), for
 * latency analysis: stages_ms[0] queue wait (submit to the launch of its
 * batch), [1] the launch calls of the batch, [2] launch returned to the
 * batch's completion seen by the scheduler (stream queueing, transfers,
 * kernels, polling), [3] of that the GPU time of the batch (its events),
 * [4] delivery (outputs copied to the caller, waiter woken), [5] total. */
prosper_status prosper_serve_wait_stages(prosper_server* srv, uint64_t req_id,
                                         int64_t timeout_us, double* stages_ms);

/* Drain the queue, stop the scheduler thread and free the server. */
prosper_status prosper_serve_stop(prosper_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* PROSPER_H */
