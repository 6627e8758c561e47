/*
 * rbp.h -- C ABI of librbp: Monte-Carlo logical-error estimation with Relay-BP
 * decoding of detector error models, on AMD Instinct MI355X (gfx950).
 *
 * The operations follow the paper's decoding problem (Sec. 6.1 and Table
 * "decoding latency"): a detector error model is a binary matrix H with
 * N_det rows (detectors, here M) and N_loc columns (error mechanisms, here N),
 * per-mechanism probabilities p_j and an observable matrix O (k x N).  Shots
 * are sampled as independent Bernoulli faults; decoding maps a syndrome to a
 * correction with Relay-BP (flooding min-sum with memory-damped marginals,
 * sequential relay legs, the lowest-weight of stop_nconv solutions,
 * single-precision messages; parameters named as in Sec. 6.1).
 *
 * Conventions shared by every call
 *   - Bit vectors are packed LSB-first into uint32 words, row-major
 *     [shot][word]: bit b of vector v is bit (b % 32) of word b / 32.  Unused
 *     high bits of the last word are written as zero.
 *   - Pointers named *_dev are device memory owned by the caller; host
 *     pointers are read during the call only.  The library owns only the
 *     handle-internal buffers it creates.
 *   - `stream` is a hipStream_t (NULL = default stream).  Sampling and decoding
 *     are asynchronous on that stream; create/destroy/info are synchronous.
 *   - A handle may be used by one host thread at a time.  Calls that overlap
 *     on different streams with one handle are not supported.
 *   - Outputs are a pure function of the inputs, the seeds and the
 *     parameters: they do not depend on the stream, the launch configuration
 *     or the order in which the device processes shots.
 *   - Errors are returned as negative status codes; rbp_last_error() gives
 *     the message of the last failing call on the calling thread.
 */
#ifndef RBP_H_
#define RBP_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rbp_status;
#define RBP_OK 0
#define RBP_ERR_INVALID_ARG (-1) /* NULL pointer, bad enum or parameter range */
#define RBP_ERR_SHAPE (-2)       /* inconsistent sizes, unsorted or duplicate CSC entries */
#define RBP_ERR_UNSUPPORTED (-3) /* row degree outside [2, 1024] (0 allowed), p outside (0, 0.5] */
#define RBP_ERR_OOM (-4)         /* device or host allocation failed */
#define RBP_ERR_HIP (-5)         /* HIP runtime error (message in rbp_last_error) */
#define RBP_ERR_ABORTED (-6)     /* a latency-mode launch stopped on an expired barrier wait */

typedef struct rbp_code* rbp_code_t;

/* Detector error model handle.
 * H: M x N in CSC form, host arrays col_ptr[N+1], row_idx[nnz] (rows strictly
 * ascending within each column, 0 <= row < M).  O: k x N in CSC form
 * (obs_col_ptr[N+1], obs_row_idx), k may be 0 (then both may be NULL).
 * Every row of H must have degree 0 or 2..1024 (the sum-product decoder,
 * rbp_decode_spa, takes rows of at most 32).  The handle keeps device copies
 * of H in CSR and CSC order and of O. */
rbp_status rbp_code_create(int32_t M, int32_t N, const int32_t* col_ptr, const int32_t* row_idx, int32_t k,
                           const int32_t* obs_col_ptr, const int32_t* obs_row_idx, rbp_code_t* out);
rbp_status rbp_code_destroy(rbp_code_t code);
/* Sizes of a handle; any output pointer may be NULL. */
rbp_status rbp_code_info(rbp_code_t code, int32_t* M, int32_t* N, int32_t* nnz, int32_t* k, int32_t* max_row_deg,
                         int32_t* max_col_deg);

/* sample(H, priors, shots, seed)  -- Bernoulli faults and their syndromes.
 * priors: host double[N], each in (0, 0.5]; mechanism j faults independently
 * with probability p_j (to 2^-32).  The mechanisms are cut into 64 segments of
 * L = ceil(N/64).  In segment g, with pmax = max_j p_j, candidate positions
 * follow geometric gaps: the gap G before the next candidate is the number of
 * k in 1..len(g) with T_k > w, w the next 32-bit word and
 * T_k = min(floor(exp(k log1p(-pmax)) 2^32), 2^32 - 1) (double precision); a
 * candidate j with p_j < pmax is kept iff the next word is below
 * A_j = min(floor(p_j / pmax 2^32), 2^32 - 2), one with p_j = pmax always.
 * Word d of segment g of shot s is word (d mod 4) of Philox4x32-10 with key
 * (seed lo, seed hi) and counter (g 2^24 + d / 4, shot lo, shot hi, 3),
 * shot = shot_offset + s, so any shot range is reproducible on its own.
 * Outputs (device): syndromes_dev uint32[shots][ceil(M/32)] = H e,
 * obs_dev uint32[shots][ceil(k/32)] = O e (may be NULL when k = 0),
 * errors_dev uint32[shots][ceil(N/32)] = e (may be NULL). */
rbp_status rbp_sample(rbp_code_t code, const double* priors, uint64_t shots, uint64_t seed, uint64_t shot_offset,
                      uint32_t* syndromes_dev, uint32_t* obs_dev, uint32_t* errors_dev, void* stream);

/* Relay-BP settings; names follow Sec. 6.1 of the paper.  Marginals saturate
 * at +-2^90 (the paper leaves FP32 overflow open; without a bound, shots that
 * never converge reach inf and NaN); the bounds below keep every message finite
 * under that saturation. */
typedef struct {
    float gamma0;               /* memory strength of leg 0 (paper: 0.125), |gamma0| <= 16 */
    float gamma_min, gamma_max; /* gamma_dist of the relay legs, e.g. [-0.24, 0.66], |gamma| <= 16 */
    int32_t pre_iter;           /* iteration budget of leg 0 (80), 1..65536 */
    int32_t max_iterations;     /* iteration budget of each relay leg (60), 1..65536 */
    int32_t num_sets;           /* number of relay legs after leg 0 (paper 1000), >= 0 */
    int32_t stop_nconv;         /* solutions to collect before stopping (5), 1..255 */
    int32_t stopping_criterion; /* 0: stop after stop_nconv solutions; 1: run every leg */
    uint64_t gamma_seed;        /* relay-leg memory strengths: gamma_j^(r) = fmaf(u, gamma_max - gamma_min,
                                   gamma_min), u = (Philox4x32-10(gamma_seed; j/4, r, 0, 1)_{j mod 4} >> 8)
                                   * 2^-24, shared by every shot */
} rbp_relay_params;

/* Per-shot decode statistics (32 bytes). */
typedef struct {
    uint8_t converged; /* 1 if some leg converged (or the syndrome was zero) */
    uint8_t nconv;     /* solutions found */
    uint8_t path;      /* 0 plain Relay-BP, 1 learned proposal accepted, 2 proposal failed -> plain,
                          3 zero syndrome */
    uint8_t reserved;
    uint16_t legs;     /* legs run (both phases) */
    uint16_t reserved2;
    uint32_t iters;    /* BP iterations run (both phases) */
    uint32_t reserved3;
    uint64_t t_start, t_end; /* device wall clock (100 MHz ticks) when the shot was taken and finished */
} rbp_shot_stats;

/* decode(H, priors, syndromes, relay params) -> corrections and logical flips.
 * priors: host double[N] in (0, 0.5]; the decoder uses Lambda_j =
 * (float) ln((1-p_j)/p_j).  syndromes_dev: uint32[shots][ceil(M/32)].
 * prior_delta_dev: optional float[shots][N]; when given, each shot first runs
 * one proposal leg (leg 0 with priors Lambda + delta, gamma0, pre_iter); if it
 * converges its solution is returned (path 1), else plain Relay-BP runs from
 * scratch (path 2).  Solution weights always use Lambda.
 * Outputs (device): corrections_dev uint32[shots][ceil(N/32)] (the lowest
 * weight solution, or the last hard decision when no leg converged),
 * obs_pred_dev uint32[shots][ceil(k/32)] = O * correction (may be NULL when
 * k = 0), stats_dev rbp_shot_stats[shots] (may be NULL).  Without a prior
 * delta, batches of 8192 shots or more are decoded heaviest syndrome first (a
 * counting sort on the device, into a per-handle buffer of 4 bytes per shot),
 * so that the longest decodes do not finish last; no output depends on it. */
rbp_status rbp_decode(rbp_code_t code, const double* priors, const uint32_t* syndromes_dev, uint64_t shots,
                      const rbp_relay_params* params, const float* prior_delta_dev, uint32_t* corrections_dev,
                      uint32_t* obs_pred_dev, rbp_shot_stats* stats_dev, void* stream);

/* The learned-proposal decode with BF16 adjustments, the network's own output
 * type (rbp_mlp_forward_bf16): identical to rbp_decode with prior_delta_dev
 * holding the same values widened to float (every BF16 value is exact in
 * FP32), but delta_bf16_dev uint16[shots][N] (BF16 bit patterns, required)
 * moves half the bytes, and the compact state copies a shot's adjustments to
 * LDS once instead of reading them on every iteration of the proposal leg.
 * Outputs as rbp_decode. */
rbp_status rbp_decode_proposal(rbp_code_t code, const double* priors, const uint32_t* syndromes_dev, uint64_t shots,
                               const rbp_relay_params* params, const uint16_t* delta_bf16_dev,
                               uint32_t* corrections_dev, uint32_t* obs_pred_dev, rbp_shot_stats* stats_dev,
                               void* stream);

/* The same decode with the BF16 adjustments laid out by decoder position
 * instead of by mechanism: delta_bf16_pos_dev uint16[shots][Np] (16-byte
 * aligned), entry p the adjustment of mechanism var_of_position[p]
 * (rbp_code_positions), entries of padding positions ignored (taken as 0).
 * Results are identical to rbp_decode_proposal with the same values by
 * mechanism; the decoder then copies each row with contiguous loads instead
 * of a gather (a network whose output layer is ordered by position writes
 * this layout directly: rbp_mlp_set_output_order). */
rbp_status rbp_decode_proposal_pos(rbp_code_t code, const double* priors, const uint32_t* syndromes_dev,
                                   uint64_t shots, const rbp_relay_params* params, const uint16_t* delta_bf16_pos_dev,
                                   uint32_t* corrections_dev, uint32_t* obs_pred_dev, rbp_shot_stats* stats_dev,
                                   void* stream);

/* The decoder's position order of a handle: *np = Np (N rounded up to whole
 * groups of 64; positions N..Np-1 are padding) and, if var_of_position is not
 * NULL (host, Np entries), the mechanism decoded at each position (-1 for
 * padding).  Positions 0..N-1 hold every mechanism once. */
rbp_status rbp_code_positions(rbp_code_t code, int32_t* np, int32_t* var_of_position);

/* rbp_decode for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same decode, arguments, outputs and results, but its scratch -- the shot
 * counter, the ordering histogram and the heaviest-first shot order -- lives
 * in a fixed 4 MiB device array per GPU, so the call allocates nothing.
 * Limits: at most 1,048,064 shots per call (UNSUPPORTED beyond); the handle's
 * per-shot state must fit in LDS (UNSUPPORTED for models decoded with the
 * state in device memory); the handle must already have decoded with the same
 * priors and relay parameters through rbp_decode, which builds its tables
 * (INVALID_ARG otherwise).  Every call on one GPU shares that array and
 * clears what must start at zero itself, with kernels (no memset); calls
 * that overlap on one GPU (several streams or threads) race and must not be
 * issued. */
rbp_status rbp_decode_noalloc(rbp_code_t code, const double* priors, const uint32_t* syndromes_dev, uint64_t shots,
                              const rbp_relay_params* params, const float* prior_delta_dev, uint32_t* corrections_dev,
                              uint32_t* obs_pred_dev, rbp_shot_stats* stats_dev, void* stream);

/* Batched decode of several detector error models in one persistent launch.
 * Shot s belongs to model shot_code_dev[s] (uint8, < n_codes) and is the
 * shot_index_dev[s]-th row of that model's syndrome / output arrays
 * (syndromes_dev[c], corrections_dev[c], obs_pred_dev[c]; device pointers held
 * in host arrays).  priors[c] are host arrays as in rbp_decode; stats_dev is
 * indexed by s.  Every model uses the same params. */
rbp_status rbp_decode_multi(int32_t n_codes, const rbp_code_t* codes, const double* const* priors,
                            const uint8_t* shot_code_dev, const uint32_t* shot_index_dev, uint64_t shots,
                            const uint32_t* const* syndromes_dev, const rbp_relay_params* params,
                            uint32_t* const* corrections_dev, uint32_t* const* obs_pred_dev,
                            rbp_shot_stats* stats_dev, void* stream);

/* Batched decode of several detector error models, each in a persistent
 * launch of its own with its own launch shape (the handle's rbp_launch_config:
 * waves per shot, state, slots), all issued at once on side streams forked
 * from `stream` and joined back into it (the largest model first), so that
 * each launch's tail is filled by the others' work (the batched uneven decode
 * of several codes; one launch over all models, rbp_decode_multi, must size
 * every slot for the largest model).  Model c decodes shots[c] rows (shots is
 * a host array; 0 skips the model) of its own arrays syndromes_dev[c],
 * corrections_dev[c], obs_pred_dev[c] and stats_dev[c] (may be NULL, or hold
 * NULL entries), exactly as rbp_decode would, with the same params.  Each
 * handle may appear once.  The side streams (8 per device, non-blocking,
 * default priority) are created on first use and kept until the process
 * ends.  Errors as rbp_decode: arguments, priors and tables are checked for
 * every model before anything is launched; a launch shape that cannot run
 * (UNSUPPORTED) stops the issue at that model, and the launches issued
 * before it still complete before later work on `stream`. */
rbp_status rbp_decode_each(int32_t n_codes, const rbp_code_t* codes, const double* const* priors,
                           const uint64_t* shots, const uint32_t* const* syndromes_dev,
                           const rbp_relay_params* params, uint32_t* const* corrections_dev,
                           uint32_t* const* obs_pred_dev, rbp_shot_stats* const* stats_dev, void* stream);

/* Block failures of a decoded batch (paper Sec. 6.1: a shot fails when any
 * logical observable is predicted wrong or the decoder did not converge):
 * *count_dev (uint64, device) += number of shots s with obs_pred_dev[s] !=
 * obs_dev[s] in any of obs_words words, or stats_dev[s].converged == 0.
 * Arrays as written by rbp_sample / rbp_decode. */
rbp_status rbp_count_failures(const uint32_t* obs_pred_dev, const uint32_t* obs_dev, const rbp_shot_stats* stats_dev,
                              uint64_t shots, int32_t obs_words, unsigned long long* count_dev, void* stream);

/* The LLRs Lambda_j = (float) ln((1-p_j)/p_j) the decoder uses for these
 * priors, written to llr_dev float[N] (device), e.g. as the prior term of the
 * proposal network's loss. */
rbp_status rbp_code_llr(rbp_code_t code, const double* priors, float* llr_dev, void* stream);

/* Launch shape of the persistent decoder for one handle (chosen by the
 * autotuner; 0 = library default).  waves_per_shot: wavefronts that share one
 * shot (1..16).  state: 0 auto, 1 per-shot state in LDS (one float per edge
 * and per variable), 2 the same state in device memory, 3 compact state in LDS
 * (one 16-byte record per check row -- its two least |nu|, the edge attaining
 * the least and the outgoing message signs -- and one float per variable;
 * rows of at most 16 edges; the messages are those of the per-edge form bit
 * for bit).  Auto takes 1 when it fits in LDS, else 3 when it fits, else 2.
 * max_slots: cap on the resident shot slots (0 = as many as fit; with several
 * shots per workgroup it caps the workgroups).  shots_per_wg: 0 or 1, one shot
 * per workgroup; 2 or 4, the workgroup decodes that many shots in lockstep,
 * one flooding iteration of each per round, sharing every group's table loads
 * (compact state only; applies to rbp_decode and rbp_decode_noalloc without a
 * prior delta, one model; identical results).  Out-of-range values return
 * RBP_ERR_INVALID_ARG; a decode whose K shots do not fit in LDS together
 * returns RBP_ERR_UNSUPPORTED. */
typedef struct {
    int32_t waves_per_shot;
    int32_t state;
    int32_t max_slots;
    int32_t shots_per_wg;
} rbp_launch_config;
rbp_status rbp_set_launch_config(rbp_code_t code, const rbp_launch_config* cfg);
/* Launch shape rbp_decode would use for this handle (after defaults). */
rbp_status rbp_get_launch_config(rbp_code_t code, rbp_launch_config* cfg, int32_t* slots, int32_t* lds_bytes);

/* Latency mode: decode shots one after another, each by several workgroups
 * together (the paper's sequential single-shot decoding, Sec. 6.1 Table
 * "decoding latency").  The row and variable groups of every sweep are spread
 * over all participating wavefronts; the sweeps are separated by grid
 * barriers.  Results are those of rbp_decode without a prior delta
 * (identical arithmetic); outputs and statistics as there, shot s at row s.
 * workgroups: participating workgroups (0: one per CU of one XCD, CUs / 8).
 * stride: participants are the workgroups whose index is a multiple of it
 * (0: 8 while workgroups * 8 <= CUs, which keeps them on one XCD, else 1).
 * waves: wavefronts per workgroup, 1..8 (0: 8).  spin_limit: bound on the polls of
 * one barrier wait (0: 2^21, about 2 s); when a wait expires the launch stops
 * at the next barrier, leaving later shots unwritten.
 * When all participants run on one XCD (checked at the start of each launch
 * from the hardware XCD id) the barriers only wait for stores and invalidate
 * the L1, since the participants share one L2; otherwise, or with
 * device_fences = 1, they use device-scope fences (L2 write-back and
 * invalidation).
 * The call returns when the launch has ended (it synchronizes the stream, as
 * a latency measurement needs): RBP_ERR_ABORTED if a barrier wait expired
 * (the outputs of the shots not reached are not written), else RBP_OK.
 * Uses per-handle scratch (one shot's state, bit arrays and barrier words).
 * Returns UNSUPPORTED when the workgroups cannot all be resident (cooperative
 * launch). */
typedef struct {
    int32_t workgroups;
    int32_t stride;
    int32_t waves;
    uint32_t spin_limit;
    int32_t device_fences;
} rbp_coop_params;
rbp_status rbp_decode_coop(rbp_code_t code, const double* priors, const uint32_t* syndromes_dev, uint64_t shots,
                           const rbp_relay_params* params, const rbp_coop_params* coop, uint32_t* corrections_dev,
                           uint32_t* obs_pred_dev, rbp_shot_stats* stats_dev, void* stream);
/* 1 in *aborted if the last rbp_decode_coop launch on this handle stopped on an
 * expired barrier wait, else 0 (the same fact rbp_decode_coop returns as
 * RBP_ERR_ABORTED).  Synchronizes the stream. */
rbp_status rbp_coop_aborted(rbp_code_t code, void* stream, int32_t* aborted);

/* Resident decoder: the sequential single-shot decoding of the latency tables
 * (Sec. 6.1, Table "decoding latency"; one shot at a time) without a kernel
 * launch per shot.  rbp_resident_start launches the latency-mode kernel (the
 * decoder of rbp_decode_coop, same arithmetic and results) once, on a
 * non-blocking stream of its own; the kernel stays on the GPU and takes shots
 * from a mailbox in pinned, coherent host memory.  rbp_resident_decode copies
 * one syndrome into the mailbox, raises its shot counter and spins on the host
 * until the kernel has written the correction, observable prediction and
 * statistics back: a shot's latency holds no launch, no stream
 * synchronization and no copy call, only the mailbox's PCIe round trips.
 *
 * coop: workgroups, stride, waves, spin_limit, device_fences as for
 *   rbp_decode_coop (0 = its defaults; workgroups = 1 decodes on one CU).
 * idle_seconds: the kernel ends itself when no shot comes for this long
 *   (0: 1 s), so a forgotten handle never holds the GPU; the next
 *   rbp_resident_decode launches it again (that shot's latency then includes
 *   the launch).  wait_seconds: bound on one rbp_resident_decode's wait
 *   (0: 60 s); on expiry the kernel is stopped and ABORTED returned.
 *
 * While a resident decoder runs: its kernel occupies `workgroups` CUs; calls
 * that synchronize the whole device (hipDeviceSynchronize, a hipFree that
 * waits for the device) wait until it ends (rbp_resident_stop, or
 * idle_seconds without a shot); decode calls on the same code handle that
 * would change its priors or relay parameters, and rbp_code_destroy, return
 * INVALID_ARG.  One host thread at a time per resident handle.
 * Errors: INVALID_ARG (NULL pointers, parameter ranges), UNSUPPORTED (the
 * workgroups cannot all be resident), OOM (pinned mailbox), ABORTED (a
 * barrier wait expired or wait_seconds passed; the kernel has ended, the next
 * decode relaunches it). */
typedef struct rbp_resident* rbp_resident_t;
typedef struct {
    rbp_coop_params coop;
    double idle_seconds;
    double wait_seconds;
} rbp_resident_params;
rbp_status rbp_resident_start(rbp_code_t code, const double* priors, const rbp_relay_params* params,
                              const rbp_resident_params* rp, rbp_resident_t* out);
/* One shot: syndrome (host, WM words) in; correction (host, WN words),
 * obs_pred (host, WK words; may be NULL when k = 0) and stats (host, may be
 * NULL) out, each laid out as one row of rbp_decode's outputs.  Blocks until
 * the shot is decoded. */
rbp_status rbp_resident_decode(rbp_resident_t r, const uint32_t* syndrome, uint32_t* correction, uint32_t* obs_pred,
                               rbp_shot_stats* stats);
/* Shots decoded so far, kernel launches so far (1 + relaunches after idle or
 * aborted ends), whether the kernel is running now, and the bit mask of the
 * XCDs its participating workgroups run on (0 until the current launch has
 * started); any pointer may be NULL. */
rbp_status rbp_resident_info(rbp_resident_t r, uint64_t* shots, int32_t* launches, int32_t* running,
                             uint32_t* xcds);
/* Ends the kernel (after the shot it is decoding, if any), waits for it and
 * frees the handle and its mailbox.  NULL is a no-op. */
rbp_status rbp_resident_stop(rbp_resident_t r);

/* Debug trace of one shot: the marginals M (float[N]) and check-to-variable
 * messages (float[nnz], CSC edge order of H) right after iteration t (>= 1) of
 * leg `leg` of phase `phase` (0 plain Relay-BP, 1 proposal leg).  syndrome_dev
 * holds one shot; prior_delta_dev is float[N] or NULL.  *reached (host) is 1 if
 * the decode got there, else 0.  Synchronizes the stream. */
rbp_status rbp_trace(rbp_code_t code, const double* priors, const uint32_t* syndrome_dev,
                     const rbp_relay_params* params, const float* prior_delta_dev, int32_t phase, int32_t leg,
                     int32_t t, float* M_out_dev, float* mu_out_dev, int32_t* reached, void* stream);

/* ---- learned proposal network ------------------------------------------- *
 * A multilayer perceptron x -> delta with x_i = syndrome bit i (0/1),
 * two hidden ReLU layers and a linear output of one log-prior adjustment per
 * mechanism: delta = W3 relu(W2 relu(W1 x + b1) + b2) + b3.  Weights are kept
 * as FP32 masters and used as BF16 copies with FP32 accumulation. */
typedef struct rbp_mlp* rbp_mlp_t;
/* in_dim = M, out_dim = N of the model it serves; hidden >= 1.  Weights are
 * initialised from `seed` (uniform in +-1/sqrt(fan_in)), biases zero. */
rbp_status rbp_mlp_create(int32_t in_dim, int32_t hidden, int32_t out_dim, uint64_t seed, rbp_mlp_t* out);
rbp_status rbp_mlp_destroy(rbp_mlp_t mlp);
/* delta_dev float[shots][out_dim] from syndromes_dev uint32[shots][ceil(in_dim/32)]. */
rbp_status rbp_mlp_forward(rbp_mlp_t mlp, const uint32_t* syndromes_dev, uint64_t shots, float* delta_dev,
                           void* stream);
/* The same forward pass with the output rounded to BF16 (round to nearest
 * even, from the FP32 value rbp_mlp_forward writes): delta_dev
 * uint16[shots][out_dim] of BF16 bit patterns, the input of
 * rbp_decode_proposal. */
rbp_status rbp_mlp_forward_bf16(rbp_mlp_t mlp, const uint32_t* syndromes_dev, uint64_t shots, uint16_t* delta_dev,
                                void* stream);
/* Column order of rbp_mlp_forward_bf16's output: with n > 0 it writes n
 * columns, column p the output order[p] (host array of n entries, each -1 for
 * a column of zeros, or an output index < out_dim), e.g. the decoder's
 * position order (rbp_code_positions) so that rbp_decode_proposal_pos can
 * take the network's rows directly.  The output layer's rows are gathered
 * into that order once here and again whenever the weights change.  n = 0
 * restores the natural order.  rbp_mlp_forward (FP32) and training are not
 * affected.  Synchronizes the device's default stream. */
rbp_status rbp_mlp_set_output_order(rbp_mlp_t mlp, const int32_t* order, int32_t n);
/* One Adam step on a batch: loss = mean over the batch of
 * sum_j BCEWithLogits(z_j, y_j), z_j = -(Lambda_j + delta_j), y = target bits
 * (uint32[batch][ceil(out_dim/32)]), Lambda = llr_dev float[out_dim].
 * loss_out_dev (float[1], may be NULL) receives the batch loss. */
rbp_status rbp_mlp_train_step(rbp_mlp_t mlp, const uint32_t* syndromes_dev, const uint32_t* targets_dev,
                              const float* llr_dev, uint64_t batch, float lr, float* loss_out_dev, void* stream);
/* Gradients of the same loss on a batch without updating the weights:
 * grads_dev float[num_params] in the parameter layout below, loss_out_dev
 * float[1] (may be NULL).  For checking the backward pass. */
rbp_status rbp_mlp_gradients(rbp_mlp_t mlp, const uint32_t* syndromes_dev, const uint32_t* targets_dev,
                             const float* llr_dev, uint64_t batch, float* grads_dev, float* loss_out_dev,
                             void* stream);
/* Copy parameters between the handle and a caller buffer (host float array
 * laid out W1[h][in], b1[h], W2[h][h], b2[h], W3[out][h], b3[out]).  Set
 * replaces the masters and resets the Adam state. */
rbp_status rbp_mlp_num_params(rbp_mlp_t mlp, int64_t* n);
rbp_status rbp_mlp_get_params(rbp_mlp_t mlp, float* host_out);
rbp_status rbp_mlp_set_params(rbp_mlp_t mlp, const float* host_in);
/* Checkpoint of the training state, for an exact resume: save writes to the
 * file at `path` the dimensions, the Adam step count, the FP32 master weights
 * and both Adam moment vectors (layout of rbp_mlp_get_params); load reads such
 * a file into a handle of the same dimensions (SHAPE otherwise; INVALID_ARG
 * for a file that is not a checkpoint) and refreshes the BF16 copies, so that
 * training continued after a load takes exactly the steps it would have
 * taken without the save.  File format (little-endian): "RBPMLP01", int32 in,
 * hidden, out, 0, int64 number of parameters, int64 step, then float32
 * masters, first moments, second moments.  Both synchronize the device. */
rbp_status rbp_mlp_save(rbp_mlp_t mlp, const char* path);
rbp_status rbp_mlp_load(rbp_mlp_t mlp, const char* path);

/* ---- sliding-window decoding --------------------------------------------- *
 * The paper's latency discussion (Sec. 6.1) argues for sliding-window decoding
 * with a commit region: a window decodes the syndrome of w consecutive rounds
 * and commits the mechanisms that start in its first c rounds; their effect is
 * removed from the running syndrome before the next window, c rounds later.
 * Windows are decoded with rbp_decode on handles of the window matrices; these
 * two calls move the bits in between. */

/* dst_dev[s] (dst_words words) = bits [bit_offset, bit_offset + nbits) of
 * src_dev[s] (src_words words), shifted to bit 0, LSB-first, zero above nbits.
 * Requires nbits <= 32 dst_words and bit_offset + nbits <= 32 src_words. */
rbp_status rbp_bits_extract(const uint32_t* src_dev, int32_t src_words, uint64_t shots, int64_t bit_offset,
                            int32_t nbits, uint32_t* dst_dev, int32_t dst_words, void* stream);

/* Commit a window's decoded mechanisms to the full model `code`.  For each shot
 * s and each set bit j < n_win of win_corr_dev[s] (win_words words) whose
 * cmap_dev[j] = J is a column of `code` (entries outside [0, N) mean "not
 * committed"): set bit J of corrections_dev[s] (uint32[shots][ceil(N/32)]),
 * XOR column J of H into syndromes_dev[s] (uint32[shots][ceil(M/32)]) and
 * column J of O into obs_pred_dev[s] (uint32[shots][ceil(k/32)]; may be NULL
 * when k = 0).  acc_stats_dev (may be NULL) accumulates the windows' decode
 * statistics: first != 0 copies win_stats_dev[s]; later windows AND
 * `converged`, take the minimum `nconv`, add `legs` and `iters` and set t_end. */
rbp_status rbp_window_commit(rbp_code_t code, uint64_t shots, const uint32_t* win_corr_dev, int32_t win_words,
                             const int32_t* cmap_dev, int32_t n_win, uint32_t* syndromes_dev, uint32_t* obs_pred_dev,
                             uint32_t* corrections_dev, const rbp_shot_stats* win_stats_dev,
                             rbp_shot_stats* acc_stats_dev, int32_t first, void* stream);

/* Bit gather (parallel-window decoding: windows whose rows are not one
 * contiguous range, and rows above a gap that fix single columns): bit t of
 * dst_dev[s] is bit rows_dev[t] of src_dev[s], t < nrows (device int32;
 * a row outside 0 .. 32 src_words - 1 reads as 0); higher bits are 0.
 * src_dev uint32[shots][src_words], dst_dev uint32[shots][dst_words], nrows <=
 * 32 dst_words (SHAPE otherwise). */
rbp_status rbp_bits_gather(const uint32_t* src_dev, int32_t src_words, uint64_t shots, const int32_t* rows_dev,
                           int32_t nrows, uint32_t* dst_dev, int32_t dst_words, void* stream);

/* Final check of windowed decoding: a shot whose running syndrome
 * syn_dev[s] (uint32[shots][words]) still has a set bit gets
 * acc_stats_dev[s].converged = 0. */
rbp_status rbp_window_residual(const uint32_t* syn_dev, int32_t words, uint64_t shots, rbp_shot_stats* acc_stats_dev,
                               void* stream);

/* ---- classical channel coding: sum-product BP over BPSK-AWGN ------------ *
 * The paper's classical benchmark of its ZSZ-2BGA codes (numerics appendix,
 * "classical channel coding", with eq. "bpsk awgn capacity"): the all-zero
 * codeword is sent as +1 symbols over an additive white Gaussian noise
 * channel, y_j = 1 + sigma z_j, and decoded by flooding sum-product BP with the
 * phi-domain ("boxplus-phi") check update and single-precision messages.  A
 * handle for this use is made by rbp_code_create from the parity-check matrix
 * with k = 0; rows of degree 2..32 (0 allowed; UNSUPPORTED otherwise). */

/* Channel LLRs of the all-zero codeword: llr_dev float[shots][N] =
 * 2 y / sigma^2 with y = 1 + sigma z (log P(bit 0 | y) / P(bit 1 | y)).
 * z_j comes from Philox4x32-10 (key = seed, counter = (j / 4, shot lo, shot hi,
 * 2)) by the Box-Muller transform: words 2h and 2h+1 give
 * u1 = ((w >> 8) + 1) 2^-24 in (0, 1] and u2 = (w >> 8) 2^-24, and
 * z_{4q+2h} = sqrt(-2 ln u1) cos(2 pi u2), z_{4q+2h+1} = sqrt(-2 ln u1) sin(2 pi u2),
 * evaluated in single precision.  Shot s uses counter index shot_offset + s,
 * so ranges of shots can be drawn independently.  sigma > 0. */
rbp_status rbp_sample_awgn(rbp_code_t code, uint64_t shots, double sigma, uint64_t seed, uint64_t shot_offset,
                           float* llr_dev, void* stream);

typedef struct {
    int32_t max_iterations; /* num_iter (paper: 100), >= 1 */
    float llr_max;          /* clipping of the channel LLRs and of the variable-to-check messages (paper: 20), > 0 */
    int32_t stop;           /* 1: stop after the first iteration whose hard decision satisfies every check;
                               0: always run max_iterations */
    int32_t waves_per_shot; /* wavefronts sharing one shot, 1..16; 0 = library default */
} rbp_spa_params;

/* Sum-product BP on channel LLRs llr_dev float[shots][N].  With L_j =
 * clip(llr_j, +-llr_max) and nu(0) = L_j on every edge, one iteration is
 *   mu_{i->j} = prod_{j' != j} s(nu_{j'->i}) * phi(sum_{j' != j} phi(|nu_{j'->i}|)),
 *   phi(x) = -ln tanh(x/2), the sum taken in ascending column order, s(x) = -1 iff x < 0;
 *   M_j = L_j + sum_i mu_{i->j} (ascending check order);
 *   nu_{j->i} = clip(M_j - mu_{i->j}, +-llr_max);  c_j = [M_j < 0].
 * Outputs (device, may be NULL except bits_dev): bits_dev uint32[shots][ceil(N/32)]
 * = c when decoding stops; marginals_dev float[shots][N] = M then; stats_dev
 * rbp_shot_stats[shots] with converged = (H c = 0), iters, path = 0 if c is the
 * zero word and 1 otherwise, t_start/t_end; counts_dev uint64[3] +=
 * {shots with c != 0 (block errors when the zero word was sent), shots with
 * c != 0 and H c = 0 (undetected errors), shots with H c != 0}. */
rbp_status rbp_decode_spa(rbp_code_t code, const float* llr_dev, uint64_t shots, const rbp_spa_params* params,
                          uint32_t* bits_dev, float* marginals_dev, rbp_shot_stats* stats_dev,
                          unsigned long long* counts_dev, void* stream);

/* ---- device ceilings ---------------------------------------------------- *
 * Aggregate LDS read bandwidth of the current device, measured: two
 * 1024-thread workgroups per compute unit read a 64 KB LDS buffer with
 * width_bytes (4, 8 or 16) per lane and instruction, every wave on 64
 * consecutive cells (no bank conflicts); *bytes_per_s (host) receives the best
 * of three timed launches.  The denominator of the decoder's LDS roofline.
 * Synchronous; allocates and frees a small device buffer. */
rbp_status rbp_measure_lds_bandwidth(int32_t width_bytes, double* bytes_per_s);

/* Message of the last failing call on this thread ("" if none). */
const char* rbp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RBP_H_ */
