/*
 * ptqmc.h -- C ABI of the MI355X (gfx950) parallel-tempering quantum Monte Carlo sampler.
 *
 * The library runs the data-parallel hot path of parallel tempering (PT) over
 * Suzuki-Trotter replicas of transverse-field Ising problems: Metropolis single-spin
 * sweeps of many independent Markov chains ("replicas"), each at its own rung of a
 * ladder, alternating with swaps between neighbouring rungs (paper, Section 2; the
 * quantum system is represented by M coupled copies of the classical one, Section 6).
 * Its loop is the paper's Figure 6 -- allocate, sweep k times, swap, measure, free --
 * with every step on the GPU and the state resident in device memory between calls.
 *
 * Model, for one instance with N spins, M Trotter slices and R replicas:
 *   E(s)  = sum_{edges (i,j)} J_ij s_i s_j + sum_i h_i s_i            (integer)
 *   E_cl  = sum_k E(s^k),   C = sum_k sum_i s_i^k s_i^{(k+1) mod M}   (C = 0 if M == 1)
 *   S_r   = b_r E_cl - K_r C   is the action of a replica at rung r; weight exp(-S_r).
 * For a temperature ladder at transverse field Gamma: b_r = beta_r / M and
 * K_r = -1/2 ln tanh(beta_r Gamma / M).  A rung is only the pair (b_r, K_r).
 *
 * Trajectory contract.  For a given (instances, seed) the sampler's trajectory is
 * unique: spins, swap decisions, integer energies, labels and accumulators do not
 * depend on launch shapes, tiles, encodings or the number of calls they are split over.
 *   sweep t      : for p in slice parities (2 if M >= 2, else 1), for g in colours,
 *                  attempt a flip at every (replica c, slice k = p mod 2, site i of colour
 *                  g).  Field f = h_i + sum_j J_ij s_j^k, t' = s_i^{k-1} + s_i^{k+1};
 *                  dE = -2 s f, dC = -2 s t', dS = b*dE - K*dC (FP64, no fused ops);
 *                  flip iff u <= thr(dS).  With k = 2m + p (M == 1: p = m = 0),
 *                  Mh = M/2 (1 if M == 1) and G = ceil(Mh/4), u = word (m mod 4) of
 *                  Philox4x32-10(ctr = ((2i + p)*G + m/4, t, c, n), key = (lo(seed), hi(seed))):
 *                  one call serves four same-parity slices of one site.
 *   thr(dS)      : 2^32-1 if dS <= 0, else clamp(floor(exp(-dS) * 2^32), 1, 2^32-1) - 1,
 *                  with exp evaluated by a fixed sequence of IEEE operations.
 *   exchange e   : pairs (r, r+1), r = e mod 2, e mod 2 + 2, ...; with x, y the replicas at
 *                  r, r+1: D = (b_r - b_{r+1})(E_x - E_y) - (K_r - K_{r+1})(C_x - C_y);
 *                  swap the rung labels iff u <= thr(-D), u = word 0 of
 *                  Philox(ctr = (r, e, 0, n), key = (lo(seed), hi(seed) ^ 0x53574150)).
 *                  Then: the replica at rung 0 labelled DOWN completes a round trip and
 *                  becomes UP (NONE becomes UP); the replica at rung R-1 labelled UP becomes
 *                  DOWN; per rung, E_cl, C and their squares are accumulated, and the
 *                  label of the replica there is counted (UP / DOWN).
 *   init         : s = +1 iff the top bit of word (m mod 4) of
 *                  Philox(ctr = ((2i + p)*G + m/4, 0, c, n), key = (lo, hi ^ 0x494E4954)).
 * Vertex labels and colours are used as given (any proper colouring).
 *
 * Conventions.  Every function returning int returns PT_OK (0) or a negative PT_E*
 * code; nothing aborts or throws across this boundary.  pt_last_error() returns a
 * thread-local message for the last failure on the calling thread.  A context is used
 * by one host thread at a time.  All calls that launch work are asynchronous on the
 * context's stream; pt_observables, pt_get_spins, pt_save and pt_sync synchronise it.
 * A slice-block launch with resident blocks bounds its waits for neighbouring blocks so
 * that every launch ends; if one gave up since the last of those four calls, the next of
 * them restores the state of the last clean synchronisation (a device copy the context
 * keeps when resident launches are possible), replays the calls since with slice blocks
 * launched per sweep (or per parity), and then runs them that way for the rest of the
 * context (pt_info.recoveries counts this).  PT_ESTATE is returned only if that replay
 * fails too.
 */
#ifndef PTQMC_H
#define PTQMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define PT_OK 0
#define PT_EINVAL (-1)  /* invalid argument or instance                                  */
#define PT_ENOMEM (-2)  /* device or host allocation failed, or workspace too small       */
#define PT_EHIP (-3)    /* a HIP runtime call failed (the message names the call and code) */
#define PT_ELAUNCH (-4) /* a kernel could not be launched in any fallback configuration    */
#define PT_ESTATE (-5)  /* call not valid in the context's state (e.g. bad checkpoint)     */

/* spin encodings (the trajectory is identical under every encoding) */
#define PT_INT8 0       /* one byte per spin                                                */
#define PT_BITPACK32 1  /* 32 replica slots per uint32 word: bit (c mod 32) of word group
                           c/32 holds slot c's spin at (k, i); device memory 8x smaller.
                           Instances with +-1 couplings, |h| <= 1, one degree D <= 8 and
                           M a power-of-two multiple of 8 are swept by octets (8 slots, one
                           byte of each word) staged in LDS with bit-sliced local fields;
                           others one colour class per launch in device memory.  The chain
                           is the same as under PT_INT8                                  */

/* Imaginary-time correlation lags: with PT_FLAG_TAU_CORR every exchange step adds, for
 * each rung r and l < PT_TAU_LAGS, Ct_l = sum_k sum_i s_i^k s_i^{(k + lag_l) mod M} of
 * the replica at rung r to sumCt[r][l], lag_l = max(1, floor((l + 1) M / 16)) slices.
 * Ct_l / (N M) estimates (1/N) sum_i <sigma^z_i(tau) sigma^z_i(0)> at imaginary time
 * tau = lag_l beta / M, whose decay gives the gap above the ground state (the quantity
 * the paper's application computes, Section 1). */
#define PT_TAU_LAGS 8

/* round-trip labels */
#define PT_LABEL_NONE 0
#define PT_LABEL_UP 1
#define PT_LABEL_DOWN 2

/* option flags */
#define PT_FLAG_TIMING 0x1u        /* bracket every sweep/exchange launch with HIP events   */
#define PT_FLAG_NO_GRAPH 0x2u      /* pt_run launches eagerly instead of replaying a graph  */
#define PT_FLAG_INJECT_LAUNCH_OOR_ONCE 0x4u /* test hook: the first sweep launch is treated
                                             as out of resources, exercising the fallback */
#define PT_FLAG_SLICE_BLOCKS 0x8u  /* split every replica that could use them into slice
                                      blocks, as replicas too large for one workgroup's
                                      LDS always are                                   */
#define PT_FLAG_FOUR_SLICE_LANES 0x10u /* fast path: one four-slice word per lane (the
                                          default only for batches too small to give every
                                          SIMD a wave per colour class; same chain; a
                                          measurement and test hook)                   */
#define PT_FLAG_TWO_WORD_LANES 0x200u /* fast path: two four-slice words per lane whatever
                                          the batch size (same chain; a measurement and
                                          test hook)                                   */
#define PT_FLAG_BLOCK_LAUNCH_PER_SWEEP 0x20u /* slice blocks: one launch per sweep (octet
                                          slice blocks: per parity of every sweep) even
                                          when all blocks could be resident at once (same
                                          chain; a measurement and test hook)          */
#define PT_FLAG_TAU_CORR 0x80u     /* accumulate imaginary-time spin correlations per rung
                                      at every exchange step (pt_obs.sumCt); PT_INT8 only */
#define PT_FLAG_WORK_QUEUE 0x100u /* PT_BITPACK32: each whole-octet workgroup takes its
                                          octet from device work queues (one per XCD,
                                          largest first) as it starts, instead of
                                          workgroup b sweeping list position b, which
                                          the hardware already hands out largest first
                                          (measured 4 % faster on config 3); the same
                                          chain (a measurement and test hook)          */
#define PT_FLAG_NO_LATENCY_PATH 0x400u /* fast path: sweep batches of at most one tile per
                                          compute unit like any other instead of forming
                                          each thread's next item during the current one
                                          (same chain; a measurement and test hook)    */
#define PT_FLAG_DEVICE_SCOPE_RECORDS 0x800u /* resident slice blocks (both encodings):
                                          pass boundary records with device-scope
                                          operations even when every ring of blocks
                                          runs on one XCD, instead of through its L2
                                          (same chain; a measurement and test hook)    */
#define PT_FLAG_TEST_XCD_MISMATCH 0x1000u /* test hook: resident slice blocks whose rings
                                          share an XCD report the launch's XCDs as
                                          mismatched, so the next synchronising call
                                          recovers (pt_info.recoveries)                */
#define PT_FLAG_TEST_BLOCK_WAIT_TIMEOUT 0x40u /* test hook: resident slice blocks wait for a
                                          progress count that never comes, under a tiny
                                          poll bound, so every wait gives up; the next
                                          synchronising call recovers (pt_info.recoveries)
                                          */

typedef struct pt_ctx pt_ctx;

/* One problem instance and its ladder.  The caller owns every pointer (host memory)
 * and may free it after pt_init returns: the library copies what it needs.
 *   N >= 1 spins; M == 1 (classical) or M even >= 2 slices; R >= 2 replicas.
 *   edges: n_edges pairs (edge_i[e], edge_j[e]) with 0 <= i < j < N, no duplicates;
 *   edge_J[e] the coupling; h[i] the field; color[i] < n_colors a proper colouring
 *   (no edge joins two sites of one colour).  max_i(|h_i| + sum_j |J_ij|) <= 1023.
 *   rung_b[r], rung_K[r] finite, K > 0 when M >= 2 (ignored when M == 1); rung 0 is
 *   the first (coldest) rung of the ladder.                                          */
typedef struct {
    int32_t N, M, R, n_edges, n_colors;
    const int32_t *edge_i, *edge_j;
    const int8_t *edge_J;
    const int8_t *h;
    const uint8_t *color;
    const double *rung_b, *rung_K;
} pt_instance;

/* Sampler options.  seed keys every draw; sweeps_per_exchange (k >= 1) is the number of
 * sweeps per pt_run cycle.  Launch shape: a workgroup sweeps a tile of replicas of one
 * instance held in LDS.  tile_replicas (replicas per tile) or tile_bytes (target spin
 * bytes per tile) and block_threads (a multiple of 64, at most 1024) fix the shape when
 * positive.  When all three are 0 the library tunes itself: its first sweep launches try
 * a few shapes, timed with HIP events, and keep the fastest (the trajectory does not
 * depend on the shape, so nothing is repeated or lost). */
typedef struct {
    uint64_t seed;
    int32_t sweeps_per_exchange;
    int32_t encoding;
    uint32_t flags;
    int32_t tile_replicas;
    int32_t tile_bytes;
    int32_t block_threads;
} pt_options;

/* Observables of one instance, written into caller-owned host arrays.  Any pointer may
 * be NULL to skip that array.  Sizes: [R] unless noted. */
typedef struct {
    int64_t *E_cl, *C;        /* by replica slot                                      */
    int32_t *rung_of;         /* slot -> rung                                         */
    int32_t *replica_of;      /* rung -> slot                                         */
    uint64_t *acc, *att;      /* [R-1] accepted / attempted swaps of pair (r, r+1)    */
    uint64_t *roundtrips;     /* by slot                                              */
    int8_t *label;            /* by slot                                              */
    int64_t *sumE, *sumC, *sumE2, *sumC2; /* by rung, accumulated at every exchange   */
    uint64_t *nup, *ndown;    /* by rung: exchange steps at which the replica there was
                                 labelled UP / DOWN (feedback-optimised ladders use
                                 f(r) = nup / (nup + ndown))                          */
    uint64_t t, e, n_acc;     /* sweeps done, exchange steps done, accumulated samples */
    int64_t *sumCt;           /* [R][PT_TAU_LAGS] by rung (zero without PT_FLAG_TAU_CORR) */
} pt_obs;

/* Launch and timing record of a context. */
typedef struct {
    int32_t n_instances, n_tiles, block_threads, lds_bytes;
    int32_t max_tile_replicas, fallbacks, encoding, device_cus;
    int32_t tile_bytes, tuned;        /* chosen target tile bytes; 1 once tuning ended */
    uint64_t flips_per_sweep;         /* sum over instances of R*N*M                 */
    double sweep_ms;                  /* summed event time of timed sweep launches   */
    int64_t sweep_launches;           /* number of timed sweep launches              */
    double exchange_ms;
    int64_t exchange_launches;
    int32_t sweep_groups;             /* launches of whole-replica tiles per sweep call:
                                         one per occupancy class of the tiles          */
    int32_t block_tiles;              /* slice-block tiles                             */
    int32_t block_resident;           /* 1: the last slice-block sweep call ran as one
                                         launch with every block resident (halos passed
                                         between blocks in device memory); 0: one launch
                                         per sweep                                      */
    int32_t class_launches;           /* PT_BITPACK32: sweep launches per sweep (one per
                                         colour class); 0 under PT_INT8                 */
    int64_t multi_launches;           /* pt_run launches that ran several PT cycles each
                                         (batches whose instances each fit one tile)    */
    int64_t multi_cycles;             /* PT cycles those launches ran                  */
    double multi_ms;                  /* their summed event time under PT_FLAG_TIMING
                                         (not part of sweep_ms / exchange_ms)           */
    int32_t oct_tiles;                /* PT_BITPACK32: whole octets (8 replica slots of one
                                         word group) swept resident in LDS, all sweeps of
                                         a call in one launch                           */
    int32_t oct_blocks;               /* PT_BITPACK32: octet slice blocks (octets too
                                         large for one workgroup's LDS, split in time)  */
    int32_t oct_tile_launches;        /* launches per call of the whole octets (0 or 1) */
    int32_t oct_resident;             /* 1: the octet slice blocks run all sweeps of a
                                         call in one launch, every block resident and
                                         boundary groups passed between neighbouring
                                         blocks in device memory; 0: one launch per
                                         parity of every sweep                          */
    int32_t oct_queue;                /* whole octets: 1 when each workgroup takes its
                                         octet from the device work queues
                                         (PT_FLAG_WORK_QUEUE), 0 when workgroup b sweeps
                                         list position b                                */
    int32_t oct_fused;                /* 1: a PT cycle of the batch is one launch, the
                                         exchange step run by the octet that completes
                                         each instance                                  */
    int32_t oct_ring_xcd;             /* 1: every ring of resident octet slice blocks
                                         runs on one XCD (workgroups b and b + 8 of a
                                         launch share one) and passes boundary records
                                         through its L2; a launch whose workgroups do
                                         not keep to that fails, and the call recovers
                                         as after a wait that gave up                   */
    int32_t block_ring_xcd;           /* 1: the same for PT_INT8 resident slice blocks,
                                         one ring of blocks per replica                 */
    int64_t recoveries;               /* synchronising calls that found a resident
                                         launch's wait given up, restored the state of
                                         the last clean synchronisation and replayed
                                         the calls since with slice blocks launched per
                                         sweep (resident launches stay off after one)   */
    int32_t lane_words;               /* PT_INT8 whole-replica tiles: four-slice words per
                                         lane (2, or 1 for batches too small to give
                                         every SIMD one wave per colour class; always 2
                                         when an instance has 16-bit entries)           */
    int32_t ent16_instances;          /* PT_INT8 instances whose neighbour entries are
                                         16 bits (regular, unit |J|, replicas of more
                                         than half a compute unit's LDS)                */
    uint32_t last_device_error;       /* the device error word the last failed
                                         synchronisation found (0: none): 1 a resident
                                         wait gave up, 2 an octet kernel found its LDS
                                         away from address 0, 4 a whole-octet workgroup
                                         found the work queues empty, 8 the workgroups
                                         of a resident launch left round-robin XCDs     */
    int32_t latency_path;             /* 1: whole-replica tiles sweep on the latency path
                                         (at most one tile per compute unit; tiles whose
                                         colour classes fit one pass of the workgroup
                                         form each thread's next item, site, entries and
                                         Philox words, while the current one is in
                                         flight)                                        */
} pt_info;

/* Device bytes pt_init needs for these instances and options (for a caller-provided
 * workspace).  Does not touch the GPU. */
int pt_workspace_bytes(const pt_instance *inst, int32_t n_inst, const pt_options *opt,
                       size_t *bytes);

/* Validate the instances, build neighbour lists, colour blocks and threshold tables,
 * place the state in device memory and draw the initial spins (then energies from
 * scratch).  stream: a hipStream_t to run on, or NULL for a library-owned stream.
 * workspace: device memory of at least pt_workspace_bytes() bytes that the caller keeps
 * alive until pt_free (the library never frees it), or NULL to let the library
 * allocate.  On error *out is NULL and nothing is leaked. */
int pt_init(pt_ctx **out, const pt_instance *inst, int32_t n_inst, const pt_options *opt,
            void *stream, void *workspace, size_t workspace_bytes);

/* n_sweeps >= 0 sweeps of every replica of every instance (t += n_sweeps). */
int pt_sweep(pt_ctx *ctx, int32_t n_sweeps);

/* One replica-exchange step of every instance (e += 1). */
int pt_exchange(pt_ctx *ctx);

/* n_cycles x (sweeps_per_exchange sweeps, then one exchange step), the same chain as
 * pt_sweep(k) + pt_exchange() per cycle (Figure 6's loop).  Cycles are replayed from a HIP
 * graph; for batches of at most 64 tiles each cycle is a single set of launches in which
 * the workgroup that finishes an instance's last tile runs that instance's exchange step
 * (per-instance completion counts), larger batches launch the exchange separately.  When
 * every instance fits one tile (and neither PT_FLAG_TAU_CORR nor PT_FLAG_NO_GRAPH is set)
 * up to 1024 cycles run in one launch instead, each workgroup doing its instance's exchange
 * steps itself; pt_info counts these launches (multi_launches, multi_cycles) and, with
 * PT_FLAG_TIMING, times them apart from the sweep and exchange launches (multi_ms).  With
 * PT_FLAG_NO_GRAPH every cycle is launched eagerly.  The chain is the same in every case. */
int pt_run(pt_ctx *ctx, int32_t n_cycles);

/* Wait for all work queued on the context's stream. */
int pt_sync(pt_ctx *ctx);

/* Copy instance inst's observables to the host (synchronising). */
int pt_observables(pt_ctx *ctx, int32_t inst, pt_obs *out);

/* Copy instance inst's spins to host int8 out[R][M][N] by replica slot (synchronising). */
int pt_get_spins(pt_ctx *ctx, int32_t inst, int8_t *out);

/* Replace instance inst's spins from host int8 in[R][M][N] (values must be +1/-1) and
 * recompute its E_cl and C. */
int pt_set_spins(pt_ctx *ctx, int32_t inst, const int8_t *in);

/* Checkpoint: with buf == NULL, *len receives the size; otherwise the mutable state is
 * written to buf (*len >= size).  pt_load restores it into a context created with the
 * same instances and options; the continued run is identical to an uninterrupted one. */
int pt_save(pt_ctx *ctx, void *buf, size_t *len);
int pt_load(pt_ctx *ctx, const void *buf, size_t len);

/* The checks pt_load makes before it copies anything, without a context or a GPU: with
 * buf == NULL only *need (if not NULL) receives the checkpoint size for these instances
 * and options.  Otherwise the checkpoint must have that size and a header written for
 * them (magic, version, seed, instance count, encoding), PT_INT8 spin bytes must be 0 or
 * 1, replica_of and rung_of of every instance inverse permutations of [0, R), and labels
 * PT_LABEL_*: the kernels use these values as indices, so a corrupt checkpoint is refused
 * with PT_ESTATE rather than loaded.  Layout: a 40-byte header (uint32 magic 0x51505450,
 * uint32 version, uint64 state bytes, uint64 seed, int32 instances, int32 encoding,
 * uint64 sum of R*N*M) followed by the state bytes. */
int pt_checkpoint_validate(const pt_instance *inst, int32_t n_inst, const pt_options *opt,
                           const void *buf, size_t len, size_t *need);

/* Tuning and timing record; pt_timing_reset zeroes the timing fields (synchronising).
 * pt_timing_enable switches PT_FLAG_TIMING on (on != 0) or off for the calls that follow
 * (synchronising): while it is on, pt_run launches cycle by cycle with events around
 * every launch instead of replaying its graph, so a caller can time the graph route with
 * it off and take per-launch durations in a separate pass with it on. */
int pt_get_info(pt_ctx *ctx, pt_info *out);
int pt_timing_reset(pt_ctx *ctx);
int pt_timing_enable(pt_ctx *ctx, int32_t on);

void pt_free(pt_ctx *ctx);
const char *pt_strerror(int code);
const char *pt_last_error(void);

/* The acceptance threshold thr(dS) of the trajectory contract as the library's host code
 * builds its tables (no GPU needed). */
uint32_t pt_threshold(double dS);

/* The same rule evaluated by the device code that decides swaps, for n values: dS and
 * out are device pointers; runs on stream (NULL: default stream) and synchronises. */
int pt_threshold_device(const double *dS, uint32_t *out, int32_t n, void *stream);

/* ---------------------------------------------------------------- ladder network
 * The ladder is data (b_r, K_r) for the sampler; choosing it is outside the Markov chain
 * (the paper defers ladder selection to its reference [7], Section 2).  The library
 * carries the FP32 kernels of a small network that proposes ladders from instance
 * features: 32 -> 128 -> 128 -> 64 with ReLU after the hidden layers; its 64 outputs are
 * per-rung values (how the caller turns them into (b_r, K_r) is the caller's choice).
 * Parameters are pt_mlp_param_count() floats: W1[128][32], b1[128], W2[128][128],
 * b2[128], W3[64][128], b3[64].  All pointers are device pointers; work runs on stream
 * (NULL: default stream) asynchronously; workspace holds pt_mlp_workspace_bytes(batch)
 * bytes.  The dense products run on the matrix cores (v_mfma_f32_16x16x4f32). */
#define PT_MLP_LOSS_SOFTMAX 0 /* -sum_j q_j log softmax(z)_j, rows of q sum to 1        */
#define PT_MLP_LOSS_SIGMOID 1 /* per-output logistic cross entropy, q in [0, 1]          */
int32_t pt_mlp_param_count(void);
size_t pt_mlp_workspace_bytes(int32_t batch);

/* logits[batch][64] for features x[batch][32]. */
int pt_mlp_forward(const float *params, const float *x, float *logits, int32_t batch,
                   void *workspace, void *stream);

/* pt_mlp_forward without a workspace, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same kernels, with the hidden activations in a fixed array of device memory that
 * the library holds on each GPU it runs on until the process ends (2 x 4096 x 128 floats,
 * 4 MiB).  Nothing is allocated or freed by the call.  batch must be in
 * [1, PT_MLP_STATIC_MAX_BATCH], else PT_EINVAL.  Every call on one GPU shares that GPU's
 * array: calls that overlap in time on one GPU (other streams, other host threads) race
 * and must be serialised by the caller.  The device is the calling thread's current
 * device; its array's address is looked up on the first call there. */
#define PT_MLP_STATIC_MAX_BATCH 4096
int pt_mlp_forward_static(const float *params, const float *x, float *logits, int32_t batch,
                          void *stream);

/* Loss loss_kind (PT_MLP_LOSS_*) against targets target[batch][64]: writes grads
 * (pt_mlp_param_count() floats) of the batch mean, and loss[0] = the batch sum of the
 * per-sample losses. */
int pt_mlp_loss_grad(const float *params, const float *x, const float *target, int32_t batch,
                     int32_t loss_kind, float *grads, float *loss, void *workspace,
                     void *stream);

/* One Adam step (Kingma & Ba, bias-corrected, step >= 1) over n parameters. */
int pt_mlp_adam(float *params, const float *grads, float *m, float *v, int32_t n, float lr,
                float beta1, float beta2, float eps, int32_t step, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PTQMC_H */
