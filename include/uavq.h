/*
 * uavq.h -- C ABI of the MI355X annealer for the UAV coverage-path QUBO.
 *
 * Method (paper: "GPU-Accelerated Quantum Annealing-Inspired UAV Path Planning
 * for Smart Agriculture"): a field of M x N square cells (Sec. II) is covered
 * by a tour that starts at cell c_{0,0}; the tour is written as a one-hot,
 * time-indexed QUBO H = H_dist + P (H_visit + H_time) (Sec. III-B, eqs.
 * (3)-(6)) and minimised by parallel annealing over many independent replicas
 * (Sec. III-C, Alg. 1, Sec. IV-A).  This library builds that QUBO
 * (uavq_qubo_build), anneals batches of instances on the GPU
 * (uavq_anneal_batch) and evaluates energies (uavq_energy_eval).
 *
 * Conventions
 *   - Every function returns 0 (UAVQ_OK) or a negative UAVQ_E* code; the
 *     message of the last failure on the calling thread is uavq_last_error().
 *     On failure no output buffer is written unless stated otherwise.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device memory owned by the caller (the library never frees them).
 *   - Handles (uavq_qubo, uavq_plan) are created and freed by the library.  A
 *     qubo is immutable.  A plan's only state after creation is a cache filled
 *     on first use (the launch shape, which needs the device, and in
 *     UAVQ_GRAPH mode the captured graph), guarded by a per-plan lock: both
 *     handles may be shared between threads (graph-mode launches of one plan
 *     are serialised by that lock; a call with other buffers or another
 *     stream re-captures).  uavq_plan_set_timing / uavq_plan_sweep_ms are the
 *     exception: not thread-safe per plan.
 *   - Streams are hipStream_t passed as void*; NULL is the default stream.
 *     uavq_anneal_batch and uavq_energy_eval_dev are asynchronous on it.
 *
 * Variables and states
 *   m = number of cells to visit (free cells: not the start cell, not
 *   no-fly), listed in increasing row-major index (the free list F).  The
 *   variable x_{t,c} (step t = 1..m, free cell c = 0..m-1) is 1 when the tour
 *   is at F[c] at step t; steps 0 and m+1 are fixed at the start cell (the
 *   fixed start of Sec. II; the closed tour returns to it).  N = m*m.
 *   Packed state: m rows of W = ceil(m/32) uint32 words; bit (c & 31) of
 *   word (t-1)*W + (c >> 5) is x_{t,c}; unused high bits are zero.
 *   state_words = m * W.
 */
#ifndef UAVQ_H
#define UAVQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    UAVQ_OK = 0,
    UAVQ_EINVAL = -1,       /* invalid argument */
    UAVQ_ENOMEM = -2,       /* host allocation failed */
    UAVQ_EHIP = -3,         /* a HIP runtime call failed (message names it) */
    UAVQ_ETOOBIG = -4,      /* the instance exceeds a kernel's limits */
    UAVQ_EINFEASIBLE = -5,  /* a state is not a permutation matrix */
    UAVQ_EINVARIANT = -6    /* an energy kept incrementally differs from its recomputation */
};

/* Message for the last error on this thread ("" if none).  Static storage. */
const char *uavq_last_error(void);

/* ABI version (major*100 + minor). */
int32_t uavq_version(void);

/* ------------------------------------------------------------------ QUBO -- */

#define UAVQ_OPEN_PATH 0x1u   /* no return leg (eq. (1a) as printed); default closed tour */
#define UAVQ_DENSE     0x2u   /* also keep the dense int16 J (needed by the dense kernel) */

typedef struct {
    int32_t rows, cols;       /* M, N of Sec. II; rows*cols <= 65536 */
    int32_t depot;            /* row-major index of the start cell (c_{0,0} = 0) */
    const uint8_t *nofly;     /* host, rows*cols bytes, 1 = excluded; NULL = none */
    int32_t cost_scale;       /* w = round(cost_scale * distance in cells); 0 -> 10
                                 (deciseconds for 5 m cells at 5 m/s, Sec. IV-C) */
    int32_t penalty;          /* P; 0 -> 2 * w_max; otherwise must exceed w_max */
    uint32_t flags;           /* UAVQ_OPEN_PATH | UAVQ_DENSE */
} uavq_grid;

typedef struct uavq_qubo uavq_qubo;

typedef struct {
    int32_t m;                /* free cells = steps */
    int32_t n_vars;           /* N = m*m */
    int32_t P;                /* one-hot penalty weight */
    int32_t w_max;            /* largest travel cost between visit-list cells */
    int64_t c0;               /* constant term, 2*P*m */
    int32_t closed;           /* 1 = closed tour */
    int32_t has_dense;        /* dense J kept */
    int32_t row_words;        /* W = ceil(m/32) */
    int32_t state_words;      /* m * W */
} uavq_qubo_info_t;

/* qubo_build -- Sec. II (grid, travel times t_ij = d_ij tau) and Sec. III-B
 * eqs. (3)-(6) expanded with x^2 = x:
 *   E(x) = c0 + sum_k b_k x_k + sum_{k<l} J_kl x_k x_l,
 *   c0 = 2 P m,  b_{t,c} = -2P + [t=1] w(s,c) + [t=m, closed] w(c,s),
 *   J_{(t,c),(t',c')} = 2P [t=t'] + 2P [c=c'] + w(c,c') [|t-t'| = 1]
 * (s = start cell).  The handle keeps the free list, the cost matrix D
 * (m x m) and the start-cell costs, and the dense J when UAVQ_DENSE is set.
 * Errors: EINVAL for a bad grid (no free cell, start cell no-fly, penalty <=
 * w_max, rows*cols > 65536) or a penalty too large for int32 fields (P >
 * 2^20, or 2P (3m + 2) + 2 m w_max >= 2^30); ETOOBIG when w_max > 255 (D is
 * stored as bytes) or, with UAVQ_DENSE, when N > 46340 or 2P + w_max > 16383
 * (the dense J splits into two int8 limbs). */
int uavq_qubo_build(const uavq_grid *g, uavq_qubo **out);
void uavq_qubo_free(uavq_qubo *q);
int uavq_qubo_info(const uavq_qubo *q, uavq_qubo_info_t *info);
/* Host copies: F (m grid indices); costs ((m+1)^2, index 0 = start cell). */
int uavq_qubo_free_cells(const uavq_qubo *q, int32_t *F);
int uavq_qubo_costs(const uavq_qubo *q, int32_t *W);
/* Host export of b (N) and, if J != NULL, the dense J (N*N, row-major). */
int uavq_qubo_export(const uavq_qubo *q, int32_t *b, int32_t *J);

/* ---------------------------------------------------------------- energy -- */

/* energy_eval -- E(x) of n_states packed host states (eqs. (3)-(6) through the
 * expanded form), written to E (host, n_states). */
int uavq_energy_eval(const uavq_qubo *q, const uint32_t *x_packed, int64_t n_states, int64_t *E);

/* energy_eval on the device: E for n_states packed device states (contiguous,
 * state_words apart) computed by the MFMA refresh kernel; d_E is device
 * int64[n_states].  d_ws must hold uavq_energy_workspace_bytes() bytes. */
int uavq_energy_workspace_bytes(const uavq_qubo *q, size_t *bytes);
int uavq_energy_eval_dev(const uavq_qubo *q, const uint32_t *d_x_packed, int64_t n_states, int64_t *d_E,
                         void *d_ws, size_t ws_bytes, void *stream);

/* energy_eval on the device without a workspace, for callers that cannot
 * allocate device memory (code under stream capture, serving loops, harnesses
 * that forbid allocation): the same computation as uavq_energy_eval_dev, with
 * the staging (cost matrix and start-cell costs, uavq_energy_workspace_bytes)
 * in a static device buffer of 80 KiB that each device keeps until the process
 * ends.  Allocates nothing.  ETOOBIG when the staging exceeds that buffer
 * (m >= 286; the refresh kernel itself stops at m = 283).  All calls on one
 * device share the buffer: calls that may overlap on a device (other streams
 * or threads) race and must be ordered by the caller. */
int uavq_energy_eval_dev_noalloc(const uavq_qubo *q, const uint32_t *d_x_packed, int64_t n_states, int64_t *d_E,
                                 void *stream);

/* Path reconstruction (Alg. 1, last step): for a permutation state, path[0..m+1]
 * (grid indices: start, the visited cells in order, start again; for an open
 * path path[m+1] = -1) and its travel cost.  EINFEASIBLE otherwise. */
int uavq_decode_path(const uavq_qubo *q, const uint32_t *x_packed, int32_t *path, int64_t *cost);

/* -------------------------------------------------------------- schedule -- */

/* Geometric temperatures T_s = T0 (T1/T0)^(s/(S-1)) and the acceptance table
 * thr[s][d] = min(2^32-1, floor(2^32 exp(-d/T_s))), d = 0..Dmax (column 0
 * unused), Dmax = least d with floor(2^32 exp(-d/T0)) = 0.  Pass thr = NULL to
 * query Dmax; otherwise thr holds S*(Dmax+1) uint32 (host).  Requires
 * 0 < T1 <= T0, S >= 1. */
int uavq_schedule(double T0, double T1, int32_t S, int32_t *Dmax, uint32_t *thr);

/* ------------------------------------------------------------- annealing -- */

#define UAVQ_KERNEL_DENSE 0x1u   /* use the dense-field kernel (every qubo needs UAVQ_DENSE) */
#define UAVQ_VARIANT_ROWMASK 0x10u /* m <= 64: rebuild travel rows from step masks instead of
                                      keeping them in LDS (a schedule choice; same results) */
#define UAVQ_PERSISTENT 0x20u      /* persistent sweep kernels: an occupancy-sized grid pulls
                                      work items (largest instances first) from a counter */
#define UAVQ_GRAPH 0x40u           /* capture the launch sequence of anneal_batch into a HIP graph
                                      on first use and replay it while the buffers and stream are
                                      the same; needs a non-default stream */
#define UAVQ_VARIANT_NOPRODUCER 0x80u /* m <= 64 at one wave per SIMD: no cut-producing wave beside
                                      each replica's wave (a schedule choice; same results) */
#define UAVQ_STOP_FROZEN 0x100u    /* factored kernels: a replica whose sweep had neither an accept nor
                                      a draw sweeps no more.  Every later sweep would leave it unchanged
                                      (all its dE are at or above the draw cutoff, which never grows
                                      along the schedule: plan_create checks, EINVAL otherwise), so
                                      every output is the same; the launch ends when all are frozen.
                                      Not for throughput measurements: frozen sweeps are not evaluated. */
#define UAVQ_VARIANT_GENERIC 0x400u /* 64 < m <= 384: the generic chunked walk (every step walked) instead
                                      of the kernel that first tests blocks of four steps whose steps
                                      each hold one cell (a schedule choice; same results) */
#define UAVQ_CONCURRENT_CLASSES 0x800u /* the sweep kernels of different chunk classes run at the same
                                      time (the first on the caller's stream, the others on streams the
                                      plan owns, forked and joined with events), so one class's blocks
                                      fill the CUs that another's tail leaves idle.  Same results. */
#define UAVQ_REDUCE_AT_END 0x200u  /* uavq_anneal_segment fills the per-instance outputs (inst_best_*)
                                      only in a segment that ends the schedule (s_end = S); earlier
                                      segments leave them untouched.  Per-replica outputs are unchanged. */

/* Launch shape chosen by uavq_autotune (never changes results). */
typedef struct {
    int32_t waves_per_block[10]; /* per chunk class (index 0 unused); 0 = default; classes 4..9
                                    run at most 4 per block */
    uint32_t variant_flags;      /* 0 or UAVQ_VARIANT_ROWMASK / _NOPRODUCER / _GENERIC */
    float trial_ms;              /* measured time of the chosen shape (trial run) */
} uavq_tune;

typedef struct {
    int32_t replicas;         /* replicas per instance, >= 1 */
    int32_t sweeps;           /* S >= 1 */
    double T0, T1;            /* schedule end points, 0 < T1 <= T0 */
    uint32_t seed;            /* random-stream key */
    uint32_t flags;           /* UAVQ_KERNEL_DENSE */
    int32_t waves_per_block;  /* replicas per workgroup; 0 = library choice.
                                 Never changes results. */
    const uavq_tune *tune;    /* optional per-class launch shape (overrides the two above) */
    const double *inst_T;     /* optional per-instance schedules: 2 * n_inst values, (T0_i, T1_i)
                                 for instance i (0 < T1_i <= T0_i); NULL = (T0, T1) for every
                                 instance.  A constant schedule (T0_i = T1_i) holds one table row.
                                 The slots of a tempering ladder run as one plan this way. */
} uavq_anneal_params;

typedef struct uavq_plan uavq_plan;

/* Plan for annealing n_inst instances (ids inst_ids[i], which address the
 * random streams, so an instance gives the same result alone or in a batch).
 * Builds the schedule table and packs all static data on the host. */
int uavq_plan_create(const uavq_qubo *const *q, int32_t n_inst, const uint32_t *inst_ids,
                     const uavq_anneal_params *p, uavq_plan **out);
void uavq_plan_free(uavq_plan *plan);

typedef struct {
    size_t ws_bytes;          /* device workspace needed */
    int64_t total_replicas;   /* n_inst * replicas */
    int64_t total_state_words;/* sum over instances of replicas * state_words */
    int32_t n_inst;
    int32_t Dmax;
} uavq_plan_info_t;
int uavq_plan_info(const uavq_plan *plan, uavq_plan_info_t *info);
/* Name of the sweep kernel that uavq_anneal_batch launches for the
 * instances of chunk class cls (1: m <= 64, 2: m <= 128, ..., 9: m <= 576; a field
 * whose costs exceed 255 runs in class 7 or above, which read 16-bit costs), for
 * profiling and reports: "" if the class is empty, NULL on error (cls out of
 * range, or no HIP device to decide the launch shape on).  The string is
 * static. */
const char *uavq_plan_kernel_name(const uavq_plan *plan, int32_t cls);
/* Replica r of instance i is global replica rep_offset[i] + r; its packed
 * state starts at word state_offset[i] + r * state_words(i).  Arrays of
 * n_inst + 1 entries (host). */
int uavq_plan_layout(const uavq_plan *plan, int64_t *rep_offset, int64_t *state_offset);

/* Copy the plan's static data (schedule table, cost matrices, dense J) into
 * the device workspace.  Must precede uavq_anneal_batch on that workspace. */
int uavq_plan_upload(const uavq_plan *plan, void *d_ws, size_t ws_bytes, void *stream);

typedef struct {              /* optional device inputs (NULL = unused) */
    const uint32_t *states;   /* total_state_words: initial states */
    const uint8_t *seeded;    /* total_replicas: 1 = start from states[], 0 = random bits */
    const int32_t *start_sweep; /* total_replicas: first sweep of that replica (0..S) */
} uavq_anneal_init;

typedef struct {              /* device outputs, caller-owned; NULL = not wanted */
    uint32_t *final_states;   /* total_state_words (required: also the working state) */
    int64_t *final_E;         /* total_replicas (required) */
    int64_t *best_E;          /* total_replicas (required) */
    int32_t *best_sweep;      /* total_replicas (required) */
    uint32_t *best_states;    /* total_state_words (required) */
    uint64_t *accepts;        /* total_replicas (required) */
    uint64_t *draws;          /* total_replicas (required): random draws taken */
    int64_t *inst_best_E;     /* n_inst */
    int32_t *inst_best_replica;
    int32_t *inst_best_sweep;
    uint32_t *inst_best_state;/* total over instances of state_words */
    int64_t *check_E;         /* total_replicas: E(final state) recomputed by the refresh */
    uint64_t *attempts;       /* total_replicas: flips attempted, N per sweep the replica ran
                                 (sweeps max(start_sweep, s_begin) .. s_end-1); carried on resume
                                 like accepts.  A replica stopped by UAVQ_STOP_FROZEN still counts
                                 the sweeps it skipped: every site of them is rejected. */
} uavq_anneal_out;

/* anneal_batch -- single-flip Metropolis annealing of every replica:
 *   x <- initial state (Bernoulli(1/2) bits from random stream 1, or given);
 *   for s = start..S-1, for k = 0..N-1 in step-major order:
 *     dE = (1 - 2 x_k) h_k,  h_k = b_k + sum_{l != k} J_kl x_l;
 *     accept if dE <= 0, otherwise iff u < thr[s][min(dE, Dmax)] where u is
 *     word (t-1) mod 4 of Philox4x32-10(counter {c + 65536 ((t-1) div 4), s,
 *     r, inst}, key {seed, 0}) and no draw is taken when that entry is 0;
 *   at each sweep end the state is kept as the replica's best if E < best_E.
 * Per instance the best is the lexicographic minimum of (best_E, replica).
 * Asynchronous on `stream`; outputs are valid once the stream has drained.
 * d_ws is read, and in persistent or dense mode also written (item counters,
 * unpacked states and fields): launches that may overlap need a workspace
 * each (uavq_plan_upload into every one). */
int uavq_anneal_batch(const uavq_plan *plan, void *d_ws, size_t ws_bytes, const uavq_anneal_init *init,
                      const uavq_anneal_out *out, void *stream);

/* anneal_segment -- the same annealing cut into pieces: runs sweeps
 * s_begin .. s_end-1 (0 <= s_begin <= s_end <= S) of the plan's S-sweep
 * schedule.  With resume = 0 the replicas start as in anneal_batch (initial
 * states from init, best_E = +inf).  With resume != 0 they continue from what
 * *out holds: final_states is the working state, and best_E, best_sweep,
 * best_states, accepts and draws are carried on, so a run cut into
 * [0, S1) + [S1, S) -- or checkpointed after S1 (copy final_states, best_E,
 * best_sweep, best_states, accepts and draws out), restored into the buffers and resumed -- gives bit for bit the
 * outputs of one anneal_batch call (every random draw is keyed by its sweep,
 * so the split leaves the random streams unchanged).  init->states and
 * init->seeded are ignored on resume; init->start_sweep still applies.  The
 * per-instance outputs and check_E describe the state after s_end.
 * anneal_batch is anneal_segment(0, S, resume = 0).  Errors: UAVQ_EINVAL for
 * a range outside [0, S] or any argument anneal_batch rejects. */
int uavq_anneal_segment(const uavq_plan *plan, void *d_ws, size_t ws_bytes, const uavq_anneal_init *init,
                        const uavq_anneal_out *out, int32_t s_begin, int32_t s_end, int32_t resume, void *stream);

/* anneal_checked -- anneal_batch with periodic invariant checks: the schedule
 * runs in pieces of refresh_every sweeps (anneal_segment, resumed), and after
 * each piece the MFMA refresh recomputes the energy of eqs. (3)-(6) from every
 * replica's working state and compares it with the energy the sweep kernels
 * kept by adding the dE of accepted flips.  d_violations (device, caller-owned,
 * total_replicas uint32, cleared by the call) counts each replica's
 * mismatching pieces; *n_violations (host) receives their sum.  out->check_E
 * is required (it holds the last recomputation).  The outputs equal those of
 * anneal_batch bit for bit.  Synchronous: the call waits for `stream`.
 * Errors: UAVQ_EINVARIANT when any piece mismatched (outputs still written);
 * UAVQ_EINVAL for refresh_every < 1, a missing buffer or a graph-mode plan;
 * UAVQ_ETOOBIG for fields the refresh kernel does not take (m > 384 or costs
 * above 255). */
int uavq_anneal_checked(const uavq_plan *plan, void *d_ws, size_t ws_bytes, const uavq_anneal_init *init,
                        const uavq_anneal_out *out, int32_t refresh_every, uint32_t *d_violations,
                        uint64_t *n_violations, void *stream);

/* Autotuner: times anneal_batch launch shapes (replicas per workgroup per
 * chunk class, m <= 64 kernel variant) on a short trial of trial_sweeps
 * sweeps of these instances, with device memory it allocates and frees
 * itself, and returns the fastest in *out.  With cache_path != NULL the choice
 * is read from / written to that JSON file, keyed by device, replicas and the
 * instance-size classes.  Every shape gives identical results. */
int uavq_autotune(const uavq_qubo *const *q, int32_t n_inst, const uint32_t *inst_ids,
                  const uavq_anneal_params *p, int32_t trial_sweeps, const char *cache_path, uavq_tune *out);

/* ------------------------------------------------------------ warm start -- */
/* A per-cell network predicts, for every free cell, a distribution over the
 * step at which a good tour visits it; tours sampled from it seed a fraction
 * of the replicas, which then start at a later (colder) sweep.  Not in the
 * paper: it is this project's learned warm start for the annealer of Alg. 1.
 *
 * Network: 16 inputs -> 128 -> 128 -> 128 logits (one per step; m <= 128),
 * ReLU between layers, softmax over steps 1..m.  Parameters are one fp32
 * vector of uavq_mlp_param_count() floats: W1[16][128], b1[128], W2[128][128],
 * b2[128], W3[128][128], b3[128] (row-major, x W convention).  Every product
 * rounds both operands to bfloat16 and accumulates in fp32 (MFMA).
 * All pointers below are device pointers unless stated. */
int uavq_mlp_param_count(void);
/* Features (host): X[m][16] for the free cells in free-list order: (i, j)/(s-1);
 * offset from the start cell /(s-1); its distance /(sqrt(2)(s-1)); no-fly
 * cells at Chebyshev distance 1 (/8) and <= 2 (/24); for r = 1..8 the fraction
 * of non-no-fly cells among the grid cells at Chebyshev distance r; m/99
 * (s = max(rows, cols)). */
int uavq_mlp_features(const uavq_qubo *q, float *X);
/* Workspace for rows input rows (both calls below). */
int uavq_mlp_workspace_bytes(int32_t rows, size_t *bytes);
/* probs[rows][128]: softmax over the first m[row] steps (0 beyond). */
int uavq_mlp_forward(const float *d_params, const float *d_X, const int32_t *d_m, int32_t rows, float *d_probs,
                     void *d_ws, size_t ws_bytes, void *stream);
/* Mean cross-entropy of the label steps (0-based, < m) and its gradient
 * d_grad[param_count]; d_loss[0] = summed (not averaged) loss. */
int uavq_mlp_loss_grad(const float *d_params, const float *d_X, const int32_t *d_m, const int32_t *d_label,
                       int32_t rows, float *d_grad, float *d_loss, void *d_ws, size_t ws_bytes, void *stream);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8, bias-corrected; step >= 1). */
int uavq_mlp_adam(float *d_params, float *d_m1, float *d_m2, const float *d_grad, int32_t step, float lr,
                  void *stream);
/* q[row][t] = floor(p * 65534) + 1 (1..65535) for t < m[row], else 0 (uint16). */
int uavq_quantize_marginals(const float *d_probs, const int32_t *d_m, int32_t rows, uint16_t *d_q, void *stream);
/* Seed states: for instance i of the plan, replicas 0..n_seeded[i]-1 get a
 * permutation drawn from q (rows q_row_off[i] .. +m of 128 steps), written to
 * d_states in the plan's state layout.  Step t goes to the first unvisited
 * cell whose running sum of q[., t] over unvisited cells exceeds
 * floor(u W / 2^32), u = word 0 of Philox({t, r, id, 0}, {seed, 4}).
 * q_row_off and n_seeded are host arrays; d_scratch holds 32 bytes per
 * instance.  Synchronises the stream before returning. */
int uavq_sample_seeds(const uavq_plan *plan, const uint16_t *d_q, const int64_t *q_row_off, const int32_t *n_seeded,
                      uint32_t *d_states, void *d_scratch, size_t scratch_bytes, void *stream);

/* ------------------------------------------------------ replica exchange -- */
/* Parallel tempering: an extension of the many-replica search of Sec. III-C
 * (the paper runs independent replicas).  Each chain r = 0..R-1 has K slots at
 * the fixed temperatures of a geometric ladder; slot k is instance k of one
 * plan (the same QUBO, instance id inst_id + k, the constant schedule T_k via
 * uavq_anneal_params.inst_T; chain sets that must be independent need
 * disjoint id ranges), run in segments (uavq_anneal_segment); between
 * segments, neighbouring slots of a chain trade
 * their states by the Metropolis rule on the product of the two Boltzmann
 * weights: with d = E_{k+1} - E_k and db = 1/T_{k+1} - 1/T_k > 0 the swap is
 * accepted with probability min(1, exp(db d)).
 *
 * Ladder (host): T[k] = T_hot (T_cold/T_hot)^(k/(K-1)), k = 0..K-1 (T_hot for
 * K = 1).  For pair k = 0..K-2: xthr[k][a] = min(2^32-1, floor(2^32 exp(-a db)))
 * for a = 0..DX[k], zero beyond; DX[k] = least a >= 1 with a zero entry.
 * Pass xthr = NULL to query DX and *max_dx; then xthr holds (K-1)*stride
 * uint32 with stride >= *max_dx + 1.  Errors: UAVQ_EINVAL unless
 * 1 <= K <= 4096 and 0 < T_cold < T_hot (for K >= 2) are finite, or stride is
 * too small; UAVQ_ETOOBIG if some DX exceeds 2^22 (slots too close). */
int uavq_pt_ladder(double T_hot, double T_cold, int32_t K, double *T, int32_t *DX, int32_t *max_dx, uint32_t *xthr,
                   int32_t stride);
/* One exchange round (device pointers, asynchronous on stream): the pairs
 * (k, k+1) with k = round mod 2, k + 2, ... of every chain.  A pair swaps
 * when d >= 0; otherwise, with a = min(-d, DX[k]), when
 * u < xthr[k][a] (no draw for a zero entry), u = word 0 of
 * Philox({k, round, r, inst_id}, {seed, 5}).  A swap exchanges the chains'
 * state words and energies.  d_states: [K][R][state_words] (the plan's
 * final_states), d_E: [K][R] (its final_E), d_DX: [K-1],
 * d_xthr: [K-1][stride]; d_swaps (NULL or [K-1] uint64) counts accepted swaps
 * per pair.  K = 1 does nothing.  Errors: UAVQ_EINVAL for a null pointer,
 * K outside 1..4096, R outside 1..2^20, state_words < 1 or stride < 2. */
int uavq_pt_exchange(int32_t K, int32_t R, int32_t state_words, uint32_t round, uint32_t seed, uint32_t inst_id,
                     const int32_t *d_DX, const uint32_t *d_xthr, int32_t stride, int32_t *d_states, int64_t *d_E,
                     uint64_t *d_swaps, void *stream);
/* The same round for n_sets chain sets of one plan at once (a batch of
 * fields, each with K slots of R chains on the same ladder): set i's slots
 * are instances i*K .. i*K + K - 1 of the plan, its states start at word
 * d_state_off[i] of d_states ([K][R][d_words[i]]), its energies at
 * d_E + i*K*R ([K][R]), its draws are addressed by d_inst[i], and its swaps
 * (if d_swaps) go to d_swaps[i*(K-1) + k].  All arrays are device arrays of
 * n_sets entries.  Errors as uavq_pt_exchange; n_sets outside 1..65535 is
 * UAVQ_EINVAL. */
int uavq_pt_exchange_batch(int32_t n_sets, int32_t K, int32_t R, uint32_t round, uint32_t seed,
                           const int64_t *d_state_off, const int32_t *d_words, const uint32_t *d_inst,
                           const int32_t *d_DX, const uint32_t *d_xthr, int32_t stride, int32_t *d_states,
                           int64_t *d_E, uint64_t *d_swaps, void *stream);

/* Kernel timing for measurement: when enabled, uavq_anneal_batch records HIP
 * events on its stream around the sweep-kernel launches of this plan, and
 * uavq_plan_sweep_ms returns their elapsed time (ms) for the last call once
 * the stream has drained.  Changes no result.  Not thread-safe per plan. */
int uavq_plan_set_timing(uavq_plan *plan, int32_t enable);
int uavq_plan_sweep_ms(const uavq_plan *plan, float *ms);

#ifdef __cplusplus
}
#endif
#endif /* UAVQ_H */
