/*
 * tapt.h -- C ABI of the MI355X (gfx950) TAPT hot-path library, libtapt.so.
 *
 * Transformer-Augmented Parallel Tempering (arXiv:2509.23043, Algorithm 1):
 * replicas of a sparse Ising problem on a fixed inverse-temperature ladder
 * run graph-colored single-spin Monte Carlo sweeps, accept pre-generated
 * global proposals with the Delta-E-only rule (Eq. 2) and exchange states
 * between neighbouring temperatures with alternating parity (Eq. 1).
 *
 * Conventions used by every entry point:
 *   - spins are int8 in {-1, +1}; configurations are [n] arrays in site order;
 *     replica arrays are [R][n], row r = beta slot r, slot 0 the hottest.
 *   - energy E(m) = -sum_{i<j} J_ij m_i m_j - sum_i h_i m_i (Supp. S4), int32.
 *   - "host pointer" arguments are caller-owned host memory, read or written
 *     during the call only. "device pointer" arguments are device memory of
 *     the context's GPU (e.g. a torch tensor's data_ptr()), used on the
 *     context's stream and complete when the call returns.
 *   - every call returns PT_OK (0) or a negative PT_E* code; on error
 *     pt_last_error() returns a message (thread-local) and no state changed,
 *     except PT_EDEVICE, after which the context is unusable.
 *   - a context is used by one host thread at a time; different contexts may
 *     be used concurrently.
 *
 * Random numbers follow a fixed counter-based contract (Philox4x32-10 keyed
 * by pt_opts.seed, counters from site, sweep, beta slot and a stream tag), so
 * results do not depend on tiling, batching or co-tenancy: the same problem,
 * ladder, options and seed give bit-identical chains on every path.
 */
#ifndef TAPT_H
#define TAPT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PT_OK 0
#define PT_EINVAL (-1)        /* bad argument */
#define PT_ENOMEM (-2)        /* device or host allocation failed, or over budget */
#define PT_EDEVICE (-3)       /* HIP error; the context is unusable afterwards */
#define PT_ESTATE (-4)        /* call not valid in the current state */
#define PT_EUNSUPPORTED (-5)  /* problem shape not supported by the kernels */
#define PT_ETIMEOUT (-6)      /* a cross-workgroup wait exceeded its bound */

#define PT_METROPOLIS 0       /* flip with min(1, exp(-beta dE)) */
#define PT_GIBBS 1            /* heat bath, Methods Eq. 5: flip with 1/(1+exp(beta dE)) */

typedef struct pt_ctx pt_ctx;
typedef struct pt_batch pt_batch;
typedef struct pt_server pt_server;

/* A sparse Ising problem (Methods, Eq. 4; Supp. S4). All pointers are host
 * pointers, copied by pt_create.
 *   lattice_L > 0: periodic L^3 cubic lattice, n = L^3, even L >= 4,
 *     site i = x + L*(y + L*z); J holds 3n bond couplings, J[d*n + i] for
 *     the bond from i to its +x (d=0), +y (1), +z (2) neighbour. row_ptr and
 *     col are ignored; colors are the checkerboard (x+y+z) mod 2.
 *   lattice_L == 0: general graph in CSR form with both directions of every
 *     edge stored, symmetric values, no self loops; J[nnz] couplings.
 *   h: [n] fields or NULL (all 0). clamp: [n] 0 = free, +-1 = fixed, or NULL.
 *   color: [n] proper coloring with colors 0..C-1 (C <= 64) for CSR graphs,
 *     required there (sites of a color are updated in parallel, colors in
 *     increasing order -- Methods, Graph coloring).
 * Limits: |J| <= 127, |h| <= 32767, n <= 32768, lattice L <= 32. */
typedef struct {
    int32_t n;
    int32_t lattice_L;
    int32_t nnz;
    const int32_t *row_ptr;
    const int32_t *col;
    const int32_t *J;
    const int32_t *h;
    const int8_t *clamp;
    const int32_t *color;
} pt_graph;

/* Run options (Algorithm 1 inputs). sweeps_per_cycle = 0 makes the slots
 * independent chains: no swap stage and no proposal stage ever runs, the
 * betas need only be positive (equal values allowed), and a context may run
 * at most 2^31 - 2 sweeps. This is the long-run MCMC that generates proposal
 * banks (Supp. Table S3 and the bank protocol after it: each sample from its
 * own randomly initialised chain after a burn-in). prop_period = 0 disables proposals;
 * otherwise a proposal stage runs at the end of sweep t when t >= prop_start,
 * (t - prop_start) % prop_period == 0 and (prop_stop < 0 or t <= prop_stop);
 * prop_start and prop_period must be multiples of sweeps_per_cycle.
 * target: first_hit records the first sweep with min_r E_r <= target. */
typedef struct {
    int32_t rule;              /* PT_METROPOLIS or PT_GIBBS */
    int32_t sweeps_per_cycle;  /* M >= 1: sweeps between swap stages; 0: independent chains */
    int64_t prop_start;
    int64_t prop_period;
    int64_t prop_stop;
    uint64_t seed;
    int32_t has_target;
    int32_t target;
} pt_opts;

/* Accept / attempt counters and best-energy record of a context. */
typedef struct {
    uint64_t t;                 /* completed sweeps */
    int32_t best_energy;        /* lowest min_r E_r seen (after init included) */
    int64_t best_t;             /* sweep when best_energy was first reached */
    int32_t best_slot;          /* lowest slot holding it at best_t */
    int64_t first_hit;          /* first sweep with min_r E_r <= target, or -1 */
} pt_summary;

/* Create a context: validate and copy the problem, build the uint32
 * acceptance tables on the host in FP64 (Eqs. 1, 2, 5), allocate device
 * state and initialise the replicas randomly (Algorithm 1, first line).
 * betas: host [R], strictly increasing, > 0 (slot 0 hottest); any positive
 * values for independent chains. R in 1..1024. */
int pt_create(const pt_graph *g, const double *betas, int32_t R, const pt_opts *o, pt_ctx **out);
int pt_destroy(pt_ctx *c);

/* Install (or replace) the proposal bank of the slot whose beta equals
 * ``beta`` exactly; n_configs = 0 clears it. configs: host pointer to
 * [n_configs][n] spins; every entry must be +-1 and match the clamps.
 * Entry energies are computed once on the device; the slot's cursor starts
 * at the contract's seeded offset and advances by one per proposal. */
int pt_propose(pt_ctx *c, double beta, const int8_t *configs, int32_t n_configs);
/* Same with configs in device memory (not validated entry by entry). */
int pt_propose_device(pt_ctx *c, double beta, const int8_t *configs_dev, int32_t n_configs);

/* Contextual proposals (Supp., ablation of proposal context, Fig. S4b):
 * with fraction > 0 or sweeps > 0, the proposal of a slot at cycle n is
 * built on the device rather than taken from the bank as is. It starts from
 * the slot's bank entry; K = round(fraction * n_free) free sites join the
 * context and take the slot's current values: the K of smallest key, site i's
 * key being word i&3 of Philox tag 7, ctr (i>>2, n, r, 7), ties to the lower
 * index (a uniformly random K-subset); `sweeps` colored
 * sweeps at the slot's beta, with the context's rule, update the other free
 * sites (Philox tag 8, ctr (i>>2, n, r + 65536 j, 8) for sweep j = 1..sweeps,
 * word i&3 as the 32-bit uniform); its energy is recomputed and the Delta-E
 * rule of Eq. 2 decides as for a bank entry, and the cursor advances as
 * usual. fraction = 0 and sweeps = 0 restore plain bank proposals.
 * fraction in [0, 1], sweeps in 0..65535, else PT_EINVAL. Contextual
 * contexts run in batches and the server only: pt_sweep returns
 * PT_EUNSUPPORTED for them, and a batch built before the mode changed
 * returns PT_ESTATE (build it again). */
int pt_set_context(pt_ctx *c, double fraction, int32_t sweeps);

/* Plain path: run n_sweeps more sweeps of Algorithm 1's main loop on this
 * context alone -- per sweep, one colored local sweep of every replica
 * (Methods, Eq. 4 and Graph coloring), then at the end of every cycle of
 * sweeps_per_cycle sweeps the proposal stage (Eq. 2) when the schedule says
 * so and the alternating-parity exchange stage (Eq. 1) -- with one launch
 * sequence per sweep (sweep kernel, cycle-end kernel). Blocks until done.
 * PT_EINVAL if the sweep counter would pass 2^32 - 1 (2^31 - 2 for
 * independent chains); PT_EUNSUPPORTED with contextual proposals. */
int pt_sweep(pt_ctx *c, uint64_t n_sweeps);

/* Current replica energies E(S_r) by slot (the energies Algorithm 1 holds
 * at the end of a cycle; Supp. S4 convention): host [R] int32, written
 * before the call returns. */
int pt_energies(pt_ctx *c, int32_t *out);
/* Current replica states S_r by slot (Algorithm 1's output): host [R][n]
 * int8 +-1, row r = slot r; the completed sweep count to *t if non-NULL.
 * spins may be NULL to read t alone. */
int pt_state(pt_ctx *c, int8_t *spins, uint64_t *t);
/* Same into device memory [R][n]. */
int pt_state_device(pt_ctx *c, int8_t *spins_dev);
/* Replace the spins (a fresh chain from a given state): host [R][n] spins
 * and sweep counter t. The counters and the best record restart; energies
 * are recomputed; bank cursors keep their values. For an exact resume use
 * pt_save / pt_restore. */
int pt_set_state(pt_ctx *c, const int8_t *spins, uint64_t t);

/* Checkpoint and resume. pt_save writes the whole chain state of a context
 * into a host buffer of pt_save_size bytes: spins and energies by slot, the
 * sweep counter, every bank cursor, the swap, proposal and flip counters and
 * the best record (energy, sweep, slot, first hit, configuration). Since
 * every random number is keyed by (seed, site, sweep, slot), pt_restore into
 * a context created with the same problem, ladder, options and seed, with
 * banks of the same sizes installed (the same banks, for the same chain) and
 * the same proposal mode, continues Algorithm 1 bit for bit as if the run had
 * never stopped, on any path (plain, batched, served). pt_restore checks the
 * blob's format, shape and fingerprint (problem, ladder, options, seed, bank
 * sizes, proposal mode), the spins (+-1, clamps), the cursors and that the
 * energies are those of the spins; on any mismatch it returns PT_EINVAL and
 * leaves the context unchanged. The blob is plain host memory in the
 * machine's byte order, owned by the caller. */
int pt_save_size(pt_ctx *c, uint64_t *bytes);
int pt_save(pt_ctx *c, void *buf, uint64_t bytes);
int pt_restore(pt_ctx *c, const void *buf, uint64_t bytes);

/* Summary and counters. swap_att/swap_acc: host [R-1] per pair (r, r+1);
 * prop_att/prop_acc/flips: host [R]; any may be NULL. best_spins: host [n]
 * or NULL. */
int pt_summary_get(pt_ctx *c, pt_summary *s, int8_t *best_spins);
int pt_counters(pt_ctx *c, uint64_t *swap_att, uint64_t *swap_acc, uint64_t *prop_att,
                uint64_t *prop_acc, uint64_t *flips);

/* Energies of configurations under the context's problem: device pointers,
 * configs [k][n] -> energies [k] (the full-recompute reduction kernel). */
int pt_energy_device(pt_ctx *c, const int8_t *configs_dev, int32_t k, int32_t *energies_dev);

/* Use a HIP stream (hipStream_t passed as void*, e.g. torch's current
 * stream) for this context's work; NULL = the library's own stream. */
int pt_set_stream(pt_ctx *c, void *stream);

/* ---- batched path: many contexts in one persistent launch per chunk ---- */
typedef struct {
    int32_t replicas_per_wg;     /* slots per workgroup (0 = choose) */
    int32_t replicas_per_thread; /* 1, 2 or 4 (0 = choose) */
    int32_t chunk_sweeps;        /* sweeps per persistent launch (0 = 1000) */
    int32_t use_graph;           /* 1: replay the chunk launches as a hipGraph */
    int32_t kernel;              /* 0 = choose; 1 = workgroup-synchronous kernel (general
                                        graphs with their LDS-resident CSR sweepers);
                                    2 = wave-per-replica kernel (lattices with n = 512);
                                    3 = +-J 8^3 kernel, two slots per wavefront (every
                                        coupling +-1, even R);
                                    4 = the same kernel with one slot per wavefront
                                        (at most 8 slots per workgroup);
                                    5 = workgroup-synchronous kernel, general graphs
                                        swept from packed rows, one storage per lane;
                                    6 = the same, four storages per lane. 5 and 6 fail
                                        with PT_EUNSUPPORTED where the rows do not fit;
                                        0 takes 6, else 5, where they fit;
                                    7 = +-J row kernel, one slot per wavefront, lattices
                                        of every even L in 6..16 in one launch (every
                                        coupling +-1, no fields), at most 8 slots per
                                        workgroup. 0 takes 7 where every context fits
                                        it and not all are 8^3 lattices (those take 3),
                                        else the other kernels;
                                    8 = general graphs, one slot per wavefront (n <= 4095,
                                        |J| <= 127, degree <= 64, colour classes of at most
                                        256 sites, at most 64 groups of 64 sites of one
                                        class), at most 8 slots per workgroup; 0 takes 8
                                        where every context fits it */
} pt_batch_opts;

/* Group contexts for batched execution. The contexts stay owned by the
 * caller and must outlive the batch; they may differ in size, ladder and
 * options. Results are bit-identical to running each context alone. */
int pt_batch_create(pt_ctx *const *ctxs, int32_t k, const pt_batch_opts *o, pt_batch **out);
int pt_batch_sweep(pt_batch *b, uint64_t n_sweeps);
int pt_batch_destroy(pt_batch *b);
/* Launch the batch's work on ``stream`` (hipStream_t as void*, e.g. torch's
 * current stream); NULL restores the batch's own stream. */
int pt_batch_set_stream(pt_batch *b, void *stream);
/* Total device time of the persistent chunk-kernel launches since the last
 * call, measured with HIP events recorded around each launch on the batch's
 * stream (launches replayed from a hipGraph are not timed), and their count.
 * Resets both. */
int pt_batch_kernel_time(pt_batch *b, double *ms, uint64_t *launches);
/* The launch plan of the batch as text, one line per launch group (contexts
 * that share a kernel): "kernel=K sweeper=S contexts=N grid=G block=B lds=L".
 * K is chunk, ctx, mixed, wave, pm or pm1; S names the sweeper of a chunk or
 * ctx launch (latticeLxRPT, csr, csr-wide, csr-quad, csr-row) or "-". The
 * text is truncated to len - 1 bytes and NUL-terminated. */
int pt_batch_describe(pt_batch *b, char *buf, int32_t len);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): run the k
 * contexts batched for n_sweeps sweeps exactly as pt_batch_create +
 * pt_batch_sweep + pt_batch_destroy would (bit-identical results, same
 * tilings and kernels; o as for pt_batch_create, use_graph ignored), with no
 * pt_batch object and no device allocation: the launch's work items, block
 * order, per-workgroup best records and snapshots, exchange words, status
 * and error flag live in a static device array of 32 MiB that the library
 * holds on each GPU it runs on until the process ends. A launch that needs
 * more returns PT_ENOMEM. stream: hipStream_t as void*, or NULL for the
 * stream of ctxs[0]; the call returns when the work is complete. Every call
 * on one GPU shares that GPU's array, so calls that overlap on one GPU (from
 * several threads) race and must be serialised by the caller. Host-side
 * planning uses ordinary host memory. */
int pt_batch_run_static(pt_ctx *const *ctxs, int32_t k, const pt_batch_opts *o, uint64_t n_sweeps, void *stream);

/* ---- serving: continuous batching of solve requests ----
 *
 * A server owns a worker thread and a stream. Callers register problems
 * (a context created with pt_create, with its proposal banks installed by
 * pt_propose: the paper reuses one bank across runs, Supp. S6) and submit
 * solve requests against them from any thread. A request is a fresh set of
 * replicas of a registered problem with its own seed, energy target and sweep
 * cap. It shares the problem's couplings, tables and banks in device memory
 * and owns only its replica state, which stays resident until it finishes.
 *
 * The worker runs rounds of chunk_sweeps sweeps over every admitted request.
 * Running requests are grouped in launch lanes: each lane is one persistent
 * launch, co-resident on its own, of the fastest kernel for its requests
 * (requests of one kind share a lane while it has room, so their work
 * overlaps on the device); a round runs the lanes' launches in turn. Between
 * rounds the worker retires the requests that reached their target or their
 * cap and admits waiting ones, first come first served, while their state
 * fits the device-memory budget (and max_active); a request that fits no
 * launch even alone is rejected with that launch's error.
 *
 * Results do not depend on co-tenants or arrival times. A request admitted at
 * sweep 0 stops at the first multiple of chunk_sweeps at or after its first
 * hit, or at its cap. All its random numbers are keyed by its seed (the
 * contract of pt_create). So first_hit, the best energy, the best
 * configuration and the sweep count equal those of the same context run
 * alone. */
typedef struct {
    uint64_t mem_budget;         /* device bytes for request state (0 = 1 GiB) */
    int32_t chunk_sweeps;        /* sweeps per round (0 = 500) */
    int32_t max_active;          /* cap on concurrent requests (0 = none) */
    int32_t replicas_per_wg;     /* tiling as in pt_batch_opts (0 = choose) */
    int32_t replicas_per_thread;
    int32_t pipeline;            /* 1: enqueue each round before retiring the requests
                                    the previous one finished (the device does not wait
                                    for the host between rounds; a new request joins one
                                    round later); 0: one round at a time */
} pt_serve_opts;

typedef struct {
    int32_t problem;             /* id from pt_serve_register */
    int32_t has_target;
    int32_t target;              /* done when min_r E_r <= target */
    int32_t pad;
    uint64_t seed;               /* Philox key of this request's chain */
    uint64_t sweep_cap;          /* done after this many sweeps in any case (>= 1) */
    int8_t *best_out;            /* host [n] or NULL: receives the best configuration
                                    before the result is published; caller-owned,
                                    must stay valid until the result is polled */
    uint64_t user_tag;
} pt_request;

typedef struct {
    uint64_t id;                 /* from pt_serve_submit */
    uint64_t user_tag;
    int32_t status;              /* PT_OK, or the PT_E* code that rejected it */
    int32_t hit;                 /* 1 if the target was reached */
    int64_t first_hit;           /* sweep of the first hit, or -1 */
    int32_t best_energy;
    int32_t best_slot;
    int64_t best_t;
    uint64_t sweeps;             /* sweeps run */
    double t_submit, t_admit, t_done;  /* seconds on the server clock (pt_serve_clock) */
} pt_result;

typedef struct {
    uint64_t submitted, admitted, completed, rejected;
    uint64_t rounds;
    double busy_s;               /* wall time of the rounds (launch to results) */
    double attempts;             /* spin-flip attempts run for requests */
    int32_t active, waiting, peak_active;
    int32_t peak_lanes;          /* most launches in one round */
    uint64_t mem_used, mem_peak;
    double gpu_busy_s;           /* device time of the rounds' sweep launches (HIP events) */
} pt_serve_stats;

int pt_serve_start(const pt_serve_opts *o, pt_server **out);
/* Register a problem: the server keeps a pointer to ctx (it must outlive the
 * server and not be used by the caller while the server runs). Its banks,
 * ladder and options (rule, sweeps_per_cycle, proposal schedule) apply to
 * every request on it. */
int pt_serve_register(pt_server *s, pt_ctx *ctx, int32_t *problem);
/* Queue a request (thread-safe; copies *rq). */
int pt_serve_submit(pt_server *s, const pt_request *rq, uint64_t *id);
/* Move up to max finished results into out; wait up to wait_ms for the
 * first one (0 = do not wait). *n_out receives the count. */
int pt_serve_poll(pt_server *s, pt_result *out, int32_t max, int32_t wait_ms, int32_t *n_out);
int pt_serve_stats_get(pt_server *s, pt_serve_stats *st);
/* Seconds since the server started (the clock of pt_result). */
double pt_serve_clock(pt_server *s);
/* Finish every queued and running request, then stop the worker and free
 * the server. Results not polled are dropped. */
int pt_serve_stop(pt_server *s);

/* ---- measurement ----
 * LDS read bandwidth of the current device in TB/s (the measured peak beside
 * the nominal one in the LDS roofline): blocks_per_cu x CUs workgroups of 256
 * threads, each reading its 32 KiB of LDS with unrolled, conflict-free
 * bytes_per_read (8 or 16) byte reads for iters rounds of 16 reads per lane;
 * the second of two timed launches counts. *ms (may be NULL) receives its
 * duration. blocks_per_cu in 1..8. Allocates and frees a small output
 * buffer. */
int pt_probe_lds(int32_t bytes_per_read, int32_t blocks_per_cu, uint32_t iters, double *tbps, double *ms);
/* VALU issue rate of one instruction (op 0: v_xor_b32, 1: v_mul_hi_u32,
 * 2: v_mul_lo_u32, 3: v_mad_u64_u32) in wave-instructions per clock per CU,
 * from 4 (op 3) or 8 independent
 * chains per lane, eight waves per SIMD; the clock is the device's
 * reported peak. A full-rate 32-bit operation issues 1 per clock per CU (4
 * SIMDs, 4 clocks per wave64 instruction). */
int pt_probe_valu(int32_t op, uint32_t iters, double *instr_per_clk_per_cu, double *ms);

const char *pt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TAPT_H */
