/*
 * CPU oracle for the TAPT hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded implementation of Transformer-Augmented
 * Parallel Tempering (arXiv:2509.23043, Algorithm 1) over a general sparse
 * Ising problem. It exists to check the HIP path bit for bit. Only the tests,
 * the smoke check and the benchmark's CPU-baseline leg may load it; the
 * product library never links or calls it. It shares no code with the HIP
 * path: the Philox generator, the FP64 acceptance thresholds and the energy
 * function are all written out again here.
 *
 * Conventions (each cited where it is used):
 *   spins m_i in {-1,+1}; E(m) = -sum_{i<j} J_ij m_i m_j - sum_i h_i m_i
 *   (Supp. S4, energy convention); local field I_i = sum_j J_ij m_j + h_i
 *   (Methods, Eq. 4).
 *
 * Random-number contract (shared definition, two independent implementations):
 *   Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key = (lo32, hi32) of
 *   the run seed, counter = (c0, c1, c2, c3) with c3 a stream tag:
 *     INIT   (1): spin i of slot r at start:  word (i&3) of ctr (i>>2, 0, r, 1);
 *                 m = +1 iff word >= 2^31.
 *     SWEEP  (2): attempt on site i of slot r in sweep t (1-based):
 *                 16-bit half (i&7) of ctr (i>>3, t, r, 2)   -> high half of u;
 *     REFINE (3): same half of ctr (i>>3, t, r, 3)            -> low half of u.
 *                 Half k of the 4 output words is word k>>1, bits 16*(k&1)...
 *     PROPOSE(4): proposal at cycle n on slot r: word 0 of ctr (r, n, 0, 4).
 *     SWAP   (5): swap at cycle n of pair (r, r+1): word 0 of ctr (r, n, 0, 5).
 *     BANK   (6): start cursor of a B-entry bank on slot r:
 *                 word 0 of ctr (r, 0, 0, 6) mod B.
 *     CONTEXT(7): contextual proposal at cycle n on slot r: the key of site i
 *                 is word (i&3) of ctr (i>>2, n, r, 7); the context is the
 *                 round(f n_free) free sites of smallest (key, index).
 *     CTXSWEEP(8): attempt on site i in completion sweep j (1-based) of that
 *                 proposal: u = word (i&3) of ctr (i>>2, n, r + 65536 j, 8).
 *   An event with probability p is accepted iff T(p) == 0xFFFFFFFF or u < T(p),
 *   T(p) = 0xFFFFFFFF for p >= 1, else min(floor(p * 2^32), 0xFFFFFFFF).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define TAG_INIT 1u
#define TAG_SWEEP 2u
#define TAG_REFINE 3u
#define TAG_PROPOSE 4u
#define TAG_SWAP 5u
#define TAG_BANK 6u
#define TAG_CONTEXT 7u
#define TAG_CTXSWEEP 8u

#define RULE_METROPOLIS 0
#define RULE_GIBBS 1

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 as published: each round multiplies counter words 0 and 2 by
 * the two round multipliers, mixes the high products with the other counter
 * words and the key, and the key advances by the Weyl constants between
 * rounds. */

void orc_philox(const uint32_t ctr[4], uint64_t seed, uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int round = 0; round < 10; ++round) {
        uint64_t a = (uint64_t)0xD2511F53u * x0;
        uint64_t b = (uint64_t)0xCD9E8D57u * x2;
        uint32_t y0 = (uint32_t)(b >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)b;
        uint32_t y2 = (uint32_t)(a >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)a;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static uint32_t philox_word(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                            uint64_t seed, int word)
{
    uint32_t ctr[4] = {c0, c1, c2, c3}, out[4];
    orc_philox(ctr, seed, out);
    return out[word];
}

static uint32_t philox_half(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                            uint64_t seed, int half)
{
    uint32_t w = philox_word(c0, c1, c2, c3, seed, half >> 1);
    return (half & 1) ? (w >> 16) : (w & 0xFFFFu);
}

/* the 32-bit uniform of one single-spin attempt */
uint32_t orc_sweep_uniform(uint64_t seed, uint32_t site, uint32_t t, uint32_t slot)
{
    uint32_t hi = philox_half(site >> 3, t, slot, TAG_SWEEP, seed, (int)(site & 7));
    uint32_t lo = philox_half(site >> 3, t, slot, TAG_REFINE, seed, (int)(site & 7));
    return (hi << 16) | lo;
}

/* ------------------------------------------------------------------------ */
/* Probability -> 32-bit threshold, and the acceptance test. */

uint32_t orc_threshold(double p)
{
    if (p >= 1.0) return 0xFFFFFFFFu;
    if (!(p > 0.0)) return 0u;
    double x = floor(ldexp(p, 32));
    if (x >= 4294967295.0) return 0xFFFFFFFFu;
    return (uint32_t)x;
}

static int accept(uint32_t T, uint32_t u) { return T == 0xFFFFFFFFu || u < T; }

/* Single-spin flip probability for an energy change dE = 2 m_i I_i.
 * Metropolis: min(1, exp(-beta dE)).
 * Gibbs (heat bath, Methods Eq. 5): the new spin is +1 with probability
 * (1 + tanh(beta I))/2 whatever the old one, so the flip probability is
 * 1/(1 + exp(beta dE)). */
double orc_flip_prob(int rule, double beta, int64_t dE)
{
    if (rule == RULE_GIBBS) return 1.0 / (1.0 + exp(beta * (double)dE));
    if (dE <= 0) return 1.0;
    return exp(-(beta * (double)dE));
}

/* ------------------------------------------------------------------------ */
/* Problem and state */

typedef struct {
    int32_t n;
    const int32_t *row_ptr; /* [n+1] */
    const int32_t *col;     /* [nnz], both directions */
    const int32_t *J;       /* [nnz] */
    const int32_t *h;       /* [n] */
    const int8_t *clamp;    /* [n]: 0 free, +-1 fixed */
    const int32_t *color;   /* [n] proper coloring, colors 0..ncolors-1 */
    int32_t ncolors;
    int32_t R;
    const double *beta;     /* [R] strictly increasing: slot 0 hottest (any
                               positive values when M == 0) */
    int32_t rule;           /* RULE_METROPOLIS | RULE_GIBBS */
    int32_t M;              /* sweeps per cycle (between swap stages); 0: the
                               slots are independent chains with no cycle end
                               (the bank-generation runs of Supp. Table S3) */
    int64_t prop_start, prop_period, prop_stop; /* proposal schedule, sweeps */
    uint64_t seed;
    const int8_t *const *bank; /* [R]: NULL or [bank_n[r]][n] configurations */
    const int32_t *bank_n;     /* [R] */
    int32_t has_target;
    int64_t target;
    int32_t check_energy;   /* 1: compare incremental and recomputed energies */
    /* contextual proposals (Supp. context ablation): when ctx_fraction or
     * ctx_sweeps is nonzero, a proposal starts from its bank entry, takes the
     * slot's current spins on the context sites -- a random choice of
     * round(ctx_fraction * n_free) of the free sites -- and completes the
     * other free sites by ctx_sweeps MCMC sweeps at the slot's beta
     * (1..65535, or 0 for none) */
    double ctx_fraction;
    int32_t ctx_sweeps;
} orc_problem;

typedef struct {
    uint64_t t;             /* completed sweeps */
    int8_t *spins;          /* [R][n] in slot order */
    int64_t *E;             /* [R] */
    int32_t *cursor;        /* [R] next bank entry per slot */
    int64_t best;           /* lowest min_r E_r seen */
    int64_t best_t;         /* sweep at which best was first reached */
    int32_t best_slot;      /* lowest slot holding best at best_t */
    int8_t *best_spins;     /* [n] that configuration */
    int64_t first_hit;      /* first sweep with min_r E_r <= target, -1 none */
    uint64_t *swap_att, *swap_acc;  /* [R-1] per pair (r, r+1) */
    uint64_t *prop_att, *prop_acc;  /* [R] */
    uint64_t *flips;                /* [R] accepted single-spin flips */
    int64_t energy_mismatch;        /* number of failed energy checks */
} orc_state;

/* E(m) = -sum_{i<j} J_ij m_i m_j - sum_i h_i m_i (Supp. S4). Each undirected
 * bond is stored twice in the CSR, so the pair sum counts i<j via col > i. */
int64_t orc_energy(const orc_problem *P, const int8_t *m)
{
    int64_t e = 0;
    for (int32_t i = 0; i < P->n; ++i) {
        for (int32_t k = P->row_ptr[i]; k < P->row_ptr[i + 1]; ++k) {
            int32_t j = P->col[k];
            if (j > i) e -= (int64_t)P->J[k] * m[i] * m[j];
        }
        e -= (int64_t)P->h[i] * m[i];
    }
    return e;
}

/* I_i = sum_j J_ij m_j + h_i (Methods, Eq. 4) */
static int64_t local_field(const orc_problem *P, const int8_t *m, int32_t i)
{
    int64_t I = P->h[i];
    for (int32_t k = P->row_ptr[i]; k < P->row_ptr[i + 1]; ++k)
        I += (int64_t)P->J[k] * m[P->col[k]];
    return I;
}

static int32_t bank_start(const orc_problem *P, int32_t r)
{
    return (int32_t)(philox_word((uint32_t)r, 0, 0, TAG_BANK, P->seed, 0) % (uint32_t)P->bank_n[r]);
}

static void track_best(const orc_problem *P, orc_state *S)
{
    int64_t lo = S->E[0];
    int32_t arg = 0;
    for (int32_t r = 1; r < P->R; ++r)
        if (S->E[r] < lo) { lo = S->E[r]; arg = r; }
    if (lo < S->best) {
        S->best = lo;
        S->best_t = (int64_t)S->t;
        S->best_slot = arg;
        memcpy(S->best_spins, S->spins + (size_t)arg * P->n, (size_t)P->n);
    }
    if (P->has_target && S->first_hit < 0 && lo <= P->target) S->first_hit = (int64_t)S->t;
}

/* Random initial replica states (Algorithm 1, initialisation step). Clamped spins
 * take their clamp value. Counters and bank cursors start here too. */
int orc_init(const orc_problem *P, orc_state *S)
{
    int32_t n = P->n;
    for (int32_t r = 0; r < P->R; ++r) {
        int8_t *m = S->spins + (size_t)r * n;
        for (int32_t i = 0; i < n; ++i) {
            if (P->clamp[i]) {
                m[i] = P->clamp[i];
            } else {
                uint32_t w = philox_word((uint32_t)i >> 2, 0, (uint32_t)r, TAG_INIT, P->seed, i & 3);
                m[i] = (w >= 0x80000000u) ? 1 : -1;
            }
        }
        S->E[r] = orc_energy(P, m);
        S->cursor[r] = (P->bank && P->bank[r] && P->bank_n[r] > 0) ? bank_start(P, r) : 0;
        S->prop_att[r] = S->prop_acc[r] = S->flips[r] = 0;
        if (r + 1 < P->R) S->swap_att[r] = S->swap_acc[r] = 0;
    }
    S->t = 0;
    S->best = INT64_MAX;
    S->best_t = -1;
    S->best_slot = -1;
    S->first_hit = -1;
    S->energy_mismatch = 0;
    track_best(P, S);
    return 0;
}

/* One Monte Carlo sweep of slot r at beta_r: every free spin once, color
 * classes in increasing color, sites of a class in increasing index
 * (Methods, Graph coloring: a class holds no neighbours, so this order gives
 * the same result as updating a class in parallel). */
static void sweep_slot(const orc_problem *P, orc_state *S, int32_t r, uint32_t t)
{
    int8_t *m = S->spins + (size_t)r * P->n;
    for (int32_t c = 0; c < P->ncolors; ++c) {
        for (int32_t i = 0; i < P->n; ++i) {
            if (P->color[i] != c || P->clamp[i]) continue;
            int64_t I = local_field(P, m, i);
            int64_t dE = 2 * (int64_t)m[i] * I; /* E(flipped) - E(current) */
            uint32_t T = orc_threshold(orc_flip_prob(P->rule, P->beta[r], dE));
            uint32_t u = orc_sweep_uniform(P->seed, (uint32_t)i, t, (uint32_t)r);
            if (accept(T, u)) {
                m[i] = (int8_t)-m[i];
                S->E[r] += dE;
                S->flips[r] += 1;
            }
        }
    }
}

/* Number of context sites: the fraction f of the free spins, rounded to the
 * nearest count (halves up). */
static int32_t context_count(const orc_problem *P)
{
    int32_t nfree = 0;
    for (int32_t i = 0; i < P->n; ++i) nfree += P->clamp[i] ? 0 : 1;
    return (int32_t)floor(P->ctx_fraction * (double)nfree + 0.5);
}

typedef struct {
    uint32_t key;
    int32_t site;
} ctx_key;

static int ctx_key_order(const void *a, const void *b)
{
    const ctx_key *x = (const ctx_key *)a, *y = (const ctx_key *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->site < y->site ? -1 : (x->site > y->site ? 1 : 0);
}

/* Contextual proposal of slot r at cycle cyc (Supp. context ablation): a
 * randomly chosen fraction of the spins is clamped to the slot's current
 * values and the remaining spins are generated by MCMC under those clamps.
 * The context is the K = round(f n_free) free sites whose CONTEXT keys
 * (word i&3 of Philox ctr (i>>2, cyc, r, 7)) are smallest, ties going to the
 * lower index: with independent uniform keys, a uniformly random K-subset.
 * The generation starts from the bank entry (a sample of the unconstrained
 * long-run MCMC at beta_r) and runs ctx_sweeps sweeps at beta_r with the
 * run's rule, color classes in increasing color and sites in increasing
 * index, as in sweep_slot. ctx_mask[i] = 1 marks the context sites. */
void orc_context_candidate(const orc_problem *P, int32_t r, uint32_t cyc, const int8_t *start,
                           const int8_t *current, int8_t *out, uint8_t *ctx_mask)
{
    const int32_t n = P->n;
    ctx_key *keys = (ctx_key *)malloc(sizeof(ctx_key) * (size_t)(n > 0 ? n : 1));
    int32_t nfree = 0;
    for (int32_t i = 0; i < n; ++i) {
        ctx_mask[i] = 0;
        if (P->clamp[i]) continue;
        keys[nfree].key = philox_word((uint32_t)i >> 2, cyc, (uint32_t)r, TAG_CONTEXT, P->seed, i & 3);
        keys[nfree].site = i;
        ++nfree;
    }
    qsort(keys, (size_t)nfree, sizeof(ctx_key), ctx_key_order);
    const int32_t K = context_count(P);
    for (int32_t k = 0; k < K && k < nfree; ++k) ctx_mask[keys[k].site] = 1;
    free(keys);
    for (int32_t i = 0; i < n; ++i) out[i] = ctx_mask[i] ? current[i] : start[i];
    for (int32_t j = 1; j <= P->ctx_sweeps; ++j) {
        for (int32_t c = 0; c < P->ncolors; ++c) {
            for (int32_t i = 0; i < n; ++i) {
                if (P->color[i] != c || P->clamp[i] || ctx_mask[i]) continue;
                int64_t dE = 2 * (int64_t)out[i] * local_field(P, out, i);
                uint32_t T = orc_threshold(orc_flip_prob(P->rule, P->beta[r], dE));
                uint32_t u = philox_word((uint32_t)i >> 2, cyc, (uint32_t)r + 65536u * (uint32_t)j, TAG_CTXSWEEP,
                                         P->seed, i & 3);
                if (accept(T, u)) out[i] = (int8_t)-out[i];
            }
        }
    }
}

static int is_proposal_sweep(const orc_problem *P, uint64_t t)
{
    if (P->prop_period <= 0 || !P->bank) return 0;
    if ((int64_t)t < P->prop_start) return 0;
    if (P->prop_stop >= 0 && (int64_t)t > P->prop_stop) return 0;
    return (((int64_t)t - P->prop_start) % P->prop_period) == 0;
}

/* Run n_sweeps more sweeps of Algorithm 1. The state must come from orc_init
 * or an earlier orc_run. */
int orc_run(const orc_problem *P, orc_state *S, uint64_t n_sweeps)
{
    int32_t n = P->n, R = P->R;
    int8_t *tmp = (int8_t *)malloc((size_t)n);
    int8_t *cand = (int8_t *)malloc((size_t)n);
    uint8_t *mask = (uint8_t *)malloc((size_t)n);
    const int contextual = P->ctx_fraction > 0.0 || P->ctx_sweeps != 0;
    if (!tmp || !cand || !mask) {
        free(tmp);
        free(cand);
        free(mask);
        return -1;
    }
    for (uint64_t step = 0; step < n_sweeps; ++step) {
        uint64_t t = S->t + 1;
        /* local MCMC sweeps: every replica, one sweep each */
        for (int32_t r = 0; r < R; ++r) sweep_slot(P, S, r, (uint32_t)t);
        S->t = t;
        if (P->M > 0 && t % (uint64_t)P->M == 0) {
            uint64_t cyc = t / (uint64_t)P->M; /* cycle n of Algorithm 1, 1-based */
            /* energies of all replicas (Algorithm 1, cycle-end energy step) */
            for (int32_t r = 0; r < R; ++r) {
                int64_t e = orc_energy(P, S->spins + (size_t)r * n);
                if (P->check_energy && e != S->E[r]) S->energy_mismatch++;
                S->E[r] = e;
            }
            /* proposals on the proposal-enabled slots, hottest first:
             * P_accept = min[1, exp(beta_r (E_r - E_r^T))]  (Eq. 2) */
            if (is_proposal_sweep(P, t)) {
                for (int32_t r = 0; r < R; ++r) {
                    if (!P->bank[r] || P->bank_n[r] <= 0) continue;
                    int32_t k = S->cursor[r];
                    S->cursor[r] = (k + 1) % P->bank_n[r];
                    const int8_t *prop = P->bank[r] + (size_t)k * n;
                    if (contextual) {
                        orc_context_candidate(P, r, (uint32_t)cyc, prop, S->spins + (size_t)r * n, cand, mask);
                        prop = cand;
                    }
                    int64_t ET = orc_energy(P, prop);
                    int64_t d = ET - S->E[r];
                    double p = (d <= 0) ? 1.0 : exp(-(P->beta[r] * (double)d));
                    uint32_t u = philox_word((uint32_t)r, (uint32_t)cyc, 0, TAG_PROPOSE, P->seed, 0);
                    S->prop_att[r]++;
                    if (accept(orc_threshold(p), u)) {
                        memcpy(S->spins + (size_t)r * n, prop, (size_t)n);
                        S->E[r] = ET;
                        S->prop_acc[r]++;
                    }
                }
            }
            /* replica exchange: odd n swaps pairs (1,2),(3,4),... of the
             * paper's 1-based ladder, even n swaps (2,3),(4,5),...;
             * P_swap = min[1, exp((beta_{r+1} - beta_r)(E_{r+1} - E_r))] (Eq. 1) */
            int32_t first = (cyc % 2 == 1) ? 0 : 1;
            for (int32_t r = first; r + 1 < R; r += 2) {
                int64_t dE = S->E[r + 1] - S->E[r];
                double db = P->beta[r + 1] - P->beta[r];
                double p = (dE >= 0) ? 1.0 : exp(-(db * (double)(-dE)));
                uint32_t u = philox_word((uint32_t)r, (uint32_t)cyc, 0, TAG_SWAP, P->seed, 0);
                S->swap_att[r]++;
                if (accept(orc_threshold(p), u)) {
                    int8_t *a = S->spins + (size_t)r * n, *b = S->spins + (size_t)(r + 1) * n;
                    memcpy(tmp, a, (size_t)n);
                    memcpy(a, b, (size_t)n);
                    memcpy(b, tmp, (size_t)n);
                    int64_t e = S->E[r];
                    S->E[r] = S->E[r + 1];
                    S->E[r + 1] = e;
                    S->swap_acc[r]++;
                }
            }
        }
        track_best(P, S);
    }
    free(tmp);
    free(cand);
    free(mask);
    return 0;
}

/* Threshold tables as the oracle would use them, for cross-checks in tests. */
void orc_flip_table(int32_t rule, double beta, int32_t dmax, uint32_t *out /*[2*dmax+1]*/)
{
    for (int32_t d = -dmax; d <= dmax; ++d)
        out[d + dmax] = orc_threshold(orc_flip_prob(rule, beta, 2 * (int64_t)d));
}

/* Run n_sweeps sweeps and, after every ``thin``-th sweep, count the state of
 * each slot in hist[r][state] where state = sum_i [m_i = +1] 2^i (n <= 20).
 * Used by the distribution tests only. */
int orc_run_sampled(const orc_problem *P, orc_state *S, uint64_t n_sweeps,
                    uint64_t thin, uint64_t *hist)
{
    if (P->n > 20 || thin == 0) return -2;
    size_t ns = (size_t)1 << P->n;
    for (uint64_t k = 0; k < n_sweeps; ++k) {
        int rc = orc_run(P, S, 1);
        if (rc) return rc;
        if (S->t % thin) continue;
        for (int32_t r = 0; r < P->R; ++r) {
            const int8_t *m = S->spins + (size_t)r * P->n;
            size_t idx = 0;
            for (int32_t i = 0; i < P->n; ++i)
                if (m[i] > 0) idx |= (size_t)1 << i;
            hist[(size_t)r * ns + idx]++;
        }
    }
    return 0;
}
