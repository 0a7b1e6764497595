// Host runtime of libtapt: the C ABI declared in include/tapt.h.
//
// pt_create validates and copies a problem, builds the uint32 acceptance
// tables in FP64 (Eqs. 1, 2 and the single-spin rule of Methods Eq. 5 or its
// Metropolis counterpart), uploads everything and initialises the replicas
// on the device. pt_sweep is the plain path (per-sweep launches of one
// context). pt_batch_* run many contexts in persistent chunk launches whose
// workgroups each own a contiguous range of beta slots of one instance.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <set>
#include <tuple>
#include <string>
#include <vector>

#include "tapt.h"
#include "tapt_dev.h"

namespace tapt {
bool lattice_supported(int L);
int lattice_max_threads();
int lattice_threads(int L, int G, int rpt);
size_t chunk_lds_bytes(int kind, int n, int G, int stride, int tsw_entries, int nnz, int nfree, int ncolors,
                       bool contextual, int sparse, size_t row_graph);
hipError_t launch_chunk(int kind, int L, int rpt, int sparse, const ChunkArgs &a, int block, size_t lds, hipStream_t s);
hipError_t chunk_occupancy(int kind, int L, int rpt, int sparse, int block, size_t lds, int *blocks_per_cu);
hipError_t launch_chunk_ctx(int kind, int L, const ChunkArgs &a, int block, size_t lds, hipStream_t s);
hipError_t chunk_occupancy_ctx(int kind, int L, int block, size_t lds, int *blocks_per_cu);
hipError_t launch_finish(const WorkItem *items, const int *first_item, int n_inst, uint32_t K, InstStatus *status,
                         hipStream_t s);
int mixed_max_threads();
int mixed_variant_of(int kind, int L, int rpt);
hipError_t launch_chunk_mixed(const ChunkArgs &a, int block, size_t lds, hipStream_t s);
hipError_t chunk_occupancy_mixed(int block, size_t lds, int *blocks_per_cu);
bool wave_supported(int L);
int wave_max_storages();
size_t wave_lds_bytes(int n, int G, int stride, int tsw_entries);
hipError_t launch_wave(int L, const ChunkArgs &a, int block, size_t lds, hipStream_t s);
hipError_t wave_occupancy(int L, int block, size_t lds, int *blocks_per_cu);
int pm_max_storages(int spw);
size_t pm_lds_bytes(int G, int tsw_entries);
hipError_t launch_pm(int spw, const ChunkArgs &a, int block, size_t lds, hipStream_t s);
hipError_t pm_occupancy(int spw, int block, size_t lds, int *blocks_per_cu);
bool pml_supported(int L);
int pml_max_storages();
size_t pml_lds_bytes(int L, int G, int tsw_entries);
int pml_xwords(int L);
hipError_t launch_pml(const ChunkArgs &a, int block, size_t lds, hipStream_t s);
hipError_t pml_occupancy(int block, size_t lds, int *blocks_per_cu);
int csrw_max_storages();
bool csrw_supported(int n, int maxabsj, int chunks, int maxcnt);
size_t csrw_lds_bytes(int n, int ncolors, int maxcnt, int chunks, int G, int stride, int tsw_entries);
int csrw_xwords(int n);
hipError_t launch_csrw(const ChunkArgs &a, int block, size_t lds, hipStream_t s);
hipError_t csrw_occupancy(int block, size_t lds, int *blocks_per_cu);
hipError_t launch_plain(int kind, int L, const InstDev *dI, int R, int n, int stride, int nnz, int nfree, int ncolors,
                        uint32_t t, hipStream_t s);
hipError_t launch_init(const InstDev *dI, int R, int n, hipStream_t s);
hipError_t launch_energy(const InstDev *dI, const int8_t *cfg, int k, int32_t *out, hipStream_t s);
hipError_t launch_init_best(const InstDev *dI, hipStream_t s);
hipError_t launch_set_caps(InstDev *const *insts, const unsigned long long *caps, int n, hipStream_t s);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t s);
uint32_t host_philox_word0(uint32_t c0, uint32_t c1, uint32_t c3, uint32_t k0, uint32_t k1);
} // namespace tapt

using namespace tapt;

// ---------------------------------------------------------------------------
// errors

static thread_local std::string g_err;

static int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                                 \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) return fail(PT_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));       \
    } while (0)

extern "C" const char *pt_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// acceptance thresholds: accept iff T == 0xFFFFFFFF or u < T for a uniform
// u32 u; T(p) = 0xFFFFFFFF for p >= 1, else min(floor(p 2^32), 0xFFFFFFFF).

static uint32_t threshold(double p)
{
    if (p >= 1.0) return ALWAYS;
    if (!(p > 0.0)) return 0u;
    double x = std::floor(std::ldexp(p, 32));
    if (x >= 4294967295.0) return ALWAYS;
    return (uint32_t)x;
}

// probability of flipping a spin whose flip changes the energy by dE
static double flip_probability(int rule, double beta, long long dE)
{
    if (rule == PT_GIBBS) return 1.0 / (1.0 + std::exp(beta * (double)dE));
    if (dE <= 0) return 1.0;
    return std::exp(-(beta * (double)dE));
}

// Longest single proposal or swap table, and the most entries all of a
// context's tables may hold together. A table is never truncated: a cut
// table would reject moves whose probability is not zero.
static const size_t TAIL_TABLE_MAX = (size_t)1 << 22;
static const size_t TAIL_TABLES_TOTAL_MAX = (size_t)1 << 26;

// Appends the entries T(exp(-a d)) for d = 1, 2, ... up to the last nonzero
// one. Returns false, leaving `out` as it was, if that table would be longer
// than TAIL_TABLE_MAX or push `out` past TAIL_TABLES_TOTAL_MAX.
static bool tail_table(double a, std::vector<uint32_t> &out)
{
    const size_t start = out.size();
    for (long long d = 1;; ++d) {
        uint32_t T = threshold(std::exp(-(a * (double)d)));
        if (T == 0) return true;
        if (out.size() - start >= TAIL_TABLE_MAX || out.size() >= TAIL_TABLES_TOTAL_MAX) {
            out.resize(start);
            return false;
        }
        out.push_back(T);
    }
}

// ---------------------------------------------------------------------------
// device buffer helper

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    bool owned = true;                // false: a view of memory owned elsewhere
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes), owned(o.owned)
    {
        o.p = nullptr;
        o.bytes = 0;
        o.owned = true;
    }
    ~DevBuf() { release(); }
    void release()
    {
        if (p && owned) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        owned = true;
    }
    hipError_t alloc(size_t b)
    {
        release();
        bytes = b;
        return hipMalloc(&p, b ? b : 16);
    }
    void view(void *q, size_t b)
    {
        release();
        p = q;
        bytes = b;
        owned = false;
    }
    template <class T> T *as() const { return (T *)p; }
};

// Page-locked host memory (hipHostMalloc): the source or target of copies
// that run after the call that enqueued them has returned.
struct HostPinned {
    void *p = nullptr;
    size_t bytes = 0;
    HostPinned() = default;
    HostPinned(const HostPinned &) = delete;
    HostPinned &operator=(const HostPinned &) = delete;
    ~HostPinned()
    {
        if (p) (void)hipHostFree(p);
    }
    // at least b bytes (contents not kept when it grows)
    hipError_t reserve(size_t b)
    {
        if (b <= bytes) return hipSuccess;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
        hipError_t e = hipHostMalloc(&p, b, hipHostMallocDefault);
        if (e == hipSuccess) bytes = b;
        return e;
    }
    template <class T> T *as() const { return (T *)p; }
};

struct Bank {
    DevBuf cfg, E;
    int32_t n = 0;
};

struct pt_ctx {
    // problem (host copies)
    int32_t n = 0, L = 0, R = 0, kind = KIND_CSR, D = 0, ncolors = 0;
    std::vector<double> betas;
    std::vector<int32_t> h_tswap_len; // host copy: swap-table length per pair
    pt_opts opts{};
    std::vector<int8_t> clamp;
    int64_t nfree = 0;
    uint64_t problem_fp = 0;          // FNV-1a of the problem, ladder, options and seed

    // device allocations
    DevBuf J3, row_ptr, col, Jc, h, clampd, color_sites, color_off, csrw_grp;
    DevBuf tflip, tprop, tprop_off, tprop_len, tswap, tswap_off, tswap_len;
    DevBuf spins, E, t, cursor, bank_ptrs, bankE_ptrs, bank_n;
    DevBuf swap_att, swap_acc, prop_att, prop_acc, flips, best, best_spins;
    DevBuf inst;                      // device InstDev
    InstDev hI{};                     // host mirror of the device InstDev
    std::vector<Bank> banks;          // per slot
    std::vector<const int8_t *> h_bank_ptrs;
    std::vector<const int32_t *> h_bankE_ptrs;
    std::vector<int32_t> h_bank_n;

    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool broken = false;
    uint64_t t_host = 0;
    int device = 0;
    bool pmJ = false;                 // 8^3 lattice with every coupling +-1 (the +-J kernel applies)
    bool pmL = false;                 // even L in 6..16, every coupling +-1 (the +-J row kernel applies)
    DevBuf arena;                     // a served request's state, carved into the views above
    std::vector<int32_t> h_cursor0;   // a served request's start cursors (source of an async copy)
};

static int push_inst(pt_ctx *c)
{
    HIPCHK(hipMemcpyAsync(c->inst.p, &c->hI, sizeof(InstDev), hipMemcpyHostToDevice, c->stream));
    return PT_OK;
}

// Independent chains (sweeps_per_cycle 0) run with a cycle this long, so
// that no cycle ends within the sweeps such a context may run.
constexpr int32_t INDEPENDENT_M = 0x7FFFFFFF;

// Largest sweep counter a context may reach.
static uint64_t sweep_limit(const pt_ctx *c)
{
    return c->opts.sweeps_per_cycle == 0 ? (uint64_t)INDEPENDENT_M - 1 : 0xFFFFFFFFull;
}

// Proposals of this context are contextual (built on the device from the
// bank entry and the slot's current state) rather than plain bank entries.
static bool contextual(const pt_ctx *c) { return c->hI.ctx_on != 0; }

static int check_ctx(pt_ctx *c)
{
    if (!c) return fail(PT_EINVAL, "null context");
    if (c->broken) return fail(PT_ESTATE, "context is unusable after a device error");
    HIPCHK(hipSetDevice(c->device));
    return PT_OK;
}

template <class T>
static hipError_t upload(DevBuf &b, const std::vector<T> &v, hipStream_t s)
{
    hipError_t e = b.alloc(v.size() * sizeof(T));
    if (e != hipSuccess || v.empty()) return e;
    return hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

// ---------------------------------------------------------------------------
// problem validation and preparation

// 64-bit FNV-1a, used to fingerprint a context for its checkpoints
struct Fnv {
    uint64_t h = 1469598103934665603ull;
    void add(const void *p, size_t bytes)
    {
        const unsigned char *b = (const unsigned char *)p;
        for (size_t k = 0; k < bytes; ++k) h = (h ^ b[k]) * 1099511628211ull;
    }
    template <class T> void add(const std::vector<T> &v)
    {
        uint64_t k = v.size();
        add(&k, sizeof k);
        if (!v.empty()) add(v.data(), v.size() * sizeof(T));
    }
    template <class T> void val(T x) { add(&x, sizeof x); }
};

struct Prepared {
    int kind, L, n, D, ncolors;
    std::vector<int8_t> J3;                 // lattice
    std::vector<int32_t> row_ptr;           // CSR over all sites
    std::vector<int16_t> col;
    std::vector<int8_t> Jc;
    std::vector<int16_t> h;
    std::vector<int8_t> clamp;
    std::vector<int16_t> color_sites;
    std::vector<int32_t> color_off;
    std::vector<int32_t> csrw_groups;       // rank groups of the one-slot-per-wavefront sparse kernel
    int csrw_chunks = 0;
    int64_t nfree;
    int maxdeg = 0, maxcnt = 0, maxabsj = 0;   // over free sites / colour classes / bonds
};

static int prepare(const pt_graph *g, Prepared &P)
{
    if (!g) return fail(PT_EINVAL, "null graph");
    const int n = g->n;
    if (n < 1 || n > 32768) return fail(PT_EINVAL, "n must be in 1..32768 (got %d)", n);
    P.n = n;
    P.h.assign(n, 0);
    P.clamp.assign(n, 0);
    if (g->h)
        for (int i = 0; i < n; ++i) {
            if (g->h[i] < -32767 || g->h[i] > 32767) return fail(PT_EINVAL, "|h[%d]| > 32767", i);
            P.h[i] = (int16_t)g->h[i];
        }
    if (g->clamp)
        for (int i = 0; i < n; ++i) {
            int v = g->clamp[i];
            if (v != 0 && v != 1 && v != -1) return fail(PT_EINVAL, "clamp[%d] must be 0 or +-1", i);
            P.clamp[i] = (int8_t)v;
        }
    std::vector<int32_t> color(n, 0);
    // adjacency (both directions) for validation, D and the CSR kernel
    std::vector<int32_t> rp(n + 1, 0);
    std::vector<int32_t> cl;
    std::vector<int32_t> jv;
    if (g->lattice_L > 0) {
        const int L = g->lattice_L;
        if (L < 4 || L % 2 || L > 32 || L * L * L != n)
            return fail(PT_EINVAL, "lattice needs even L in 4..32 with n = L^3 (L=%d, n=%d)", L, n);
        if (!g->J) return fail(PT_EINVAL, "lattice couplings J missing");
        P.L = L;
        P.J3.resize(3 * (size_t)n);
        for (size_t k = 0; k < 3 * (size_t)n; ++k) {
            if (g->J[k] < -127 || g->J[k] > 127) return fail(PT_EINVAL, "|J| > 127 at bond %zu", k);
            P.J3[k] = (int8_t)g->J[k];
        }
        for (int i = 0; i < n; ++i) {
            int x = i % L, y = (i / L) % L, z = i / (L * L);
            int nb[6] = {(x + 1) % L + L * (y + L * z), (x + L - 1) % L + L * (y + L * z),
                         x + L * ((y + 1) % L + L * z), x + L * ((y + L - 1) % L + L * z),
                         x + L * (y + L * ((z + 1) % L)), x + L * (y + L * ((z + L - 1) % L))};
            int jj[6] = {P.J3[i], P.J3[nb[1]], P.J3[n + i], P.J3[n + nb[3]], P.J3[2 * n + i], P.J3[2 * n + nb[5]]};
            for (int d = 0; d < 6; ++d) {
                cl.push_back(nb[d]);
                jv.push_back(jj[d]);
            }
            rp[i + 1] = (int32_t)cl.size();
            color[i] = (x + y + z) & 1;
        }
        bool plain = true;
        for (int i = 0; i < n; ++i)
            if (P.h[i] || P.clamp[i]) plain = false;
        P.kind = (plain && lattice_supported(L)) ? KIND_LATTICE : KIND_CSR;
    } else {
        P.L = 0;
        P.kind = KIND_CSR;
        if (!g->row_ptr || !g->col || !g->J) return fail(PT_EINVAL, "CSR arrays missing");
        if (g->row_ptr[0] != 0 || g->row_ptr[n] != g->nnz || g->nnz < 0)
            return fail(PT_EINVAL, "row_ptr must start at 0 and end at nnz");
        for (int i = 0; i < n; ++i) {
            if (g->row_ptr[i + 1] < g->row_ptr[i]) return fail(PT_EINVAL, "row_ptr not monotone at %d", i);
            for (int k = g->row_ptr[i]; k < g->row_ptr[i + 1]; ++k) {
                int j = g->col[k];
                if (j < 0 || j >= n) return fail(PT_EINVAL, "col[%d] out of range", k);
                if (j == i) return fail(PT_EINVAL, "self loop at site %d", i);
                if (g->J[k] < -127 || g->J[k] > 127) return fail(PT_EINVAL, "|J| > 127 at entry %d", k);
                cl.push_back(j);
                jv.push_back(g->J[k]);
            }
            rp[i + 1] = (int32_t)cl.size();
        }
        // symmetry: every (i, j, J) has its (j, i, J)
        std::map<std::pair<int, int>, long long> w;
        for (int i = 0; i < n; ++i)
            for (int k = rp[i]; k < rp[i + 1]; ++k) w[{i, cl[k]}] += jv[k];
        for (auto &kv : w) {
            auto it = w.find({kv.first.second, kv.first.first});
            if (it == w.end() || it->second != kv.second)
                return fail(PT_EINVAL, "couplings not symmetric at (%d, %d)", kv.first.first, kv.first.second);
        }
        if (!g->color) return fail(PT_EINVAL, "CSR graphs need a coloring");
        for (int i = 0; i < n; ++i) color[i] = g->color[i];
    }
    // coloring checks
    int nc = 0;
    for (int i = 0; i < n; ++i) {
        if (color[i] < 0 || color[i] >= MAX_COLORS) return fail(PT_EINVAL, "color[%d] out of 0..63", i);
        nc = std::max(nc, color[i] + 1);
    }
    for (int i = 0; i < n; ++i)
        for (int k = rp[i]; k < rp[i + 1]; ++k)
            if (color[cl[k]] == color[i]) return fail(PT_EINVAL, "coloring not proper at edge (%d, %d)", i, cl[k]);
    P.ncolors = nc;
    // flip-table half width: |m_i I_i| <= sum_j |J_ij| + |h_i| over free sites
    int D = 0;
    P.nfree = 0;
    for (int i = 0; i < n; ++i) {
        if (P.clamp[i]) continue;
        ++P.nfree;
        long long s = std::abs((long long)P.h[i]);
        for (int k = rp[i]; k < rp[i + 1]; ++k) s += std::abs((long long)jv[k]);
        if (s > 4096) return fail(PT_EUNSUPPORTED, "local field bound %lld at site %d exceeds 4096", s, i);
        D = std::max(D, (int)s);
    }
    P.D = D;
    for (int i = 0; i < n; ++i)
        if (!P.clamp[i]) P.maxdeg = std::max(P.maxdeg, rp[i + 1] - rp[i]);
    for (int v : jv) P.maxabsj = std::max(P.maxabsj, std::abs(v));
    P.row_ptr = rp;
    P.col.resize(cl.size());
    P.Jc.resize(jv.size());
    for (size_t k = 0; k < cl.size(); ++k) {
        P.col[k] = (int16_t)cl[k];
        P.Jc[k] = (int8_t)jv[k];
    }
    // the free sites of each colour, largest degree first (sites of one colour
    // share no bond, so their order within the class changes no result; this
    // one lets the one-slot-per-wavefront kernel give the few high-degree
    // sites their own rank groups)
    P.color_off.assign(nc + 1, 0);
    for (int c = 0; c < nc; ++c) {
        const size_t from = P.color_sites.size();
        for (int i = 0; i < n; ++i)
            if (color[i] == c && !P.clamp[i]) P.color_sites.push_back((int16_t)i);
        std::stable_sort(P.color_sites.begin() + from, P.color_sites.end(), [&](int16_t a, int16_t b) {
            return rp[a + 1] - rp[a] > rp[b + 1] - rp[b];
        });
        P.color_off[c + 1] = (int32_t)P.color_sites.size();
        P.maxcnt = std::max(P.maxcnt, P.color_off[c + 1] - P.color_off[c]);
    }
    // rank groups (c, k) of 64 sites: chunks of CSRW_CHUNK bonds for the
    // largest degree in the group, numbered in group order
    const int ipl = (P.maxcnt + 63) / 64;
    if (P.maxdeg <= CSRW_MAXDEG && P.maxcnt >= 1 && nc * ipl <= CSRW_MAXGROUPS) {
        int base = 0;
        for (int c = 0; c < nc; ++c)
            for (int k = 0; k < ipl; ++k) {
                int md = 1;
                for (int s = P.color_off[c] + 64 * k; s < std::min(P.color_off[c + 1], P.color_off[c] + 64 * k + 64); ++s)
                    md = std::max(md, rp[P.color_sites[s] + 1] - rp[P.color_sites[s]]);
                const int nch = (md + CSRW_CHUNK - 1) / CSRW_CHUNK;
                P.csrw_groups.push_back((base << 8) | nch);
                base += nch;
            }
        P.csrw_chunks = base;
    }
    if (P.color_sites.empty()) P.color_sites.push_back(0);
    return PT_OK;
}

static void fill_inst_pointers(pt_ctx *c)
{
    InstDev &I = c->hI;
    I.J3 = c->J3.as<int8_t>();
    I.row_ptr = c->row_ptr.as<int32_t>();
    I.col = c->col.as<int16_t>();
    I.Jc = c->Jc.as<int8_t>();
    I.h = c->h.as<int16_t>();
    I.clamp = c->clampd.as<int8_t>();
    I.color_sites = c->color_sites.as<int16_t>();
    I.color_off = c->color_off.as<int32_t>();
    I.csrw_groups = c->csrw_grp.as<int32_t>();
    I.tflip = c->tflip.as<uint32_t>();
    I.tprop = c->tprop.as<uint32_t>();
    I.tprop_off = c->tprop_off.as<int32_t>();
    I.tprop_len = c->tprop_len.as<int32_t>();
    I.tswap = c->tswap.as<uint32_t>();
    I.tswap_off = c->tswap_off.as<int32_t>();
    I.tswap_len = c->tswap_len.as<int32_t>();
    I.spins = c->spins.as<int8_t>();
    I.E = c->E.as<int32_t>();
    I.t = c->t.as<unsigned long long>();
    I.cursor = c->cursor.as<int32_t>();
    I.bank = c->bank_ptrs.as<const int8_t *>();
    I.bankE = c->bankE_ptrs.as<const int32_t *>();
    I.bank_n = c->bank_n.as<int32_t>();
    I.swap_att = c->swap_att.as<unsigned long long>();
    I.swap_acc = c->swap_acc.as<unsigned long long>();
    I.prop_att = c->prop_att.as<unsigned long long>();
    I.prop_acc = c->prop_acc.as<unsigned long long>();
    I.flips = c->flips.as<unsigned long long>();
    I.best = c->best.as<BestRec>();
    I.best_spins = c->best_spins.as<int8_t>();
}

// zero counters, initialise spins (or take them from `spins`), energies, best.
// sync = false (fresh spins at t = 0 only): everything is enqueued on the
// context's stream and nothing waits, so that a server can set up many
// requests at once; every host source then lives in the context.
static int reset_state(pt_ctx *c, const int8_t *spins, uint64_t t, bool sync = true)
{
    hipStream_t s = c->stream;
    const int R = c->R, n = c->n;
    if (!sync && (spins || t)) return fail(PT_EINVAL, "an unsynchronised reset starts fresh chains at t = 0");
    HIPCHK(hipMemsetAsync(c->swap_att.p, 0, c->swap_att.bytes, s));
    HIPCHK(hipMemsetAsync(c->swap_acc.p, 0, c->swap_acc.bytes, s));
    HIPCHK(hipMemsetAsync(c->prop_att.p, 0, c->prop_att.bytes, s));
    HIPCHK(hipMemsetAsync(c->prop_acc.p, 0, c->prop_acc.bytes, s));
    HIPCHK(hipMemsetAsync(c->flips.p, 0, c->flips.bytes, s));
    unsigned long long tt = t;
    if (sync) HIPCHK(hipMemcpyAsync(c->t.p, &tt, 8, hipMemcpyHostToDevice, s));
    else HIPCHK(hipMemsetAsync(c->t.p, 0, 8, s));
    c->hI.epoch += 1;
    int rc = push_inst(c);
    if (rc) return rc;
    if (spins)
        HIPCHK(hipMemcpyAsync(c->spins.p, spins, (size_t)R * n, hipMemcpyHostToDevice, s));
    else
        HIPCHK(launch_init(c->inst.as<InstDev>(), R, n, s));
    HIPCHK(launch_energy(c->inst.as<InstDev>(), c->spins.as<int8_t>(), R, c->E.as<int32_t>(), s));
    HIPCHK(launch_init_best(c->inst.as<InstDev>(), s));
    if (sync) HIPCHK(hipStreamSynchronize(s));
    c->t_host = t;
    return PT_OK;
}

extern "C" int pt_create(const pt_graph *g, const double *betas, int32_t R, const pt_opts *o, pt_ctx **out)
{
    if (!out) return fail(PT_EINVAL, "null output pointer");
    *out = nullptr;
    if (!betas || !o) return fail(PT_EINVAL, "null betas or options");
    if (R < 1 || R > 1024) return fail(PT_EINVAL, "R must be in 1..1024 (got %d)", R);
    // sweeps_per_cycle == 0: independent chains (no swap stage, no proposals),
    // where any positive betas are allowed, equal ones included
    const bool independent = o->sweeps_per_cycle == 0;
    for (int r = 0; r < R; ++r) {
        if (!(betas[r] > 0.0) || !std::isfinite(betas[r])) return fail(PT_EINVAL, "beta[%d] must be finite and > 0", r);
        if (!independent && r && !(betas[r] > betas[r - 1])) return fail(PT_EINVAL, "betas must be strictly increasing");
    }
    if (o->rule != PT_METROPOLIS && o->rule != PT_GIBBS) return fail(PT_EINVAL, "unknown rule %d", o->rule);
    if (o->sweeps_per_cycle < 0) return fail(PT_EINVAL, "sweeps_per_cycle must be >= 0");
    if (independent && o->prop_period != 0) return fail(PT_EINVAL, "independent chains (sweeps_per_cycle 0) take no proposals");
    if (o->prop_period < 0) return fail(PT_EINVAL, "prop_period must be >= 0");
    if (o->prop_period > 0) {
        if (o->prop_start < 0) return fail(PT_EINVAL, "prop_start must be >= 0");
        if (o->prop_start % o->sweeps_per_cycle || o->prop_period % o->sweeps_per_cycle)
            return fail(PT_EINVAL, "prop_start and prop_period must be multiples of sweeps_per_cycle");
    }
    Prepared P;
    int rc = prepare(g, P);
    if (rc) return rc;

    pt_ctx *c = new pt_ctx();
    c->n = P.n;
    c->L = P.L;
    c->R = R;
    c->kind = P.kind;
    c->D = P.D;
    c->ncolors = P.ncolors;
    c->betas.assign(betas, betas + R);
    c->opts = *o;
    c->clamp = P.clamp;
    c->nfree = P.nfree;
    {
        Fnv f;
        f.val(P.kind); f.val(P.L); f.val(P.n); f.val(P.D); f.val(P.ncolors);
        f.add(P.J3); f.add(P.row_ptr); f.add(P.col); f.add(P.Jc); f.add(P.h); f.add(P.clamp);
        f.add(P.color_sites); f.add(P.color_off); f.add(c->betas);
        f.val(o->rule); f.val(o->sweeps_per_cycle); f.val(o->prop_start); f.val(o->prop_period);
        f.val(o->prop_stop); f.val(o->seed); f.val(o->has_target); f.val(o->target);
        c->problem_fp = f.h;
    }
    c->pmJ = P.kind == KIND_LATTICE && P.L == 8 && P.D == 6 && R % 2 == 0;
    c->pmL = P.kind == KIND_LATTICE && pml_supported(P.L) && P.D == 6;
    for (int8_t j : P.J3)
        if (j != 1 && j != -1) c->pmJ = c->pmL = false;
    auto bail = [&](int code) {
        if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
        delete c;
        return code;
    };
    // tables (on the host, before any device call)
    // Flip thresholds [R][stride], then per slot the FP32 bits of 2 beta / ln 2,
    // from which the sparse one-slot-per-wavefront kernel evaluates the flip
    // probability itself and reads a threshold only near a uniform's edge.
    const int stride = 2 * P.D + 1;
    std::vector<uint32_t> tflip((size_t)R * stride + R);
    for (int r = 0; r < R; ++r) {
        for (int k = 0; k < stride; ++k)
            tflip[(size_t)r * stride + k] = threshold(flip_probability(o->rule, betas[r], 2LL * (k - P.D)));
        const float cf = (float)(2.0 * betas[r] / std::log(2.0));
        memcpy(&tflip[(size_t)R * stride + r], &cf, 4);
    }
    std::vector<uint32_t> tprop, tswap;
    std::vector<int32_t> tprop_off(R), tprop_len(R), tswap_off(std::max(R - 1, 1)), tswap_len(std::max(R - 1, 1));
    for (int r = 0; r < R; ++r) {
        tprop_off[r] = (int32_t)tprop.size();
        if (!tail_table(betas[r], tprop))
            return bail(fail(PT_EUNSUPPORTED, "proposal table of slot %d (beta %g) has more than %zu entries "
                             "(or all tables more than %zu)", r, betas[r], TAIL_TABLE_MAX, TAIL_TABLES_TOTAL_MAX));
        tprop_len[r] = (int32_t)tprop.size() - tprop_off[r];
    }
    for (int r = 0; r + 1 < R; ++r) {
        tswap_off[r] = (int32_t)tswap.size();
        if (!independent && !tail_table(betas[r + 1] - betas[r], tswap))
            return bail(fail(PT_EUNSUPPORTED, "swap table of pair (%d, %d) (beta gap %g) has more than %zu entries "
                             "(or all tables more than %zu)", r, r + 1, betas[r + 1] - betas[r], TAIL_TABLE_MAX,
                             TAIL_TABLES_TOTAL_MAX));
        tswap_len[r] = (int32_t)tswap.size() - tswap_off[r];
    }
    if (hipGetDevice(&c->device) != hipSuccess) return bail(fail(PT_EDEVICE, "no HIP device"));
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(PT_EDEVICE, "stream creation failed"));
    c->own_stream = true;
    hipStream_t s = c->stream;

    if (tprop.empty()) tprop.push_back(0);
    if (tswap.empty()) tswap.push_back(0);

    c->h_tswap_len.assign(tswap_len.begin(), tswap_len.begin() + std::max(R - 1, 0));
    std::vector<int16_t> colsites = P.color_sites;
    hipError_t e = hipSuccess;
#define UP(buf, vec) if (e == hipSuccess) e = upload(c->buf, vec, s)
    UP(J3, P.J3.empty() ? std::vector<int8_t>(1, 0) : P.J3);
    UP(row_ptr, P.row_ptr);
    UP(col, P.col.empty() ? std::vector<int16_t>(1, 0) : P.col);
    UP(Jc, P.Jc.empty() ? std::vector<int8_t>(1, 0) : P.Jc);
    UP(h, P.h);
    UP(clampd, P.clamp);
    UP(color_sites, colsites);
    UP(color_off, P.color_off);
    UP(csrw_grp, P.csrw_groups.empty() ? std::vector<int32_t>(1, 0) : P.csrw_groups);
    UP(tflip, tflip);
    UP(tprop, tprop);
    UP(tprop_off, tprop_off);
    UP(tprop_len, tprop_len);
    UP(tswap, tswap);
    UP(tswap_off, tswap_off);
    UP(tswap_len, tswap_len);
#undef UP
    c->h_bank_ptrs.assign(R, nullptr);
    c->h_bankE_ptrs.assign(R, nullptr);
    c->h_bank_n.assign(R, 0);
    c->banks.resize(R);
    if (e == hipSuccess) e = c->spins.alloc((size_t)R * P.n);
    if (e == hipSuccess) e = c->E.alloc((size_t)R * 4);
    if (e == hipSuccess) e = c->t.alloc(8);
    if (e == hipSuccess) e = c->cursor.alloc((size_t)R * 4);
    if (e == hipSuccess) e = c->bank_ptrs.alloc((size_t)R * 8);
    if (e == hipSuccess) e = c->bankE_ptrs.alloc((size_t)R * 8);
    if (e == hipSuccess) e = c->bank_n.alloc((size_t)R * 4);
    if (e == hipSuccess) e = c->swap_att.alloc((size_t)std::max(R - 1, 1) * 8);
    if (e == hipSuccess) e = c->swap_acc.alloc((size_t)std::max(R - 1, 1) * 8);
    if (e == hipSuccess) e = c->prop_att.alloc((size_t)R * 8);
    if (e == hipSuccess) e = c->prop_acc.alloc((size_t)R * 8);
    if (e == hipSuccess) e = c->flips.alloc((size_t)R * 8);
    if (e == hipSuccess) e = c->best.alloc(sizeof(BestRec));
    if (e == hipSuccess) e = c->best_spins.alloc((size_t)P.n);
    if (e == hipSuccess) e = c->inst.alloc(sizeof(InstDev));
    if (e == hipSuccess) e = hipMemsetAsync(c->cursor.p, 0, (size_t)R * 4, s);
    if (e == hipSuccess) e = hipMemsetAsync(c->bank_ptrs.p, 0, (size_t)R * 8, s);
    if (e == hipSuccess) e = hipMemsetAsync(c->bankE_ptrs.p, 0, (size_t)R * 8, s);
    if (e == hipSuccess) e = hipMemsetAsync(c->bank_n.p, 0, (size_t)R * 4, s);
    if (e != hipSuccess)
        return bail(fail(e == hipErrorOutOfMemory ? PT_ENOMEM : PT_EDEVICE, "device setup: %s", hipGetErrorString(e)));

    InstDev &I = c->hI;
    memset(&I, 0, sizeof I);
    I.n = P.n;
    I.L = P.L;
    I.R = R;
    I.kind = P.kind;
    I.rule = o->rule;
    // independent chains: a cycle longer than any run the sweep counter allows
    I.M = independent ? INDEPENDENT_M : o->sweeps_per_cycle;
    I.D = P.D;
    I.tflip_stride = stride;
    I.has_target = o->has_target ? 1 : 0;
    I.target = o->target;
    I.ncolors = P.ncolors;
    I.nfree = (int32_t)P.nfree;
    I.nnz = (int32_t)P.col.size();
    I.maxdeg = P.maxdeg;
    I.maxcnt = P.maxcnt;
    I.maxabsj = P.maxabsj;
    I.csrw_chunks = P.csrw_chunks;
    I.seed_lo = (uint32_t)o->seed;
    I.seed_hi = (uint32_t)(o->seed >> 32);
    I.epoch = 0;
    I.prop_start = o->prop_start;
    I.prop_period = o->prop_period;
    I.prop_stop = o->prop_stop;
    I.sweep_cap = ~0ull;
    fill_inst_pointers(c);
    rc = reset_state(c, nullptr, 0);
    if (rc) return bail(rc);
    *out = c;
    return PT_OK;
}

extern "C" int pt_destroy(pt_ctx *c)
{
    if (!c) return PT_OK;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return PT_OK;
}

extern "C" int pt_set_stream(pt_ctx *c, void *stream)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(c->stream));
    if (c->own_stream) HIPCHK(hipStreamDestroy(c->stream));
    c->own_stream = false;
    if (stream) {
        c->stream = (hipStream_t)stream;
    } else {
        HIPCHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        c->own_stream = true;
    }
    return PT_OK;
}

static int slot_of_beta(pt_ctx *c, double beta)
{
    for (int r = 0; r < c->R; ++r)
        if (c->betas[r] == beta) return r;
    return -1;
}

static int install_bank(pt_ctx *c, int r, const int8_t *cfg, int32_t k, bool device_src)
{
    hipStream_t s = c->stream;
    Bank &b = c->banks[r];
    if (k == 0) {
        HIPCHK(hipStreamSynchronize(s));
        b.cfg.release();
        b.E.release();
        b.n = 0;
        c->h_bank_ptrs[r] = nullptr;
        c->h_bankE_ptrs[r] = nullptr;
        c->h_bank_n[r] = 0;
    } else {
        HIPCHK(hipStreamSynchronize(s));
        HIPCHK(b.cfg.alloc((size_t)k * c->n));
        HIPCHK(b.E.alloc((size_t)k * 4));
        HIPCHK(hipMemcpyAsync(b.cfg.p, cfg, (size_t)k * c->n,
                              device_src ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
        HIPCHK(launch_energy(c->inst.as<InstDev>(), b.cfg.as<int8_t>(), k, b.E.as<int32_t>(), s));
        b.n = k;
        c->h_bank_ptrs[r] = b.cfg.as<int8_t>();
        c->h_bankE_ptrs[r] = b.E.as<int32_t>();
        c->h_bank_n[r] = k;
    }
    // start cursor: BANK stream word 0 mod B
    int32_t cur = k ? (int32_t)(host_philox_word0((uint32_t)r, 0, TAG_BANK, c->hI.seed_lo, c->hI.seed_hi) % (uint32_t)k) : 0;
    HIPCHK(hipMemcpyAsync(c->bank_ptrs.as<const int8_t *>() + r, &c->h_bank_ptrs[r], 8, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->bankE_ptrs.as<const int32_t *>() + r, &c->h_bankE_ptrs[r], 8, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->bank_n.as<int32_t>() + r, &c->h_bank_n[r], 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->cursor.as<int32_t>() + r, &cur, 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return PT_OK;
}

extern "C" int pt_propose(pt_ctx *c, double beta, const int8_t *configs, int32_t n_configs)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    int r = slot_of_beta(c, beta);
    if (r < 0) return fail(PT_EINVAL, "no slot has beta %.17g", beta);
    if (n_configs < 0) return fail(PT_EINVAL, "n_configs must be >= 0");
    if (n_configs > 0 && !configs) return fail(PT_EINVAL, "null configs");
    for (int64_t b = 0; b < n_configs; ++b)
        for (int i = 0; i < c->n; ++i) {
            int v = configs[b * c->n + i];
            if (v != 1 && v != -1) return fail(PT_EINVAL, "config %lld site %d is not +-1", (long long)b, i);
            if (c->clamp[i] && v != c->clamp[i])
                return fail(PT_EINVAL, "config %lld violates the clamp at site %d", (long long)b, i);
        }
    rc = install_bank(c, r, configs, n_configs, false);
    if (rc) c->broken = true;
    return rc;
}

extern "C" int pt_propose_device(pt_ctx *c, double beta, const int8_t *configs_dev, int32_t n_configs)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    int r = slot_of_beta(c, beta);
    if (r < 0) return fail(PT_EINVAL, "no slot has beta %.17g", beta);
    if (n_configs < 0 || (n_configs > 0 && !configs_dev)) return fail(PT_EINVAL, "bad device bank");
    rc = install_bank(c, r, configs_dev, n_configs, true);
    if (rc) c->broken = true;
    return rc;
}

extern "C" int pt_set_context(pt_ctx *c, double fraction, int32_t sweeps)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!(fraction >= 0.0 && fraction <= 1.0)) return fail(PT_EINVAL, "context fraction must lie in [0, 1]");
    if (sweeps < 0 || sweeps > 65535) return fail(PT_EINVAL, "completion sweeps must lie in 0..65535");
    // the context is round(fraction * n_free) free sites (halves round up)
    c->hI.ctx_K = (int32_t)std::floor(fraction * (double)c->nfree + 0.5);
    c->hI.ctx_on = (fraction > 0.0 || sweeps > 0) ? 1 : 0;
    c->hI.ctx_sweeps = sweeps;
    return push_inst(c);
}

extern "C" int pt_sweep(pt_ctx *c, uint64_t n_sweeps)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (contextual(c)) return fail(PT_EUNSUPPORTED, "contextual proposals run in batches (pt_batch_*), not on the plain path");
    if (c->t_host + n_sweeps > sweep_limit(c)) return fail(PT_EINVAL, "sweep counter would exceed %llu",
                                                            (unsigned long long)sweep_limit(c));
    hipStream_t s = c->stream;
    const int stride = 2 * c->D + 1;
    for (uint64_t k = 0; k < n_sweeps; ++k) {
        uint32_t t = (uint32_t)(c->t_host + k + 1);
        hipError_t e = launch_plain(c->kind, c->L, c->inst.as<InstDev>(), c->R, c->n, stride, c->hI.nnz, c->hI.nfree,
                                    c->ncolors, t, s);
        if (e != hipSuccess) {
            c->broken = true;
            return fail(PT_EDEVICE, "plain sweep launch: %s", hipGetErrorString(e));
        }
    }
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        c->broken = true;
        return fail(PT_EDEVICE, "plain sweep: %s", hipGetErrorString(e));
    }
    c->t_host += n_sweeps;
    return PT_OK;
}

extern "C" int pt_energies(pt_ctx *c, int32_t *out)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!out) return fail(PT_EINVAL, "null output");
    HIPCHK(hipMemcpyAsync(out, c->E.p, (size_t)c->R * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return PT_OK;
}

extern "C" int pt_state(pt_ctx *c, int8_t *spins, uint64_t *t)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (spins) HIPCHK(hipMemcpyAsync(spins, c->spins.p, (size_t)c->R * c->n, hipMemcpyDeviceToHost, c->stream));
    unsigned long long tt = 0;
    HIPCHK(hipMemcpyAsync(&tt, c->t.p, 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (t) *t = tt;
    return PT_OK;
}

extern "C" int pt_state_device(pt_ctx *c, int8_t *spins_dev)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!spins_dev) return fail(PT_EINVAL, "null output");
    HIPCHK(hipMemcpyAsync(spins_dev, c->spins.p, (size_t)c->R * c->n, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return PT_OK;
}

extern "C" int pt_set_state(pt_ctx *c, const int8_t *spins, uint64_t t)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!spins) return fail(PT_EINVAL, "null spins");
    for (size_t k = 0; k < (size_t)c->R * c->n; ++k) {
        int v = spins[k];
        int i = (int)(k % c->n);
        if ((v != 1 && v != -1) || (c->clamp[i] && v != c->clamp[i]))
            return fail(PT_EINVAL, "invalid spin at %zu", k);
    }
    rc = reset_state(c, spins, t);
    if (rc) c->broken = true;
    return rc;
}

extern "C" int pt_summary_get(pt_ctx *c, pt_summary *s, int8_t *best_spins)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    BestRec b;
    unsigned long long tt = 0;
    HIPCHK(hipMemcpyAsync(&b, c->best.p, sizeof b, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(&tt, c->t.p, 8, hipMemcpyDeviceToHost, c->stream));
    if (best_spins) HIPCHK(hipMemcpyAsync(best_spins, c->best_spins.p, c->n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (s) {
        s->t = tt;
        s->best_energy = b.E;
        s->best_t = b.t;
        s->best_slot = b.slot;
        s->first_hit = b.first_hit;
    }
    return PT_OK;
}

extern "C" int pt_counters(pt_ctx *c, uint64_t *swap_att, uint64_t *swap_acc, uint64_t *prop_att,
                           uint64_t *prop_acc, uint64_t *flips)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    hipStream_t s = c->stream;
    size_t R = c->R, P = R > 1 ? R - 1 : 0;
    if (swap_att && P) HIPCHK(hipMemcpyAsync(swap_att, c->swap_att.p, P * 8, hipMemcpyDeviceToHost, s));
    if (swap_acc && P) HIPCHK(hipMemcpyAsync(swap_acc, c->swap_acc.p, P * 8, hipMemcpyDeviceToHost, s));
    if (prop_att) HIPCHK(hipMemcpyAsync(prop_att, c->prop_att.p, R * 8, hipMemcpyDeviceToHost, s));
    if (prop_acc) HIPCHK(hipMemcpyAsync(prop_acc, c->prop_acc.p, R * 8, hipMemcpyDeviceToHost, s));
    if (flips) HIPCHK(hipMemcpyAsync(flips, c->flips.p, R * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return PT_OK;
}

// ---------------------------------------------------------------------------
// checkpoints: the whole chain state of a context as one host blob

namespace {
struct CkptHeader {
    char magic[8];            // "TAPTCKP" + format version byte
    uint64_t bytes;           // whole blob
    uint64_t fingerprint;     // problem, ladder, options, seed, bank sizes, proposal mode
    int32_t n, R;
    uint64_t t;
    BestRec best;
};
const char CKPT_MAGIC[8] = {'T', 'A', 'P', 'T', 'C', 'K', 'P', 1};

// Layout after the header, each array in slot order: int32 E[R],
// int32 cursor[R], uint64 swap_att[P], swap_acc[P] (P = max(R - 1, 1)),
// uint64 prop_att[R], prop_acc[R], flips[R], int8 spins[R][n], int8 best_spins[n].
uint64_t ckpt_bytes(int R, int n)
{
    uint64_t P = (uint64_t)std::max(R - 1, 1);
    return sizeof(CkptHeader) + 8ull * R + 16ull * P + 24ull * R + (uint64_t)R * n + (uint64_t)n;
}
} // namespace

// what a checkpoint must match: the problem and options fixed at creation,
// the bank sizes and the contextual-proposal mode
static uint64_t ckpt_fingerprint(const pt_ctx *c)
{
    Fnv f;
    f.val(c->problem_fp);
    f.add(c->h_bank_n);
    f.val(c->hI.ctx_K);
    f.val(c->hI.ctx_on);
    f.val(c->hI.ctx_sweeps);
    return f.h;
}

extern "C" int pt_save_size(pt_ctx *c, uint64_t *bytes)
{
    if (!c) return fail(PT_EINVAL, "null context");
    if (!bytes) return fail(PT_EINVAL, "null output");
    *bytes = ckpt_bytes(c->R, c->n);
    return PT_OK;
}

extern "C" int pt_save(pt_ctx *c, void *buf, uint64_t bytes)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    const int R = c->R, n = c->n;
    const size_t P = (size_t)std::max(R - 1, 1);
    if (!buf) return fail(PT_EINVAL, "null buffer");
    if (bytes < ckpt_bytes(R, n)) return fail(PT_EINVAL, "checkpoint needs %llu bytes (got %llu)",
                                               (unsigned long long)ckpt_bytes(R, n), (unsigned long long)bytes);
    hipStream_t s = c->stream;
    CkptHeader hd;
    memset(&hd, 0, sizeof hd);
    memcpy(hd.magic, CKPT_MAGIC, 8);
    hd.bytes = ckpt_bytes(R, n);
    hd.fingerprint = ckpt_fingerprint(c);
    hd.n = n;
    hd.R = R;
    char *q = (char *)buf + sizeof hd;
    unsigned long long tt = 0;
    HIPCHK(hipMemcpyAsync(&tt, c->t.p, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&hd.best, c->best.p, sizeof(BestRec), hipMemcpyDeviceToHost, s));
    auto take = [&](const DevBuf &b, size_t nbytes) -> hipError_t {
        hipError_t e = hipMemcpyAsync(q, b.p, nbytes, hipMemcpyDeviceToHost, s);
        q += nbytes;
        return e;
    };
    HIPCHK(take(c->E, 4 * (size_t)R));
    HIPCHK(take(c->cursor, 4 * (size_t)R));
    HIPCHK(take(c->swap_att, 8 * P));
    HIPCHK(take(c->swap_acc, 8 * P));
    HIPCHK(take(c->prop_att, 8 * (size_t)R));
    HIPCHK(take(c->prop_acc, 8 * (size_t)R));
    HIPCHK(take(c->flips, 8 * (size_t)R));
    HIPCHK(take(c->spins, (size_t)R * n));
    HIPCHK(take(c->best_spins, (size_t)n));
    HIPCHK(hipStreamSynchronize(s));
    hd.t = tt;
    memcpy(buf, &hd, sizeof hd);
    return PT_OK;
}

extern "C" int pt_restore(pt_ctx *c, const void *buf, uint64_t bytes)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    const int R = c->R, n = c->n;
    const size_t P = (size_t)std::max(R - 1, 1);
    if (!buf) return fail(PT_EINVAL, "null buffer");
    if (bytes < sizeof(CkptHeader)) return fail(PT_EINVAL, "checkpoint too short");
    CkptHeader hd;
    memcpy(&hd, buf, sizeof hd);
    if (memcmp(hd.magic, CKPT_MAGIC, 8)) return fail(PT_EINVAL, "not a checkpoint of this format");
    if (hd.n != n || hd.R != R || hd.bytes != ckpt_bytes(R, n) || bytes < hd.bytes)
        return fail(PT_EINVAL, "checkpoint shape (n=%d, R=%d, %llu bytes) does not fit this context", hd.n, hd.R,
                    (unsigned long long)hd.bytes);
    if (hd.fingerprint != ckpt_fingerprint(c))
        return fail(PT_EINVAL, "checkpoint was taken on a different problem, ladder, options, seed, bank sizes "
                               "or proposal mode");
    if (hd.t > sweep_limit(c)) return fail(PT_EINVAL, "checkpoint sweep counter out of range");
    const char *q = (const char *)buf + sizeof hd;
    std::vector<int32_t> E(R), cursor(R);
    memcpy(E.data(), q, 4 * (size_t)R);
    memcpy(cursor.data(), q + 4 * (size_t)R, 4 * (size_t)R);
    const char *counters = q + 8 * (size_t)R;
    const size_t counter_bytes = 16 * P + 24 * (size_t)R;
    const int8_t *spins = (const int8_t *)(counters + counter_bytes);
    const int8_t *bspins = spins + (size_t)R * n;
    for (int r = 0; r < R; ++r)
        if (c->h_bank_n[r] ? (cursor[r] < 0 || cursor[r] >= c->h_bank_n[r]) : cursor[r] < 0)
            return fail(PT_EINVAL, "checkpoint cursor of slot %d out of range", r);
    for (size_t k = 0; k < (size_t)R * n + n; ++k) {
        int v = spins[k];
        int i = (int)(k % n);
        if ((v != 1 && v != -1) || (c->clamp[i] && v != c->clamp[i]))
            return fail(PT_EINVAL, "checkpoint spin %zu is invalid", k);
    }
    // the energies must be those of the spins: recompute them aside first,
    // so that a corrupt checkpoint leaves the context as it was
    hipStream_t s = c->stream;
    DevBuf tmp_spins, tmp_E;
    HIPCHK(tmp_spins.alloc((size_t)R * n));
    HIPCHK(tmp_E.alloc(4 * (size_t)R));
    HIPCHK(hipMemcpyAsync(tmp_spins.p, spins, (size_t)R * n, hipMemcpyHostToDevice, s));
    HIPCHK(launch_energy(c->inst.as<InstDev>(), tmp_spins.as<int8_t>(), R, tmp_E.as<int32_t>(), s));
    std::vector<int32_t> E_dev(R);
    HIPCHK(hipMemcpyAsync(E_dev.data(), tmp_E.p, 4 * (size_t)R, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (E_dev != E) return fail(PT_EINVAL, "checkpoint energies do not match its spins");
    unsigned long long tt = hd.t;
    const char *cq = counters;
    auto put = [&](DevBuf &b, size_t nbytes) -> hipError_t {
        hipError_t e = hipMemcpyAsync(b.p, cq, nbytes, hipMemcpyHostToDevice, s);
        cq += nbytes;
        return e;
    };
    hipError_t e = hipMemcpyAsync(c->spins.p, tmp_spins.p, (size_t)R * n, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(c->E.p, tmp_E.p, 4 * (size_t)R, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(c->cursor.p, cursor.data(), 4 * (size_t)R, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = put(c->swap_att, 8 * P);
    if (e == hipSuccess) e = put(c->swap_acc, 8 * P);
    if (e == hipSuccess) e = put(c->prop_att, 8 * (size_t)R);
    if (e == hipSuccess) e = put(c->prop_acc, 8 * (size_t)R);
    if (e == hipSuccess) e = put(c->flips, 8 * (size_t)R);
    if (e == hipSuccess) e = hipMemcpyAsync(c->best_spins.p, bspins, (size_t)n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(c->best.p, &hd.best, sizeof(BestRec), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(c->t.p, &tt, 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        c->hI.epoch += 1;       // batches clear their exchange words for the new state
        e = hipMemcpyAsync(c->inst.p, &c->hI, sizeof(InstDev), hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        c->broken = true;
        return fail(PT_EDEVICE, "restore: %s", hipGetErrorString(e));
    }
    c->t_host = hd.t;
    return PT_OK;
}

extern "C" int pt_energy_device(pt_ctx *c, const int8_t *configs_dev, int32_t k, int32_t *energies_dev)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (k < 0 || (k > 0 && (!configs_dev || !energies_dev))) return fail(PT_EINVAL, "bad arguments");
    HIPCHK(launch_energy(c->inst.as<InstDev>(), configs_dev, k, energies_dev, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return PT_OK;
}

// ---------------------------------------------------------------------------
// batched path

struct LaunchGroup {
    int kind, L, rpt, block, grid = 0, tsw_entries = 0;
    bool mixed = false;               // one launch of chunk_kernel_mixed for several sweepers
    bool wave = false;                // wave-per-replica kernel
    bool pm = false;                  // +-J 8^3 kernel
    bool pml = false;                 // +-J row kernel, even L in 6..16, one slot per wavefront
    bool csrw = false;                // sparse graphs, one slot per wavefront
    int spw = 2;                      // its slots per wavefront (1 or 2)
    bool ctx = false;                 // some context has contextual proposals (chunk_kernel_ctx)
    int sparse = SPARSE_CSR;          // sparse graphs: the sweeper of the chunk kernel
    int sparse_req = 0;               // the caller's choice: 0 any, -1 no packed rows, SPARSE_ROW, SPARSE_ROW4
    size_t lds;
    std::vector<pt_ctx *> ctxs;
    std::vector<int> Gs;              // per context: slots per workgroup (max)
    std::vector<int> rpts;            // per context: slots per thread
    DevBuf items, order, first_item, best, best_spins, xbuf, status;
    std::vector<size_t> x_off, x_bytes;   // per context: its exchange words
    std::vector<uint32_t> x_epoch;        // epoch the exchange words were cleared for
    std::vector<char> ctx_mode;           // contextual proposals at build time (sizes the LDS)
    int n_items = 0;
};

struct pt_batch {
    std::vector<pt_ctx *> ctxs;
    std::vector<LaunchGroup *> groups;
    pt_batch_opts opts{};
    hipStream_t stream = nullptr;
    DevBuf err;
    DevBuf gmem;                      // the launch group's device buffers (grows, never shrinks)
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    uint32_t graph_K = 0;
    int device = 0;
    int cus = 0;
    hipStream_t own_stream = nullptr;
    std::vector<hipEvent_t> ev_pool;  // start/stop pairs of timed launches
    size_t ev_used = 0;
    // builds that do not wait for the stream: the work-item tables go to the
    // device from pinned staging, alternating between two, so a build never
    // overwrites the staging of the launch before the one still running
    bool async_build = false;
    unsigned build_gen = 0;
    HostPinned stage[2];
    double kernel_ms = 0.0;
    uint64_t kernel_launches = 0;
    ~pt_batch()
    {
        for (auto e : ev_pool) (void)hipEventDestroy(e);
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        for (auto *g : groups) delete g;
        if (own_stream) (void)hipStreamDestroy(own_stream);
    }
};

// Choose (slots per workgroup, slots per thread) for a context. What the
// caller leaves free comes from one of TILING_LEVELS automatic tilings,
// finest (most workgroups, fewest sites per thread: the shortest sweep) at
// level 0, coarsest at the last level; a launch takes the finest level whose
// workgroups can all be co-resident. At the last two levels a mixed launch
// gives large lattices 4 slots per thread, so that a batch of many sizes fits.
static constexpr int TILING_LEVELS = 5;

static void choose_tiling(const pt_ctx *c, const pt_batch_opts &o, bool mixed, bool ctx_group, int level, int &G,
                          int &rpt)
{
    const int R = c->R;
    rpt = o.replicas_per_thread > 0 ? o.replicas_per_thread : 0;
    if (rpt == 3) rpt = 2;      // the kernels come with 1, 2 or 4 slots per thread
    if (rpt > 4) rpt = 4;
    G = o.replicas_per_wg > 0 ? std::min(std::min(o.replicas_per_wg, R), 64) : 0;
    if (c->kind == KIND_CSR) {
        static const int csr_g[TILING_LEVELS] = {2, 4, 8, 16, 32};
        rpt = 1;
        if (!G) G = std::min(R, csr_g[level]);
        return;
    }
    if (!rpt) rpt = level < 2 ? 1 : (level >= TILING_LEVELS - 2 && mixed && c->n >= 1000) ? 4 : 2;
    if (ctx_group) rpt = 1;   // the contextual kernels hold one slot per thread
    // the cycle-end stages keep one slot per lane of a wavefront: G <= 64
    const int NC = c->n / 8;
    const int maxt = mixed ? mixed_max_threads() : lattice_max_threads();
    if (!G) {
        // whole ladder in one workgroup when it fits the block limit, else split
        int maxg = (maxt / NC) * rpt;
        G = std::min(R, std::max(rpt, maxg));
    }
    G = std::min(G, 64);
    while (((G + rpt - 1) / rpt) * NC > maxt && G > 1) --G;
}

// Host-side layout of one launch: the work items (one workgroup each, with
// near-equal slot counts per instance), the XCD-aware block order, the block
// size, the LDS carve-up, and whether every workgroup can be co-resident.
struct GroupPlan {
    std::vector<WorkItem> items;
    std::vector<int> first;
    std::vector<int32_t> order;
    struct Ctx { int first, W, n, xwords, gmax; size_t bs_off, x_off; };
    std::vector<Ctx> ctx;
    size_t nbest = 0, nbs = 0, nx = 0, lds = 0;
    int block = 64, grid = 0, tsw_max = 0, per_cu = 0;
    int sparse = SPARSE_CSR;
};

// Fewest slots per workgroup for the four-storages-per-lane sparse sweeper.
constexpr int QUAD_MIN_G = 12;

static int plan_group(const pt_batch *b, const LaunchGroup *g, GroupPlan &P)
{
    // Sparse graphs take a packed-row sweeper where every context fits it
    // (the four-storages-per-lane one first): its block holds one thread per
    // item (site and storage, or site and four storages) and bond share of
    // the largest colour class.
    const bool sparse_sync = g->kind == KIND_CSR && !g->mixed && !g->ctx && !g->csrw;
    bool row_ok = sparse_sync, row4_ok = sparse_sync;
    int row_block = 64, row4_block = 64;
    for (size_t k = 0; k < g->ctxs.size() && sparse_sync; ++k) {
        const InstDev &I = g->ctxs[k]->hI;
        if (I.n > CSR_ROW_MAXN || I.maxdeg > 2 * CSR_ROW_BPL || I.maxcnt < 1) row_ok = row4_ok = false;
        if (I.maxabsj > CSR_ROW_MAXJ) row_ok = false;
        if (I.D > 255) row4_ok = false;
    }
    for (size_t k = 0; k < g->ctxs.size(); ++k) {
        pt_ctx *c = g->ctxs[k];
        // the two-slot +-J kernel splits the ladder into whole slot pairs (even G, even s0)
        const int unit = g->pm ? g->spw : 1;
        int R = c->R / unit, W = (R + g->Gs[k] / unit - 1) / (g->Gs[k] / unit);
        int xwords = ((g->pml ? pml_xwords(c->L) : g->csrw ? csrw_xwords(c->n) : ((c->n + 31) >> 5) + 1) + 7) & ~7;
        P.ctx.push_back({(int)P.items.size(), W, c->n, xwords, unit * ((R + W - 1) / W), P.nbs, P.nx});
        P.first.push_back((int)P.items.size());
        int base = R / W, extra = R % W, s0 = 0;
        for (int w = 0; w < W; ++w) {
            int G = unit * (base + (w < extra ? 1 : 0));
            WorkItem it{};
            it.inst = c->inst.as<InstDev>();
            it.s0 = s0;
            it.G = G;
            it.w = w;
            it.W = W;
            it.xwords = xwords;
            it.variant = g->pml ? c->L : mixed_variant_of(c->kind, c->L, g->rpts[k]);
            P.items.push_back(it);
            s0 += G;
            P.nbs += (g->wave || g->pm || g->pml || g->csrw) ? (size_t)G * c->n : (size_t)((c->n + 15) & ~15);   // one snapshot per slot
        }
        P.nbest += W;
        P.nx += (size_t)W * 4 * xwords * 8;
        // LDS swap-table rows: pairs s0-1 .. s0+G-1 of each workgroup
        for (int w = 0; w < W; ++w) {
            const WorkItem &it = P.items[P.ctx[k].first + w];
            int tot = 0;
            for (int r = it.s0 - 1; r <= it.s0 + it.G - 1; ++r)
                if (r >= 0 && r + 1 < c->R) tot += c->h_tswap_len[r];
            P.tsw_max = std::max(P.tsw_max, tot);
        }
        // a block covers the largest item's threads
        int need = g->pm     ? 64 * (P.ctx[k].gmax / g->spw)
                   : (g->wave || g->pml || g->csrw) ? 64 * P.ctx[k].gmax
                             : c->kind == KIND_LATTICE ? lattice_threads(c->L, P.ctx[k].gmax, g->rpts[k])
                             // sparse graphs: a few slots per workgroup (the latency tilings) get 512
                             // threads, so that 2 or 4 lanes can share a site's bonds
                             : P.ctx[k].gmax <= 2 ? 512 : 256;
        P.block = std::max(P.block, (need + 63) & ~63);
        if (sparse_sync) {
            const int gmax = P.ctx[k].gmax, gs = (gmax + 3) & ~3;
            row_block = std::max(row_block, (c->hI.maxcnt * gmax * csr_row_lanes(c->hI.maxdeg) + 63) & ~63);
            row4_block = std::max(row4_block, (c->hI.maxcnt * (gs / 4) * csr_row4_lanes(c->hI.maxdeg) + 63) & ~63);
            if ((c->n - 1) * gs + 3 >= 65536) row4_ok = false;
        }
    }
    if (row_block > 512) row_ok = false;
    if (row4_block > 512) row4_ok = false;
    // independent chains (bank generation) take the coarsest tiling, where the
    // four-storages-per-lane LDS sweeper outruns the packed rows; the rows
    // only where the caller asks for them
    bool any_waits = false;
    for (pt_ctx *c : g->ctxs) any_waits = any_waits || c->opts.sweeps_per_cycle != 0;
    if (!any_waits && g->sparse_req == 0) row_ok = row4_ok = false;
    if (g->sparse_req == SPARSE_ROW4 && !row4_ok)
        return fail(PT_EUNSUPPORTED, "the four-storage packed-row sweeper does not fit this batch");
    if (g->sparse_req == SPARSE_ROW && !row_ok)
        return fail(PT_EUNSUPPORTED, "the packed-row sweeper does not fit this batch");
    if (g->sparse_req == SPARSE_ROW || g->sparse_req < 0) row4_ok = false;
    if (g->sparse_req == SPARSE_ROW4 || g->sparse_req < 0) row_ok = false;
    if (row4_ok) {
        P.sparse = SPARSE_ROW4;
        P.block = row4_block;
    } else if (row_ok) {
        P.sparse = SPARSE_ROW;
        P.block = row_block;
    }
    // XCD-aware order: workgroups are dispatched round-robin over the 8 XCDs,
    // so blockIdx b runs on XCD b % 8. Each XCD gets a contiguous run of the
    // instance-ordered items (so the workgroups of one instance share an L2);
    // blocks past the end of a run are padding that exits at once.
    const int nx8 = 8, n_items = (int)P.items.size();
    int per = (n_items + nx8 - 1) / nx8;
    P.order.assign((size_t)per * nx8, -1);
    for (int idx = 0; idx < n_items; ++idx) P.order[(size_t)(idx % per) * nx8 + idx / per] = idx;
    P.grid = per * nx8;
    // Sparse graphs in the coarse tilings (every workgroup at least
    // QUAD_MIN_G slots, 256 threads, no contextual proposals, every site's
    // field bound below 256) take the four-storages-per-lane sweeper. With
    // fewer slots a colour class has too few (site, quad) items to fill a
    // workgroup, and the sweep is bound by each item's chain of LDS reads,
    // which the quad layout does not shorten.
    bool quad = P.sparse == SPARSE_CSR && sparse_sync && P.block <= 256;
    for (size_t k = 0; k < g->ctxs.size() && quad; ++k) {
        if (g->ctxs[k]->D > 255) quad = false;
        for (int w = 0; w < P.ctx[k].W; ++w)
            if (P.items[P.ctx[k].first + w].G < QUAD_MIN_G) quad = false;
    }
    if (quad) P.sparse = SPARSE_QUAD;
    // LDS: the largest carve-up over the items (every item lays out its own
    // region with the common swap-table capacity)
    for (size_t k = 0; k < g->ctxs.size(); ++k) {
        pt_ctx *c = g->ctxs[k];
        P.lds = std::max(P.lds, g->pm     ? pm_lds_bytes(P.ctx[k].gmax, P.tsw_max)
                                : g->pml ? pml_lds_bytes(c->L, P.ctx[k].gmax, P.tsw_max)
                                : g->csrw ? csrw_lds_bytes(c->n, c->ncolors, c->hI.maxcnt, c->hI.csrw_chunks, P.ctx[k].gmax, 2 * c->D + 1,
                                                           P.tsw_max)
                                : g->wave ? wave_lds_bytes(c->n, P.ctx[k].gmax, 2 * c->D + 1, P.tsw_max)
                                          : chunk_lds_bytes(c->kind, c->n, P.ctx[k].gmax, 2 * c->D + 1, P.tsw_max,
                                                            c->hI.nnz, c->hI.nfree, c->ncolors, contextual(c), P.sparse,
                                                            P.sparse == SPARSE_ROW4
                                                                ? csr_row4_graph_bytes(c->ncolors, c->hI.maxcnt,
                                                                                       csr_row4_lanes(c->hI.maxdeg))
                                                            : P.sparse == SPARSE_ROW
                                                                ? csr_row_graph_bytes(c->ncolors, c->hI.maxcnt,
                                                                                      csr_row_lanes(c->hI.maxdeg))
                                                                : 0));
    }
    if (P.lds > 160 * 1024) return fail(PT_EUNSUPPORTED, "tiling needs %zu B of LDS per workgroup", P.lds);
    if (g->ctx && g->mixed)
        return fail(PT_EUNSUPPORTED, "contextual proposals need a batch of one lattice size or of general graphs");
    for (int r : g->rpts)
        if (g->ctx && r != 1) return fail(PT_EUNSUPPORTED, "contextual proposals take one slot per thread");
    if (g->pm)
        HIPCHK(pm_occupancy(g->spw, P.block, P.lds, &P.per_cu));
    else if (g->pml)
        HIPCHK(pml_occupancy(P.block, P.lds, &P.per_cu));
    else if (g->csrw)
        HIPCHK(csrw_occupancy(P.block, P.lds, &P.per_cu));
    else if (g->wave)
        HIPCHK(wave_occupancy(g->L, P.block, P.lds, &P.per_cu));
    else if (g->mixed)
        HIPCHK(chunk_occupancy_mixed(P.block, P.lds, &P.per_cu));
    else if (g->ctx)
        HIPCHK(chunk_occupancy_ctx(g->kind, g->L, P.block, P.lds, &P.per_cu));
    else {
        // a specialised sparse-graph launch at 512 threads takes the lane-sharing sweeper
        if (P.sparse == SPARSE_CSR && g->kind == KIND_CSR && P.block == 512) P.sparse = SPARSE_WIDE;
        HIPCHK(chunk_occupancy(g->kind, g->L, g->rpt, P.sparse, P.block, P.lds, &P.per_cu));
    }
    if (P.per_cu < 1) return fail(PT_EUNSUPPORTED, "kernel cannot run with block %d, LDS %zu", P.block, P.lds);
    // the cross-workgroup waits need every workgroup of the launch resident
    // (counted with the padding blocks, so that every XCD's share fits its CUs);
    // independent chains never wait, so their workgroups may queue
    bool waits = false;
    for (pt_ctx *c : g->ctxs) waits = waits || c->opts.sweeps_per_cycle != 0;
    if (waits && (long long)P.per_cu * b->cus < (long long)P.grid)
        return fail(PT_EUNSUPPORTED, "%d workgroups exceed the %d that can be co-resident; use fewer contexts per batch",
                    P.grid, P.per_cu * b->cus);
    return PT_OK;
}

// Where a launch group's device buffers come from: fresh allocations, or
// 256-byte aligned views into a region the caller provides (the static
// scratch of pt_batch_run_static), in which case nothing is allocated.
struct GroupMem {
    char *base = nullptr;             // null: allocate
    size_t cap = 0, used = 0;
    hipError_t take(DevBuf &b, size_t bytes)
    {
        if (!base) return b.alloc(bytes);
        const size_t at = (used + 255) & ~(size_t)255;
        const size_t len = (bytes + 7) & ~(size_t)7;
        if (at + len > cap) return hipErrorOutOfMemory;
        b.view(base + at, len);
        used = at + len;
        return hipSuccess;
    }
    template <class T> hipError_t put(DevBuf &b, const std::vector<T> &v, hipStream_t s)
    {
        hipError_t e = take(b, v.size() * sizeof(T));
        if (e != hipSuccess || v.empty()) return e;
        return hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
    }
    // the same from a copy in pinned staging at *at (advanced past it)
    template <class T> hipError_t put_staged(DevBuf &b, const std::vector<T> &v, char *&at, hipStream_t s)
    {
        hipError_t e = take(b, v.size() * sizeof(T));
        if (e != hipSuccess || v.empty()) return e;
        memcpy(at, v.data(), v.size() * sizeof(T));
        e = hipMemcpyAsync(b.p, at, v.size() * sizeof(T), hipMemcpyHostToDevice, s);
        at += (v.size() * sizeof(T) + 15) & ~(size_t)15;
        return e;
    }
};

// Bytes build_group takes from a GroupMem region for this plan (the same
// sequence of 256-byte aligned, 8-byte padded parts).
static size_t group_bytes(const LaunchGroup *g, const GroupPlan &P)
{
    size_t used = 0;
    auto take = [&](size_t bytes) { used = ((used + 255) & ~(size_t)255) + ((bytes + 7) & ~(size_t)7); };
    take(g->ctxs.size() * sizeof(InstStatus));
    take(P.nbest * sizeof(BestRec));
    take(P.nbs);
    take(P.nx);
    take(P.items.size() * sizeof(WorkItem));
    take(P.order.size() * sizeof(int32_t));
    take(P.first.size() * sizeof(int));
    return used;
}

static int build_group(pt_batch *b, LaunchGroup *g, GroupMem &mem)
{
    hipStream_t s = b->stream;
    GroupPlan P;
    int rc = plan_group(b, g, P);
    if (rc) return rc;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = mem.take(g->status, g->ctxs.size() * sizeof(InstStatus));
    if (e == hipSuccess) e = mem.take(g->best, P.nbest * sizeof(BestRec));
    if (e == hipSuccess) e = mem.take(g->best_spins, P.nbs);
    if (e == hipSuccess) e = mem.take(g->xbuf, P.nx);
    if (e == hipErrorOutOfMemory && mem.base)
        return fail(PT_ENOMEM, "the launch needs more than the %zu bytes of static scratch", mem.cap);
    HIPCHK(e);
    HIPCHK(launch_zero(g->xbuf.p, g->xbuf.bytes, s));
    size_t bi = 0;
    for (size_t k = 0; k < g->ctxs.size(); ++k) {
        const GroupPlan::Ctx &p = P.ctx[k];
        size_t bs_off = p.bs_off;
        for (int w = 0; w < p.W; ++w) {
            WorkItem &it = P.items[p.first + w];
            it.best = g->best.as<BestRec>() + bi++;
            it.best_spins = g->best_spins.as<int8_t>() + bs_off;
            bs_off += (g->wave || g->pm || g->pml || g->csrw) ? (size_t)it.G * p.n : (size_t)((p.n + 15) & ~15);
            it.xbuf = (unsigned long long *)(g->xbuf.as<int8_t>() + p.x_off);
        }
        g->x_off.push_back(p.x_off);
        g->x_bytes.push_back((size_t)p.W * 4 * p.xwords * 8);
        g->x_epoch.push_back(g->ctxs[k]->hI.epoch);
        g->ctx_mode.push_back(contextual(g->ctxs[k]) ? 1 : 0);
    }
    g->n_items = (int)P.items.size();
    g->sparse = P.sparse;
    g->grid = P.grid;
    g->block = P.block;
    g->lds = P.lds;
    g->tsw_entries = P.tsw_max;
    if (b->async_build) {
        auto padded = [](size_t x) { return (x + 15) & ~(size_t)15; };
        HostPinned &st = b->stage[b->build_gen++ & 1];
        if (e == hipSuccess)
            e = st.reserve(padded(P.items.size() * sizeof(WorkItem)) + padded(P.order.size() * sizeof(int32_t)) +
                           padded(P.first.size() * sizeof(int)));
        char *at = st.as<char>();
        if (e == hipSuccess) e = mem.put_staged(g->items, P.items, at, s);
        if (e == hipSuccess) e = mem.put_staged(g->order, P.order, at, s);
        if (e == hipSuccess) e = mem.put_staged(g->first_item, P.first, at, s);
    } else {
        if (e == hipSuccess) e = mem.put(g->items, P.items, s);
        if (e == hipSuccess) e = mem.put(g->order, P.order, s);
        if (e == hipSuccess) e = mem.put(g->first_item, P.first, s);
    }
    if (e == hipErrorOutOfMemory && mem.base)
        return fail(PT_ENOMEM, "the launch needs more than the %zu bytes of static scratch", mem.cap);
    HIPCHK(e);
    // the host vectors must outlive their copies (staged copies do not read them)
    if (!b->async_build) HIPCHK(hipStreamSynchronize(s));
    return PT_OK;
}

static void clear_groups(pt_batch *b)
{
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
    for (auto *g : b->groups) delete g;
    b->groups.clear();
    b->ctxs.clear();
}

// The launch group for a set of contexts (host fields only). Contexts that
// share one sweeper instantiation run in the specialised kernel; a set that
// needs several sweepers runs as a single launch of the mixed kernel.
static LaunchGroup *make_group(const pt_batch_opts &o, const std::vector<pt_ctx *> &ctxs, int level, bool pml_auto,
                               bool force_mixed = false)
{
    bool any_ctx = false;
    for (pt_ctx *c : ctxs) any_ctx = any_ctx || contextual(c);
    std::map<std::tuple<int, int, int>, int> keys;
    for (pt_ctx *c : ctxs) {
        int G, rpt;
        choose_tiling(c, o, false, any_ctx, level, G, rpt);
        keys[std::make_tuple(c->kind, c->kind == KIND_LATTICE ? c->L : 0, rpt)] += 1;
    }
    LaunchGroup *g = new LaunchGroup();
    // the +-J row kernel runs lattices of several sizes in one launch: where
    // every context is a +-J lattice with even L in 6..16, when the caller
    // asks for it (kernel 7) or leaves the kernel open (kernel 0, one slot
    // per thread) and the batch is not one of 8^3 lattices only (the +-J 8^3
    // kernel's)
    bool all_pml = !any_ctx, all_pm8 = true;
    for (pt_ctx *c : ctxs) {
        all_pml = all_pml && c->pmL;
        all_pm8 = all_pm8 && c->pmJ;
    }
    g->pml = all_pml && (o.kernel == 7 || (pml_auto && o.kernel == 0 && !all_pm8 && o.replicas_per_thread <= 1));
    // the one-slot-per-wavefront sparse kernel where every context is a
    // general graph that fits it (its mailbox carries energies of 24 bits),
    // when the caller asks for it (kernel 8) or leaves the kernel open for
    // chains that exchange (independent chains never wait, and wide
    // workgroups of the workgroup-synchronous kernel sweep them faster)
    bool waits = false;
    for (pt_ctx *c : ctxs) waits = waits || c->opts.sweeps_per_cycle != 0;
    bool all_csrw = !any_ctx && (o.kernel == 8 || (pml_auto && o.kernel == 0 && waits));
    for (pt_ctx *c : ctxs)
        all_csrw = all_csrw && c->kind == KIND_CSR &&
                   csrw_supported(c->n, c->hI.maxabsj, c->hI.csrw_chunks, c->hI.maxcnt) && (long long)c->n * c->D < (1 << 23);
    g->csrw = all_csrw;
    g->mixed = (keys.size() > 1 || force_mixed) && !g->pml;
    g->kind = ctxs[0]->kind;
    g->L = g->kind == KIND_LATTICE ? ctxs[0]->L : 0;
    // the wave-per-replica kernel: one lattice size whose storage is exactly
    // one wavefront, unless the caller asks for the workgroup-synchronous one
    bool all_pm = !g->mixed;
    for (pt_ctx *c : ctxs) all_pm = all_pm && c->pmJ;
    // contextual proposals run in the workgroup-synchronous kernels only
    all_pm = all_pm && !any_ctx;
    g->ctx = any_ctx;
    g->pm = !g->pml && all_pm && (o.kernel == 3 || o.kernel == 4 || (o.kernel == 0 && o.replicas_per_thread <= 1));
    g->spw = o.kernel == 4 ? 1 : 2;
    g->sparse_req = o.kernel == 1 ? -1 : o.kernel == 5 ? SPARSE_ROW : o.kernel == 6 ? SPARSE_ROW4 : 0;
    g->wave = !g->pm && !g->pml && !g->mixed && !any_ctx && g->kind == KIND_LATTICE && wave_supported(g->L) &&
              o.kernel != 1 && o.kernel != 5 && o.kernel != 6 && (o.kernel == 2 || o.replicas_per_thread <= 1);
    for (pt_ctx *c : ctxs) {
        int G, rpt;
        if (g->pm) {
            rpt = 1;
            G = o.replicas_per_wg > 0 ? o.replicas_per_wg : 8;
            G = std::min(std::min(G, c->R), pm_max_storages(g->spw));
            if (g->spw == 2) G = std::max(G & ~1, 2);
        } else if (g->pml) {
            // left open, a large lattice takes 4 slots per workgroup: its
            // wavefronts keep a SIMD's issue slots busy alone, so a workgroup
            // of 4 gives each its own SIMD; smaller ones take 8
            rpt = 1;
            G = o.replicas_per_wg > 0 ? o.replicas_per_wg : (c->n > 2000 ? 4 : pml_max_storages());
            G = std::min(std::min(G, c->R), pml_max_storages());
        } else if (g->csrw) {
            rpt = 1;
            G = o.replicas_per_wg > 0 ? o.replicas_per_wg : csrw_max_storages();
            G = std::min(std::min(G, c->R), csrw_max_storages());
        } else if (g->wave) {
            rpt = 1;
            G = o.replicas_per_wg > 0 ? o.replicas_per_wg : wave_max_storages();
            G = std::min(std::min(G, c->R), wave_max_storages());
        } else {
            choose_tiling(c, o, g->mixed, any_ctx, level, G, rpt);
        }
        g->rpt = rpt;
        g->ctxs.push_back(c);
        g->Gs.push_back(G);
        g->rpts.push_back(rpt);
    }
    return g;
}

// The launch group of a set of contexts at the finest automatic tiling
// level whose workgroups fit (the caller's fixed tiling choices hold at
// every level). Independent chains never wait for one another, so nothing
// bounds their workgroup count and they take the coarsest level, which
// fills the workgroups best. On failure *out is null and the last level's
// error stands.
static int pick_group(const pt_batch *b, const std::vector<pt_ctx *> &ctxs, LaunchGroup **out)
{
    *out = nullptr;
    int rc = PT_OK;
    bool waits = false;
    for (pt_ctx *c : ctxs) waits = waits || c->opts.sweeps_per_cycle != 0;
    // first the one-slot-per-wavefront kernels (+-J rows, general graphs)
    // where the caller leaves the kernel open (their tiling does not depend on
    // the level), then the others, then the mixed kernel for any set. A set
    // that fits the mixed kernel keeps fitting it when contexts leave it
    // (fewer workgroups, no more LDS), so a server that admitted a set can
    // always run what remains of it.
    const bool open = b->opts.kernel == 0 || b->opts.kernel == 1;
    for (int pass = 0; pass < 3; ++pass) {
        if (pass == 2 && !open) break;
        for (int level = waits ? 0 : TILING_LEVELS - 1; level < TILING_LEVELS; ++level) {
            LaunchGroup *g = make_group(b->opts, ctxs, level, pass == 0, pass == 2);
            if (pass == 0 && !((g->pml || g->csrw) && b->opts.kernel == 0)) {
                delete g;
                break;
            }
            if (pass == 2 && (!g->mixed || g->ctx)) {   // the mixed kernel takes no contextual proposals
                delete g;
                break;
            }
            GroupPlan P;
            const int r = plan_group(b, g, P);
            if (r == PT_OK) {
                g->sparse = P.sparse;   // the sweeper it would run (build_group sets it again)
                *out = g;
                return PT_OK;
            }
            rc = r;
            delete g;
            if (pass == 0) break;
        }
    }
    return rc;
}

// (Re)build the launch group of a batch for the contexts ctxs[0..k).
static int batch_set_contexts(pt_batch *b, pt_ctx *const *ctxs, int32_t k)
{
    clear_groups(b);
    for (int i = 0; i < k; ++i) {
        if (!ctxs[i] || ctxs[i]->broken) return fail(PT_EINVAL, "context %d missing or unusable", i);
        if (ctxs[i]->device != b->device) return fail(PT_EINVAL, "context %d lives on another device", i);
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return fail(PT_EINVAL, "context %d appears twice", i);
        b->ctxs.push_back(ctxs[i]);
    }
    LaunchGroup *g = nullptr;
    int rc = pick_group(b, b->ctxs, &g);
    if (rc) return rc;
    b->groups.push_back(g);
    // the buffers are views into the batch's region, which grows when a
    // launch needs more (a rebuilt batch, as in serving, allocates nothing
    // while its launches fit the region)
    GroupPlan P;
    rc = plan_group(b, g, P);
    if (rc) return rc;
    const size_t need = group_bytes(g, P);
    if (b->gmem.bytes < need) {
        HIPCHK(hipStreamSynchronize(b->stream));
        HIPCHK(b->gmem.alloc(std::max(need, 2 * b->gmem.bytes)));
    }
    GroupMem mem;
    mem.base = b->gmem.as<char>();
    mem.cap = b->gmem.bytes;
    return build_group(b, g, mem);
}

// PT_OK if the contexts could run in one launch of this batch (no allocation).
static int batch_fits(const pt_batch *b, const std::vector<pt_ctx *> &ctxs)
{
    LaunchGroup *g = nullptr;
    int rc = pick_group(b, ctxs, &g);
    delete g;
    return rc;
}

// shared: run on that stream (not owned), else on a stream of the batch's own
static int batch_init(pt_batch *b, int device, hipStream_t shared = nullptr)
{
    b->device = device;
    if (hipSetDevice(b->device) != hipSuccess) return fail(PT_EDEVICE, "hipSetDevice");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, b->device) != hipSuccess) return fail(PT_EDEVICE, "device properties");
    b->cus = prop.multiProcessorCount;
    if (shared) {
        b->stream = shared;
    } else {
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess)
            return fail(PT_EDEVICE, "stream creation failed");
        b->own_stream = b->stream;
    }
    if (b->err.alloc(32) != hipSuccess) return fail(PT_ENOMEM, "error flag");
    if (hipMemset(b->err.p, 0, 32) != hipSuccess) return fail(PT_EDEVICE, "memset");
    return PT_OK;
}

extern "C" int pt_batch_create(pt_ctx *const *ctxs, int32_t k, const pt_batch_opts *o, pt_batch **out)
{
    if (!out) return fail(PT_EINVAL, "null output pointer");
    *out = nullptr;
    if (!ctxs || k < 1) return fail(PT_EINVAL, "need at least one context");
    if (!ctxs[0]) return fail(PT_EINVAL, "context 0 missing");
    if (o && (o->kernel < 0 || o->kernel > 8)) return fail(PT_EINVAL, "kernel must be in 0..8 (got %d)", o->kernel);
    pt_batch *b = new pt_batch();
    if (o) b->opts = *o;
    if (b->opts.chunk_sweeps <= 0) b->opts.chunk_sweeps = 1000;
    int rc = batch_init(b, ctxs[0]->device);
    if (!rc) rc = batch_set_contexts(b, ctxs, k);
    if (rc) {
        delete b;
        return rc;
    }
    *out = b;
    return PT_OK;
}

static hipError_t enqueue_round(pt_batch *b, uint32_t K, bool timed)
{
    for (auto *g : b->groups) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (timed) {
            while (b->ev_pool.size() < b->ev_used + 2) {
                hipEvent_t ev;
                hipError_t ee = hipEventCreate(&ev);
                if (ee != hipSuccess) return ee;
                b->ev_pool.push_back(ev);
            }
            e0 = b->ev_pool[b->ev_used++];
            e1 = b->ev_pool[b->ev_used++];
            hipError_t ee = hipEventRecord(e0, b->stream);
            if (ee != hipSuccess) return ee;
        }
        ChunkArgs a{};
        a.items = g->items.as<WorkItem>();
        a.order = g->order.as<int32_t>();
        a.n_items = g->grid;
        a.K = K;
        a.err = b->err.as<int32_t>();
        a.spin_limit = 1u << 22;
        a.tsw_entries = g->tsw_entries;
        hipError_t e = g->pm      ? launch_pm(g->spw, a, g->block, g->lds, b->stream)
                       : g->pml   ? launch_pml(a, g->block, g->lds, b->stream)
                       : g->csrw  ? launch_csrw(a, g->block, g->lds, b->stream)
                       : g->wave  ? launch_wave(g->L, a, g->block, g->lds, b->stream)
                       : g->mixed ? launch_chunk_mixed(a, g->block, g->lds, b->stream)
                       : g->ctx   ? launch_chunk_ctx(g->kind, g->L, a, g->block, g->lds, b->stream)
                                  : launch_chunk(g->kind, g->L, g->rpt, g->sparse, a, g->block, g->lds,
                                                 b->stream);
        if (e != hipSuccess) return e;
        if (timed) {
            e = hipEventRecord(e1, b->stream);
            if (e != hipSuccess) return e;
        }
        e = launch_finish(g->items.as<WorkItem>(), g->first_item.as<int>(), (int)g->ctxs.size(), K,
                          g->status.as<InstStatus>(), b->stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Run n_sweeps sweeps of every context of a built batch. timed: record HIP
// events around the chunk launches (pt_batch_kernel_time); untimed eager
// launches create nothing. The graph path is taken when the batch asks for it.
static int batch_sweep(pt_batch *b, uint64_t n_sweeps, bool timed)
{
    if (n_sweeps == 0) return PT_OK;
    // every context stops exactly at its own t + n_sweeps: the caps go to the
    // device in one small launch per 64 contexts rather than one copy each
    std::vector<InstDev *> insts;
    std::vector<unsigned long long> caps;
    for (pt_ctx *c : b->ctxs) {
        if (c->broken) return fail(PT_ESTATE, "a context of the batch is unusable");
        if (c->t_host + n_sweeps > sweep_limit(c))
            return fail(PT_EINVAL, "sweep counter would exceed %llu", (unsigned long long)sweep_limit(c));
        if (c->stream != b->stream && hipStreamQuery(c->stream) != hipSuccess) HIPCHK(hipStreamSynchronize(c->stream));
        c->hI.sweep_cap = c->t_host + n_sweeps;
        insts.push_back(c->inst.as<InstDev>());
        caps.push_back(c->hI.sweep_cap);
    }
    HIPCHK(launch_set_caps(insts.data(), caps.data(), (int)insts.size(), b->stream));
    for (auto *g : b->groups)
        for (size_t k = 0; k < g->ctxs.size(); ++k)
            if (g->ctx_mode[k] != (contextual(g->ctxs[k]) ? 1 : 0))
                return fail(PT_ESTATE, "a context's proposal mode changed after the batch was built");
    // a replaced state restarts the cycle count: clear that instance's exchange words
    for (auto *g : b->groups)
        for (size_t k = 0; k < g->ctxs.size(); ++k)
            if (g->x_epoch[k] != g->ctxs[k]->hI.epoch) {
                HIPCHK(launch_zero(g->xbuf.as<int8_t>() + g->x_off[k], g->x_bytes[k], b->stream));
                g->x_epoch[k] = g->ctxs[k]->hI.epoch;
            }
    const uint32_t K = (uint32_t)b->opts.chunk_sweeps;
    uint64_t rounds = (n_sweeps + K - 1) / K;
    if (b->opts.use_graph) {
        if (!b->gexec || b->graph_K != K) {
            if (b->gexec) {
                HIPCHK(hipGraphExecDestroy(b->gexec));
                b->gexec = nullptr;
            }
            if (b->graph) {
                HIPCHK(hipGraphDestroy(b->graph));
                b->graph = nullptr;
            }
            HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            hipError_t e = enqueue_round(b, K, false);
            hipGraph_t gr = nullptr;
            hipError_t e2 = hipStreamEndCapture(b->stream, &gr);
            if (e != hipSuccess) return fail(PT_EDEVICE, "capture: %s", hipGetErrorString(e));
            if (e2 != hipSuccess) return fail(PT_EDEVICE, "end capture: %s", hipGetErrorString(e2));
            b->graph = gr;
            HIPCHK(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
            b->graph_K = K;
        }
        for (uint64_t k = 0; k < rounds; ++k) HIPCHK(hipGraphLaunch(b->gexec, b->stream));
    } else {
        b->ev_used = 0;
        for (uint64_t k = 0; k < rounds; ++k) {
            hipError_t e = enqueue_round(b, K, timed);
            if (e != hipSuccess) return fail(PT_EDEVICE, "chunk launch: %s", hipGetErrorString(e));
        }
    }
    int err[8] = {0};
    HIPCHK(hipMemcpyAsync(err, b->err.p, 32, hipMemcpyDeviceToHost, b->stream));
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        for (pt_ctx *c : b->ctxs) c->broken = true;
        return fail(PT_EDEVICE, "batched sweep: %s", hipGetErrorString(e));
    }
    for (size_t k = 0; k + 1 < b->ev_used; k += 2) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, b->ev_pool[k], b->ev_pool[k + 1]));
        b->kernel_ms += ms;
        b->kernel_launches += 1;
    }
    b->ev_used = 0;
    for (pt_ctx *c : b->ctxs) c->t_host += n_sweeps;
    if (err[0]) {
        for (pt_ctx *c : b->ctxs) c->broken = true;
        return fail(PT_ETIMEOUT,
                    "exchange wait timed out (kind %d): item %d (workgroup %d of its instance) waiting on side %d "
                    "at cycle %d saw word %08x:%08x, epoch %d",
                    err[0], err[1], err[2], err[3], err[4], (unsigned)err[6], (unsigned)err[5], err[7]);
    }
    return PT_OK;
}

extern "C" int pt_batch_sweep(pt_batch *b, uint64_t n_sweeps)
{
    if (!b) return fail(PT_EINVAL, "null batch");
    HIPCHK(hipSetDevice(b->device));
    return batch_sweep(b, n_sweeps, true);
}

extern "C" int pt_batch_set_stream(pt_batch *b, void *stream)
{
    if (!b) return fail(PT_EINVAL, "null batch");
    HIPCHK(hipSetDevice(b->device));
    HIPCHK(hipStreamSynchronize(b->stream));
    b->stream = stream ? (hipStream_t)stream : b->own_stream;
    if (b->gexec) {
        HIPCHK(hipGraphExecDestroy(b->gexec));
        b->gexec = nullptr;
    }
    if (b->graph) {
        HIPCHK(hipGraphDestroy(b->graph));
        b->graph = nullptr;
    }
    return PT_OK;
}

extern "C" int pt_batch_kernel_time(pt_batch *b, double *ms, uint64_t *launches)
{
    if (!b) return fail(PT_EINVAL, "null batch");
    if (ms) *ms = b->kernel_ms;
    if (launches) *launches = b->kernel_launches;
    b->kernel_ms = 0.0;
    b->kernel_launches = 0;
    return PT_OK;
}

// The kernel and sweeper a launch group runs, as pt_batch_describe names them.
static std::string group_identity(const LaunchGroup *g)
{
    const char *kern = g->pm    ? (g->spw == 1 ? "pm1" : "pm")
                       : g->pml ? "pml"
                       : g->csrw ? "csrw"
                       : g->wave ? "wave"
                       : g->mixed ? "mixed"
                       : g->ctx ? "ctx"
                                : "chunk";
    std::string sw;
    if (g->pm || g->pml || g->csrw || g->wave || g->mixed) sw = "-";
    else if (g->kind == KIND_LATTICE) sw = "lattice" + std::to_string(g->L) + "x" + std::to_string(g->rpt);
    else sw = g->sparse == SPARSE_ROW4  ? "csr-row4"
              : g->sparse == SPARSE_ROW ? "csr-row"
              : g->sparse == SPARSE_QUAD ? "csr-quad"
              : g->sparse == SPARSE_WIDE ? "csr-wide"
                                         : "csr";
    return std::string("kernel=") + kern + " sweeper=" + sw;
}

extern "C" int pt_batch_describe(pt_batch *b, char *buf, int32_t len)
{
    if (!b || !buf || len < 1) return fail(PT_EINVAL, "null batch or buffer");
    std::string out;
    for (const LaunchGroup *g : b->groups) {
        char line[256];
        snprintf(line, sizeof line, "%s contexts=%zu grid=%d block=%d lds=%zu\n", group_identity(g).c_str(),
                 g->ctxs.size(), g->grid, g->block, g->lds);
        out += line;
    }
    snprintf(buf, (size_t)len, "%s", out.c_str());
    return PT_OK;
}

extern "C" int pt_batch_destroy(pt_batch *b)
{
    if (!b) return PT_OK;
    (void)hipSetDevice(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    delete b;
    return PT_OK;
}

// ---------------------------------------------------------------------------
// batched runs that allocate nothing: the launch's device buffers live in a
// file-scope static device array. In host code the array's name is only a
// stand-in for it; its device address (one per GPU) comes from
// hipGetSymbolAddress and is the only form in which host code uses it.

constexpr size_t STATIC_SCRATCH_BYTES = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[MAX_DEVICES];

// Device address of `scratch` on the current device `dev`, looked up once
// per device.
static int static_scratch(int dev, char **out)
{
    if (dev < 0 || dev >= MAX_DEVICES) return fail(PT_EUNSUPPORTED, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(PT_EDEVICE, "static scratch address: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = (char *)g_scratch_ptr[dev];
    return PT_OK;
}

extern "C" int pt_batch_run_static(pt_ctx *const *ctxs, int32_t k, const pt_batch_opts *o, uint64_t n_sweeps,
                                   void *stream)
{
    if (!ctxs || k < 1) return fail(PT_EINVAL, "need at least one context");
    if (!ctxs[0]) return fail(PT_EINVAL, "context 0 missing");
    const int dev = ctxs[0]->device;
    HIPCHK(hipSetDevice(dev));
    char *base = nullptr;
    int rc = static_scratch(dev, &base);
    if (rc) return rc;
    pt_batch b;                        // on the stack: owns no stream and no device memory
    if (o) b.opts = *o;
    b.opts.use_graph = 0;
    if (b.opts.chunk_sweeps <= 0) b.opts.chunk_sweeps = 1000;
    b.device = dev;
    HIPCHK(hipDeviceGetAttribute(&b.cus, hipDeviceAttributeMultiprocessorCount, dev));
    b.stream = stream ? (hipStream_t)stream : ctxs[0]->stream;
    for (int i = 0; i < k; ++i) {
        if (!ctxs[i] || ctxs[i]->broken) return fail(PT_EINVAL, "context %d missing or unusable", i);
        if (ctxs[i]->device != dev) return fail(PT_EINVAL, "context %d lives on another device", i);
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return fail(PT_EINVAL, "context %d appears twice", i);
        b.ctxs.push_back(ctxs[i]);
    }
    LaunchGroup *g = nullptr;
    rc = pick_group(&b, b.ctxs, &g);
    if (rc) return rc;
    b.groups.push_back(g);
    GroupMem mem;
    mem.base = base;
    mem.cap = STATIC_SCRATCH_BYTES;
    // the error flag, cleared: a previous call may have left it set
    HIPCHK(mem.take(b.err, 32));
    HIPCHK(launch_zero(b.err.p, 32, b.stream));
    rc = build_group(&b, g, mem);
    if (rc) return rc;
    return batch_sweep(&b, n_sweeps, false);
}

// ---------------------------------------------------------------------------
// serving: continuous batching of solve requests

namespace {

// One allocation holds a served request's state; the parts are 256-byte aligned.
struct ArenaLayout {
    size_t spins, E, t, cursor, bank_ptrs, bankE_ptrs, bank_n, swap_att, swap_acc, prop_att, prop_acc, flips, best,
        best_spins, inst, total;
};

ArenaLayout arena_layout(int R, int n)
{
    ArenaLayout A;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = (o + bytes + 255) & ~(size_t)255;
        return at;
    };
    const size_t P = (size_t)std::max(R - 1, 1);
    A.spins = take((size_t)R * n);
    A.E = take((size_t)R * 4);
    A.t = take(8);
    A.cursor = take((size_t)R * 4);
    A.bank_ptrs = take((size_t)R * 8);
    A.bankE_ptrs = take((size_t)R * 8);
    A.bank_n = take((size_t)R * 4);
    A.swap_att = take(P * 8);
    A.swap_acc = take(P * 8);
    A.prop_att = take((size_t)R * 8);
    A.prop_acc = take((size_t)R * 8);
    A.flips = take((size_t)R * 8);
    A.best = take(sizeof(BestRec));
    A.best_spins = take((size_t)n);
    A.inst = take(sizeof(InstDev));
    A.total = o;
    return A;
}

// A context that reads the problem, tables and banks of `tm` (device data the
// template owns) and owns only its replica state, on stream s.
// The state lives in `mem` (arena_layout(R, n).total bytes, owned by the
// caller), and the setup is only enqueued on s: nothing waits for it.
int clone_ctx(const pt_ctx *tm, uint64_t seed, int has_target, int32_t target, uint64_t cap, hipStream_t s,
              void *mem, pt_ctx **out)
{
    *out = nullptr;
    pt_ctx *c = new pt_ctx();
    c->n = tm->n;
    c->L = tm->L;
    c->R = tm->R;
    c->kind = tm->kind;
    c->D = tm->D;
    c->ncolors = tm->ncolors;
    c->betas = tm->betas;
    c->h_tswap_len = tm->h_tswap_len;
    c->opts = tm->opts;
    c->opts.seed = seed;
    c->opts.has_target = has_target;
    c->opts.target = target;
    c->clamp = tm->clamp;
    c->nfree = tm->nfree;
    c->pmJ = tm->pmJ;
    c->pmL = tm->pmL;
    c->device = tm->device;
    c->stream = s;
    c->own_stream = false;
#define VIEW(f) c->f.view(tm->f.p, tm->f.bytes)
    VIEW(J3); VIEW(row_ptr); VIEW(col); VIEW(Jc); VIEW(h); VIEW(clampd); VIEW(color_sites); VIEW(color_off); VIEW(csrw_grp);
    VIEW(tflip); VIEW(tprop); VIEW(tprop_off); VIEW(tprop_len); VIEW(tswap); VIEW(tswap_off); VIEW(tswap_len);
#undef VIEW
    const int R = c->R, n = c->n;
    const ArenaLayout A = arena_layout(R, n);
    hipError_t e = hipSuccess;
    c->arena.view(mem, A.total);
    char *base = c->arena.as<char>();
    const size_t P = (size_t)std::max(R - 1, 1);
    c->spins.view(base + A.spins, (size_t)R * n);
    c->E.view(base + A.E, (size_t)R * 4);
    c->t.view(base + A.t, 8);
    c->cursor.view(base + A.cursor, (size_t)R * 4);
    c->bank_ptrs.view(base + A.bank_ptrs, (size_t)R * 8);
    c->bankE_ptrs.view(base + A.bankE_ptrs, (size_t)R * 8);
    c->bank_n.view(base + A.bank_n, (size_t)R * 4);
    c->swap_att.view(base + A.swap_att, P * 8);
    c->swap_acc.view(base + A.swap_acc, P * 8);
    c->prop_att.view(base + A.prop_att, (size_t)R * 8);
    c->prop_acc.view(base + A.prop_acc, (size_t)R * 8);
    c->flips.view(base + A.flips, (size_t)R * 8);
    c->best.view(base + A.best, sizeof(BestRec));
    c->best_spins.view(base + A.best_spins, (size_t)n);
    c->inst.view(base + A.inst, sizeof(InstDev));
    c->banks.resize(R);
    c->h_bank_ptrs = tm->h_bank_ptrs;
    c->h_bankE_ptrs = tm->h_bankE_ptrs;
    c->h_bank_n = tm->h_bank_n;
    c->hI = tm->hI;
    c->hI.seed_lo = (uint32_t)seed;
    c->hI.seed_hi = (uint32_t)(seed >> 32);
    c->hI.has_target = has_target ? 1 : 0;
    c->hI.target = target;
    c->hI.sweep_cap = cap;
    c->hI.epoch = 0;
    c->hI.stop_at_hit = 1;     // a request ends at its first hit: later rounds leave it as it is
    fill_inst_pointers(c);
    // the request's bank cursors start at its own seeded offsets
    std::vector<int32_t> &cur = c->h_cursor0;
    cur.assign(R, 0);
    for (int r = 0; r < R; ++r)
        if (c->h_bank_n[r] > 0)
            cur[r] = (int32_t)(host_philox_word0((uint32_t)r, 0, TAG_BANK, c->hI.seed_lo, c->hI.seed_hi) %
                               (uint32_t)c->h_bank_n[r]);
    auto bail = [&](hipError_t ee) {
        delete c;
        return fail(PT_EDEVICE, "request setup: %s", hipGetErrorString(ee));
    };
    if ((e = hipMemcpyAsync(c->bank_ptrs.p, c->h_bank_ptrs.data(), (size_t)R * 8, hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(c->bankE_ptrs.p, c->h_bankE_ptrs.data(), (size_t)R * 8, hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(c->bank_n.p, c->h_bank_n.data(), (size_t)R * 4, hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(c->cursor.p, cur.data(), (size_t)R * 4, hipMemcpyHostToDevice, s)))
        return bail(e);
    int rc = reset_state(c, nullptr, 0, false);
    if (rc) {
        delete c;
        return rc;
    }
    *out = c;
    return PT_OK;
}

double seconds_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

struct SrvReq {
    uint64_t id;
    pt_request rq;
    double t_submit;
};

struct SrvActive {
    SrvReq r;
    pt_ctx *c;
    size_t bytes;
    double t_admit;
    uint64_t t_last;
    int lane;                         // the launch lane it runs in
    int cur;                          // its index in that lane's launch group as last built
    int slot[2];                      // its index in the round of each parity (-1: not in it)
    int lane_at[2];                   // its lane in the round of each parity
    int pace;                         // rank groups per sweep (sparse one-slot-per-wavefront requests), else 0
};

// A launch lane of a server: a batch over some of the running requests whose
// launch is co-resident on its own. A round runs every non-empty lane's launch
// in turn on the server's stream, so each lane keeps the fastest kernel for
// its requests (the +-J row kernel for lattices, the one-slot-per-wavefront
// sparse kernel for general graphs) instead of one mixed launch over all.
struct SrvLane {
    pt_batch *b = nullptr;
    std::string ident;                // kernel and sweeper of its launch (group_identity)
    int members = 0;
    int pace = -2;                    // its members' pace (SrvActive::pace); -1 mixed, -2 none yet
    bool dirty = false;               // membership changed since the last build
    std::set<std::string> full_for;   // request kinds it had no room for (cleared when one leaves)
    // by round parity: status records and error flag copied after its launch,
    // and events around the launch
    HostPinned status[2], err[2];
    hipEvent_t ev[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    bool ran[2] = {false, false};
    ~SrvLane()
    {
        pt_batch_destroy(b);
        for (auto &pe : ev)
            for (hipEvent_t e : pe)
                if (e) (void)hipEventDestroy(e);
    }
};

} // namespace

struct pt_server {
    pt_serve_opts opts{};
    int device = 0;
    std::chrono::steady_clock::time_point t0;
    std::vector<pt_ctx *> problems;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<SrvReq> pending;
    std::deque<pt_result> done;
    bool stopping = false;
    std::string fail_msg;             // why a failed round stopped the server
    uint64_t next_id = 1;
    pt_serve_stats st{};
    std::thread worker;
    // worker-only
    hipStream_t stream = nullptr;
    hipStream_t copy_stream = nullptr; // best configurations to callers beside a running round
    hipEvent_t round_end[2] = {nullptr, nullptr};   // after the status copies of the round of each parity
    pt_batch *probe = nullptr;        // plans single requests (no contexts of its own)
    std::vector<std::unique_ptr<SrvLane>> lanes;
    std::vector<std::string> solo;    // per problem: the kernel a request of it runs alone
    std::vector<SrvActive> active;
    // request-state arenas of retired requests, reused by later ones of the
    // same size (no device allocation or free, and so no device-wide
    // synchronisation, per request once the pool is warm); grave[q]: arenas
    // of requests retired while the round of parity q still ran over them
    // (no-ops there), pooled once it ends
    std::vector<std::pair<size_t, void *>> pool, grave[2];
    ~pt_server()
    {
        if (stream) (void)hipStreamSynchronize(stream);
        lanes.clear();
        pt_batch_destroy(probe);
        for (auto &m : pool) (void)hipFree(m.second);
        for (auto &g : grave)
            for (auto &m : g) (void)hipFree(m.second);
        for (hipEvent_t e : round_end)
            if (e) (void)hipEventDestroy(e);
        if (copy_stream) (void)hipStreamDestroy(copy_stream);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

// An arena of `bytes` for a new request: from the pool, else allocated.
static void *arena_take(pt_server *S, size_t bytes)
{
    for (size_t k = 0; k < S->pool.size(); ++k)
        if (S->pool[k].first == bytes) {
            void *p = S->pool[k].second;
            S->pool[k] = S->pool.back();
            S->pool.pop_back();
            return p;
        }
    void *p = nullptr;
    return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
}

static void serve_publish(pt_server *S, std::vector<pt_result> &res)
{
    if (res.empty()) return;
    std::lock_guard<std::mutex> lk(S->mu);
    for (auto &r : res) S->done.push_back(r);
    res.clear();
    S->cv_done.notify_all();
}

static pt_result serve_result(const SrvReq &r, int status, double t_admit, double t_done)
{
    pt_result o{};
    o.id = r.id;
    o.user_tag = r.rq.user_tag;
    o.status = status;
    o.first_hit = -1;
    o.best_energy = 0x7FFFFFFF;
    o.best_slot = -1;
    o.best_t = -1;
    o.t_submit = r.t_submit;
    o.t_admit = t_admit;
    o.t_done = t_done;
    return o;
}

// A batch object on the server's stream with its tiling options and no
// contexts: a lane (builds that do not wait for the running round), or the
// probe that plans single requests.
static int serve_new_batch(pt_server *S, pt_batch **out)
{
    *out = nullptr;
    pt_batch *b = new pt_batch();
    b->opts.replicas_per_wg = S->opts.replicas_per_wg;
    b->opts.replicas_per_thread = S->opts.replicas_per_thread;
    b->opts.chunk_sweeps = S->opts.chunk_sweeps;
    b->async_build = true;
    int rc = batch_init(b, S->device, S->stream);
    if (rc) {
        delete b;
        return rc;
    }
    *out = b;
    return PT_OK;
}

// A new empty lane, its events created.
static int serve_new_lane(pt_server *S, const std::string &ident, int &index)
{
    std::unique_ptr<SrvLane> ln(new SrvLane());
    int rc = serve_new_batch(S, &ln->b);
    if (rc) return rc;
    for (auto &pe : ln->ev)
        for (hipEvent_t &e : pe)
            if (hipEventCreate(&e) != hipSuccess) return fail(PT_EDEVICE, "event creation failed");
    ln->ident = ident;
    S->lanes.push_back(std::move(ln));
    index = (int)S->lanes.size() - 1;
    return PT_OK;
}

// The contexts of lane l in the order of the active list.
static std::vector<pt_ctx *> lane_set(const pt_server *S, int l)
{
    std::vector<pt_ctx *> set;
    for (auto &a : S->active)
        if (a.lane == l) set.push_back(a.c);
    return set;
}

// The kernel a request of problem p runs alone (empty, with the error code in
// rc, if it fits no launch by itself).
static std::string serve_solo(pt_server *S, int p, int &rc)
{
    rc = PT_OK;
    if ((int)S->solo.size() <= p) S->solo.resize(p + 1);
    if (S->solo[p].empty()) {
        LaunchGroup *g = nullptr;
        rc = pick_group(S->probe, {S->problems[p]}, &g);
        if (rc) return std::string();
        S->solo[p] = group_identity(g);
        delete g;
    }
    return S->solo[p];
}

// A request's pace in the sparse one-slot-per-wavefront kernel: the rank
// groups it sweeps per colour pass (colour classes of more than 64 sites take
// two or more). A launch lasts as long as its slowest request, so lanes keep
// requests of one pace apart where that costs no extra launch. 0 elsewhere.
static int serve_pace(const pt_ctx *c, const std::string &solo)
{
    if (solo.rfind("kernel=csrw ", 0) != 0) return 0;
    return c->ncolors * ((c->hI.maxcnt + 63) / 64);
}

// The lane a request of template tm joins: the first lane of its kind, of its
// pace first, whose launch keeps its kernel and stays co-resident with it
// added, else an empty lane (reused or new). -1 with the error code in rc
// when none can be had.
static int serve_place(pt_server *S, pt_ctx *tm, const std::string &solo, int pace, int &rc)
{
    rc = PT_OK;
    for (int pass = 0; pass < 2; ++pass)
        for (int l = 0; l < (int)S->lanes.size(); ++l) {
            SrvLane &ln = *S->lanes[l];
            // 8^3 +-J lattices run in the row kernel's lanes beside other sizes
            const bool kin = ln.ident == solo || (ln.ident.rfind("kernel=pml ", 0) == 0 && solo.rfind("kernel=pm ", 0) == 0);
            if (ln.members == 0 || !kin || ln.full_for.count(solo)) continue;
            if (pass == 0 && ln.pace != pace) continue;
            std::vector<pt_ctx *> set = lane_set(S, l);
            set.push_back(tm);
            LaunchGroup *g = nullptr;
            const bool ok = pick_group(ln.b, set, &g) == PT_OK && group_identity(g) == ln.ident;
            delete g;
            if (ok) return l;
            ln.full_for.insert(solo);
        }
    for (int l = 0; l < (int)S->lanes.size(); ++l)
        if (S->lanes[l]->members == 0) {
            S->lanes[l]->ident = solo;
            S->lanes[l]->full_for.clear();
            return l;
        }
    int l = -1;
    rc = serve_new_lane(S, solo, l);
    return rc ? -1 : l;
}

// Admit waiting requests, first come first served, while their state fits
// the memory budget (and the cap on running requests). Each joins a launch
// lane (serve_place); a request that fits no launch even alone is rejected.
static void serve_admit(pt_server *S, std::vector<pt_result> &out)
{
    for (;;) {
        SrvReq r;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            if (S->pending.empty()) return;
            r = S->pending.front();
        }
        if (S->opts.max_active > 0 && (int)S->active.size() >= S->opts.max_active) return;
        pt_ctx *tm = S->problems[r.rq.problem];
        const size_t need = arena_layout(tm->R, tm->n).total;
        int rc = PT_OK;
        if (S->st.mem_used + need > S->opts.mem_budget) {
            if (!S->active.empty()) return;   // wait for running requests to finish
            rc = fail(PT_ENOMEM, "request state of %zu bytes exceeds the memory budget", need);
        }
        int lane = -1, pace = 0;
        if (!rc) {
            // the template has the clone's shape: plan with it
            const std::string solo = serve_solo(S, r.rq.problem, rc);
            pace = serve_pace(tm, solo);
            if (!rc) lane = serve_place(S, tm, solo, pace, rc);
        }
        pt_ctx *c = nullptr;
        void *mem = nullptr;
        if (!rc) {
            mem = arena_take(S, need);
            if (!mem) rc = fail(PT_ENOMEM, "request state of %zu bytes: device allocation failed", need);
        }
        if (!rc) rc = clone_ctx(tm, r.rq.seed, r.rq.has_target, r.rq.target, r.rq.sweep_cap, S->stream, mem, &c);
        if (rc && mem) S->pool.push_back({need, mem});
        const double now = seconds_since(S->t0);
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->pending.pop_front();
            S->st.waiting = (int32_t)S->pending.size();
            if (rc) {
                S->st.rejected += 1;
            } else {
                S->st.admitted += 1;
                S->st.mem_used += need;
                S->st.mem_peak = std::max(S->st.mem_peak, S->st.mem_used);
                S->st.active = (int32_t)S->active.size() + 1;
                S->st.peak_active = std::max(S->st.peak_active, S->st.active);
            }
        }
        if (rc) {
            out.push_back(serve_result(r, rc, now, now));
            continue;
        }
        S->active.push_back({r, c, need, now, 0, lane, -1, {-1, -1}, {-1, -1}, pace});
        SrvLane &ln = *S->lanes[lane];
        ln.pace = ln.members == 0 ? pace : ln.pace == pace ? pace : -1;
        ln.members += 1;
        ln.dirty = true;
    }
}

// Keep the paces of the sparse one-slot-per-wavefront requests apart: when
// lanes of that kernel mix paces and their membership changed, refill them
// pace by pace (each lane filled to its co-resident limit) if that takes no
// more lanes than they now are. Which lane a request runs in changes none of
// its results.
static void serve_rebalance(pt_server *S)
{
    std::vector<int> ls;
    bool mixed = false, dirty = false;
    for (int l = 0; l < (int)S->lanes.size(); ++l) {
        const SrvLane &ln = *S->lanes[l];
        if (ln.members == 0 || ln.ident.rfind("kernel=csrw ", 0) != 0) continue;
        ls.push_back(l);
        mixed = mixed || ln.pace == -1;
        dirty = dirty || ln.dirty;
    }
    if (ls.size() < 2 || !mixed || !dirty) return;
    std::map<int, std::vector<int>> by_pace;   // active indices, in arrival order
    for (int k = 0; k < (int)S->active.size(); ++k)
        if (std::find(ls.begin(), ls.end(), S->active[k].lane) != ls.end()) by_pace[S->active[k].pace].push_back(k);
    std::vector<std::pair<int, std::vector<int>>> fill;   // (pace, members) per lane
    for (auto &kv : by_pace) {
        // the co-resident work items of a lane of this pace: a plan of one request
        LaunchGroup *g = nullptr;
        GroupPlan P;
        if (pick_group(S->probe, {S->active[kv.second[0]].c}, &g) != PT_OK) return;
        const int prc = g->csrw ? plan_group(S->probe, g, P) : PT_EUNSUPPORTED;
        delete g;
        if (prc) return;
        const long cap = (long)P.per_cu * S->probe->cus / 8 * 8;
        std::vector<int> cur;
        long items = 0;
        for (int k : kv.second) {
            const pt_ctx *c = S->active[k].c;
            int G = S->opts.replicas_per_wg > 0 ? S->opts.replicas_per_wg : csrw_max_storages();
            G = std::min(std::min(G, c->R), csrw_max_storages());
            const long w = (c->R + G - 1) / G;
            if (!cur.empty() && items + w > cap) {
                fill.push_back({kv.first, cur});
                cur.clear();
                items = 0;
            }
            cur.push_back(k);
            items += w;
        }
        if (!cur.empty()) fill.push_back({kv.first, cur});
    }
    if (fill.size() > ls.size()) return;   // keeping paces apart would take another launch
    for (int l : ls) {
        SrvLane &ln = *S->lanes[l];
        ln.members = 0;
        ln.pace = -2;
        ln.dirty = true;
        ln.full_for.clear();
    }
    for (size_t i = 0; i < fill.size(); ++i) {
        SrvLane &ln = *S->lanes[ls[i]];
        for (int k : fill[i].second) S->active[k].lane = ls[i];
        ln.members = (int)fill[i].second.size();
        ln.pace = fill[i].first;
    }
}

// Build the launch of every lane whose membership changed (without waiting
// for the running round: the new tables reach the device behind it). A lane
// whose remaining requests no longer fit its launch (its kernel can change as
// requests leave) gives its later half to a new lane, until every lane
// builds; a single admitted request always fits alone.
static int serve_build(pt_server *S)
{
    serve_rebalance(S);
    for (int l = 0; l < (int)S->lanes.size(); ++l) {
        SrvLane &ln = *S->lanes[l];
        if (!ln.dirty || ln.members == 0) {
            ln.dirty = false;
            continue;
        }
        std::vector<pt_ctx *> set = lane_set(S, l);
        int rc = batch_set_contexts(ln.b, set.data(), (int32_t)set.size());
        if (rc == PT_EUNSUPPORTED && set.size() > 1) {
            int nidx = -1;
            rc = serve_new_lane(S, std::string(), nidx);
            if (rc) return rc;
            int k = 0;
            const int keep = (int)set.size() / 2;
            for (auto &a : S->active)
                if (a.lane == l && k++ >= keep) a.lane = nidx;
            S->lanes[nidx]->members = (int)set.size() - keep;
            S->lanes[nidx]->pace = S->lanes[l]->pace;
            S->lanes[nidx]->dirty = true;
            S->lanes[l]->members = keep;
            --l;   // rebuild this lane with its first half
            continue;
        }
        if (rc) return rc;
        SrvLane &lb = *S->lanes[l];
        lb.ident = group_identity(lb.b->groups[0]);
        lb.dirty = false;
        int k = 0;
        for (auto &a : S->active)
            if (a.lane == l) a.cur = k++;
    }
    return PT_OK;
}

// Enqueue the round of parity q: each lane's persistent launch of
// chunk_sweeps sweeps over its requests, in turn on the server's stream,
// with its status records and error flag copied to pinned memory behind it.
static int serve_launch(pt_server *S, int q, int &lanes)
{
    const uint32_t K = (uint32_t)S->opts.chunk_sweeps;
    lanes = 0;
    for (auto &lp : S->lanes) {
        SrvLane &ln = *lp;
        ln.ran[q] = ln.members > 0;
        if (!ln.ran[q]) continue;
        LaunchGroup *g = ln.b->groups[0];
        const size_t sb = g->ctxs.size() * sizeof(InstStatus);
        HIPCHK(ln.status[q].reserve(sb));
        HIPCHK(ln.err[q].reserve(32));
        HIPCHK(hipEventRecord(ln.ev[q][0], S->stream));
        hipError_t e = enqueue_round(ln.b, K, false);
        if (e != hipSuccess) return fail(PT_EDEVICE, "serving round: %s", hipGetErrorString(e));
        HIPCHK(hipEventRecord(ln.ev[q][1], S->stream));
        HIPCHK(hipMemcpyAsync(ln.status[q].p, g->status.p, sb, hipMemcpyDeviceToHost, S->stream));
        HIPCHK(hipMemcpyAsync(ln.err[q].p, ln.b->err.p, 32, hipMemcpyDeviceToHost, S->stream));
        lanes += 1;
    }
    HIPCHK(hipEventRecord(S->round_end[q], S->stream));
    for (auto &a : S->active) {
        a.slot[q] = a.cur;
        a.lane_at[q] = a.lane;
    }
    return PT_OK;
}

// Wait for the round of parity q and retire the requests that are done. The
// round of parity q ^ 1, if next_running, was enqueued before this wait and
// runs over the retired requests as no-ops (they stop at their target or
// cap), so their arenas wait in grave[q ^ 1] until it ends; their best
// configurations go to the callers now, on the copy stream.
static int serve_finish(pt_server *S, int q, bool next_running, std::vector<pt_result> &out)
{
    HIPCHK(hipEventSynchronize(S->round_end[q]));
    for (auto &m : S->grave[q]) S->pool.push_back(m);
    S->grave[q].clear();
    double gpu_ms = 0.0;
    for (auto &lp : S->lanes) {
        SrvLane &ln = *lp;
        if (!ln.ran[q]) continue;
        if (ln.err[q].as<int>()[0]) return fail(PT_ETIMEOUT, "cross-workgroup exchange timed out in a serving round");
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, ln.ev[q][0], ln.ev[q][1]));
        gpu_ms += ms;
    }
    double attempts = 0.0;
    std::vector<SrvActive> keep, retired;
    for (auto &a : S->active) {
        if (a.slot[q] < 0) {     // admitted after the round was enqueued
            keep.push_back(a);
            continue;
        }
        const InstStatus &st = S->lanes[a.lane_at[q]]->status[q].as<InstStatus>()[a.slot[q]];
        const uint64_t t = (uint64_t)st.t;
        attempts += (double)(t - a.t_last) * (double)a.c->R * (double)a.c->nfree;
        a.t_last = t;
        const bool hit = a.r.rq.has_target && st.first_hit >= 0;
        if (!hit && t < a.r.rq.sweep_cap) {
            keep.push_back(a);
            continue;
        }
        if (a.r.rq.best_out)
            HIPCHK(hipMemcpyAsync(a.r.rq.best_out, a.c->best_spins.p, (size_t)a.c->n, hipMemcpyDeviceToHost,
                                  S->copy_stream));
        pt_result o = serve_result(a.r, PT_OK, a.t_admit, 0.0);
        o.hit = hit ? 1 : 0;
        o.first_hit = st.first_hit;
        o.best_energy = st.best_E;
        o.best_slot = st.best_slot;
        o.best_t = st.best_t;
        o.sweeps = t;
        out.push_back(o);
        retired.push_back(a);
        SrvLane &ln = *S->lanes[a.lane];
        ln.members -= 1;
        ln.dirty = true;
        ln.full_for.clear();
    }
    if (!retired.empty()) HIPCHK(hipStreamSynchronize(S->copy_stream));
    const double t_done = seconds_since(S->t0);
    for (size_t k = out.size() - retired.size(); k < out.size(); ++k) out[k].t_done = t_done;
    for (auto &a : retired) {
        (next_running ? S->grave[q ^ 1] : S->pool).push_back({a.bytes, a.c->arena.p});
        delete a.c;                  // views only: frees no device memory
    }
    S->active.swap(keep);
    std::lock_guard<std::mutex> lk(S->mu);
    for (auto &a : retired) {
        S->st.mem_used -= a.bytes;
        S->st.completed += 1;
    }
    S->st.gpu_busy_s += gpu_ms * 1e-3;
    S->st.attempts += attempts;
    S->st.active = (int32_t)S->active.size();
    return PT_OK;
}

// The worker. Each turn admits waiting requests, builds the lanes that
// changed and enqueues a round. One round at a time (the default), it then
// waits for that round and retires what it finished. Pipelined, it waits
// instead for the round before, so the device runs the next round while the
// host handles the last; a request is then in the round after the one that
// finished it as a no-op, which changes nothing it reports, and a new request
// joins one round later.
static void serve_worker(pt_server *S)
{
    (void)hipSetDevice(S->device);
    std::vector<pt_result> out;
    int q = 0;                   // parity of the next round
    bool running = false;        // the round of parity q ^ 1 is in flight
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->active.empty() && S->pending.empty() && !running) {
                if (S->stopping) break;
                S->cv_work.wait(lk, [&] { return S->stopping || !S->pending.empty(); });
                continue;
            }
        }
        const double ta = seconds_since(S->t0);
        serve_admit(S, out);
        serve_publish(S, out);
        int rc = PT_OK, lanes = 0;
        bool launched = false;
        if (!S->active.empty()) {
            rc = serve_build(S);
            if (!rc) rc = serve_launch(S, q, lanes);
            launched = rc == PT_OK;
        }
        if (!rc && running) rc = serve_finish(S, q ^ 1, launched, out);
        if (!rc && launched && !S->opts.pipeline) {   // one round at a time
            rc = serve_finish(S, q, false, out);
            launched = false;
            if (!rc) {
                std::lock_guard<std::mutex> lk(S->mu);
                S->st.rounds += 1;
                S->st.peak_lanes = std::max(S->st.peak_lanes, (int32_t)lanes);
            }
        }
        if (rc) {
            // a failed round fails every request in it; the device state of
            // the launch is unknown, so the server takes no more work
            (void)hipStreamSynchronize(S->stream);
            const double now = seconds_since(S->t0);
            for (auto &a : S->active) {
                out.push_back(serve_result(a.r, rc, a.t_admit, now));
                a.c->broken = true;
                S->pool.push_back({a.bytes, a.c->arena.p});
                pt_destroy(a.c);
            }
            S->active.clear();
            for (auto &ln : S->lanes) ln->members = 0;
            const std::string why = pt_last_error();
            std::lock_guard<std::mutex> lk(S->mu);
            S->fail_msg = why;
            for (auto &r : S->pending) out.push_back(serve_result(r, rc, now, now));
            S->st.rejected += S->pending.size();
            S->pending.clear();
            S->stopping = true;
            running = false;
        } else {
            running = launched;
            if (launched) q ^= 1;
            std::lock_guard<std::mutex> lk(S->mu);
            if (launched) {
                S->st.rounds += 1;
                S->st.peak_lanes = std::max(S->st.peak_lanes, (int32_t)lanes);
            }
            S->st.busy_s += seconds_since(S->t0) - ta;
        }
        serve_publish(S, out);
    }
}

extern "C" int pt_serve_start(const pt_serve_opts *o, pt_server **out)
{
    if (!out) return fail(PT_EINVAL, "null output pointer");
    *out = nullptr;
    pt_server *S = new pt_server();
    if (o) S->opts = *o;
    if (S->opts.mem_budget == 0) S->opts.mem_budget = 1ull << 30;
    if (S->opts.chunk_sweeps <= 0) S->opts.chunk_sweeps = 500;
    if (hipGetDevice(&S->device) != hipSuccess) {
        delete S;
        return fail(PT_EDEVICE, "no HIP device");
    }
    int rc = PT_OK;
    if (hipSetDevice(S->device) != hipSuccess || hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&S->copy_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&S->round_end[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&S->round_end[1], hipEventDisableTiming) != hipSuccess)
        rc = fail(PT_EDEVICE, "stream or event creation failed");
    if (!rc) rc = serve_new_batch(S, &S->probe);
    if (rc) {
        delete S;
        return rc;
    }
    S->t0 = std::chrono::steady_clock::now();
    S->worker = std::thread(serve_worker, S);
    *out = S;
    return PT_OK;
}

extern "C" int pt_serve_register(pt_server *s, pt_ctx *ctx, int32_t *problem)
{
    if (!s || !ctx || !problem) return fail(PT_EINVAL, "null argument");
    if (ctx->broken) return fail(PT_ESTATE, "context is unusable");
    if (ctx->device != s->device) return fail(PT_EINVAL, "context lives on another device");
    HIPCHK(hipStreamSynchronize(ctx->stream));
    std::lock_guard<std::mutex> lk(s->mu);
    s->problems.push_back(ctx);
    *problem = (int32_t)s->problems.size() - 1;
    return PT_OK;
}

extern "C" int pt_serve_submit(pt_server *s, const pt_request *rq, uint64_t *id)
{
    if (!s || !rq) return fail(PT_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping)
        return fail(PT_ESTATE, s->fail_msg.empty() ? "server is stopping" : "server stopped after a failed round: %s",
                    s->fail_msg.c_str());
    if (rq->problem < 0 || rq->problem >= (int32_t)s->problems.size()) return fail(PT_EINVAL, "unknown problem %d", rq->problem);
    if (rq->sweep_cap < 1 || rq->sweep_cap > 0xFFFFFFFFull) return fail(PT_EINVAL, "sweep_cap must be in 1..2^32-1");
    SrvReq r;
    r.id = s->next_id++;
    r.rq = *rq;
    r.t_submit = seconds_since(s->t0);
    s->pending.push_back(r);
    s->st.submitted += 1;
    s->st.waiting = (int32_t)s->pending.size();
    if (id) *id = r.id;
    s->cv_work.notify_one();
    return PT_OK;
}

extern "C" int pt_serve_poll(pt_server *s, pt_result *out, int32_t max, int32_t wait_ms, int32_t *n_out)
{
    if (!s || !n_out || (max > 0 && !out)) return fail(PT_EINVAL, "null argument");
    std::unique_lock<std::mutex> lk(s->mu);
    if (wait_ms > 0 && s->done.empty())
        s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !s->done.empty(); });
    int n = 0;
    while (n < max && !s->done.empty()) {
        out[n++] = s->done.front();
        s->done.pop_front();
    }
    *n_out = n;
    return PT_OK;
}

extern "C" int pt_serve_stats_get(pt_server *s, pt_serve_stats *st)
{
    if (!s || !st) return fail(PT_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *st = s->st;
    return PT_OK;
}

extern "C" double pt_serve_clock(pt_server *s) { return s ? seconds_since(s->t0) : 0.0; }

extern "C" int pt_serve_stop(pt_server *s)
{
    if (!s) return PT_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
        s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    for (auto &a : s->active) {
        s->pool.push_back({a.bytes, a.c->arena.p});
        pt_destroy(a.c);
    }
    delete s;
    return PT_OK;
}
