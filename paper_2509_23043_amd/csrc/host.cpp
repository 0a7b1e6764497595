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
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "tapt.h"
#include "tapt_dev.h"

namespace tapt {
bool lattice_supported(int L);
int lattice_max_threads();
int lattice_threads(int L, int G, int rpt);
size_t chunk_lds_bytes(int kind, int n, int G, int stride, int tsw_entries);
hipError_t launch_chunk(int kind, int L, int rpt, const ChunkArgs &a, int block, size_t lds, hipStream_t s);
hipError_t chunk_occupancy(int kind, int L, int rpt, int block, size_t lds, int *blocks_per_cu);
hipError_t launch_finish(const WorkItem *items, const int *first_item, int n_inst, uint32_t K, hipStream_t s);
hipError_t launch_plain(int kind, int L, const InstDev *dI, int R, int n, int stride, uint32_t t, hipStream_t s);
hipError_t launch_init(const InstDev *dI, int R, int n, hipStream_t s);
hipError_t launch_energy(const InstDev *dI, const int8_t *cfg, int k, int32_t *out, hipStream_t s);
hipError_t launch_init_best(const InstDev *dI, hipStream_t s);
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

// entries T(exp(-a d)) for d = 1, 2, ... up to the last nonzero one
static void tail_table(double a, std::vector<uint32_t> &out)
{
    for (long long d = 1;; ++d) {
        uint32_t T = threshold(std::exp(-(a * (double)d)));
        if (T == 0) break;
        out.push_back(T);
        if (out.size() > (1u << 22)) break;
    }
}

// ---------------------------------------------------------------------------
// device buffer helper

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    ~DevBuf() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    hipError_t alloc(size_t b)
    {
        release();
        bytes = b;
        return hipMalloc(&p, b ? b : 16);
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

    // device allocations
    DevBuf J3, row_ptr, col, Jc, h, clampd, color_sites, color_off;
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
};

static int push_inst(pt_ctx *c)
{
    HIPCHK(hipMemcpyAsync(c->inst.p, &c->hI, sizeof(InstDev), hipMemcpyHostToDevice, c->stream));
    return PT_OK;
}

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
    int64_t nfree;
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
    P.row_ptr = rp;
    P.col.resize(cl.size());
    P.Jc.resize(jv.size());
    for (size_t k = 0; k < cl.size(); ++k) {
        P.col[k] = (int16_t)cl[k];
        P.Jc[k] = (int8_t)jv[k];
    }
    P.color_off.assign(nc + 1, 0);
    for (int c = 0; c < nc; ++c) {
        for (int i = 0; i < n; ++i)
            if (color[i] == c && !P.clamp[i]) P.color_sites.push_back((int16_t)i);
        P.color_off[c + 1] = (int32_t)P.color_sites.size();
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

// zero counters, initialise spins (or take them from `spins`), energies, best
static int reset_state(pt_ctx *c, const int8_t *spins, uint64_t t)
{
    hipStream_t s = c->stream;
    const int R = c->R, n = c->n;
    HIPCHK(hipMemsetAsync(c->swap_att.p, 0, c->swap_att.bytes, s));
    HIPCHK(hipMemsetAsync(c->swap_acc.p, 0, c->swap_acc.bytes, s));
    HIPCHK(hipMemsetAsync(c->prop_att.p, 0, c->prop_att.bytes, s));
    HIPCHK(hipMemsetAsync(c->prop_acc.p, 0, c->prop_acc.bytes, s));
    HIPCHK(hipMemsetAsync(c->flips.p, 0, c->flips.bytes, s));
    unsigned long long tt = t;
    HIPCHK(hipMemcpyAsync(c->t.p, &tt, 8, hipMemcpyHostToDevice, s));
    c->hI.epoch += 1;
    int rc = push_inst(c);
    if (rc) return rc;
    if (spins)
        HIPCHK(hipMemcpyAsync(c->spins.p, spins, (size_t)R * n, hipMemcpyHostToDevice, s));
    else
        HIPCHK(launch_init(c->inst.as<InstDev>(), R, n, s));
    HIPCHK(launch_energy(c->inst.as<InstDev>(), c->spins.as<int8_t>(), R, c->E.as<int32_t>(), s));
    HIPCHK(launch_init_best(c->inst.as<InstDev>(), s));
    HIPCHK(hipStreamSynchronize(s));
    c->t_host = t;
    return PT_OK;
}

extern "C" int pt_create(const pt_graph *g, const double *betas, int32_t R, const pt_opts *o, pt_ctx **out)
{
    if (!out) return fail(PT_EINVAL, "null output pointer");
    *out = nullptr;
    if (!betas || !o) return fail(PT_EINVAL, "null betas or options");
    if (R < 1 || R > 1024) return fail(PT_EINVAL, "R must be in 1..1024 (got %d)", R);
    for (int r = 0; r < R; ++r) {
        if (!(betas[r] > 0.0) || !std::isfinite(betas[r])) return fail(PT_EINVAL, "beta[%d] must be finite and > 0", r);
        if (r && !(betas[r] > betas[r - 1])) return fail(PT_EINVAL, "betas must be strictly increasing");
    }
    if (o->rule != PT_METROPOLIS && o->rule != PT_GIBBS) return fail(PT_EINVAL, "unknown rule %d", o->rule);
    if (o->sweeps_per_cycle < 1) return fail(PT_EINVAL, "sweeps_per_cycle must be >= 1");
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
    auto bail = [&](int code) {
        delete c;
        return code;
    };
    if (hipGetDevice(&c->device) != hipSuccess) return bail(fail(PT_EDEVICE, "no HIP device"));
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(PT_EDEVICE, "stream creation failed"));
    c->own_stream = true;
    hipStream_t s = c->stream;

    // tables
    const int stride = 2 * P.D + 1;
    std::vector<uint32_t> tflip((size_t)R * stride);
    for (int r = 0; r < R; ++r)
        for (int k = 0; k < stride; ++k)
            tflip[(size_t)r * stride + k] = threshold(flip_probability(o->rule, betas[r], 2LL * (k - P.D)));
    std::vector<uint32_t> tprop, tswap;
    std::vector<int32_t> tprop_off(R), tprop_len(R), tswap_off(std::max(R - 1, 1)), tswap_len(std::max(R - 1, 1));
    for (int r = 0; r < R; ++r) {
        tprop_off[r] = (int32_t)tprop.size();
        tail_table(betas[r], tprop);
        tprop_len[r] = (int32_t)tprop.size() - tprop_off[r];
    }
    for (int r = 0; r + 1 < R; ++r) {
        tswap_off[r] = (int32_t)tswap.size();
        tail_table(betas[r + 1] - betas[r], tswap);
        tswap_len[r] = (int32_t)tswap.size() - tswap_off[r];
    }
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
    I.M = o->sweeps_per_cycle;
    I.D = P.D;
    I.tflip_stride = stride;
    I.has_target = o->has_target ? 1 : 0;
    I.target = o->target;
    I.ncolors = P.ncolors;
    I.nfree = (int32_t)P.nfree;
    I.nnz = (int32_t)P.col.size();
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

extern "C" int pt_sweep(pt_ctx *c, uint64_t n_sweeps)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (c->t_host + n_sweeps > 0xFFFFFFFFull) return fail(PT_EINVAL, "sweep counter would exceed 2^32-1");
    hipStream_t s = c->stream;
    const int stride = 2 * c->D + 1;
    for (uint64_t k = 0; k < n_sweeps; ++k) {
        uint32_t t = (uint32_t)(c->t_host + k + 1);
        hipError_t e = launch_plain(c->kind, c->L, c->inst.as<InstDev>(), c->R, c->n, stride, t, s);
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
    size_t lds;
    std::vector<pt_ctx *> ctxs;
    std::vector<int> Gs;              // per context: slots per workgroup (max)
    DevBuf items, order, first_item, best, best_spins, xbuf;
    std::vector<size_t> x_off, x_bytes;   // per context: its exchange words
    std::vector<uint32_t> x_epoch;        // epoch the exchange words were cleared for
    int n_items = 0;
};

struct pt_batch {
    std::vector<pt_ctx *> ctxs;
    std::vector<LaunchGroup *> groups;
    pt_batch_opts opts{};
    hipStream_t stream = nullptr;
    DevBuf err;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    uint32_t graph_K = 0;
    int device = 0;
    int cus = 0;
    hipStream_t own_stream = nullptr;
    std::vector<hipEvent_t> ev_pool;  // start/stop pairs of timed launches
    size_t ev_used = 0;
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

// Choose (slots per workgroup, slots per thread) for a context.
static void choose_tiling(const pt_ctx *c, const pt_batch_opts &o, int &G, int &rpt)
{
    const int R = c->R;
    rpt = o.replicas_per_thread > 0 ? o.replicas_per_thread : 0;
    G = o.replicas_per_wg > 0 ? std::min(std::min(o.replicas_per_wg, R), 64) : 0;
    if (c->kind == KIND_CSR) {
        rpt = 1;
        if (!G) G = std::min(R, 32);
        return;
    }
    // the cycle-end stages keep one slot per lane of a wavefront: G <= 64
    const int NC = c->n / 8;
    const int maxt = lattice_max_threads();
    if (!rpt) rpt = 2;
    if (!G) {
        // whole ladder in one workgroup when it fits the block limit, else split
        int maxg = (maxt / NC) * rpt;
        G = std::min(R, std::max(rpt, maxg));
    }
    G = std::min(G, 64);
    while (((G + rpt - 1) / rpt) * NC > maxt && G > 1) --G;
}

static int build_group(pt_batch *b, LaunchGroup *g)
{
    hipStream_t s = b->stream;
    // items: per context, W workgroups with near-equal slot counts
    std::vector<WorkItem> items;
    std::vector<int> first;
    int maxG = 1;
    size_t nbest = 0, nbs = 0, nx = 0;
    struct Pend { int first, W, n, xwords; size_t bs_off, x_off; };
    std::vector<Pend> pend;
    for (size_t k = 0; k < g->ctxs.size(); ++k) {
        pt_ctx *c = g->ctxs[k];
        int R = c->R, W = (R + g->Gs[k] - 1) / g->Gs[k];
        int xwords = (((c->n + 31) >> 5) + 1 + 7) & ~7;
        pend.push_back({(int)items.size(), W, c->n, xwords, nbs, nx});
        first.push_back((int)items.size());
        int base = R / W, extra = R % W, s0 = 0;
        for (int w = 0; w < W; ++w) {
            int G = base + (w < extra ? 1 : 0);
            WorkItem it{};
            it.inst = c->inst.as<InstDev>();
            it.s0 = s0;
            it.G = G;
            it.w = w;
            it.W = W;
            it.xwords = xwords;
            items.push_back(it);
            maxG = std::max(maxG, G);
            s0 += G;
            nbs += (size_t)((c->n + 15) & ~15);
        }
        nbest += W;
        nx += (size_t)W * 4 * xwords * 8;
    }
    HIPCHK(g->best.alloc(nbest * sizeof(BestRec)));
    HIPCHK(g->best_spins.alloc(nbs));
    HIPCHK(g->xbuf.alloc(nx));
    HIPCHK(hipMemsetAsync(g->xbuf.p, 0, nx, s));
    size_t bi = 0;
    for (size_t k = 0; k < g->ctxs.size(); ++k) {
        const Pend &p = pend[k];
        size_t bs_off = p.bs_off;
        for (int w = 0; w < p.W; ++w) {
            WorkItem &it = items[p.first + w];
            it.best = g->best.as<BestRec>() + bi++;
            it.best_spins = g->best_spins.as<int8_t>() + bs_off;
            bs_off += (size_t)((p.n + 15) & ~15);
            it.xbuf = (unsigned long long *)(g->xbuf.as<int8_t>() + p.x_off);
        }
        g->x_off.push_back(p.x_off);
        g->x_bytes.push_back((size_t)p.W * 4 * p.xwords * 8);
        g->x_epoch.push_back(g->ctxs[k]->hI.epoch);
    }
    g->n_items = (int)items.size();
    // XCD-aware order: workgroups are dispatched round-robin over the 8 XCDs,
    // so blockIdx b runs on XCD b % 8. Each XCD gets a contiguous run of the
    // instance-ordered items (so the workgroups of one instance share an L2);
    // blocks past the end of a run are padding that exits at once.
    const int nx8 = 8;
    int per = (g->n_items + nx8 - 1) / nx8;
    std::vector<int32_t> order((size_t)per * nx8, -1);
    for (int idx = 0; idx < g->n_items; ++idx) order[(size_t)(idx % per) * nx8 + idx / per] = idx;
    g->grid = per * nx8;
    HIPCHK(upload(g->items, items, s));
    HIPCHK(upload(g->order, order, s));
    HIPCHK(upload(g->first_item, first, s));
    // launch shape
    int stride_max = 1;
    for (auto *c : g->ctxs) stride_max = std::max(stride_max, 2 * c->D + 1);
    int n = g->ctxs[0]->n;
    if (g->kind == KIND_LATTICE) {
        g->block = (lattice_threads(g->L, maxG, g->rpt) + 63) & ~63;
    } else {
        int nmax = 0;
        for (auto *c : g->ctxs) nmax = std::max(nmax, c->n);
        n = nmax;
        g->block = 256;
    }
    // LDS swap-table rows: pairs s0-1 .. s0+G-1 of each workgroup
    int tsw_max = 0;
    for (size_t k = 0; k < g->ctxs.size(); ++k) {
        const Pend &p = pend[k];
        pt_ctx *c = g->ctxs[k];
        for (int w = 0; w < p.W; ++w) {
            const WorkItem &it = items[p.first + w];
            int tot = 0;
            for (int r = it.s0 - 1; r <= it.s0 + it.G - 1; ++r)
                if (r >= 0 && r + 1 < c->R) tot += c->h_tswap_len[r];
            tsw_max = std::max(tsw_max, tot);
        }
    }
    g->tsw_entries = tsw_max;
    g->lds = chunk_lds_bytes(g->kind, n, maxG, stride_max, tsw_max);
    if (g->lds > 160 * 1024) return fail(PT_EUNSUPPORTED, "tiling needs %zu B of LDS per workgroup", g->lds);
    int per_cu = 0;
    HIPCHK(chunk_occupancy(g->kind, g->L, g->rpt, g->block, g->lds, &per_cu));
    if (per_cu < 1) return fail(PT_EUNSUPPORTED, "kernel cannot run with block %d, LDS %zu", g->block, g->lds);
    if ((long long)per_cu * b->cus < g->grid)
        return fail(PT_EUNSUPPORTED, "%d workgroups exceed the %d that can be co-resident; use fewer contexts per batch",
                    g->grid, per_cu * b->cus);
    HIPCHK(hipStreamSynchronize(s));
    return PT_OK;
}

extern "C" int pt_batch_create(pt_ctx *const *ctxs, int32_t k, const pt_batch_opts *o, pt_batch **out)
{
    if (!out) return fail(PT_EINVAL, "null output pointer");
    *out = nullptr;
    if (!ctxs || k < 1) return fail(PT_EINVAL, "need at least one context");
    pt_batch *b = new pt_batch();
    if (o) b->opts = *o;
    if (b->opts.chunk_sweeps <= 0) b->opts.chunk_sweeps = 1000;
    auto bail = [&](int code) {
        delete b;
        return code;
    };
    for (int i = 0; i < k; ++i) {
        if (!ctxs[i] || ctxs[i]->broken) return bail(fail(PT_EINVAL, "context %d missing or unusable", i));
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return bail(fail(PT_EINVAL, "context %d appears twice", i));
        b->ctxs.push_back(ctxs[i]);
    }
    b->device = ctxs[0]->device;
    if (hipSetDevice(b->device) != hipSuccess) return bail(fail(PT_EDEVICE, "hipSetDevice"));
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, b->device) != hipSuccess) return bail(fail(PT_EDEVICE, "device properties"));
    b->cus = prop.multiProcessorCount;
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(PT_EDEVICE, "stream creation failed"));
    b->own_stream = b->stream;
    if (b->err.alloc(32) != hipSuccess) return bail(fail(PT_ENOMEM, "error flag"));
    if (hipMemset(b->err.p, 0, 32) != hipSuccess) return bail(fail(PT_EDEVICE, "memset"));
    // group contexts by kernel instantiation
    std::map<std::tuple<int, int, int>, LaunchGroup *> gm;
    for (pt_ctx *c : b->ctxs) {
        int G, rpt;
        choose_tiling(c, b->opts, G, rpt);
        auto key = std::make_tuple(c->kind, c->kind == KIND_LATTICE ? c->L : 0, rpt);
        LaunchGroup *&g = gm[key];
        if (!g) {
            g = new LaunchGroup();
            g->kind = c->kind;
            g->L = c->kind == KIND_LATTICE ? c->L : 0;
            g->rpt = rpt;
            b->groups.push_back(g);
        }
        g->ctxs.push_back(c);
        g->Gs.push_back(G);
    }
    for (auto *g : b->groups) {
        int rc = build_group(b, g);
        if (rc) return bail(rc);
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
        hipError_t e = launch_chunk(g->kind, g->L, g->rpt, a, g->block, g->lds, b->stream);
        if (e != hipSuccess) return e;
        if (timed) {
            e = hipEventRecord(e1, b->stream);
            if (e != hipSuccess) return e;
        }
        e = launch_finish(g->items.as<WorkItem>(), g->first_item.as<int>(), (int)g->ctxs.size(), K, b->stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

extern "C" int pt_batch_sweep(pt_batch *b, uint64_t n_sweeps)
{
    if (!b) return fail(PT_EINVAL, "null batch");
    HIPCHK(hipSetDevice(b->device));
    if (n_sweeps == 0) return PT_OK;
    // every context stops exactly at its own t + n_sweeps
    for (pt_ctx *c : b->ctxs) {
        if (c->broken) return fail(PT_ESTATE, "a context of the batch is unusable");
        if (c->t_host + n_sweeps > 0xFFFFFFFFull) return fail(PT_EINVAL, "sweep counter would exceed 2^32-1");
        HIPCHK(hipStreamSynchronize(c->stream));
        c->hI.sweep_cap = c->t_host + n_sweeps;
        HIPCHK(hipMemcpyAsync(c->inst.p, &c->hI, sizeof(InstDev), hipMemcpyHostToDevice, b->stream));
    }
    // a replaced state restarts the cycle count: clear that instance's exchange words
    for (auto *g : b->groups)
        for (size_t k = 0; k < g->ctxs.size(); ++k)
            if (g->x_epoch[k] != g->ctxs[k]->hI.epoch) {
                HIPCHK(hipMemsetAsync(g->xbuf.as<int8_t>() + g->x_off[k], 0, g->x_bytes[k], b->stream));
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
            hipError_t e = enqueue_round(b, K, true);
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
                    "cross-workgroup exchange timed out: item %d (workgroup %d of its instance) waiting on side %d "
                    "at cycle %d saw word %08x:%08x, epoch %d",
                    err[1], err[2], err[3], err[4], (unsigned)err[6], (unsigned)err[5], err[7]);
    }
    return PT_OK;
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

extern "C" int pt_batch_destroy(pt_batch *b)
{
    if (!b) return PT_OK;
    (void)hipSetDevice(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    delete b;
    return PT_OK;
}
