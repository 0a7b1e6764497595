// Persistent kernel for general sparse graphs with one beta slot per
// wavefront. Where the workgroup-synchronous sweepers separate every colour
// class with a workgroup barrier and spread a slot over several wavefronts,
// here a wavefront sweeps its own slot alone: the colour classes follow one
// another in program order (LDS operations of a wavefront complete in order),
// so a class costs the chain of its items' LDS reads and nothing more.
//
// Sweep. Lane q takes the sites of rank q, q + 64, ... of every colour class
// (Methods, Graph coloring). Their rows are packed once per launch in LDS,
// shared by the workgroup's slots of the instance: record (c, s) holds the
// s-th site of class c with h_i, and its bonds in chunks of CSRW_CHUNK: the
// neighbours as 16-bit words and the couplings as bytes (unused bonds: site
// 0 with J = 0). A neighbour's LDS address is one add of a 16-bit half to the
// slot's base, and four spins packed by v_perm meet their four couplings in
// one 8-bit dot product. The 64 sites of a rank group (c, k) take the chunks their
// largest degree needs; within a class the host orders sites by degree, so
// the few high-degree sites of a circuit (a multiplier's input bits) share
// groups and the rest take one chunk. A lane reads the next item's first two
// chunks while it decides the current one, so an item costs one LDS round
// trip: the neighbour spins with the own spin and random half. The flip
// decision (Eqs. 4-5) comes from the flip probability evaluated in FP32 with a
// relative margin, which settles it as the slot's uint32 threshold table would
// for all but about one uniform in 10^4; only those items read the table (a
// second round trip). The slot's sweep uniforms (Philox call q serves sites
// 8q .. 8q + 7) are staged in LDS in site order, drawn at the start of the
// sweep or, after a cycle end with a partner, while the slot waits for it.
//
// Slots and states as in the +-J row kernel: states move between LDS buffers,
// pairs inside the workgroup meet in an LDS mailbox (energy, buffer index),
// pairs across a workgroup boundary exchange cycle-tagged words through
// global memory and copy the state on acceptance (Eq. 1); here lane q's word
// holds the signs of its sites q + 64k, bit k mod 32. Proposals (Eq. 2) copy
// the bank configuration into the slot's buffer.
#include "sweep.h"

namespace tapt {

namespace csrw {

constexpr int MAXG = 8;   // slots (wavefronts) per workgroup
constexpr int RULE_GIBBS = 1;              // heat-bath rule (Methods Eq. 5); 0: Metropolis
constexpr float MARGIN = 1.0f / 4096.0f;   // relative margin of the FP32 flip decision

struct Off {
    size_t sp, rnd, bw, bj, info, tab, toff, tsw, mail, xst, total;
};

// n sites, ncolors classes of at most ipl * 64 sites, chunks bond chunks, G slots
__host__ __device__ inline Off offsets(int n, int ncolors, int ipl, int chunks, int G, int stride, int tsw_entries)
{
    const int SB = (n + 16) & ~15, nr = (n + 7) & ~7;     // spins, then at least one padding byte
    const int wpl = (n + 64 * 32 - 1) / (64 * 32);        // exchange words per lane
    const size_t nrec = (size_t)ncolors * 64 * ipl;
    Off f;
    size_t o = 0;
    f.sp = o; o = align16(o + (size_t)G * SB);
    f.rnd = o; o = align16(o + (size_t)G * nr * 2);
    // one chunk of padding: a group's second chunk is read whether or not it has one
    f.bw = o; o = align16(o + (size_t)(chunks + 1) * 64 * 16);
    f.bj = o; o = align16(o + (size_t)(chunks + 1) * 64 * 8);
    f.info = o; o = align16(o + nrec * 4);
    f.tab = o; o = align16(o + (size_t)G * stride * 4);
    f.toff = o; o = align16(o + (size_t)(G + 2) * 4);
    f.tsw = o; o = align16(o + (size_t)tsw_entries * 4);
    f.mail = o; o = align16(o + (size_t)4 * G * 8);
    f.xst = o; o = align16(o + (size_t)2 * G * (64 * wpl + 1) * 4);
    f.total = o;
    return f;
}

// a rank group's first two bond chunks and its site word, read one group ahead
struct Rows {
    uint4 b0, b1;
    uint2 j0, j1;
    uint32_t inf;
    int gcb;
};

struct Rec {
    int E, slot;
    long long t, hit;
};

// The low bytes of four values (spins +-1) as one word, a in byte 0.
__device__ __forceinline__ uint32_t pack4(int a, int b, int c, int d)
{
    return __builtin_amdgcn_perm((uint32_t)b, (uint32_t)a, 0x0c0c0400u) |
           (__builtin_amdgcn_perm((uint32_t)d, (uint32_t)c, 0x0c0c0400u) << 16);
}

// Swap acceptance (Eq. 1) for dE = E_{r+1} - E_r with the pair's LDS table
// row (off, len); every input is wave-uniform and the result is a scalar.
__device__ __forceinline__ bool swap_ok(int dE, uint32_t u, int off, int len, const uint32_t *tsw)
{
    const int d = -dE;
    const bool in_row = d >= 1 && d <= len;
    const uint32_t Tr = tsw[in_row ? off + d - 1 : 0];
    const uint32_t T = dE >= 0 ? ALWAYS : (in_row ? Tr : 0u);
    const bool ok = T == ALWAYS || u < T;
    return __builtin_amdgcn_readfirstlane(ok ? 1 : 0) != 0;
}

} // namespace csrw

__global__ void __launch_bounds__(64 * csrw::MAXG) csrw_kernel(ChunkArgs a)
{
    using namespace csrw;
    constexpr int NP = 2;                     // pairs a slot takes part in
    const int item = a.order[blockIdx.x];
    if (item < 0) return;
    const WorkItem it = a.items[item];
    const InstDev &I = *it.inst;
    RunParams P;
    P.load(I);
    const int G = it.G, s0 = it.s0, n = P.n;
    const int tid = threadIdx.x, bs = blockDim.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const uint64_t t0 = *I.t;
    const uint64_t cap = chunk_cap(I, t0);
    const uint64_t tend = (t0 + a.K < cap) ? t0 + a.K : cap;
    if (t0 >= tend) {
        if (tid == 0) idle_best(it.best);
        return;
    }
    const int ncol = I.ncolors, ipl = (I.maxcnt + 63) / 64, ngr = ncol * ipl;
    const int SB = (n + 16) & ~15, nr = (n + 7) & ~7;     // spins, then at least one padding byte
    const int spl = (n + 63) / 64;                            // sites per lane
    const int wpl = (spl + 31) / 32;                          // exchange words per lane
    const int NXW = 64 * wpl;                                 // words of a state, before the energy word
    const int stride = P.stride, D = P.D;
    const Off lof = offsets(n, ncol, ipl, I.csrw_chunks, G, stride, a.tsw_entries);
    int8_t *sp = (int8_t *)(lds_raw + lof.sp);                 // [G][SB] spins +-1, site order
    uint16_t *rnd = (uint16_t *)(lds_raw + lof.rnd);          // [G][nr] sweep uniforms (upper halves)
    uint4 *bw = (uint4 *)(lds_raw + lof.bw);                  // [chunks][64] neighbours, CSRW_CHUNK 16-bit words
    uint2 *bj = (uint2 *)(lds_raw + lof.bj);                  // [chunks][64] couplings, CSRW_CHUNK bytes
    uint32_t *info = (uint32_t *)(lds_raw + lof.info);        // [ncol][64 ipl] site | h << 16; 0xFFF: none
    uint32_t *tab = (uint32_t *)(lds_raw + lof.tab);          // [G][stride] flip thresholds
    int *tsw_off = (int *)(lds_raw + lof.toff);
    uint32_t *tsw = (uint32_t *)(lds_raw + lof.tsw);
    unsigned long long *mail = (unsigned long long *)(lds_raw + lof.mail);   // [4][G]
    uint32_t *xstage = (uint32_t *)(lds_raw + lof.xst);       // [G][2 sides][NXW + 1]

    // ---- stage: states (slot l in buffer l), packed rows, tables ----
    for (int x = tid; x < G * n; x += bs) {
        const int l = x / n, i = x - l * n;
        sp[l * SB + i] = I.spins[(size_t)(s0 + l) * n + i];
    }
    // record x = 64 g + q: lane q of rank group g = (c, k), class c's site 64 k + q
    for (int x = tid; x < 64 * ngr; x += bs) {
        const int g = x >> 6, q = x & 63;
        const int c = g / ipl, s = (g - c * ipl) * 64 + q;
        const int gcb = I.csrw_groups[g], cb = gcb >> 8, nch = gcb & 255;
        const int off = I.color_off[c], cnt = I.color_off[c + 1] - off;
        uint32_t inf = 0xFFFu;
        int e0 = 0, e1 = 0;
        if (s < cnt) {
            const int i = I.color_sites[off + s];
            e0 = I.row_ptr[i];
            e1 = I.row_ptr[i + 1];
            inf = (uint32_t)i | ((uint32_t)(uint16_t)I.h[i] << 16);
        }
        for (int j = 0; j < nch; ++j) {
            uint32_t w[4] = {0, 0, 0, 0}, jv[2] = {0, 0};
            for (int b = 0; b < CSRW_CHUNK; ++b) {
                const int e = e0 + CSRW_CHUNK * j + b;
                if (e < e1) {
                    w[b >> 1] |= (uint32_t)(uint16_t)I.col[e] << (16 * (b & 1));
                    jv[b >> 2] |= (uint32_t)(uint8_t)I.Jc[e] << (8 * (b & 3));
                }
            }
            bw[(cb + j) * 64 + q] = make_uint4(w[0], w[1], w[2], w[3]);
            bj[(cb + j) * 64 + q] = make_uint2(jv[0], jv[1]);
        }
        info[x] = inf;
    }
    // group g's first chunk << 8 | chunks, in lane g
    const int gcb_v = lane < ngr ? I.csrw_groups[lane] : 0;
    for (int x = tid; x < G * stride; x += bs) tab[x] = I.tflip[(size_t)s0 * stride + x];
    if (tid == 0) {
        int o = 0;
        for (int p = 0; p <= G; ++p) {
            tsw_off[p] = o;
            const int r = s0 - 1 + p;
            if (r >= 0 && r + 1 < P.R) o += I.tswap_len[r];
        }
        tsw_off[G + 1] = o;
    }
    for (int x = tid; x < 4 * G; x += bs) mail[x] = 0ull;
    __syncthreads();
    for (int p = 0; p <= G; ++p) {
        const int r = s0 - 1 + p;
        if (r < 0 || r + 1 >= P.R) continue;
        const int lo = tsw_off[p], len = tsw_off[p + 1] - lo;
        for (int x = tid; x < len; x += bs) tsw[lo + x] = I.tswap[I.tswap_off[r] + x];
    }
    __syncthreads();

    // swap-table rows of the slot's two pairs, lane i: pair s0 - 1 + wv + i
    const int prow_w = wv < G ? wv + (lane < NP ? lane : 0) : 0;
    const int row_off_v = tsw_off[prow_w];
    const int row_len_v = tsw_off[prow_w + 1] - row_off_v;
    const bool active = wv < G;
    // the wavefronts at the workgroup's ends carry the cross-workgroup
    // exchanges that pace the whole ladder: they issue first on their SIMD
    if (it.W > 1) {
        const int dist = wv < G - 1 - wv ? wv : G - 1 - wv;
        if (dist == 0) __builtin_amdgcn_s_setprio(3);
        else if (dist == 1) __builtin_amdgcn_s_setprio(2);
        else if (dist == 2) __builtin_amdgcn_s_setprio(1);
    }
    const bool has_down = it.w > 0, has_up = it.w + 1 < it.W;
    bool failed = false;

    int buf = wv, E = active ? I.E[s0 + wv] : 0, bestE = I.best->E, bestSlot = -1;
    long long bestT = -1, hit = -1;
    unsigned nflip = 0, satt = 0, sacc = 0, patt = 0, pacc = 0;
    const bool want_hit = P.has_target && I.best->first_hit < 0;
    uint32_t n_prop = 0;

    if (active) {
        const int slot = s0 + wv;
        const uint32_t *tab_w = tab + wv * stride + D;        // flip threshold by m_i I_i
        const float cfl = __uint_as_float(__builtin_amdgcn_readfirstlane(I.tflip[(size_t)P.R * stride + slot]));   // 2 beta / ln 2
        const bool gibbs = I.rule == RULE_GIBBS;
        uint16_t *rnd_w = rnd + (size_t)wv * nr;
        uint32_t cyc = (uint32_t)(t0 / (uint64_t)P.M), phase = (uint32_t)(t0 % (uint64_t)P.M);
        uint64_t prop_at = P.first_prop_from(t0 + 1);
        // the slot's exchange by cycle parity (1: lower member of its pair,
        // 2: partner in this workgroup, 4: partner across a boundary)
        int xflags = 0;
#pragma unroll
        for (int par = 0; par < 2; ++par) {
            const bool lower = ((slot ^ par) & 1) != 0;
            const bool paired = lower ? slot + 1 < P.R : slot >= 1;
            const bool intra = paired && (lower ? wv + 1 < G : wv > 0);
            const bool cross = paired && !intra && (lower ? has_up : has_down);
            xflags |= ((lower ? 1 : 0) | (intra ? 2 : 0) | (cross ? 4 : 0)) << (3 * par);
        }
        xflags = __builtin_amdgcn_readfirstlane(xflags);
        constexpr uint32_t UCYC = 64 / NP;
        uint32_t u_vec = 0, u_base = (uint32_t)-100;
        const uint32_t u_i = (uint32_t)lane % (uint32_t)NP, u_c = (uint32_t)lane / (uint32_t)NP;

        // sweep tt's uniforms: Philox call q serves sites 8q .. 8q + 7
        auto draw = [&](uint64_t tt) {
            for (int q = lane; q < nr / 8; q += 64) {
                const P4 rr = philox_v((uint32_t)q, (uint32_t)tt, (uint32_t)slot, TAG_SWEEP, P.k0, P.k1);
                *(uint4 *)(rnd_w + 8 * q) = make_uint4(rr.v[0], rr.v[1], rr.v[2], rr.v[3]);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
        };
        auto load_rows = [&](Rows &r, int g) {
            r.gcb = __builtin_amdgcn_readlane(gcb_v, g);
            r.b0 = bw[(r.gcb >> 8) * 64 + lane];
            r.b1 = bw[((r.gcb >> 8) + 1) * 64 + lane];      // unused where the group has one chunk
            r.j0 = bj[(r.gcb >> 8) * 64 + lane];
            r.j1 = bj[((r.gcb >> 8) + 1) * 64 + lane];
            r.inf = info[g * 64 + lane];
        };
        bool drawn = false;
        for (uint64_t t = t0 + 1; t <= tend && !failed; ++t) {
            const bool ends = phase + 1 == (uint32_t)P.M;
            if (ends && cyc + 1 - u_base >= UCYC) {
                u_base = cyc + 1;
                u_vec = philox_v((uint32_t)(slot - 1) + u_i, u_base + u_c, 0, TAG_SWAP, P.k0, P.k1).v[0];
            }
            // the first group's rows, in flight while the uniforms are drawn
            Rows ra, rb;
            load_rows(ra, 0);
            // ---- the sweep's uniforms, staged in site order (at a cycle end
            // they were drawn while the slot waited for its partner) ----
            if (!drawn) draw(t);
            drawn = false;

            // ---- the sweep: colour classes in order, item ranks lane + 64 k ----
            int8_t *m_w = sp + buf * SB;
            int dE = 0, nf = 0;
            // groups in pairs with two register sets, so that the rows read
            // one group ahead never need copying
            auto sweep_group = [&](const Rows &cur, Rows &nxt, int g) {
                // this group's rows have arrived (read one group ago); waiting
                // here keeps the compiler from waiting for the next group's
                // rows below, after they are requested (lgkmcnt(0))
                __builtin_amdgcn_s_waitcnt(0xc07f);
                const uint32_t ci = cur.inf;
                const int cb = cur.gcb >> 8, nch = cur.gcb & 255;
                const uint32_t ws[8] = {cur.b0.x, cur.b0.y, cur.b0.z, cur.b0.w, cur.b1.x, cur.b1.y, cur.b1.z, cur.b1.w};
                const uint32_t jz[4] = {cur.j0.x, cur.j0.y, cur.j1.x, cur.j1.y};
                // the next group's first chunks, in flight while this one is decided
                if (g + 1 < ngr) load_rows(nxt, g + 1);
                const int i = (int)(ci & 0xFFFu);
                // the item, with the reads of its first NC chunks issued
                // before any is summed (one LDS round trip); a group takes
                // one straight-line body by its chunk count, so no read is
                // waited for at a branch
                auto decide = [&](auto nc_const) {
                    constexpr int NC = decltype(nc_const)::value;
                    // a lane without an item works on the padding byte n (its
                    // bonds are site 0 with J = 0) and decides nothing, so the
                    // lanes need no divergent region
                    const bool has = i != 0xFFF;
                    const int ii = has ? i : n;
                    const int m = m_w[ii];
                    const uint32_t ur = rnd_w[ii], hs = ur << 16;
                    int v[8 * NC];                      // 4 words of 2 neighbours per chunk
#pragma unroll
                    for (int q = 0; q < 4 * NC; ++q) {
                        v[2 * q] = m_w[ws[q] & 0xFFFFu];
                        v[2 * q + 1] = m_w[ws[q] >> 16];
                    }
                    // keep the scheduler from splitting the reads around a wait
                    __builtin_amdgcn_sched_barrier(0);
                    int f = (int)ci >> 16;
#pragma unroll
                    for (int q = 0; q < 2 * NC; ++q)
                        f = __builtin_amdgcn_sdot4((int)pack4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]),
                                                   (int)jz[q], f, false);
                    // chunks past the second: the rare high-degree groups
                    for (int j = 2; j < nch; ++j) {
                        const uint4 wc = bw[(cb + j) * 64 + lane];
                        const uint2 jc = bj[(cb + j) * 64 + lane];
                        const uint32_t wj[4] = {wc.x, wc.y, wc.z, wc.w};
                        int u[8];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            u[2 * q] = m_w[wj[q] & 0xFFFFu];
                            u[2 * q + 1] = m_w[wj[q] >> 16];
                        }
                        f = __builtin_amdgcn_sdot4((int)pack4(u[0], u[1], u[2], u[3]), (int)jc.x, f, false);
                        f = __builtin_amdgcn_sdot4((int)pack4(u[4], u[5], u[6], u[7]), (int)jc.y, f, false);
                    }
                    const int d = __mul24(m, f);            // m = +-1, |f| <= 4096
                    // The table's coarse test accepts iff floor(65536 p) > u_hi
                    // and leaves u open iff floor(65536 p) == u_hi. X = 65536 p
                    // in FP32 is within 3e-6 of the host's FP64 value wherever
                    // X >= 1/2 (the exponent stays below 17), so X (1 - MARGIN)
                    // >= u_hi + 1 accepts and X (1 + MARGIN) < u_hi rejects as the
                    // table would; the rest (about one uniform in 10^4, and a
                    // NaN X) read the slot's threshold.
                    const float uf = (float)ur, y = (float)d * cfl;
                    // one exponential for either rule, no branch
                    const float ex = __builtin_amdgcn_exp2f(gibbs ? y : 16.0f - y);
                    const float X = gibbs ? 65536.0f * __builtin_amdgcn_rcpf(1.0f + ex) : ex;
                    bool acc = has && ((!gibbs && d <= 0) || X * (1.0f - MARGIN) >= uf + 1.0f);
                    const bool open = has && !acc && !(X * (1.0f + MARGIN) < uf);
                    if (__builtin_expect(any_lane(open), 0)) {
                        bool maybe = false;
                        uint32_t T = 0;
                        if (open) {
                            T = tab_w[d];
                            acc = coarse_accept(T, hs, maybe);
                        }
                        if (any_lane(maybe)) {
                            if (maybe) {
                                const P4 r2 = philox(opaque((uint32_t)(i >> 3)), (uint32_t)t, (uint32_t)slot,
                                                     TAG_REFINE, P.k0, P.k1);
                                const int wq = (i & 7) >> 1;
                                const uint32_t wd = wq == 0 ? r2.v[0] : wq == 1 ? r2.v[1] : wq == 2 ? r2.v[2] : r2.v[3];
                                const uint32_t lo = ((i & 1) ? (wd >> 16) : wd) & 0xFFFFu;
                                acc = (T == ALWAYS) || ((hs | lo) < T);
                            }
                        }
                    }
                    // every lane with an item writes its spin back, so the
                    // common path takes no branch
                    m_w[ii] = (int8_t)(acc ? -m : m);
                    dE += acc ? 2 * d : 0;
                    nf += acc ? 1 : 0;
                };
                if (__builtin_expect(nch == 1, 1)) decide(std::integral_constant<int, 1>{});
                else decide(std::integral_constant<int, 2>{});
                // the next class reads what this one wrote (in-order LDS
                // within a wavefront)
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
            };
            for (int g = 0; g < ngr; g += 2) {
                sweep_group(ra, rb, g);
                if (g + 1 < ngr) sweep_group(rb, ra, g + 1);
            }
            nflip += (unsigned)nf;
            E += wave_sum(dE);

            if (ends) {
                phase = 0;
                ++cyc;
                // ---- proposal (Eq. 2) ----
                const bool prop_now = t == prop_at;
                if (prop_now) {
                    prop_at = P.next_prop(prop_at);
                    const int Bn = I.bank_n[slot];
                    if (Bn > 0) {
                        const int cur0 = I.cursor[slot];
                        const int kk = (int)(((uint32_t)cur0 + n_prop % (uint32_t)Bn) % (uint32_t)Bn);
                        patt += 1;
                        const int ET = I.bankE[slot][kk];
                        const long long dd = (long long)ET - (long long)E;
                        uint32_t T;
                        if (dd <= 0) T = ALWAYS;
                        else if (dd <= I.tprop_len[slot]) T = I.tprop[I.tprop_off[slot] + (int)dd - 1];
                        else T = 0;
                        const uint32_t u = philox_word0((uint32_t)slot, cyc, TAG_PROPOSE, P.k0, P.k1);
                        if (T == ALWAYS || u < T) {
                            const int8_t *src = I.bank[slot] + (size_t)kk * n;
                            int8_t *dst = sp + buf * SB;
                            for (int i = lane; i < n; i += 64) dst[i] = src[i];
                            E = ET;
                            pacc += 1;
                        }
                    }
                    ++n_prop;
                }
                // ---- swap (Eq. 1), alternating parity ----
                const int xf = (xflags >> (3 * (int)(cyc & 1))) & 7;
                const bool lower = (xf & 1) != 0;
                const int side = xf & 1;                          // 1: partner slot + 1
                const bool intra = (xf & 2) != 0;
                const bool cross = (xf & 4) != 0;
                const int pi = xf & 1;                            // pair slot - 1 + pi
                unsigned long long *mb = mail + (cyc & 3) * G;
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                if (intra && lane == 0)
                    __hip_atomic_store(mb + wv, ((unsigned long long)cyc << 32) | ((uint32_t)buf << 24) |
                                                    ((uint32_t)E & 0xFFFFFFu),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                const int buf_x = (cyc >> 1) & 1;
                if (cross) {
                    // lane q's word m: bit k - 32 m set when site q + 64 k is -1; word NXW the energy
                    unsigned long long *out = it.xbuf + ((size_t)(it.w * 2 + side) * 2 + buf_x) * it.xwords;
                    const int8_t *src = sp + buf * SB;
                    uint32_t w0 = 0, w1 = 0;
                    for (int k = 0; k < spl; ++k) {
                        const int i = lane + 64 * k;
                        const uint32_t bit = (i < n && src[i] < 0) ? 1u : 0u;
                        if (k < 32) w0 |= bit << k;
                        else w1 |= bit << (k - 32);
                    }
                    const unsigned long long tg = (unsigned long long)cyc << 32;
                    __hip_atomic_store(out + lane, tg | w0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (wpl > 1) __hip_atomic_store(out + 64 + lane, tg | w1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (lane == 0)
                        __hip_atomic_store(out + NXW, tg | (uint32_t)E, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                // the next sweep's uniforms do not depend on the swap: draw
                // them while the partner's word is on its way
                if ((intra || cross) && t < tend) {
                    draw(t + 1);
                    drawn = true;
                }
                if (intra) {
                    uint32_t polls = 0;
                    unsigned long long v;
                    for (;;) {
                        v = __hip_atomic_load(mb + wv + (lower ? 1 : -1), __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
                        if ((uint32_t)(v >> 32) == cyc) break;
                        __builtin_amdgcn_s_sleep(1);
                        if (++polls > a.spin_limit) break;
                    }
                    if ((uint32_t)(v >> 32) != cyc) {
                        if (lane == 0 && atomicCAS(a.err, 0, 2) == 0) {
                            a.err[1] = item; a.err[2] = it.w; a.err[3] = 2; a.err[4] = (int)cyc;
                            a.err[5] = (int)(v & 0xFFFFFFFFu); a.err[6] = (int)(v >> 32); a.err[7] = (int)I.epoch;
                        }
                        failed = true;
                    } else {
                        const uint32_t lo32 = __builtin_amdgcn_readfirstlane((uint32_t)v);
                        const int pE = ((int)(lo32 << 8)) >> 8;      // 24-bit signed energy
                        const int pb = (int)((lo32 >> 24) & 0xFFu);
                        const int dEs = lower ? pE - E : E - pE;
                        const bool okx = swap_ok(dEs, __builtin_amdgcn_readlane(u_vec, NP * (cyc - u_base) + pi),
                                                 __builtin_amdgcn_readlane(row_off_v, pi),
                                                 __builtin_amdgcn_readlane(row_len_v, pi), tsw);
                        if (lower) {   // the lower member owns the pair's counters
                            satt += 1;
                            sacc += okx ? 1u : 0u;
                        }
                        buf = okx ? pb : buf;
                        E = okx ? pE : E;
                    }
                }
                if (cross && !failed) {
                    const int pw = lower ? it.w + 1 : it.w - 1;
                    const unsigned long long *in = it.xbuf + ((size_t)(pw * 2 + (1 - side)) * 2 + buf_x) * it.xwords;
                    uint32_t *stage = xstage + (size_t)(wv * 2 + side) * (NXW + 1);
                    uint32_t polls = 0;
                    bool ok_all = false;
                    unsigned long long bad = 0;
                    for (;;) {
                        bool ok = true;
                        for (int m = 0; m <= wpl; ++m) {
                            const int w = lane + 64 * m;
                            if (w <= NXW) {
                                const unsigned long long v =
                                    __hip_atomic_load(in + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                                if ((uint32_t)(v >> 32) == cyc) stage[w] = (uint32_t)v;
                                else {
                                    ok = false;
                                    bad = v;
                                }
                            }
                        }
                        if (__all(ok)) {
                            ok_all = true;
                            break;
                        }
                        if (++polls > a.spin_limit) break;
                    }
                    if (!ok_all) {
                        if (lane == 0 && atomicCAS(a.err, 0, 1) == 0) {
                            a.err[1] = item; a.err[2] = it.w; a.err[3] = side; a.err[4] = (int)cyc;
                            a.err[5] = (int)(bad & 0xFFFFFFFFu); a.err[6] = (int)(bad >> 32); a.err[7] = (int)I.epoch;
                        }
                        failed = true;
                    } else {
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        const int pE = __builtin_amdgcn_readfirstlane((int)stage[NXW]);
                        const int dEs = lower ? pE - E : E - pE;
                        const bool okx = swap_ok(dEs, __builtin_amdgcn_readlane(u_vec, NP * (cyc - u_base) + pi),
                                                 __builtin_amdgcn_readlane(row_off_v, pi),
                                                 __builtin_amdgcn_readlane(row_len_v, pi), tsw);
                        if (lower) {   // the lower workgroup owns the pair's counters
                            satt += 1;
                            if (okx) sacc += 1;
                        }
                        E = okx ? pE : E;
                        if (okx) {
                            // the lane's sites from its own words
                            const uint32_t w0 = stage[lane], w1 = wpl > 1 ? stage[64 + lane] : 0u;
                            int8_t *dst = sp + buf * SB;
                            for (int k = 0; k < spl; ++k) {
                                const int i = lane + 64 * k;
                                const uint32_t bit = k < 32 ? (w0 >> k) & 1u : (w1 >> (k - 32)) & 1u;
                                if (i < n) dst[i] = bit ? (int8_t)-1 : (int8_t)1;
                            }
                        }
                    }
                }
            } else {
                ++phase;
            }
            // ---- best energy and first hit ----
            if (want_hit && hit < 0 && E <= P.target) hit = (long long)t;
            if (E < bestE) {
                bestE = E;
                bestT = (long long)t;
                bestSlot = slot;
                const int8_t *src = sp + buf * SB;
                int8_t *dst = it.best_spins + (size_t)wv * n;
                for (int i = lane; i < n; i += 64) dst[i] = src[i];
            }
        }
    }

    // ---- end of launch ----
    __shared__ int any_failed, win;
    __shared__ int slot_buf[MAXG], slot_E[MAXG];
    __shared__ Rec rec[MAXG];
    __shared__ unsigned cnt[MAXG][5];
    if (tid == 0) any_failed = 0;
    __syncthreads();
    if (active) {
        const unsigned nfw = (unsigned)wave_sum((int)nflip);
        if (failed && lane == 0) any_failed = 1;
        if (lane == 0) {
            slot_buf[wv] = buf;
            slot_E[wv] = E;
            Rec rr;
            rr.E = bestE;
            rr.slot = bestSlot;
            rr.t = bestT;
            rr.hit = hit;
            rec[wv] = rr;
            cnt[wv][0] = nfw;
            cnt[wv][1] = satt;
            cnt[wv][2] = sacc;
            cnt[wv][3] = patt;
            cnt[wv][4] = pacc;
        }
    }
    __syncthreads();
    if (any_failed) return;   // the host reports the error; the launch's state is abandoned
    for (int x = tid; x < G * n; x += bs) {
        const int l = x / n, i = x - l * n;
        I.spins[(size_t)(s0 + l) * n + i] = sp[slot_buf[l] * SB + i];
    }
    for (int l = tid; l < G; l += bs) {
        const int slot = s0 + l;
        I.E[slot] = slot_E[l];
        I.flips[slot] += cnt[l][0];
        I.prop_att[slot] += cnt[l][3];
        I.prop_acc[slot] += cnt[l][4];
        const int Bn = I.bank_n[slot];
        if (Bn > 0) I.cursor[slot] = (int)(((uint32_t)I.cursor[slot] + n_prop % (uint32_t)Bn) % (uint32_t)Bn);
        if (slot + 1 < P.R) {
            I.swap_att[slot] += cnt[l][1];
            I.swap_acc[slot] += cnt[l][2];
        }
    }
    if (tid == 0) {
        int wb = -1;
        long long h = -1;
        for (int l = 0; l < G; ++l) {
            const Rec r = rec[l];
            if (r.hit >= 0 && (h < 0 || r.hit < h)) h = r.hit;
            if (r.t < 0) continue;
            if (wb < 0 || r.E < rec[wb].E || (r.E == rec[wb].E && (r.t < rec[wb].t || (r.t == rec[wb].t && r.slot < rec[wb].slot))))
                wb = l;
        }
        BestRec b;
        b.E = wb >= 0 ? rec[wb].E : 0x7FFFFFFF;
        b.slot = wb >= 0 ? rec[wb].slot : -1;
        b.t = wb >= 0 ? rec[wb].t : -1;
        b.first_hit = h;
        b.pad = 0;
        *it.best = b;
        win = wb;
    }
    __syncthreads();
    if (win > 0)
        for (int i = tid; i < n; i += bs) it.best_spins[i] = it.best_spins[(size_t)win * n + i];
}

// ---------------------------------------------------------------------------
// Host-side launchers (C++ linkage, used by the runtime in host.cpp).

int csrw_max_storages() { return csrw::MAXG; }

// where the kernel applies: n <= 4095, |J| <= 127, classes of at most 256 sites,
// and the host packed the rows (chunks > 0: degree <= CSRW_MAXDEG, at most
// CSRW_MAXGROUPS rank groups)
bool csrw_supported(int n, int maxabsj, int chunks, int maxcnt)
{
    return n >= 1 && n <= 4095 && maxabsj <= 127 && chunks > 0 && maxcnt >= 1 && maxcnt <= 256;
}

size_t csrw_lds_bytes(int n, int ncolors, int maxcnt, int chunks, int G, int stride, int tsw_entries)
{
    return csrw::offsets(n, ncolors, (maxcnt + 63) / 64, chunks, G, stride, tsw_entries).total;
}

// 64-bit exchange words of one state (bits and energy)
int csrw_xwords(int n) { return 64 * (((n + 63) / 64 + 31) / 32) + 1; }

hipError_t launch_csrw(const ChunkArgs &a, int block, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL(csrw_kernel, dim3(a.n_items), dim3(block), lds, s, a);
    return hipGetLastError();
}

hipError_t csrw_occupancy(int block, size_t lds, int *blocks_per_cu)
{
    hipError_t e = hipFuncSetAttribute((const void *)csrw_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, csrw_kernel, block, lds);
}

} // namespace tapt
