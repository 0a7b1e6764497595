// Persistent kernel for +-J couplings on the periodic 8^3 lattice (no
// fields): every wavefront owns SPW adjacent beta slots (SPW = 2: slots 2w,
// 2w+1 of its workgroup; SPW = 1: slot w) and sweeps them with byte-parallel
// arithmetic. Two slots per wavefront give each wavefront two independent
// chains to interleave; one slot per wavefront gives the SIMDs twice as many
// wavefronts to switch between.
//
// Storage. A replica is 64 rows of 8 sites (row q = y + 8z holds x = 0..7,
// site index i = 8q + x), one byte per site that is 1 when the spin is -1.
// Lane q of a wavefront owns row q, which is also the row of Philox call q,
// so its 8 uniforms are the lane's own.
//
// Local field. With b the down-bit of a site, n the down-bit of a neighbour
// and j = 1 when the bond is -1, the bond is unsatisfied (J m_i m_j = -1)
// exactly when j ^ b ^ n = 1. A colour phase updates the four sites
// x = p, p+2, p+4, p+6 of the row (p = (colour + y + z) mod 2). Their
// neighbours along x come from the lane's own row and those along y and z
// from four whole-row LDS reads; v_perm gathers the four relevant bytes of
// each into one dword, three-input XORs form the six unsatisfied-bond flags
// and byte-wise adds count them (U <= 6, no carries). Then m_i I_i = 6 - 2U,
// the flip changes E by 12 - 4U, and the threshold is the slot's table entry
// for that m_i I_i. The upper halves of the slot's eight thresholds (by U)
// sit in registers as byte tables, so one v_perm looks up all four sites and
// saturating 16-bit subtractions test them against their uniforms at once;
// the rare tie of the upper halves takes the exact 32-bit test.
//
// Slots and states. A wavefront's slots are fixed; states move between LDS
// buffers. With two slots, the pair (2w, 2w+1) is decided inside the
// wavefront with no communication. A pair that spans two wavefronts meets in
// an LDS mailbox that carries the energy and the buffer index, and an
// accepted swap trades buffer indices. Pairs across a workgroup boundary go
// through cycle-tagged global words and copy the state. Best energy, first
// hit and all counters are per slot and live in registers.
#include "sweep.h"

namespace tapt {

namespace pm {

constexpr int L = 8, N = 512, ROWB = 8;

// v_perm selectors ({hi, lo}: bytes 0-3 from lo, 4-7 from hi)
__device__ __forceinline__ uint32_t sel_sites(int p) { return p ? 0x07050301u : 0x06040200u; }   // x = p + 2j
__device__ __forceinline__ uint32_t sel_xp(int p) { return p ? 0x00060402u : 0x07050301u; }      // x + 1
__device__ __forceinline__ uint32_t sel_xm(int p) { return p ? 0x06040200u : 0x05030107u; }      // x - 1
// high half of word j moved to the top: (w >> 16p) << 16 (0x0c selects a zero byte)
__device__ __forceinline__ uint32_t sel_half(int p) { return p ? 0x03020c0cu : 0x01000c0cu; }
// halves p of words j and j+1 side by side: {hi: word j+1, lo: word j}
__device__ __forceinline__ uint32_t sel_pair(int p) { return p ? 0x07060302u : 0x05040100u; }
// compact flags (byte j) to row bytes x = p + 2j, low and high dword
__device__ __forceinline__ uint32_t sel_flo(int p) { return p ? 0x010c000cu : 0x0c010c00u; }
__device__ __forceinline__ uint32_t sel_fhi(int p) { return p ? 0x030c020cu : 0x0c030c02u; }

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel)
{
    return __builtin_amdgcn_perm(hi, lo, sel);
}

struct Off {
    size_t buf, tabu, toff, tsw, mail, xst, total;
};

__host__ __device__ inline Off offsets(int G, int tsw_entries)
{
    Off f;
    size_t o = 0;
    f.buf = o; o = align16(o + (size_t)G * N);
    f.tabu = o; o = align16(o + (size_t)G * 8 * 4);
    f.toff = o; o = align16(o + (size_t)(G + 2) * 4);
    f.tsw = o; o = align16(o + (size_t)tsw_entries * 4);
    f.mail = o; o = align16(o + (size_t)4 * G * 8);
    f.xst = o; o = align16(o + (size_t)2 * G * ((N >> 5) + 1) * 4);   // [2 G][17] staged words
    f.total = o;
    return f;
}

struct Rec {
    int E, slot;
    long long t, hit;
};

// Swap acceptance (Eq. 1) for dE = E_{r+1} - E_r with the pair's LDS table
// row (off, len). Every input is wave-uniform; the table is read
// unconditionally (clamped index) and the result is returned through an SGPR,
// so that callers select on a scalar instead of branching per lane.
__device__ __forceinline__ bool swap_ok(int dE, uint32_t u, int off, int len, const uint32_t *tsw)
{
    const int d = -dE;
    const bool in_row = d >= 1 && d <= len;
    const uint32_t Tr = tsw[in_row ? off + d - 1 : 0];
    const uint32_t T = dE >= 0 ? ALWAYS : (in_row ? Tr : 0u);
    const bool ok = T == ALWAYS || u < T;
    return __builtin_amdgcn_readfirstlane(ok ? 1 : 0) != 0;
}

} // namespace pm

template <int SPW>
__global__ void __launch_bounds__(512) pm_kernel(ChunkArgs a)
{
    using namespace pm;
    constexpr int NP = SPW + 1;               // pairs a wavefront takes part in
    const int item = a.order[blockIdx.x];
    if (item < 0) return;
    const WorkItem it = a.items[item];
    const InstDev &I = *it.inst;
    RunParams P;
    P.load(I);
    const int G = it.G, s0 = it.s0;          // G even, s0 even
    const int tid = threadIdx.x, bs = blockDim.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int NWV = G / SPW;
    const uint64_t t0 = *I.t;
    const uint64_t cap = chunk_cap(I, t0);
    const uint64_t tend = (t0 + a.K < cap) ? t0 + a.K : cap;
    if (t0 >= tend) {
        if (tid == 0) idle_best(it.best);
        return;
    }
    const Off lof = offsets(G, a.tsw_entries);
    uint8_t *bufs = (uint8_t *)(lds_raw + lof.buf);
    uint32_t *tabu = (uint32_t *)(lds_raw + lof.tabu);          // [G][8] threshold by U
    int *tsw_off = (int *)(lds_raw + lof.toff);
    uint32_t *tsw = (uint32_t *)(lds_raw + lof.tsw);
    unsigned long long *mail = (unsigned long long *)(lds_raw + lof.mail);   // [4][G]
    uint32_t *xstage = (uint32_t *)(lds_raw + lof.xst);
    constexpr int NWD = N >> 5;                                   // 32-bit words of a packed state

    // ---- stage: states as down-bits (slot l in buffer l), tables ----
    for (int x = tid; x < G * N / 4; x += bs) {
        const int l = x / (N / 4), w4 = x - l * (N / 4);
        const uint32_t v = *(const uint32_t *)(I.spins + (size_t)(s0 + l) * N + 4 * w4);
        *(uint32_t *)(bufs + l * N + 4 * w4) = (v >> 7) & 0x01010101u;
    }
    for (int x = tid; x < G * 8; x += bs) {
        const int l = x >> 3, U = x & 7;
        // m_i I_i = 6 - 2U indexes the flip row at D + 6 - 2U (D = 6 here)
        tabu[x] = U <= 6 ? I.tflip[(size_t)(s0 + l) * P.stride + P.D + 6 - 2 * U] : 0u;
    }
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

    // swap-table rows of this wavefront's NP pairs, lane i: pair s0 - 1 + SPW wv + i
    // (i = 0: below its first slot, NP - 1: above its last, 1 between two slots)
    const int prow_w = wv < G / SPW ? SPW * wv + (lane < NP ? lane : 0) : 0;
    const int row_off_v = tsw_off[prow_w];
    const int row_len_v = tsw_off[prow_w + 1] - row_off_v;
    const bool active = wv < NWV;
    // the wavefronts at the workgroup's ends carry the cross-workgroup
    // exchanges that pace the whole ladder: the closer a wavefront is to an
    // end, the earlier it issues on its SIMD
    if (it.W > 1) {
        const int dist = wv < NWV - 1 - wv ? wv : NWV - 1 - wv;
        if (dist == 0) __builtin_amdgcn_s_setprio(3);
        else if (dist == 1) __builtin_amdgcn_s_setprio(2);
        else if (dist == 2) __builtin_amdgcn_s_setprio(1);
    }
    const bool has_down = it.w > 0, has_up = it.w + 1 < it.W;
    bool failed = false;

    // per-slot state of this wavefront (k = 0, 1: local slots 2wv + k)
    int buf[SPW], E[SPW], bestE[SPW], bestSlot[SPW];
    long long bestT[SPW], hit[SPW];
    unsigned nflip[SPW], satt[SPW], sacc[SPW], patt[SPW], pacc[SPW];
    const int best0 = I.best->E;
    const bool want_hit = P.has_target && I.best->first_hit < 0;
#pragma unroll
    for (int k = 0; k < SPW; ++k) {
        buf[k] = SPW * wv + k;
        E[k] = active ? I.E[s0 + SPW * wv + k] : 0;
        bestE[k] = best0;
        bestSlot[k] = -1;
        bestT[k] = -1;
        hit[k] = -1;
        nflip[k] = satt[k] = sacc[k] = patt[k] = pacc[k] = 0;
    }
    uint32_t n_prop = 0;

    if (active) {
        // lane geometry: row q = lane, y = q & 7, z = q >> 3
        const int y = lane & 7, z = lane >> 3;
        const int rel_yp = ROWB * (((y + 1) & 7) + 8 * z), rel_ym = ROWB * (((y + 7) & 7) + 8 * z);
        const int rel_zp = ROWB * (y + 8 * ((z + 1) & 7)), rel_zm = ROWB * (y + 8 * ((z + 7) & 7));
        const int rel_me = ROWB * lane;
        int par[2];
        par[0] = (y + z) & 1;
        par[1] = par[0] ^ 1;
        // unsatisfied-bond bits of the couplings: JN[c][d] byte j = 1 when the
        // bond of site x = par[c] + 2j in direction d is -1 (d: +x, -x, +y, -y, +z, -z)
        uint32_t JN[2][6];
        const int8_t *J3 = I.J3;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
#pragma unroll
            for (int d = 0; d < 6; ++d) JN[c][d] = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int x = par[c] + 2 * j;
                const int i = x + 8 * lane;
                const int xm = (x + 7) & 7;
                const int iym = x + 8 * (((y + 7) & 7) + 8 * z);
                const int izm = x + 8 * (y + 8 * ((z + 7) & 7));
                const int jb[6] = {J3[i], J3[xm + 8 * lane], J3[N + i], J3[N + iym], J3[2 * N + i], J3[2 * N + izm]};
#pragma unroll
                for (int d = 0; d < 6; ++d) JN[c][d] |= (uint32_t)(jb[d] < 0 ? 1 : 0) << (8 * j);
            }
        }
        const uint32_t S0 = sel_sites(par[0]), S1 = sel_sites(par[1]);
        const uint32_t XP0 = sel_xp(par[0]), XP1 = sel_xp(par[1]);
        const uint32_t XM0 = sel_xm(par[0]), XM1 = sel_xm(par[1]);
        const uint32_t H0 = sel_half(par[0]), H1 = sel_half(par[1]);
        const uint32_t FL0 = sel_flo(par[0]), FL1 = sel_flo(par[1]);
        const uint32_t FH0 = sel_fhi(par[0]), FH1 = sel_fhi(par[1]);
        const uint32_t HP0 = sel_pair(par[0]), HP1 = sel_pair(par[1]);
        // coarse thresholds (upper 16 bits of each slot's threshold by U) as
        // byte tables for v_perm: tb* hold the high bytes, tl* the low bytes,
        // *lo for U = 0..3 and *hi for U = 4..7
        uint32_t tbl[SPW], tbh[SPW], tll[SPW], tlh[SPW];
#pragma unroll
        for (int k = 0; k < SPW; ++k) {
            const uint32_t *tu = tabu + (SPW * wv + k) * 8;
            tbl[k] = tbh[k] = tll[k] = tlh[k] = 0;
#pragma unroll
            for (int U = 0; U < 4; ++U) {
                tbl[k] |= (tu[U] >> 24) << (8 * U);
                tbh[k] |= (tu[U + 4] >> 24) << (8 * U);
                tll[k] |= ((tu[U] >> 16) & 0xFFu) << (8 * U);
                tlh[k] |= ((tu[U + 4] >> 16) & 0xFFu) << (8 * U);
            }
        }
        const uint32_t ONE2 = 0x00010001u;

        uint32_t cyc = (uint32_t)(t0 / (uint64_t)P.M), phase = (uint32_t)(t0 % (uint64_t)P.M);
        uint64_t prop_at = P.first_prop_from(t0 + 1);
        const int lab0 = s0 + SPW * wv;          // this wavefront's slots: lab0 .. lab0 + SPW - 1
        // one slot per wavefront: its exchange by cycle parity, three bits per
        // parity (1: lower member of its pair, 2: partner in this workgroup,
        // 4: partner across a workgroup boundary), so that the cycle end tests
        // bits of one scalar
        int xflags = 0;
        if constexpr (SPW == 1) {
#pragma unroll
            for (int par = 0; par < 2; ++par) {
                const bool lower = ((lab0 ^ par) & 1) != 0;
                const bool paired = lower ? lab0 + 1 < P.R : lab0 >= 1;
                const bool intra = paired && (lower ? wv + 1 < NWV : wv > 0);
                const bool cross = paired && !intra && (lower ? has_up : has_down);
                xflags |= ((lower ? 1 : 0) | (intra ? 2 : 0) | (cross ? 4 : 0)) << (3 * par);
            }
            xflags = __builtin_amdgcn_readfirstlane(xflags);
        }
        // swap uniforms of this wavefront's NP pairs for UCYC cycles: lane
        // NP c + i holds pair lab0 - 1 + i at cycle u_base + c
        constexpr uint32_t UCYC = 64 / NP;
        uint32_t u_vec = 0, u_base = (uint32_t)-100;
        const uint32_t u_i = (uint32_t)lane % (uint32_t)NP, u_c = (uint32_t)lane / (uint32_t)NP;
        // the sweep uniforms of the next sweep: slots are fixed per wavefront,
        // so they are drawn ahead, where the cycle end waits for a partner
        P4 rn[SPW];
#pragma unroll
        for (int k = 0; k < SPW; ++k)
            rn[k] = philox_v((uint32_t)lane, (uint32_t)(t0 + 1), (uint32_t)(lab0 + k), TAG_SWEEP, P.k0, P.k1);

        for (uint64_t t = t0 + 1; t <= tend && !failed; ++t) {
            bool drawn = false;   // rn holds sweep t + 1's uniforms
            const bool ends = phase + 1 == (uint32_t)P.M;
            // one Philox call per UCYC cycles, drawn before the sweep so that
            // its latency hides behind it
            if (ends && cyc + 1 - u_base >= UCYC) {
                u_base = cyc + 1;
                u_vec = philox_v((uint32_t)(lab0 - 1) + u_i, u_base + u_c, 0, TAG_SWAP, P.k0, P.k1).v[0];
            }

            // ---- sweep both slots (colour phases outermost, so that the two
            // slots' independent work interleaves) ----
            P4 r[SPW];
            uint2 me[SPW];
            int nf[SPW], su[SPW];
            uint32_t a_me[SPW], a_yp[SPW], a_ym[SPW], a_zp[SPW], a_zm[SPW];   // row addresses in bufs
#pragma unroll
            for (int k = 0; k < SPW; ++k) {
                r[k] = rn[k];
                const uint32_t B = (uint32_t)(buf[k] * N);
                a_me[k] = B + rel_me;
                a_yp[k] = B + rel_yp;
                a_ym[k] = B + rel_ym;
                a_zp[k] = B + rel_zp;
                a_zm[k] = B + rel_zm;
                me[k] = *(const uint2 *)(bufs + a_me[k]);
                nf[k] = 0;
                su[k] = 0;
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const uint32_t Ss = c ? S1 : S0, Xp = c ? XP1 : XP0, Xm = c ? XM1 : XM0;
                const uint32_t Hs = c ? H1 : H0, FL = c ? FL1 : FL0, FH = c ? FH1 : FH0;
                const uint32_t Hp = c ? HP1 : HP0;
                // both slots' neighbour rows first (the slots use different
                // buffers), so that all eight reads are in flight together
                uint2 yp[SPW], ym[SPW], zp[SPW], zm[SPW];
#pragma unroll
                for (int k = 0; k < SPW; ++k) {
                    yp[k] = *(const uint2 *)(bufs + a_yp[k]);
                    ym[k] = *(const uint2 *)(bufs + a_ym[k]);
                    zp[k] = *(const uint2 *)(bufs + a_zp[k]);
                    zm[k] = *(const uint2 *)(bufs + a_zm[k]);
                }
#pragma unroll
                for (int k = 0; k < SPW; ++k) {
                    const uint32_t b = perm(me[k].y, me[k].x, Ss);
                    const uint32_t x0 = xor3(JN[c][0], b, perm(me[k].y, me[k].x, Xp));
                    const uint32_t x1 = xor3(JN[c][1], b, perm(me[k].y, me[k].x, Xm));
                    const uint32_t x2 = xor3(JN[c][2], b, perm(yp[k].y, yp[k].x, Ss));
                    const uint32_t x3 = xor3(JN[c][3], b, perm(ym[k].y, ym[k].x, Ss));
                    const uint32_t x4 = xor3(JN[c][4], b, perm(zp[k].y, zp[k].x, Ss));
                    const uint32_t x5 = xor3(JN[c][5], b, perm(zm[k].y, zm[k].x, Ss));
                    const uint32_t U = x0 + x1 + x2 + x3 + x4 + x5;
                    // Coarse test of all four sites at once, on 16-bit halves:
                    // site j flips when its uniform's upper half is below the
                    // upper half of its threshold, and stays when above; equal
                    // halves (or an always-accept entry, whose upper half is
                    // 0xFFFF) leave the decision to the exact test below.
                    const uint32_t TB = perm(tbh[k], tbl[k], U);        // U <= 6 selects a table byte
                    const uint32_t TL = perm(tlh[k], tll[k], U);
                    const uint32_t T01 = perm(TB, TL, 0x05010400u), T23 = perm(TB, TL, 0x07030602u);
                    const uint32_t U01 = perm(r[k].v[1], r[k].v[0], Hp), U23 = perm(r[k].v[3], r[k].v[2], Hp);
                    uint32_t F = perm(pk_min_u16(pk_sub_sat_u16(T23, U23), ONE2),
                                      pk_min_u16(pk_sub_sat_u16(T01, U01), ONE2), 0x06040200u);
                    const uint32_t Z = pk_min_u16(pk_min_u16(T01 ^ U01, T23 ^ U23), ONE2);
                    if (any_lane(Z != ONE2)) {
                        // exact test: u = (upper << 16) | lower, the lower half
                        // from the refinement call
                        const uint32_t *tu = tabu + (SPW * wv + k) * 8;
                        const P4 r2 = philox_v(opaque((uint32_t)lane), (uint32_t)t, (uint32_t)(lab0 + k), TAG_REFINE, P.k0, P.k1);
                        uint32_t Fx = 0;
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const uint32_t T = tu[(U >> (8 * j)) & 0xFFu];
                            const uint32_t u = perm(r[k].v[j], r[k].v[j], Hs) | (perm(r2.v[j], r2.v[j], Hs) >> 16);
                            Fx |= (T == ALWAYS || u < T) ? (1u << (8 * j)) : 0u;
                        }
                        F = Fx;
                    }
                    me[k].x ^= perm(0u, F, FL);
                    me[k].y ^= perm(0u, F, FH);
                    *(uint2 *)(bufs + a_me[k]) = me[k];
                    nf[k] += __builtin_popcount(F);
                    su[k] = (int)__builtin_amdgcn_udot4(U, F, (uint32_t)su[k], false);
                }
                // the next colour reads what this one wrote (in-order LDS within a wavefront)
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
            int dEl[SPW];
#pragma unroll
            for (int k = 0; k < SPW; ++k) {
                nflip[k] += (unsigned)nf[k];   // per lane; reduced at the end
                dEl[k] = 12 * nf[k] - 4 * su[k];
            }
#pragma unroll
            for (int k = 0; k < SPW; ++k) E[k] += wave_sum(dEl[k]);

            if (ends) {
                phase = 0;
                ++cyc;
                // ---- proposals (Eq. 2), this wavefront's slots ----
                const bool prop_now = t == prop_at;
                if (prop_now) {
                    prop_at = P.next_prop(prop_at);
#pragma unroll
                    for (int k = 0; k < SPW; ++k) {
                        const int slot = lab0 + k;
                        const int Bn = I.bank_n[slot];
                        if (Bn <= 0) continue;
                        const int cur0 = I.cursor[slot];
                        const int kk = (int)(((uint32_t)cur0 + n_prop % (uint32_t)Bn) % (uint32_t)Bn);
                        patt[k] += 1;
                        const int ET = I.bankE[slot][kk];
                        const long long dd = (long long)ET - (long long)E[k];
                        uint32_t T;
                        if (dd <= 0) T = ALWAYS;
                        else if (dd <= I.tprop_len[slot]) T = I.tprop[I.tprop_off[slot] + (int)dd - 1];
                        else T = 0;
                        const uint32_t u = philox_word0((uint32_t)slot, cyc, TAG_PROPOSE, P.k0, P.k1);
                        if (T == ALWAYS || u < T) {
                            const uint2 v = *(const uint2 *)(I.bank[slot] + (size_t)kk * N + rel_me);
                            uint2 d;
                            d.x = (v.x >> 7) & 0x01010101u;
                            d.y = (v.y >> 7) & 0x01010101u;
                            *(uint2 *)(bufs + buf[k] * N + rel_me) = d;
                            E[k] = ET;
                            pacc[k] += 1;
                        }
                    }
                    ++n_prop;
                }
                // ---- swaps (Eq. 1), alternating parity ----
                if constexpr (SPW == 1) {
                    // the slot is the lower member of its pair when its parity
                    // differs from the cycle's
                    const int xf = (xflags >> (3 * (int)(cyc & 1))) & 7;
                    const bool lower = (xf & 1) != 0;
                    const int side = xf & 1;                          // 1: partner lab0 + 1
                    const bool intra = (xf & 2) != 0;
                    const bool cross = (xf & 4) != 0;
                    const int pi = xf & 1;                            // pair lab0 - 1 + pi
                    unsigned long long *mb = mail + (cyc & 3) * G;
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                    if (intra && lane == 0)
                        __hip_atomic_store(mb + wv, ((unsigned long long)cyc << 32) | ((uint32_t)buf[0] << 24) |
                                                        ((uint32_t)E[0] & 0xFFFFFFu),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    const int buf_x = (cyc >> 1) & 1;
                    if (cross) {
                        unsigned long long *out = it.xbuf + ((size_t)(it.w * 2 + side) * 2 + buf_x) * it.xwords;
                        const uint2 row = *(const uint2 *)(bufs + buf[0] * N + rel_me);
                        uint32_t pay = (uint32_t)E[0];
                        // lane >> 1 made opaque here: otherwise the compiler keeps the eight
                        // lane masks (lane >> 1) == x in SGPRs for the whole launch
                        const uint32_t lh = opaque((uint32_t)lane >> 1);
#pragma unroll
                        for (int x = 0; x < 8; ++x) {
                            const uint32_t byte = ((x < 4 ? row.x : row.y) >> (8 * (x & 3))) & 0xFFu;
                            const unsigned long long bal = __ballot(byte == 0);
                            const uint32_t half = (lane & 1) ? (uint32_t)(bal >> 32) : (uint32_t)bal;
                            pay = lh == (uint32_t)x ? half : pay;
                        }
                        if (lane <= NWD)
                            __hip_atomic_store(out + lane, ((unsigned long long)cyc << 32) | pay, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                    }
                    // next sweep's uniforms while the partners' words travel
                    if (intra || cross) {
                        rn[0] = philox_v((uint32_t)lane, (uint32_t)(t + 1), (uint32_t)lab0, TAG_SWEEP, P.k0, P.k1);
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
                            const int dEs = lower ? pE - E[0] : E[0] - pE;
                            const bool okx = swap_ok(dEs, __builtin_amdgcn_readlane(u_vec, NP * (cyc - u_base) + pi),
                                                     __builtin_amdgcn_readlane(row_off_v, pi),
                                                     __builtin_amdgcn_readlane(row_len_v, pi), tsw);
                            if (lower) {   // the lower member owns the pair's counters
                                satt[0] += 1;
                                sacc[0] += okx ? 1u : 0u;
                            }
                            buf[0] = okx ? pb : buf[0];
                            E[0] = okx ? pE : E[0];
                        }
                    }
                    if (cross && !failed) {
                        const int pw = lower ? it.w + 1 : it.w - 1;
                        const unsigned long long *in =
                            it.xbuf + ((size_t)(pw * 2 + (1 - side)) * 2 + buf_x) * it.xwords;
                        uint32_t *stage = xstage + (size_t)(wv * 2 + side) * (NWD + 1);
                        uint32_t polls = 0;
                        bool ok_all = false;
                        unsigned long long bad = 0;
                        for (;;) {
                            bool ok = true;
                            if (lane <= NWD) {
                                const unsigned long long v =
                                    __hip_atomic_load(in + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                                if ((uint32_t)(v >> 32) == cyc) stage[lane] = (uint32_t)v;
                                else {
                                    ok = false;
                                    bad = v;
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
                            const int pE = __builtin_amdgcn_readfirstlane((int)stage[NWD]);
                            const int dEs = lower ? pE - E[0] : E[0] - pE;
                            const bool okx = swap_ok(dEs, __builtin_amdgcn_readlane(u_vec, NP * (cyc - u_base) + pi),
                                                     __builtin_amdgcn_readlane(row_off_v, pi),
                                                     __builtin_amdgcn_readlane(row_len_v, pi), tsw);
                            if (lower) {
                                satt[0] += 1;
                                if (okx) sacc[0] += 1;
                            }
                            E[0] = okx ? pE : E[0];
                            if (okx) {
                                // this lane's row: bit (lane & 31) of words 2x + (lane >> 5)
                                const int h = lane >> 5, bit = lane & 31;
                                uint32_t wx[8];
#pragma unroll
                                for (int x = 0; x < 8; ++x) wx[x] = stage[2 * x + h];
                                uint2 d;
                                d.x = d.y = 0;
#pragma unroll
                                for (int x = 0; x < 8; ++x) {
                                    const uint32_t down = ((wx[x] >> bit) & 1u) ^ 1u;
                                    if (x < 4) d.x |= down << (8 * x);
                                    else d.y |= down << (8 * (x - 4));
                                }
                                *(uint2 *)(bufs + buf[0] * N + rel_me) = d;
                            }
                        }
                    }
                } else {
                    if (cyc & 1) {
                        // pairs (2w, 2w+1): inside this wavefront
                        const int r = lab0;
                        if (r + 1 < P.R) {
                            const bool ok = swap_ok(E[1] - E[0], __builtin_amdgcn_readlane(u_vec, NP * (cyc - u_base) + 1),
                                                    __builtin_amdgcn_readlane(row_off_v, 1),
                                                    __builtin_amdgcn_readlane(row_len_v, 1), tsw);
                            satt[0] += 1;
                            sacc[0] += ok ? 1u : 0u;
                            const int b0 = buf[0], b1 = buf[1], e0 = E[0], e1 = E[1];
                            buf[0] = ok ? b1 : b0;
                            buf[1] = ok ? b0 : b1;
                            E[0] = ok ? e1 : e0;
                            E[1] = ok ? e0 : e1;
                        }
                    } else {
                        // pairs (2w+1, 2w+2): with the next wavefront or across the upper
                        // boundary; (2w-1, 2w): with the previous one or across the lower
                        const int lu = SPW * wv + 1;                 // local slot of the upper one
                        unsigned long long *mb = mail + (cyc & 3) * G;
                        const bool up_here = lab0 + 2 < P.R && wv + 1 < NWV;
                        const bool dn_here = wv > 0;
                        // publish (energy, buffer) of the slots that meet a neighbour wavefront
                        // LDS operations of a wavefront complete in order, so the row
                        // writes of the sweep land before these words; only the
                        // compiler must not move them past (signal fence)
                        __atomic_signal_fence(__ATOMIC_SEQ_CST);
                        if (lane == 0) {
                            if (up_here)
                                __hip_atomic_store(mb + lu, ((unsigned long long)cyc << 32) | ((uint32_t)buf[1] << 24) |
                                                                ((uint32_t)E[1] & 0xFFFFFFu),
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                            if (dn_here)
                                __hip_atomic_store(mb + lu - 1, ((unsigned long long)cyc << 32) | ((uint32_t)buf[0] << 24) |
                                                                    ((uint32_t)E[0] & 0xFFFFFFu),
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        }
                        // across the workgroup boundaries: publish first (one store of
                        // 17 tagged words: lane 2x + h holds the sites 8q + x of rows
                        // q = 32h .. 32h + 31, one ballot per x, bit set = spin +1;
                        // lane 16 the energy), then settle the pairs inside the
                        // workgroup while the words travel, then poll
                        const int buf_x = (cyc >> 1) & 1;
                        const unsigned long long tag = (unsigned long long)cyc << 32;
#pragma unroll
                        for (int side = 0; side < 2; ++side) {
                            const int k = side == 0 ? 0 : 1;
                            const bool cross = side == 0 ? (wv == 0 && has_down && lab0 >= 1)
                                                         : (wv + 1 == NWV && has_up && lab0 + 2 < P.R);
                            if (!cross || failed) continue;
                            unsigned long long *out = it.xbuf + ((size_t)(it.w * 2 + side) * 2 + buf_x) * it.xwords;
                            const uint2 row = *(const uint2 *)(bufs + buf[k] * N + rel_me);
                            uint32_t pay = (uint32_t)E[k];
                            // lane >> 1 made opaque here: otherwise the compiler keeps the eight
                            // lane masks (lane >> 1) == x in SGPRs for the whole launch
                            const uint32_t lh = opaque((uint32_t)lane >> 1);
#pragma unroll
                            for (int x = 0; x < 8; ++x) {
                                const uint32_t byte = ((x < 4 ? row.x : row.y) >> (8 * (x & 3))) & 0xFFu;
                                const unsigned long long bal = __ballot(byte == 0);
                                const uint32_t half = (lane & 1) ? (uint32_t)(bal >> 32) : (uint32_t)bal;
                                pay = lh == (uint32_t)x ? half : pay;
                            }
                            if (lane <= NWD)
                                __hip_atomic_store(out + lane, tag | pay, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        }
                        if (!failed) {
                            // inside the workgroup: read the neighbour wavefronts' words
#pragma unroll
                            for (int side = 0; side < 2; ++side) {
                                const bool here = side == 0 ? dn_here : up_here;
                                if (!here || failed) continue;
                                const int k = side == 0 ? 0 : 1;
                                const int pl = side == 0 ? SPW * wv - 1 : SPW * wv + 2;   // partner local slot
                                uint32_t polls = 0;
                                unsigned long long v;
                                for (;;) {
                                    v = __hip_atomic_load(mb + pl, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
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
                                    continue;
                                }
                                // every value here is wave-uniform: keep it scalar
                                const uint32_t lo32 = __builtin_amdgcn_readfirstlane((uint32_t)v);
                                const int pE = ((int)(lo32 << 8)) >> 8;      // 24-bit signed energy
                                const int pb = (int)((lo32 >> 24) & 0xFFu);
                                const int slot = lab0 + k;
                                const int r = side == 0 ? slot - 1 : slot;
                                const int pi = r - (lab0 - 1);                // 0 or 2
                                const int dEs = side == 0 ? E[k] - pE : pE - E[k];
                                const bool okx = swap_ok(dEs, __builtin_amdgcn_readlane(u_vec, NP * (cyc - u_base) + pi),
                                                         __builtin_amdgcn_readlane(row_off_v, pi),
                                                         __builtin_amdgcn_readlane(row_len_v, pi), tsw);
                                if (side == 1) {
                                    satt[1] += 1;
                                    sacc[1] += okx ? 1u : 0u;
                                }
                                // trade buffers on acceptance: the partner takes ours
                                buf[k] = okx ? pb : buf[k];
                                E[k] = okx ? pE : E[k];
                            }
                        }
                        // across the workgroup boundaries: poll, decide, copy
#pragma unroll
                        for (int side = 0; side < 2; ++side) {
                            const int k = side == 0 ? 0 : 1;
                            const bool cross = side == 0 ? (wv == 0 && has_down && lab0 >= 1)
                                                         : (wv + 1 == NWV && has_up && lab0 + 2 < P.R);
                            if (!cross || failed) continue;
                            const int pw = side == 0 ? it.w - 1 : it.w + 1;
                            const unsigned long long *in =
                                it.xbuf + ((size_t)(pw * 2 + (side == 0 ? 1 : 0)) * 2 + buf_x) * it.xwords;
                            uint32_t *stage = xstage + (size_t)(wv * 2 + side) * (NWD + 1);
                            uint32_t polls = 0;
                            bool ok_all = false;
                            unsigned long long bad = 0;
                            for (;;) {
                                bool ok = true;
                                if (lane <= NWD) {
                                    const unsigned long long v =
                                        __hip_atomic_load(in + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                                    if ((uint32_t)(v >> 32) == cyc) stage[lane] = (uint32_t)v;
                                    else {
                                        ok = false;
                                        bad = v;
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
                                continue;
                            }
                            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                            __builtin_amdgcn_wave_barrier();
                            const int pE = __builtin_amdgcn_readfirstlane((int)stage[NWD]);
                            const int slot = lab0 + k;
                            const int r = side == 0 ? slot - 1 : slot;
                            const int pi = r - (lab0 - 1);                    // 0 or 2
                            const int dEs = side == 0 ? E[k] - pE : pE - E[k];
                            const bool okx = swap_ok(dEs, __builtin_amdgcn_readlane(u_vec, NP * (cyc - u_base) + pi),
                                                     __builtin_amdgcn_readlane(row_off_v, pi),
                                                     __builtin_amdgcn_readlane(row_len_v, pi), tsw);
                            if (side == 1) {   // the lower workgroup owns the pair's counters
                                satt[1] += 1;
                                if (okx) sacc[1] += 1;
                            }
                            E[k] = okx ? pE : E[k];
                            if (okx) {
                                // this lane's row: bit (lane & 31) of words 2x + (lane >> 5)
                                const int h = lane >> 5, bit = lane & 31;
                                uint32_t wx[8];
#pragma unroll
                                for (int x = 0; x < 8; ++x) wx[x] = stage[2 * x + h];
                                uint2 d;
                                d.x = d.y = 0;
#pragma unroll
                                for (int x = 0; x < 8; ++x) {
                                    const uint32_t down = ((wx[x] >> bit) & 1u) ^ 1u;
                                    if (x < 4) d.x |= down << (8 * x);
                                    else d.y |= down << (8 * (x - 4));
                                }
                                *(uint2 *)(bufs + buf[k] * N + rel_me) = d;
                            }
                        }
                    }
                }
            } else {
                ++phase;
            }
            if (!drawn) {
#pragma unroll
                for (int k = 0; k < SPW; ++k)
                    rn[k] = philox_v((uint32_t)lane, (uint32_t)(t + 1), (uint32_t)(lab0 + k), TAG_SWEEP, P.k0, P.k1);
            }
            // ---- best energy and first hit, per slot ----
#pragma unroll
            for (int k = 0; k < SPW; ++k) {
                if (want_hit && hit[k] < 0 && E[k] <= P.target) hit[k] = (long long)t;
                if (E[k] < bestE[k]) {
                    bestE[k] = E[k];
                    bestT[k] = (long long)t;
                    bestSlot[k] = lab0 + k;
                    const uint2 v = *(const uint2 *)(bufs + buf[k] * N + rel_me);
                    uint2 o;
                    o.x = v.x * 0xFEu + 0x01010101u;       // down-bit 1 -> -1 (0xFF), 0 -> +1
                    o.y = v.y * 0xFEu + 0x01010101u;
                    *(uint2 *)(it.best_spins + (size_t)(SPW * wv + k) * N + rel_me) = o;
                }
            }
        }
    }

    // ---- end of launch ----
    __shared__ int any_failed, win;
    __shared__ int slot_buf[64], slot_E[64];
    __shared__ Rec rec[64];
    __shared__ unsigned cnt[64][5];
    if (tid == 0) any_failed = 0;
    __syncthreads();
    if (active) {
        unsigned nfw[SPW];
#pragma unroll
        for (int k = 0; k < SPW; ++k) nfw[k] = (unsigned)wave_sum((int)nflip[k]);
        if (failed && lane == 0) any_failed = 1;
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < SPW; ++k) {
                const int l = SPW * wv + k;
                slot_buf[l] = buf[k];
                slot_E[l] = E[k];
                Rec rr;
                rr.E = bestE[k];
                rr.slot = bestSlot[k];
                rr.t = bestT[k];
                rr.hit = hit[k];
                rec[l] = rr;
                cnt[l][0] = nfw[k];
                cnt[l][1] = satt[k];
                cnt[l][2] = sacc[k];
                cnt[l][3] = patt[k];
                cnt[l][4] = pacc[k];
            }
        }
    }
    __syncthreads();
    if (any_failed) return;   // the host reports the error; the launch's state is abandoned
    for (int x = tid; x < G * N / 4; x += bs) {
        const int l = x / (N / 4), w4 = x - l * (N / 4);
        const uint32_t v = *(const uint32_t *)(bufs + slot_buf[l] * N + 4 * w4);
        *(uint32_t *)(I.spins + (size_t)(s0 + l) * N + 4 * w4) = v * 0xFEu + 0x01010101u;
    }
    for (int l = tid; l < G; l += bs) {
        const int slot = s0 + l;
        I.E[slot] = slot_E[l];
        I.flips[slot] += cnt[l][0];
        I.prop_att[slot] += cnt[l][3];
        I.prop_acc[slot] += cnt[l][4];
        const int Bn = I.bank_n[slot];
        if (Bn > 0) I.cursor[slot] = (int)(((uint32_t)I.cursor[slot] + n_prop % (uint32_t)Bn) % (uint32_t)Bn);
    }
    // swap counters: pair (2w, 2w+1) in slot 2w's k=0 entry; pair (2w+1, 2w+2) in k=1
    for (int l = tid; l < G; l += bs) {
        const int slot = s0 + l;
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
        for (int i = tid; i < N; i += bs) it.best_spins[i] = it.best_spins[(size_t)win * N + i];
}

// ---------------------------------------------------------------------------
// Host-side launchers (C++ linkage, used by the runtime in host.cpp).

// spw: slots per wavefront (1 or 2); a workgroup holds at most 8 wavefronts
int pm_max_storages(int spw) { return spw == 1 ? 8 : 16; }

size_t pm_lds_bytes(int G, int tsw_entries) { return pm::offsets(G, tsw_entries).total; }

hipError_t launch_pm(int spw, const ChunkArgs &a, int block, size_t lds, hipStream_t s)
{
    if (spw == 1) hipLaunchKernelGGL(pm_kernel<1>, dim3(a.n_items), dim3(block), lds, s, a);
    else hipLaunchKernelGGL(pm_kernel<2>, dim3(a.n_items), dim3(block), lds, s, a);
    return hipGetLastError();
}

hipError_t pm_occupancy(int spw, int block, size_t lds, int *blocks_per_cu)
{
    const void *f = spw == 1 ? (const void *)pm_kernel<1> : (const void *)pm_kernel<2>;
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return spw == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, pm_kernel<1>, block, lds)
                    : hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, pm_kernel<2>, block, lds);
}

} // namespace tapt
