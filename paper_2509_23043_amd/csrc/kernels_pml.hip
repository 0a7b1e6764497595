// Persistent kernel for +-J couplings on periodic L^3 lattices of any even L
// from 6 to 16 (no fields): one beta slot per wavefront, byte-parallel
// arithmetic over rows of sites, and lattices of several sizes in one launch
// (each workgroup runs the body of its own instance's L).
//
// Storage. A replica is L^2 rows of L sites (row r = y + L z holds x = 0..L-1,
// site index i = x + L r), one byte per site that is 1 when the spin is -1,
// each row padded to RB = 8 (L <= 8) or 16 bytes with zero bytes. Lane q of
// the wavefront owns the rows q, q + 64, ... . The slot's sweep uniforms
// (Philox call q serves sites 8q .. 8q + 7, Methods) are drawn at the start of
// each sweep by the lane of each row: a row of L sites (L even) starts at a
// whole 32-bit word of a call, so the row's uniforms are whole words of at
// most three consecutive calls and stay in the lane's registers.
//
// Local field. With b the down-bit of a site, n that of a neighbour and j = 1
// when their bond is -1, the bond is unsatisfied exactly when j ^ b ^ n = 1.
// A colour phase updates the sites x = p, p + 2, ... of each row (p = (colour
// + y + z) mod 2), four sites per 8-byte chunk: v_perm gathers their bytes,
// and those of their neighbours along y and z from whole-row LDS reads and
// along x from the own row rotated by one byte (periodic in L), three-input
// XORs with the bond-sign bytes (precomputed per row in LDS) form the six
// unsatisfied-bond flags, and byte-wise adds count them (U <= 6, no carries).
// Then m_i I_i = 6 - 2U and the flip changes E by 12 - 4U (Methods, Eq. 4).
// The upper halves of the slot's thresholds by U sit in registers as byte
// tables, so one v_perm looks up four sites and saturating 16-bit
// subtractions test them against their uniforms' upper halves; a tie takes
// the exact 32-bit test with the lower half from the refinement draw.
//
// Slots and states. The slot of a wavefront is fixed; states move between LDS
// buffers. A pair that spans two wavefronts meets in an LDS mailbox carrying
// the energy and the buffer index, and an accepted swap (Eq. 1) trades buffer
// indices. A pair across a workgroup boundary exchanges cycle-tagged words
// through global memory (the state as bits, each lane its own rows, and the
// energy) and copies the state on acceptance. Proposals (Eq. 2) read
// the bank configuration into the slot's buffer. Best energy, first hit and
// every counter are per slot and live in registers.
#include "sweep.h"

namespace tapt {

namespace pml {

constexpr int MAXG = 8;   // slots (wavefronts) per workgroup

template <int L>
struct Geo {
    static_assert(L % 2 == 0 && L >= 6 && L <= 16, "even L in 6..16");
    static constexpr int N = L * L * L;
    static constexpr int NR = L * L;                 // rows
    static constexpr int RB = L <= 8 ? 8 : 16;       // LDS bytes per row
    static constexpr int NW = RB / 4;                // dwords per row
    static constexpr int NCH = RB / 8;               // 8-byte chunks per row
    static constexpr int RPL = (NR + 63) / 64;       // rows per lane
    static constexpr int SBUF = NR * RB;             // bytes per state buffer
    static constexpr int JW = 2 * NCH * 6;           // bond-sign words per row
    // A state crosses a workgroup boundary as XW words per lane (lane q's
    // rows, RB bits each: bit x of row j at bit RB j + x of its bit stream),
    // word k of lane q at q + 64 k; the energy word follows at NXW.
    static constexpr int XW = (RPL * RB + 31) / 32;
    static constexpr int NXW = 64 * XW;
    // A row's first site L r sits at half (L r) mod 8 of Philox call (L r) / 8;
    // L is even, so that offset is a whole 32-bit word, TOFF words at most,
    // and the row's uniforms are NCALL consecutive calls' words from there.
    static constexpr int TOFF = L % 8 == 0 ? 0 : L % 4 == 0 ? 2 : 3;
    static constexpr int NCALL = (L + 2 * TOFF + 7) / 8;
};

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel)
{
    return __builtin_amdgcn_perm(hi, lo, sel);
}

// v_perm selectors on an 8-byte chunk {hi, lo} (bytes 0-3 from lo, 4-7 from hi)
__device__ __forceinline__ uint32_t sel_sites(int p) { return p ? 0x07050301u : 0x06040200u; }   // x = p + 2j
// the 16-bit halves p of words j and j + 1 side by side
__device__ __forceinline__ uint32_t sel_pair(int p) { return p ? 0x07060302u : 0x05040100u; }
// compact flags (byte j for x = p + 2j) back to the chunk's low and high dword (0x0c: zero byte)
__device__ __forceinline__ uint32_t sel_flo(int p) { return p ? 0x010c000cu : 0x0c010c00u; }
__device__ __forceinline__ uint32_t sel_fhi(int p) { return p ? 0x030c020cu : 0x0c030c02u; }

// LDS carve-up of one workgroup of G slots of an L^3 lattice
struct Off {
    size_t buf, jn, tabu, toff, tsw, mail, total;
};

template <int L>
__host__ __device__ inline Off offsets(int G, int tsw_entries)
{
    using Gm = Geo<L>;
    Off f;
    size_t o = 0;
    f.buf = o; o = align16(o + (size_t)G * Gm::SBUF);
    f.jn = o; o = align16(o + (size_t)Gm::NR * Gm::JW * 4);
    f.tabu = o; o = align16(o + (size_t)G * 8 * 4);
    f.toff = o; o = align16(o + (size_t)(G + 2) * 4);
    f.tsw = o; o = align16(o + (size_t)tsw_entries * 4);
    f.mail = o; o = align16(o + (size_t)4 * G * 8);
    f.total = o;
    return f;
}

struct Rec {
    int E, slot;
    long long t, hit;
};

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

// The row rotated by one site along x, periodic in L: xp[x] = o[(x + 1) % L]
// and xm[x] = o[(x - 1) % L] for x < L (padding bytes are don't-care).
template <int L>
__device__ __forceinline__ void rotate_row(const uint32_t (&o)[Geo<L>::NW], uint32_t (&xp)[Geo<L>::NW],
                                           uint32_t (&xm)[Geo<L>::NW])
{
    constexpr int NW = Geo<L>::NW, RB = Geo<L>::RB;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        xp[w] = __builtin_amdgcn_alignbyte(o[(w + 1) % NW], o[w], 1);           // bytes 4w+1 .. 4w+4
        xm[w] = __builtin_amdgcn_alignbyte(o[w], o[(w + NW - 1) % NW], 3);      // bytes 4w-1 .. 4w+2
    }
    if constexpr (RB != L) {
        // x = L - 1 takes site 0; x = 0 takes site L - 1
        constexpr int wp = (L - 1) / 4, bp = (L - 1) % 4;
        constexpr uint32_t selp = (0x03020100u & ~(0xFFu << (8 * bp))) | (0x04u << (8 * bp));
        xp[wp] = perm(o[0], xp[wp], selp);
        constexpr uint32_t selm = 0x03020100u & ~0xFFu;
        xm[0] = perm(o[wp], xm[0], selm | (uint32_t)(4 + bp));
    }
}

} // namespace pml

template <int L>
__device__ __forceinline__ void pml_body(const ChunkArgs a, const int item)
{
    using namespace pml;
    using Gm = Geo<L>;
    constexpr int N = Gm::N, NR = Gm::NR, RB = Gm::RB, NW = Gm::NW, NCH = Gm::NCH, RPL = Gm::RPL;
    constexpr int SBUF = Gm::SBUF, JW = Gm::JW, NXW = Gm::NXW;
    constexpr int NP = 2;                     // pairs a slot takes part in
    const WorkItem it = a.items[item];
    const InstDev &I = *it.inst;
    RunParams P;
    P.load(I);
    const int G = it.G, s0 = it.s0;
    const int tid = threadIdx.x, bs = blockDim.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const uint64_t t0 = *I.t;
    const uint64_t cap = chunk_cap(I, t0);
    const uint64_t tend = (t0 + a.K < cap) ? t0 + a.K : cap;
    if (t0 >= tend) {
        if (tid == 0) idle_best(it.best);
        return;
    }
    const Off lof = offsets<L>(G, a.tsw_entries);
    uint8_t *bufs = (uint8_t *)(lds_raw + lof.buf);
    uint32_t *jn = (uint32_t *)(lds_raw + lof.jn);              // [NR][2 colours][NCH][6 directions]
    uint32_t *tabu = (uint32_t *)(lds_raw + lof.tabu);          // [G][8] threshold by U
    int *tsw_off = (int *)(lds_raw + lof.toff);
    uint32_t *tsw = (uint32_t *)(lds_raw + lof.tsw);
    unsigned long long *mail = (unsigned long long *)(lds_raw + lof.mail);   // [4][G]

    // ---- stage: states as down-bits in row layout (slot l in buffer l), bond signs, tables ----
    for (int x = tid; x < G * SBUF / 4; x += bs) ((uint32_t *)bufs)[x] = 0u;
    __syncthreads();
    for (int x = tid; x < G * N; x += bs) {
        const int l = x / N, i = x - l * N;
        const int r = i / L, xx = i - r * L;
        bufs[l * SBUF + r * RB + xx] = I.spins[(size_t)(s0 + l) * N + i] < 0 ? 1 : 0;
    }
    const int8_t *J3 = I.J3;
    for (int e = tid; e < NR * JW; e += bs) {
        const int r = e / JW, q = e - r * JW;
        const int c = q / (NCH * 6), ch = (q / 6) % NCH, d = q % 6;
        const int y = r % L, z = r / L;
        const int p = (c + y + z) & 1;
        uint32_t w = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int x = p + 2 * j + 8 * ch;
            if (x >= L) continue;
            const int i = x + L * r;
            int jb;
            if (d == 0) jb = J3[i];
            else if (d == 1) jb = J3[(x + L - 1) % L + L * r];
            else if (d == 2) jb = J3[N + i];
            else if (d == 3) jb = J3[N + x + L * ((y + L - 1) % L + L * z)];
            else if (d == 4) jb = J3[2 * N + i];
            else jb = J3[2 * N + x + L * (y + L * ((z + L - 1) % L))];
            w |= (uint32_t)(jb < 0 ? 1 : 0) << (8 * j);
        }
        jn[e] = w;
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
        // coarse thresholds (upper 16 bits by U) as byte tables for v_perm:
        // tb* the high bytes, tl* the low bytes, *l for U = 0..3, *h for U = 4..7
        uint32_t tbl = 0, tbh = 0, tll = 0, tlh = 0;
        {
            const uint32_t *tu = tabu + wv * 8;
#pragma unroll
            for (int U = 0; U < 4; ++U) {
                tbl |= (tu[U] >> 24) << (8 * U);
                tbh |= (tu[U + 4] >> 24) << (8 * U);
                tll |= ((tu[U] >> 16) & 0xFFu) << (8 * U);
                tlh |= ((tu[U + 4] >> 16) & 0xFFu) << (8 * U);
            }
        }
        const uint32_t ONE2 = 0x00010001u;
        uint32_t cyc = (uint32_t)(t0 / (uint64_t)P.M), phase = (uint32_t)(t0 % (uint64_t)P.M);
        uint64_t prop_at = P.first_prop_from(t0 + 1);
        // the slot's exchange by cycle parity, three bits per parity (1: lower
        // member of its pair, 2: partner in this workgroup, 4: partner across
        // a workgroup boundary), tested as bits of one scalar
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
        // swap uniforms of the slot's two pairs for UCYC cycles: lane NP c + i
        // holds pair slot - 1 + i at cycle u_base + c
        constexpr uint32_t UCYC = 64 / NP;
        uint32_t u_vec = 0, u_base = (uint32_t)-100;
        const uint32_t u_i = (uint32_t)lane % (uint32_t)NP, u_c = (uint32_t)lane / (uint32_t)NP;

        for (uint64_t t = t0 + 1; t <= tend && !failed; ++t) {
            const bool ends = phase + 1 == (uint32_t)P.M;
            if (ends && cyc + 1 - u_base >= UCYC) {
                u_base = cyc + 1;
                u_vec = philox_v((uint32_t)(slot - 1) + u_i, u_base + u_c, 0, TAG_SWAP, P.k0, P.k1).v[0];
            }
            // ---- the sweep's uniforms: word k of row j holds sites x = 2k, 2k + 1 ----
            uint32_t rwr[RPL][RB / 2];
#pragma unroll
            for (int j = 0; j < RPL; ++j) {
                const int base = L * (lane + 64 * j);            // first site of the row
                const uint32_t q0 = (uint32_t)(base >> 3);
                uint32_t W[4 * Gm::NCALL];
#pragma unroll
                for (int k = 0; k < Gm::NCALL; ++k) {
                    const P4 rr = philox_v(q0 + (uint32_t)k, (uint32_t)t, (uint32_t)slot, TAG_SWEEP, P.k0, P.k1);
#pragma unroll
                    for (int v = 0; v < 4; ++v) W[4 * k + v] = rr.v[v];
                }
                const int toff = (base & 7) >> 1;                // 0 .. TOFF
#pragma unroll
                for (int k = 0; k < RB / 2; ++k) {
                    uint32_t w = W[k < 4 * Gm::NCALL ? k : 4 * Gm::NCALL - 1];
#pragma unroll
                    for (int d = 1; d <= Gm::TOFF; ++d) {
                        const int src = k + d < 4 * Gm::NCALL ? k + d : 4 * Gm::NCALL - 1;   // past x = L - 1: unused
                        w = toff == d ? W[src] : w;
                    }
                    rwr[j][k] = w;
                }
            }

            // ---- the sweep: colour phases, the lane's rows ----
            const uint32_t B = (uint32_t)(buf * SBUF);
            int nf = 0, su = 0;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                // a row's reads (its own row, the four y and z neighbour rows, its
                // bond-sign words): issued for row j + 1 before row j is decided and
                // written back, which they never alias (row j + 1's neighbours are
                // rows r + 64 +- 1 and +- L, none of them r)
                struct RowIn {
                    uint32_t o[NW], yp[NW], ym[NW], zp[NW], zm[NW], jw[NCH * 6];
                };
                auto row_in = [&](int j, RowIn &v) {
                    const int r = lane + 64 * j;
                    if (NR % 64 != 0 && r >= NR) return;
                    const int y = r % L, z = r / L;
                    const uint32_t a_me = B + r * RB;
                    const uint32_t a_yp = B + (((y + 1) % L) + L * z) * RB, a_ym = B + (((y + L - 1) % L) + L * z) * RB;
                    const uint32_t a_zp = B + (y + L * ((z + 1) % L)) * RB, a_zm = B + (y + L * ((z + L - 1) % L)) * RB;
                    if constexpr (NW == 2) {
                        const uint2 v0 = *(const uint2 *)(bufs + a_me), v1 = *(const uint2 *)(bufs + a_yp);
                        const uint2 v2 = *(const uint2 *)(bufs + a_ym), v3 = *(const uint2 *)(bufs + a_zp);
                        const uint2 v4 = *(const uint2 *)(bufs + a_zm);
                        v.o[0] = v0.x; v.o[1] = v0.y; v.yp[0] = v1.x; v.yp[1] = v1.y; v.ym[0] = v2.x; v.ym[1] = v2.y;
                        v.zp[0] = v3.x; v.zp[1] = v3.y; v.zm[0] = v4.x; v.zm[1] = v4.y;
                    } else {
                        const uint4 v0 = *(const uint4 *)(bufs + a_me), v1 = *(const uint4 *)(bufs + a_yp);
                        const uint4 v2 = *(const uint4 *)(bufs + a_ym), v3 = *(const uint4 *)(bufs + a_zp);
                        const uint4 v4 = *(const uint4 *)(bufs + a_zm);
                        v.o[0] = v0.x; v.o[1] = v0.y; v.o[2] = v0.z; v.o[3] = v0.w;
                        v.yp[0] = v1.x; v.yp[1] = v1.y; v.yp[2] = v1.z; v.yp[3] = v1.w;
                        v.ym[0] = v2.x; v.ym[1] = v2.y; v.ym[2] = v2.z; v.ym[3] = v2.w;
                        v.zp[0] = v3.x; v.zp[1] = v3.y; v.zp[2] = v3.z; v.zp[3] = v3.w;
                        v.zm[0] = v4.x; v.zm[1] = v4.y; v.zm[2] = v4.z; v.zm[3] = v4.w;
                    }
                    const uint32_t *js = jn + r * JW + c * NCH * 6;
#pragma unroll
                    for (int q = 0; q < NCH * 6; q += 2) {
                        const uint2 w = *(const uint2 *)(js + q);
                        v.jw[q] = w.x;
                        v.jw[q + 1] = w.y;
                    }
                };
                RowIn nxt;
                row_in(0, nxt);
#pragma unroll
                for (int j = 0; j < RPL; ++j) {
                    const int r = lane + 64 * j;
                    if (NR % 64 != 0 && r >= NR) continue;
                    const RowIn cur = nxt;
                    if (j + 1 < RPL) row_in(j + 1, nxt);
                    // keep the scheduler from sinking those reads below row j's work
                    __builtin_amdgcn_sched_barrier(0);
                    const int y = r % L, z = r / L;
                    const int p = (c + y + z) & 1;
                    const uint32_t a_me = B + r * RB;
                    uint32_t o[NW], yp[NW], ym[NW], zp[NW], zm[NW], rw[2 * NW], jw[NCH * 6];
#pragma unroll
                    for (int k = 0; k < RB / 2; ++k) rw[k] = rwr[j][k];
#pragma unroll
                    for (int w = 0; w < NW; ++w) {
                        o[w] = cur.o[w];
                        yp[w] = cur.yp[w];
                        ym[w] = cur.ym[w];
                        zp[w] = cur.zp[w];
                        zm[w] = cur.zm[w];
                    }
#pragma unroll
                    for (int q = 0; q < NCH * 6; ++q) jw[q] = cur.jw[q];
                    uint32_t xp[NW], xm[NW];
                    rotate_row<L>(o, xp, xm);
                    const uint32_t S = sel_sites(p), Hp = sel_pair(p);
#pragma unroll
                    for (int ch = 0; ch < NCH; ++ch) {
                        const int w0 = 2 * ch, w1 = 2 * ch + 1;
                        const uint32_t b = perm(o[w1], o[w0], S);
                        const uint32_t U = xor3(jw[6 * ch + 0], b, perm(xp[w1], xp[w0], S)) +
                                           xor3(jw[6 * ch + 1], b, perm(xm[w1], xm[w0], S)) +
                                           xor3(jw[6 * ch + 2], b, perm(yp[w1], yp[w0], S)) +
                                           xor3(jw[6 * ch + 3], b, perm(ym[w1], ym[w0], S)) +
                                           xor3(jw[6 * ch + 4], b, perm(zp[w1], zp[w0], S)) +
                                           xor3(jw[6 * ch + 5], b, perm(zm[w1], zm[w0], S));
                        const uint32_t TB = perm(tbh, tbl, U), TL = perm(tlh, tll, U);
                        const uint32_t T01 = perm(TB, TL, 0x05010400u), T23 = perm(TB, TL, 0x07030602u);
                        const uint32_t U01 = perm(rw[4 * ch + 1], rw[4 * ch], Hp);
                        const uint32_t U23 = perm(rw[4 * ch + 3], rw[4 * ch + 2], Hp);
                        uint32_t F = perm(pk_min_u16(pk_sub_sat_u16(T23, U23), ONE2),
                                          pk_min_u16(pk_sub_sat_u16(T01, U01), ONE2), 0x06040200u);
                        const uint32_t Z = pk_min_u16(pk_min_u16(T01 ^ U01, T23 ^ U23), ONE2);
                        if (__builtin_expect(any_lane(Z != ONE2), 0)) {
                            // exact test of the four sites: u = (upper << 16) | lower,
                            // the lower half from the refinement draw of the site's call
                            uint32_t Fx = 0;
#pragma unroll
                            for (int k = 0; k < 4; ++k) {
                                const int x = p + 2 * k + 8 * ch;
                                const int i = x + L * r;
                                const uint32_t T = tabu[wv * 8 + ((U >> (8 * k)) & 0xFFu)];
                                const uint32_t hi = ((k < 2 ? U01 : U23) >> (16 * (k & 1))) & 0xFFFFu;
                                const P4 r2 = philox(opaque((uint32_t)(i >> 3)), (uint32_t)t, (uint32_t)slot, TAG_REFINE,
                                                     P.k0, P.k1);
                                const int h = i & 7;
                                const uint32_t wd = h < 2 ? r2.v[0] : h < 4 ? r2.v[1] : h < 6 ? r2.v[2] : r2.v[3];
                                const uint32_t lo = (h & 1) ? (wd >> 16) : (wd & 0xFFFFu);
                                const uint32_t u = (hi << 16) | lo;
                                Fx |= (T == ALWAYS || u < T) ? (1u << (8 * k)) : 0u;
                            }
                            F = Fx;
                        }
                        if constexpr (L % 8 != 0) {
                            // sites past x = L - 1 are padding
                            if (ch == NCH - 1) {
                                uint32_t vm = 0;
#pragma unroll
                                for (int k = 0; k < 4; ++k)
                                    vm |= (p + 2 * k + 8 * ch < L) ? (0xFFu << (8 * k)) : 0u;
                                F &= vm;
                            }
                        }
                        o[w0] ^= perm(0u, F, sel_flo(p));
                        o[w1] ^= perm(0u, F, sel_fhi(p));
                        nf += __builtin_popcount(F);
                        su = (int)__builtin_amdgcn_udot4(U, F, (uint32_t)su, false);
                    }
                    // the row goes back whether or not a site flipped: no branch
                    if constexpr (NW == 2) *(uint2 *)(bufs + a_me) = make_uint2(o[0], o[1]);
                    else *(uint4 *)(bufs + a_me) = make_uint4(o[0], o[1], o[2], o[3]);
                }
                // the next colour reads what this one wrote (in-order LDS within a wavefront)
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
            nflip += (unsigned)nf;
            E += wave_sum(12 * nf - 4 * su);

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
                            const int8_t *src = I.bank[slot] + (size_t)kk * N;
#pragma unroll
                            for (int j = 0; j < RPL; ++j) {
                                const int r = lane + 64 * j;
                                if (NR % 64 != 0 && r >= NR) continue;
                                uint32_t o[NW];
#pragma unroll
                                for (int w = 0; w < NW; ++w) o[w] = 0;
#pragma unroll
                                for (int x = 0; x < L; ++x)
                                    o[x >> 2] |= (uint32_t)(src[L * r + x] < 0 ? 1 : 0) << (8 * (x & 3));
                                if constexpr (NW == 2) *(uint2 *)(bufs + buf * SBUF + r * RB) = make_uint2(o[0], o[1]);
                                else *(uint4 *)(bufs + buf * SBUF + r * RB) = make_uint4(o[0], o[1], o[2], o[3]);
                            }
                            E = ET;
                            pacc += 1;
                        }
                    }
                    ++n_prop;
                }
                // ---- swap (Eq. 1), alternating parity: the slot is the lower
                // member of its pair when its parity differs from the cycle's ----
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
                    // the state as bits, each lane its own rows: a row's down-bytes
                    // (0 or 1) fold four at a time into bits by a dot product with
                    // 1, 2, 4, 8 (bit x of the row is site x)
                    unsigned long long *out = it.xbuf + ((size_t)(it.w * 2 + side) * 2 + buf_x) * it.xwords;
                    uint32_t pay[Gm::XW];
#pragma unroll
                    for (int k = 0; k < Gm::XW; ++k) pay[k] = 0u;
#pragma unroll
                    for (int j = 0; j < RPL; ++j) {
                        const int r = lane + 64 * j;
                        uint32_t bits = 0;
                        if (NR % 64 == 0 || r < NR) {
                            uint32_t o[NW];
                            if constexpr (NW == 2) {
                                const uint2 v = *(const uint2 *)(bufs + buf * SBUF + r * RB);
                                o[0] = v.x; o[1] = v.y;
                            } else {
                                const uint4 v = *(const uint4 *)(bufs + buf * SBUF + r * RB);
                                o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
                            }
#pragma unroll
                            for (int w = 0; w < NW; ++w) bits |= __builtin_amdgcn_udot4(o[w], 0x08040201u, 0u, false) << (4 * w);
                        }
                        pay[(j * RB) >> 5] |= bits << ((j * RB) & 31);
                    }
                    const unsigned long long tg = (unsigned long long)cyc << 32;
#pragma unroll
                    for (int k = 0; k < Gm::XW; ++k)
                        __hip_atomic_store(out + lane + 64 * k, tg | pay[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (lane == 0)
                        __hip_atomic_store(out + NXW, tg | (uint32_t)E, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
                    uint32_t got[Gm::XW + 1];   // this lane's words, and the energy (lane 0)
                    uint32_t polls = 0;
                    bool ok_all = false;
                    unsigned long long bad = 0;
                    for (;;) {
                        bool ok = true;
#pragma unroll
                        for (int k = 0; k <= Gm::XW; ++k) {
                            if (k == Gm::XW && lane != 0) continue;
                            const unsigned long long v = __hip_atomic_load(in + (k == Gm::XW ? NXW : lane + 64 * k),
                                                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            if ((uint32_t)(v >> 32) == cyc) got[k] = (uint32_t)v;
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
                        const int pE = __builtin_amdgcn_readfirstlane((int)got[Gm::XW]);
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
                            // bits back to down-bytes: a nibble times 1 + 2^7 + 2^14 + 2^21
                            // puts bit i at bit 8 i (the copies do not overlap)
#pragma unroll
                            for (int j = 0; j < RPL; ++j) {
                                const int r = lane + 64 * j;
                                if (NR % 64 != 0 && r >= NR) continue;
                                const uint32_t bits = got[(j * RB) >> 5] >> ((j * RB) & 31);
                                uint32_t o[NW];
#pragma unroll
                                for (int w = 0; w < NW; ++w)
                                    o[w] = (((bits >> (4 * w)) & 15u) * 0x00204081u) & 0x01010101u;
                                if constexpr (NW == 2) *(uint2 *)(bufs + buf * SBUF + r * RB) = make_uint2(o[0], o[1]);
                                else *(uint4 *)(bufs + buf * SBUF + r * RB) = make_uint4(o[0], o[1], o[2], o[3]);
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
#pragma unroll
                for (int j = 0; j < RPL; ++j) {
                    const int r = lane + 64 * j;
                    if (NR % 64 != 0 && r >= NR) continue;
                    int8_t *dst = it.best_spins + (size_t)wv * N + (size_t)L * r;
#pragma unroll
                    for (int x = 0; x < L; ++x) dst[x] = bufs[buf * SBUF + r * RB + x] ? (int8_t)-1 : (int8_t)1;
                }
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
    for (int x = tid; x < G * N; x += bs) {
        const int l = x / N, i = x - l * N;
        const int r = i / L, xx = i - r * L;
        I.spins[(size_t)(s0 + l) * N + i] = bufs[slot_buf[l] * SBUF + r * RB + xx] ? (int8_t)-1 : (int8_t)1;
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
        for (int i = tid; i < N; i += bs) it.best_spins[i] = it.best_spins[(size_t)win * N + i];
}

#define TAPT_PML_LIST(X) X(6) X(8) X(10) X(12) X(14) X(16)

// One launch for +-J lattices of one or several sizes: each workgroup runs
// the body of its instance's L (the work item's variant).
__global__ void __launch_bounds__(64 * pml::MAXG) pml_kernel(ChunkArgs a)
{
    const int item = a.order[blockIdx.x];
    if (item < 0) return;
    switch (a.items[item].variant) {
#define X(LL)                             \
    case LL: pml_body<LL>(a, item); break;
        TAPT_PML_LIST(X)
#undef X
    default: break;
    }
}

// ---------------------------------------------------------------------------
// Host-side launchers (C++ linkage, used by the runtime in host.cpp).

bool pml_supported(int L) { return L % 2 == 0 && L >= 6 && L <= 16; }

int pml_max_storages() { return pml::MAXG; }

size_t pml_lds_bytes(int L, int G, int tsw_entries)
{
    switch (L) {
#define X(LL)     \
    case LL: return pml::offsets<LL>(G, tsw_entries).total;
        TAPT_PML_LIST(X)
#undef X
    default: return 0;
    }
}

// 64-bit exchange words of one state (bits and energy)
// 64-bit exchange words of one state: XW per lane and the energy
int pml_xwords(int L)
{
    const int rpl = (L * L + 63) / 64, rb = L <= 8 ? 8 : 16;
    return 64 * ((rpl * rb + 31) / 32) + 1;
}

hipError_t launch_pml(const ChunkArgs &a, int block, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL(pml_kernel, dim3(a.n_items), dim3(block), lds, s, a);
    return hipGetLastError();
}

hipError_t pml_occupancy(int block, size_t lds, int *blocks_per_cu)
{
    hipError_t e = hipFuncSetAttribute((const void *)pml_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, pml_kernel, block, lds);
}

} // namespace tapt
