// Device code shared by the persistent-kernel translation units of libtapt:
// Philox4x32-10, the sweepers, the LDS carve-up and the body of the
// persistent chunk kernel (one workgroup, K sweeps and their cycle ends).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tapt_dev.h"

namespace tapt {

typedef short short2v __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11). The 32x32->64 products
// compile to v_mad_u64_u32; the key schedule is wave-uniform (SGPRs).
struct P4 {
    uint32_t v[4];
};

__host__ __device__ __forceinline__ P4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t a = (uint64_t)c0 * 0xD2511F53u;
        uint64_t b = (uint64_t)c2 * 0xCD9E8D57u;
        uint32_t n0 = (uint32_t)(b >> 32) ^ c1 ^ k0;
        uint32_t n2 = (uint32_t)(a >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)b;
        c3 = (uint32_t)a;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    P4 o;
    o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
    return o;
}

__host__ __device__ __forceinline__ uint32_t philox_word0(uint32_t c0, uint32_t c1, uint32_t c3,
                                                          uint32_t k0, uint32_t k1)
{
    return philox(c0, c1, 0, c3, k0, k1).v[0];
}

// An opaque copy of x. A rarely taken branch passes its Philox counter
// through it, so that the compiler cannot hoist the (pure) draw out of the
// branch and pay for it on every pass.
__device__ __forceinline__ uint32_t opaque(uint32_t x)
{
    asm volatile("" : "+v"(x));
    return x;
}

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// a * b + c on the two 16-bit halves of each word (v_pk_mad_u16)
__device__ __forceinline__ uint32_t pk_mad_u16(uint32_t a, uint32_t b, uint32_t c)
{
    const u16x2 r = __builtin_bit_cast(u16x2, a) * __builtin_bit_cast(u16x2, b) + __builtin_bit_cast(u16x2, c);
    return __builtin_bit_cast(uint32_t, r);
}

// Three-input XOR in one instruction (gfx950 v_bitop3_b32, truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// The same generator as philox(), for device code whose counter word 0 varies
// by lane and whose other counter words are wave-uniform: the first two
// rounds keep their uniform XORs on the scalar unit, the remaining eight
// fold each pair of XORs into one v_bitop3.
__device__ __forceinline__ P4 philox_v(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                       uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t a = (uint64_t)c0 * 0xD2511F53u;
        uint64_t b = (uint64_t)c2 * 0xCD9E8D57u;
        uint32_t n0, n2;
        if (r < 2) {
            n0 = (uint32_t)(b >> 32) ^ c1 ^ k0;
            n2 = (uint32_t)(a >> 32) ^ c3 ^ k1;
        } else {
            n0 = xor3((uint32_t)(b >> 32), c1, k0);
            n2 = xor3((uint32_t)(a >> 32), c3, k1);
        }
        c1 = (uint32_t)b;
        c3 = (uint32_t)a;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    P4 o;
    o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
    return o;
}

// Packed unsigned 16-bit operations on two lanes of a dword.
__device__ __forceinline__ uint32_t pk_sub_sat_u16(uint32_t a, uint32_t b)   // max(a - b, 0) per half
{
    uint32_t r;
    asm("v_pk_sub_u16 %0, %1, %2 clamp" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ uint32_t pk_min_u16(uint32_t a, uint32_t b)
{
    uint32_t r;
    asm("v_pk_min_u16 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// accept iff T == ALWAYS or u < T, with u = (hi << 16) | lo and the low half
// drawn only when the high half leaves the decision open.
__device__ __forceinline__ bool coarse_accept(uint32_t T, uint32_t hs, bool &maybe)
{
    bool acc = (hs | 0xFFFFu) < T;
    maybe = !acc && hs < T;
    return acc;
}

__device__ __forceinline__ bool any_lane(bool p) { return __any(p); }

// Minimum of x over the 64 lanes of a wavefront with DPP row shifts and row
// broadcasts (no LDS round trips); every lane receives the result.
__device__ __forceinline__ int wave_min(int x)
{
    const int id = 0x7FFFFFFF;
    x = min(x, __builtin_amdgcn_update_dpp(id, x, 0x111, 0xf, 0xf, false));   // row_shr:1
    x = min(x, __builtin_amdgcn_update_dpp(id, x, 0x112, 0xf, 0xf, false));   // row_shr:2
    x = min(x, __builtin_amdgcn_update_dpp(id, x, 0x114, 0xf, 0xf, false));   // row_shr:4
    x = min(x, __builtin_amdgcn_update_dpp(id, x, 0x118, 0xf, 0xf, false));   // row_shr:8
    x = min(x, __builtin_amdgcn_update_dpp(id, x, 0x142, 0xa, 0xf, false));   // row_bcast:15
    x = min(x, __builtin_amdgcn_update_dpp(id, x, 0x143, 0xc, 0xf, false));   // row_bcast:31
    return __builtin_amdgcn_readlane(x, 63);
}

// x of the next (lane + 1) and the previous (lane - 1) lane by DPP wave
// shifts; the last and the first lane keep their own value.
__device__ __forceinline__ int from_next_lane(int x) { return __builtin_amdgcn_update_dpp(x, x, 0x130, 0xf, 0xf, false); }
__device__ __forceinline__ int from_prev_lane(int x) { return __builtin_amdgcn_update_dpp(x, x, 0x138, 0xf, 0xf, false); }

// Sum of x over the 64 lanes of a wavefront (same DPP pattern as wave_min).
__device__ __forceinline__ int wave_sum(int x)
{
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);   // row_bcast:15
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);   // row_bcast:31
    return __builtin_amdgcn_readlane(x, 63);
}

// ---------------------------------------------------------------------------
// Sweepers. Each provides: storage size and LDS index of a site, per-thread
// setup, and one sweep of every storage of the workgroup (all threads call it;
// it contains the workgroup barriers between color classes).

// Periodic L^3 cubic lattice, checkerboard colors (x+y+z) mod 2, even L.
// Thread (group g, call q) owns sites 8q..8q+7 -- the 8 sites whose uniforms
// come from Philox call q -- of RPT storages. Every such call holds exactly 4
// sites of each color (a row has even length and calls start at even x), so a
// thread updates 4 sites per color phase. Neighbour LDS addresses and packed
// couplings of those 8 sites are computed once and stay in VGPRs.
// LDS layout of a storage: site i at byte (i & 7) * (N/8) + (i >> 3), so
// lanes (consecutive q) touch consecutive bytes for every neighbour direction.
template <int L, int RPT>
struct LatSweep {
    static constexpr int N = L * L * L;
    static constexpr int NC = N / 8;
    static_assert(L % 2 == 0 && L >= 4, "even L >= 4");
    static constexpr int SB = N;   // bytes per storage
    static constexpr int MAXT = 512;  // block limit: leaves up to 256 VGPRs per lane
    static constexpr int MINW = 1;    // waves per SIMD the register budget must allow
    static constexpr bool RND = false;  // no staged random halves

    __host__ __device__ static constexpr int lidx(int i) { return (i & 7) * NC + (i >> 3); }
    static int threads(int G) { return ((G + RPT - 1) / RPT) * NC; }

    int q, grp;
    bool active;
    int own[2][4];
    int nb[2][4][6];
    short2v J[2][4][3];
    int sh[2][4];

    __device__ static int site(int x, int y, int z)
    {
        x = (x + L) % L; y = (y + L) % L; z = (z + L) % L;
        return x + L * (y + L * z);
    }

    __device__ __forceinline__ void setup(const InstDev &I, int G)
    {
        int tid = threadIdx.x;
        grp = tid / NC;
        q = tid % NC;
        active = grp < (G + RPT - 1) / RPT;
        const int8_t *J3 = I.J3;
        for (int c = 0; c < 2; ++c) {
            for (int s = 0; s < 4; ++s) {
                int i0 = 8 * q + 2 * s;
                int x = i0 % L, y = (i0 / L) % L, z = i0 / (L * L);
                int p = (((x + y + z) & 1) == c) ? 0 : 1;
                int i = i0 + p;
                x = i % L;
                int nbs[6] = {site(x + 1, y, z), site(x - 1, y, z), site(x, y + 1, z),
                              site(x, y - 1, z), site(x, y, z + 1), site(x, y, z - 1)};
                int jj[6] = {J3[i], J3[nbs[1]], J3[N + i], J3[N + nbs[3]], J3[2 * N + i], J3[2 * N + nbs[5]]};
                own[c][s] = lidx(i) + grp * RPT * SB;
                for (int d = 0; d < 6; ++d) nb[c][s][d] = lidx(nbs[d]) + grp * RPT * SB;
                for (int d = 0; d < 3; ++d) {
                    short2v v;
                    v.x = (short)jj[2 * d];
                    v.y = (short)jj[2 * d + 1];
                    J[c][s][d] = v;
                }
                sh[c][s] = 16 * p;
            }
        }
    }

    // One sweep at sweep index t of every storage this workgroup holds.
    // slot_of: storage -> local slot; global slot = s0 + local slot.
    __device__ __forceinline__ void sweep(const InstDev &I, int G, int s0, uint32_t t, const int *slot_of,
                                          int8_t *sp, const uint32_t *tab, int stride, int *Elds,
                                          unsigned *flips_lds)
    {
        uint32_t w[RPT][4];
        int sl[RPT], dE[RPT], nf[RPT];
        bool ok[RPT];
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            int stor = grp * RPT + k;
            ok[k] = active && stor < G;
            sl[k] = ok[k] ? slot_of[stor] : 0;
            P4 r = philox_v((uint32_t)q, t, (uint32_t)(s0 + sl[k]), TAG_SWEEP, I.seed_lo, I.seed_hi);
#pragma unroll
            for (int j = 0; j < 4; ++j) w[k][j] = r.v[j];
            dE[k] = 0;
            nf[k] = 0;
        }
        const int D = I.D;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
#pragma unroll
            for (int k = 0; k < RPT; ++k) {
                if (ok[k]) {
                    // the 4 same-color sites are independent: decide all, then flip
                    const uint32_t *trow = tab + sl[k] * stride + D;
                    int mm[4], dd[4];
                    uint32_t TT[4], hs[4];
                    bool acc[4], maybe[4];
                    bool any_maybe = false;
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        int m = sp[own[c][s] + k * SB];
                        short2v m01, m23, m45;
                        m01.x = sp[nb[c][s][0] + k * SB];
                        m01.y = sp[nb[c][s][1] + k * SB];
                        m23.x = sp[nb[c][s][2] + k * SB];
                        m23.y = sp[nb[c][s][3] + k * SB];
                        m45.x = sp[nb[c][s][4] + k * SB];
                        m45.y = sp[nb[c][s][5] + k * SB];
                        int f = __builtin_amdgcn_sdot2(m01, J[c][s][0], 0, false);
                        f = __builtin_amdgcn_sdot2(m23, J[c][s][1], f, false);
                        f = __builtin_amdgcn_sdot2(m45, J[c][s][2], f, false);
                        mm[s] = m;
                        dd[s] = m * f;                      // dE / 2
                        TT[s] = trow[dd[s]];
                        hs[s] = (w[k][s] >> sh[c][s]) << 16;
                        acc[s] = coarse_accept(TT[s], hs[s], maybe[s]);
                        any_maybe |= maybe[s];
                    }
                    if (any_lane(any_maybe)) {
                        P4 r2 = philox(opaque((uint32_t)q), t, (uint32_t)(s0 + sl[k]), TAG_REFINE, I.seed_lo, I.seed_hi);
#pragma unroll
                        for (int s = 0; s < 4; ++s) {
                            uint32_t lo = (r2.v[s] >> sh[c][s]) & 0xFFFFu;
                            if (maybe[s]) acc[s] = (TT[s] == ALWAYS) || ((hs[s] | lo) < TT[s]);
                        }
                    }
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        if (acc[s]) {
                            sp[own[c][s] + k * SB] = (int8_t)(-mm[s]);
                            dE[k] += 2 * dd[s];
                            nf[k] += 1;
                        }
                    }
                }
            }
            if (c == 0) __syncthreads();
        }
        // per-storage energy change and flip count, then the barrier that
        // ends the sweep (Elds is final after it)
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            int e = dE[k], f = nf[k];
            if constexpr (NC % 64 == 0) {
                // a wave belongs to one storage group: DPP sums, no LDS round trips
                e = wave_sum(e);
                f = wave_sum(f);
                if (ok[k] && (threadIdx.x & 63) == 0) {
                    atomicAdd(&Elds[grp * RPT + k], e);
                    atomicAdd(&flips_lds[sl[k]], (unsigned)f);
                }
            } else if constexpr (NC >= 64) {
                // a wave spans at most two storage groups: one DPP sum for each
                const int lane = threadIdx.x & 63;
                const bool first = grp == (int)(threadIdx.x - lane) / NC;
                const int e0 = wave_sum(first ? e : 0), f0 = wave_sum(first ? f : 0);
                const int e1 = wave_sum(first ? 0 : e), f1 = wave_sum(first ? 0 : f);
                if (ok[k] && lane == 0) {
                    atomicAdd(&Elds[grp * RPT + k], e0);
                    atomicAdd(&flips_lds[sl[k]], (unsigned)f0);
                }
                if (ok[k] && lane == 63 && !first) {
                    atomicAdd(&Elds[grp * RPT + k], e1);
                    atomicAdd(&flips_lds[sl[k]], (unsigned)f1);
                }
            } else {
                if (ok[k] && (e != 0 || f != 0)) {
                    atomicAdd(&Elds[grp * RPT + k], e);
                    atomicAdd(&flips_lds[sl[k]], (unsigned)f);
                }
            }
        }
        __syncthreads();
    }
};

// LDS copy of a general graph, staged once per launch: row offsets, packed
// (column << 8 | coupling) words, fields, free sites sorted by colour and the
// colour offsets. Sizes come from the instance, so host and device agree.
struct CsrGraph {
    int *rp;
    uint32_t *cw;
    int16_t *h;
    int16_t *cs;
    int *coff;
};

__host__ __device__ inline size_t csr_graph_bytes(int n, int nnz, int nfree, int ncolors)
{
    size_t o = 0;
    o = (o + (size_t)(n + 1) * 4 + 15) & ~(size_t)15;
    o = (o + (size_t)(nnz > 0 ? nnz : 1) * 4 + 15) & ~(size_t)15;
    o = (o + (size_t)n * 2 + 15) & ~(size_t)15;
    o = (o + (size_t)(nfree > 0 ? nfree : 1) * 2 + 15) & ~(size_t)15;
    o = (o + (size_t)(ncolors + 1) * 4 + 15) & ~(size_t)15;
    return o;
}

__device__ __forceinline__ CsrGraph csr_graph_carve(unsigned char *base, int n, int nnz, int nfree, int ncolors)
{
    CsrGraph g;
    size_t o = 0;
    g.rp = (int *)(base + o); o = (o + (size_t)(n + 1) * 4 + 15) & ~(size_t)15;
    g.cw = (uint32_t *)(base + o); o = (o + (size_t)(nnz > 0 ? nnz : 1) * 4 + 15) & ~(size_t)15;
    g.h = (int16_t *)(base + o); o = (o + (size_t)n * 2 + 15) & ~(size_t)15;
    g.cs = (int16_t *)(base + o); o = (o + (size_t)(nfree > 0 ? nfree : 1) * 2 + 15) & ~(size_t)15;
    g.coff = (int *)(base + o);
    (void)ncolors;
    return g;
}

__device__ __forceinline__ void csr_graph_stage(const InstDev &I, const CsrGraph &g, int tid, int bs)
{
    for (int i = tid; i <= I.n; i += bs) g.rp[i] = I.row_ptr[i];
    for (int e = tid; e < I.nnz; e += bs) g.cw[e] = ((uint32_t)I.col[e] << 8) | ((uint32_t)I.Jc[e] & 0xFFu);
    for (int i = tid; i < I.n; i += bs) g.h[i] = I.h[i];
    for (int k = tid; k < I.nfree; k += bs) g.cs[k] = I.color_sites[k];
    for (int c = tid; c <= I.ncolors; c += bs) g.coff[c] = I.color_off[c];
}

// General sparse graph (CSR, any proper coloring, clamps, fields). Random
// halves for every site of every storage are staged in LDS at the start of
// the sweep (one Philox call per 8 sites), then each color class is spread
// over all threads of the workgroup. WIDE lets a colour class with few
// (site, storage) items share each site's bonds among 2 or 4 lanes; it is
// instantiated for the latency tilings (512 threads, at most 2 slots per
// workgroup), and left out elsewhere, where it would only cost registers.
template <bool WIDE>
struct CsrSweepT {
    static constexpr int RPTV = 1;
    static constexpr int MAXT = 512;    // block limit
    static constexpr int MINW = WIDE ? 3 : 1;   // wide: at most 168 VGPRs, as the plain one needs anyway
    static constexpr bool RND = true;   // random halves staged in LDS
    int n, SB, nr;
    CsrGraph gr;

    __host__ __device__ static int storage_bytes(int n) { return (n + 15) & ~15; }
    __device__ int lidx(int i) const { return i; }
    __device__ static size_t graph_bytes(const InstDev &I) { return csr_graph_bytes(I.n, I.nnz, I.nfree, I.ncolors); }

    __device__ void setup(const InstDev &I, int G)
    {
        (void)G;
        n = I.n;
        SB = storage_bytes(n);
        nr = (n + 7) & ~7;
    }

    // carve and fill the LDS copy of the graph (before the staging barrier)
    __device__ __forceinline__ void bind(const InstDev &I, unsigned char *base, int tid, int bs)
    {
        gr = csr_graph_carve(base, I.n, I.nnz, I.nfree, I.ncolors);
        csr_graph_stage(I, gr, tid, bs);
    }

    __device__ __forceinline__ void sweep(const InstDev &I, int G, int s0, uint32_t t, const int *slot_of,
                                          int8_t *sp, const uint32_t *tab, int stride, int *Elds,
                                          unsigned *flips_lds, uint16_t *rnd)
    {
        const int tid = threadIdx.x, bs = blockDim.x;
        const int ncall = nr >> 3;
        for (int idx = tid; idx < G * ncall; idx += bs) {
            int k = idx / ncall, q = idx - k * ncall;
            P4 r = philox_v((uint32_t)q, t, (uint32_t)(s0 + slot_of[k]), TAG_SWEEP, I.seed_lo, I.seed_hi);
            uint4 v = make_uint4(r.v[0], r.v[1], r.v[2], r.v[3]);
            *(uint4 *)(rnd + (size_t)k * nr + 8 * q) = v;
        }
        __syncthreads();
        const int D = I.D;
        const int ncol = I.ncolors;
        // Work item idx = s * G + k (site s of the colour, storage k): the G
        // lanes of a site read the same graph words (LDS broadcasts). When G
        // divides the block, a thread keeps one storage for the whole sweep
        // and sums its energy change and flips in registers.
        const bool fixed_k = bs % G == 0;
        const int dq = bs / G, dr = bs - dq * G;
        int dE_acc = 0;
        unsigned nf_acc = 0;
        for (int c = 0; c < ncol; ++c) {
            const int off = gr.coff[c], cnt = gr.coff[c + 1] - off;
            // A colour class with few (site, storage) items spreads each site's
            // bonds over 2 or 4 adjacent lanes (a contiguous share each, summed
            // by DPP), which shortens the chain of dependent LDS reads per item.
            const int items = cnt * G;
            const int lp = !WIDE ? 0 : (items * 4 <= bs) ? 2 : (items * 2 <= bs) ? 1 : 0;
            if (lp == 0) {
                int s = tid / G, k = tid - (tid / G) * G;
                while (s < cnt) {
                    const int i = gr.cs[off + s];
                    int8_t *m_k = sp + k * SB;
                    int f = gr.h[i];
                    const int e1 = gr.rp[i + 1];
                    int e = gr.rp[i];
                    // four neighbours per step: their words, then their spins, are
                    // independent loads (two LDS round trips per four bonds)
                    for (; e + 4 <= e1; e += 4) {
                        const uint32_t w0 = gr.cw[e], w1 = gr.cw[e + 1], w2 = gr.cw[e + 2], w3 = gr.cw[e + 3];
                        const int n0 = m_k[w0 >> 8], n1 = m_k[w1 >> 8], n2 = m_k[w2 >> 8], n3 = m_k[w3 >> 8];
                        f += (int)(int8_t)(w0 & 0xFFu) * n0 + (int)(int8_t)(w1 & 0xFFu) * n1 +
                             (int)(int8_t)(w2 & 0xFFu) * n2 + (int)(int8_t)(w3 & 0xFFu) * n3;
                    }
                    for (; e < e1; ++e) {
                        const uint32_t w = gr.cw[e];
                        f += (int)(int8_t)(w & 0xFFu) * (int)m_k[w >> 8];
                    }
                    const int m = m_k[i];
                    const int d = m * f;
                    const int sl = slot_of[k];
                    const uint32_t T = tab[sl * stride + D + d];
                    const uint32_t hs = (uint32_t)rnd[(size_t)k * nr + i] << 16;
                    bool maybe;
                    bool acc = coarse_accept(T, hs, maybe);
                    if (any_lane(maybe)) {
                        if (maybe) {
                            P4 r2 = philox(opaque((uint32_t)(i >> 3)), t, (uint32_t)(s0 + sl), TAG_REFINE, I.seed_lo, I.seed_hi);
                            const int wq = (i & 7) >> 1;   // word of the half (no dynamic indexing)
                            const uint32_t wd = wq == 0 ? r2.v[0] : wq == 1 ? r2.v[1] : wq == 2 ? r2.v[2] : r2.v[3];
                            const uint32_t lo = ((i & 1) ? (wd >> 16) : wd) & 0xFFFFu;
                            acc = (T == ALWAYS) || ((hs | lo) < T);
                        }
                    }
                    if (acc) {
                        m_k[i] = (int8_t)(-m);
                        if (fixed_k) {
                            dE_acc += 2 * d;
                            nf_acc += 1;
                        } else {
                            atomicAdd(&Elds[k], 2 * d);
                            atomicAdd(&flips_lds[sl], 1u);
                        }
                    }
                    s += dq;
                    k += dr;
                    if (k >= G) {
                        k -= G;
                        ++s;
                    }
                }
            } else {
                const int sub = tid & ((1 << lp) - 1), it = tid >> lp;
                if (it < items) {
                    const int s = it / G, k = it - s * G;
                    const int i = gr.cs[off + s];
                    int8_t *m_k = sp + k * SB;
                    const int e0 = gr.rp[i], e1 = gr.rp[i + 1];
                    const int ch = (e1 - e0 + (1 << lp) - 1) >> lp;
                    int e = e0 + sub * ch;
                    const int ee = e + ch < e1 ? e + ch : e1;
                    int f = sub == 0 ? (int)gr.h[i] : 0;
                    for (; e + 4 <= ee; e += 4) {
                        const uint32_t w0 = gr.cw[e], w1 = gr.cw[e + 1], w2 = gr.cw[e + 2], w3 = gr.cw[e + 3];
                        const int n0 = m_k[w0 >> 8], n1 = m_k[w1 >> 8], n2 = m_k[w2 >> 8], n3 = m_k[w3 >> 8];
                        f += (int)(int8_t)(w0 & 0xFFu) * n0 + (int)(int8_t)(w1 & 0xFFu) * n1 +
                             (int)(int8_t)(w2 & 0xFFu) * n2 + (int)(int8_t)(w3 & 0xFFu) * n3;
                    }
                    for (; e < ee; ++e) {
                        const uint32_t w = gr.cw[e];
                        f += (int)(int8_t)(w & 0xFFu) * (int)m_k[w >> 8];
                    }
                    f += __builtin_amdgcn_update_dpp(0, f, 0xB1, 0xf, 0xf, false);       // quad_perm 1,0,3,2
                    if (lp == 2) f += __builtin_amdgcn_update_dpp(0, f, 0x4E, 0xf, 0xf, false);   // 2,3,0,1
                    const int m = m_k[i];
                    const int d = m * f;
                    const int sl = slot_of[k];
                    const uint32_t T = tab[sl * stride + D + d];
                    const uint32_t hs = (uint32_t)rnd[(size_t)k * nr + i] << 16;
                    bool maybe;
                    bool acc = coarse_accept(T, hs, maybe);
                    if (any_lane(maybe)) {
                        if (maybe) {
                            P4 r2 = philox(opaque((uint32_t)(i >> 3)), t, (uint32_t)(s0 + sl), TAG_REFINE, I.seed_lo,
                                           I.seed_hi);
                            const int wq = (i & 7) >> 1;
                            const uint32_t wd = wq == 0 ? r2.v[0] : wq == 1 ? r2.v[1] : wq == 2 ? r2.v[2] : r2.v[3];
                            const uint32_t lo = ((i & 1) ? (wd >> 16) : wd) & 0xFFFFu;
                            acc = (T == ALWAYS) || ((hs | lo) < T);
                        }
                    }
                    if (acc && sub == 0) {   // the lanes of an item agree; one of them writes
                        m_k[i] = (int8_t)(-m);
                        atomicAdd(&Elds[k], 2 * d);
                        atomicAdd(&flips_lds[sl], 1u);
                    }
                }
            }
            __syncthreads();
        }
        if (fixed_k) {
            const int k = tid - (tid / G) * G;
            if (dE_acc) atomicAdd(&Elds[k], dE_acc);
            if (nf_acc) atomicAdd(&flips_lds[slot_of[k]], nf_acc);
            __syncthreads();
        }
    }
};
using CsrSweep = CsrSweepT<false>;
using CsrSweepWide = CsrSweepT<true>;

// ---------------------------------------------------------------------------
// General sparse graph, packed rows ("row" sweeper). The same (site, storage)
// items and storage layout as CsrSweepT, with a fixed item per thread: the
// thread's storage k and rank s never change (item s * G + k of every colour
// class), and the graph is laid out for that map. Record (c, s, sub) holds
// the s-th site of class c and its bonds sub * BPL .. sub * BPL + BPL - 1 as
// 16-bit words (neighbour in bits 0-11, J in bits 12-15), so that a thread
// reads its class-c row with two 16-byte and one 4-byte LDS read at an index
// it computes itself. The rows of class c + 1 are read while class c is
// swept, which leaves two dependent LDS round trips per class on the critical
// path (the neighbour spins with the own spin and random half; then the flip
// threshold), where the CSR layout needs site -> row bounds -> bond words ->
// neighbour spins first. A site's bonds are split over LP = 1 or 2 adjacent
// lanes, summed by DPP; unused bond words are 0 (site 0 with J = 0), so every
// lane reads all BPL neighbours without a branch.
// Requirements (checked by the runtime): n <= CSR_ROW_MAXN, |J| <=
// CSR_ROW_MAXJ, degree <= 2 BPL, and a block of at least (largest class) x G x
// LP threads.
struct RowGraph {
    uint4 *bw;        // [ncolors][maxcnt][LP][2]: 16 bonds of 16 bits
    uint32_t *info;   // [ncolors][maxcnt][LP]: site i | h_i << 16 (h on sub 0); 0xFFF: no site
};

struct CsrRowSweep {
    static constexpr int RPTV = 1;
    static constexpr int MAXT = 512;
    static constexpr int MINW = 1;
    static constexpr bool RND = true;
    static constexpr int BPL = CSR_ROW_BPL;
    int n, SB, nr, G, k, sub, lp, s, maxcnt;
    RowGraph gr;

    __device__ static size_t graph_bytes(const InstDev &I)
    {
        return csr_row_graph_bytes(I.ncolors, I.maxcnt, csr_row_lanes(I.maxdeg));
    }

    __device__ void setup(const InstDev &I, int G_)
    {
        n = I.n;
        SB = CsrSweepT<false>::storage_bytes(n);
        nr = (n + 7) & ~7;
        G = G_;
    }

    __device__ __forceinline__ void bind(const InstDev &I, unsigned char *base, int tid, int bs)
    {
        lp = csr_row_lanes(I.maxdeg);
        maxcnt = I.maxcnt;
        sub = tid & (lp - 1);
        const int it = tid / lp;
        s = it / G;
        k = it - s * G;
        const int nrec = I.ncolors * maxcnt * lp;
        gr.bw = (uint4 *)base;
        gr.info = (uint32_t *)(base + (size_t)nrec * 32);
        for (int x = tid; x < nrec; x += bs) {
            const int c = x / (maxcnt * lp), rest = x - c * maxcnt * lp;
            const int ss = rest / lp, sb = rest - ss * lp;
            const int off = I.color_off[c], cnt = I.color_off[c + 1] - off;
            uint32_t w[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            uint32_t info = 0xFFFu;
            if (ss < cnt) {
                const int i = I.color_sites[off + ss];
                const int r1 = I.row_ptr[i + 1];
                const int e0 = I.row_ptr[i] + sb * BPL;
                for (int b = 0; b < BPL && e0 + b < r1; ++b)
                    w[b >> 1] |= ((uint32_t)I.col[e0 + b] | (((uint32_t)I.Jc[e0 + b] & 15u) << 12)) << (16 * (b & 1));
                info = (uint32_t)i | ((sb == 0 ? (uint32_t)(uint16_t)I.h[i] : 0u) << 16);
            }
            gr.bw[2 * x] = make_uint4(w[0], w[1], w[2], w[3]);
            gr.bw[2 * x + 1] = make_uint4(w[4], w[5], w[6], w[7]);
            gr.info[x] = info;
        }
    }

    __device__ __forceinline__ void sweep(const InstDev &I, int G_, int s0, uint32_t t, const int *slot_of,
                                          int8_t *sp, const uint32_t *tab, int stride, int *Elds,
                                          unsigned *flips_lds, uint16_t *rnd)
    {
        (void)G_;
        const int tid = threadIdx.x, bs = blockDim.x;
        const int ncol = I.ncolors;
        const bool on = s < maxcnt;             // threads past the last item only keep the barriers
        const int xs = on ? s * lp + sub : 0;   // record of this thread in class 0
        const int xstep = maxcnt * lp;          // records per class
        // class 0's row, read while the random halves are drawn
        uint4 w0 = gr.bw[2 * xs], w1 = gr.bw[2 * xs + 1];
        uint32_t info = on ? gr.info[xs] : 0xFFFu;
        const int ncall = nr >> 3;
        for (int idx = tid; idx < G * ncall; idx += bs) {
            const int kk = idx / ncall, q = idx - kk * ncall;
            const P4 r = philox_v((uint32_t)q, t, (uint32_t)(s0 + slot_of[kk]), TAG_SWEEP, I.seed_lo, I.seed_hi);
            *(uint4 *)(rnd + (size_t)kk * nr + 8 * q) = make_uint4(r.v[0], r.v[1], r.v[2], r.v[3]);
        }
        __syncthreads();
        const int sl = slot_of[k];
        const int tb = sl * stride + I.D;
        int8_t *m_k = sp + k * SB;
        const uint16_t *r_k = rnd + (size_t)k * nr;
        int dE_acc = 0;
        unsigned nf_acc = 0;
        for (int c = 0; c < ncol; ++c) {
            const int i = (int)(info & 0xFFFu);
            const bool valid = i != 0xFFF;
            int f = 0, m = 0;
            uint32_t hs = 0;
            if (valid) {
                // the item's reads are independent: one LDS round trip
                m = m_k[i];
                hs = (uint32_t)r_k[i] << 16;
                f = (int)info >> 16;
                const uint32_t ws[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const uint32_t wq = ws[q];
                    f += ((int)(wq << 16) >> 28) * (int)m_k[wq & 0xFFFu] + ((int)wq >> 28) * (int)m_k[(wq >> 16) & 0xFFFu];
                }
            }
            // the next class's row, in flight while this class is decided
            if (c + 1 < ncol) {
                const int xn = xs + (c + 1) * xstep;
                w0 = gr.bw[2 * xn];
                w1 = gr.bw[2 * xn + 1];
                info = on ? gr.info[xn] : 0xFFFu;
            }
            if (lp == 2) f += __builtin_amdgcn_update_dpp(0, f, 0xB1, 0xf, 0xf, false);   // quad_perm 1,0,3,2
            if (valid) {
                const int d = m * f;
                const uint32_t T = tab[tb + d];
                bool maybe;
                bool acc = coarse_accept(T, hs, maybe);
                if (any_lane(maybe)) {
                    if (maybe) {
                        P4 r2 = philox(opaque((uint32_t)(i >> 3)), t, (uint32_t)(s0 + sl), TAG_REFINE, I.seed_lo, I.seed_hi);
                        const int wq = (i & 7) >> 1;
                        const uint32_t wd = wq == 0 ? r2.v[0] : wq == 1 ? r2.v[1] : wq == 2 ? r2.v[2] : r2.v[3];
                        const uint32_t lo = ((i & 1) ? (wd >> 16) : wd) & 0xFFFFu;
                        acc = (T == ALWAYS) || ((hs | lo) < T);
                    }
                }
                if (acc && sub == 0) {   // the lanes of an item agree; the first one writes
                    m_k[i] = (int8_t)(-m);
                    dE_acc += 2 * d;
                    nf_acc += 1;
                }
            }
            __syncthreads();
        }
        if (dE_acc) atomicAdd(&Elds[k], dE_acc);
        if (nf_acc) atomicAdd(&flips_lds[sl], nf_acc);
        __syncthreads();
    }
};

// ---------------------------------------------------------------------------
// General sparse graph, packed rows and four storages per lane ("row-quad"
// sweeper). The storages are interleaved as in CsrQuadSweep (byte k of site
// i's GS-byte group is storage k's down-bit), so one dword read gives a
// neighbour's spins in four storages and a lane decides one site of four
// storages at once (U summed byte-parallel, d = D_i - 2 U per storage). The
// rows are packed as in CsrRowSweep, for a fixed (site rank s, quad) item per
// thread: record (c, s, sub) holds the s-th site of class c and 16 of its
// bonds as words (neighbour byte offset j * GS in bits 0-15, 1 in byte 2 if
// J < 0, |J| in byte 3), read with four 16-byte LDS reads and prefetched one
// class ahead. A bond costs an add, a dword read, a byte permute, a shift and
// a multiply, a three-input XOR and a packed multiply-add; unused bond words are 0 (the
// dword at offset 0 with |J| = 0). Requirements (checked by the runtime):
// every D_i <= 255, (n - 1) * GS + 3 < 65536, degree <= 32 (LP = 1 or 2
// lanes per item, U partial sums added after DPP: no byte exceeds D_i), and a
// block of at least (largest class) x GS / 4 x LP threads.
struct RowQuadGraph {
    uint4 *bw;        // [ncolors][maxcnt][LP][4]: 16 bond words
    uint32_t *info;   // [ncolors][maxcnt][LP]: i | D_i << 12 | |h_i| << 20 | [h_i < 0] << 28 (h on sub 0); 0xFFF: none
};

struct CsrRowQuadSweep {
    static constexpr int RPTV = 1;
    static constexpr int MAXT = 512;
    static constexpr int MINW = 1;
    static constexpr bool RND = true;
    static constexpr int BPL = CSR_ROW4_BPL;
    int n, G, GS, nr, qd, sub, lp, s, maxcnt;
    RowQuadGraph gr;

    __host__ __device__ static int group_bytes(int G) { return (G + 3) & ~3; }
    __device__ static size_t graph_bytes(const InstDev &I)
    {
        return csr_row4_graph_bytes(I.ncolors, I.maxcnt, csr_row4_lanes(I.maxdeg));
    }

    __device__ void setup(const InstDev &I, int G_)
    {
        n = I.n;
        G = G_;
        GS = group_bytes(G_);
        nr = (n + 7) & ~7;
    }

    __device__ __forceinline__ void bind(const InstDev &I, unsigned char *base, int tid, int bs)
    {
        lp = csr_row4_lanes(I.maxdeg);
        maxcnt = I.maxcnt;
        const int nq = GS >> 2;
        sub = tid & (lp - 1);
        const int it = tid / lp;
        s = it / nq;
        qd = it - s * nq;
        const int nrec = I.ncolors * maxcnt * lp;
        gr.bw = (uint4 *)base;
        gr.info = (uint32_t *)(base + (size_t)nrec * 64);
        for (int x = tid; x < nrec; x += bs) {
            const int c = x / (maxcnt * lp), rest = x - c * maxcnt * lp;
            const int ss = rest / lp, sb = rest - ss * lp;
            const int off = I.color_off[c], cnt = I.color_off[c + 1] - off;
            uint32_t w[16];
#pragma unroll
            for (int b = 0; b < 16; ++b) w[b] = 0;
            uint32_t info = 0xFFFu;
            if (ss < cnt) {
                const int i = I.color_sites[off + ss];
                const int r0 = I.row_ptr[i], r1 = I.row_ptr[i + 1];
                int D = 0;
                for (int e = r0; e < r1; ++e) D += abs((int)I.Jc[e]);
                const int h = sb == 0 ? (int)I.h[i] : 0;
                D += abs((int)I.h[i]);
                const int e0 = r0 + sb * BPL;
#pragma unroll
                for (int b = 0; b < 16; ++b) {
                    if (e0 + b < r1) {
                        const int J = I.Jc[e0 + b];
                        w[b] = (uint32_t)I.col[e0 + b] * (uint32_t)GS | (J < 0 ? 0x10000u : 0u) |
                               ((uint32_t)abs(J) << 24);
                    }
                }
                info = (uint32_t)i | ((uint32_t)D << 12) | ((uint32_t)abs(h) << 20) | (h < 0 ? 1u << 28 : 0u);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) gr.bw[4 * x + q] = make_uint4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
            gr.info[x] = info;
        }
    }

    __device__ __forceinline__ void sweep(const InstDev &I, int G_, int s0, uint32_t t, const int *slot_of,
                                          int8_t *sp, const uint32_t *tab, int stride, int *Elds,
                                          unsigned *flips_lds, uint16_t *rnd)
    {
        (void)G_;
        const int tid = threadIdx.x, bs = blockDim.x;
        const int ncol = I.ncolors;
        const bool on = s < maxcnt;             // threads past the last item only keep the barriers
        const int xs = on ? s * lp + sub : 0;   // record of this thread in class 0
        const int xstep = maxcnt * lp;          // records per class
        uint4 w0 = gr.bw[4 * xs], w1 = gr.bw[4 * xs + 1], w2 = gr.bw[4 * xs + 2], w3 = gr.bw[4 * xs + 3];
        uint32_t info = on ? gr.info[xs] : 0xFFFu;
        // random halves of every (site, storage), interleaved like the spins
        const int ncall = nr >> 3;
        for (int idx = tid; idx < G * ncall; idx += bs) {
            const int k = idx / ncall, q = idx - k * ncall;
            const P4 r = philox_v((uint32_t)q, t, (uint32_t)(s0 + slot_of[k]), TAG_SWEEP, I.seed_lo, I.seed_hi);
            uint16_t *dst = rnd + (size_t)(8 * q) * GS + k;
#pragma unroll
            for (int j = 0; j < 8; ++j) dst[j * GS] = (uint16_t)(r.v[j >> 1] >> (16 * (j & 1)));
        }
        __syncthreads();
        const int D = I.D;
        const int qo = 4 * qd;                  // byte offset of this lane's quad in a site group
        int tb[4];
        uint32_t vm = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int st = qo + k;
            const bool ok = st < G;
            tb[k] = ok ? slot_of[st] * stride + D : D;
            vm |= ok ? (1u << (8 * k)) : 0u;
        }
        int e_acc[4] = {0, 0, 0, 0};
        unsigned f_acc[4] = {0, 0, 0, 0};
        for (int c = 0; c < ncol; ++c) {
            const int i = (int)(info & 0xFFFu);
            const bool valid = i != 0xFFF;
            uint32_t U = 0, own = 0;
            uint2 hh = make_uint2(0, 0);
            const uint32_t a_own = (uint32_t)i * (uint32_t)GS + (uint32_t)qo;
            if (valid) {
                // the item's reads are independent: one LDS round trip
                own = *(const uint32_t *)(sp + a_own);
                hh = *(const uint2 *)(rnd + a_own);
                U = pk_mad_u16(own ^ ((info >> 28) * 0x01010101u), ((info >> 20) & 0xFFu) * 0x10001u, 0u);
                const uint32_t ws[16] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w,
                                         w2.x, w2.y, w2.z, w2.w, w3.x, w3.y, w3.z, w3.w};
#pragma unroll
                for (int b = 0; b < 16; ++b) {
                    const uint32_t w = ws[b];
                    const uint32_t nb = *(const uint32_t *)(sp + (w & 0xFFFFu) + (uint32_t)qo);
                    // sign byte to all four bytes; |J| to both 16-bit halves
                    const uint32_t sg = __builtin_amdgcn_perm(w, w, 0x02020202u);
                    const uint32_t aj = (w >> 24) * 0x10001u;
                    U = pk_mad_u16(xor3(own, nb, sg), aj, U);
                }
            }
            const uint32_t info_c = info;
            // the next class's row, in flight while this class is decided
            if (c + 1 < ncol) {
                const int xn = xs + (c + 1) * xstep;
                w0 = gr.bw[4 * xn];
                w1 = gr.bw[4 * xn + 1];
                w2 = gr.bw[4 * xn + 2];
                w3 = gr.bw[4 * xn + 3];
                info = on ? gr.info[xn] : 0xFFFu;
            }
            if (lp == 2) U += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)U, 0xB1, 0xf, 0xf, false);   // quad_perm 1,0,3,2
            if (valid) {
                const int Dsite = (int)((info_c >> 12) & 0xFFu);
                uint32_t T[4], hs[4];
                int d[4];
                bool acc[4], maybe[4];
                bool any_maybe = false;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    d[k] = Dsite - 2 * (int)((U >> (8 * k)) & 0xFFu);   // m_i I_i of storage qo + k
                    T[k] = tab[tb[k] + d[k]];
                    const uint32_t wv = k < 2 ? hh.x : hh.y;
                    hs[k] = (k & 1) ? (wv & 0xFFFF0000u) : (wv << 16);
                    acc[k] = coarse_accept(T[k], hs[k], maybe[k]) && ((vm >> (8 * k)) & 1u);
                    maybe[k] = maybe[k] && ((vm >> (8 * k)) & 1u);
                    any_maybe |= maybe[k];
                }
                if (any_lane(any_maybe)) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        if (maybe[k]) {
                            const P4 r2 = philox(opaque((uint32_t)(i >> 3)), t, (uint32_t)(s0 + slot_of[qo + k]), TAG_REFINE,
                                                 I.seed_lo, I.seed_hi);
                            const int wq = (i & 7) >> 1;
                            const uint32_t wd = wq == 0 ? r2.v[0] : wq == 1 ? r2.v[1] : wq == 2 ? r2.v[2] : r2.v[3];
                            const uint32_t lo = ((i & 1) ? (wd >> 16) : wd) & 0xFFFFu;
                            acc[k] = (T[k] == ALWAYS) || ((hs[k] | lo) < T[k]);
                        }
                    }
                }
                if (sub == 0) {   // the lanes of an item agree; the first one writes
                    uint32_t F = 0;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        F |= acc[k] ? (1u << (8 * k)) : 0u;
                        e_acc[k] += acc[k] ? 2 * d[k] : 0;       // the flip changes E by 2 d
                        f_acc[k] += acc[k] ? 1u : 0u;
                    }
                    if (F) *(uint32_t *)(sp + a_own) = own ^ F;
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int st = qo + k;
            if (on && st < G && (e_acc[k] != 0 || f_acc[k] != 0)) {
                atomicAdd(&Elds[st], e_acc[k]);
                atomicAdd(&flips_lds[slot_of[st]], f_acc[k]);
            }
        }
        __syncthreads();
    }
};

// ---------------------------------------------------------------------------
// General sparse graph, four storages per lane ("quad" sweeper). The storages
// of a workgroup are interleaved: byte k of site i's GS-byte group (GS = G
// rounded up to a multiple of 4) holds storage k's spin as a down-bit (1 for
// -1). One dword read gives a site's spins in four storages, so a lane
// updates one site of four storages at once:
//   with u = b_i ^ b_j ^ [J_ij < 0] (1 when the bond is unsatisfied, per
//   byte) and u_h = b_i ^ [h_i < 0], the four energy changes of flipping
//   site i are 2 d, d = m_i I_i = D_i - 2 U, with D_i = sum_j |J_ij| + |h_i|
//   and U = sum_j |J_ij| u_ij + |h_i| u_h (Methods, Eq. 4),
// and U is summed byte-parallel by 24-bit multiply-adds (no byte carries
// while D_i <= 255). The bond records hold the neighbour's byte offset, the
// sign mask and |J|, so a bond costs an add, a three-input XOR and a
// multiply-add. Each storage's decision then reads its own slot's flip
// table. Used for throughput tilings of general graphs (G >= 4, n <= 4096,
// every site bound D_i <= 255); random halves are staged per sweep as in
// CsrSweepT, interleaved like the storages.
struct QuadGraph {
    uint4 *site;     // [n]: x, y bond range; z = D_i | |h_i| << 16; w = 0x01010101 if h_i < 0
    uint4 *bond;     // [nnz]: x = j * GS, y = 0x01010101 if J < 0, z = |J| in both 16-bit halves
    int16_t *cs;     // free sites sorted by colour [nfree]
    int *coff;       // [ncolors + 1]
};

__host__ __device__ inline size_t quad_graph_bytes(int n, int nnz, int nfree, int ncolors)
{
    size_t o = 0;
    o = (o + (size_t)n * 16 + 15) & ~(size_t)15;
    o = (o + (size_t)(nnz > 0 ? nnz : 1) * 16 + 15) & ~(size_t)15;
    o = (o + (size_t)(nfree > 0 ? nfree : 1) * 2 + 15) & ~(size_t)15;
    o = (o + (size_t)(ncolors + 1) * 4 + 15) & ~(size_t)15;
    return o;
}

struct CsrQuadSweep {
    static constexpr int RPTV = 1;
    static constexpr int MAXT = 256;
    static constexpr int MINW = 4;      // at most 128 VGPRs: four waves per SIMD
    static constexpr bool RND = true;
    int n, G, GS, nr;
    QuadGraph gr;

    __host__ __device__ static int group_bytes(int G) { return (G + 3) & ~3; }
    __device__ static size_t graph_bytes(const InstDev &I) { return quad_graph_bytes(I.n, I.nnz, I.nfree, I.ncolors); }

    __device__ void setup(const InstDev &I, int G_)
    {
        n = I.n;
        G = G_;
        GS = group_bytes(G_);
        nr = (n + 7) & ~7;
    }

    __device__ __forceinline__ void bind(const InstDev &I, unsigned char *base, int tid, int bs)
    {
        size_t o = 0;
        gr.site = (uint4 *)(base + o); o = (o + (size_t)n * 16 + 15) & ~(size_t)15;
        gr.bond = (uint4 *)(base + o); o = (o + (size_t)(I.nnz > 0 ? I.nnz : 1) * 16 + 15) & ~(size_t)15;
        gr.cs = (int16_t *)(base + o); o = (o + (size_t)(I.nfree > 0 ? I.nfree : 1) * 2 + 15) & ~(size_t)15;
        gr.coff = (int *)(base + o);
        for (int i = tid; i < n; i += bs) {
            const int e0 = I.row_ptr[i], e1 = I.row_ptr[i + 1];
            int D = 0;
            for (int e = e0; e < e1; ++e) D += abs((int)I.Jc[e]);
            const int h = I.h[i];
            D += abs(h);
            gr.site[i] = make_uint4((uint32_t)e0, (uint32_t)e1, (uint32_t)D | ((uint32_t)abs(h) << 16),
                                    h < 0 ? 0x01010101u : 0u);
        }
        for (int e = tid; e < I.nnz; e += bs) {
            const int J = I.Jc[e];
            gr.bond[e] = make_uint4((uint32_t)I.col[e] * (uint32_t)GS, J < 0 ? 0x01010101u : 0u,
                                    (uint32_t)abs(J) * 0x10001u, 0u);
        }
        for (int k = tid; k < I.nfree; k += bs) gr.cs[k] = I.color_sites[k];
        for (int c = tid; c <= I.ncolors; c += bs) gr.coff[c] = I.color_off[c];
    }

    __device__ __forceinline__ void sweep(const InstDev &I, int G_, int s0, uint32_t t, const int *slot_of,
                                          int8_t *sp, const uint32_t *tab, int stride, int *Elds,
                                          unsigned *flips_lds, uint16_t *rnd)
    {
        (void)G_;
        const int tid = threadIdx.x, bs = blockDim.x;
        const int ncall = nr >> 3;
        // random halves of every (site, storage), interleaved like the spins
        for (int idx = tid; idx < G * ncall; idx += bs) {
            const int k = idx / ncall, q = idx - k * ncall;
            const P4 r = philox_v((uint32_t)q, t, (uint32_t)(s0 + slot_of[k]), TAG_SWEEP, I.seed_lo, I.seed_hi);
            uint16_t *dst = rnd + (size_t)(8 * q) * GS + k;
#pragma unroll
            for (int s = 0; s < 8; ++s) dst[s * GS] = (uint16_t)(r.v[s >> 1] >> (16 * (s & 1)));
        }
        __syncthreads();
        const int D = I.D;
        const int nq = GS >> 2;                 // storage quads
        const int qd = tid % nq, j0 = tid / nq, dj = bs / nq;
        const bool lane_on = j0 < dj;           // threads past the last whole quad row idle
        const int qo = 4 * qd;                  // byte offset of this lane's quad in a site group
        int tb[4];
        uint32_t vm = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int st = qo + k;
            const bool ok = st < G;
            tb[k] = ok ? slot_of[st] * stride + D : D;
            vm |= ok ? (1u << (8 * k)) : 0u;
        }
        int e_acc[4] = {0, 0, 0, 0};
        unsigned f_acc[4] = {0, 0, 0, 0};
        const int ncol = I.ncolors;
        for (int c = 0; c < ncol; ++c) {
            const int off = gr.coff[c], cnt = gr.coff[c + 1] - off;
            for (int s = lane_on ? j0 : cnt; s < cnt; s += dj) {
                const int i = gr.cs[off + s];
                const uint4 si = gr.site[i];
                const uint32_t a_own = (uint32_t)i * (uint32_t)GS + (uint32_t)qo;
                uint32_t own = *(const uint32_t *)(sp + a_own);
                uint32_t U = pk_mad_u16(own ^ si.w, (si.z >> 16) * 0x10001u, 0u);
                uint32_t e = si.x;
                // four bonds a step: their records, then their neighbours, are
                // independent reads (two LDS round trips per four bonds)
                for (; e + 4 <= si.y; e += 4) {
                    const uint4 b0 = gr.bond[e], b1 = gr.bond[e + 1], b2 = gr.bond[e + 2], b3 = gr.bond[e + 3];
                    const uint32_t n0 = *(const uint32_t *)(sp + b0.x + (uint32_t)qo);
                    const uint32_t n1 = *(const uint32_t *)(sp + b1.x + (uint32_t)qo);
                    const uint32_t n2 = *(const uint32_t *)(sp + b2.x + (uint32_t)qo);
                    const uint32_t n3 = *(const uint32_t *)(sp + b3.x + (uint32_t)qo);
                    U = pk_mad_u16(xor3(own, n0, b0.y), b0.z, U);
                    U = pk_mad_u16(xor3(own, n1, b1.y), b1.z, U);
                    U = pk_mad_u16(xor3(own, n2, b2.y), b2.z, U);
                    U = pk_mad_u16(xor3(own, n3, b3.y), b3.z, U);
                }
                for (; e < si.y; ++e) {
                    const uint4 b = gr.bond[e];
                    const uint32_t nb = *(const uint32_t *)(sp + b.x + (uint32_t)qo);
                    U = pk_mad_u16(xor3(own, nb, b.y), b.z, U);
                }
                const int Dsite = (int)(si.z & 0xFFFFu);
                const uint2 hh = *(const uint2 *)(rnd + a_own);
                uint32_t T[4], hs[4];
                int d[4];
                bool acc[4], maybe[4];
                bool any_maybe = false;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    d[k] = Dsite - 2 * (int)((U >> (8 * k)) & 0xFFu);   // m_i I_i of storage 4 qd + k
                    T[k] = tab[tb[k] + d[k]];
                    const uint32_t w = k < 2 ? hh.x : hh.y;
                    hs[k] = (k & 1) ? (w & 0xFFFF0000u) : (w << 16);
                    acc[k] = coarse_accept(T[k], hs[k], maybe[k]) && ((vm >> (8 * k)) & 1u);
                    maybe[k] = maybe[k] && ((vm >> (8 * k)) & 1u);
                    any_maybe |= maybe[k];
                }
                if (any_lane(any_maybe)) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        if (maybe[k]) {
                            const P4 r2 = philox(opaque((uint32_t)(i >> 3)), t, (uint32_t)(s0 + slot_of[qo + k]), TAG_REFINE,
                                                 I.seed_lo, I.seed_hi);
                            const int wq = (i & 7) >> 1;
                            const uint32_t wd = wq == 0 ? r2.v[0] : wq == 1 ? r2.v[1] : wq == 2 ? r2.v[2] : r2.v[3];
                            const uint32_t lo = ((i & 1) ? (wd >> 16) : wd) & 0xFFFFu;
                            acc[k] = (T[k] == ALWAYS) || ((hs[k] | lo) < T[k]);
                        }
                    }
                }
                uint32_t F = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    F |= acc[k] ? (1u << (8 * k)) : 0u;
                    e_acc[k] += acc[k] ? 2 * d[k] : 0;       // the flip changes E by 2 d
                    f_acc[k] += acc[k] ? 1u : 0u;
                }
                *(uint32_t *)(sp + a_own) = own ^ F;
            }
            __syncthreads();
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int st = qo + k;
            if (lane_on && st < G && (e_acc[k] != 0 || f_acc[k] != 0)) {
                atomicAdd(&Elds[st], e_acc[k]);
                atomicAdd(&flips_lds[slot_of[st]], f_acc[k]);
            }
        }
        __syncthreads();
    }
};

// ---------------------------------------------------------------------------
// LDS carve-up shared by the persistent kernel and the host's size query.
// tsw: swap-threshold rows of the pairs a workgroup decides, pair slot p for
// global pair r = s0 - 1 + p (p = 0 and p = G are the cross-workgroup pairs).
struct ChunkLds {
    int8_t *sp;
    uint32_t *tab;
    int *slot_of, *stor_of, *Elds;
    unsigned *flips, *satt, *sacc;
    int *misc;
    long long *src;
    uint16_t *rnd;
    int *tsw_off;              // [G + 2]: row p spans [tsw_off[p], tsw_off[p+1])
    uint32_t *tsw;
    uint32_t *xstage;          // [2][ceil(n/32) + 1] validated exchange words
    uint32_t *usw;             // [2][65] swap uniforms by cycle parity (lane l: pair s0+l; 64: pair s0-1)
    int8_t *cx;                // contextual proposal: candidate storage [SB]
    uint8_t *cm;               // and its context mask [SB], both in the storage layout
    uint32_t *ckey;            // and the CONTEXT keys of its sites [n], site order
    int *chist;                // radix-select histogram [256]
};

struct ChunkOff {
    size_t sp, tab, ints, src, rnd, toff, tsw, xst, usw, graph, ctx, cmask, ckey, chist, total;
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

__host__ __device__ __forceinline__ ChunkOff chunk_lds_offsets(int G, int SB, int stride, int nr_csr, int tsw_entries,
                                                                int n, size_t graph_bytes = 0, bool contextual = false)
{
    ChunkOff f;
    size_t o = 0;
    f.sp = o; o = align16(o + (size_t)G * SB);
    f.tab = o; o = align16(o + (size_t)G * stride * 4);
    f.ints = o; o = align16(o + (size_t)G * 4 * 7 + 64);
    f.src = o; o = align16(o + (size_t)G * 8);
    f.rnd = o; o = align16(o + (size_t)G * nr_csr * 2);
    f.toff = o; o = align16(o + (size_t)(G + 2) * 4);
    f.tsw = o; o = align16(o + (size_t)tsw_entries * 4);
    f.xst = o; o = align16(o + (size_t)2 * (((n + 31) >> 5) + 1) * 4);
    f.usw = o; o = align16(o + (size_t)2 * 65 * 4);
    f.graph = o; o = align16(o + graph_bytes);
    f.ctx = o; o = align16(o + (contextual ? (size_t)SB : 0));     // contextual candidate
    f.cmask = o; o = align16(o + (contextual ? (size_t)SB : 0));   // and its context mask
    f.ckey = o; o = align16(o + (contextual ? (size_t)n * 4 : 0)); // context keys
    f.chist = o; o = align16(o + (contextual ? (size_t)256 * 4 : 0));
    f.total = o;
    return f;
}

// Pointers into the dynamic LDS block, built from the kernel's own
// __shared__ array so that every access compiles to ds_* instructions.
#define CHUNK_LDS_POINTERS(c, f, G, base)                         \
    ChunkLds c;                                                   \
    c.sp = (int8_t *)((base) + (f).sp);                           \
    c.tab = (uint32_t *)((base) + (f).tab);                       \
    c.slot_of = (int *)((base) + (f).ints);                       \
    c.stor_of = c.slot_of + (G);                                  \
    c.Elds = c.slot_of + 2 * (G);                                 \
    c.flips = (unsigned *)(c.slot_of + 3 * (G));                  \
    c.satt = (unsigned *)(c.slot_of + 4 * (G));                   \
    c.sacc = (unsigned *)(c.slot_of + 5 * (G));                   \
    c.misc = c.slot_of + 7 * (G);                                 \
    c.src = (long long *)((base) + (f).src);                      \
    c.rnd = (uint16_t *)((base) + (f).rnd);                       \
    c.tsw_off = (int *)((base) + (f).toff);                       \
    c.tsw = (uint32_t *)((base) + (f).tsw);                       \
    c.xstage = (uint32_t *)((base) + (f).xst);                    \
    c.usw = (uint32_t *)((base) + (f).usw);                       \
    c.cx = (int8_t *)((base) + (f).ctx);                          \
    c.cm = (uint8_t *)((base) + (f).cmask);                       \
    c.ckey = (uint32_t *)((base) + (f).ckey);                     \
    c.chist = (int *)((base) + (f).chist)

// Run parameters of one instance, read once per launch (kept in SGPRs).
struct RunParams {
    int n, R, M, D, stride, has_target, target;
    uint32_t k0, k1;
    int64_t prop_start, prop_period, prop_stop;
    __device__ __forceinline__ void load(const InstDev &I)
    {
        n = I.n; R = I.R; M = I.M; D = I.D; stride = I.tflip_stride;
        has_target = I.has_target; target = I.target;
        k0 = I.seed_lo; k1 = I.seed_hi;
        prop_start = I.prop_start; prop_period = I.prop_period; prop_stop = I.prop_stop;
    }
    // First proposal sweep at or after t, or ~0 if none is left. The loops
    // step from it by prop_period, so no 64-bit division runs per sweep.
    __device__ __forceinline__ uint64_t first_prop_from(uint64_t t) const
    {
        if (prop_period <= 0) return ~0ull;
        uint64_t k = 0;
        if ((int64_t)t > prop_start) k = ((uint64_t)((int64_t)t - prop_start) + (uint64_t)prop_period - 1) / (uint64_t)prop_period;
        uint64_t at = (uint64_t)prop_start + k * (uint64_t)prop_period;
        if (prop_stop >= 0 && (int64_t)at > prop_stop) return ~0ull;
        return at;
    }
    __device__ __forceinline__ uint64_t next_prop(uint64_t at) const
    {
        uint64_t nx = at + (uint64_t)prop_period;
        if (prop_stop >= 0 && (int64_t)nx > prop_stop) return ~0ull;
        return nx;
    }
    __device__ __forceinline__ bool prop_sweep(uint64_t t) const
    {
        if (prop_period <= 0) return false;
        if ((int64_t)t < prop_start) return false;
        if (prop_stop >= 0 && (int64_t)t > prop_stop) return false;
        return (((int64_t)t - prop_start) % prop_period) == 0;
    }
};

__device__ inline bool is_prop_sweep(const InstDev &I, uint64_t t)
{
    if (I.prop_period <= 0) return false;
    if ((int64_t)t < I.prop_start) return false;
    if (I.prop_stop >= 0 && (int64_t)t > I.prop_stop) return false;
    return (((int64_t)t - I.prop_start) % I.prop_period) == 0;
}

// swap threshold for pair r and dE = E_{r+1} - E_r from an LDS row
__device__ __forceinline__ uint32_t swap_threshold(const ChunkLds &c, int p, int dE)
{
    if (dE >= 0) return ALWAYS;
    int d = -dE, lo = c.tsw_off[p], len = c.tsw_off[p + 1] - lo;
    return d <= len ? c.tsw[lo + d - 1] : 0u;
}

// ---------------------------------------------------------------------------
// Persistent chunk kernel: K sweeps (and the cycle-end stages they reach) of
// the slots [s0, s0+G) of one instance per workgroup.
template <class Sw>
struct SweepCall;

template <int L, int RPT>
struct SweepCall<LatSweep<L, RPT>> {
    static __device__ __forceinline__ void run(LatSweep<L, RPT> &sw, const InstDev &I, int G, int s0, uint32_t t, ChunkLds &c,
                               int stride)
    {
        sw.sweep(I, G, s0, t, c.slot_of, c.sp, c.tab, stride, c.Elds, c.flips);
    }
    static __device__ int SB(const LatSweep<L, RPT> &) { return LatSweep<L, RPT>::SB; }
    static __device__ int lidx(const LatSweep<L, RPT> &, int i) { return LatSweep<L, RPT>::lidx(i); }
    // storages are consecutive blocks of SB bytes holding the spins as +-1
    static __device__ int layout_g(const LatSweep<L, RPT> &, int G) { return G; }
    static __device__ int pos(const LatSweep<L, RPT> &, int st, int p) { return st * LatSweep<L, RPT>::SB + p; }
    static __device__ int8_t enc(int m) { return (int8_t)m; }
    static __device__ int dec(int8_t v) { return v; }
    static __device__ size_t graph_bytes(const InstDev &) { return 0; }
    static __device__ void bind(LatSweep<L, RPT> &, const InstDev &, unsigned char *, int, int) {}

    // Contextual proposals work on one candidate storage X (same layout),
    // through a view of the graph that is passed by value (a lattice needs
    // none). ctx_sites calls f(i) for the sites of colour col this thread updates.
    struct CtxView {};
    static __device__ CtxView ctx_view(const LatSweep<L, RPT> &) { return CtxView{}; }
    static __device__ __forceinline__ int ctx_lidx(int i) { return LatSweep<L, RPT>::lidx(i); }
    template <class F>
    static __device__ __forceinline__ void ctx_sites(const CtxView &, const InstDev &, int col, int tid, int bs, F f)
    {
        constexpr int N = L * L * L;
        for (int i = tid; i < N; i += bs) {
            const int x = i % L, y = (i / L) % L, z = i / (L * L);
            if (((x + y + z) & 1) == col) f(i);
        }
    }
    // local field of site i (Eq. 4; a lattice has no fields)
    static __device__ __forceinline__ int ctx_field(const CtxView &, const InstDev &I, const int8_t *X, int i)
    {
        constexpr int N = L * L * L;
        using S = LatSweep<L, RPT>;
        const int x = i % L, y = (i / L) % L, z = i / (L * L);
        const int xm = (x + L - 1) % L + L * (y + L * z), xp = (x + 1) % L + L * (y + L * z);
        const int ym = x + L * ((y + L - 1) % L + L * z), yp = x + L * ((y + 1) % L + L * z);
        const int zm = x + L * (y + L * ((z + L - 1) % L)), zp = x + L * (y + L * ((z + 1) % L));
        const int8_t *J = I.J3;
        return J[i] * X[S::lidx(xp)] + J[xm] * X[S::lidx(xm)] + J[N + i] * X[S::lidx(yp)] + J[N + ym] * X[S::lidx(ym)] +
               J[2 * N + i] * X[S::lidx(zp)] + J[2 * N + zm] * X[S::lidx(zm)];
    }
    // twice site i's share of E(X): its +x, +y, +z bonds
    static __device__ __forceinline__ int ctx_energy2(const CtxView &, const InstDev &I, const int8_t *X, int i)
    {
        constexpr int N = L * L * L;
        using S = LatSweep<L, RPT>;
        const int x = i % L, y = (i / L) % L, z = i / (L * L);
        const int xp = (x + 1) % L + L * (y + L * z), yp = x + L * ((y + 1) % L + L * z);
        const int zp = x + L * (y + L * ((z + 1) % L));
        const int8_t *J = I.J3;
        return -2 * X[S::lidx(i)] * (J[i] * X[S::lidx(xp)] + J[N + i] * X[S::lidx(yp)] + J[2 * N + i] * X[S::lidx(zp)]);
    }
};

template <bool W>
struct SweepCall<CsrSweepT<W>> {
    static __device__ __forceinline__ void run(CsrSweepT<W> &sw, const InstDev &I, int G, int s0, uint32_t t, ChunkLds &c, int stride)
    {
        sw.sweep(I, G, s0, t, c.slot_of, c.sp, c.tab, stride, c.Elds, c.flips, c.rnd);
    }
    static __device__ int SB(const CsrSweepT<W> &s) { return s.SB; }
    static __device__ int lidx(const CsrSweepT<W> &, int i) { return i; }
    static __device__ int layout_g(const CsrSweepT<W> &, int G) { return G; }
    static __device__ int pos(const CsrSweepT<W> &s, int st, int p) { return st * s.SB + p; }
    static __device__ int8_t enc(int m) { return (int8_t)m; }
    static __device__ int dec(int8_t v) { return v; }
    static __device__ size_t graph_bytes(const InstDev &I) { return CsrSweepT<W>::graph_bytes(I); }
    static __device__ void bind(CsrSweepT<W> &sw, const InstDev &I, unsigned char *base, int tid, int bs)
    {
        sw.bind(I, base, tid, bs);
    }

    // Contextual proposals: the free sites of colour col from the LDS graph
    using CtxView = CsrGraph;
    static __device__ CtxView ctx_view(const CsrSweepT<W> &sw) { return sw.gr; }
    static __device__ __forceinline__ int ctx_lidx(int i) { return i; }
    template <class F>
    static __device__ __forceinline__ void ctx_sites(const CtxView &g, const InstDev &, int col, int tid, int bs, F f)
    {
        const int end = g.coff[col + 1];
        for (int q = g.coff[col] + tid; q < end; q += bs) f((int)g.cs[q]);
    }
    static __device__ __forceinline__ int ctx_field(const CtxView &g, const InstDev &, const int8_t *X, int i)
    {
        int f = g.h[i];
        for (int e = g.rp[i]; e < g.rp[i + 1]; ++e) {
            const uint32_t w = g.cw[e];
            f += (int)(int8_t)(w & 0xFFu) * (int)X[w >> 8];
        }
        return f;
    }
    // twice site i's share of E(X): half of each of its bonds, all of its field
    static __device__ __forceinline__ int ctx_energy2(const CtxView &g, const InstDev &, const int8_t *X, int i)
    {
        int s = 0;
        for (int e = g.rp[i]; e < g.rp[i + 1]; ++e) {
            const uint32_t w = g.cw[e];
            s += (int)(int8_t)(w & 0xFFu) * (int)X[w >> 8];
        }
        const int m = X[i];
        return -m * s - 2 * (int)g.h[i] * m;
    }
};

template <>
struct SweepCall<CsrRowSweep> {
    static __device__ __forceinline__ void run(CsrRowSweep &sw, const InstDev &I, int G, int s0, uint32_t t, ChunkLds &c,
                                               int stride)
    {
        sw.sweep(I, G, s0, t, c.slot_of, c.sp, c.tab, stride, c.Elds, c.flips, c.rnd);
    }
    static __device__ int SB(const CsrRowSweep &s) { return s.SB; }
    static __device__ int lidx(const CsrRowSweep &, int i) { return i; }
    static __device__ size_t graph_bytes(const InstDev &I) { return CsrRowSweep::graph_bytes(I); }
    static __device__ void bind(CsrRowSweep &sw, const InstDev &I, unsigned char *base, int tid, int bs)
    {
        sw.bind(I, base, tid, bs);
    }
    static __device__ int layout_g(const CsrRowSweep &, int G) { return G; }
    static __device__ int pos(const CsrRowSweep &s, int st, int p) { return st * s.SB + p; }
    static __device__ int8_t enc(int m) { return (int8_t)m; }
    static __device__ int dec(int8_t v) { return v; }
    struct CtxView {};
};

template <>
struct SweepCall<CsrRowQuadSweep> {
    static __device__ __forceinline__ void run(CsrRowQuadSweep &sw, const InstDev &I, int G, int s0, uint32_t t,
                                               ChunkLds &c, int stride)
    {
        sw.sweep(I, G, s0, t, c.slot_of, c.sp, c.tab, stride, c.Elds, c.flips, c.rnd);
    }
    // the carve-up takes GS slots of n bytes each, as for CsrQuadSweep
    static __device__ int SB(const CsrRowQuadSweep &s) { return s.n; }
    static __device__ int lidx(const CsrRowQuadSweep &, int i) { return i; }
    static __device__ size_t graph_bytes(const InstDev &I) { return CsrRowQuadSweep::graph_bytes(I); }
    static __device__ void bind(CsrRowQuadSweep &sw, const InstDev &I, unsigned char *base, int tid, int bs)
    {
        sw.bind(I, base, tid, bs);
    }
    static __device__ int layout_g(const CsrRowQuadSweep &s, int) { return s.GS; }
    static __device__ int pos(const CsrRowQuadSweep &s, int st, int p) { return p * s.GS + st; }
    static __device__ int8_t enc(int m) { return m < 0 ? 1 : 0; }
    static __device__ int dec(int8_t v) { return v ? -1 : 1; }
    struct CtxView {};
};

template <>
struct SweepCall<CsrQuadSweep> {
    static __device__ __forceinline__ void run(CsrQuadSweep &sw, const InstDev &I, int G, int s0, uint32_t t, ChunkLds &c,
                                               int stride)
    {
        sw.sweep(I, G, s0, t, c.slot_of, c.sp, c.tab, stride, c.Elds, c.flips, c.rnd);
    }
    // the carve-up takes GS slots of n bytes each: the interleaved storages
    // fill GS * n bytes and the staged random halves GS * nr
    static __device__ int SB(const CsrQuadSweep &s) { return s.n; }
    static __device__ int lidx(const CsrQuadSweep &, int i) { return i; }
    static __device__ size_t graph_bytes(const InstDev &I) { return CsrQuadSweep::graph_bytes(I); }
    static __device__ void bind(CsrQuadSweep &sw, const InstDev &I, unsigned char *base, int tid, int bs)
    {
        sw.bind(I, base, tid, bs);
    }
    static __device__ int layout_g(const CsrQuadSweep &s, int) { return s.GS; }
    static __device__ int pos(const CsrQuadSweep &s, int st, int p) { return p * s.GS + st; }
    static __device__ int8_t enc(int m) { return m < 0 ? 1 : 0; }
    static __device__ int dec(int8_t v) { return v ? -1 : 1; }
    struct CtxView {};
};

__device__ __forceinline__ uint32_t pick4(const P4 &r, int k)
{
    return k == 0 ? r.v[0] : k == 1 ? r.v[1] : k == 2 ? r.v[2] : r.v[3];
}

// Contextual proposals of the slots this workgroup holds (Supp. context
// ablation), at the proposal stage of cycle cyc. For each proposal-enabled
// slot, in increasing order: the candidate starts from the slot's bank entry;
// the ctx_K free sites of smallest CONTEXT key join the context and hold the
// slot's current values; ctx_sweeps colored sweeps
// at the slot's beta (Philox CTXSWEEP, one 32-bit word per attempt) update
// the other free sites; the Delta-E rule of Eq. 2 judges the candidate's
// recomputed energy. Every thread of the block takes part. Only the
// kernels instantiated for contextual batches compile it in, so the others
// keep their register allocation.
template <class Sw>
__device__ __forceinline__ void ctx_proposals(const typename SweepCall<Sw>::CtxView &gv, const InstDev &I, int G, int s0,
                                              uint32_t cyc, ChunkLds &c, int SB, int stride)
{
    const int tid = threadIdx.x, bs = blockDim.x, n = I.n, D = I.D;
    const uint32_t k0 = I.seed_lo, k1 = I.seed_hi;
    const int K = I.ctx_sweeps;
    const int KC = I.ctx_K;        // context sites per proposal
    for (int l = 0; l < G; ++l) {
        const int r = s0 + l;
        const int B = I.bank_n[r];
        if (B <= 0) continue;
        if (tid == 0) {
            c.misc[8] = I.cursor[r];
            c.misc[6] = 0;
        }
        __syncthreads();
        const int k = c.misc[8];
        const int st = c.stor_of[l];
        const int8_t *cur = c.sp + st * SB;
        const int8_t *src = I.bank[r] + (size_t)k * n;
        // the context: the KC free sites of smallest (key, index), found by a
        // radix select of the KC-th smallest key (8 bits a pass, highest first)
        for (int i = tid; i < n; i += bs)
            c.ckey[i] = pick4(philox((uint32_t)i >> 2, cyc, (uint32_t)r, TAG_CONTEXT, k0, k1), i & 3);
        uint32_t tau = 0;
        int take_eq = 0;                 // sites with key == tau that join, lowest index first
        if (KC > 0 && KC < I.nfree) {
            uint32_t prefix = 0;
            int remaining = KC;
            for (int pass = 0; pass < 4; ++pass) {
                const int shift = 24 - 8 * pass;
                for (int x = tid; x < 256; x += bs) c.chist[x] = 0;
                __syncthreads();
                for (int i = tid; i < n; i += bs) {
                    const uint32_t key = c.ckey[i];
                    if (I.clamp[i] == 0 && (pass == 0 || (key >> (shift + 8)) == prefix))
                        atomicAdd(&c.chist[(key >> shift) & 255u], 1);
                }
                __syncthreads();
                if (tid == 0) {
                    int below = 0, b = 0;
                    while (below + c.chist[b] < remaining) below += c.chist[b++];
                    c.misc[9] = b;
                    c.misc[10] = remaining - below;
                    c.misc[11] = c.chist[b];
                }
                __syncthreads();
                prefix = (prefix << 8) | (uint32_t)c.misc[9];
                remaining = c.misc[10];
            }
            tau = prefix;
            take_eq = remaining;             // of the c.misc[11] sites whose key is tau
        }
        const bool all_eq = KC >= I.nfree || take_eq >= c.misc[11];
        for (int i = tid; i < n; i += bs) {
            const int li = SweepCall<Sw>::ctx_lidx(i);
            const uint32_t key = c.ckey[i];
            const bool ctx = I.clamp[i] == 0 && KC > 0 &&
                             (KC >= I.nfree || key < tau || (key == tau && all_eq));
            c.cm[li] = ctx ? 1 : 0;
            c.cx[li] = ctx ? cur[li] : src[i];
        }
        __syncthreads();
        if (!all_eq && tid == 0) {
            // equal keys at the cut (rare): the lowest indices among them join
            int left = take_eq;
            for (int i = 0; i < n && left > 0; ++i) {
                if (I.clamp[i] != 0 || c.ckey[i] != tau) continue;
                const int li = SweepCall<Sw>::ctx_lidx(i);
                c.cm[li] = 1;
                c.cx[li] = cur[li];
                --left;
            }
        }
        __syncthreads();
        const uint32_t *trow = c.tab + l * stride + D;
        for (int j = 1; j <= K; ++j) {
            const uint32_t c2 = (uint32_t)r + 65536u * (uint32_t)j;
            for (int col = 0; col < I.ncolors; ++col) {
                SweepCall<Sw>::ctx_sites(gv, I, col, tid, bs, [&](int i) {
                    const int li = SweepCall<Sw>::ctx_lidx(i);
                    if (c.cm[li]) return;
                    const int m = c.cx[li];
                    const int d = m * SweepCall<Sw>::ctx_field(gv, I, c.cx, i);
                    const uint32_t T = trow[d];
                    const uint32_t u = pick4(philox((uint32_t)i >> 2, cyc, c2, TAG_CTXSWEEP, k0, k1), i & 3);
                    if (T == ALWAYS || u < T) c.cx[li] = (int8_t)(-m);
                });
                __syncthreads();
            }
        }
        // E of the candidate: twice each site's share, summed over the block
        int e2 = 0;
        for (int i = tid; i < n; i += bs) e2 += SweepCall<Sw>::ctx_energy2(gv, I, c.cx, i);
        e2 = wave_sum(e2);
        if ((tid & 63) == 0) atomicAdd(&c.misc[6], e2);
        __syncthreads();
        if (tid == 0) {
            const int ET = c.misc[6] / 2;
            const long long dd = (long long)ET - (long long)c.Elds[st];
            uint32_t T;
            if (dd <= 0) T = ALWAYS;
            else if (dd <= I.tprop_len[r]) T = I.tprop[I.tprop_off[r] + (int)dd - 1];
            else T = 0;
            const uint32_t u = philox_word0((uint32_t)r, cyc, TAG_PROPOSE, k0, k1);
            I.cursor[r] = (k + 1 == B) ? 0 : k + 1;
            I.prop_att[r] += 1;
            const bool acc = T == ALWAYS || u < T;
            if (acc) {
                I.prop_acc[r] += 1;
                c.Elds[st] = ET;
            }
            c.misc[7] = acc ? 1 : 0;
        }
        __syncthreads();
        if (c.misc[7]) {
            int8_t *dst = c.sp + st * SB;
            for (int x = tid; x < n; x += bs) dst[x] = c.cx[x];
        }
        __syncthreads();
    }
}


#define TAPT_LATTICE_LIST(X) X(4) X(6) X(8) X(10) X(12) X(14) X(16)
#define TAPT_MIXED_LATTICE_LIST(X) TAPT_LATTICE_LIST(X)

// Dynamic LDS of the persistent and plain kernels.
extern __shared__ __align__(16) unsigned char lds_raw[];

template <class Sw, bool CTX = false>
__device__ __forceinline__ void chunk_body(const ChunkArgs &a, const int item)
{
    const WorkItem it = a.items[item];
    const InstDev &I = *it.inst;
    RunParams P;
    P.load(I);
    const int G = it.G, s0 = it.s0, n = P.n;
    const int tid = threadIdx.x, bs = blockDim.x, lane = tid & 63;
    const uint64_t t0 = *I.t;
    const uint64_t cap = chunk_cap(I, t0);
    const uint64_t tend = (t0 + a.K < cap) ? t0 + a.K : cap;
    if (t0 >= tend) {
        if (tid == 0) idle_best(it.best);
        return;
    }

    Sw sw;
    sw.setup(I, G);
    const int SB = SweepCall<Sw>::SB(sw);
    const int GL = SweepCall<Sw>::layout_g(sw, G);   // slots the LDS carve-up is sized for
    const int stride = P.stride;
    const bool contextual = CTX && I.ctx_on != 0;
    const ChunkOff lof = chunk_lds_offsets(GL, SB, stride, Sw::RND ? ((n + 7) & ~7) : 0, a.tsw_entries, n,
                                           SweepCall<Sw>::graph_bytes(I), contextual);
    CHUNK_LDS_POINTERS(c, lof, GL, lds_raw);
    SweepCall<Sw>::bind(sw, I, lds_raw + lof.graph, tid, bs);

    // stage tables and state
    for (int x = tid; x < G * stride; x += bs) c.tab[x] = I.tflip[(size_t)s0 * stride + x];
    for (int x = tid; x < GL * SB; x += bs) c.sp[x] = SweepCall<Sw>::enc(1);   // padding storages too
    __syncthreads();
    for (int x = tid; x < G * n; x += bs) {
        int l = x / n, i = x - l * n;
        c.sp[SweepCall<Sw>::pos(sw, l, SweepCall<Sw>::lidx(sw, i))] = SweepCall<Sw>::enc(I.spins[(size_t)(s0 + l) * n + i]);
    }
    if (tid == 0) {
        int o = 0;
        for (int p = 0; p <= G; ++p) {
            c.tsw_off[p] = o;
            int r = s0 - 1 + p;
            if (r >= 0 && r + 1 < P.R) o += I.tswap_len[r];
        }
        c.tsw_off[G + 1] = o;
    }
    for (int l = tid; l < G; l += bs) {
        c.slot_of[l] = l;
        c.stor_of[l] = l;
        c.Elds[l] = I.E[s0 + l];
        c.flips[l] = 0;
        c.satt[l] = 0;
        c.sacc[l] = 0;
    }
    // misc[12]: the cycle end's outcome for the whole block, written by
    // wavefront 0 every sweep (bit 0: a wait timed out; bits 8-15 / 16-23:
    // storage + 1 that takes the partner's state across the lower / upper
    // boundary; bits 24-31: storage + 1 of a new best state). misc[13]: the
    // storages of slots 0 and G - 1 (bits 0-7, 8-15), which the next cycle
    // end publishes.
    if (tid < 16) c.misc[tid] = tid == 13 ? (G - 1) << 8 : 0;
    __syncthreads();
    for (int p = 0; p <= G; ++p) {
        int r = s0 - 1 + p;
        if (r < 0 || r + 1 >= P.R) continue;
        int lo = c.tsw_off[p], len = c.tsw_off[p + 1] - lo;
        for (int x = tid; x < len; x += bs) c.tsw[lo + x] = I.tswap[I.tswap_off[r] + x];
    }
    // best-energy bookkeeping lives in registers of wave 0
    int bestE = I.best->E;
    int64_t bestT = -1;
    int bestSlot = -1;
    int64_t hit = I.best->first_hit;
    const int64_t hit0 = hit;
    const bool has_down = it.w > 0, has_up = it.w + 1 < it.W;
    __syncthreads();

    // Wave-0 registers for the cycle-end stages (G <= 64): lane l is local
    // slot l; my_st is the storage holding it; (row_off, row_len) is the LDS
    // swap-threshold row of pair (s0+l, s0+l+1) -- for l = G-1 that is the
    // pair across the upper boundary; (dn_off, dn_len) the one across the lower.
    int my_st = lane, row_off = 0, row_len = 0, dn_off = 0, dn_len = 0;
    unsigned my_att = 0, my_acc = 0;
    if (tid < 64) {
        if (lane < G) {
            row_off = c.tsw_off[lane + 1];
            row_len = c.tsw_off[lane + 2] - row_off;
        }
        dn_off = c.tsw_off[0];
        dn_len = c.tsw_off[1] - dn_off;
    }
    const int nw = (n + 31) >> 5;
    if (tid < 64) {   // swap uniforms of the first cycle end of this launch
        const uint32_t c1 = (uint32_t)((t0 + (uint64_t)P.M) / (uint64_t)P.M);
        c.usw[(c1 & 1) * 65 + lane] = philox_word0((uint32_t)(s0 + lane), c1, TAG_SWAP, P.k0, P.k1);
        if (lane == 0 && has_down) c.usw[(c1 & 1) * 65 + 64] = philox_word0((uint32_t)(s0 - 1), c1, TAG_SWAP, P.k0, P.k1);
    }
    __syncthreads();

    bool failed = false;
    int xst = c.misc[13];
    // cycle bookkeeping by counting (t0 / M once per launch)
    uint32_t cyc = (uint32_t)(t0 / (uint64_t)P.M), phase = (uint32_t)(t0 % (uint64_t)P.M);
    uint64_t prop_at = P.first_prop_from(t0 + 1);
    for (uint64_t t = t0 + 1; t <= tend && !failed; ++t) {
        const bool cyc_end = ++phase == (uint32_t)P.M;
        if (cyc_end) {
            phase = 0;
            ++cyc;
        }
        SweepCall<Sw>::run(sw, I, G, s0, (uint32_t)t, c, stride);   // ends with a barrier
        // ---- proposals (Eq. 2), slots in increasing order ----
        const bool prop_now = t == prop_at;
        if (prop_now) prop_at = P.next_prop(prop_at);
        bool bank_prop = prop_now;
        if constexpr (CTX) {
            if (prop_now && contextual) {
                const typename SweepCall<Sw>::CtxView gv = SweepCall<Sw>::ctx_view(sw);
                ctx_proposals<Sw>(gv, I, G, s0, cyc, c, SB, stride);
                bank_prop = false;
            }
        }
        if (bank_prop) {
            if (tid < 64) {
                for (int l = lane; l < G; l += 64) {
                    int r = s0 + l;
                    c.src[l] = 0;
                    int B = I.bank_n[r];
                    if (B > 0) {
                        int k = I.cursor[r];
                        I.cursor[r] = (k + 1 == B) ? 0 : k + 1;
                        int ET = I.bankE[r][k];
                        int st = c.stor_of[l];
                        long long dd = (long long)ET - (long long)c.Elds[st];
                        uint32_t T;
                        if (dd <= 0) T = ALWAYS;
                        else if (dd <= I.tprop_len[r]) T = I.tprop[I.tprop_off[r] + (int)dd - 1];
                        else T = 0;
                        uint32_t u = philox_word0((uint32_t)r, cyc, TAG_PROPOSE, P.k0, P.k1);
                        I.prop_att[r] += 1;
                        if (T == ALWAYS || u < T) {
                            c.Elds[st] = ET;
                            c.src[l] = (long long)(I.bank[r] + (size_t)k * n);
                            I.prop_acc[r] += 1;
                        }
                    }
                }
            }
            __syncthreads();
            for (int l = 0; l < G; ++l) {
                const int8_t *src = (const int8_t *)c.src[l];
                if (src) {
                    const int st = c.stor_of[l];
                    for (int i = tid; i < n; i += bs)
                        c.sp[SweepCall<Sw>::pos(sw, st, SweepCall<Sw>::lidx(sw, i))] = SweepCall<Sw>::enc(src[i]);
                }
            }
            __syncthreads();
        }
        // the boundary slots in a cross pair this cycle (alternating parity)
        const int first = (cyc & 1) ? 0 : 1;
        const bool down = cyc_end && has_down && (((s0 - 1 - first) & 1) == 0);
        const bool up = cyc_end && has_up && (((s0 + G - 1 - first) & 1) == 0);
        const int buf = (cyc >> 1) & 1;
        const unsigned long long tag = (unsigned long long)cyc << 32;
        // wavefront 0's reads of the cycle end, in flight during the publish
        int e = 0x7FFFFFFF;
        uint32_t u_pair = 0, u_dn = 0;
        if (tid < 64) {
            if (lane < G) e = c.Elds[my_st];
            if (cyc_end) {
                u_pair = c.usw[(cyc & 1) * 65 + lane];
                u_dn = c.usw[(cyc & 1) * 65 + 64];
            }
        }
        if (down || up) {
            // publish the boundary states, every wavefront a share of the 64-byte
            // chunks. A boundary slot in a cross pair is in no local pair this
            // cycle. Bit j of the words is the sign of storage byte j (both sides
            // of a pair run the same sweeper, so they share the storage layout).
            // Every 64-bit word carries 32 spin bits (or the energy) and the cycle
            // number, written with relaxed device-scope atomics; the reader takes a
            // word only when its tag is this cycle, so no fence or flag is needed.
            // Buffers alternate with the cycle parity: a partner is at most one
            // exchange ahead.
            const int nch = (n + 63) >> 6, wv = tid >> 6, nwv = bs >> 6;
            for (int side = 0; side < 2; ++side) {
                if (!(side == 0 ? down : up)) continue;
                const int st = side == 0 ? (xst & 0xFF) : ((xst >> 8) & 0xFF);
                unsigned long long *out = it.xbuf + ((size_t)(it.w * 2 + side) * 2 + buf) * it.xwords;
                if (tid == 0)
                    __hip_atomic_store(out + nw, tag | (uint32_t)c.Elds[st], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                for (int ch0 = wv; ch0 < nch; ch0 += 4 * nwv) {
                    int8_t v[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {   // four chunks' reads in flight
                        const int j = 64 * (ch0 + q * nwv) + lane;
                        v[q] = c.sp[SweepCall<Sw>::pos(sw, st, j < n ? j : n - 1)];
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int ch = ch0 + q * nwv;
                        if (ch >= nch) break;
                        const unsigned long long m = __ballot(64 * ch + lane < n && SweepCall<Sw>::dec(v[q]) > 0);
                        const int wd = 2 * ch + lane;
                        if (lane < 2 && wd < nw)
                            __hip_atomic_store(out + wd, tag | (lane ? (m >> 32) : (m & 0xFFFFFFFFull)),
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
            }
        }
        if (tid >= 64 && tid < 128 && cyc_end) {
            // wave 1 draws the next cycle's swap uniforms while wave 0 works
            const uint32_t nx = cyc + 1;
            c.usw[(nx & 1) * 65 + lane] = philox_word0((uint32_t)(s0 + lane), nx, TAG_SWAP, P.k0, P.k1);
            if (lane == 0 && has_down) c.usw[(nx & 1) * 65 + 64] = philox_word0((uint32_t)(s0 - 1), nx, TAG_SWAP, P.k0, P.k1);
        }
        if (tid < 64) {
            int fl = 0;   // the block's outcome word (misc[12])
            // first poll of the partners' words (three per lane: n <= 6112 in
            // one round), issued before the local pairs are settled so that
            // its memory latency overlaps them
            unsigned long long pv[2][3] = {{0, 0, 0}, {0, 0, 0}};
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                if (!(side == 0 ? down : up)) continue;
                const int pw = side == 0 ? it.w - 1 : it.w + 1;
                const unsigned long long *in = it.xbuf + ((size_t)(pw * 2 + (side == 0 ? 1 : 0)) * 2 + buf) * it.xwords;
#pragma unroll
                for (int q = 0; q < 3; ++q)
                    if (lane + 64 * q <= nw)
                        pv[side][q] = __hip_atomic_load(in + lane + 64 * q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (cyc_end) {
                // ---- replica exchange (Eq. 1): the boundary states are published ----
                // pairs inside the workgroup: exchange labels (lane l decides (l, l+1))
                const int e_nx = from_next_lane(e), st_nx = from_next_lane(my_st);
                const bool act = lane + 1 < G && (((s0 + lane - first) & 1) == 0);
                bool acc = false;
                if (act) {
                    const int dE = e_nx - e;
                    const uint32_t T = dE >= 0 ? ALWAYS : (-dE <= row_len ? c.tsw[row_off - dE - 1] : 0u);
                    acc = T == ALWAYS || u_pair < T;
                    my_att += 1;
                    my_acc += acc ? 1u : 0u;
                }
                const bool acc_pv = (from_prev_lane((int)acc) != 0) && lane > 0;
                const int st_pv = from_prev_lane(my_st), e_pv = from_prev_lane(e);
                if (acc) {
                    my_st = st_nx;
                    e = e_nx;
                } else if (acc_pv) {
                    my_st = st_pv;
                    e = e_pv;
                }
                if ((acc || acc_pv) && lane < G) {
                    c.stor_of[lane] = my_st;
                    c.slot_of[my_st] = lane;
                }
                // pairs across a workgroup boundary: the partner's words and the
                // decision (both sides draw the same uniform); the block copies the
                // accepted states after the barrier
                if (down || up) {
                    int timeout = 0;
#pragma unroll
                    for (int side = 0; side < 2; ++side) {
                        if (!(side == 0 ? down : up) || timeout) continue;
                        const int pw = side == 0 ? it.w - 1 : it.w + 1;
                        const unsigned long long *in =
                            it.xbuf + ((size_t)(pw * 2 + (side == 0 ? 1 : 0)) * 2 + buf) * it.xwords;
                        uint32_t *stage = c.xstage + side * (nw + 1);
                        uint32_t polls = 0;
                        for (bool first = true;; first = false) {
                            bool ok = true;
                            unsigned long long bad = 0;
                            for (int wd = lane, q = 0; wd <= nw; wd += 64, ++q) {
                                // the first round takes the words read above
                                const unsigned long long v =
                                    (first && q < 3) ? (q == 0 ? pv[side][0] : q == 1 ? pv[side][1] : pv[side][2])
                                                     : __hip_atomic_load(in + wd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                                if ((uint32_t)(v >> 32) == cyc) {
                                    stage[wd] = (uint32_t)v;
                                } else {
                                    ok = false;
                                    bad = v;
                                }
                            }
                            if (__all(ok)) break;
                            __builtin_amdgcn_s_sleep(1);
                            if (++polls > a.spin_limit) {
                                timeout = 1;
                                if (!ok && atomicCAS(a.err, 0, 1) == 0) {
                                    a.err[1] = item;
                                    a.err[2] = it.w;
                                    a.err[3] = side;
                                    a.err[4] = (int)cyc;
                                    a.err[5] = (int)(bad & 0xFFFFFFFFu);
                                    a.err[6] = (int)(bad >> 32);
                                    a.err[7] = (int)I.epoch;
                                }
                                break;
                            }
                        }
                    }
                    timeout = __builtin_amdgcn_readlane(timeout, 0);
                    if (timeout) {
                        fl |= 1;
                    } else {
                        for (int side = 0; side < 2; ++side) {
                            if (!(side == 0 ? down : up)) continue;
                            const uint32_t *stage = c.xstage + side * (nw + 1);
                            const int pE = (int)stage[nw];
                            const int bl = side == 0 ? 0 : G - 1;            // my boundary slot
                            const int st = __builtin_amdgcn_readlane(my_st, bl);
                            const int myE = __builtin_amdgcn_readlane(e, bl);
                            const int dE = side == 0 ? myE - pE : pE - myE; // E_{r+1} - E_r
                            const int off = side == 0 ? dn_off : __builtin_amdgcn_readlane(row_off, G - 1);
                            const int len = side == 0 ? dn_len : __builtin_amdgcn_readlane(row_len, G - 1);
                            const uint32_t T = dE >= 0 ? ALWAYS : (-dE <= len ? c.tsw[off - dE - 1] : 0u);
                            const uint32_t u = side == 0 ? u_dn : (uint32_t)__builtin_amdgcn_readlane((int)u_pair, G - 1);
                            const bool sacc = (T == ALWAYS || u < T);
                            if (side == 1 && lane == G - 1) {   // the lower workgroup owns the pair's counters
                                my_att += 1;
                                my_acc += sacc ? 1u : 0u;
                            }
                            if (sacc) {
                                if (lane == bl) {
                                    e = pE;
                                    c.Elds[st] = pE;
                                }
                                fl |= (st + 1) << (8 + 8 * side);
                            }
                        }
                    }
                }
            }
            if (cyc_end && bs <= 64) {   // a one-wave workgroup draws the next uniforms itself
                const uint32_t nx = cyc + 1;
                c.usw[(nx & 1) * 65 + lane] = philox_word0((uint32_t)(s0 + lane), nx, TAG_SWAP, P.k0, P.k1);
                if (lane == 0 && has_down) c.usw[(nx & 1) * 65 + 64] = philox_word0((uint32_t)(s0 - 1), nx, TAG_SWAP, P.k0, P.k1);
            }
            // ---- best energy and first hit, after every stage of this sweep ----
            // key e*64 + lane orders by energy, then by slot (|E| < 2^24)
            const int key = wave_min(lane < G ? e * 64 + lane : 0x7FFFFFFF);
            const int em = key >> 6, lm = key & 63;
            if (P.has_target && hit < 0 && em <= P.target) hit = (int64_t)t;
            if (em < bestE) {
                bestE = em;
                bestT = (int64_t)t;
                bestSlot = s0 + lm;
                const int st = __builtin_amdgcn_readlane(my_st, lm);
                fl |= (st + 1) << 24;   // the whole block copies it below
            }
            if (lane == 0) {
                c.misc[12] = fl;
                c.misc[13] = __builtin_amdgcn_readlane(my_st, 0) | (__builtin_amdgcn_readlane(my_st, G - 1) << 8);
            }
        }
        __syncthreads();
        const int fl = c.misc[12];
        xst = c.misc[13];
        if (cyc_end && (has_down || has_up)) failed = (fl & 1) != 0;
        if (down || up) {   // accepted cross swaps: the partner's state into the storage
            const int x0 = (fl >> 8) & 0xFF, x1 = (fl >> 16) & 0xFF;
            if (x0 | x1) {
                for (int side = 0; side < 2; ++side) {
                    const int xs = side == 0 ? x0 : x1;
                    if (!xs) continue;
                    const uint32_t *stage = c.xstage + side * (nw + 1);
                    for (int j = tid; j < n; j += bs)
                        c.sp[SweepCall<Sw>::pos(sw, xs - 1, j)] =
                            SweepCall<Sw>::enc(((stage[j >> 5] >> (j & 31)) & 1u) ? 1 : -1);
                }
                __syncthreads();
            }
        }
        const int bst = (fl >> 24) & 0xFF;
        if (bst) {   // snapshot of the new best state, before the next sweep changes it
            for (int i = tid; i < n; i += bs)
                it.best_spins[i] = (int8_t)SweepCall<Sw>::dec(c.sp[SweepCall<Sw>::pos(sw, bst - 1, SweepCall<Sw>::lidx(sw, i))]);
            __syncthreads();
        }
    }
    if (tid < 64 && lane < G) {
        c.satt[lane] = my_att;
        c.sacc[lane] = my_acc;
    }
    __syncthreads();

    // write the state back by slot
    for (int x = tid; x < G * n; x += bs) {
        int l = x / n, i = x - l * n;
        I.spins[(size_t)(s0 + l) * n + i] =
            (int8_t)SweepCall<Sw>::dec(c.sp[SweepCall<Sw>::pos(sw, c.stor_of[l], SweepCall<Sw>::lidx(sw, i))]);
    }
    for (int l = tid; l < G; l += bs) {
        I.E[s0 + l] = c.Elds[c.stor_of[l]];
        I.flips[s0 + l] += c.flips[l];
        if (s0 + l + 1 < P.R) {
            I.swap_att[s0 + l] += c.satt[l];
            I.swap_acc[s0 + l] += c.sacc[l];
        }
    }
    if (tid == 0) {
        BestRec b;
        b.E = bestT >= 0 ? bestE : 0x7FFFFFFF;
        b.slot = bestSlot;
        b.t = bestT;
        b.first_hit = (hit0 < 0) ? hit : -1;
        b.pad = 0;
        *it.best = b;
    }
}


} // namespace tapt
