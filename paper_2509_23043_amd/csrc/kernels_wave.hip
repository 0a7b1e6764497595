// Wave-per-replica persistent kernel for L^3 lattices with n / 8 == 64
// (L = 8): every wavefront owns one replica storage and runs Algorithm 1 for
// it with no workgroup barrier inside the sweep loop.
//
// A wavefront sweeps its storage under its current beta slot (its label, a
// wave-uniform value), reduces the energy change with DPP, runs the proposal
// stage of its slot (Eq. 2) and then settles the swap pair of its slot for
// this cycle (Eq. 1):
//   - partner slot in the same workgroup: both wavefronts publish their
//     energy in an LDS mailbox tagged with the cycle, read the other's, draw
//     the same uniform and, on acceptance, exchange labels;
//   - partner slot in the neighbouring workgroup: the boundary state and
//     energy go through cycle-tagged 64-bit words in global memory, as in
//     the workgroup-synchronous kernel, and an accepted swap copies the state.
// Only the two wavefronts of a pair wait for each other, so a slow exchange
// delays its pair and not the whole workgroup. Best energy and first hit are
// tracked per storage (its own record below the best known at launch start)
// and merged at the end; the merged record equals the lowest (E, t, slot)
// over the ladder because a storage reaches a new global minimum first
// exactly when the ladder does.
#include "sweep.h"

namespace tapt {

template <int L>
struct WaveLat {
    static constexpr int N = L * L * L;
    static constexpr int NC = N / 8;
    static_assert(NC == 64, "one wavefront per storage");
    static constexpr int SB = N;

    __host__ __device__ static constexpr int lidx(int i) { return (i & 7) * NC + (i >> 3); }

    int own[2][4];
    int nb[2][4][6];
    short2v J[2][4][3];
    int sh[2][4];

    __device__ static int site(int x, int y, int z)
    {
        x = (x + L) % L; y = (y + L) % L; z = (z + L) % L;
        return x + L * (y + L * z);
    }

    // lane q owns sites 8q..8q+7 of the storage at LDS byte offset base
    __device__ __forceinline__ void setup(const int8_t *J3, int q, int base)
    {
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
                own[c][s] = lidx(i) + base;
                for (int d = 0; d < 6; ++d) nb[c][s][d] = lidx(nbs[d]) + base;
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

    // One sweep of this lane's 8 sites under global slot `slot`; trow points at
    // the slot's flip-table row offset by D. Returns the lane's energy change
    // and flip count.
    __device__ __forceinline__ void sweep(uint32_t q, uint32_t t, uint32_t slot, uint32_t k0, uint32_t k1,
                                          int8_t *sp, const uint32_t *trow, int &dE, int &nf)
    {
        P4 r = philox(q, t, slot, TAG_SWEEP, k0, k1);
        dE = 0;
        nf = 0;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            int mm[4], dd[4];
            uint32_t TT[4], hs[4];
            bool acc[4], maybe[4];
            bool any_maybe = false;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                int m = sp[own[c][s]];
                short2v m01, m23, m45;
                m01.x = sp[nb[c][s][0]];
                m01.y = sp[nb[c][s][1]];
                m23.x = sp[nb[c][s][2]];
                m23.y = sp[nb[c][s][3]];
                m45.x = sp[nb[c][s][4]];
                m45.y = sp[nb[c][s][5]];
                int f = __builtin_amdgcn_sdot2(m01, J[c][s][0], 0, false);
                f = __builtin_amdgcn_sdot2(m23, J[c][s][1], f, false);
                f = __builtin_amdgcn_sdot2(m45, J[c][s][2], f, false);
                mm[s] = m;
                dd[s] = m * f;
                TT[s] = trow[dd[s]];
                hs[s] = (r.v[s] >> sh[c][s]) << 16;
                acc[s] = coarse_accept(TT[s], hs[s], maybe[s]);
                any_maybe |= maybe[s];
            }
            if (any_lane(any_maybe)) {
                P4 r2 = philox(opaque(q), t, slot, TAG_REFINE, k0, k1);
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    uint32_t lo = (r2.v[s] >> sh[c][s]) & 0xFFFFu;
                    if (maybe[s]) acc[s] = (TT[s] == ALWAYS) || ((hs[s] | lo) < TT[s]);
                }
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                if (acc[s]) {
                    sp[own[c][s]] = (int8_t)(-mm[s]);
                    dE += 2 * dd[s];
                    nf += 1;
                }
            }
            // the next color reads what this one wrote (same wavefront: LDS
            // operations complete in order; keep the compiler from moving them)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
    }
};

// LDS carve-up of the wave kernel.
struct WaveOff {
    size_t sp, tab, toff, tsw, mail, ints, xst, total;
};

__host__ __device__ inline WaveOff wave_lds_offsets(int G, int n, int stride, int tsw_entries)
{
    WaveOff f;
    size_t o = 0;
    f.sp = o; o = align16(o + (size_t)G * n);
    f.tab = o; o = align16(o + (size_t)G * stride * 4);
    f.toff = o; o = align16(o + (size_t)(G + 2) * 4);
    f.tsw = o; o = align16(o + (size_t)tsw_entries * 4);
    f.mail = o; o = align16(o + (size_t)4 * G * 8);
    f.ints = o; o = align16(o + (size_t)G * 4 * 16);   // 8 ints + a 6-int record per storage
    f.xst = o; o = align16(o + (size_t)G * 2 * (((n + 31) >> 5) + 1) * 4);
    f.total = o;
    return f;
}

// per-wave best record kept in LDS for the final merge
struct WaveRec {
    int E, slot;
    long long t, hit;
};

template <int L>
__global__ void __launch_bounds__(512) wave_kernel(ChunkArgs a)
{
    using Sw = WaveLat<L>;
    constexpr int N = Sw::N;
    const int item = a.order[blockIdx.x];
    if (item < 0) return;
    const WorkItem it = a.items[item];
    const InstDev &I = *it.inst;
    RunParams P;
    P.load(I);
    const int G = it.G, s0 = it.s0;
    const int tid = threadIdx.x, bs = blockDim.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);   // storage of this wavefront
    const uint64_t t0 = *I.t;
    const uint64_t cap = chunk_cap(I, t0);
    const uint64_t tend = (t0 + a.K < cap) ? t0 + a.K : cap;
    if (t0 >= tend) {
        if (tid == 0) idle_best(it.best);
        return;
    }
    const int stride = P.stride;
    const WaveOff lof = wave_lds_offsets(G, N, stride, a.tsw_entries);
    int8_t *sp = (int8_t *)(lds_raw + lof.sp);
    uint32_t *tab = (uint32_t *)(lds_raw + lof.tab);
    int *tsw_off = (int *)(lds_raw + lof.toff);
    uint32_t *tsw = (uint32_t *)(lds_raw + lof.tsw);
    unsigned long long *mail = (unsigned long long *)(lds_raw + lof.mail);   // [4][G]
    int *ints = (int *)(lds_raw + lof.ints);
    unsigned *flips = (unsigned *)ints;              // [G] by local slot
    unsigned *satt = flips + G, *sacc = flips + 2 * G;   // [G] by pair (s0 + l, s0 + l + 1)
    unsigned *patt = flips + 3 * G, *pacc = flips + 4 * G;
    int *cursor = ints + 5 * G;                      // [G] bank cursor by local slot at launch start
    int *stor_of = ints + 6 * G;                     // [G] final slot -> storage
    int *Efin = ints + 7 * G;                        // [G] final energy by storage
    WaveRec *rec = (WaveRec *)(ints + 8 * G);        // [G] (4 ints each)
    uint32_t *xstage = (uint32_t *)(lds_raw + lof.xst);

    // ---- stage tables, state and bookkeeping ----
    for (int x = tid; x < G * stride; x += bs) tab[x] = I.tflip[(size_t)s0 * stride + x];
    for (int x = tid; x < G * N; x += bs) {
        int l = x / N, i = x - l * N;
        sp[l * N + Sw::lidx(i)] = I.spins[(size_t)(s0 + l) * N + i];
    }
    if (tid == 0) {
        int o = 0;
        for (int p = 0; p <= G; ++p) {
            tsw_off[p] = o;
            int r = s0 - 1 + p;
            if (r >= 0 && r + 1 < P.R) o += I.tswap_len[r];
        }
        tsw_off[G + 1] = o;
    }
    for (int x = tid; x < 4 * G; x += bs) mail[x] = 0ull;
    for (int l = tid; l < G; l += bs) {
        flips[l] = 0;
        satt[l] = 0;
        sacc[l] = 0;
        patt[l] = 0;
        pacc[l] = 0;
        cursor[l] = I.cursor[s0 + l];
    }
    __syncthreads();
    for (int p = 0; p <= G; ++p) {
        int r = s0 - 1 + p;
        if (r < 0 || r + 1 >= P.R) continue;
        int lo = tsw_off[p], len = tsw_off[p + 1] - lo;
        for (int x = tid; x < len; x += bs) tsw[lo + x] = I.tswap[I.tswap_off[r] + x];
    }
    __syncthreads();

    // lane p of every wavefront: LDS swap-table row (offset, length) of pair s0 - 1 + p
    const int row_off_v = lane <= G ? tsw_off[lane] : 0;
    const int row_len_v = lane <= G ? tsw_off[lane + 1] - row_off_v : 0;
    const bool active = wv < G;
    int label = s0 + wv;                // global slot held by this storage
    uint32_t n_prop = 0;                // proposal stages run in this launch (every banked slot's
                                        // cursor advances by one per stage)
    int E = active ? I.E[s0 + wv] : 0;
    int bestE = I.best->E;
    long long bestT = -1, hit = -1;
    int bestSlot = -1;
    const bool want_hit = P.has_target && I.best->first_hit < 0;
    const bool has_down = it.w > 0, has_up = it.w + 1 < it.W;
    const int nw = (N + 31) >> 5;
    bool failed = false;
    int8_t *mine = sp + wv * N;
    int8_t *snap = it.best_spins + (size_t)wv * N;

    if (active) {
        Sw sw;
        sw.setup(I.J3, lane, wv * N);
        // cycle bookkeeping by counting (t0 / M once per launch)
        uint32_t cyc = (uint32_t)(t0 / (uint64_t)P.M), phase = (uint32_t)(t0 % (uint64_t)P.M);
        uint64_t prop_at = P.first_prop_from(t0 + 1);
        for (uint64_t t = t0 + 1; t <= tend && !failed; ++t) {
            const int l = label - s0;
            // swap uniforms of every pair this workgroup touches (lane p: pair s0 - 1 + p)
            // for the cycle this sweep ends, drawn before the sweep so that their
            // latency hides behind it
            uint32_t u_vec = 0;
            if (phase + 1 == (uint32_t)P.M)
                u_vec = philox_word0((uint32_t)(s0 - 1 + lane), cyc + 1, TAG_SWAP, P.k0, P.k1);
            int dE, nf;
            sw.sweep((uint32_t)lane, (uint32_t)t, (uint32_t)label, P.k0, P.k1, sp, tab + l * stride + P.D, dE, nf);
            dE = wave_sum(dE);
            nf = wave_sum(nf);
            E += dE;
            if (lane == 0 && nf) atomicAdd(&flips[l], (unsigned)nf);
            if (++phase == (uint32_t)P.M) {
                phase = 0;
                ++cyc;
                // ---- proposal of this slot (Eq. 2) ----
                const bool prop_now = t == prop_at;
                if (prop_now) prop_at = P.next_prop(prop_at);
                if (prop_now) {
                    const int B = I.bank_n[label];
                    if (B > 0) {
                        const int k = (int)(((uint32_t)cursor[l] + n_prop % (uint32_t)B) % (uint32_t)B);
                        if (lane == 0) atomicAdd(&patt[l], 1u);
                        const int ET = I.bankE[label][k];
                        const long long dd = (long long)ET - (long long)E;
                        uint32_t T;
                        if (dd <= 0) T = ALWAYS;
                        else if (dd <= I.tprop_len[label]) T = I.tprop[I.tprop_off[label] + (int)dd - 1];
                        else T = 0;
                        const uint32_t u = philox_word0((uint32_t)label, cyc, TAG_PROPOSE, P.k0, P.k1);
                        if (T == ALWAYS || u < T) {
                            const int8_t *src = I.bank[label] + (size_t)k * N;
                            for (int i = lane; i < N; i += 64) mine[Sw::lidx(i)] = src[i];
                            E = ET;
                            if (lane == 0) atomicAdd(&pacc[l], 1u);
                        }
                    }
                }
                if (prop_now) ++n_prop;
                // ---- swap of this slot's pair (Eq. 1), alternating parity ----
                const int first = (cyc & 1) ? 0 : 1;
                const bool lower = ((label - first) & 1) == 0;
                const int partner = lower ? label + 1 : label - 1;
                if (partner >= 0 && partner < P.R) {
                    const int pl = partner - s0;
                    const int r = lower ? label : partner;           // the pair's lower slot
                    const int prow = r - (s0 - 1);                   // its LDS swap-table row
                    int pE;
                    if (pl >= 0 && pl < G) {
                        // same workgroup: LDS mailboxes by (cycle mod 4, local slot)
                        unsigned long long *mb = mail + (cyc & 3) * G;
                        // (the word itself is the message: relaxed accesses suffice)
                        if (lane == 0)
                            __hip_atomic_store(mb + l, ((unsigned long long)cyc << 32) | (uint32_t)E, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
                        uint32_t polls = 0;
                        unsigned long long v;
                        for (;;) {
                            v = __hip_atomic_load(mb + pl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
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
                            break;
                        }
                        pE = (int)(uint32_t)v;
                        const int dEs = lower ? pE - E : E - pE;    // E_{r+1} - E_r
                        const int off = __builtin_amdgcn_readlane(row_off_v, prow);
                        const int len = __builtin_amdgcn_readlane(row_len_v, prow);
                        const uint32_t T = dEs >= 0 ? ALWAYS : (-dEs <= len ? tsw[off - dEs - 1] : 0u);
                        const uint32_t u = __builtin_amdgcn_readlane(u_vec, prow);
                        const bool acc = T == ALWAYS || u < T;
                        if (lower && lane == 0) {
                            atomicAdd(&satt[l], 1u);
                            if (acc) atomicAdd(&sacc[l], 1u);
                        }
                        if (acc) label = partner;
                    } else {
                        // across the workgroup boundary: tagged global words, state copy
                        const int side = pl < 0 ? 0 : 1;
                        if (side == 0 ? !has_down : !has_up) {
                            failed = true;   // cannot happen: the ladder split covers every slot
                            break;
                        }
                        const int buf = (cyc >> 1) & 1;
                        const unsigned long long tag = (unsigned long long)cyc << 32;
                        unsigned long long *out = it.xbuf + ((size_t)(it.w * 2 + side) * 2 + buf) * it.xwords;
                        for (int k0 = 0; k0 < (N >> 6); k0 += 8) {
                            int8_t v8[8];
#pragma unroll
                            for (int j = 0; j < 8; ++j) v8[j] = mine[Sw::lidx(64 * (k0 + j) + lane)];
#pragma unroll
                            for (int j = 0; j < 8; ++j) {
                                const unsigned long long m = __ballot(v8[j] > 0);
                                const int wd = 2 * (k0 + j) + lane;
                                if (lane < 2)
                                    __hip_atomic_store(out + wd, tag | (lane ? (m >> 32) : (m & 0xFFFFFFFFull)),
                                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            }
                        }
                        if (lane == 0)
                            __hip_atomic_store(out + nw, tag | (uint32_t)E, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        const int pw = side == 0 ? it.w - 1 : it.w + 1;
                        const unsigned long long *in =
                            it.xbuf + ((size_t)(pw * 2 + (side == 0 ? 1 : 0)) * 2 + buf) * it.xwords;
                        uint32_t *stage = xstage + (size_t)(wv * 2 + side) * (nw + 1);
                        uint32_t polls = 0;
                        bool ok_all = false;
                        unsigned long long bad = 0;
                        for (;;) {
                            bool ok = true;
                            for (int wd = lane; wd <= nw; wd += 64) {
                                unsigned long long v = __hip_atomic_load(in + wd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                                if ((uint32_t)(v >> 32) == cyc) {
                                    stage[wd] = (uint32_t)v;
                                } else {
                                    ok = false;
                                    bad = v;
                                }
                            }
                            if (__all(ok)) {
                                ok_all = true;
                                break;
                            }
                            __builtin_amdgcn_s_sleep(1);
                            if (++polls > a.spin_limit) break;
                        }
                        if (!ok_all) {
                            if (lane == 0 && atomicCAS(a.err, 0, 1) == 0) {
                                a.err[1] = item; a.err[2] = it.w; a.err[3] = side; a.err[4] = (int)cyc;
                                a.err[5] = (int)(bad & 0xFFFFFFFFu); a.err[6] = (int)(bad >> 32); a.err[7] = (int)I.epoch;
                            }
                            failed = true;
                            break;
                        }
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        pE = (int)stage[nw];
                        const int dEs = lower ? pE - E : E - pE;
                        const int off = __builtin_amdgcn_readlane(row_off_v, prow);
                        const int len = __builtin_amdgcn_readlane(row_len_v, prow);
                        const uint32_t T = dEs >= 0 ? ALWAYS : (-dEs <= len ? tsw[off - dEs - 1] : 0u);
                        const uint32_t u = __builtin_amdgcn_readlane(u_vec, prow);
                        const bool acc = T == ALWAYS || u < T;
                        if (side == 1 && lane == 0) {   // the lower workgroup owns the pair's counters
                            atomicAdd(&satt[l], 1u);
                            if (acc) atomicAdd(&sacc[l], 1u);
                        }
                        if (acc) {
                            uint32_t wd8[N >> 6];
#pragma unroll
                            for (int j = 0; j < (N >> 6); ++j) wd8[j] = stage[(64 * j + lane) >> 5];
#pragma unroll
                            for (int j = 0; j < (N >> 6); ++j) {
                                const int i = 64 * j + lane;
                                mine[Sw::lidx(i)] = ((wd8[j] >> (i & 31)) & 1u) ? 1 : -1;
                            }
                            E = pE;
                        }
                    }
                }
            }
            // ---- best energy and first hit of this storage ----
            if (want_hit && hit < 0 && E <= P.target) hit = (long long)t;
            if (E < bestE) {
                bestE = E;
                bestT = (long long)t;
                bestSlot = label;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                for (int i = lane; i < N; i += 64) snap[i] = mine[Sw::lidx(i)];
            }
        }
        if (lane == 0) {
            stor_of[label - s0] = wv;
            Efin[wv] = E;
            WaveRec w;
            w.E = bestE;
            w.slot = bestSlot;
            w.t = bestT;
            w.hit = hit;
            rec[wv] = w;
        }
    }
    __shared__ int win, any_failed;
    if (tid == 0) any_failed = 0;
    __syncthreads();
    if (failed && lane == 0) any_failed = 1;
    __syncthreads();
    if (any_failed) return;   // the host reports the error; the launch's state is abandoned
    // write the state back by slot
    for (int x = tid; x < G * N; x += bs) {
        int l = x / N, i = x - l * N;
        I.spins[(size_t)(s0 + l) * N + i] = sp[stor_of[l] * N + Sw::lidx(i)];
    }
    for (int l = tid; l < G; l += bs) {
        I.E[s0 + l] = Efin[stor_of[l]];
        I.flips[s0 + l] += flips[l];
        {   // every wavefront ran the same proposal stages; these threads are in wavefront 0
            const int B = I.bank_n[s0 + l];
            if (B > 0) I.cursor[s0 + l] = (int)(((uint32_t)cursor[l] + n_prop % (uint32_t)B) % (uint32_t)B);
        }
        I.prop_att[s0 + l] += patt[l];
        I.prop_acc[s0 + l] += pacc[l];
        if (s0 + l + 1 < P.R) {
            I.swap_att[s0 + l] += satt[l];
            I.swap_acc[s0 + l] += sacc[l];
        }
    }
    // merge the storages' records: lowest (E, t, slot); earliest hit
    if (tid == 0) {
        int wb = -1;
        long long h = -1;
        for (int w = 0; w < G; ++w) {
            const WaveRec r = rec[w];
            if (r.hit >= 0 && (h < 0 || r.hit < h)) h = r.hit;
            if (r.t < 0) continue;
            if (wb < 0 || r.E < rec[wb].E || (r.E == rec[wb].E && (r.t < rec[wb].t || (r.t == rec[wb].t && r.slot < rec[wb].slot))))
                wb = w;
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

bool wave_supported(int L) { return L == 8; }

int wave_max_storages() { return 8; }

size_t wave_lds_bytes(int n, int G, int stride, int tsw_entries)
{
    return wave_lds_offsets(G, n, stride, tsw_entries).total;
}

hipError_t launch_wave(int L, const ChunkArgs &a, int block, size_t lds, hipStream_t s)
{
    if (L != 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(wave_kernel<8>, dim3(a.n_items), dim3(block), lds, s, a);
    return hipGetLastError();
}

hipError_t wave_occupancy(int L, int block, size_t lds, int *blocks_per_cu)
{
    if (L != 8) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute((const void *)wave_kernel<8>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, wave_kernel<8>, block, lds);
}

} // namespace tapt
