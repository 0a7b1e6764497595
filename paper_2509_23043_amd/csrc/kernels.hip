// HIP kernels of the TAPT hot path for gfx950 (MI355X).
//
// Algorithm 1 of arXiv:2509.23043: replicas sweep their spins with a
// single-spin rule (Methods, Eqs. 4-5) over color classes of the coupling
// graph (Methods, Graph coloring); at the end of each cycle of M sweeps the
// proposal-enabled replicas test a pre-generated configuration with the
// Delta-E-only rule (Eq. 2) and neighbouring replicas exchange states with
// alternating parity (Eq. 1).
//
// Everything on the device is integer: int8 spins and couplings, int32
// energies, uint32 uniforms from Philox4x32-10 compared with uint32 threshold
// tables that the host built in FP64. No step is a dense contraction, so no
// MFMA is used; the sweep is bound by LDS instruction issue and VALU.
//
// Persistent chunk kernel: each workgroup owns G consecutive beta slots of one
// instance and keeps their spins in LDS for K sweeps. Swaps between slots of
// the same workgroup exchange labels (slot <-> storage maps in LDS); swaps
// across a workgroup boundary copy the boundary state through global memory
// as cycle-tagged 64-bit words (relaxed device-scope atomics, no cache
// maintenance on the critical path). All random numbers are keyed by
// (seed, site, sweep, slot, stream tag), never by thread or storage, so the
// chain is the same for every tiling, batch and launch sequence.
#include "sweep.h"

namespace tapt {

template <class Sw>
__global__ void __launch_bounds__(Sw::MAXT, Sw::MINW) chunk_kernel(ChunkArgs a)
{
    const int item = a.order[blockIdx.x];
    if (item < 0) return;   // padding block that keeps the XCD placement aligned
    chunk_body<Sw>(a, item);
}


// Merge the per-workgroup best records of one instance into its canonical
// record, and advance its sweep counter. One workgroup per instance.
__global__ void finish_kernel(const WorkItem *items, const int *first_item, int n_inst, uint32_t K,
                              InstStatus *status)
{
    int inst = blockIdx.x;
    if (inst >= n_inst) return;
    const WorkItem *its = items + first_item[inst];
    const InstDev &I = *its[0].inst;
    const int W = its[0].W;
    __shared__ int win;
    if (threadIdx.x == 0) {
        BestRec cb = *I.best;
        // as the round's sweep launch saw it (chunk_cap)
        const bool stopped = I.stop_at_hit && cb.first_hit >= 0;
        int wbest = -1;
        long long hit = -1;
        for (int w = 0; w < W; ++w) {
            BestRec b = *its[w].best;
            if (b.first_hit >= 0 && (hit < 0 || b.first_hit < hit)) hit = b.first_hit;
            if (b.t < 0) continue;
            if (b.E < cb.E || (b.E == cb.E && (b.t < cb.t || (b.t == cb.t && b.slot < cb.slot)))) {
                cb.E = b.E;
                cb.t = b.t;
                cb.slot = b.slot;
                wbest = w;
            }
        }
        if (cb.first_hit < 0 && hit >= 0) cb.first_hit = hit;
        *I.best = cb;
        win = wbest;
        uint64_t t0 = *I.t;
        const uint64_t cap = stopped ? t0 : I.sweep_cap;
        uint64_t t1 = t0 + K < cap ? t0 + K : cap;
        if (t0 < t1) *I.t = t1;
        if (status) {
            InstStatus st;
            st.t = (int64_t)(t0 < t1 ? t1 : t0);
            st.best_t = cb.t;
            st.first_hit = cb.first_hit;
            st.best_E = cb.E;
            st.best_slot = cb.slot;
            status[inst] = st;
        }
    }
    __syncthreads();
    if (win >= 0)
        for (int i = threadIdx.x; i < I.n; i += blockDim.x) I.best_spins[i] = its[win].best_spins[i];
}

// ---------------------------------------------------------------------------
// Plain path: one launch per sweep (every replica, one workgroup each), then a
// one-workgroup tail launch for the cycle-end stages and best tracking.
template <class Sw>
__global__ void __launch_bounds__(Sw::MAXT) plain_sweep_kernel(const InstDev *Ip, uint32_t t)
{
    const InstDev &I = *Ip;
    const int r = blockIdx.x, n = I.n, tid = threadIdx.x, bs = blockDim.x;
    Sw sw;
    sw.setup(I, 1);
    const int SB = SweepCall<Sw>::SB(sw);
    const int stride = I.tflip_stride;
    const ChunkOff lof = chunk_lds_offsets(1, SB, stride, Sw::RND ? ((n + 7) & ~7) : 0, 0, n,
                                           SweepCall<Sw>::graph_bytes(I));
    CHUNK_LDS_POINTERS(c, lof, 1, lds_raw);
    SweepCall<Sw>::bind(sw, I, lds_raw + lof.graph, tid, bs);
    for (int x = tid; x < stride; x += bs) c.tab[x] = I.tflip[(size_t)r * stride + x];
    for (int i = tid; i < n; i += bs) c.sp[SweepCall<Sw>::lidx(sw, i)] = I.spins[(size_t)r * n + i];
    if (tid == 0) {
        c.slot_of[0] = 0;
        c.stor_of[0] = 0;
        c.Elds[0] = 0;
        c.flips[0] = 0;
    }
    __syncthreads();
    SweepCall<Sw>::run(sw, I, 1, r, t, c, stride);
    __syncthreads();
    for (int i = tid; i < n; i += bs) I.spins[(size_t)r * n + i] = c.sp[SweepCall<Sw>::lidx(sw, i)];
    if (tid == 0) {
        I.E[r] += c.Elds[0];
        I.flips[r] += c.flips[0];
    }
}

__global__ void __launch_bounds__(256) plain_tail_kernel(const InstDev *Ip, uint32_t t)
{
    const InstDev &I = *Ip;
    const int n = I.n, R = I.R, tid = threadIdx.x, bs = blockDim.x;
    const uint32_t k0 = I.seed_lo, k1 = I.seed_hi;
    __shared__ int acc_s[1024];
    __shared__ int bank_k[1024];
    if (t % (uint32_t)I.M == 0) {
        const uint32_t cyc = t / (uint32_t)I.M;
        if (is_prop_sweep(I, t)) {
            for (int r = tid; r < R; r += bs) {
                acc_s[r] = 0;
                int B = I.bank_n[r];
                if (B <= 0) continue;
                int k = I.cursor[r];
                I.cursor[r] = (k + 1 == B) ? 0 : k + 1;
                int ET = I.bankE[r][k];
                long long dd = (long long)ET - (long long)I.E[r];
                uint32_t T;
                if (dd <= 0) T = ALWAYS;
                else if (dd <= I.tprop_len[r]) T = I.tprop[I.tprop_off[r] + (int)dd - 1];
                else T = 0;
                uint32_t u = philox_word0((uint32_t)r, cyc, TAG_PROPOSE, k0, k1);
                I.prop_att[r] += 1;
                if (T == ALWAYS || u < T) {
                    acc_s[r] = 1;
                    bank_k[r] = k;
                    I.E[r] = ET;
                    I.prop_acc[r] += 1;
                }
            }
            __syncthreads();
            for (int r = 0; r < R; ++r) {
                if (!acc_s[r]) continue;
                const int8_t *src = I.bank[r] + (size_t)bank_k[r] * n;
                for (int i = tid; i < n; i += bs) I.spins[(size_t)r * n + i] = src[i];
            }
            __syncthreads();
        }
        const int first = (cyc & 1) ? 0 : 1;
        for (int r = tid; r + 1 < R; r += bs) {
            acc_s[r] = 0;
            if (((r - first) & 1) != 0) continue;
            int dE = I.E[r + 1] - I.E[r];
            uint32_t T;
            if (dE >= 0) T = ALWAYS;
            else if (-dE <= I.tswap_len[r]) T = I.tswap[I.tswap_off[r] - dE - 1];
            else T = 0;
            uint32_t u = philox_word0((uint32_t)r, cyc, TAG_SWAP, k0, k1);
            I.swap_att[r] += 1;
            if (T == ALWAYS || u < T) {
                acc_s[r] = 1;
                I.swap_acc[r] += 1;
                int e = I.E[r];
                I.E[r] = I.E[r + 1];
                I.E[r + 1] = e;
            }
        }
        __syncthreads();
        for (int r = 0; r + 1 < R; ++r) {
            if (!acc_s[r]) continue;
            int8_t *a = I.spins + (size_t)r * n, *b = I.spins + (size_t)(r + 1) * n;
            for (int i = tid; i < n; i += bs) {
                int8_t x = a[i];
                a[i] = b[i];
                b[i] = x;
            }
        }
        __syncthreads();
    }
    // best energy and first hit
    __shared__ int be[256], bl[256];
    int e = 0x7FFFFFFF, ls = 0x7FFFFFFF;
    for (int r = tid; r < R; r += bs) {
        int v = I.E[r];
        if (v < e) { e = v; ls = r; }
    }
    be[tid] = e;
    bl[tid] = ls;
    __syncthreads();
    for (int off = bs / 2; off > 0; off >>= 1) {
        if (tid < off) {
            int e2 = be[tid + off], l2 = bl[tid + off];
            if (e2 < be[tid] || (e2 == be[tid] && l2 < bl[tid])) { be[tid] = e2; bl[tid] = l2; }
        }
        __syncthreads();
    }
    __shared__ int better_s;
    if (tid == 0) {
        BestRec b = *I.best;
        if (I.has_target && b.first_hit < 0 && be[0] <= I.target) b.first_hit = t;
        better_s = be[0] < b.E;
        if (better_s) {
            b.E = be[0];
            b.t = t;
            b.slot = bl[0];
        }
        *I.best = b;
        *I.t = t;
    }
    __syncthreads();
    if (better_s)
        for (int i = tid; i < n; i += bs) I.best_spins[i] = I.spins[(size_t)bl[0] * n + i];
}

// ---------------------------------------------------------------------------
// Initialization (Algorithm 1, random initial replica states): spin i
// of slot r is +1 iff word (i & 3) of Philox(i >> 2, 0, r, INIT) >= 2^31;
// clamped sites take their clamp value.
__global__ void init_kernel(const InstDev *Ip)
{
    const InstDev &I = *Ip;
    const int n = I.n;
    const int ng = (n + 3) >> 2;
    int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= ng * I.R) return;
    int r = gid / ng, g = gid - r * ng;
    P4 w = philox((uint32_t)g, 0, (uint32_t)r, TAG_INIT, I.seed_lo, I.seed_hi);
    for (int j = 0; j < 4; ++j) {
        int i = 4 * g + j;
        if (i >= n) break;
        int cl = I.clamp[i];
        I.spins[(size_t)r * n + i] = cl ? (int8_t)cl : (int8_t)(w.v[j] >= 0x80000000u ? 1 : -1);
    }
}

// Full energy E(m) = -sum_{i<j} J_ij m_i m_j - sum_i h_i m_i (Supp. S4) of k
// configurations: one workgroup per configuration, lane partial sums reduced
// across the wavefront and then through LDS.
__global__ void __launch_bounds__(256) energy_kernel(const InstDev *Ip, const int8_t *cfg, int k, int32_t *out)
{
    const InstDev &I = *Ip;
    const int b = blockIdx.x;
    if (b >= k) return;
    const int n = I.n;
    const int8_t *m = cfg + (size_t)b * n;
    int e = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        int mi = m[i];
        int f = I.h[i];
        if (I.kind == KIND_LATTICE) {
            int L = I.L;
            int x = i % L, y = (i / L) % L, z = i / (L * L);
            int jx = x + 1 == L ? i - (L - 1) : i + 1;
            int jy = y + 1 == L ? i - (L - 1) * L : i + L;
            int jz = z + 1 == L ? i - (L - 1) * L * L : i + L * L;
            f = f + I.J3[i] * m[jx] + I.J3[n + i] * m[jy] + I.J3[2 * n + i] * m[jz];
        } else {
            for (int q = I.row_ptr[i]; q < I.row_ptr[i + 1]; ++q) {
                int j = I.col[q];
                if (j > i) f += (int)I.Jc[q] * (int)m[j];
            }
        }
        e -= mi * f;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off);
    __shared__ int part[16];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) s += part[w];
        out[b] = s;
    }
}

// Record the state right after initialization as the first best (t = 0).
__global__ void init_best_kernel(const InstDev *Ip)
{
    const InstDev &I = *Ip;
    __shared__ int slot_s;
    if (threadIdx.x == 0) {
        int e = 0x7FFFFFFF, ls = 0;
        for (int r = 0; r < I.R; ++r)
            if (I.E[r] < e) { e = I.E[r]; ls = r; }
        BestRec b;
        b.E = e;
        b.slot = ls;
        b.t = 0;
        b.first_hit = (I.has_target && e <= I.target) ? 0 : -1;
        b.pad = 0;
        *I.best = b;
        slot_s = ls;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < I.n; i += blockDim.x) I.best_spins[i] = I.spins[(size_t)slot_s * I.n + i];
}

// ---------------------------------------------------------------------------
// Host-side launchers (C++ linkage, used by the runtime in host.cpp).

bool lattice_supported(int L) { return L >= 4 && L <= 16 && L % 2 == 0; }

int lattice_max_threads() { return 512; }

int lattice_threads(int L, int G, int rpt) { return ((G + rpt - 1) / rpt) * (L * L * L / 8); }

size_t chunk_lds_bytes(int kind, int n, int G, int stride, int tsw_entries, int nnz, int nfree, int ncolors,
                       bool contextual, int sparse, size_t row_graph)
{
    if (kind == KIND_CSR && sparse == SPARSE_ROW4)   // interleaved storages, packed rows of row_graph bytes
        return chunk_lds_offsets(CsrRowQuadSweep::group_bytes(G), n, stride, (n + 7) & ~7, tsw_entries, n, row_graph,
                                 false).total;
    if (kind == KIND_CSR && sparse == SPARSE_ROW)    // per-storage bytes, packed rows of row_graph bytes
        return chunk_lds_offsets(G, CsrSweep::storage_bytes(n), stride, (n + 7) & ~7, tsw_entries, n, row_graph,
                                 false).total;
    if (kind == KIND_CSR && sparse == SPARSE_QUAD)
        return chunk_lds_offsets(CsrQuadSweep::group_bytes(G), n, stride, (n + 7) & ~7, tsw_entries, n,
                                 quad_graph_bytes(n, nnz, nfree, ncolors), false).total;
    int SB = kind == KIND_LATTICE ? n : CsrSweep::storage_bytes(n);
    int nr = kind == KIND_LATTICE ? 0 : ((n + 7) & ~7);
    size_t gb = kind == KIND_LATTICE ? 0 : csr_graph_bytes(n, nnz, nfree, ncolors);
    return chunk_lds_offsets(G, SB, stride, nr, tsw_entries, n, gb, contextual).total;
}

template <class K>
static hipError_t set_lds(K kern, size_t lds)
{
    return hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

// The dynamic-LDS attribute is set by chunk_occupancy, which the runtime calls
// before the first launch, so nothing here is illegal under stream capture.
template <class Sw>
static hipError_t launch_chunk_t(const ChunkArgs &a, int block, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL(chunk_kernel<Sw>, dim3(a.n_items), dim3(block), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_chunk(int kind, int L, int rpt, int sparse, const ChunkArgs &a, int block, size_t lds, hipStream_t s)
{
    if (kind == KIND_CSR) {
        switch (sparse) {
        case SPARSE_ROW4: return launch_chunk_t<CsrRowQuadSweep>(a, block, lds, s);
        case SPARSE_ROW: return launch_chunk_t<CsrRowSweep>(a, block, lds, s);
        case SPARSE_QUAD: return launch_chunk_t<CsrQuadSweep>(a, block, lds, s);
        case SPARSE_WIDE: return launch_chunk_t<CsrSweepWide>(a, block, lds, s);
        default: return launch_chunk_t<CsrSweep>(a, block, lds, s);
        }
    }
#define X(LL)                                                                         \
    if (L == LL) {                                                                    \
        if (rpt == 1) return launch_chunk_t<LatSweep<LL, 1>>(a, block, lds, s);       \
        if (rpt == 2) return launch_chunk_t<LatSweep<LL, 2>>(a, block, lds, s);       \
        if (rpt == 4) return launch_chunk_t<LatSweep<LL, 4>>(a, block, lds, s);       \
    }
    TAPT_LATTICE_LIST(X)
#undef X
    return hipErrorInvalidValue;
}

template <class Sw>
static hipError_t occupancy_t(int block, size_t lds, int *blocks_per_cu)
{
    hipError_t e = set_lds(chunk_kernel<Sw>, lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, chunk_kernel<Sw>, block, lds);
}

hipError_t chunk_occupancy(int kind, int L, int rpt, int sparse, int block, size_t lds, int *blocks_per_cu)
{
    if (kind == KIND_CSR) {
        switch (sparse) {
        case SPARSE_ROW4: return occupancy_t<CsrRowQuadSweep>(block, lds, blocks_per_cu);
        case SPARSE_ROW: return occupancy_t<CsrRowSweep>(block, lds, blocks_per_cu);
        case SPARSE_QUAD: return occupancy_t<CsrQuadSweep>(block, lds, blocks_per_cu);
        case SPARSE_WIDE: return occupancy_t<CsrSweepWide>(block, lds, blocks_per_cu);
        default: return occupancy_t<CsrSweep>(block, lds, blocks_per_cu);
        }
    }
#define X(LL)                                                                      \
    if (L == LL) {                                                                 \
        if (rpt == 1) return occupancy_t<LatSweep<LL, 1>>(block, lds, blocks_per_cu); \
        if (rpt == 2) return occupancy_t<LatSweep<LL, 2>>(block, lds, blocks_per_cu); \
        if (rpt == 4) return occupancy_t<LatSweep<LL, 4>>(block, lds, blocks_per_cu); \
    }
    TAPT_LATTICE_LIST(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_finish(const WorkItem *items, const int *first_item, int n_inst, uint32_t K, InstStatus *status,
                         hipStream_t s)
{
    hipLaunchKernelGGL(finish_kernel, dim3(n_inst), dim3(256), 0, s, items, first_item, n_inst, K, status);
    return hipGetLastError();
}


template <class Sw>
static hipError_t launch_plain_sweep_t(const InstDev *dI, int R, int block, size_t lds, uint32_t t, hipStream_t s)
{
    hipError_t e = set_lds(plain_sweep_kernel<Sw>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(plain_sweep_kernel<Sw>, dim3(R), dim3(block), lds, s, dI, t);
    return hipGetLastError();
}

hipError_t launch_plain(int kind, int L, const InstDev *dI, int R, int n, int stride, int nnz, int nfree, int ncolors,
                        uint32_t t, hipStream_t s)
{
    size_t lds = chunk_lds_bytes(kind, n, 1, stride, 0, nnz, nfree, ncolors, false, SPARSE_CSR, 0);
    hipError_t e;
    if (kind == KIND_CSR) {
        e = launch_plain_sweep_t<CsrSweep>(dI, R, 256, lds, t, s);
    } else {
        e = hipErrorInvalidValue;
        int block = (lattice_threads(L, 1, 1) + 63) & ~63;
#define X(LL) \
        if (L == LL) e = launch_plain_sweep_t<LatSweep<LL, 1>>(dI, R, block, lds, t, s);
        TAPT_LATTICE_LIST(X)
#undef X
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(plain_tail_kernel, dim3(1), dim3(256), 0, s, dI, t);
    return hipGetLastError();
}

hipError_t launch_init(const InstDev *dI, int R, int n, hipStream_t s)
{
    int ng = (n + 3) >> 2;
    int total = ng * R;
    hipLaunchKernelGGL(init_kernel, dim3((total + 255) / 256), dim3(256), 0, s, dI);
    return hipGetLastError();
}

hipError_t launch_energy(const InstDev *dI, const int8_t *cfg, int k, int32_t *out, hipStream_t s)
{
    if (k <= 0) return hipSuccess;
    hipLaunchKernelGGL(energy_kernel, dim3(k), dim3(256), 0, s, dI, cfg, k, out);
    return hipGetLastError();
}

// Zero `words` 64-bit words (a fill kernel rather than hipMemsetAsync, so that
// the clear may sit in a captured stream).
__global__ void zero_kernel(unsigned long long *p, size_t words)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride) p[i] = 0ull;
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t s)
{
    const size_t words = (bytes + 7) / 8;      // callers pass 8-byte aligned regions padded to 8 bytes
    if (words == 0) return hipSuccess;
    const size_t want = (words + 255) / 256, blocks = want < 1024 ? want : 1024;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (unsigned long long *)p, words);
    return hipGetLastError();
}

// Sweep caps of up to CAPS_PER_LAUNCH contexts of a batch, set on the device
// in one launch (the caps travel as kernel arguments).
constexpr int CAPS_PER_LAUNCH = 64;
struct CapSet {
    InstDev *inst[CAPS_PER_LAUNCH];
    unsigned long long cap[CAPS_PER_LAUNCH];
    int n;
};

__global__ void set_caps_kernel(CapSet cs)
{
    const int k = threadIdx.x;
    if (k < cs.n) cs.inst[k]->sweep_cap = cs.cap[k];
}

hipError_t launch_set_caps(InstDev *const *insts, const unsigned long long *caps, int n, hipStream_t s)
{
    for (int a = 0; a < n; a += CAPS_PER_LAUNCH) {
        CapSet cs{};
        cs.n = n - a < CAPS_PER_LAUNCH ? n - a : CAPS_PER_LAUNCH;
        for (int k = 0; k < cs.n; ++k) {
            cs.inst[k] = insts[a + k];
            cs.cap[k] = caps[a + k];
        }
        hipLaunchKernelGGL(set_caps_kernel, dim3(1), dim3(CAPS_PER_LAUNCH), 0, s, cs);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_init_best(const InstDev *dI, hipStream_t s)
{
    hipLaunchKernelGGL(init_best_kernel, dim3(1), dim3(256), 0, s, dI);
    return hipGetLastError();
}

uint32_t host_philox_word0(uint32_t c0, uint32_t c1, uint32_t c3, uint32_t k0, uint32_t k1)
{
    return philox_word0(c0, c1, c3, k0, k1);
}

} // namespace tapt
