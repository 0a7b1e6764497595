// The mixed persistent kernel: one launch for a batch whose instances need
// different sweepers. Kept in its own translation unit so that it compiles
// in parallel with the specialised kernels.
#include "sweep.h"

namespace tapt {

// One persistent launch for a batch whose instances need different sweepers
// (lattices of several sizes, general graphs): each workgroup runs the body
// of its own item's variant. The block is sized for the largest item; the
// others leave the surplus threads idle (they still take part in barriers).
constexpr int MIXED_MAXT = 512;

__host__ __device__ constexpr int mixed_variant(int kind, int L, int rpt)
{
    return kind == KIND_CSR ? 0 : 1 + ((L - 4) / 2) * 3 + (rpt == 4 ? 2 : rpt - 1);
}

// Each variant is a separate (not inlined) function, so that it gets its own
// register allocation instead of one shared by every variant's live values.
template <class Sw>
__device__ __noinline__ void chunk_body_call(const ChunkArgs a, const int item)
{
    chunk_body<Sw>(a, item);
}

__global__ void __launch_bounds__(MIXED_MAXT) chunk_kernel_mixed(ChunkArgs a)
{
    const int item = a.order[blockIdx.x];
    if (item < 0) return;
    switch (a.items[item].variant) {
    case 0: chunk_body_call<CsrSweep>(a, item); break;
#define X(LL)                                                                      \
    case mixed_variant(KIND_LATTICE, LL, 1): chunk_body_call<LatSweep<LL, 1>>(a, item); break; \
    case mixed_variant(KIND_LATTICE, LL, 2): chunk_body_call<LatSweep<LL, 2>>(a, item); break; \
    case mixed_variant(KIND_LATTICE, LL, 4): chunk_body_call<LatSweep<LL, 4>>(a, item); break;
        TAPT_MIXED_LATTICE_LIST(X)
#undef X
    default: break;
    }
}

// ---------------------------------------------------------------------------
// Host-side launchers (C++ linkage, used by the runtime in host.cpp).

int mixed_max_threads() { return MIXED_MAXT; }

int mixed_variant_of(int kind, int L, int rpt) { return mixed_variant(kind, L, rpt); }

hipError_t launch_chunk_mixed(const ChunkArgs &a, int block, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL(chunk_kernel_mixed, dim3(a.n_items), dim3(block), lds, s, a);
    return hipGetLastError();
}

hipError_t chunk_occupancy_mixed(int block, size_t lds, int *blocks_per_cu)
{
    hipError_t e = hipFuncSetAttribute((const void *)chunk_kernel_mixed, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, chunk_kernel_mixed, block, lds);
}

} // namespace tapt
