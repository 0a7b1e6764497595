// Persistent chunk kernels for batches with contextual proposals (the
// context ablation of the paper's supplement): the workgroup-synchronous
// body with the contextual proposal stage compiled in, for general graphs
// and for lattices with one slot per thread. Kept in their own translation
// unit and instantiation, so that the kernels of every other batch keep
// their register allocation.
#include "sweep.h"

namespace tapt {

template <class Sw>
__global__ void __launch_bounds__(Sw::MAXT) chunk_kernel_ctx(ChunkArgs a)
{
    const int item = a.order[blockIdx.x];
    if (item < 0) return;   // padding block that keeps the XCD placement aligned
    chunk_body<Sw, true>(a, item);
}

template <class Sw>
static hipError_t launch_t(const ChunkArgs &a, int block, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL(chunk_kernel_ctx<Sw>, dim3(a.n_items), dim3(block), lds, s, a);
    return hipGetLastError();
}

template <class Sw>
static hipError_t occupancy_t(int block, size_t lds, int *blocks_per_cu)
{
    hipError_t e = hipFuncSetAttribute((const void *)chunk_kernel_ctx<Sw>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, chunk_kernel_ctx<Sw>, block, lds);
}

// Host-side launchers (C++ linkage, used by the runtime in host.cpp).
hipError_t launch_chunk_ctx(int kind, int L, const ChunkArgs &a, int block, size_t lds, hipStream_t s)
{
    if (kind == KIND_CSR) return launch_t<CsrSweep>(a, block, lds, s);
#define X(LL) \
    if (L == LL) return launch_t<LatSweep<LL, 1>>(a, block, lds, s);
    TAPT_LATTICE_LIST(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t chunk_occupancy_ctx(int kind, int L, int block, size_t lds, int *blocks_per_cu)
{
    if (kind == KIND_CSR) return occupancy_t<CsrSweep>(block, lds, blocks_per_cu);
#define X(LL) \
    if (L == LL) return occupancy_t<LatSweep<LL, 1>>(block, lds, blocks_per_cu);
    TAPT_LATTICE_LIST(X)
#undef X
    return hipErrorInvalidValue;
}

} // namespace tapt
