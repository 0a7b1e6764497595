// LDS read-bandwidth probe: the measured side of the LDS roofline that the
// benchmark reports. Every workgroup fills 32 KiB of LDS, then each lane
// issues unrolled, independent 8- or 16-byte LDS reads at conflict-free
// addresses (consecutive lanes read consecutive words) and folds them with
// XORs (three-input ones for 16-byte reads), so that the reads, not the
// folding, set the pace. The folded value is stored only when it equals one
// fixed word (a chance of 2^-32 per thread), which keeps the reads alive
// without a store per thread.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tapt.h"

namespace tapt {

constexpr int PROBE_THREADS = 256;
constexpr int PROBE_BYTES = 32 * 1024;         // LDS per workgroup

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Eight reads of 16 (or 8) bytes per lane at offsets of 4096 (or 2048) bytes,
// in one asm block that waits for its own reads, so that the compiler can
// neither merge, split nor drop them. The caller keeps
// lds_addr + 7 * offset + 16 (or 8) within the workgroup's PROBE_BYTES.
__device__ __forceinline__ uint32_t read8_b128(uint32_t lds_addr)
{
    u32x4 q0, q1, q2, q3, q4, q5, q6, q7;
    asm volatile(
        "ds_read_b128 %0, %8\n"
        "ds_read_b128 %1, %8 offset:4096\n"
        "ds_read_b128 %2, %8 offset:8192\n"
        "ds_read_b128 %3, %8 offset:12288\n"
        "ds_read_b128 %4, %8 offset:16384\n"
        "ds_read_b128 %5, %8 offset:20480\n"
        "ds_read_b128 %6, %8 offset:24576\n"
        "ds_read_b128 %7, %8 offset:28672\n"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(q0), "=&v"(q1), "=&v"(q2), "=&v"(q3), "=&v"(q4), "=&v"(q5), "=&v"(q6), "=&v"(q7)
        : "v"(lds_addr)
        : "memory");
    // one word of each read is folded (the reads completed inside the block);
    // folding all of them would make the XORs, not the reads, the bound
    return q0.x ^ q1.y ^ q2.z ^ q3.w ^ q4.x ^ q5.y ^ q6.z ^ q7.w;
}

__device__ __forceinline__ uint32_t read8_b64(uint32_t lds_addr)
{
    u32x2 q0, q1, q2, q3, q4, q5, q6, q7;
    asm volatile(
        "ds_read_b64 %0, %8\n"
        "ds_read_b64 %1, %8 offset:2048\n"
        "ds_read_b64 %2, %8 offset:4096\n"
        "ds_read_b64 %3, %8 offset:6144\n"
        "ds_read_b64 %4, %8 offset:8192\n"
        "ds_read_b64 %5, %8 offset:10240\n"
        "ds_read_b64 %6, %8 offset:12288\n"
        "ds_read_b64 %7, %8 offset:14336\n"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(q0), "=&v"(q1), "=&v"(q2), "=&v"(q3), "=&v"(q4), "=&v"(q5), "=&v"(q6), "=&v"(q7)
        : "v"(lds_addr)
        : "memory");
    return q0.x ^ q1.y ^ q2.x ^ q3.y ^ q4.x ^ q5.y ^ q6.x ^ q7.y;
}

// Per round each lane issues two asm blocks of eight reads (16 reads).
// Lane addresses: (lane slot) * BYTES, lane slot = (tid + 97 i) mod 256, so
// the lanes of a wavefront read consecutive, distinct words.
template <int BYTES>
__global__ void __launch_bounds__(PROBE_THREADS) lds_probe_kernel(uint32_t iters, uint32_t *out)
{
    __shared__ __align__(16) uint32_t buf[PROBE_BYTES / 4];
    const uint32_t tid = threadIdx.x;
    for (uint32_t w = tid; w < PROBE_BYTES / 4; w += PROBE_THREADS) buf[w] = w * 2654435761u + blockIdx.x;
    __syncthreads();
    const uint32_t lds0 = (uint32_t)(uintptr_t)buf;     // LDS byte address of buf
    uint32_t acc = tid;
    for (uint32_t i = 0; i < iters; ++i) {
        const uint32_t slot = (tid + 97u * i) & (PROBE_THREADS - 1);
        if constexpr (BYTES == 16) {
            acc ^= read8_b128(lds0 + slot * 16u);
            acc ^= read8_b128(lds0 + ((slot + 128u) & (PROBE_THREADS - 1)) * 16u);
        } else {
            acc ^= read8_b64(lds0 + slot * 8u);
            acc ^= read8_b64(lds0 + 16384u + slot * 8u);
        }
    }
    if (acc == 0x9e3779b9u) out[blockIdx.x] = acc;
}

} // namespace tapt

using namespace tapt;

extern "C" int pt_probe_lds(int32_t bytes_per_read, int32_t blocks_per_cu, uint32_t iters, double *tbps, double *ms)
{
    if ((bytes_per_read != 8 && bytes_per_read != 16) || blocks_per_cu < 1 || blocks_per_cu > 8 || iters < 1 ||
        !tbps)
        return PT_EINVAL;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PT_EDEVICE;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return PT_EDEVICE;
    const int blocks = cus * blocks_per_cu;
    uint32_t *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&out, (size_t)blocks * 4);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float t = 0.f;
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {   // the first launch warms up
        e = hipEventRecord(e0, nullptr);
        if (e != hipSuccess) break;
        if (bytes_per_read == 16)
            hipLaunchKernelGGL(lds_probe_kernel<16>, dim3(blocks), dim3(PROBE_THREADS), 0, nullptr, iters, out);
        else
            hipLaunchKernelGGL(lds_probe_kernel<8>, dim3(blocks), dim3(PROBE_THREADS), 0, nullptr, iters, out);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (out) (void)hipFree(out);
    if (e != hipSuccess) return PT_EDEVICE;
    const double bytes = (double)blocks * PROBE_THREADS * (double)iters * 16.0 * bytes_per_read;
    *tbps = bytes / (t * 1e-3) / 1e12;
    if (ms) *ms = t;
    return PT_OK;
}
