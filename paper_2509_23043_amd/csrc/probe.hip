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

// VALU issue-rate probe: eight independent chains per lane of one
// instruction (asm, so that the compiler neither folds nor reorders them);
// the kernel's wave-instructions per cycle per CU give the instruction's rate
// relative to the 64 lanes-per-clock of a full-rate 32-bit operation.
__global__ void __launch_bounds__(256) valu_probe_kernel(int op, uint32_t iters, uint32_t *out)
{
    uint32_t a0 = threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4, a5 = a0 + 5, a6 = a0 + 6,
             a7 = a0 + 7;
    const uint32_t c = 0xD2511F53u + blockIdx.x;
    if (op == 0) {
        for (uint32_t i = 0; i < iters; ++i) {
            asm volatile("v_xor_b32 %0, %8, %0\n v_xor_b32 %1, %8, %1\n v_xor_b32 %2, %8, %2\n v_xor_b32 %3, %8, %3\n"
                         "v_xor_b32 %4, %8, %4\n v_xor_b32 %5, %8, %5\n v_xor_b32 %6, %8, %6\n v_xor_b32 %7, %8, %7"
                         : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)
                         : "v"(c));
        }
    } else if (op == 1) {
        for (uint32_t i = 0; i < iters; ++i) {
            asm volatile("v_mul_hi_u32 %0, %8, %0\n v_mul_hi_u32 %1, %8, %1\n v_mul_hi_u32 %2, %8, %2\n"
                         "v_mul_hi_u32 %3, %8, %3\n v_mul_hi_u32 %4, %8, %4\n v_mul_hi_u32 %5, %8, %5\n"
                         "v_mul_hi_u32 %6, %8, %6\n v_mul_hi_u32 %7, %8, %7"
                         : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)
                         : "v"(c));
        }
    } else if (op == 3) {
        // four independent 32x32 -> 64 multiply-add chains (the Philox round's
        // instruction); eight instructions per iteration as for the others
        uint64_t b0 = a0, b1 = a1, b2 = a2, b3 = a3;
        uint64_t cy0, cy1, cy2, cy3;
        for (uint32_t i = 0; i < iters; ++i) {
            asm volatile("v_mad_u64_u32 %0, %4, %8, %9, %0\n v_mad_u64_u32 %1, %5, %8, %9, %1\n"
                         "v_mad_u64_u32 %2, %6, %8, %9, %2\n v_mad_u64_u32 %3, %7, %8, %9, %3\n"
                         "v_mad_u64_u32 %0, %4, %8, %9, %0\n v_mad_u64_u32 %1, %5, %8, %9, %1\n"
                         "v_mad_u64_u32 %2, %6, %8, %9, %2\n v_mad_u64_u32 %3, %7, %8, %9, %3"
                         : "+v"(b0), "+v"(b1), "+v"(b2), "+v"(b3), "=s"(cy0), "=s"(cy1), "=s"(cy2), "=s"(cy3)
                         : "v"(c), "v"(a4));
        }
        a0 = (uint32_t)b0 ^ (uint32_t)(b0 >> 32);
        a1 = (uint32_t)b1 ^ (uint32_t)(b1 >> 32);
        a2 = (uint32_t)b2 ^ (uint32_t)(b2 >> 32);
        a3 = (uint32_t)b3 ^ (uint32_t)(b3 >> 32);
        a4 = a5 = a6 = a7 = 0;
    } else {
        for (uint32_t i = 0; i < iters; ++i) {
            asm volatile("v_mul_lo_u32 %0, %8, %0\n v_mul_lo_u32 %1, %8, %1\n v_mul_lo_u32 %2, %8, %2\n"
                         "v_mul_lo_u32 %3, %8, %3\n v_mul_lo_u32 %4, %8, %4\n v_mul_lo_u32 %5, %8, %5\n"
                         "v_mul_lo_u32 %6, %8, %6\n v_mul_lo_u32 %7, %8, %7"
                         : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)
                         : "v"(c));
        }
    }
    const uint32_t x = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;
    if (x == 0x9e3779b9u) out[blockIdx.x] = x;
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

extern "C" int pt_probe_valu(int32_t op, uint32_t iters, double *instr_per_clk_per_cu, double *ms)
{
    if (op < 0 || op > 3 || iters < 1 || !instr_per_clk_per_cu) return PT_EINVAL;
    int dev = 0, cus = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PT_EDEVICE;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return PT_EDEVICE;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeClockRate, dev) != hipSuccess) return PT_EDEVICE;
    const int blocks = cus * 8;                // 32 waves per CU: 8 per SIMD
    uint32_t *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&out, (size_t)blocks * 4);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float t = 0.f;
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
        e = hipEventRecord(e0, nullptr);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(valu_probe_kernel, dim3(blocks), dim3(256), 0, nullptr, (int)op, iters, out);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (out) (void)hipFree(out);
    if (e != hipSuccess) return PT_EDEVICE;
    // wave-instructions issued: blocks x 4 waves x iters x 8; clocks: t x clock rate
    const double instrs = (double)blocks * 4.0 * (double)iters * 8.0;
    const double clocks = (double)t * 1e-3 * (double)khz * 1e3;
    *instr_per_clk_per_cu = instrs / clocks / (double)cus;
    if (ms) *ms = t;
    return PT_OK;
}
