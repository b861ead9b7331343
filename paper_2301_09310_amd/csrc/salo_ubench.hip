// Ceiling microbenchmarks for gfx950 (a separate library, libsalo_ubench.so,
// loaded only by the benchmark): the sustained VALU rate of the two integer
// forms the DP kernels use, and the HBM copy bandwidth.
//
//  * packed 16-bit: v_pk_add_u16 / v_pk_max_u16 on independent chains, two
//    16-bit elements per lane per instruction;
//  * 32-bit: v_add_u32 / v_max_i32 on independent chains;
//  * copy: a streaming device-to-device copy in 16-byte vector loads and
//    stores (bytes read plus bytes written per second).
//
// The measured rates are the peaks the DP kernels' roofline fractions can be
// read against, beside the nominal 256 CUs x 64 lanes x 2.4 GHz.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

constexpr int kChains = 16;
constexpr int kUnroll = 8;

// Every lane runs kChains independent chains of (add, max) pairs; the
// operands come from the kernel arguments so nothing folds at compile time.
__global__ __launch_bounds__(256) void valu_pk16(uint32_t *sink, int iters, uint32_t a,
                                                 uint32_t b) {
    u16x2 x[kChains];
    const u16x2 va = __builtin_bit_cast(u16x2, a), vb = __builtin_bit_cast(u16x2, b);
#pragma unroll
    for (int c = 0; c < kChains; ++c)
        x[c] = __builtin_bit_cast(u16x2, (uint32_t)(threadIdx.x * 7 + c));
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
            for (int c = 0; c < kChains; ++c) {
                x[c] = x[c] + va;
                x[c] = __builtin_elementwise_max(x[c], vb);
            }
        }
    }
    uint32_t acc = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc ^= __builtin_bit_cast(uint32_t, x[c]);
    if (acc == 0x12345678u) sink[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

__global__ __launch_bounds__(256) void valu_i32(uint32_t *sink, int iters, int a, int b) {
    int x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = (int)threadIdx.x * 7 + c;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
            for (int c = 0; c < kChains; ++c) {
                x[c] = x[c] + a;
                x[c] = max(x[c], b);
            }
        }
    }
    int acc = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc ^= x[c];
    if (acc == 0x12345678) sink[blockIdx.x * blockDim.x + threadIdx.x] = (uint32_t)acc;
}

__global__ __launch_bounds__(256) void copy16(const uint4 *__restrict__ src,
                                              uint4 *__restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] = src[i];
}

}  // namespace

extern "C" {

// kind 0: packed 16-bit VALU; 1: 32-bit VALU -- `work` is the loop count per
// lane, *out_units the element-operations executed.  kind 2: copy of `work`
// bytes (a multiple of 16) between two device buffers allocated here --
// *out_units the bytes read plus written.  *out_ms: the mean duration of
// `reps` launches after one warm-up, from HIP events on the null stream.
// Returns 0, or a HIP error code.
int salo_ubench(int kind, int64_t work, int reps, double *out_ms, double *out_units) {
    if (!out_ms || !out_units || reps < 1 || work < 1) return (int)hipErrorInvalidValue;
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return (int)e;
    const int threads = 256;
    const int blocks = cus * 8;              // 32 waves per CU
    uint32_t *sink = nullptr;
    void *src = nullptr, *dst = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int64_t n16 = work / 16;
    e = hipMalloc(&sink, sizeof(uint32_t) * blocks * threads);
    if (e == hipSuccess && kind == 2) {
        if (n16 < 1) e = hipErrorInvalidValue;
        if (e == hipSuccess) e = hipMalloc(&src, (size_t)n16 * 16);
        if (e == hipSuccess) e = hipMalloc(&dst, (size_t)n16 * 16);
        if (e == hipSuccess) e = hipMemset(src, 1, (size_t)n16 * 16);
    }
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    auto launch = [&]() -> hipError_t {
        if (kind == 0)
            hipLaunchKernelGGL(valu_pk16, dim3(blocks), dim3(threads), 0, 0, sink, (int)work,
                               0x00010001u, 0x00030003u);
        else if (kind == 1)
            hipLaunchKernelGGL(valu_i32, dim3(blocks), dim3(threads), 0, 0, sink, (int)work, 1,
                               3);
        else
            hipLaunchKernelGGL(copy16, dim3(cus * 16), dim3(threads), 0, 0,
                               static_cast<const uint4 *>(src), static_cast<uint4 *>(dst), n16);
        return hipGetLastError();
    };
    if (e == hipSuccess && kind != 0 && kind != 1 && kind != 2) e = hipErrorInvalidValue;
    if (e == hipSuccess && (kind == 0 || kind == 1) && work > (1 << 24)) e = hipErrorInvalidValue;
    if (e == hipSuccess) e = launch();                 // warm-up
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipEventRecord(e0, 0);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e1, 0);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess) {
        *out_ms = (double)ms / reps;
        const double lanes = (double)blocks * threads;
        if (kind == 0)       // two packed instructions per chain step, 2 elements each
            *out_units = lanes * (double)work * kUnroll * kChains * 2.0 * 2.0;
        else if (kind == 1)  // two instructions per chain step
            *out_units = lanes * (double)work * kUnroll * kChains * 2.0;
        else
            *out_units = 2.0 * (double)n16 * 16.0;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (sink) (void)hipFree(sink);
    if (src) (void)hipFree(src);
    if (dst) (void)hipFree(dst);
    return (int)e;
}

}  // extern "C"
