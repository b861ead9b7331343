// salo_align_batch_noalloc: salo_align_batch for callers that cannot
// allocate device memory (code under HIP graph capture, serving loops that
// must not call hipMalloc, harnesses that forbid it).  Every workspace
// buffer of the persistent path -- counters, bin table, plan buffers and
// the chunk-boundary slots -- is carved from one file-scope device array,
// `scratch`, that each GPU holds from the library's load to the end of the
// process.  The kernels are the same as salo_align_batch's.
#include <mutex>

#include "salo.h"
#include "salo_internal.h"

namespace {

// At most 4,194,304 pairs per call; 3,072 boundary slots (256 CUs x 12
// resident waves) of 96 KiB, so one pair group's column holds 12,288 target
// rows (longer targets are flagged invalid: score, q_end and t_end -1).
constexpr int64_t kNoAllocMaxPairs = int64_t(1) << 22;
constexpr int64_t kNoAllocSlots = 3072;
constexpr int32_t kNoAllocSlotWords = 96 * 1024 / 4;
constexpr int64_t kNoAllocBytes =
    salo::fixed_scratch_bytes(kNoAllocMaxPairs, kNoAllocSlots, kNoAllocSlotWords);

static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

// The array's device address on each GPU, looked up once per device (the
// name `scratch` in host code is a host-side stand-in, not that address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

extern "C" salo_status_t salo_align_batch_noalloc(const uint8_t *q_seqs,
                                                  const int64_t *q_offsets,
                                                  const uint8_t *t_seqs,
                                                  const int64_t *t_offsets, int64_t n_pairs,
                                                  salo_scoring_t scoring, int32_t *out_score,
                                                  int32_t *out_qend, int32_t *out_tend,
                                                  hipStream_t stream) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return salo::set_error(SALO_ERR_HIP, "hipGetDevice failed");
    if (dev < 0 || dev >= kMaxDevices)
        return salo::set_error(SALO_ERR_UNSUPPORTED, "device index above 63");
    void *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            void *p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p)
                return salo::set_error(SALO_ERR_HIP, "hipGetSymbolAddress(scratch) failed");
            g_scratch_ptr[dev] = p;
        }
        ptr = g_scratch_ptr[dev];
    }
    return salo::align_batch_fixed_scratch(q_seqs, q_offsets, t_seqs, t_offsets, n_pairs,
                                           scoring, out_score, out_qend, out_tend, stream, ptr,
                                           kNoAllocBytes, kNoAllocMaxPairs, kNoAllocSlots,
                                           kNoAllocSlotWords);
}
