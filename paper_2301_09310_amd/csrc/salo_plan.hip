// Planning kernels of the persistent mode: length bins, sort keys and a
// counting sort that orders pairs so that every unit of work holds pairs of
// near-equal shape, heaviest first.
//
// Why: pair lengths in a batch vary by an order of magnitude and work grows
// with the product of the two lengths (SALoBa, Section III-A), so a wave
// that takes pairs in input order waits for its longest pair.  Binning by
// query length picks the lane-group width per bin (the subwarp trade-off of
// Section IV-C); sorting within a bin by chunk count and target length makes
// the pairs that share a wave (and a packed register) nearly equal.
//
// Steps (all device-side, no host synchronisation):
//   plan_zero        clear the histograms and the per-bin statistics
//   plan_bins        per pair: bin; per bin: count and target length range
//                    (reduced per block in LDS before one global update)
//   plan_keys        per pair: 16-bit key = bin | relative chunk count | length code,
//                    counted in sub-histogram blockIdx % kSubHist
//   plan_scan_*      exclusive scan of all sub-histograms in descending key
//                    order (block sums, their scan, then the cursors) and
//                    the per-bin unit table
//   plan_scatter     order[cursor[key][sub]++] = pair
#include "salo_internal.h"

namespace salo {
namespace {

constexpr int kTpb = 256;          // threads per block of the per-pair kernels
constexpr int kScanThreads = 1024;

struct PairLen {
    int64_t m, n;
};

__device__ __forceinline__ PairLen pair_len(const KParams &P, int64_t p) {
    const int64_t q0 = P.q_off[p], t0 = P.t_off[p];
    const int64_t m = P.q_off[p + 1] - q0;
    const int64_t n = P.t_off[p + 1] - t0;
    const bool valid = m >= 0 && n >= 0 && m <= SALO_MAX_LEN_DEV && n <= SALO_MAX_LEN_DEV &&
                       q0 >= 0 && t0 >= 0;
    if (!valid) return {0, 0};
    if (P.in_qstart) {
        // trace pass: the span from the answer's start to its end
        const int32_t sc = P.in_score[p], qe = P.in_qend[p], te = P.in_tend[p];
        const int32_t qs = P.in_qstart[p], ts = P.in_tstart[p];
        if (sc <= 0 || qs < 0 || qs > qe || qe >= m || ts < 0 || ts > te || te >= n)
            return {0, 0};
        return {(int64_t)qe - qs + 1, (int64_t)te - ts + 1};
    }
    if (P.in_score) {
        // start pass: the reversed prefixes ending at the forward answer
        const int32_t sc = P.in_score[p], qe = P.in_qend[p], te = P.in_tend[p];
        if (sc <= 0 || qe < 0 || qe >= m || te < 0 || te >= n) return {0, 0};
        return {(int64_t)qe + 1, (int64_t)te + 1};
    }
    return {m, n};
}

__device__ __forceinline__ bool pair_packed(const KParams &P, int64_t m, int64_t n) {
    if (!P.packed_ok || P.force_int32) return false;
    return packed_bound_ok(P.match, P.mismatch, m < n ? m : n);
}

// First bin of the pair's kind (16- or 32-bit) whose query range holds m
// and whose lane-group width keeps the boundary columns of a whole unit in
// one slot (n rows, or the banded ring, x 64/W groups x 2 words); else the
// last bin of the kind.
__device__ __forceinline__ int pair_bin(const KParams &P, const BinTable &bt, int64_t m,
                                        int64_t n) {
    const int want = pair_packed(P, m, n) ? 1 : 0;
    if (P.band >= 0) {
        uint32_t wrap = 0;
        n = band_slot_rows((int)n, P.band, &wrap);
    }
    int last = 0;
    for (int b = 0; b < bt.n_bins; ++b) {
        if (bt.packed[b] != want) continue;
        last = b;
        const int64_t row_cap = (int64_t)P.slot_words * bt.lanes[b] / (2 * 64);
        if (m <= bt.m_hi[b] && n <= row_cap) return b;
    }
    return last;
}

// position of (key, sub) in the scan order: descending key, ascending sub
__device__ __forceinline__ int64_t hist_index(uint32_t key, int sub) {
    return (int64_t)(kKeys - 1 - key) * kSubHist + sub;
}

__global__ void plan_zero(PlanBuffers pb, int32_t *counters) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kHistEntries / 4)
        reinterpret_cast<uint4 *>(pb.hist)[i] = make_uint4(0u, 0u, 0u, 0u);
    if (i < kMaxBins) {
        pb.binstat[3 * i + 0] = 0;
        pb.binstat[3 * i + 1] = 0x7FFFFFFF;
        pb.binstat[3 * i + 2] = 0;
    }
    if (i < kCounterWords) counters[i] = 0;
}

__global__ __launch_bounds__(kTpb) void plan_bins(KParams P, BinTable bt, PlanBuffers pb) {
    __shared__ int32_t s_cnt[kMaxBins], s_min[kMaxBins], s_max[kMaxBins];
    const int t = threadIdx.x;
    if (t < kMaxBins) {
        s_cnt[t] = 0;
        s_min[t] = 0x7FFFFFFF;
        s_max[t] = 0;
    }
    __syncthreads();
    constexpr int kPer = 8;
    const int64_t base = (int64_t)blockIdx.x * kTpb * kPer + t;
    for (int k = 0; k < kPer; ++k) {
        const int64_t p = base + (int64_t)k * kTpb;
        if (p >= P.n_pairs) break;
        const PairLen L = pair_len(P, p);
        const int b = pair_bin(P, bt, L.m, L.n);
        atomicAdd(&s_cnt[b], 1);
        atomicMin(&s_min[b], (int32_t)L.n);
        atomicMax(&s_max[b], (int32_t)L.n);
    }
    __syncthreads();
    if (t < kMaxBins && s_cnt[t] > 0) {
        atomicAdd(&pb.binstat[3 * t + 0], s_cnt[t]);
        atomicMin(&pb.binstat[3 * t + 1], s_min[t]);
        atomicMax(&pb.binstat[3 * t + 2], s_max[t]);
    }
}

__global__ __launch_bounds__(kTpb) void plan_keys(KParams P, BinTable bt, PlanBuffers pb) {
    const int64_t p = (int64_t)blockIdx.x * kTpb + threadIdx.x;
    if (p >= P.n_pairs) return;
    const PairLen L = pair_len(P, p);
    const int b = pair_bin(P, bt, L.m, L.n);
    const int64_t width = (int64_t)bt.lanes[b] * bt.cols[b];
    const int64_t c_min = (bt.m_lo[b] + width) / width;   // chunks of the bin's shortest query
    int64_t c = (L.m + width - 1) / width - c_min;
    c = c < 0 ? 0 : (c > 15 ? 15 : c);
    const int32_t nmin = pb.binstat[3 * b + 1], nmax = pb.binstat[3 * b + 2];
    const int64_t span = (int64_t)nmax - nmin + 1;
    int64_t nc = span > 0 ? ((L.n - nmin) * 256) / span : 0;
    nc = nc < 0 ? 0 : (nc > 255 ? 255 : nc);
    const uint32_t key = ((uint32_t)b << 12) | ((uint32_t)c << 8) | (uint32_t)nc;
    pb.keys[p] = (uint16_t)key;
    atomicAdd(&pb.hist[hist_index(key, blockIdx.x % kSubHist)], 1u);
}

// block-wide exclusive scan of one value per thread (kScanThreads threads)
__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *part) {
    const int t = threadIdx.x;
    part[t] = v;
    __syncthreads();
    for (int o = 1; o < kScanThreads; o <<= 1) {
        const uint32_t x = t >= o ? part[t - o] : 0u;
        __syncthreads();
        part[t] += x;
        __syncthreads();
    }
    const uint32_t incl = part[t];
    __syncthreads();
    return incl - v;
}

// sums of kScanBlock consecutive histogram entries
__global__ __launch_bounds__(kScanThreads) void plan_scan_sums(PlanBuffers pb) {
    __shared__ uint32_t part[kScanThreads];
    const uint4 *h = reinterpret_cast<const uint4 *>(pb.hist + (int64_t)blockIdx.x * kScanBlock);
    const uint4 v = h[threadIdx.x];
    part[threadIdx.x] = v.x + v.y + v.z + v.w;
    __syncthreads();
    for (int o = kScanThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) pb.block_sums[blockIdx.x] = part[0];
}

// exclusive scan of the block sums, then the bin table
__global__ __launch_bounds__(kScanThreads) void plan_scan_top(KParams P, BinTable bt,
                                                              PlanBuffers pb) {
    __shared__ uint32_t part[kScanThreads];
    static_assert(kScanBlocks % kScanThreads == 0, "scan geometry");
    constexpr int per = kScanBlocks / kScanThreads;
    const int t = threadIdx.x;
    uint32_t loc[per];
    uint32_t sum = 0;
    for (int k = 0; k < per; ++k) {
        loc[k] = pb.block_sums[t * per + k];
        sum += loc[k];
    }
    uint32_t run = block_exclusive_scan(sum, part);
    for (int k = 0; k < per; ++k) {
        pb.block_sums[t * per + k] = run;
        run += loc[k];
    }
    if (t == 0) {
        // bins appear in descending index order in the sorted list; units
        // are numbered within each bin's column class
        int32_t first = 0, unit0[kColClasses] = {0, 0, 0, 0};
        for (int b = kMaxBins - 1; b >= 0; --b) {
            BinDesc d;
            const bool on = b < bt.n_bins;
            d.lanes = on ? bt.lanes[b] : 64;
            d.cols = on ? bt.cols[b] : 16;
            d.packed = on ? bt.packed[b] : 1;
            d.pairs = 2 * (64 / d.lanes);
            d.count = on ? pb.binstat[3 * b + 0] : 0;
            d.first = first;
            d.units = (d.count + d.pairs - 1) / d.pairs;
            d.split = on ? bt.split[b] : 0;
            const int kc = bin_class(d.cols, d.split);
            d.unit0 = unit0[kc];
            d.n_min = on ? pb.binstat[3 * b + 1] : 0;
            d.n_max = on ? pb.binstat[3 * b + 2] : 0;
            first += d.count;
            unit0[kc] += d.units;
            P.bins[b] = d;
        }
        for (int kc = 0; kc < kColClasses; ++kc) {
            P.total_units[kc] = unit0[kc];
            P.unit_counter[kc] = 0;
        }
    }
}

// cursors: block offset + exclusive scan within the block
__global__ __launch_bounds__(kScanThreads) void plan_scan_apply(PlanBuffers pb) {
    __shared__ uint32_t part[kScanThreads];
    uint4 *h = reinterpret_cast<uint4 *>(pb.hist + (int64_t)blockIdx.x * kScanBlock);
    const uint4 v = h[threadIdx.x];
    const uint32_t s = v.x + v.y + v.z + v.w;
    const uint32_t run = pb.block_sums[blockIdx.x] + block_exclusive_scan(s, part);
    h[threadIdx.x] = make_uint4(run, run + v.x, run + v.x + v.y, run + v.x + v.y + v.z);
}

__global__ __launch_bounds__(kTpb) void plan_scatter(KParams P, PlanBuffers pb) {
    const int64_t p = (int64_t)blockIdx.x * kTpb + threadIdx.x;
    if (p >= P.n_pairs) return;
    const uint32_t pos = atomicAdd(&pb.hist[hist_index(pb.keys[p], blockIdx.x % kSubHist)], 1u);
    if (pos < (uint64_t)P.n_pairs) pb.order[pos] = (int32_t)p;   // always, for consistent counts
}

}  // namespace

hipError_t launch_plan(const KParams &p, const BinTable &bt, const PlanBuffers &pb,
                       hipStream_t stream) {
    const int64_t nb = (p.n_pairs + kTpb - 1) / kTpb;
    const int64_t nb8 = (p.n_pairs + kTpb * 8 - 1) / (kTpb * 8);
    const int64_t zero_blocks = (kHistEntries / 4 + kTpb - 1) / kTpb;
    hipLaunchKernelGGL(plan_zero, dim3((unsigned)zero_blocks), dim3(kTpb), 0, stream, pb,
                       p.unit_counter);
    hipLaunchKernelGGL(plan_bins, dim3((unsigned)nb8), dim3(kTpb), 0, stream, p, bt, pb);
    hipLaunchKernelGGL(plan_keys, dim3((unsigned)nb), dim3(kTpb), 0, stream, p, bt, pb);
    hipLaunchKernelGGL(plan_scan_sums, dim3(kScanBlocks), dim3(kScanThreads), 0, stream, pb);
    hipLaunchKernelGGL(plan_scan_top, dim3(1), dim3(kScanThreads), 0, stream, p, bt, pb);
    hipLaunchKernelGGL(plan_scan_apply, dim3(kScanBlocks), dim3(kScanThreads), 0, stream, pb);
    hipLaunchKernelGGL(plan_scatter, dim3((unsigned)nb), dim3(kTpb), 0, stream, p, pb);
    return hipGetLastError();
}

}  // namespace salo
