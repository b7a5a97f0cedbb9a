// Batched persistent Recoil decoding: thousands of independent streams (own
// tables, uint8 or uint16 symbols, W = 32 or 64) decoded by one launch.
//
// Host planning cuts every stream into work items (runs of consecutive unit
// pairs of one stream) and orders them largest stream first. Each persistent
// workgroup pops an item from a device counter, restages the decode table in
// LDS only when the item belongs to a different stream than its previous item,
// and its waves decode the item's pairs with the same per-pair decoder as the
// single-stream kernel. The queue head lives in device memory and is reset by
// a one-thread kernel launched just before, so the pair of launches can be
// captured in a HIP graph and replayed.
#include <algorithm>
#include <mutex>

#include "batch.hpp"
#include "decode_core.hpp"

namespace recoil {

// Queue heads of recoil_decode_batch_noalloc: one per table class, kStaticHeadStride
// words apart (one 128-byte line each). Every decode on a device shares its copy.
static __device__ __align__(256) uint32_t scratch[kStaticScratchWords];

namespace {

using namespace dev;

template <int W, typename Sym, int K, int SS = 64 / W, int VAR = kPlain>
__device__ inline void run_item(const DecodeParams &p, uint32_t lut, uint32_t ring0,
                                uint32_t lane, uint32_t wave, uint32_t waves, uint32_t first, uint32_t count) {
    PairDecoder<W, Sym, K, SS, VAR> d(p, lut, ring0, lane);
    const uint32_t share = wave < count ? (count - 1 - wave) / waves + 1 : 0u;
    uint32_t left = share;
    for (uint32_t q = first + wave; q < first + count; q += waves) d.run(q, --left, share);
}

// VAR: kPlain (one-level tables, n <= 12) or kWide (two-level, 13 <= n <= 16), one
// kernel each so that the wide decode does not weigh on the common one's registers.
template <int K, int WAVES, int VAR = kPlain>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_num_sgpr(RECOIL_SGPR_BUDGET), amdgpu_waves_per_eu(8, 8))) void decode_batch(
    BatchParams bp) {
    using L = Lds<16, K, WAVES>;
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned char *lut = smem + L::TABLE;
    const uint32_t base = lds_addr(smem);   // the first word of the pad holds the popped item
    const uint32_t wave = uni(threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t ring0 = base + L::PAD + wave * L::WAVE_LDS;
    int32_t cur = -1;
    for (;;) {
        if (threadIdx.x == 0) lds_st<uint32_t>(base, atomicAdd(bp.head, 1u));
        __syncthreads();
        const uint32_t it = uni(lds_ld<uint32_t>(base));
        if (it >= bp.n_items) break;
        const WorkItem wi = uni_load(bp.items + it);
        const StreamDesc d = uni_load(bp.streams + wi.stream);
        if ((int32_t)wi.stream != cur) {
            const uint32_t chunks = d.lut_chunks;
            const uint4 *src = reinterpret_cast<const uint4 *>(bp.ws + d.lut_off);
            for (uint32_t i = threadIdx.x; i < chunks; i += 64 * WAVES) reinterpret_cast<uint4 *>(lut)[i] = src[i];
            cur = (int32_t)wi.stream;
        }
        __syncthreads();
        DecodeParams p;
        p.words = reinterpret_cast<const uint16_t *>(bp.ws + d.words_off);
        p.lut = nullptr;
        p.counts = nullptr;
        p.tidx = nullptr;
        p.tables = 1;
        p.meta = reinterpret_cast<const UnitMeta *>(bp.ws + d.meta_off);
        p.lanes = reinterpret_cast<const uint32_t *>(bp.ws + d.lanes_off);
        p.out = bp.out + d.out_off;
        p.err = bp.err + wi.stream * bp.err_stride;
        p.n_symbols = d.n_symbols;
        p.units = d.units;
        const bool single = (wi.run & kItemSingle) != 0;
        const uint32_t run = wi.run & ~kItemSingle;
        p.run = run > 1 ? run : 1u;
        p.runs = (d.units + p.run - 1) / p.run;
        p.quant_bits = d.quant_bits;
        p.fill_symbol = d.fill_symbol;
        p.single_symbol = d.single_symbol;
        p.partitioned = d.partitioned;
        if (d.single_symbol) {
            for (uint64_t i = threadIdx.x; i < d.n_symbols; i += 64 * WAVES) {
                if (d.symbol_bytes == 1) static_cast<uint8_t *>(p.out)[i] = (uint8_t)d.fill_symbol;
                else static_cast<uint16_t *>(p.out)[i] = (uint16_t)d.fill_symbol;
            }
        } else if (d.lanes == 32) {
            if (single) {
                if (lane < 32) {   // one unit per wave: the upper half-wave idles until the item ends
                    if (d.symbol_bytes == 1) run_item<32, uint8_t, K, 1, VAR>(p, base + L::TABLE, ring0, lane, wave, WAVES, wi.first, wi.count);
                    else run_item<32, uint16_t, K, 1, VAR>(p, base + L::TABLE, ring0, lane, wave, WAVES, wi.first, wi.count);
                }
            } else if (d.symbol_bytes == 1) {
                run_item<32, uint8_t, K, 2, VAR>(p, base + L::TABLE, ring0, lane, wave, WAVES, wi.first, wi.count);
            } else {
                run_item<32, uint16_t, K, 2, VAR>(p, base + L::TABLE, ring0, lane, wave, WAVES, wi.first, wi.count);
            }
        } else {
            if (d.symbol_bytes == 1) run_item<64, uint8_t, K, 1, VAR>(p, base + L::TABLE, ring0, lane, wave, WAVES, wi.first, wi.count);
            else run_item<64, uint16_t, K, 1, VAR>(p, base + L::TABLE, ring0, lane, wave, WAVES, wi.first, wi.count);
        }
        if (bp.remaining) {
            // Publish the stream's completion once its last item is done: every
            // thread's stores reach device scope before the count drops, and the
            // finishing workgroup makes them system-visible before the flag.
            __threadfence();
            __syncthreads();
            if (threadIdx.x == 0 && atomicSub(bp.remaining + wi.stream, 1u) == 1u) {
                __threadfence_system();
                const uint32_t e = __hip_atomic_load(p.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(bp.host_done + wi.stream, kHostDone | e, __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_SYSTEM);
            }
        } else {
            __syncthreads();   // every wave is done with this table before the next item may replace it
        }
    }
}

__global__ void reset_head(uint32_t *head) {
    if (threadIdx.x == 0) *head = 0u;
}

template <int K, int WAVES>
size_t batch_lds(uint32_t lut_bytes) {
    return Lds<16, K, WAVES>::TABLE + lut_bytes;
}

template <int K, int WAVES, int VAR = kPlain>
int occupancy(uint32_t lut_bytes) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, decode_batch<K, WAVES, VAR>, 64 * WAVES,
                                                     batch_lds<K, WAVES>(lut_bytes)) != hipSuccess)
        return 0;
    return per_cu;
}

template <int K, int WAVES, int VAR>
hipError_t launch_var(const BatchParams &bp, uint32_t blocks_per_cu, hipStream_t stream) {
    const int cus = device_cus();
    int per_cu = occupancy<K, WAVES, VAR>(bp.lut_bytes);
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    if (blocks_per_cu > 0) per_cu = std::min<int>(per_cu, (int)blocks_per_cu);
    const uint32_t blocks = std::max<uint32_t>(1, std::min<uint32_t>(bp.n_items, (uint32_t)(cus * per_cu)));
    hipLaunchKernelGGL(reset_head, dim3(1), dim3(64), 0, stream, bp.head);
    const size_t lds = batch_lds<K, WAVES>(bp.lut_bytes);
    hipLaunchKernelGGL((decode_batch<K, WAVES, VAR>), dim3(blocks), dim3(64 * WAVES), lds, stream, bp);
    return hipGetLastError();
}

template <int K, int WAVES>
hipError_t launch(const BatchParams &bp, uint32_t blocks_per_cu, hipStream_t stream) {
    return bp.wide ? launch_var<K, WAVES, kWide>(bp, blocks_per_cu, stream)
                   : launch_var<K, WAVES, kPlain>(bp, blocks_per_cu, stream);
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t *g_scratch_ptr[kMaxDevices];

}  // namespace

hipError_t static_scratch(uint32_t **ptr) {
    *ptr = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        // The array's device address on this device; the host-side name is only a stand-in.
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = static_cast<uint32_t *>(p);
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

hipError_t launch_batch(const BatchParams &bp, const BatchTuning &t, hipStream_t stream) {
    if (bp.n_items == 0) return hipSuccess;
    if (t.chunk_groups == 4 && t.waves == 8) return launch<4, 8>(bp, t.blocks_per_cu, stream);
    if (t.chunk_groups == 4 && t.waves == 16) return launch<4, 16>(bp, t.blocks_per_cu, stream);
    if (t.chunk_groups == 8 && t.waves == 8) return launch<8, 8>(bp, t.blocks_per_cu, stream);
    if (t.chunk_groups == 8 && t.waves == 16) return launch<8, 16>(bp, t.blocks_per_cu, stream);
    return hipErrorInvalidValue;
}

int batch_blocks_per_cu(const BatchTuning &t, uint32_t lut_bytes, bool wide) {
    if (wide) {
        if (t.chunk_groups == 4 && t.waves == 8) return occupancy<4, 8, kWide>(lut_bytes);
        if (t.chunk_groups == 4 && t.waves == 16) return occupancy<4, 16, kWide>(lut_bytes);
        if (t.chunk_groups == 8 && t.waves == 8) return occupancy<8, 8, kWide>(lut_bytes);
        if (t.chunk_groups == 8 && t.waves == 16) return occupancy<8, 16, kWide>(lut_bytes);
        return 0;
    }
    if (t.chunk_groups == 4 && t.waves == 8) return occupancy<4, 8>(lut_bytes);
    if (t.chunk_groups == 4 && t.waves == 16) return occupancy<4, 16>(lut_bytes);
    if (t.chunk_groups == 8 && t.waves == 8) return occupancy<8, 8>(lut_bytes);
    if (t.chunk_groups == 8 && t.waves == 16) return occupancy<8, 16>(lut_bytes);
    return 0;
}

}  // namespace recoil
