// Host-to-device copies of pageable host memory through pinned staging buffers.
#include <algorithm>
#include <cstring>

#include "plan.hpp"

namespace recoil {

namespace {

constexpr size_t kStageBytes = 16u << 20;   // per buffer; two per thread
constexpr size_t kDirectBytes = 256u << 10; // smaller copies go straight from pageable memory

struct Staging {
    void *buf[2] = {nullptr, nullptr};
    hipEvent_t done[2] = {nullptr, nullptr};
    bool pending[2] = {false, false};
    bool ready = false;

    hipError_t init() {
        if (ready) return hipSuccess;
        for (int i = 0; i < 2; ++i) {
            hipError_t e = hipHostMalloc(&buf[i], kStageBytes, hipHostMallocDefault);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&done[i], hipEventDisableTiming);
            if (e != hipSuccess) return e;
        }
        ready = true;
        return hipSuccess;
    }
    ~Staging() {
        for (int i = 0; i < 2; ++i) {
            if (done[i]) {
                (void)hipEventSynchronize(done[i]);
                (void)hipEventDestroy(done[i]);
            }
            if (buf[i]) (void)hipHostFree(buf[i]);
        }
    }
};

thread_local Staging t_staging;

}  // namespace

hipError_t stage_h2d(void *dst, const void *src, size_t bytes, hipStream_t stream) {
    if (bytes == 0) return hipSuccess;
    if (bytes <= kDirectBytes) return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream);
    Staging &st = t_staging;
    hipError_t e = st.init();
    if (e != hipSuccess) return e;
    const char *s = static_cast<const char *>(src);
    char *d = static_cast<char *>(dst);
    for (size_t off = 0, i = 0; off < bytes; off += kStageBytes, ++i) {
        const int k = (int)(i & 1);
        const size_t n = std::min(kStageBytes, bytes - off);
        if (st.pending[k]) {
            e = hipEventSynchronize(st.done[k]);   // the buffer's previous copy has left it
            if (e != hipSuccess) return e;
        }
        std::memcpy(st.buf[k], s + off, n);
        e = hipMemcpyAsync(d + off, st.buf[k], n, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipEventRecord(st.done[k], stream);
        if (e != hipSuccess) return e;
        st.pending[k] = true;
    }
    return hipSuccess;
}

}  // namespace recoil
