// cloth_debug_candidates_noalloc: the broad-phase candidate query of cloth_debug_candidates
// with every device buffer it needs (the points, their candidate counts and offsets, the
// scan's partial sums and the pairs) carved out of one fixed, file-scope device array
// instead of allocated per call, for callers that cannot allocate device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "sim.h"

namespace cloth {
namespace {

// The call's device memory.  Each GPU the library runs on holds its own copy until the
// process ends; every call on that GPU uses it, so calls that overlap on one GPU race.
constexpr size_t kScratchBytes = 8u << 20;
constexpr int kNoallocMaxPoints = 1 << 16;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` per device, looked up once per device with that device
// current (the array's host-side name is only a stand-in for it).
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

hipError_t scratch_for_current_device(unsigned char** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_addr[dev] = p;
    }
    *out = static_cast<unsigned char*>(g_scratch_addr[dev]);
    return hipSuccess;
}

constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// AoS [n][3] points -> SoA [3][n].
__global__ void k_points_soa(int n, const float* __restrict__ aos, float* __restrict__ soa) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    soa[i] = aos[3 * (size_t)i];
    soa[n + i] = aos[3 * (size_t)i + 1];
    soa[2 * (size_t)n + i] = aos[3 * (size_t)i + 2];
}

// Where each buffer of a call over n points sits in the scratch array (byte offsets); the
// pairs take the rest.
struct Layout {
    size_t aos, soa, counts, offsets, scan, pairs, pair_capacity;
};
Layout layout(size_t n) {
    Layout L{};
    size_t at = 0;
    L.aos = at;
    at += align256(12 * n);
    L.soa = at;
    at += align256(12 * n);
    L.counts = at;
    at += align256(4 * n);
    L.offsets = at;
    at += align256(4 * (n + 1));
    L.scan = at;
    at += align256(4 * scan_tmp_words(n));
    L.pairs = at;
    L.pair_capacity = at < kScratchBytes ? (kScratchBytes - at) / 8 : 0;
    return L;
}

}  // namespace
}  // namespace cloth

using namespace cloth;

extern "C" {

int cloth_debug_candidates_noalloc(cloth_sim* s, int n_points, const float* points,
                                   int* pairs_out, long long cap, long long* n_out) {
    if (!s || !n_out) return fail(CLOTH_EINVAL, "NULL argument");
    if (n_points < 0 || cap < 0) return fail(CLOTH_EINVAL, "negative size");
    if (n_points > 0 && !points) return fail(CLOTH_EINVAL, "points is NULL");
    if (cap > 0 && !pairs_out) return fail(CLOTH_EINVAL, "pairs_out is NULL");
    const SurfaceView& sv = s->surfs[0].view;
    if (sv.n_tris == 0) return fail(CLOTH_EINVAL, "collision is disabled for this handle");
    if (s->surface_broken) return fail(CLOTH_ESTATE, "a surface update failed; update it again first");
    *n_out = 0;
    if (n_points > kNoallocMaxPoints)
        return fail(CLOTH_ENOMEM, "at most 65536 points per call (fixed device scratch)");
    if (n_points == 0) return CLOTH_OK;
    unsigned char* base = nullptr;
    hipError_t e = scratch_for_current_device(&base);
    if (e != hipSuccess) return hip_fail(e, "scratch address");
    const size_t n = (size_t)n_points;
    const Layout L = layout(n);
    float* d_aos = reinterpret_cast<float*>(base + L.aos);
    float* d_soa = reinterpret_cast<float*>(base + L.soa);
    uint32_t* d_cnt = reinterpret_cast<uint32_t*>(base + L.counts);
    uint32_t* d_off = reinterpret_cast<uint32_t*>(base + L.offsets);
    uint32_t* d_scan = reinterpret_cast<uint32_t*>(base + L.scan);
    int* d_pairs = reinterpret_cast<int*>(base + L.pairs);
    uint32_t total = 0;
    StreamFence fence{s->stream};
    // every count is written by the count pass and every offset by the scan, so nothing in
    // the scratch needs clearing between calls
    if ((e = hipMemcpyAsync(d_aos, points, 12 * n, hipMemcpyHostToDevice, s->stream)))
        return hip_fail(e, "copy points");
    k_points_soa<<<(unsigned)((n + 255) / 256), 256, 0, s->stream>>>(n_points, d_aos, d_soa);
    if ((e = hipGetLastError()) ||
        (e = launch_candidates_count(n_points, n_points, d_soa, sv, s->launch.hit_slots, d_cnt,
                                     s->stream)) ||
        (e = scan_exclusive_u32(d_cnt, d_off, n, d_scan, s->stream)) ||
        (e = hipMemcpyAsync(&total, d_off + n, 4, hipMemcpyDeviceToHost, s->stream)) ||
        (e = hipStreamSynchronize(s->stream)))
        return hip_fail(e, "candidate count");
    *n_out = total;
    if (total == 0 || cap == 0) return CLOTH_OK;
    if (total > L.pair_capacity)
        return fail(CLOTH_ENOMEM, "more candidate pairs than the fixed device scratch holds");
    const size_t ncopy = (size_t)std::min<long long>(cap, total);
    if ((e = launch_candidates_write(n_points, n_points, d_soa, sv, s->launch.hit_slots, d_off,
                                     d_pairs, s->stream)) ||
        (e = hipMemcpyAsync(pairs_out, d_pairs, 8 * ncopy, hipMemcpyDeviceToHost, s->stream)) ||
        (e = hipStreamSynchronize(s->stream)))
        return hip_fail(e, "candidate write");
    return CLOTH_OK;
}

}  // extern "C"
