// Stand-in HIP runtime for running the library's host code under AddressSanitizer and
// UndefinedBehaviorSanitizer on a machine without a GPU.
//
// Device memory is host memory.  Copies and fills are not performed when they are enqueued:
// they wait in a queue until the program synchronises (a stream, an event, or a free), as
// the HIP runtime may do with copies from or to pageable host memory that are queued behind
// other work on a stream.  A host buffer that the library releases before its copy has run
// is therefore read or written after it was freed, which AddressSanitizer reports.
// Kernel launches do nothing; the one whose result the host reads back (the reference count
// of a surface grid) writes zero.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>
#include <deque>

#include "../../paper_2507_11794_amd/csrc/cloth_internal.h"

namespace {

struct Op {
    void* dst;
    const void* src;  // nullptr: a fill with `value`
    size_t bytes;
    int value;
};
std::deque<Op> g_ops;

void drain() {
    while (!g_ops.empty()) {
        const Op o = g_ops.front();
        g_ops.pop_front();
        if (o.src)
            std::memcpy(o.dst, o.src, o.bytes);
        else
            std::memset(o.dst, o.value, o.bytes);
    }
}

struct Handle {
    int tag;
};

}  // namespace

extern "C" {

hipError_t hipMalloc(void** p, size_t n) {
    *p = std::calloc(1, n ? n : 1);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* p) {
    drain();  // the runtime's free waits for the device
    std::free(p);
    return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t n, unsigned int) {
    *p = std::calloc(1, n ? n : 1);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipHostFree(void* p) {
    drain();
    std::free(p);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t) {
    if (bytes) g_ops.push_back(Op{dst, src, bytes, 0});
    return hipSuccess;
}
hipError_t hipMemsetAsync(void* dst, int value, size_t bytes, hipStream_t) {
    if (bytes) g_ops.push_back(Op{dst, nullptr, bytes, value});
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) {
    drain();
    return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) {
    *s = reinterpret_cast<hipStream_t>(new Handle{1});
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    delete reinterpret_cast<Handle*>(s);
    return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipSuccess; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) {
    *g = reinterpret_cast<hipGraph_t>(new Handle{2});
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t, hipGraphNode_t*, char*, size_t) {
    *e = reinterpret_cast<hipGraphExec_t>(new Handle{3});
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
    delete reinterpret_cast<Handle*>(g);
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t e) {
    delete reinterpret_cast<Handle*>(e);
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t) {
    return reinterpret_cast<Handle*>(e)->tag == 3 ? hipSuccess : hipErrorInvalidValue;
}
hipError_t hipGetLastError(void) { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) {
    *e = reinterpret_cast<hipEvent_t>(new Handle{4});
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) {
    drain();
    return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
    static float t = 1.0f;
    *ms = (t += 0.125f);  // later candidates look slower: the first one wins
    return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
    delete reinterpret_cast<Handle*>(e);
    return hipSuccess;
}
hipError_t hipGetDevice(int* d) {
    *d = 0;
    return hipSuccess;
}
hipError_t hipGetDevicePropertiesR0600(hipDeviceProp_t* prop, int) {
    std::memset(prop, 0, sizeof(*prop));
    std::strcpy(prop->gcnArchName, "gfx950 stub");
    prop->multiProcessorCount = 256;
    return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t, int) {
    *v = 256;
    return hipSuccess;
}
const char* hipGetErrorString(hipError_t) { return "stub error"; }

}  // extern "C"

// Kernel launchers of the HIP sources: no device work.
namespace cloth {

hipError_t prepare_substep_kernels(size_t) { return hipSuccess; }
hipError_t prepare_tile_kernels(size_t) { return hipSuccess; }
hipError_t prepare_scatter_kernels(size_t) { return hipSuccess; }
hipError_t launch_tiles(const TileView&, int, int, const StepParams&, const float*, const float*,
                        float*, float*, int, int, hipStream_t) {
    return hipSuccess;
}
hipError_t launch_substep(const ClothView&, int, const StepParams&, const float*, const float*,
                          float*, float*, int, hipStream_t, const SurfaceView*, const int*, int,
                          int, int, int*, int, float*) {
    return hipSuccess;
}
hipError_t launch_scatter_substep(const ClothView&, const SpringList&, int, int,
                                  const StepParams&, float*, const float*, const float*, float*,
                                  float*, int, hipStream_t, const SurfaceView*, const int*, int,
                                  int) {
    return hipSuccess;
}
hipError_t launch_mt_substep(const ClothView&, const StepParams&, const MtTopology&,
                             const SurfaceView*, const float*, const float*, float*, float*,
                             float*, int, hipStream_t) {
    return hipSuccess;
}
hipError_t launch_mt_debug_contacts(const ClothView&, const StepParams&, const MtTopology&,
                                    const SurfaceView*, const float*, const float*, float*, int*,
                                    int*, int, hipStream_t) {
    return hipSuccess;
}
hipError_t launch_adj_node(const ClothView&, const SurfaceView&, const StepParams&, const float*,
                           const float*, const float*, const float*, float*, float*, float*, int,
                           const float*, hipStream_t) {
    return hipSuccess;
}
hipError_t launch_adj_fused(const ClothView&, const SurfaceView&, const StepParams&, const float*,
                            const float*, const float*, const float*, const float*, const float*,
                            float*, float*, float*, float*, float*, double*, double*,
                            const float*, const int*, int, hipStream_t) {
    return hipSuccess;
}
hipError_t launch_adj_springs(const ClothView&, const float*, const float*, const float*,
                              const float*, const float*, float*, float*, double*, double*,
                              hipStream_t) {
    return hipSuccess;
}
hipError_t launch_debug_contacts(const ClothView&, const SurfaceView&, const StepParams&,
                                 const float*, const float*, int*, int*, int, int, hipStream_t) {
    return hipSuccess;
}
hipError_t launch_debug_volume(const ClothView&, const SurfaceView&, const StepParams&,
                               const float*, const float*, int, uint32_t*, uint32_t*,
                               unsigned long long*, hipStream_t) {
    return hipSuccess;
}
hipError_t launch_substep_lanes(int, const ClothView&, int, const StepParams&, const float*,
                                const float*, float*, float*, int, hipStream_t,
                                const SurfaceView*, const int*, int, int, float*) {
    return hipSuccess;
}
size_t lanes_lds_bytes(int block, int hit_slots) {
    return (size_t)(block / 64) * ((size_t)(hit_slots + 1) * 256 + 5 * 1024);
}
hipError_t prepare_lanes_kernels(size_t) { return hipSuccess; }
hipError_t launch_grid_substep(const ClothView&, const GridView&, int, const StepParams&,
                               const float*, const float*, float*, float*, hipStream_t,
                               const SurfaceView*, int, int, int, int, float*) {
    return hipSuccess;
}
hipError_t prepare_grid_kernels(size_t) { return hipSuccess; }
size_t grid_lds_bytes(int hit_slots) { return (size_t)(hit_slots + 1) * 256; }
hipError_t launch_set_stencil_entries(int, const int*, const int*, const int*, const int*,
                                      uint32_t*, uint32_t*, hipStream_t) {
    return hipSuccess;
}
hipError_t launch_import(int, int, const int*, const float*, float*, int, hipStream_t) {
    return hipSuccess;
}
hipError_t launch_export(int, int, const int*, const float*, float*, hipStream_t) {
    return hipSuccess;
}
hipError_t launch_set_params(size_t, const int*, const float*, const float*, float*, float*,
                             hipStream_t) {
    return hipSuccess;
}
hipError_t launch_set_entries(size_t, const int*, int, const int*, uint2*, hipStream_t) {
    return hipSuccess;
}
hipError_t launch_d2f(size_t, const double*, float*, hipStream_t) { return hipSuccess; }
hipError_t launch_vertex_normals(int, int, const float*, const int*, const int*, const int*,
                                 const int4*, float*, hipStream_t) {
    return hipSuccess;
}
hipError_t launch_tri_prep(int, const float*, const int*, float, const float*, float, const int*,
                           float4*, float4*, float4*, float4*, unsigned long long* total,
                           hipStream_t stream) {
    return hipMemsetAsync(total, 0, sizeof(*total), stream);  // no grid references
}
hipError_t launch_grid_count(int, const float4*, const float4*, const float*, float, const int*,
                             uint32_t*, hipStream_t) {
    return hipSuccess;
}
hipError_t launch_grid_fill(int, const float4*, const float4*, const float*, float, const int*,
                            const uint32_t*, uint32_t*, uint32_t*, hipStream_t) {
    return hipSuccess;
}
hipError_t launch_grid_finish(int, const float*, float, const int*, const uint32_t*, uint32_t*,
                              const float4*, const float4*, float4*, float4*, uint4*,
                              hipStream_t) {
    return hipSuccess;
}
hipError_t scan_exclusive_u32(const uint32_t*, uint32_t* out, size_t n, uint32_t*,
                              hipStream_t stream) {
    return hipMemsetAsync(out, 0, 4 * (n + 1), stream);  // all cells empty
}
hipError_t launch_candidates_count(int, int, const float*, const SurfaceView&, int, uint32_t*,
                                   hipStream_t) {
    return hipSuccess;
}
hipError_t launch_candidates_write(int, int, const float*, const SurfaceView&, int,
                                   const uint32_t*, int*, hipStream_t) {
    return hipSuccess;
}

}  // namespace cloth
