// Host-side building blocks shared by the plain, batched and rollout entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/cloth.h"
#include "cloth_internal.h"

namespace cloth {

// Sets the calling thread's last-error message and returns code.
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);
extern thread_local std::string g_last_error;

// Waits for a stream when it goes out of scope.  The runtime may perform a copy from or to
// pageable host memory after hipMemcpyAsync has returned (when the stream still has work
// queued ahead of it), so a host buffer must outlive every copy that uses it.  Declared
// after such buffers, a fence is destroyed before them on every return path, error returns
// included.
struct StreamFence {
    hipStream_t stream;
    StreamFence(const StreamFence&) = delete;
    StreamFence& operator=(const StreamFence&) = delete;
    ~StreamFence() { (void)hipStreamSynchronize(stream); }
};

// Device allocations owned by one handle, released together.
struct DeviceArena {
    std::vector<void*> ptrs;
    DeviceArena() = default;
    DeviceArena(const DeviceArena&) = delete;
    DeviceArena& operator=(const DeviceArena&) = delete;
    ~DeviceArena();
    void release();
    hipError_t alloc_bytes(void** p, size_t bytes);
    template <class T>
    hipError_t alloc(T** p, size_t n) {
        void* q = nullptr;
        hipError_t e = alloc_bytes(&q, n * sizeof(T));
        *p = static_cast<T*>(q);
        return e;
    }
    void free_one(void* p);
};

// The cloth_create arguments of one cloth (borrowed host pointers).
struct ClothHostInput {
    int nx, ny;
    const float* x0;
    const float* v0;
    const float* mass;
    const unsigned char* pinned;
    int n_springs;
    const int* ends;
    const float* rest;
    const float* k;
    const float* c;
    int n_verts;
    const float* verts;
    int n_tris;
    const int* tris;
};

// Host copies of one cloth in internal node order (see ClothView for the layout).
struct ClothHost {
    int n = 0, ld = 0;
    std::vector<int> order, slot;  // order[slot] = node id; slot[node id] = internal slot
    std::vector<float> x, v, w;
    std::vector<int> deg, slice_ptr, nbr, inc_spring;
    // the distinct (k, c, rest length) triples of each cloth and each spring's entry
    // (param_table); tab_span: the most entries any one cloth has
    std::vector<float4> ptab;
    std::vector<int> spring_entry;
    int tab_span = 0;
    // The state copies are only needed for the upload; the incidence lists stay for
    // rebuilding tile plans.
    void release_state() {
        std::vector<float>().swap(x);
        std::vector<float>().swap(v);
    }
};

struct ClothDevice {
    int n = 0, ld = 0;
    float* x[2] = {nullptr, nullptr};
    float* v[2] = {nullptr, nullptr};
    int cur = 0;
    float* w = nullptr;
    int* deg = nullptr;
    int* slice_ptr = nullptr;
    uint2* inc2 = nullptr;
    int* inc_spring = nullptr;
    float4* ptab = nullptr;       // room for one entry per spring (at least one)
    int* spring_entry = nullptr;  // [springs]: re-points the records after a parameter update
    int n_springs = 0;
    int* n_tab = nullptr;         // [1]: the most entries one cloth has in ptab (stencil kernel)
    // grid stencil (build_stencil), when every cloth of the handle has one
    int n_tiles = 0;
    int4 one_cloth{};                // the cloth of a one-cloth handle (GridView::one)
    int4* tiles = nullptr;           // [n_tiles] per-tile cloth (batches), else NULL
    int* sten_code = nullptr;        // [kStencilDirs][ld] spring or -1
    uint32_t* sten_idx = nullptr;    // [kStencilDirs][ld] ptab entry or kNoSpring
    uint32_t* sten_idx8 = nullptr;   // [kStencilDirs / 4][ld] the entries as bytes, relative
                                     // to the cloth's first (GridView)
    int* tab_base = nullptr;         // [cloths] first ptab entry of each cloth (batches), else NULL
    const int* slot_cloth = nullptr; // [ld] cloth of each slot (batches), else NULL
    GridView grid_view() const;
    ClothView view() const;
};

// Device copy of a tile plan (build_tile_plan) and its schedule (build_schedule).
struct TilePlanDevice {
    DeviceArena arena;
    DeviceArena sched_arena;
    std::vector<TileMeta> meta_host;
    int schedule = -1, sched_workgroups = 0;
    int tile_nodes = 0, K = 0;
    TileView view{};
    int* inc_sid = nullptr;  // spring id per incidence entry (-1 = padding)
    size_t inc_count = 0;
    size_t bytes = 0;
    long long computed_per_launch_first = 0;  // nodes computed in the first substep of a launch
};

struct SurfaceDevice {
    SurfaceView view{};
    double cell = 0.0;
    long long n_cells = 0, n_refs = 0;
    int n_verts = 0;
    // build buffers, kept for rebuilds (capacities in elements)
    float* verts = nullptr;
    int* tris = nullptr;
    unsigned long long* total = nullptr;
    float4 *box_lo = nullptr, *box_hi = nullptr, *geo = nullptr, *tri_v = nullptr;
    uint32_t *counts = nullptr, *cell_start = nullptr, *tmp = nullptr, *refs = nullptr;
    float4 *ref_lo = nullptr, *ref_hi = nullptr;
    uint4* ref_q = nullptr;
    size_t cap_cells = 0, cap_refs = 0;
    bool dirty = false;  // a rebuild started rewriting the arrays and has not completed
};

std::vector<int> tile_order(int nx, int ny);
// The 8x8 tiles of an nx-by-ny grid as (column, row) tile coordinates, in slot order
// (row by row).
std::vector<std::pair<int, int>> tile_list(int nx, int ny);
// One cloth of a handle, for build_stencil: grid shape, first node id, first internal slot,
// first spring and spring count.
struct StencilCloth {
    int nx, ny, node_off, slot_off, spring_off, n_springs;
};
bool build_stencil(const std::vector<StencilCloth>& cloths, const std::vector<int>& ends,
                   const std::vector<int>& slot, int ld, std::vector<int>* code,
                   std::vector<int4>* tiles);
int validate_cloth(const ClothHostInput& in);
int validate_params(const cloth_params* p);
void stability_bounds(const ClothHostInput& in, double* omega2, double* gamma);
bool unstable(double omega2, double gamma, double h);
// order: internal slot -> node id; NULL = the 8x8-tile Morton order of (nx, ny).  segs: the
// first spring of each cloth of a merged input, then the spring count (NULL = one cloth).
int build_cloth_host(const ClothHostInput& in, ClothHost* out,
                     const std::vector<int>* order = nullptr,
                     const std::vector<int>* segs = nullptr);
int upload_cloth(const ClothHost& h, DeviceArena& arena, hipStream_t stream, ClothDevice* d);
// The distinct (k, c, rest length) triples of S springs, compared by their exact FP32 bits,
// in order of first occurrence, and each spring's entry in that table.  The triples are
// distinct per segment of springs (segs: each segment's first spring, then S; NULL or empty =
// one segment), so each segment's entries are one contiguous range starting at the entry of
// its first spring; *span gets the largest range.
void param_table(const float* k, const float* c, const float* rest, int S,
                 const std::vector<int>* segs, std::vector<float4>* tab,
                 std::vector<int>* entry, int* span);
// First entry of each segment (the entry of its first spring; 0 for a segment without
// springs).
std::vector<int> segment_bases(const std::vector<int>& segs, const std::vector<int>& entry);
// Upload a parameter table and the springs' entries, then re-point the cloth's incidence
// records (and the tile plan's records, if rec/sid are given) at them; synchronises.
// span: the most entries one segment (cloth) has; bases: each cloth's first entry, uploaded
// to d->tab_base when the handle has one.
int upload_param_table(const std::vector<float4>& tab, const std::vector<int>& entry, int span,
                       const std::vector<int>& bases, ClothDevice* d, size_t n_inc,
                       uint2* plan_rec, const int* plan_sid, size_t n_plan, hipStream_t stream);
int build_surface(const ClothHostInput& in, const cloth_params& p, DeviceArena& arena,
                  hipStream_t stream, SurfaceDevice* sd);
// Rebuild the grid and every per-triangle array for new vertex positions [n_verts][3] (host)
// of the same triangles; synchronises the stream once (to size the reference array).
int rebuild_surface(SurfaceDevice* sd, const float* verts, DeviceArena& arena,
                    hipStream_t stream);
int build_tile_plan(const ClothHost& h, const std::vector<int>& group_off, int tile_nodes, int K,
                    hipStream_t stream, TilePlanDevice* out);
int build_schedule(TilePlanDevice* plan, int mode, int n_workgroups, hipStream_t stream);

}  // namespace cloth
