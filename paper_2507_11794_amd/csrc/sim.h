// The simulation handle shared by the plain, rollout, batch and autotune entry points
// (private).  One handle holds one or more independent cloths ("groups"): node slots
// [group_off[g], group_off[g+1]) belong to cloth g, each cloth has its own surface grid, and
// no spring or tile crosses two cloths.  A plain handle is a batch of one.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/cloth.h"
#include "cloth_internal.h"
#include "host_common.h"

namespace cloth {

// Spring list and force accumulator of the spring-centric (scatter) kernels.
struct SpringDevice {
    DeviceArena arena;
    SpringList view{};
    int* sid = nullptr;  // caller spring id of each list entry
    float* k = nullptr;
    float* c = nullptr;
    float* F = nullptr;  // [3][ld], zero between substeps
    bool ready = false;
};

struct GraphEntry {
    unsigned h_bits;
    int K, chunk, parity;
    long long plan_version;
    hipGraphExec_t exec;
};

// Differentiable-rollout buffers (cloth_rollout_forward / cloth_rollout_backward).
struct RolloutState {
    DeviceArena arena;
    bool ready = false;  // a forward pass whose checkpoints are still valid
    float h = 0.0f;
    long long n_sub = 0;             // substeps of the forward pass
    long long ckpt = 0;              // substeps between checkpoints
    std::vector<long long> out_sub;  // substep index of each recorded output
    float* ck = nullptr;             // checkpoints: [n_ck][6][ld] (x then v)
    long long n_ck = 0;
    float* seg = nullptr;    // one segment of states: [ckpt + 1][6][ld]
    float* pred = nullptr;   // the segment's predictions before collision: [ckpt][3][ld]
    float* adj = nullptr;    // xb, vb, fb[2], (unused), xb_part, vb_part: 7 x [3][ld]
    double* kb = nullptr;    // [S]
    double* cb = nullptr;    // [S]
};

// Per-cloth bookkeeping of a handle.
struct GroupInfo {
    int nx = 0, ny = 0;
    int node_off = 0;    // first node id (caller numbering) of this cloth in the handle
    int slot_off = 0;    // first internal slot
    int n = 0;           // nodes
    int n_springs = 0;
    int spring_off = 0;  // first spring of this cloth in the handle's spring list
    double omega2 = 0.0, gamma = 0.0;  // stability bounds
};

}  // namespace cloth

struct cloth_sim {
    cloth_params p{};
    hipStream_t stream = nullptr;
    hipStream_t capture = nullptr;  // private stream used only for graph capture
    int n_nodes = 0, n_springs = 0;
    std::vector<cloth::GroupInfo> groups;
    std::vector<int> group_off;  // slot offsets, groups.size() + 1 entries
    cloth::ClothHost host;
    cloth::ClothDevice dev;
    std::vector<cloth::SurfaceDevice> surfs;  // per group
    cloth::SurfaceView* svs_dev = nullptr;    // per group, on the device
    int* node_group_dev = nullptr;            // per slot (batches only)
    int any_collision = 0;
    cloth::DeviceArena arena;
    cloth::TilePlanDevice plan;
    cloth::SpringDevice springs;
    long long plan_version = 0;
    std::vector<cloth::GraphEntry> graphs;
    cloth_launch launch{CLOTH_KERNEL_DIRECT, 256, 1, 64, 1, CLOTH_SCHED_GRID, 0, 32, 0, 0};
    int* heavy_dev = nullptr;  // the second pass's counters and node lists (first use)
    bool launch_ready = false;  // plan, schedule and LDS limits match `launch`
    int* nan_flag = nullptr;
    // host copies kept for the stability bound and parameter updates (caller numbering)
    std::vector<float> x0, mass, k, c, rest;
    std::vector<unsigned char> pinned;
    std::vector<int> ends;
    // device: initial state (SoA, internal order) and node id -> internal slot
    float* x_init = nullptr;
    float* v_init = nullptr;
    int* slot_dev = nullptr;
    // allocated by the first normals call: slot -> node id, per-cloth (node_off, nx, ny, 0)
    int* order_dev = nullptr;
    int4* group_desc_dev = nullptr;
    // external forces (SoA [3][ld], internal slots), allocated by the first set call
    float* fext_dev = nullptr;
    bool fext_on = false;
    bool surface_broken = false;
    bool mt = false;             // triangle-triangle narrow phase (CLOTH_F_NARROW_MT)
    float* mt_pred = nullptr;    // its prediction scratch, [6][ld]  // a surface rebuild failed part-way: stepping is refused
    cloth::RolloutState roll;
    // read-back staging, allocated by the first read of the state (the handle is used by one
    // thread at a time): device AoS x then v of the largest cloth in node-id order, and its
    // pinned host copy followed by the status flag
    mutable float* export_dev = nullptr;
    mutable float* export_host = nullptr;

    void drop_graphs() {
        for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
        graphs.clear();
    }
    ~cloth_sim() {
        (void)hipStreamSynchronize(stream);
        drop_graphs();
        if (capture) (void)hipStreamDestroy(capture);
        if (export_dev) (void)hipFree(export_dev);
        if (export_host) (void)hipHostFree(export_host);
    }
};

// A batch handle is a multi-cloth simulation handle.
struct cloth_batch {
    cloth_sim* sim = nullptr;
};

namespace cloth {

// Build a handle holding the given cloths (validated), on `stream`.
int create_sim(const std::vector<ClothHostInput>& cloths, const cloth_params* p,
               hipStream_t stream, cloth_sim** out);
int check_launch(const cloth_launch& c);
// Make sure the tile plan and its schedule match the launch configuration.
int ensure_plan(cloth_sim* s, const cloth_launch& c);
// Build the spring list and force accumulator of the scatter kernels (once).
int ensure_springs(cloth_sim* s);
// Apply a launch configuration (validates, replans, drops stale graphs).
int set_launch(cloth_sim* s, const cloth_launch& c);
// Advance `total` substeps of length h with the handle's launch configuration.
int run_substeps(cloth_sim* s, float h, long long total);
// Validates dt / counts and the stability bound of every cloth, then runs.
int step_sim(cloth_sim* s, float dt, int n_substeps, int n_steps);
// Recompute the stability bounds from the handle's host copies.
void refresh_stability(cloth_sim* s);
// Copy the state of slots [slot_off, slot_off + n) to the host in caller numbering
// (node id - node_off).
int read_state_range(const cloth_sim* s, int group, float* x_out, float* v_out);
// New vertex positions for cloth `group`'s surface (same triangles): rebuilds its grid.
int update_surface(cloth_sim* s, int group, const float* verts, int n_verts);
// First spring of each cloth of the handle, then the spring count (param_table's segments).
std::vector<int> spring_segments(const cloth_sim* s);
// Per-node external forces [n_nodes][3] in caller numbering (NULL removes them).
int set_external_force(cloth_sim* s, const float* f);
// Device tables of the cloth-grid topology (node order, per-cloth sizes), made once.
int ensure_topology(cloth_sim* s);
// Substeps one launch of the current configuration advances.
int substeps_per_launch(const cloth_sim* s);
// Per-vertex normals of the current state of every cloth into n_out (device, AoS, caller
// numbering), on the handle's stream.
int vertex_normals(cloth_sim* s, float* n_out);
// Measured search over launch configurations (autotune.cpp).
int autotune_sim(cloth_sim* s, float dt, int n_substeps, int frames, cloth_launch* best);

}  // namespace cloth
