// Internal declarations shared by the host API (api.cpp) and the HIP kernel sources.
// Not part of the public ABI (include/cloth.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cloth {

// Static collision surface and its uniform grid, as the kernels see them.
//   cell of a point p: c_a = clamp(floor((p_a - org_a) * inv_cell), 0, dim_a - 1) per axis,
//   linear id (c_z * dim_y + c_y) * dim_x + c_x; refs[cell_start[c] .. cell_start[c+1]) are
//   the triangles whose inflated box overlaps cell c, in ascending triangle id.
struct SurfaceView {
    int n_tris;                  // 0 = collision disabled
    float org[3];
    float inv_cell;
    int dim[3];
    float thickness;
    float thickness2;            // thickness^2
    const uint32_t* cell_start;  // [cells + 1]
    const uint32_t* refs;        // [refs]
    const float4* ref_lo;        // [refs]: inflated box of refs[r]; .w = triangle id (int bits)
    const float4* ref_hi;        // [refs]: .w unused
    const uint4* ref_q;          // [refs]: the box coded against its cell (ref_code), and
                                 // the triangle id in .w
    const float4* box_lo;        // [T] inflated box, .w unused
    const float4* box_hi;        // [T]
    const float4* geo;           // [T*3]: (A, n.x), (B-A, n.y), (C-A, n.z); n = unit outward normal
    const float4* tri_v;         // [T*3]: the vertices (x, y, z, vertex id as int bits)
};

// One cloth's node and spring arrays on the device (internal node order).
//   State is SoA: x[k*ld + i].
//   Incidences use a sliced CSR layout: nodes are grouped in slices of 64 (one wavefront),
//   and the r-th incidence of node i (r < deg[i]) sits at slice_ptr[i/64] + r*64 + i%64, so
//   the 64 lanes of a wavefront read incidence r with one coalesced access.  Per incidence:
//   inc2 = (neighbour node, entry of the spring's parameters in ptab), one 8-byte record,
//   and inc_spring (spring id, bitwise-negated (~s) when node i is the spring's second end
//   b).  ptab holds the distinct (k, c, rest length) triples of the springs (a cloth has a
//   few spring types, so the table stays in cache; after per-spring parameters are set it
//   may hold one entry per spring).  Each node's incidences are in ascending (neighbour
//   node id, spring) order.
struct ClothView {
    int n;
    int ld;  // SoA leading dimension (>= n)
    const float* w;  // [n] inverse mass, 0 = pinned
    const int* deg;        // [n]
    const int* slice_ptr;  // [ceil(n/64) + 1]
    const uint2* inc2;
    const float4* ptab;  // (k, c, rest length, 0)
    const int* inc_spring;
};

// Grid stencil of cloths whose springs join only nodes at the offsets (row, column)
// (-2,0) (-1,-1) (-1,0) (-1,1) (0,-2) (0,-1) (0,1) (0,2) (1,-1) (1,0) (1,1) (2,0), in that
// order (ascending neighbour id, the order of every node's incidence list), one spring per
// node and offset at most.  The stencil kernel runs one wavefront per 8x8 tile of the
// internal order (tiles row by row, nodes row-major in a tile).  A cloth is described by
// (first slot, nx | ny << 16, first tile, cloth index): `one` for a handle of one cloth,
// tiles[t] per tile for a batch.  Each cloth's entries in the parameter table are one
// contiguous range starting at tab_base[cloth] (0 for a one-cloth handle).  idx[d * ld + p]
// is the table entry of the spring from slot p in direction d, or kNoSpring; while no cloth
// has more than kSmallTab entries, byte d % 4 of idx8[(d / 4) * ld + p] holds the same entry
// relative to its cloth's first (kNoSpring8 for none), a quarter of the bytes.  n_tab points
// at the largest number of entries of one cloth (kept on the device so captured graphs stay
// valid when parameters change); tab_cap is the table's capacity.
constexpr int kStencilDirs = 12;
constexpr uint32_t kNoSpring = 0xffffffffu;
constexpr uint32_t kNoSpring8 = 0xffu;
constexpr int kSmallTab = 255;
struct GridView {
    int n_tiles;
    int4 one;
    const int4* tiles;
    const uint32_t* idx;
    const uint32_t* idx8;
    const int* n_tab;
    int tab_cap;
    const int* tab_base;  // [cloths] first table entry of each cloth (batches), else NULL
};

// Springs for the spring-centric (scatter) force pass: ends as internal slots, parameters
// per spring, ordered by (min slot, max slot) for locality.
struct SpringList {
    int n;
    const int* a;
    const int* b;
    const float* k;
    const float* c;
    const float* L0;
};

struct StepParams {
    float h;
    float g[3];
    float restitution;
    int check_nan;
    int* nan_flag;
    const float* fext;  // external forces, SoA [3][fext_ld] by internal slot; NULL = none
    int fext_ld;
};

// Temporally blocked tiles.  The internal node order is cut into tiles of consecutive
// slots; one workgroup owns a tile and the region of nodes within K spring hops of it,
// ordered by hop level (level 0 = the tile, ascending slot within a level).  level[k] counts
// the nodes within k hops, so substep s of a launch recomputes the prefix [0, level[K - s])
// in LDS and only the tile itself is written back after K substeps.  Computed nodes
// (u < level[K - 1]) carry their incidences in region-local form: inc[inc_off + r * inc_pad
// + u] = (k, c, rest length, local neighbour index as int bits), in the same order as the
// node's global incidence list, so the arithmetic matches the one-substep kernel bit for bit.
constexpr int kMaxTileK = 8;

struct TileMeta {
    int group;       // cloth of a batch (index into TileView::svs)
    int region_off;  // into region_slot
    int region_n;    // = level[K_plan]
    int comp_off;    // into comp_deg
    int inc_off;     // float4 offset into inc
    int inc_pad;     // multiple of 64, >= level[K_plan - 1]
    int level[kMaxTileK + 1];
};

struct TileView {
    int n_tiles;
    int rmax;  // largest region (LDS sizing)
    int ld;    // global SoA leading dimension
    int n_workgroups;      // grid size of the schedule
    const int* item_ptr;   // [n_workgroups + 1]: workgroup b runs items[item_ptr[b]..item_ptr[b+1])
    const int* items;      // tile ids
    const SurfaceView* svs;  // [groups] surface of each cloth
    const TileMeta* meta;
    const int* region_slot;
    const int* comp_deg;
    const uint2* inc;     // (neighbour's region index, parameter entry)
    const float4* ptab;   // the cloth's parameter table (ClothView::ptab)
    const float* w;  // inverse mass by global slot
};

// K substeps (K <= the plan's K) of every tile; reads (xs, vs), writes (xd, vd).
// collide = 0 skips the collision stage for every cloth (no cloth has a surface).
hipError_t launch_tiles(const TileView& tv, int K, int collide, const StepParams& sp,
                        const float* xs, const float* vs, float* xd, float* vd, int block,
                        int hit_slots, hipStream_t stream);
// LDS of one tile workgroup: the region state plus the collision stage of its wavefronts.
size_t tile_lds_bytes(int rmax, int block = 256, int hit_slots = 0);
// Raise the tile kernels' dynamic LDS limit when a plan needs more than 64 KiB.
hipError_t prepare_tile_kernels(size_t lds_bytes);

// a1-a4: one substep for every node (one thread per node).  collide = 0 skips a3/a4.  The
// surfaces are read on the device: node i's is svs[node_group[i]] with node_group non-NULL
// (a batch of cloths), otherwise svs[0].  hit_slots: length of each lane's LDS list of box
// hits in the collision query (0 = no list: hits are resolved per round of references; at
// most kMaxHitSlots).  Reference boxes are tested kRefRound per round of loads.
constexpr int kMaxHitSlots = 64;
constexpr int kMaxXcdRuns = 4096;
constexpr int kRefRound = 8;
constexpr int kHitRound = 8;  // box hits whose geometry is loaded per round

// Grid size of a one-thread-per-node launch of n_logical workgroups under xcd_runs (see
// xcd_block): padded to a multiple of 8 * xcd_runs when xcd_runs >= 2.
inline int xcd_grid(int n_logical, int xcd_runs) {
    if (xcd_runs < 2) return n_logical;
    const long long c = 8LL * xcd_runs;
    return (int)((n_logical + c - 1) / c * c);
}
// A lane's hit list holds hit_slots entries plus one scratch entry that takes the writes of
// references that are not hits (so the box loop appends without a branch); the lists of a
// wavefront's 64 lanes are interleaved, list_stride(hit_slots) words per wavefront.
constexpr int list_stride(int hit_slots) { return hit_slots > 0 ? (hit_slots + 1) * 64 : 0; }
// LDS bytes one wavefront's collision query uses for its lanes' hit lists.
constexpr size_t wave_query_lds(int hit_slots) { return (size_t)list_stride(hit_slots) * 4; }
// xcd_runs: the workgroup-to-XCD mapping (see xcd_block; 0 = the hardware's order).
// pred: if non-NULL, receives every node's prediction before collision (SoA, ld).
// split_refs > 0: nodes whose cell lists more than split_refs references are resolved by a
// second launch with four lanes per node (launch_heavy).  heavy holds two counters, then two
// node lists of ld entries at kHeavyListOff; the first pass appends to list `parity`, the
// second pass reads it and clears the other parity's counter for the next substep, so
// consecutive substeps (alternating buffers) alternate lists.  Both counters must be zero when
// the scheme starts (heavy_words() ints in all).
constexpr int kHeavyListOff = 64;
constexpr size_t heavy_words(int ld) { return kHeavyListOff + 2 * (size_t)ld; }
hipError_t launch_substep(const ClothView& cv, int collide, const StepParams& sp, const float* xs,
                          const float* vs, float* xd, float* vd, int block, hipStream_t stream,
                          const SurfaceView* svs, const int* node_group = nullptr,
                          int hit_slots = 0, int xcd_runs = 0, int split_refs = 0,
                          int* heavy = nullptr, int parity = 0, float* pred = nullptr);
// launch_substep with `lanes` (2 or 4) lanes per node (lanes_step.hip): the same results,
// bit for bit; no second pass.
// launch_substep through the grid stencil (grid_step.hip): one wavefront per 8x8 tile stages
// the tile and a two-node halo in LDS and sums each node's springs from there, in the
// incidence order; the same results, bit for bit.  waves = 2 (with collision) adds a second
// wavefront per tile that takes every other round of the box hits' narrow tests (same
// results); without collision one wavefront is launched either way.
hipError_t launch_grid_substep(const ClothView& cv, const GridView& gv, int collide,
                               const StepParams& sp, const float* xs, const float* vs, float* xd,
                               float* vd, hipStream_t stream, const SurfaceView* svs,
                               int grouped, int hit_slots, int xcd_runs, int waves,
                               float* pred = nullptr);
hipError_t prepare_grid_kernels(size_t lds_bytes);
// Dynamic LDS of a stencil launch (the hit lists of each tile's first wavefront, the only
// one that lists hits).
size_t grid_lds_bytes(int hit_slots);
// Stencil parameter entries from per-spring entries: idx[q] = entry[code[q]], or kNoSpring
// where code[q] < 0, and their byte form in idx8 (q = d * ld + p, see GridView), relative to
// tab_base[slot_cloth[p]] when both are given.
hipError_t launch_set_stencil_entries(int ld, const int* code, const int* entry,
                                      const int* slot_cloth, const int* tab_base, uint32_t* idx,
                                      uint32_t* idx8, hipStream_t st);
hipError_t launch_substep_lanes(int lanes, const ClothView& cv, int collide, const StepParams& sp,
                                const float* xs, const float* vs, float* xd, float* vd, int block,
                                hipStream_t stream, const SurfaceView* svs, const int* node_group,
                                int hit_slots, int xcd_runs, float* pred = nullptr);
hipError_t prepare_lanes_kernels(size_t lds_bytes);
// Dynamic LDS of a lanes launch: hit lists and contact records of its wavefronts.
size_t lanes_lds_bytes(int block, int hit_slots);
// The second pass over list `parity` of heavy (see launch_substep): each listed node's
// prediction is in (xd, vd) and is replaced by the collision-resolved state.
hipError_t launch_heavy(const ClothView& cv, const StepParams& sp, int* heavy, int parity,
                        float* xd, float* vd, const SurfaceView* svs, const int* node_group,
                        hipStream_t st);
// Raise the one-substep kernel's dynamic LDS limit when its stage needs more than 64 KiB.
hipError_t prepare_substep_kernels(size_t lds_bytes);
// One substep with spring-centric forces: the spring pass accumulates into F (SoA [3][ld],
// FP32 or, with fix, int32 at 2^-24 N; all zero on entry), then the node pass integrates,
// collides (as launch_substep) and zeroes F.  Fixed-point overflow sets bit 2 of
// sp.nan_flag.
hipError_t launch_scatter_substep(const ClothView& cv, const SpringList& sl, int fix, int collide,
                                  const StepParams& sp, float* F, const float* xs,
                                  const float* vs, float* xd, float* vd, int block,
                                  hipStream_t st, const SurfaceView* svs, const int* node_group,
                                  int hit_slots, int xcd_runs);
hipError_t prepare_scatter_kernels(size_t lds_bytes);

// Cloth-grid topology for the triangle-triangle narrow phase: order[slot] = node id,
// slot[node id], node_group[slot] (NULL for one cloth), groups[g] = (node_off, nx, ny, 0).
struct MtTopology {
    const int* order;
    const int* slot;
    const int* node_group;
    const int4* groups;
};
// One substep with the triangle-triangle narrow phase: prediction into P ([6][ld]: x*, v*),
// then the contact search and the averaged response into xd, vd.
hipError_t launch_mt_substep(const ClothView& cv, const StepParams& sp, const MtTopology& tp,
                             const SurfaceView* svs, const float* xs, const float* vs, float* P,
                             float* xd, float* vd, int block, hipStream_t st);
// The contact sets that substep would use: counts[slot], up to cap ids per slot (in the
// kernel's candidate order).
hipError_t launch_mt_debug_contacts(const ClothView& cv, const StepParams& sp,
                                    const MtTopology& tp, const SurfaceView* svs, const float* xs,
                                    const float* vs, float* P, int* counts, int* ids, int cap,
                                    hipStream_t st);

// --- a6 adjoint ----------------------------------------------------------------------------
// Response and integration transpose of one substep at state (xs, vs): partial adjoints and
// the force adjoint fb = h w vtot (see adjoint.hip).
// hit_slots: the contact search's LDS list (0 = unlisted search); pred: the forward
// prediction stored by launch_substep, or NULL to recompute it.  The results are the same.
hipError_t launch_adj_node(const ClothView& cv, const SurfaceView& sv, const StepParams& sp,
                           const float* xs, const float* vs, const float* xb_out,
                           const float* vb_out, float* fb, float* xb_part, float* vb_part,
                           int hit_slots, const float* pred, hipStream_t st);
// Spring-force transpose: xb_in / vb_in = partial + spring terms; adds dL/dk, dL/dc.
// The spring pass of substep t and the node pass of substep t - 1 in one launch (see
// k_adj_fused); gout: an output's loss adjoint added between them, or NULL.
hipError_t launch_adj_fused(const ClothView& cv, const SurfaceView& sv, const StepParams& sp,
                            const float* xs_a, const float* vs_a, const float* xs_b,
                            const float* vs_b, const float* pred_b, const float* fb_t,
                            float* fb_prev, float* xb_part, float* vb_part, float* xb, float* vb,
                            double* kb, double* cb, const float* gout, const int* order,
                            int hit_slots, hipStream_t st);
hipError_t launch_adj_springs(const ClothView& cv, const float* xs, const float* vs,
                              const float* fb, const float* xb_part, const float* vb_part,
                              float* xb_in, float* vb_in, double* kb, double* cb, hipStream_t st);
// Contact sets of the next substep (internal slot order): counts[slot], ids[slot*cap ...],
// found with the step kernels' query (hit_slots as theirs).
hipError_t launch_debug_contacts(const ClothView& cv, const SurfaceView& sv, const StepParams& sp,
                                const float* xs, const float* vs, int* counts, int* ids, int cap,
                                int hit_slots, hipStream_t st);
// The surface data the next substep's collision query touches: bit c of cell_bits for every
// non-empty cell some node queries, bit t of tri_bits for every box hit, and totals[0..2] +=
// node queries of non-empty cells, references tested, box hits (zeroed by the caller).
hipError_t launch_debug_volume(const ClothView& cv, const SurfaceView& sv, const StepParams& sp,
                               const float* xs, const float* vs, int hit_slots,
                               uint32_t* cell_bits, uint32_t* tri_bits,
                               unsigned long long* totals, hipStream_t st);
// Node-id AoS [n][3] <-> internal SoA [3][ld] through slot[id].
hipError_t launch_import(int n, int ld, const int* slot, const float* aos, float* soa,
                         int accumulate, hipStream_t st);
hipError_t launch_export(int n, int ld, const int* slot, const float* soa, float* aos,
                         hipStream_t st);
// Per-incidence k, c from per-spring arrays (sliced CSR and tile plan forms).
hipError_t launch_set_params(size_t m, const int* code, const float* k, const float* c, float* ik,
                             float* ic, hipStream_t st);
// Re-point incidence records at new parameter-table entries: record q takes
// entry[spring of code[q]].  negated = 1: code is in inc_spring's form (~s for a second end);
// negated = 0: code is a spring id, or -1 for padding (entry 0).
hipError_t launch_set_entries(size_t m, const int* code, int negated, const int* entry,
                              uint2* rec, hipStream_t st);
hipError_t launch_d2f(size_t n, const double* a, float* b, hipStream_t st);
// Per-vertex normals of the state x (SoA [3][ld], internal slots) into out (AoS, caller
// numbering); order[slot] = node id, groups[g] = (node_off, nx, ny, 0), node_group[slot]
// (NULL for one cloth).
hipError_t launch_vertex_normals(int n, int ld, const float* x, const int* order, const int* slot,
                                 const int* node_group, const int4* groups, float* out,
                                 hipStream_t st);

// --- a3 grid build ---------------------------------------------------------------------
// Per triangle: inflated box, geometry, vertices, and the number of grid cells its box overlaps
// (clamped to 2^31-1); total_refs accumulates the sum (64-bit).
hipError_t launch_tri_prep(int n_tris, const float* verts, const int* tris, float thickness,
                           const float org[3], float inv_cell, const int dim[3], float4* box_lo,
                           float4* box_hi, float4* geo, float4* tri_v,
                           unsigned long long* total_refs, hipStream_t stream);
hipError_t launch_grid_count(int n_tris, const float4* box_lo, const float4* box_hi,
                             const float org[3], float inv_cell, const int dim[3],
                             uint32_t* counts, hipStream_t stream);
hipError_t launch_grid_fill(int n_tris, const float4* box_lo, const float4* box_hi,
                            const float org[3], float inv_cell, const int dim[3],
                            const uint32_t* cell_start, uint32_t* fill, uint32_t* refs,
                            hipStream_t stream);
// Sorts each cell's references ascending and writes their records (ref_lo, ref_hi, ref_q).
hipError_t launch_grid_finish(int n_cells, const float org[3], float inv_cell, const int dim[3],
                              const uint32_t* cell_start, uint32_t* refs, const float4* box_lo,
                              const float4* box_hi, float4* ref_lo, float4* ref_hi, uint4* ref_q,
                              hipStream_t stream);

// Exclusive prefix sum of in[0..n) into out[0..n] (out[n] = total) with wavefront scans:
// each 1024-thread workgroup scans a tile of kScanTile entries (kScanItems per thread), the
// tile totals are scanned recursively and added back.  tmp must hold scan_tmp_words(n) words.
constexpr int kScanThreads = 1024;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;
size_t scan_tmp_words(size_t n);
hipError_t scan_exclusive_u32(const uint32_t* in, uint32_t* out, size_t n, uint32_t* tmp,
                              hipStream_t stream);

// Broad-phase query for arbitrary points (SoA [3][ld]) through the step kernels' own query
// with hit_slots list entries per lane (0 = unlisted): per-point candidate counts, then the
// (point, triangle) pairs at the given offsets.
hipError_t launch_candidates_count(int n, int ld, const float* p, const SurfaceView& sv,
                                   int hit_slots, uint32_t* counts, hipStream_t stream);
hipError_t launch_candidates_write(int n, int ld, const float* p, const SurfaceView& sv,
                                   int hit_slots, const uint32_t* offsets, int* pairs,
                                   hipStream_t stream);

}  // namespace cloth
