// a1-a4 fused for grid cloths: one substep, one wavefront per 8x8 tile of the internal order,
// the same results as k_substep bit for bit.
//
// The one-thread-per-node gather issues, per node, a load for every incidence record, every
// parameter entry and every component of every neighbour's state, about a hundred scattered
// loads per wavefront, and the address units of the compute units become the limit of the
// whole substep.  On a grid cloth the neighbours sit at fixed offsets (row, column), so here
//   1. each wavefront loads its tile and a two-node halo (12 x 12 nodes, both state vectors)
//      into LDS with row-coalesced loads whose slots follow from the grid shape alone (no
//      index loads first), together with its nodes' parameter-table entries per direction
//      (one byte each, relative to the cloth's first entry, while no cloth has more than
//      255) and, when the cloth has at most 128 entries, its part of the table;
//   2. each lane sums its node's springs from LDS in the incidence order (ascending
//      neighbour id = ascending offset (row, column)), with the same spring_force
//      arithmetic as every other kernel;
//   3. integration, the grid broad phase, the narrow phase and the response are those of
//      k_substep (HR box hits per round of geometry loads).
#include "cloth_device.h"
#include "cloth_internal.h"

namespace cloth {

namespace {

constexpr int kSide = 12;                  // region side: the tile and two nodes either side
constexpr int kRegion = kSide * kSide;     // 144 nodes
constexpr int kTabLds = 128;               // tables up to this size are read from LDS
// Lists of at most kShortListSlots hits load the geometry of kShortHitRound hits per round.
constexpr int kShortListSlots = 16;
constexpr int kShortHitRound = 4;

// Offsets of the stencil's directions in the region (row * kSide + column), in incidence
// order.
__device__ __forceinline__ constexpr int region_offset(int d) {
    constexpr int off[kStencilDirs] = {-2 * kSide,     -kSide - 1, -kSide, -kSide + 1,
                                       -2,             -1,         1,      2,
                                       kSide - 1,      kSide,      kSide + 1, 2 * kSide};
    return off[d];
}

// Internal slot of node (row gr, column gc) of a cloth whose tiles start at slot `first`:
// the tile rows above hold 8 nx nodes each, the tiles to the left in its tile row 8 h nodes
// each (h: that row's tile height), and nodes are row-major within their tile (w: the tile's
// width).
__device__ __forceinline__ int grid_slot(int first, int nx, int ny, int gr, int gc) {
    const int tr = gr >> 3, tc = gc >> 3;
    const int h = min(8, ny - 8 * tr), w = min(8, nx - 8 * tc);
    return first + 8 * nx * tr + 8 * h * tc + (gr & 7) * w + (gc & 7);
}

// NW wavefronts per tile: with NW = 2 the second wavefront helps stage the region and takes
// every other round of the box hits' narrow tests, and the first visits the contacts of both
// in list order (the same arithmetic in the same order as NW = 1).
template <bool COLLIDE, bool GROUPED, int HR, int NW>
__global__ void __launch_bounds__(64 * NW, 2)
    k_grid(const ClothView cv, const GridView gv, const StepParams sp,
           const float* __restrict__ xs, const float* __restrict__ vs, float* __restrict__ xd,
           float* __restrict__ vd, const SurfaceView* __restrict__ svs, const int hit_slots,
           const int xcd_runs, float* __restrict__ pred) {
    __shared__ float reg[6 * kRegion];  // x, y, z, vx, vy, vz of the region
    __shared__ float4 tab[kTabLds];
    extern __shared__ uint32_t hit_lds[];  // wave_query_lds(hit_slots) bytes
    static_assert(NW == 1 || (NW == 2 && COLLIDE), "one wavefront, or two with collision");
    constexpr int kThreads = 64 * NW;
    const int t = xcd_block(xcd_runs, gv.n_tiles);
    if (t >= gv.n_tiles) return;  // the whole workgroup
    const int4 cd = GROUPED ? gv.tiles[t] : gv.one;
    const int nx = cd.y & 0xffff, ny = cd.y >> 16;
    const int tl = t - cd.z, tx = (nx + 7) >> 3;
    const int gr0 = 8 * (tl / tx), gc0 = 8 * (tl % tx);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ld = cv.ld;
    const int r = lane >> 3, c = lane & 7;
    const bool active = wave == 0 && gr0 + r < ny && gc0 + c < nx;
    const int i = active ? grid_slot(cd.x, nx, ny, gr0 + r, gc0 + c) : 0;

    // 1. every load of the gather in one round
    float w = 0.0f;
    uint32_t idx8[kStencilDirs / 4] = {};
    if (active) {
        w = cv.w[i];
#pragma unroll
        for (int k = 0; k < kStencilDirs / 4; ++k) idx8[k] = gv.idx8[(size_t)k * ld + i];
    }
    // the cloth's entries of the parameter table start at tb; a small table is staged in LDS
    const int n_tab = *gv.n_tab;
    const int tb = GROUPED && gv.tab_base ? gv.tab_base[cd.w] : 0;
    const int tab_here = min(gv.tab_cap - tb, kTabLds);
    constexpr int kTabIters = kTabLds / kThreads, kRegionIters = (kRegion + kThreads - 1) / kThreads;
    float4 tv[kTabIters];
#pragma unroll
    for (int j = 0; j < kTabIters; ++j) {
        tv[j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (tid + kThreads * j < tab_here) tv[j] = ldg4(cv.ptab, tb + tid + kThreads * j);
    }
    float sv_[kRegionIters][6];
#pragma unroll
    for (int j = 0; j < kRegionIters; ++j) {
        const int e = tid + kThreads * j;
        const int gr = gr0 + e / kSide - 2, gc = gc0 + e % kSide - 2;
        const bool ok = e < kRegion && gr >= 0 && gr < ny && gc >= 0 && gc < nx;
#pragma unroll
        for (int k = 0; k < 6; ++k) sv_[j][k] = 0.0f;
        if (ok) {
            const int p = grid_slot(cd.x, nx, ny, gr, gc);
            sv_[j][0] = xs[p];
            sv_[j][1] = xs[ld + p];
            sv_[j][2] = xs[2 * ld + p];
            sv_[j][3] = vs[p];
            sv_[j][4] = vs[ld + p];
            sv_[j][5] = vs[2 * ld + p];
        }
    }
#pragma unroll
    for (int j = 0; j < kRegionIters; ++j) {
        const int e = tid + kThreads * j;
        if (e < kRegion) {
#pragma unroll
            for (int k = 0; k < 6; ++k) reg[k * kRegion + e] = sv_[j][k];
        }
    }
#pragma unroll
    for (int j = 0; j < kTabIters; ++j) tab[tid + kThreads * j] = tv[j];
    __syncthreads();

    // the parameter entries of the node's springs, relative to the cloth's first: bytes
    // while every cloth has few entries, else (a second round of loads) the full entries
    uint32_t idx[kStencilDirs];
    if (n_tab <= kSmallTab) {
#pragma unroll
        for (int d = 0; d < kStencilDirs; ++d) {
            const uint32_t b = (idx8[d / 4] >> (8 * (d % 4))) & 0xffu;
            idx[d] = active && b != kNoSpring8 ? b : kNoSpring;
        }
    } else {
#pragma unroll
        for (int d = 0; d < kStencilDirs; ++d) {
            const uint32_t v = active ? gv.idx[(size_t)d * ld + i] : kNoSpring;
            idx[d] = v == kNoSpring ? kNoSpring : v - (uint32_t)tb;
        }
    }

    // 2. the springs of each node from LDS, in incidence order; 3. integration
    float px = 0.0f, py = 0.0f, pz = 0.0f, qx = 0.0f, qy = 0.0f, qz = 0.0f;
    if (active) {
        const int e0 = (r + 2) * kSide + (c + 2);
        const float xi = reg[e0], yi = reg[kRegion + e0], zi = reg[2 * kRegion + e0];
        const float vxi = reg[3 * kRegion + e0], vyi = reg[4 * kRegion + e0],
                    vzi = reg[5 * kRegion + e0];
        float fx = 0.0f, fy = 0.0f, fz = 0.0f;
        float4 e[kStencilDirs];
        if (n_tab <= kTabLds) {
#pragma unroll
            for (int d = 0; d < kStencilDirs; ++d) e[d] = tab[idx[d] == kNoSpring ? 0 : idx[d]];
        } else {
#pragma unroll
            for (int d = 0; d < kStencilDirs; ++d)
                e[d] = ldg4(cv.ptab, tb + (idx[d] == kNoSpring ? 0 : idx[d]));
        }
#pragma unroll
        for (int d = 0; d < kStencilDirs; ++d) {
            if (idx[d] == kNoSpring) continue;
            const int e2 = e0 + region_offset(d);
            spring_force(reg[e2] - xi, reg[kRegion + e2] - yi, reg[2 * kRegion + e2] - zi,
                         reg[3 * kRegion + e2] - vxi, reg[4 * kRegion + e2] - vyi,
                         reg[5 * kRegion + e2] - vzi, e[d].x, e[d].y, e[d].z, fx, fy, fz);
        }
        add_external(sp, i, fx, fy, fz);
        integrate(w, sp.h, sp.g, xi, yi, zi, vxi, vyi, vzi, fx, fy, fz, px, py, pz, qx, qy, qz);
        if (pred) {  // the prediction before collision, for the adjoint
            pred[i] = px;
            pred[ld + i] = py;
            pred[2 * ld + i] = pz;
        }
    }
    // a3 + a4: broad phase, narrow phase, response (as k_substep)
    if constexpr (NW == 1) {
        if (COLLIDE && active && w != 0.0f) {
            const SurfaceView sv = svs[GROUPED ? cd.w : 0];
            if (sv.n_tris > 0) {
                if (hit_slots > 0)
                    collide_listed<HR>(sv, hit_lds + lane, hit_slots, sp.restitution, px, py, pz,
                                       qx, qy, qz);
                else
                    collide(sv, sp.restitution, px, py, pz, qx, qy, qz);
            }
        }
    } else {
        // the first wavefront lists its nodes' box hits; the hit rounds h0 = 0, HR, 2 HR, ...
        // of each list alternate between the two wavefronts, each recording its contacts as
        // bits of the list entries; the first then visits the contacts in list order
        __shared__ float p_lds[3 * 64];
        __shared__ int nh_lds[64];
        __shared__ unsigned long long bits_lds[64];
        const SurfaceView sv = svs[GROUPED ? cd.w : 0];
        const bool coll = active && w != 0.0f && sv.n_tris > 0;
        int nh = -1;  // -1: no list (outside the grid, or no collision for this node)
        uint32_t rb = 0, re = 0;
        if (wave == 0) {
            uint32_t cx, cy, cz;
            if (coll && hit_slots > 0 && cell_refs(sv, px, py, pz, cx, cy, cz, rb, re))
                nh = list_box_hits(sv, hit_lds + lane, hit_slots, cx, cy, cz, rb, re);
            nh_lds[lane] = nh >= 0 && nh <= hit_slots ? nh : 0;
            p_lds[lane] = px;
            p_lds[64 + lane] = py;
            p_lds[128 + lane] = pz;
        }
        __syncthreads();
        unsigned long long bits = 0;
        {
            const int nl = nh_lds[lane];
            const float bx = p_lds[lane], by = p_lds[64 + lane], bz = p_lds[128 + lane];
            for (int h0 = wave * HR; h0 < nl; h0 += NW * HR)
                hit_round<HR>(sv, hit_lds + lane, nl, h0, bx, by, bz,
                              [&](int k, uint32_t id, const float4& g0, const float4& g1,
                                  const float4& g2) {
                                  narrow_visit(sv, id, g0, g1, g2, bx, by, bz,
                                               [&](const float4&, float, uint32_t) {
                                                   bits |= 1ull << k;
                                               });
                              });
        }
        if (wave == 1) bits_lds[lane] = bits;
        __syncthreads();
        if (wave == 1) return;
        if (coll) {
            if (hit_slots == 0) {
                collide(sv, sp.restitution, px, py, pz, qx, qy, qz);
            } else {
                PushSum sum(sv.thickness);
                int cnt = 0;
                if (nh > hit_slots) {
                    cnt = visit_range<true, kRefRound>(sv, rb, re, px, py, pz, sum);
                } else if (nh > 0) {
                    for (unsigned long long m = bits | bits_lds[lane]; m; m &= m - 1ull) {
                        const uint32_t id = hit_lds[lane + 64 * __builtin_ctzll(m)] & 0x7fffffffu;
                        float4 n;
                        float ax, ay, az;
                        const float s = plane_offset(ldg4(sv.geo, 3 * (size_t)id),
                                                     ldg4(sv.geo, 3 * (size_t)id + 1),
                                                     ldg4(sv.geo, 3 * (size_t)id + 2), px, py,
                                                     pz, n, ax, ay, az);
                        sum(n, s, id);
                        ++cnt;
                    }
                }
                respond(cnt, sum.x, sum.y, sum.z, sp.restitution, px, py, pz, qx, qy, qz);
            }
        }
    }
    if (!active) return;
    xd[i] = px;
    xd[ld + i] = py;
    xd[2 * ld + i] = pz;
    vd[i] = qx;
    vd[ld + i] = qy;
    vd[2 * ld + i] = qz;
    if (sp.check_nan) {
        const float sum = px + py + pz + qx + qy + qz;
        if (!__builtin_isfinite(sum)) atomicOr(sp.nan_flag, 1);
    }
}

// One thread per slot: its kStencilDirs entries, then their byte form relative to the
// slot's cloth's first entry (one word per four directions).
__global__ void k_set_stencil_entries(int ld, const int* __restrict__ code,
                                      const int* __restrict__ entry,
                                      const int* __restrict__ slot_cloth,
                                      const int* __restrict__ tab_base, uint32_t* __restrict__ idx,
                                      uint32_t* __restrict__ idx8) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= ld) return;
    const uint32_t base = slot_cloth && tab_base ? (uint32_t)tab_base[slot_cloth[p]] : 0u;
    uint32_t word = 0;
    for (int d = 0; d < kStencilDirs; ++d) {
        const int s = code[(size_t)d * ld + p];
        const uint32_t v = s >= 0 ? (uint32_t)entry[s] : kNoSpring;
        idx[(size_t)d * ld + p] = v;
        word |= (v == kNoSpring ? kNoSpring8 : ((v - base) & 0xffu)) << (8 * (d % 4));
        if (d % 4 == 3) {
            idx8[(size_t)(d / 4) * ld + p] = word;
            word = 0;
        }
    }
}

}  // namespace

size_t grid_lds_bytes(int hit_slots) { return wave_query_lds(hit_slots); }

hipError_t prepare_grid_kernels(size_t lds_bytes) {
    if (lds_bytes <= 32 * 1024) return hipSuccess;
    const void* fns[] = {(const void*)k_grid<true, false, kHitRound, 1>,
                         (const void*)k_grid<true, true, kHitRound, 1>,
                         (const void*)k_grid<true, false, kShortHitRound, 1>,
                         (const void*)k_grid<true, true, kShortHitRound, 1>,
                         (const void*)k_grid<true, false, kShortHitRound, 2>,
                         (const void*)k_grid<true, true, kShortHitRound, 2>};
    for (const void* f : fns) {
        hipError_t e =
            hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_grid_substep(const ClothView& cv, const GridView& gv, int collide,
                               const StepParams& sp, const float* xs, const float* vs, float* xd,
                               float* vd, hipStream_t stream, const SurfaceView* svs,
                               int grouped, int hit_slots, int xcd_runs, int waves, float* pred) {
    if (gv.n_tiles <= 0) return hipSuccess;
    if (xcd_runs < 0 || xcd_runs > kMaxXcdRuns) xcd_runs = 0;
    if (hit_slots < 0 || hit_slots > kMaxHitSlots) return hipErrorInvalidValue;
    if (waves != 1 && waves != 2) return hipErrorInvalidValue;
    const int grid = xcd_grid(gv.n_tiles, xcd_runs);
    const size_t lds = collide ? grid_lds_bytes(hit_slots) : 0;
    // short hit lists go with short rounds of geometry and reference loads: fewer registers,
    // more wavefronts per SIMD for workloads whose collision work is spread over many of them;
    // the two-wavefront form always takes short rounds (at about 100 registers every tile of
    // a 100K-node cloth is resident at once; rounds of eight need 166)
    const bool short_round = hit_slots <= kShortListSlots;
    if (collide && waves == 2 && grouped)
        k_grid<true, true, kShortHitRound, 2><<<grid, 128, lds, stream>>>(
            cv, gv, sp, xs, vs, xd, vd, svs, hit_slots, xcd_runs, pred);
    else if (collide && waves == 2)
        k_grid<true, false, kShortHitRound, 2><<<grid, 128, lds, stream>>>(
            cv, gv, sp, xs, vs, xd, vd, svs, hit_slots, xcd_runs, pred);
    else if (collide && grouped && short_round)
        k_grid<true, true, kShortHitRound, 1><<<grid, 64, lds, stream>>>(
            cv, gv, sp, xs, vs, xd, vd, svs, hit_slots, xcd_runs, pred);
    else if (collide && grouped)
        k_grid<true, true, kHitRound, 1><<<grid, 64, lds, stream>>>(
            cv, gv, sp, xs, vs, xd, vd, svs, hit_slots, xcd_runs, pred);
    else if (collide && short_round)
        k_grid<true, false, kShortHitRound, 1><<<grid, 64, lds, stream>>>(
            cv, gv, sp, xs, vs, xd, vd, svs, hit_slots, xcd_runs, pred);
    else if (collide)
        k_grid<true, false, kHitRound, 1><<<grid, 64, lds, stream>>>(
            cv, gv, sp, xs, vs, xd, vd, svs, hit_slots, xcd_runs, pred);
    else if (grouped)
        k_grid<false, true, kHitRound, 1><<<grid, 64, 0, stream>>>(cv, gv, sp, xs, vs, xd, vd,
                                                                   svs, 0, xcd_runs, pred);
    else
        k_grid<false, false, kHitRound, 1><<<grid, 64, 0, stream>>>(cv, gv, sp, xs, vs, xd, vd,
                                                                    svs, 0, xcd_runs, pred);
    return hipGetLastError();
}

hipError_t launch_set_stencil_entries(int ld, const int* code, const int* entry,
                                      const int* slot_cloth, const int* tab_base, uint32_t* idx,
                                      uint32_t* idx8, hipStream_t st) {
    if (ld <= 0) return hipSuccess;
    k_set_stencil_entries<<<(unsigned)((ld + 255) / 256), 256, 0, st>>>(ld, code, entry,
                                                                         slot_cloth, tab_base,
                                                                         idx, idx8);
    return hipGetLastError();
}

}  // namespace cloth
