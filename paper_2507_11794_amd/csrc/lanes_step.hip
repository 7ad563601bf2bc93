// a1-a4 fused, one launch per substep, L lanes per node (L = 2 or 4): the same substep as
// k_substep, bit for bit, with each node's work split over a group of L adjacent lanes.
//
// At the workloads' sizes the one-lane-per-node kernel is bound by per-lane latency, not by
// bandwidth: a 100K-node cloth fills only 1,561 wavefronts, so every lane's chain of
// dependent loads shows, and the few wavefronts whose nodes sit in crowded grid cells run
// their serial collision query long after the others have finished.  Here
//   a1  lane j of a group loads and evaluates the incidences r = j, j + L, j + 2L, ... of
//       its node; the group then sums all of them in incidence order, every lane reading
//       the others' terms through DPP lane moves, so each lane holds the same force as the
//       one-lane gather (the same fused multiply-adds in the same order);
//   a2  every lane integrates the node (identical values);
//   a3  lane j tests the j-th of L consecutive, equal runs of the cell's references (coded
//       boxes, its own hit list in LDS);
//   a4  lane j runs the narrow phase on its own hits and keeps up to kLaneContacts contacts
//       (push th - s and normal n) in LDS; the group then sums the contacts of lanes
//       0..L-1 in order.  The runs are consecutive and each is ascending, so the contacts
//       are summed in ascending triangle id with the same operations as the one-lane query.
//       A group with a lane holding more contacts than it keeps runs the one-lane query
//       instead (on every lane: identical values).
// Lane 0 of a group writes the node.
#include "cloth_device.h"
#include "cloth_internal.h"

namespace cloth {

namespace {

constexpr int kLaneContacts = 4;
// A lane tests a fraction of a cell's references and lists a fraction of its hits, so its
// query uses smaller rounds than the one-lane query (fewer registers: more wavefronts per
// SIMD to hide the loads' latency); the rounds do not change which contacts are found or
// their order.
constexpr int kLaneRefRound = 8;
constexpr int kLaneHitRound = 4;

// Value of lane j of this lane's group of L (L = 2 or 4) as one DPP move: quad_perm
// [j, j, j, j] for L = 4, [j, j, 2 + j, 2 + j] for L = 2.
template <int L, int J>
__device__ __forceinline__ float group_bcast(float v) {
    constexpr int ctrl = L == 4 ? J * 0x55 : (J | (J << 2) | ((2 + J) << 4) | ((2 + J) << 6));
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), ctrl, 0xF, 0xF, false));
}
template <int L, int J>
__device__ __forceinline__ int group_bcast_i(int v) {
    constexpr int ctrl = L == 4 ? J * 0x55 : (J | (J << 2) | ((2 + J) << 4) | ((2 + J) << 6));
    return __builtin_amdgcn_mov_dpp(v, ctrl, 0xF, 0xF, false);
}
template <int L, int J>
__device__ __forceinline__ float4 group_bcast4(const float4& v) {
    return make_float4(group_bcast<L, J>(v.x), group_bcast<L, J>(v.y), group_bcast<L, J>(v.z),
                       group_bcast<L, J>(v.w));
}

// a1 for node i on lane `part` of its group (see the file comment): the group's forces, in
// incidence order, on every lane of the group.  All L lanes of the group must be active.
template <int L>
__device__ __forceinline__ void gather_lanes(const ClothView& cv, const float* __restrict__ xs,
                                             const float* __restrict__ vs, int i, int part,
                                             float xi, float yi, float zi, float vxi, float vyi,
                                             float vzi, float& fx, float& fy, float& fz) {
    constexpr int R = 12, RL = R / L;  // incidences per round, per lane
    const int ld = cv.ld;
    const int deg = cv.deg[i];
    const int base = cv.slice_ptr[i >> 6] + (i & 63);
    const gptr<float> X = gmem(xs), V = gmem(vs);
    for (int r0 = 0; r0 < deg; r0 += R) {
        uint2 rec[RL];
#pragma unroll
        for (int q = 0; q < RL; ++q)
            rec[q] = ldgu2(cv.inc2, (size_t)(base + min(r0 + part + L * q, deg - 1) * 64));
        float4 e[RL];
        float nx[RL], ny[RL], nz[RL], mx[RL], my[RL], mz[RL];
#pragma unroll
        for (int q = 0; q < RL; ++q) {
            e[q] = ldg4(cv.ptab, rec[q].y);
            const int j = (int)rec[q].x;
            nx[q] = X[j];
            ny[q] = X[ld + j];
            nz[q] = X[2 * ld + j];
            mx[q] = V[j];
            my[q] = V[ld + j];
            mz[q] = V[2 * ld + j];
        }
        // this lane's terms: coefficient s and spring vector d of each of its incidences
        float4 term[RL];
#pragma unroll
        for (int q = 0; q < RL; ++q) {
            const float dx = nx[q] - xi, dy = ny[q] - yi, dz = nz[q] - zi;
            term[q] = make_float4(spring_coeff(dx, dy, dz, mx[q] - vxi, my[q] - vyi, mz[q] - vzi,
                                               e[q].x, e[q].y, e[q].z),
                                  dx, dy, dz);
        }
        // incidence r0 + L q + j is lane j's term q: sum them in incidence order
#pragma unroll
        for (int q = 0; q < RL; ++q) {
            float4 t[L];
            t[0] = group_bcast4<L, 0>(term[q]);
            t[1] = group_bcast4<L, 1>(term[q]);
            if constexpr (L == 4) {
                t[2] = group_bcast4<L, 2>(term[q]);
                t[3] = group_bcast4<L, 3>(term[q]);
            }
#pragma unroll
            for (int j = 0; j < L; ++j)
                if (r0 + L * q + j < deg) spring_accumulate(t[j].x, t[j].y, t[j].z, t[j].w, fx, fy, fz);
        }
    }
}

// LDS of one wavefront: the lanes' hit lists, then each lane's contact records (push
// th - s and normal n), kLaneContacts of them plus one scratch record that takes the writes
// past the last, interleaved as the hit lists are (record k of lane l at k * 64 + l).
constexpr size_t lanes_wave_lds(int hit_slots) {
    return wave_query_lds(hit_slots) + (size_t)(kLaneContacts + 1) * 64 * sizeof(float4);
}

// Adds the first n records of lane J of the group (group: its lane 0's records) to
// (sx, sy, sz) in order.
template <int J>
__device__ __forceinline__ void add_lane_contacts(const float4* group, int n, float& sx,
                                                  float& sy, float& sz) {
    for (int k = 0; k < n; ++k) {
        const float4 c = group[k * 64 + J];
        sx += c.x * c.y;
        sy += c.x * c.z;
        sz += c.x * c.w;
    }
}

template <int L, bool COLLIDE, bool GROUPED>
__global__ void __launch_bounds__(256)
    k_lanes(const ClothView cv, const StepParams sp, const float* __restrict__ xs,
            const float* __restrict__ vs, float* __restrict__ xd, float* __restrict__ vd,
            const SurfaceView* __restrict__ svs, const int* __restrict__ node_group,
            const int hit_slots, const int xcd_runs, float* __restrict__ pred) {
    extern __shared__ uint32_t hit_lds[];  // per wavefront: lanes_wave_lds(hit_slots) bytes
    const int nodes_per_block = blockDim.x / L;
    const int n_logical = (cv.n + nodes_per_block - 1) / nodes_per_block;
    const int i = xcd_block(xcd_runs, n_logical) * nodes_per_block + threadIdx.x / L;
    const int part = threadIdx.x % L;
    if (i >= cv.n) return;  // a whole group: every lane of a group has the same node
    const int ld = cv.ld;
    const float xi = xs[i], yi = xs[ld + i], zi = xs[2 * ld + i];
    const float vxi = vs[i], vyi = vs[ld + i], vzi = vs[2 * ld + i];
    const float w = cv.w[i];
    float fx = 0.0f, fy = 0.0f, fz = 0.0f;
    gather_lanes<L>(cv, xs, vs, i, part, xi, yi, zi, vxi, vyi, vzi, fx, fy, fz);
    add_external(sp, i, fx, fy, fz);
    float px, py, pz, qx, qy, qz;
    integrate(w, sp.h, sp.g, xi, yi, zi, vxi, vyi, vzi, fx, fy, fz, px, py, pz, qx, qy, qz);
    if (pred && part == 0) {
        pred[i] = px;
        pred[ld + i] = py;
        pred[2 * ld + i] = pz;
    }
    if (COLLIDE && w != 0.0f) {
        const SurfaceView sv = svs[GROUPED ? node_group[i] : 0];
        const int lane = threadIdx.x & 63;
        uint32_t* wave = hit_lds + (threadIdx.x >> 6) * (lanes_wave_lds(hit_slots) / 4);
        uint32_t* list = wave + lane;
        float4* recs = reinterpret_cast<float4*>(wave + list_stride(hit_slots));
        const float gx = cell_coord_raw(px, sv.org[0], sv.inv_cell);
        const float gy = cell_coord_raw(py, sv.org[1], sv.inv_cell);
        const float gz = cell_coord_raw(pz, sv.org[2], sv.inv_cell);
        const float cfx = floorf(gx), cfy = floorf(gy), cfz = floorf(gz);
        // the test of cell_of, on the same values (uniform over the group)
        if (sv.n_tris > 0 && cfx >= 0.0f && cfx <= (float)(sv.dim[0] - 1) && cfy >= 0.0f &&
            cfy <= (float)(sv.dim[1] - 1) && cfz >= 0.0f && cfz <= (float)(sv.dim[2] - 1)) {
            const int cell = ((int)cfz * sv.dim[1] + (int)cfy) * sv.dim[0] + (int)cfx;
            const uint32_t cx = point_code(gx, cfx), cy = point_code(gy, cfy),
                           cz = point_code(gz, cfz);
            const gptr<uint32_t> cs = gmem(sv.cell_start);
            const uint32_t b = cs[cell], e = cs[cell + 1];
            const uint32_t run = (e - b + L - 1) / L;
            const uint32_t r0 = min(e, b + part * run), r1 = min(e, r0 + run);
            const float th = sv.thickness;
            int nc = 0;
            auto keep = [&](const float4& n, float s, uint32_t) {
                recs[min(nc, kLaneContacts) * 64 + lane] = make_float4(th - s, n.x, n.y, n.z);
                ++nc;
            };
            if (hit_slots > 0)
                listed_range<true, kLaneRefRound, kLaneHitRound>(sv, list, hit_slots, cx, cy, cz,
                                                                 r0, r1, px, py, pz, keep);
            else
                visit_range<true, kLaneRefRound>(sv, r0, r1, px, py, pz, keep);
            // the group's lanes have reconverged: gather their counts
            const int n0 = group_bcast_i<L, 0>(nc), n1 = group_bcast_i<L, 1>(nc);
            const int n2 = L == 4 ? group_bcast_i<L, 2>(nc) : 0;
            const int n3 = L == 4 ? group_bcast_i<L, 3>(nc) : 0;
            const int most = max(max(n0, n1), max(n2, n3));
            if (most > kLaneContacts) {
                // a lane kept too few: the one-lane query over the whole cell
                PushSum sum(th);
                const int cnt =
                    hit_slots > 0
                        ? listed_range<true, kLaneRefRound, kLaneHitRound>(
                              sv, list, hit_slots, cx, cy, cz, b, e, px, py, pz, sum)
                        : visit_range<true, kLaneRefRound>(sv, b, e, px, py, pz, sum);
                respond(cnt, sum.x, sum.y, sum.z, sp.restitution, px, py, pz, qx, qy, qz);
            } else {
                // the group's records, in lane order (LDS operations of a wavefront complete
                // in order, so the other lanes' records are in place)
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                const float4* group = recs + (lane & ~(L - 1));
                float sx = 0.0f, sy = 0.0f, sz = 0.0f;
                add_lane_contacts<0>(group, n0, sx, sy, sz);
                add_lane_contacts<1>(group, n1, sx, sy, sz);
                if constexpr (L == 4) {
                    add_lane_contacts<2>(group, n2, sx, sy, sz);
                    add_lane_contacts<3>(group, n3, sx, sy, sz);
                }
                respond(n0 + n1 + n2 + n3, sx, sy, sz, sp.restitution, px, py, pz, qx, qy, qz);
            }
        }
    }
    if (part != 0) return;
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

template <int L>
hipError_t launch_l(const ClothView& cv, int collide, const StepParams& sp, const float* xs,
                    const float* vs, float* xd, float* vd, int block, hipStream_t stream,
                    const SurfaceView* svs, const int* node_group, int hit_slots, int xcd_runs,
                    float* pred) {
    const int nodes_per_block = block / L;
    const int grid = xcd_grid((cv.n + nodes_per_block - 1) / nodes_per_block, xcd_runs);
    const size_t lds = collide ? (size_t)(block / 64) * lanes_wave_lds(hit_slots) : 0;
    if (collide && node_group)
        k_lanes<L, true, true><<<grid, block, lds, stream>>>(cv, sp, xs, vs, xd, vd, svs,
                                                             node_group, hit_slots, xcd_runs, pred);
    else if (collide)
        k_lanes<L, true, false><<<grid, block, lds, stream>>>(cv, sp, xs, vs, xd, vd, svs,
                                                              nullptr, hit_slots, xcd_runs, pred);
    else
        k_lanes<L, false, false><<<grid, block, 0, stream>>>(cv, sp, xs, vs, xd, vd, svs,
                                                             nullptr, 0, xcd_runs, pred);
    return hipGetLastError();
}

template <int L>
hipError_t prepare_l(size_t lds_bytes) {
    hipError_t e = hipFuncSetAttribute((const void*)k_lanes<L, true, false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_lanes<L, true, true>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
}

}  // namespace

size_t lanes_lds_bytes(int block, int hit_slots) {
    return (size_t)(block / 64) * lanes_wave_lds(hit_slots);
}

hipError_t prepare_lanes_kernels(size_t lds_bytes) {
    if (lds_bytes <= 64 * 1024) return hipSuccess;
    hipError_t e = prepare_l<2>(lds_bytes);
    return e != hipSuccess ? e : prepare_l<4>(lds_bytes);
}

hipError_t launch_substep_lanes(int lanes, const ClothView& cv, int collide, const StepParams& sp,
                                const float* xs, const float* vs, float* xd, float* vd, int block,
                                hipStream_t stream, const SurfaceView* svs, const int* node_group,
                                int hit_slots, int xcd_runs, float* pred) {
    if (cv.n <= 0) return hipSuccess;
    if (block <= 0 || block > 256 || (block & 63)) block = 256;
    if (xcd_runs < 0 || xcd_runs > kMaxXcdRuns) xcd_runs = 0;
    if (hit_slots < 0 || hit_slots > kMaxHitSlots) return hipErrorInvalidValue;
    if (lanes == 2)
        return launch_l<2>(cv, collide, sp, xs, vs, xd, vd, block, stream, svs, node_group,
                           hit_slots, xcd_runs, pred);
    if (lanes == 4)
        return launch_l<4>(cv, collide, sp, xs, vs, xd, vd, block, stream, svs, node_group,
                           hit_slots, xcd_runs, pred);
    return hipErrorInvalidValue;
}

}  // namespace cloth
