// a1-a4 with temporal blocking: one workgroup advances its tile of nodes K substeps at a
// time.  The tile's K-hop region is gathered from HBM into LDS once per launch; every
// substep recomputes a shrinking prefix of the region entirely from LDS (spring forces of
// Alg. 1 gathered per node, semi-implicit Euler with pins, grid broad phase, point-triangle
// narrow phase and the averaged response of Alg. 2), and only the tile is written back.
// Neighbouring tiles recompute shared halo nodes with identical inputs and identical
// arithmetic, so the result equals K launches of the one-substep kernel bit for bit.  Tiles
// are independent within a launch, so a workgroup may run any list of them (the schedule).
#include "cloth_device.h"
#include "cloth_internal.h"

namespace cloth {

namespace {

template <bool COLLIDE>
__device__ __forceinline__ void run_tile(const TileView& tv, const TileMeta& m, const int K,
                                         const StepParams& sp, const float* __restrict__ xs,
                                         const float* __restrict__ vs, float* __restrict__ xd,
                                         float* __restrict__ vd, float* lds, uint32_t* hit_lds,
                                         int hit_slots) {
    const int rmax = tv.rmax, ld = tv.ld;
    float* X0 = lds;
    float* X1 = lds + 3 * rmax;
    float* V0 = lds + 6 * rmax;
    float* V1 = lds + 9 * rmax;
    const int* rs = tv.region_slot + m.region_off;
    const int n_load = m.level[K];
    for (int u = threadIdx.x; u < n_load; u += blockDim.x) {
        const int slot = rs[u];
        X0[u] = xs[slot];
        X0[rmax + u] = xs[ld + slot];
        X0[2 * rmax + u] = xs[2 * ld + slot];
        V0[u] = vs[slot];
        V0[rmax + u] = vs[ld + slot];
        V0[2 * rmax + u] = vs[2 * ld + slot];
    }
    SurfaceView sv;
    if (COLLIDE) sv = tv.svs[m.group];
    const bool collide_here = COLLIDE && sv.n_tris > 0;
    __syncthreads();
    for (int s = 1; s <= K; ++s) {
        const float* Xs = (s & 1) ? X0 : X1;
        const float* Vs = (s & 1) ? V0 : V1;
        float* Xd = (s & 1) ? X1 : X0;
        float* Vd = (s & 1) ? V1 : V0;
        const int ncomp = m.level[K - s];
        // wavefront-uniform chunks of 64 nodes, so the collision query can run per wavefront
        for (int u0 = threadIdx.x & ~63; u0 < ncomp; u0 += blockDim.x) {
            const int u = u0 + (threadIdx.x & 63);
            const bool valid = u < ncomp;
            float px = 0.0f, py = 0.0f, pz = 0.0f, qx = 0.0f, qy = 0.0f, qz = 0.0f, w = 0.0f;
            if (valid) {
                const float xi = Xs[u], yi = Xs[rmax + u], zi = Xs[2 * rmax + u];
                const float vxi = Vs[u], vyi = Vs[rmax + u], vzi = Vs[2 * rmax + u];
                w = tv.w[rs[u]];
                const int deg = tv.comp_deg[m.comp_off + u];
                const uint2* inc = tv.inc + m.inc_off + u;
                float fx = 0.0f, fy = 0.0f, fz = 0.0f;
                // records of four incidences and their parameters are loaded together, then
                // summed in order
                for (int r0 = 0; r0 < deg; r0 += 4) {
                    uint2 rec[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        rec[q] = r0 + q < deg ? inc[(r0 + q) * m.inc_pad] : make_uint2(u, 0u);
                    float4 e[4];  // (k, c, rest length, 0)
#pragma unroll
                    for (int q = 0; q < 4; ++q) e[q] = ldg4(tv.ptab, rec[q].y);
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (r0 + q < deg) {
                            const int j = (int)rec[q].x;
                            spring_force(Xs[j] - xi, Xs[rmax + j] - yi, Xs[2 * rmax + j] - zi,
                                         Vs[j] - vxi, Vs[rmax + j] - vyi,
                                         Vs[2 * rmax + j] - vzi, e[q].x, e[q].y, e[q].z, fx,
                                         fy, fz);
                        }
                }
                add_external(sp, rs[u], fx, fy, fz);
                integrate(w, sp.h, sp.g, xi, yi, zi, vxi, vyi, vzi, fx, fy, fz, px, py, pz, qx,
                          qy, qz);
            }
            if (collide_here && valid && w != 0.0f) {
                if (hit_slots > 0)
                    collide_listed(sv,
                                   hit_lds + (threadIdx.x >> 6) * list_stride(hit_slots) + (threadIdx.x & 63),
                                   hit_slots, sp.restitution, px, py, pz, qx, qy, qz);
                else
                    collide(sv, sp.restitution, px, py, pz, qx, qy, qz);
            }
            if (valid) {
                Xd[u] = px;
                Xd[rmax + u] = py;
                Xd[2 * rmax + u] = pz;
                Vd[u] = qx;
                Vd[rmax + u] = qy;
                Vd[2 * rmax + u] = qz;
                if (sp.check_nan) {
                    const float sum = px + py + pz + qx + qy + qz;
                    if (!__builtin_isfinite(sum)) atomicOr(sp.nan_flag, 1);
                }
            }
        }
        __syncthreads();
    }
    const float* Xf = (K & 1) ? X1 : X0;
    const float* Vf = (K & 1) ? V1 : V0;
    for (int u = threadIdx.x; u < m.level[0]; u += blockDim.x) {
        const int slot = rs[u];
        xd[slot] = Xf[u];
        xd[ld + slot] = Xf[rmax + u];
        xd[2 * ld + slot] = Xf[2 * rmax + u];
        vd[slot] = Vf[u];
        vd[ld + slot] = Vf[rmax + u];
        vd[2 * ld + slot] = Vf[2 * rmax + u];
    }
}

// Workgroup b runs the tiles items[item_ptr[b] .. item_ptr[b+1]) one after another (one tile
// per workgroup for the grid schedule, a work list for the persistent schedules).
template <bool COLLIDE>
__global__ void __launch_bounds__(256)
    k_tile(const TileView tv, const int K, const StepParams sp, const float* __restrict__ xs,
           const float* __restrict__ vs, float* __restrict__ xd, float* __restrict__ vd,
           const int hit_slots) {
    extern __shared__ float4 lds4[];
    float* lds = reinterpret_cast<float*>(lds4);
    uint32_t* hit_lds = reinterpret_cast<uint32_t*>(lds4 + 3 * (size_t)tv.rmax);  // after the state
    const int b0 = tv.item_ptr[blockIdx.x], b1 = tv.item_ptr[blockIdx.x + 1];
    for (int it = b0; it < b1; ++it) {
        const TileMeta& m = tv.meta[tv.items[it]];
        run_tile<COLLIDE>(tv, m, K, sp, xs, vs, xd, vd, lds, hit_lds, hit_slots);
        __syncthreads();  // LDS is reused by the next tile
    }
}

}  // namespace

hipError_t prepare_tile_kernels(size_t lds_bytes) {
    if (lds_bytes <= 64 * 1024) return hipSuccess;
    hipError_t e = hipFuncSetAttribute((const void*)k_tile<true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_tile<false>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
}

hipError_t launch_tiles(const TileView& tv, int K, int collide, const StepParams& sp,
                        const float* xs, const float* vs, float* xd, float* vd, int block,
                        int hit_slots, hipStream_t stream) {
    if (tv.n_tiles <= 0 || tv.n_workgroups <= 0) return hipSuccess;
    if (block <= 0 || block > 256 || (block & 63)) block = 256;
    if (!collide) hit_slots = 0;
    const size_t lds = tile_lds_bytes(tv.rmax, block, hit_slots);
    if (collide)
        k_tile<true><<<tv.n_workgroups, block, lds, stream>>>(tv, K, sp, xs, vs, xd, vd,
                                                              hit_slots);
    else
        k_tile<false><<<tv.n_workgroups, block, lds, stream>>>(tv, K, sp, xs, vs, xd, vd, 0);
    return hipGetLastError();
}

}  // namespace cloth
