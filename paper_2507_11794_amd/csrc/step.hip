// a1-a4 fused: one substep of the mass-spring cloth for every node, one thread per node.
//
//   a1  F_i = sum over incident springs of Alg. 1's force, gathered over the sliced CSR
//       incidence list in a fixed order (no atomics, bitwise deterministic).
//   a2  semi-implicit Euler: v* = v + h (w F + g), x* = x + h v*; pinned (w = 0): v* = 0,
//       x* = x.
//   a3  broad phase: the grid cell of x*; its triangles in ascending id; inclusive test
//       against each triangle's thickness-inflated box.
//   a4  narrow phase: contact iff point-triangle distance < thickness; response of Alg. 2
//       with the averaged direction of Sec. 3: x = x* + mean_t (th - (x* - A_t).n_t) n_t,
//       v = -restitution v*.
#include "cloth_device.h"
#include "cloth_internal.h"

namespace cloth {

template <bool COLLIDE, bool GROUPED>
__global__ void __launch_bounds__(256)
    k_substep(const ClothView cv, const StepParams sp, const float* __restrict__ xs,
              const float* __restrict__ vs, float* __restrict__ xd, float* __restrict__ vd,
              const SurfaceView* __restrict__ svs, const int* __restrict__ node_group,
              const int hit_slots, const int xcd_runs, const int split_refs,
              int* __restrict__ heavy, const int parity, float* __restrict__ pred) {
    extern __shared__ uint32_t hit_lds[];  // per wavefront: wave_query_lds(hit_slots) bytes
    const int i = xcd_block(xcd_runs, (cv.n + blockDim.x - 1) / blockDim.x) * blockDim.x +
                  threadIdx.x;
    const bool valid = i < cv.n;
    const int ld = cv.ld;
    float px = 0.0f, py = 0.0f, pz = 0.0f, qx = 0.0f, qy = 0.0f, qz = 0.0f, w = 0.0f;
    if (valid) {
        const float xi = xs[i], yi = xs[ld + i], zi = xs[2 * ld + i];
        const float vxi = vs[i], vyi = vs[ld + i], vzi = vs[2 * ld + i];
        w = cv.w[i];
        // a1: gather
        float fx = 0.0f, fy = 0.0f, fz = 0.0f;
        gather_global(cv, xs, vs, i, xi, yi, zi, vxi, vyi, vzi, fx, fy, fz);
        add_external(sp, i, fx, fy, fz);
        // a2: integrate
        integrate(w, sp.h, sp.g, xi, yi, zi, vxi, vyi, vzi, fx, fy, fz, px, py, pz, qx, qy, qz);
        if (pred) {  // the prediction before collision, for the adjoint
            pred[i] = px;
            pred[ld + i] = py;
            pred[2 * ld + i] = pz;
        }
    }
    // a3 + a4: broad phase, narrow phase, response
    int is_heavy = 0;
    if (COLLIDE && valid && w != 0.0f) {
        // the surface is read from device memory, so captured graphs stay valid when it is
        // rebuilt
        const SurfaceView sv = svs[GROUPED ? node_group[i] : 0];
        if (sv.n_tris > 0 && split_refs > 0) {
            // a node whose cell lists more than split_refs references is left to the
            // four-lane second pass (its prediction is written below)
            const int cell = cell_of(sv, px, py, pz);
            if (cell >= 0) {
                const gptr<uint32_t> cs = gmem(sv.cell_start);
                is_heavy = cs[cell + 1] - cs[cell] > (uint32_t)split_refs;
            }
        }
        if (sv.n_tris > 0 && !is_heavy) {
            if (hit_slots > 0)
                collide_listed(sv, hit_lds + (threadIdx.x >> 6) * list_stride(hit_slots) + (threadIdx.x & 63),
                               hit_slots, sp.restitution, px, py, pz, qx, qy, qz);
            else
                collide(sv, sp.restitution, px, py, pz, qx, qy, qz);
        }
    }
    if (split_refs > 0) {
        // append the wavefront's heavy nodes to this parity's list, one atomic per wavefront
        const unsigned long long m = __ballot(is_heavy != 0);
        if (m) {
            const int lane = threadIdx.x & 63, leader = __builtin_ctzll(m);
            int base = 0;
            if (lane == leader) base = atomicAdd(heavy + parity, __popcll(m));
            base = __shfl(base, leader);
            const int pos = base + __popcll(m & ((1ULL << lane) - 1ULL));
            if (is_heavy && pos < cv.ld) heavy[kHeavyListOff + (size_t)parity * cv.ld + pos] = i;
        }
    }
    if (!valid) return;
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

hipError_t prepare_substep_kernels(size_t lds_bytes) {
    if (lds_bytes <= 64 * 1024) return hipSuccess;
    hipError_t e = hipFuncSetAttribute((const void*)k_substep<true, false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_substep<true, true>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
}

hipError_t launch_substep(const ClothView& cv, int collide, const StepParams& sp, const float* xs,
                          const float* vs, float* xd, float* vd, int block, hipStream_t stream,
                          const SurfaceView* svs, const int* node_group, int hit_slots,
                          int xcd_runs, int split_refs, int* heavy, int parity, float* pred) {
    if (cv.n <= 0) return hipSuccess;
    if (block <= 0 || block > 256 || (block & 63)) block = 256;
    if (xcd_runs < 0 || xcd_runs > kMaxXcdRuns) xcd_runs = 0;
    const int grid = xcd_grid((cv.n + block - 1) / block, xcd_runs);
    if (!collide || !heavy) split_refs = 0;
    const size_t lds = collide ? (size_t)(block / 64) * wave_query_lds(hit_slots) : 0;
    if (collide && node_group) {
        k_substep<true, true><<<grid, block, lds, stream>>>(cv, sp, xs, vs, xd, vd, svs, node_group,
                                                            hit_slots, xcd_runs, split_refs, heavy, parity,
                                                            pred);
    } else if (collide) {
        k_substep<true, false><<<grid, block, lds, stream>>>(cv, sp, xs, vs, xd, vd, svs, nullptr,
                                                             hit_slots, xcd_runs, split_refs, heavy, parity,
                                                            pred);
    } else {
        k_substep<false, false><<<grid, block, 0, stream>>>(cv, sp, xs, vs, xd, vd, svs, nullptr,
                                                            0, xcd_runs, 0, nullptr, 0, pred);
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && split_refs > 0)
        e = launch_heavy(cv, sp, heavy, parity, xd, vd, svs, node_group, stream);
    return e;
}

}  // namespace cloth
