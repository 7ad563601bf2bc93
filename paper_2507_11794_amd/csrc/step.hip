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
    k_substep(const ClothView cv, const SurfaceView sv1, const StepParams sp,
              const float* __restrict__ xs, const float* __restrict__ vs, float* __restrict__ xd,
              float* __restrict__ vd, const SurfaceView* __restrict__ svs,
              const int* __restrict__ node_group) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cv.n) return;
    const int ld = cv.ld;
    const float xi = xs[i], yi = xs[ld + i], zi = xs[2 * ld + i];
    const float vxi = vs[i], vyi = vs[ld + i], vzi = vs[2 * ld + i];
    const float w = cv.w[i];

    // a1: gather
    float fx = 0.0f, fy = 0.0f, fz = 0.0f;
    const int deg = cv.deg[i];
    const int base = cv.slice_ptr[i >> 6] + (i & 63);
    for (int r = 0; r < deg; ++r) {
        const int q = base + r * 64;
        const int j = cv.nbr[q];
        spring_force(xs[j] - xi, xs[ld + j] - yi, xs[2 * ld + j] - zi, vs[j] - vxi,
                     vs[ld + j] - vyi, vs[2 * ld + j] - vzi, cv.ik[q], cv.ic[q], cv.il[q], fx, fy,
                     fz);
    }

    // a2: integrate; a3 + a4: broad phase, narrow phase, response
    float px, py, pz, qx, qy, qz;
    integrate(w, sp.h, sp.g, xi, yi, zi, vxi, vyi, vzi, fx, fy, fz, px, py, pz, qx, qy, qz);
    if (COLLIDE && w != 0.0f) {
        if (GROUPED) {
            const SurfaceView sv = svs[node_group[i]];
            if (sv.n_tris > 0) collide(sv, sp.restitution, px, py, pz, qx, qy, qz);
        } else {
            collide(sv1, sp.restitution, px, py, pz, qx, qy, qz);
        }
    }

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

hipError_t launch_substep(const ClothView& cv, const SurfaceView& sv, const StepParams& sp,
                          const float* xs, const float* vs, float* xd, float* vd, int block,
                          hipStream_t stream, const SurfaceView* svs, const int* node_group) {
    if (cv.n <= 0) return hipSuccess;
    if (block <= 0 || block > 256 || (block & 63)) block = 256;
    const int grid = (cv.n + block - 1) / block;
    if (svs && node_group)
        k_substep<true, true><<<grid, block, 0, stream>>>(cv, sv, sp, xs, vs, xd, vd, svs,
                                                          node_group);
    else if (sv.n_tris > 0)
        k_substep<true, false><<<grid, block, 0, stream>>>(cv, sv, sp, xs, vs, xd, vd, nullptr,
                                                           nullptr);
    else
        k_substep<false, false><<<grid, block, 0, stream>>>(cv, sv, sp, xs, vs, xd, vd, nullptr,
                                                            nullptr);
    return hipGetLastError();
}

}  // namespace cloth
