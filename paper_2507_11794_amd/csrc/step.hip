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

template <bool COLLIDE>
__global__ void __launch_bounds__(256)
    k_substep(const ClothView cv, const SurfaceView sv, const StepParams sp,
              const float* __restrict__ xs, const float* __restrict__ vs, float* __restrict__ xd,
              float* __restrict__ vd) {
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

    // a2: integrate
    float px = xi, py = yi, pz = zi, qx = 0.0f, qy = 0.0f, qz = 0.0f;
    if (w != 0.0f) {
        const float h = sp.h;
        qx = vxi + h * (w * fx + sp.g[0]);
        qy = vyi + h * (w * fy + sp.g[1]);
        qz = vzi + h * (w * fz + sp.g[2]);
        px = xi + h * qx;
        py = yi + h * qy;
        pz = zi + h * qz;
    }

    // a3 + a4
    if (COLLIDE && w != 0.0f) {
        const int cell = cell_of(sv, px, py, pz);
        const uint32_t b = sv.cell_start[cell], e = sv.cell_start[cell + 1];
        float sx = 0.0f, sy = 0.0f, sz = 0.0f;
        int cnt = 0;
        for (uint32_t r = b; r < e; ++r) {
            const uint32_t t = sv.refs[r];
            if (!in_box(sv.box_lo[t], sv.box_hi[t], px, py, pz)) continue;
            const float4 A = sv.geo[4 * t], e1 = sv.geo[4 * t + 1], e2 = sv.geo[4 * t + 2],
                         n = sv.geo[4 * t + 3];
            const float ax = px - A.x, ay = py - A.y, az = pz - A.z;
            const float s = ax * n.x + ay * n.y + az * n.z;
            const float d2 = point_tri_dist2(ax, ay, az, e1.x, e1.y, e1.z, e2.x, e2.y, e2.z, s);
            if (d2 < sv.thickness2) {
                const float push = sv.thickness - s;
                sx += push * n.x;
                sy += push * n.y;
                sz += push * n.z;
                ++cnt;
            }
        }
        if (cnt > 0) {
            const float inv = 1.0f / (float)cnt;
            px += sx * inv;
            py += sy * inv;
            pz += sz * inv;
            qx = -sp.restitution * qx;
            qy = -sp.restitution * qy;
            qz = -sp.restitution * qz;
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
                          hipStream_t stream) {
    if (cv.n <= 0) return hipSuccess;
    if (block <= 0 || block > 256 || (block & 63)) block = 256;
    const int grid = (cv.n + block - 1) / block;
    if (sv.n_tris > 0)
        k_substep<true><<<grid, block, 0, stream>>>(cv, sv, sp, xs, vs, xd, vd);
    else
        k_substep<false><<<grid, block, 0, stream>>>(cv, sv, sp, xs, vs, xd, vd);
    return hipGetLastError();
}

}  // namespace cloth
